// Host-visible descriptors of the propagation kernels (plane and pencil passes).
#pragma once
#include <hip/hip_runtime.h>

namespace mpe {

constexpr int MAX_K = 6;  // order 2K <= 12

enum PlaneMode { PM_FWD = 0, PM_LINK = 1, PM_TAIL = 2, PM_HTAIL = 3, PM_OUT = 4 };
enum PencilKind { PK_EXP = 0, PK_ADD = 1, PK_FFT_FWD = 2, PK_FFT_INV = 3 };
// Row-pass modes of the three-pass plans (x transforms alone): as the plane
// modes of the same names, without the y transform.
enum RowMode { RW_FWD = 0, RW_LINK = 1, RW_OUT = 2, RW_HTAIL = 3 };

// Per-state addresses for launches that cover states of several systems of
// one grid (batched uneven systems).  One entry per state of the launch.
struct StateDesc {
  const void* real_in;        // states (PM_FWD) or phi (PM_HTAIL)
  void* real_out;             // PM_TAIL / PM_HTAIL output
  void* spec;                 // this state's chain-0 half spectrum
  const void* fac;            // the state's system: base of its factor-table set
  const void* V;              // the state's system: potential in the data type (PM_HTAIL)
  const void* kin;            // the state's system: kinetic exp tables of chain 0
  const void* hk;             // the state's system: additive kinetic tables (H)
  long chain_stride;          // elements between consecutive chains' spectra
};

// One plane-pass launch.  Pointers are device addresses; element types are the
// plan's data type F (float or double) for real arrays and cx<F> for spectra.
// Without desc, state s of the launch sits at base + (state0 + s) * stride.
struct PlaneArgs {
  const void* real_in;        // PM_FWD: states; PM_HTAIL: the phi of V*phi
  void* spec;                 // half spectra of this launch's chain (PM_TAIL: chain 1)
  void* real_out;             // PM_TAIL, PM_HTAIL
  const void* fac;            // factor-table set [2K][z][y][x] (PM_HTAIL: V)
  const void* rx;             // roots of unity, length NX/2
  const void* ry;             // roots of unity, length NY
  const void* wpost;          // exp(-2 pi i k / NX), k = 0..NX/4
  const StateDesc* desc;      // optional per-state addresses (batched launches)
  long real_state_stride;     // elements between consecutive states (real arrays)
  long spec_state_stride;     // elements between consecutive states (spectra)
  long chain_stride;          // PM_TAIL, PM_FWD: elements between the chains' spectra
  long fac_table_stride;      // elements between consecutive factor tables (= N)
  int fac_index;              // PM_FWD / PM_LINK: factor table used, -1 for none
  int chain;                  // desc mode: chain of this launch
  int state0;                 // first state of this launch
  int K;                      // PM_TAIL: number of chains
  double coef[MAX_K];         // PM_TAIL: c_1..c_K
  // PM_FWD: chains formed from one read of the rows (0 or 1: one); chain c
  // takes factor table fac_index + 2c and writes spec + c * chain_stride (the
  // first potential half-steps exp(-dt V / 2k) of chains k = 1..K are tables
  // 1, 3, .., 2K - 1)
  int fwd_chains;
  // PM_FWD with fwd_chains > 1, one work-group per plane (persist_mode 0):
  // 0 = one work item per (chain, plane), the chains of a plane on one XCD;
  // 1 = each work-group forms every chain of its plane in turn, reading the
  //     rows again from its own CU's caches for chains after the first (grids
  //     of 64 points and more; smaller grids take 0).  Both give the same bits.
  int fwd_loop;
  // PM_FWD / PM_LINK launch shape (grids of 64 points and more): persist_mode
  // 0 = one work-group per (z, state) plane; 1 / 2 = persist_blocks resident
  // work-groups looping over the planes, each loading the next plane's input
  // while it transforms the current one, with the register budget of one
  // work-group per CU (1) or of the one-plane launch (2)
  int persist_mode;
  int persist_blocks;
  // PM_FWD / PM_LINK / PM_HTAIL / PM_OUT plane order: 0 = z planes fastest (neighbouring work-groups
  // take neighbouring planes of one state), 1 = states fastest (the work-groups
  // in flight share a few z planes, so each factor-table plane is fetched into
  // an XCD's L2 once and read there by every state)
  int states_fast;
  int nz, nstates;            // set by the launcher
  int ny;                     // row passes: rows per z plane
};

struct PencilArgs {
  void* data;                 // half spectra, in place
  const void* rz;             // roots of unity, length NZ
  const void* tab;            // per-axis tables [kx | ky | kz] in the data type
  const StateDesc* desc;      // optional per-state addresses
  long state_stride;          // elements between states = NZ * M
  int M;                      // columns per z = NY * NXH
  int NXH;                    // NX/2 + 1
  int NY;
  int state0;
  int chain;                  // desc mode: chain of this launch
  int desc_tables;            // desc mode: 0 = exp tables of `chain`, 1 = additive tables
  int tile;                   // work-group shape: 0 = 256 threads, 1 = 128, 2 = 512 (columns scale alike)
};

bool plane_supported(int is_double, int nx, int ny);
// Whether the fused tail pass (all K chains combined in float64 registers) runs
// out of registers for this plane; then each chain leaves the tail on its own
// (PM_OUT into a real buffer) and launch_combine forms sum_k c_k x_k.
bool tail_split(int is_double, int nx);
// dst[i] = sum_k coef[k] tmp[k * stride + i], i < n, accumulated in float64
hipError_t launch_combine(int is_double, const void* tmp, long stride, int K, const double* coef, void* dst, long n,
                          hipStream_t st);
bool pencil_supported(int nz);
bool row_supported(int nx);
// Row pass over the rows of states [state0, state0 + nstates): nstates * nz * ny rows of nx points.
hipError_t launch_rows(int is_double, int mode, int nx, const PlaneArgs& a, int ny, int nz, int nstates,
                       hipStream_t st);
hipError_t launch_plane(int is_double, int mode, int nx, const PlaneArgs& a, int nz, int nstates, hipStream_t st);
hipError_t launch_pencil(int is_double, int kind, int nz, const PencilArgs& a, int nstates, hipStream_t st);

}  // namespace mpe
