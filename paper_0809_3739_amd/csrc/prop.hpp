// Host-visible descriptors of the propagation kernels (plane and pencil passes).
#pragma once
#include <hip/hip_runtime.h>

namespace mpe {

constexpr int MAX_K = 6;  // order 2K <= 12

enum PlaneMode { PM_FWD = 0, PM_LINK = 1, PM_TAIL = 2, PM_HTAIL = 3 };
enum PencilKind { PK_EXP = 0, PK_ADD = 1 };

// One plane-pass launch.  Pointers are device addresses; element types are the
// plan's data type F (float or double) for real arrays and cx<F> for spectra.
struct PlaneArgs {
  const void* real_in;        // PM_FWD: states; PM_HTAIL: the phi of V*phi
  const void* spec_in;        // PM_LINK, PM_HTAIL: half spectra; PM_TAIL: chain 1 half spectra
  void* spec_out;             // PM_FWD, PM_LINK
  void* real_out;             // PM_TAIL, PM_HTAIL
  const void* fac;            // pointwise factor table [z][y][x] (PM_TAIL: base of the table set)
  const void* rx;             // roots of unity, length NX/2
  const void* ry;             // roots of unity, length NY
  const void* wpost;          // exp(-2 pi i k / NX), k = 0..NX/4
  long real_state_stride;     // elements between consecutive states (real arrays)
  long spec_state_stride;     // elements between consecutive states (spectra)
  long chain_stride;          // PM_TAIL: elements between the chains' spectra
  long fac_table_stride;      // PM_TAIL: elements between consecutive factor tables
  int state0;                 // first state of this launch
  int K;                      // PM_TAIL: number of chains
  double coef[MAX_K];         // PM_TAIL: c_1..c_K
};

struct PencilArgs {
  void* data;                 // half spectra, in place
  const void* rz;             // roots of unity, length NZ
  const void* tx;             // per-axis tables (kx, ky, kz) in the data type
  const void* ty;
  const void* tz;
  long state_stride;          // elements between states = NZ * M
  int M;                      // columns per z = NY * NXH
  int NXH;                    // NX/2 + 1
  int state0;
};

bool plane_supported(int is_double, int nx, int ny);
bool pencil_supported(int nz);
hipError_t launch_plane(int is_double, int mode, int nx, const PlaneArgs& a, int nz, int nstates, hipStream_t st);
hipError_t launch_pencil(int is_double, int kind, int nz, const PencilArgs& a, int nstates, hipStream_t st);

}  // namespace mpe
