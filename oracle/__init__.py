"""CPU oracle of the MPE eigensolver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call or execute anything in this package.  It shares no
code with the GPU library; the two meet only in the seeded input generators of
``workloads``.

* ``oracle.mpe``   -- the method in plain float64 NumPy/SciPy, step by step in the
  paper's order (split operator, multi-product expansion, orthonormalisation,
  Rayleigh-Ritz, variances, step-size protocol).
* ``oracle.dense`` -- exact dense references on tiny grids built without any FFT
  routine (explicit DFT matrices), used to pin ``oracle.mpe``.
"""
