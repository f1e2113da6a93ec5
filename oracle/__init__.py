"""FP64 CPU oracle: test infrastructure only.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may use
this package.  It shares no code with the GPU library (paper_1401_0838_amd) and
never imports it.  Contents:
  pic_oracle.c  plain FP64 C implementation of one PIC step
  ref.py        ctypes wrapper around it plus numpy diagnostics
  psi.py        correction-stencil coefficients by rational interpolation
                in 50-digit arithmetic (Sec. 2, Eqs. 3-5)
  brute.py      dense / DFT brute-force step for tiny grids (the oracle's pin)
  fit.py        growth-rate fit of transverse field energy
  adjoint.py    reverse-mode adjoint of the oracle step (exact transposes)
"""
