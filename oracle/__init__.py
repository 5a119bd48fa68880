"""Plain FP64 CPU oracle for the gray covariant radiative-transfer step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, calls or links anything
from here, and this package imports nothing from the product.

Every function follows the paper (arXiv 2508.15532, "Direct Solution of the
Time-Dependent Covariant Radiative Transfer Equation and its Coupling to
GRMHD with cuHARM") step by step, in the paper's order and notation, with no
blocking, fusion or reordering.  Arrays of intensities are direction-major,
shape [N_s, N1, N2, N3]; per-cell fields are [N1, N2, N3].  All floating point
is float64.

Modules
  grid         geodesic angular grid (paper Sec. 3.3)
  geometry     flat and Kerr-Schild metric / tetrad factors (Sec. 2.1, App. A)
  transport    PLI reconstruction and spatial / angular fluxes (Sec. 3.4-3.5)
  interaction  implicit radiation-fluid source step (Sec. 3.6)
  step         predictor-corrector step and moments (Sec. 3.7, Eq. R)

Parity status of each function is stated in its docstring; readings of
ambiguous passages are listed in the repository's design notes.
"""
