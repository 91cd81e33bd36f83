"""adimx: ADI isogeometric Maxwell time stepping on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libadimx.so`` (hand-written HIP
kernels, see ``include/adimx.h``); this package only marshals arguments
(``_lib``), gives a small object API (``solver``) and builds the library
(``build``).  Importing the package does not load the library; the first
use of ``solver.Solver`` does, and raises if it is missing.
"""

__all__ = ["build", "solver"]
