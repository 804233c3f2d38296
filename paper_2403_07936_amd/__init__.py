"""MI355X-native geometric multigrid for the 2-D (pressure-)Poisson equation.

The solver is the HIP library ``libmg355.so`` behind the C ABI of
``include/mg.h``; ``binding`` wraps it with ctypes under the same names and
``solver.Solver`` adds torch-tensor marshalling.  Nothing is loaded at
import time; the first call that needs the library loads it and raises if it
is missing.
"""

__all__ = ["binding", "build", "solver"]
