"""FP64 CPU oracle of the flip-free ADMM iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU
library (``paper_2107_05200_amd``); the only common input is the seeded
workload generator, which holds none of the method's arithmetic.

The oracle follows Stein, Li & Solomon, "A Splitting Scheme for Flip-Free
Distortion Energies": the three-block ADMM of Algorithm 1 (sub-steps of
Section "Our Optimization Method"), the initialisation and residuals of
Section "Implementation", and the closed-form sub-step solvers of the
supplement.  It is plain NumPy / SciPy in float64; library primitives
(SVD, symmetric eigendecomposition, sparse LU solve) serve as steps.
"""
from .admm import *  # noqa: F401,F403
from . import adjoint  # noqa: F401
from . import tutte  # noqa: F401
from . import ordering  # noqa: F401
