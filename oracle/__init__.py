"""FP64 CPU oracle for exponential discriminant analysis (EDA).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check of the entry module and the CPU-baseline leg
of the benchmark may use it.  It shares no code with the HIP library; the
only module both sides use is ``datagen`` (seeded inputs, no method
arithmetic).

Everything here is plain NumPy / SciPy in float64 and follows the paper's
definitions directly (Wu, Feng, Zhang, Yang, "Inexact Krylov subspace
algorithms for large matrix exponential eigenproblem from dimensionality
reduction", arXiv 1512.06500):

* scatter factors H_W, H_B                        -- Section 1, eqs. (1.1)-(1.2)
* exp of a symmetric matrix by eigendecomposition -- Section 2, eq. (2.3)
* exp by its power series (tiny inputs, mpmath)   -- Section 2, eq. (2.1)
* closed-form exp-vector products                 -- Section 3.1, Theorem 3.1
                                                     (eqs. (3.9)-(3.11)) and
                                                     Algorithm 2 (QR + SVD route)
* dense EDA (the plain definition of the result)  -- Algorithm 1, pencil eq. (1.7)
* exact reduction to the (n+k)-dim pencil (O2)    -- follows from Theorem 3.1
* the EDA criterion rho and the bounds used as checks -- eq. (1.6); Section 3.2
  (eigenvalue bounds of Theorem 3.2, criterion bounds of Theorem 3.4,
  unit-eigenvalue count of Theorem 3.6)
* nearest-neighbour classification and Theorem 3.7 -- Section 3.3 (oracle.nn)

Equation numbers are the printed ones (section.number).
"""
from .eda_oracle import *  # noqa: F401,F403
from .eda_oracle import __all__  # noqa: F401
from . import nn  # noqa: F401
