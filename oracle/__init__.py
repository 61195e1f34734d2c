"""Reference oracle for circulant-embedding conditional simulation with local
Kriging (Bailey, Bandyopadhyay and Nychka, arXiv 2109.11044).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation of what the method computes, written from the paper.  It exists
so that the HIP path can be checked against something obviously correct.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does, and it shares no code, tables or
helpers with the HIP library.

Modules, in the order the method uses them:

* ``covariance`` -- Matern covariance family (Section 3.3) with geometric
  anisotropy.
* ``philox``     -- Philox4x32-10 counter-based generator and Box-Muller
  normals; the one random stream both sides implement independently.
* ``ce``         -- circulant-embedding setup (torus base, eigenvalues,
  negative-eigenvalue ladder) and the unconditional grid draw (Section 1,
  Section 2.1 item (a)).
* ``localkrige`` -- local Kriging of off-grid observations from their
  (2 n_p)^2 nearest grid nodes: weights, conditional variances and synthetic
  observations (Section 2.1 items (b)-(d); Section 3.1; Section 3.6).
* ``kriging``    -- Kriging of residuals from the observations onto the grid,
  the conditioning steps 1, 4 and 5 of the algorithm in Section 2 and the
  conditional law eq. (4) of Section 3.
* ``pipeline``   -- the five-step conditional simulation put together, plus
  test-only outputs (explicit linear maps, exact conditional law).

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, brute force, printed values or the exact conditional law; see
each module's header.
"""

from . import covariance, philox, ce, localkrige, kriging, pipeline  # noqa: F401
