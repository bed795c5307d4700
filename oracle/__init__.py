"""FP64 CPU oracle for constrained-least-squares radio image formation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy (complex128 / float64) implementation of the method of Mouri
Sardarabadi, Leshem and van der Veen, "Radio Astronomical Image Formation using
Constrained Least Squares and Krylov Subspaces".  Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  The HIP
library never calls it and shares no code, table or constant with it.

Modules
-------
imaging     steering vectors, the Khatri-Rao operators (correlation /
            beamforming), matched-filter and MVDR dirty images, bounds and
            detection threshold (Sec. II, Sec. IV-B, App. A)
lsqr        Golub-Kahan bidiagonalisation with the LSQR updates (Sec. IV-A)
active_set  the active-set solver of Table I with the detection threshold
            (Sec. III)
pwls        the constrained preconditioned weighted LS problem (eq. preWLS)
            as the LS problem on whitened, D-scaled inputs
offgrid     strong off-grid sources (Sec. III-E, eq. doals): the free pixels'
            offsets by Gauss-Newton rounds around the LSQR subproblem
multi       K covariance blocks over one grid (Earth-rotation snapshots or
            frequency channels, eq. vectRtotal): MF / MVDR images, bounds,
            thresholds and the stacked solve (eqs. mfdimg, wmvdr, App. A)

Pins (what the oracle is checked against, in tests/test_oracle_*.py): the
Kronecker/Khatri-Rao identities of the Notation section against an explicitly
built dense Psi, closed forms for a single source (MF and Sherman-Morrison
MVDR), the MF >= MVDR ordering, the Jacobi-preconditioned-WLS identity for the
MVDR image (Sec. II-C), the bounds' kappa_b terms and the detection threshold
against the Monte Carlo spread of the MF and MVDR images over sample
covariances (App. A, K = 1), LSQR against SVD minimum-norm least squares,
the active-set solution against SciPy's BVLS and brute-force enumeration
(objective and KKT conditions, eqs. gradFcond/etaL/etaU), exact recovery of
on-grid sources from an exact covariance, and invariances (scale, antenna
permutation, array translation, mirror).  The thresholded path with
kappa_d > 0 beyond those pins is defined by this oracle ("parity unpinned" for
the exact add/drop sequence).  PWLS (tests/test_oracle_pwls.py): Cholesky
whitening against the R^-1/2 weighting from an eigendecomposition, the
transformed operators against the dense weighted Khatri-Rao matrix, the
gradient at zero against the unbiased MVDR image from R^-1, the box solution
against BVLS with KKT, bound pixels at gamma in image units, and the
threshold's MVDR standard deviation against a Monte Carlo.  K blocks
(tests/test_oracle_multi.py): the stacked solve against BVLS on the dense
stacked Psi with KKT, K identical blocks against the single-block problem,
the MVDR <= MF ordering and the ASSC lower bound, both App. A variances
against Monte Carlo, and adjointness of the stacked operators.
"""

from .imaging import (  # noqa: F401
    pixel_directions,
    steering,
    forward,
    adjoint,
    mf_image,
    mvdr_inverse_power,
    upper_bound,
    detection_threshold,
    NotPositiveDefinite,
)
from .lsqr import lsqr, LsqrResult  # noqa: F401
from .active_set import solve, SolveResult, STATE_L, STATE_F, STATE_U  # noqa: F401
from .pwls import pwls_problem, pwls_scaling, pwls_threshold, solve_pwls, whitening_factor  # noqa: F401
from .multi import (  # noqa: F401
    steering_blocks,
    mf_image_multi,
    mf_std_multi,
    mvdr_powers,
    upper_bound_multi,
    detection_threshold_multi,
    solve_multi,
)
from .offgrid import gauss_newton_block, offset_gradient, solve_offgrid, steering_at  # noqa: F401
