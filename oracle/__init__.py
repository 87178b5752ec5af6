"""Plain, slow, FP64 CPU oracle for the calibrated FFT-correlator.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library: it is written directly from the paper's definitions.

Modules
-------
geometry   antenna positions, baseline types, redundant groups, the subset
           selection rule (Sec. 5, eq. subredcal_frac_bls) and the
           degeneracy criterion (Sec. 5.2).
correlator the direct FX correlator (Sec. 1), the redundant average of
           eq. modelvis and the reduced X-engine (Fig. 1, calibrator box).
redcal     the redundant-calibration model (eq. redcal), chi^2 (eq. redchi),
           degrees of freedom (eq. dof), its Wirtinger gradient, logcal
           (eq. logcal), Gauss-Newton (Taylor-expansion lincal, Sec. 2),
           omnical-style damped updates (Sec. 3) and degeneracy fixing.
stats      the predicted gain covariance of eq. cov / eq. gaincov (the
           linearised system's pseudo-inverse, degeneracies projected out)
           and chi^2_r of eq. redchi.

Parity status of each function is stated in its docstring; every function
here is pinned by a `-m "not gpu"` test against something other than itself.
"""
from . import geometry, correlator, redcal, stats  # noqa: F401
