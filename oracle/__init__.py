"""FP64 CPU oracle for the exact camera covariance (test infrastructure only).

This package is the slow, obviously-correct reference that the GPU library is
checked against.  It is *test infrastructure*: only the tests, the smoke
entry point and the CPU-baseline leg of the benchmark may import it.  The
product library never calls it and shares no code with it: the Jacobians here
come from forward-mode dual numbers (the GPU uses hand-derived formulas), the
Schur complement from SciPy sparse products (the GPU uses a binned scatter),
the rotation nullspace block from a least-squares solve (the GPU uses 3x3
normal equations), the orthonormal basis from Householder QR (the GPU uses
Cholesky-QR), and the inverse from LAPACK's Cholesky (the GPU uses its own
blocked MFMA kernels).

Modules, in the order of the paper's method:

* ``dual``       forward-mode dual numbers (derivative machinery)
* ``camera``     projection function and its Jacobian blocks (Sec. 5.1)
* ``schur``      normal-equation blocks U, V, W and Z = U - W V^-1 W^T
                 (Sec. 4 normal equations; Sec. 5.2 block inversion and Schur
                 complement)
* ``nullspace``  similarity nullspace H with the rotation block solved from
                 J_r H_r = B (Sec. 5.1)
* ``covariance`` Moore-Penrose camera covariance Z^+ = (Z + a Q Q^T)^-1 - Q Q^T / a
                 with Jacobi conditioning (Sec. 4 gauge, Sec. 5.2 conditioning)
* ``pipeline``   end to end, plus the input checks shared by the error tests
* ``paper_gauge`` the paper's own gauge, (M^+)_cc: the definition on the dense
                 M, and the points eliminated with the full nullspace
                 (Sec. 4, Sec. 5.2)
* ``subrecon``   sub-reconstructions (Sec. 6): per-group sub-scenes, each solved
                 exactly, the minimum-trace block per camera
* ``screener``   the learned screener's reference: per-camera features, the
                 log-Cholesky label transform, an FP64 MLP with its gradient,
                 and Adam (not part of the paper; its labels are the exact
                 covariances above)

Parity status: every function is pinned by a CPU test against something other
than itself (complex-step derivatives, a dense brute-force Schur complement,
J H = 0, the closed-form SO(3) inverse right Jacobian, SVD and multiprecision
pseudo-inverses, Penrose conditions, gauge-invariant sub-blocks, Loewner
monotonicity and a matrix with a prescribed spectrum).  The paper prints no
worked example, so value-level agreement with its figures is unpinned.
"""
from .pipeline import OracleError, camera_covariance, validate  # noqa: F401
