"""FP64 CPU oracle for generalized-loss CP tensor completion.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_1910_02371_amd``) never imports it, and it imports nothing from the
GPU library: the two share no code.  Inputs come from the seeded generators in
``paper_1910_02371_amd.workloads``, which hold no arithmetic of the method.

Every function is the plain definition from the paper, written out in NumPy
float64 for arbitrary tensor order N:

* ``cp``      -- index (stable counting sort), TTTP, loss maps, MTTKRP, Gram,
                 row solves, Solve Factor, objective, gradient, GN operator,
                 full Hessian-vector product.
* ``solvers`` -- ALS sweep, ALS fast-loss identity, PCG Gauss-Newton step,
                 generalized alternating-minimization sweep, CCD++ sweep.
* ``bf16``    -- round-to-nearest-even emulation of bfloat16 storage.

Parity status of each function is listed in its docstring; every function here
is pinned by ``tests/test_oracle_*.py`` except where a docstring says
"parity unpinned".
"""
from .cp import (  # noqa: F401
    build_index, tttp, phi, dphi, d2phi, mttkrp, row_design, gram,
    solve_rows, solve_factor, objective, gradient, jvp, gn_matvec, newton_matvec,
    rmse, cholesky_info, LOSS_LS, LOSS_POISSON_LOG,
)
from .solvers import (  # noqa: F401
    als_sweep, als_fast_loss, pcg, gn_step, gam_sweep, ccd_sweep,
)
from .bf16 import bf16_round  # noqa: F401
