"""Plain FP64 CPU oracle for the batched constraint projection.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything here.  The
GPU library never calls into this package and shares no code with it.

What it computes, for every sample independently (the batch Jacobian is
block-diagonal across samples, paper Sec. III-B):

    u* = argmin_u 1/2 ||u - u_hat||^2   subject to  h(u) = 0

(paper eq. for the projection step in Sec. II-A and its restatement in
Sec. III-B), by Newton-Raphson on the KKT conditions

    F(u, lam) = [ u - u_hat + J(u)^T lam ;  h(u) ] = 0

whose Jacobian is the Newton-KKT matrix [[W, J^T], [J, 0]] with
W = Hessian of the Lagrangian (Appendix B).  Each Newton step assembles that
matrix explicitly as a scipy sparse matrix and solves it with a general sparse
direct solver; there is no Schur reduction, no ordering trick and no banded
factorization here, so the GPU path's structure is checked against a plain
statement of the same equations.

Modules:
  families  -- h(u), J(u) and the Hessian of lam^T h(u) for each constraint family
  kkt       -- the Newton-KKT iteration and the implicit-function adjoint
  metric    -- the per-constraint-type error of Appendix E

Parity status per function is recorded in each module's header.
"""
from .families import FAMILIES, family_of, constraint_types  # noqa: F401
from .kkt import project_sample, project_batch, adjoint_sample, adjoint_batch  # noqa: F401
from .metric import constraint_error, max_violation  # noqa: F401
