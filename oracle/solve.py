"""Full finite element solution and error measures (test infrastructure).

Problem 2.2 solved directly on the free nodes, the energy norm of the global
stiffness A(kappa), and the Galerkin-orthogonality identity of Section 7.1:
for the reduced solution u~ = Q x,  ||u - u~||_A^2 = u^T b - x^T Q^T b.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, project, reduce


def fe_solution(mesh, kappa, f_nodal):
    A, b, free, gmap = fem.global_system(mesh, kappa, f_nodal)
    uf = spla.splu(A.tocsc()).solve(b)
    u = np.zeros(mesh.n_nodes)
    u[free] = uf
    return u, A, b, free


def energy(A, free, v: np.ndarray) -> float:
    vf = v[free]
    return float(np.sqrt(max(vf @ (A @ vf), 0.0)))


def run(problem, rank=None, tol=None, workers: int = 1, pinv_rtol=None, with_fe: bool = True,
        implicit: bool = False, update_drop=None, pcg_rtol=None, order=None):
    """The whole explicit method on one problem, plus the FE reference solution.

    implicit: local reductions through the pencil's sparse factors (`reduce.reduce_local_implicit`).
    update_drop: apply the basis update of Section 6, step 2 to every local result with this
    relative drop.  pcg_rtol: solve the reduced system with the paper's diagonal-preconditioned
    conjugate gradients to this relative residual instead of a Cholesky factorization."""
    local = reduce.reduce_all(problem, rank=rank, tol=tol, workers=workers, implicit=implicit, order=order)
    results = local if update_drop is None else [reduce.basis_update(r, update_drop) for r in local]
    At, bt, off = project.reduced_system(problem.mesh, problem.kappa, problem.subdomains, results)
    pcg_iters = None
    if pcg_rtol is not None:
        x, pcg_iters, _ = project.pcg_diag(At, bt, rtol=pcg_rtol)
    else:
        x = project.solve_reduced(At, bt, pinv_rtol)
    ut = project.reconstruct(problem.mesh, results, x)
    out = dict(results=results, local=local, At=At, bt=bt, off=off, x=x, u_tilde=ut, pcg_iters=pcg_iters)
    if with_fe:
        u, A, b, free = fe_solution(problem.mesh, problem.kappa, problem.f_nodal)
        out.update(u_fe=u, A=A, b=b, free=free,
                   red_err=energy(A, free, u - ut), u_energy=energy(A, free, u))
    return out
