"""Galerkin projection of the global system and the reduced solve (test infrastructure).

Section 6, step 3: Q^T A Q is built block by block (eq. 6.1) without forming A
or Q.  Diagonal blocks come from the local step.  An off-diagonal block
Q_i^T A_ij Q_j is non-zero only for neighbouring subdomains; its entries depend
only on the elements of omega_0 (elements in two or more subdomains), so it is
computed from a stiffness matrix A_0 assembled on omega_0 and the rows of Q_i
and Q_j on the shared nodes.  The reduced system is then solved: the paper uses
conjugate gradients with a diagonal preconditioner (end of Section 6, step 3, and
the scaling runs of Section 7), given here by `pcg_diag`; a dense Cholesky
factorization (`solve_reduced`) gives the same solution.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

from . import decomp, fem


def offsets(results) -> np.ndarray:
    """Block offsets of the reduced system: each subdomain contributes its basis columns
    (k_eff + 1, or fewer after the basis update)."""
    return np.concatenate([[0], np.cumsum([r.Vloc.shape[1] for r in results])]).astype(np.int64)


def omega0_stiffness(mesh, kappa, subdomains) -> sp.csr_matrix:
    """A_0: the stiffness matrix assembled over omega_0 only, on all free nodes."""
    t0 = decomp.omega0_tets(mesh, subdomains)
    free = np.flatnonzero(mesh.dirichlet == 0)
    gmap = -np.ones(mesh.n_nodes, dtype=np.int64)
    gmap[free] = np.arange(free.size)
    Ke, _, _ = fem.element_matrices(mesh.xyz, mesh.tets[t0], kappa[t0])
    A0 = fem.assemble(Ke, mesh.tets[t0], gmap, free.size)
    return A0, free, gmap


def neighbour_blocks(mesh, kappa, subdomains, results):
    """Off-diagonal blocks {(i, j): Q_i^T A_ij Q_j} for i != j, from A_0 and the interface rows."""
    sets = [r.sets for r in results]
    owner = decomp.owner_map(mesh, sets)
    A0, free, gmap = omega0_stiffness(mesh, kappa, subdomains)
    coo = A0.tocoo()
    gi, gj = free[coo.row], free[coo.col]
    oi, oj = owner[gi], owner[gj]
    cross = oi != oj
    pos = []
    for r in results:
        m = -np.ones(mesh.n_nodes, dtype=np.int64)
        m[r.sets.P] = np.arange(r.sets.P.size)
        pos.append(m)
    blocks = {}
    pairs = np.unique(np.stack([oi[cross], oj[cross]], axis=1), axis=0)
    for i, j in pairs:
        sel = cross & (oi == i) & (oj == j)
        rows_g, cols_g, vals = gi[sel], gj[sel], coo.data[sel]
        Gij = np.unique(rows_g)       # Gamma_ij: nodes of P_i coupled to P_j
        Gji = np.unique(cols_g)
        rloc = np.searchsorted(Gij, rows_g)
        cloc = np.searchsorted(Gji, cols_g)
        Asub = sp.coo_matrix((vals, (rloc, cloc)), shape=(Gij.size, Gji.size)).toarray()
        Vi = results[i].Vloc[pos[i][Gij]]
        Vj = results[j].Vloc[pos[j][Gji]]
        blocks[(int(i), int(j))] = Vi.T @ Asub @ Vj
    return blocks


def reduced_system(mesh, kappa, subdomains, results):
    """Dense reduced matrix Q^T A Q and load Q^T b, assembled block by block."""
    off = offsets(results)
    n = int(off[-1])
    At = np.zeros((n, n))
    bt = np.zeros(n)
    for i, r in enumerate(results):
        At[off[i]:off[i + 1], off[i]:off[i + 1]] = r.Aii
        bt[off[i]:off[i + 1]] = r.bi
    for (i, j), blk in neighbour_blocks(mesh, kappa, subdomains, results).items():
        At[off[i]:off[i + 1], off[j]:off[j + 1]] = blk
    return 0.5 * (At + At.T), bt, off


def solve_reduced(At: np.ndarray, bt: np.ndarray, pinv_rtol: float | None = None) -> np.ndarray:
    """Cholesky solve; with pinv_rtol, a pseudo-inverse that drops eigenvalues below
    pinv_rtol * lambda_max (for full-rank bases whose stitched columns are dependent)."""
    if pinv_rtol is None:
        return la.cho_solve(la.cho_factor(At, lower=False), bt)
    w, U = la.eigh(At)
    keep = w > pinv_rtol * w.max()
    return U[:, keep] @ ((U[:, keep].T @ bt) / w[keep])


def pcg_diag(At: np.ndarray, bt: np.ndarray, rtol: float = 1e-12, max_iter: int = 20000, on_iter=None):
    """The paper's reduced solver (Section 6, step 3; Section 7): conjugate gradients on
    A~ x = b~ preconditioned by the diagonal D of A~, from x = 0, in the textbook order
    (Hestenes and Stiefel):

        r = b, z = D^-1 r, p = z
        repeat:  q = A p;  alpha = r.z / p.q;  x += alpha p;  r -= alpha q
                 stop if ||r|| <= rtol ||b||
                 z = D^-1 r;  beta = r.z(new) / r.z(old);  p = z + beta p

    r is the recurrence residual.  Returns (x, iterations, ||r|| / ||b|| at the stop).
    on_iter(k, x, r), if given, sees every iterate.  Raises if p.q <= 0 (A~ not SPD) or
    when max_iter is reached."""
    A = np.asarray(At, dtype=np.float64)
    b = np.asarray(bt, dtype=np.float64)
    dinv = 1.0 / np.diag(A)
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for k in range(1, max_iter + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0.0:
            raise np.linalg.LinAlgError("p'Ap <= 0: the reduced matrix is not positive definite")
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        if on_iter is not None:
            on_iter(k, x, r)
        res = np.linalg.norm(r) / nb
        if res <= rtol:
            return x, k, res
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError(f"reduced PCG did not reach {rtol} in {max_iter} iterations")


def block_pinv(At: np.ndarray, off, drop: float = 0.0) -> np.ndarray:
    """The block-diagonal preconditioner of the reduced system: for each subdomain's diagonal
    block A~_ii = U Lambda U^T, the pseudo-inverse U_r Lambda_r^-1 U_r^T over the eigenvalues
    above drop * lambda_max (the directions the basis update of Section 6, step 2 keeps)."""
    n = At.shape[0]
    M = np.zeros((n, n))
    for i in range(len(off) - 1):
        a, b = int(off[i]), int(off[i + 1])
        lam, U = np.linalg.eigh(0.5 * (At[a:b, a:b] + At[a:b, a:b].T))
        keep = lam > drop * lam.max()
        M[a:b, a:b] = (U[:, keep] / lam[keep]) @ U[:, keep].T
    return M


def pcg_block(At: np.ndarray, bt: np.ndarray, off, drop: float = 0.0, rtol: float = 1e-12, max_iter: int = 20000,
              on_iter=None):
    """Conjugate gradients on A~ x = b~ preconditioned by `block_pinv` (reading of Section 6:
    after the basis update the diagonal blocks are the identity and the paper's diagonal
    preconditioner leaves plain CG on the updated system, which is this iteration on the
    un-updated one).  Same steps as `pcg_diag`.  The stopping test is the updated system's:
    with M^-1 = T T^T its residual is T^T r, so stop when sqrt(r'M^-1 r / b'M^-1 b) <= rtol.
    With drop > 0 the preconditioner is singular: the dropped part of r never shrinks and, once
    the kept part is near rounding relative to it, the recurrence loses conjugacy (the basis
    update, which removes those directions from the system, has no such part).  drop = 0 keeps
    every positive eigenvalue.  Returns (x, iterations, that ratio)."""
    A = np.asarray(At, dtype=np.float64)
    b = np.asarray(bt, dtype=np.float64)
    Minv = block_pinv(A, off, drop)
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = Minv @ r
    p = z.copy()
    rz = r @ z
    rz0 = rz
    for k in range(1, max_iter + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0.0:
            raise np.linalg.LinAlgError("p'Ap <= 0: the reduced matrix is not positive definite")
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        if on_iter is not None:
            on_iter(k, x, r)
        z = Minv @ r
        rz_new = r @ z
        res = np.sqrt(max(rz_new, 0.0) / rz0)
        if res <= rtol:
            return x, k, res
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError(f"reduced block PCG did not reach {rtol} in {max_iter} iterations")


def reconstruct(mesh, results, x: np.ndarray) -> np.ndarray:
    """u~ = sum_i S_i (Q_i x_i): on P_i the value is Vloc_i x_i; zero on the Dirichlet nodes."""
    off = offsets(results)
    u = np.zeros(mesh.n_nodes)
    for i, r in enumerate(results):
        u[r.sets.P] = r.Vloc @ x[off[i]:off[i + 1]]
    return u


def dense_QtAQ(mesh, kappa, results):
    """The straightforward projection: form Q (free nodes x reduced) and A, multiply."""
    A, _, free, gmap = fem.global_system(mesh, kappa, None)
    off = offsets(results)
    rows, cols, vals = [], [], []
    for i, r in enumerate(results):
        k1 = r.Vloc.shape[1]
        rr = np.repeat(gmap[r.sets.P], k1)
        cc = np.tile(np.arange(off[i], off[i] + k1), r.sets.P.size)
        rows.append(rr)
        cols.append(cc)
        vals.append(r.Vloc.ravel())
    Q = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(free.size, int(off[-1])))
    return (Q.T @ (A @ Q)).toarray(), Q
