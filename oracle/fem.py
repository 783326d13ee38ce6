"""P1 tetrahedral finite elements in float64 (test infrastructure, see package docstring).

Follows the model problem and its discretisation (Section 2, Problems 2.1-2.3),
with the coefficient a(x) of Section 7.2 as a per-element constant kappa, the H1
inner product matrices of Section 4 (the bilinear form int grad w . grad v + w v,
used for R_i and for R_BB in Lemma 4.2), and the load b = M I_h f (consistent
mass matrix times the nodal interpolant of f).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def tet_geometry(xyz: np.ndarray, tets: np.ndarray):
    """Volumes |T| and barycentric gradients grad(lambda_a), a = 0..3, per tet.

    With J the 3x3 matrix whose columns are x1-x0, x2-x0, x3-x0, the map
    x = x0 + J xi gives lambda_a = xi_a (a = 1..3), so grad(lambda_a) is row a of
    J^{-1}, and lambda_0 = 1 - sum gives grad(lambda_0) = -sum of the others.
    """
    X = xyz[tets]                                   # (t, 4, 3)
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))   # columns = edge vectors
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                         # rows = grad lambda_1..3
    grads = np.empty((tets.shape[0], 4, 3))
    grads[:, 1:, :] = Jinv
    grads[:, 0, :] = -Jinv.sum(axis=1)
    return np.abs(det) / 6.0, det, grads


def element_matrices(xyz, tets, kappa):
    """Per-tet stiffness kappa|T| grad(l_a).grad(l_b), unweighted stiffness, and mass |T|(1+d_ab)/20."""
    vol, _, g = tet_geometry(xyz, tets)
    G = np.einsum("tai,tbi->tab", g, g) * vol[:, None, None]
    Ke = G * kappa[:, None, None]
    Me = (np.ones((4, 4)) + np.eye(4))[None, :, :] * (vol / 20.0)[:, None, None]
    return Ke, G, Me


def assemble(values_e: np.ndarray, tets: np.ndarray, rows_map: np.ndarray, n_rows: int,
             cols_map: np.ndarray | None = None, n_cols: int | None = None) -> sp.csr_matrix:
    """Sum element matrices into a sparse matrix.

    rows_map / cols_map send global node ids to local indices; entries whose
    node maps to -1 are dropped (Dirichlet nodes, or nodes outside the index set).
    """
    if cols_map is None:
        cols_map, n_cols = rows_map, n_rows
    r = rows_map[tets]                                  # (t, 4)
    c = cols_map[tets]
    R = np.repeat(r[:, :, None], 4, axis=2)
    C = np.repeat(c[:, None, :], 4, axis=1)
    keep = (R >= 0) & (C >= 0)
    A = sp.coo_matrix((values_e[keep], (R[keep], C[keep])), shape=(n_rows, n_cols))
    return A.tocsr()


def load_vector(Me: np.ndarray, tets: np.ndarray, f_nodal: np.ndarray | None, n_nodes_global: int,
                rows_map: np.ndarray, n_rows: int) -> np.ndarray:
    """b_a = sum over tets of sum_b M_e[a,b] f(x_b): consistent mass times the P1 interpolant."""
    if f_nodal is None:
        f_nodal = np.ones(n_nodes_global)
    be = np.einsum("tab,tb->ta", Me, f_nodal[tets])
    r = rows_map[tets]
    keep = r >= 0
    return np.bincount(r[keep], weights=be[keep], minlength=n_rows).astype(np.float64)


def global_system(mesh, kappa, f_nodal):
    """Global stiffness A and load b on the free (non-Dirichlet) nodes (Problem 2.2)."""
    free = np.flatnonzero(mesh.dirichlet == 0)
    gmap = -np.ones(mesh.n_nodes, dtype=np.int64)
    gmap[free] = np.arange(free.size)
    Ke, _, Me = element_matrices(mesh.xyz, mesh.tets, kappa)
    A = assemble(Ke, mesh.tets, gmap, free.size)
    b = load_vector(Me, mesh.tets, f_nodal, mesh.n_nodes, gmap, free.size)
    return A, b, free, gmap
