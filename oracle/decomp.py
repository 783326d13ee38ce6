"""Index sets of the overlapping decomposition (test infrastructure, see package docstring).

Section 3: subdomains omega_i overlap in one element layer; omega_i^+ is omega_i
extended by r.  Section 4: I = degrees of freedom in the interior of omega_i^+,
B = degrees of freedom on the boundary of omega_i^+ minus the Dirichlet boundary,
C_i restricts I to the degrees of freedom of V_i.  Section 6, step 2: D_i
restricts V_i to the interior of omega_i (the stitching operator of
Definition 3.1).  Section 6, step 3: omega_0 = the elements in two or more
subdomains.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_FACES = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])


def boundary_nodes(tets: np.ndarray) -> np.ndarray:
    """Nodes on the boundary of the union of the given tets: nodes of faces used exactly once."""
    f = np.sort(tets[:, _FACES].reshape(-1, 3), axis=1)
    uniq, counts = np.unique(f, axis=0, return_counts=True)
    return np.unique(uniq[counts == 1].ravel())


@dataclass
class LocalSets:
    ext_tets: np.ndarray    # global tet ids of omega_i^+
    core_tets: np.ndarray   # global tet ids of omega_i
    I: np.ndarray           # global node ids, sorted: interior of omega_i^+, not Dirichlet
    B: np.ndarray           # global node ids, sorted: boundary of omega_i^+, not Dirichlet
    V: np.ndarray           # global node ids, sorted: nodes of omega_i, not Dirichlet
    P: np.ndarray           # global node ids, sorted: free nodes whose whole star lies in omega_i


def local_sets(mesh, subdomains, i: int, star_count: np.ndarray | None = None) -> LocalSets:
    ext = subdomains.ext(i).astype(np.int64)
    core = subdomains.core(i).astype(np.int64)
    dir_ = mesh.dirichlet != 0
    ext_nodes = np.unique(mesh.tets[ext])
    bnd = boundary_nodes(mesh.tets[ext])
    on_bnd = np.zeros(mesh.n_nodes, dtype=bool)
    on_bnd[bnd] = True
    I = ext_nodes[~on_bnd[ext_nodes] & ~dir_[ext_nodes]]
    B = ext_nodes[on_bnd[ext_nodes] & ~dir_[ext_nodes]]
    core_nodes = np.unique(mesh.tets[core])
    V = core_nodes[~dir_[core_nodes]]
    if star_count is None:
        star_count = np.bincount(mesh.tets.ravel(), minlength=mesh.n_nodes)
    core_count = np.bincount(mesh.tets[core].ravel(), minlength=mesh.n_nodes)
    P = V[core_count[V] == star_count[V]]
    return LocalSets(ext_tets=ext, core_tets=core, I=I, B=B, V=V, P=P)


def all_local_sets(mesh, subdomains) -> list[LocalSets]:
    star = np.bincount(mesh.tets.ravel(), minlength=mesh.n_nodes)
    return [local_sets(mesh, subdomains, i, star) for i in range(subdomains.n_sub)]


def omega0_tets(mesh, subdomains) -> np.ndarray:
    """Elements that belong to at least two subdomains omega_i (Section 6, step 3)."""
    cnt = np.zeros(mesh.n_tets, dtype=np.int64)
    for i in range(subdomains.n_sub):
        cnt[subdomains.core(i)] += 1
    return np.flatnonzero(cnt >= 2)


def owner_map(mesh, sets: list[LocalSets]) -> np.ndarray:
    """owner[node] = i for node in P_i, -1 for Dirichlet nodes; raises if P_i is not a partition."""
    owner = -np.ones(mesh.n_nodes, dtype=np.int64)
    for i, s in enumerate(sets):
        if np.any(owner[s.P] >= 0):
            raise ValueError("P_i overlap: the decomposition is not a partition of the free nodes")
        owner[s.P] = i
    free = mesh.dirichlet == 0
    if np.any(owner[free] < 0):
        raise ValueError("some free node lies in no P_i")
    return owner
