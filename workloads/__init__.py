"""Seeded synthetic inputs: meshes, coefficients, box decompositions, request streams.

This module holds no arithmetic of the reduction method.  It only produces the
*inputs* that the problem statement of the paper (Section 6, first paragraph)
names: a tetrahedral mesh, a coefficient field, a load, and an overlapping
decomposition into subdomains omega_i with their extensions omega_i^+
(Section 3).  Both the FP64 CPU oracle and the HIP library consume these
arrays; neither side imports the other.

Workloads follow the paper's scaling tests (Section 7.1): the unit cube meshed
with evenly spaced tetrahedra and Dirichlet data on the whole boundary, split
into box subdomains with a few thousand degrees of freedom each and an
extension that roughly doubles the subdomain diameter.

Mesh: the unit cube cut into n^3 hexahedral cells, each split into the 6 Kuhn
tetrahedra {v, v+e_a, v+e_a+e_b, v+(1,1,1)} over the 6 axis orders (a,b,c).
Node (i,j,k) has id i + (n+1)*(j + (n+1)*k); cell (i,j,k) has id
i + n*(j + n*k) and owns tets 6*cell .. 6*cell+5.  Every tet is stored with
positive orientation.

Decomposition (boxes): per-axis cuts 0 = c_0 < ... < c_p = n.  Box (a,b,c)
has core cells [c_a, min(c_{a+1}+1, n)) per axis (one cell of overlap on the
+ side, so two neighbouring cores share exactly one element layer, Section 3)
and extension cells [max(c_a - r, 0), min(c_{a+1}+1+r, n)) (the extension by
r cell layers, the box analogue of the paper's r-hop extension).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# The 6 axis orders; the tet for order (a,b,c) is v, v+e_a, v+e_a+e_b, v+1.
_KUHN_ORDERS = list(itertools.permutations(range(3)))


@dataclass
class Mesh:
    n: int                      # cells per axis
    xyz: np.ndarray             # (n_nodes, 3) float64
    tets: np.ndarray            # (n_tets, 4) int32, positively oriented
    dirichlet: np.ndarray       # (n_nodes,) uint8, 1 on the boundary of the cube

    @property
    def n_nodes(self) -> int:
        return self.xyz.shape[0]

    @property
    def n_tets(self) -> int:
        return self.tets.shape[0]


@dataclass
class Subdomains:
    """Overlapping decomposition as tet lists (CSR over subdomains)."""
    ext_tet_ptr: np.ndarray     # (n_sub+1,) int64
    ext_tets: np.ndarray        # (nnz,) int32: tets of omega_i^+
    in_core: np.ndarray         # (nnz,) uint8: 1 if the tet also lies in omega_i
    boxes: list = field(default_factory=list)  # per subdomain ((lo,hi) core, (lo,hi) ext) cell ranges per axis

    @property
    def n_sub(self) -> int:
        return self.ext_tet_ptr.shape[0] - 1

    def ext(self, i: int) -> np.ndarray:
        return self.ext_tets[self.ext_tet_ptr[i]:self.ext_tet_ptr[i + 1]]

    def core(self, i: int) -> np.ndarray:
        s = slice(self.ext_tet_ptr[i], self.ext_tet_ptr[i + 1])
        return self.ext_tets[s][self.in_core[s] != 0]


@dataclass
class Problem:
    name: str
    mesh: Mesh
    kappa: np.ndarray           # (n_tets,) float64, piecewise constant per cell
    f_nodal: np.ndarray | None  # (n_nodes,) float64 nodal load values, None => f = 1
    subdomains: Subdomains
    rank: int                   # number of lifting modes kept per subdomain (plus q0)
    ranks: np.ndarray | None = None   # per-subdomain ranks (serving stream)
    precision: str = "fp64"
    meta: dict = field(default_factory=dict)


def kuhn_cube(n: int, jitter: float = 0.0, seed: int | None = None) -> Mesh:
    """Kuhn-tetrahedral mesh of [0,1]^3 with n cells per axis.

    jitter > 0 moves every interior coordinate (0 < index < n along that axis)
    by U(-jitter*h, +jitter*h), so the domain stays the unit cube.
    """
    n1 = n + 1
    h = 1.0 / n
    idx = np.arange(n1)
    k3, j3, i3 = np.meshgrid(idx, idx, idx, indexing="ij")
    ijk = np.stack([i3.ravel(), j3.ravel(), k3.ravel()], axis=1)  # node id order
    xyz = ijk.astype(np.float64) * h
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        interior = (ijk > 0) & (ijk < n)
        xyz = xyz + np.where(interior, d, 0.0)
    dirichlet = np.any((ijk == 0) | (ijk == n), axis=1).astype(np.uint8)

    c = np.arange(n)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)  # cell id order
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)

    def nid(p):
        return p[:, 0] + n1 * (p[:, 1] + n1 * p[:, 2])

    eye = np.eye(3, dtype=np.int64)
    for t, (a, b, _) in enumerate(_KUHN_ORDERS):
        v0 = base
        v1 = base + eye[a]
        v2 = v1 + eye[b]
        v3 = base + 1
        tets[:, t, :] = np.stack([nid(v0), nid(v1), nid(v2), nid(v3)], axis=1)
    tets = tets.reshape(-1, 4)
    # orient positively: swap two vertices where the signed volume is negative
    e = xyz[tets[:, 1:]] - xyz[tets[:, :1]]
    det = np.einsum("ti,ti->t", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    neg = det < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    e = xyz[tets[:, 1:]] - xyz[tets[:, :1]]
    det = np.einsum("ti,ti->t", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    if not np.all(det > 0):
        raise ValueError("mesh generation produced a degenerate or inverted tet")
    return Mesh(n=n, xyz=xyz, tets=tets.astype(np.int32), dirichlet=dirichlet)


# ----------------------------------------------------------------------------------
# coefficient fields (per cell, replicated to the 6 tets of the cell)

def kappa_constant(mesh: Mesh, value: float = 1.0) -> np.ndarray:
    return np.full(mesh.n_tets, value, dtype=np.float64)


def kappa_lognormal(mesh: Mesh, sigma: float, seed: int) -> np.ndarray:
    """kappa = exp(sigma * g), g ~ N(0,1) i.i.d. per cell."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(mesh.n ** 3)
    return np.repeat(np.exp(sigma * g), 6)


def kappa_inclusions(mesh: Mesh, seed: int, n_spheres: int = 20, high: float = 1e4,
                     rmin: float = 0.05, rmax: float = 0.15) -> np.ndarray:
    """kappa = 1 with kappa = high in cells whose centroid lies in any sphere."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_spheres, 3))
    radii = rng.uniform(rmin, rmax, size=n_spheres)
    n = mesh.n
    c = (np.arange(n) + 0.5) / n
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    cen = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    inside = np.zeros(n ** 3, dtype=bool)
    for s in range(n_spheres):
        inside |= np.sum((cen - centres[s]) ** 2, axis=1) < radii[s] ** 2
    return np.repeat(np.where(inside, high, 1.0), 6)


def load_polynomial(mesh: Mesh) -> np.ndarray:
    """Nodal values of the scaling-test load of Section 7.1,
    f = 2*sqrt(900)*((1-x)x(1-y)y + (1-x)x(1-z)z + (1-y)y(1-z)z)."""
    x, y, z = mesh.xyz.T
    gx, gy, gz = (1 - x) * x, (1 - y) * y, (1 - z) * z
    return 2.0 * 30.0 * (gx * gy + gx * gz + gy * gz)


def load_sine(mesh: Mesh) -> np.ndarray:
    """Nodal values of f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z)."""
    x, y, z = mesh.xyz.T
    return 3.0 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


# ----------------------------------------------------------------------------------
# box decompositions

def cuts_equal(n: int, parts: int) -> np.ndarray:
    if n % parts:
        raise ValueError("equal cuts need parts | n")
    return np.arange(parts + 1, dtype=np.int64) * (n // parts)


def cuts_random(n: int, parts: int, min_width: int, rng: np.random.Generator) -> np.ndarray:
    """Seeded uneven cuts: widths = min_width + multinomial share of the rest."""
    rest = n - parts * min_width
    if rest < 0:
        raise ValueError("too many parts for the minimum width")
    w = min_width + rng.multinomial(rest, [1.0 / parts] * parts)
    return np.concatenate([[0], np.cumsum(w)]).astype(np.int64)


def cuts_uniform_widths(n: int, wmin: int, wmax: int, rng: np.random.Generator) -> np.ndarray:
    """Widths drawn from U{wmin..wmax} until n is closed (all widths stay in range)."""
    widths = []
    remaining = n
    while remaining > 0:
        if remaining <= wmax:
            w = remaining
        else:
            w = int(rng.integers(wmin, wmax + 1))
            if remaining - w < wmin:
                w = remaining - wmin
        widths.append(w)
        remaining -= w
    return np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)


def box_subdomains(n: int, cuts: tuple, r: int) -> Subdomains:
    """Boxes with one-cell overlap on the + side and extension by r cell layers."""
    ptr = [0]
    ext_all = []
    core_all = []
    boxes = []
    tet6 = np.arange(6, dtype=np.int64)
    for kc in range(len(cuts[2]) - 1):
        for jc in range(len(cuts[1]) - 1):
            for ic in range(len(cuts[0]) - 1):
                core = []
                ext = []
                for ax, a in zip(range(3), (ic, jc, kc)):
                    c = cuts[ax]
                    lo, hi = int(c[a]), int(min(c[a + 1] + 1, n))
                    core.append((lo, hi))
                    ext.append((max(lo - r, 0), min(hi + r, n)))
                ranges = [np.arange(lo, hi) for lo, hi in ext]
                kk, jj, ii = np.meshgrid(ranges[2], ranges[1], ranges[0], indexing="ij")
                ci, cj, ck = ii.ravel(), jj.ravel(), kk.ravel()
                cell = ci + n * (cj + n * ck)
                incore = ((ci >= core[0][0]) & (ci < core[0][1]) &
                          (cj >= core[1][0]) & (cj < core[1][1]) &
                          (ck >= core[2][0]) & (ck < core[2][1]))
                t = (6 * cell[:, None] + tet6[None, :]).ravel()
                ext_all.append(t.astype(np.int32))
                core_all.append(np.repeat(incore, 6).astype(np.uint8))
                ptr.append(ptr[-1] + t.size)
                boxes.append((tuple(core), tuple(ext)))
    return Subdomains(ext_tet_ptr=np.asarray(ptr, dtype=np.int64),
                      ext_tets=np.concatenate(ext_all),
                      in_core=np.concatenate(core_all),
                      boxes=boxes)


# ----------------------------------------------------------------------------------
# general meshes and graph partitions

def kuhn_region(n: int, keep_cell, jitter: float = 0.0, seed: int = 0, shuffle: bool = True) -> Mesh:
    """A tetrahedral mesh of a non-box region: the Kuhn tets of the cells (i, j, k) of the
    n^3 grid with keep_cell(ci, cj, ck) true (arrays in, bool array out), Dirichlet data on
    the whole boundary of the region (nodes of faces used by one tet only), every node off
    that boundary moved by U(-jitter h, +jitter h) per coordinate.  With shuffle, nodes and
    tets are renumbered by seeded random permutations and each tet's vertex list is rotated
    by a seeded even permutation (orientation kept), so that no structured numbering
    survives."""
    full = kuhn_cube(n)
    c = np.arange(n)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    keep = np.asarray(keep_cell(ci.ravel(), cj.ravel(), ck.ravel()), dtype=bool)
    tets = full.tets.reshape(-1, 6, 4)[keep].reshape(-1, 4).astype(np.int64)
    used = np.unique(tets)
    new_id = -np.ones(full.n_nodes, dtype=np.int64)
    new_id[used] = np.arange(used.size)
    tets = new_id[tets]
    xyz = full.xyz[used].copy()
    faces = np.sort(tets[:, [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]].reshape(-1, 3), axis=1)
    uniq, counts = np.unique(faces, axis=0, return_counts=True)
    dirichlet = np.zeros(used.size, dtype=np.uint8)
    dirichlet[np.unique(uniq[counts == 1])] = 1
    rng = np.random.default_rng(seed)
    if jitter > 0.0:
        d = rng.uniform(-jitter / n, jitter / n, size=xyz.shape)
        xyz = xyz + np.where(dirichlet[:, None] == 0, d, 0.0)
    if shuffle:
        perm = rng.permutation(used.size)            # old id -> new id
        xyz_new = np.empty_like(xyz)
        xyz_new[perm] = xyz
        dir_new = np.empty_like(dirichlet)
        dir_new[perm] = dirichlet
        tets = perm[tets][rng.permutation(tets.shape[0])]
        even = np.array([[0, 1, 2, 3], [1, 2, 0, 3], [2, 0, 1, 3], [0, 2, 3, 1], [0, 3, 1, 2], [1, 0, 3, 2],
                         [2, 3, 0, 1], [3, 2, 1, 0], [3, 0, 2, 1], [1, 3, 2, 0], [2, 1, 3, 0], [3, 1, 0, 2]])
        rot = even[rng.integers(0, 12, size=tets.shape[0])]
        tets = np.take_along_axis(tets, rot, axis=1)
        xyz, dirichlet = xyz_new, dir_new
    e = xyz[tets[:, 1:]] - xyz[tets[:, :1]]
    det = np.einsum("ti,ti->t", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    if not np.all(det > 0):
        raise ValueError("region mesh has a degenerate or inverted tet")
    return Mesh(n=n, xyz=xyz, tets=tets.astype(np.int32), dirichlet=dirichlet)


def _node_graph(mesh: Mesh):
    """CSR node adjacency (mesh edges) and node -> tets incidence."""
    t = mesh.tets.astype(np.int64)
    nn = mesh.n_nodes
    a = np.concatenate([t[:, i] for i in range(4) for j in range(4) if i != j])
    b = np.concatenate([t[:, j] for i in range(4) for j in range(4) if i != j])
    key = np.unique(a * nn + b)
    a, b = key // nn, key % nn
    ptr = np.concatenate([[0], np.cumsum(np.bincount(a, minlength=nn))])
    tn = t.ravel()
    order = np.argsort(tn, kind="stable")
    tptr = np.concatenate([[0], np.cumsum(np.bincount(tn, minlength=nn))])
    return ptr, b, tptr, order // 4


def graph_parts(mesh: Mesh, n_parts: int, seed: int) -> np.ndarray:
    """Part id per node: parts grown at once by breadth-first search over the mesh edges from
    n_parts start nodes (each round, every part claims the unclaimed neighbours of its last
    claimed layer), a simple graph partition with connected, compact parts.  The first start
    is a seeded random node; each further start is a node farthest (in edge hops) from the
    starts so far."""
    ptr, adj, _, _ = _node_graph(mesh)
    rng = np.random.default_rng(seed)

    def hops(src):
        d = -np.ones(mesh.n_nodes, dtype=np.int64)
        d[src] = 0
        f = np.asarray(src)
        k = 0
        while f.size:
            k += 1
            nb = np.unique(np.concatenate([adj[ptr[v]:ptr[v + 1]] for v in f]))
            nb = nb[d[nb] < 0]
            d[nb] = k
            f = nb
        return d

    starts = [int(rng.integers(mesh.n_nodes))]
    while len(starts) < n_parts:
        d = hops(starts)
        far = np.flatnonzero(d == d.max())
        starts.append(int(far[rng.integers(far.size)]))
    part = -np.ones(mesh.n_nodes, dtype=np.int64)
    part[starts] = np.arange(n_parts)
    fronts = [np.array([s]) for s in starts]
    while any(f.size for f in fronts):
        for p in range(n_parts):
            f = fronts[p]
            if not f.size:
                continue
            nb = np.unique(np.concatenate([adj[ptr[v]:ptr[v + 1]] for v in f]))
            nb = nb[part[nb] < 0]
            part[nb] = p
            fronts[p] = nb
    return part


def graph_subdomains(mesh: Mesh, part: np.ndarray, r: int, max_rounds: int = 50) -> Subdomains:
    """Subdomains from a node partition (Section 3, the construction next to its decomposition
    figure): omega_i = the tets with at least one node in part i, so neighbouring subdomains share
    one element layer; omega_i^+ = omega_i grown by r element layers (tets sharing a node with the
    previous layer).  A free node interior to two subdomains (every tet around it touches
    both parts) moves to the part whose subdomain surrounds it, until the interiors of the
    omega_i partition the free nodes; raises if max_rounds do not settle it."""
    ptr, adj, tptr, tet_of = _node_graph(mesh)
    t = mesh.tets.astype(np.int64)
    nn, nt = mesh.n_nodes, mesh.n_tets
    n_parts = int(part.max()) + 1
    part = part.copy()
    free = mesh.dirichlet == 0
    star = np.bincount(t.ravel(), minlength=nn)
    for _ in range(max_rounds):
        cores = []
        moved = False
        inner = np.zeros(nn, dtype=np.int64)
        for p in range(n_parts):
            core = np.zeros(nt, dtype=bool)
            core[np.unique(tet_of[np.concatenate([np.arange(tptr[v], tptr[v + 1]) for v in np.flatnonzero(part == p)])])] = True
            cnt = np.bincount(t[core].ravel(), minlength=nn)
            interior = free & (cnt == star)
            inner += interior
            cores.append(core)
            intruders = np.flatnonzero(interior & (part != p))
            if intruders.size:
                part[intruders] = p
                moved = True
                break
        if not moved:
            if np.any(inner[free] != 1):
                raise ValueError("graph decomposition: free nodes not covered exactly once")
            break
    else:
        raise ValueError("graph decomposition did not settle")
    ptr_out = [0]
    ext_all, core_all = [], []
    for p in range(n_parts):
        ext = cores[p].copy()
        for _ in range(r):
            nodes = np.unique(t[ext].ravel())
            grow = np.unique(tet_of[np.concatenate([np.arange(tptr[v], tptr[v + 1]) for v in nodes])])
            ext[grow] = True
        ids = np.flatnonzero(ext)
        ext_all.append(ids.astype(np.int32))
        core_all.append(cores[p][ids].astype(np.uint8))
        ptr_out.append(ptr_out[-1] + ids.size)
    return Subdomains(ext_tet_ptr=np.asarray(ptr_out, dtype=np.int64), ext_tets=np.concatenate(ext_all),
                      in_core=np.concatenate(core_all))


def make_general_problem(n: int = 14, n_parts: int = 6, r: int = 2, rank: int = 6, kappa_sigma: float = 1.0,
                         jitter: float = 0.2, seed: int = 31, name: str = "general") -> Problem:
    """A general mesh and partition: the L-shaped region [0,1]^3 minus the quarter
    x, y > 1/2 with a cubic cavity of n/7 cells near its corner removed, jittered and
    renumbered at random (kuhn_region), lognormal kappa per tet, f = 1, a BFS graph partition
    into n_parts parts and r element layers of extension."""
    h = max(1, n // 7)
    a0 = n // 4

    def keep(ci, cj, ck):
        lshape = ~((ci >= n // 2) & (cj >= n // 2))
        cavity = (ci >= a0) & (ci < a0 + h) & (cj >= a0) & (cj < a0 + h) & (ck >= a0) & (ck < a0 + h)
        return lshape & ~cavity

    mesh = kuhn_region(n, keep, jitter=jitter, seed=seed)
    kap = np.exp(kappa_sigma * np.random.default_rng(seed + 1).standard_normal(mesh.n_tets))
    sd = graph_subdomains(mesh, graph_parts(mesh, n_parts, seed + 2), r)
    return Problem(name=name, mesh=mesh, kappa=kap, f_nodal=None, subdomains=sd, rank=rank, precision="fp64",
                   meta=dict(n=n, r=r, parts=n_parts, region="L-shape with cavity"))


# ----------------------------------------------------------------------------------
# named workloads

def make_problem(n: int, parts=(2, 2, 2), r: int = 1, rank: int = 8, kappa: str = "one",
                 kappa_sigma: float = 1.0, seed: int = 0, jitter: float = 0.0,
                 load: str = "one", cuts=None, precision: str = "fp64", name: str = "custom") -> Problem:
    mesh = kuhn_cube(n, jitter=jitter, seed=seed + 2 if jitter > 0 else None)
    if kappa == "one":
        kap = kappa_constant(mesh)
    elif kappa == "lognormal":
        kap = kappa_lognormal(mesh, kappa_sigma, seed)
    elif kappa == "inclusions":
        kap = kappa_inclusions(mesh, seed)
    else:
        raise ValueError(kappa)
    if load == "one":
        f = None
    elif load == "poly":
        f = load_polynomial(mesh)
    elif load == "sine":
        f = load_sine(mesh)
    else:
        raise ValueError(load)
    if cuts is None:
        cuts = tuple(cuts_equal(n, p) for p in parts)
    sd = box_subdomains(n, cuts, r)
    return Problem(name=name, mesh=mesh, kappa=kap, f_nodal=f, subdomains=sd, rank=rank,
                   precision=precision, meta=dict(n=n, r=r, cuts=[c.tolist() for c in cuts]))


CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5", "C6")


def make_config(name: str) -> Problem:
    """The five named workloads.

    C1  16^3 cells, kappa = 1, f = 1, 2x2x2 equal boxes, r = 1, k = 8, plain FP64.
    C2  48^3, kappa = exp(N(0,1)) per cell (seed 1), 4x4x4 boxes, r = 6, k = 16,
        FP32 block CG with FP64 refinement.
    C3  64^3 with node jitter U(+-0.2h) (seed 2), 6x5x4 boxes at seeded random cuts
        (seed 3, min width 4), r = 6, k = 24, FP32.
    C4  96^3, kappa = exp(2 N(0,1)) (seed 4), 8^3 boxes, r = 6, k = 32, BF16 Gram.
    C5  128^3, kappa = 1 with 20 spheres of kappa = 1e4 (seed 5), boxes with widths
        U{10..40} per axis (seed 6), r = 6, ranks U{8..48} per request (seed 8).
    C6  216^3 (10.2 million nodes, 9.9 million free DOFs), kappa = exp(N(0,1)) (seed 10),
        18x18x18 boxes of 12 cells (5 832 subdomains), r = 6, k = 16: the scale of the
        paper's larger scaling cases (Table 2) on one device.
    """
    if name == "C1":
        return make_problem(16, (2, 2, 2), r=1, rank=8, name="C1", precision="fp64")
    if name == "C2":
        p = make_problem(48, (4, 4, 4), r=6, rank=16, kappa="lognormal", kappa_sigma=1.0, seed=1,
                         name="C2", precision="fp32_refine")
        return p
    if name == "C3":
        rng = np.random.default_rng(3)
        cuts = tuple(cuts_random(64, p, 4, rng) for p in (6, 5, 4))
        mesh = kuhn_cube(64, jitter=0.2, seed=2)
        sd = box_subdomains(64, cuts, 6)
        return Problem(name="C3", mesh=mesh, kappa=kappa_constant(mesh), f_nodal=None, subdomains=sd,
                       rank=24, precision="fp32", meta=dict(n=64, r=6, cuts=[c.tolist() for c in cuts]))
    if name == "C4":
        return make_problem(96, (8, 8, 8), r=6, rank=32, kappa="lognormal", kappa_sigma=2.0, seed=4,
                            name="C4", precision="bf16_split")
    if name == "C6":
        return make_problem(216, (18, 18, 18), r=6, rank=16, kappa="lognormal", kappa_sigma=1.0, seed=10,
                            name="C6", precision="fp32_refine")
    if name == "C5":
        mesh = kuhn_cube(128)
        kap = kappa_inclusions(mesh, seed=5)
        rng = np.random.default_rng(6)
        cuts = tuple(cuts_uniform_widths(128, 10, 40, rng) for _ in range(3))
        sd = box_subdomains(128, cuts, 6)
        ranks = np.random.default_rng(8).integers(8, 49, size=sd.n_sub)
        return Problem(name="C5", mesh=mesh, kappa=kap, f_nodal=None, subdomains=sd, rank=int(ranks.max()),
                       ranks=ranks, precision="mixed", meta=dict(n=128, r=6, cuts=[c.tolist() for c in cuts]))
    raise ValueError(name)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea and Flood 2014) on uint64 arrays, wrapping."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def sketch_rows(n_nodes: int, node_ids: np.ndarray, cols: int, sub: int, seed: int = 13) -> np.ndarray:
    """Standard Gaussian random matrix for the randomized local reduction of subdomain `sub`:
    one row per node id in `node_ids` (the subdomain's interface nodes, in the caller's
    order), `cols` columns.  Entry (node, j) depends only on (seed, sub, global node id, j): two
    SplitMix64 draws keyed by them feed a Box-Muller transform, so every consumer that lists the
    same nodes gets the same matrix, a narrower sketch is the leading columns of a wider one, and
    only the listed rows are generated.  (n_nodes bounds the ids.)"""
    ids = np.asarray(node_ids, dtype=np.int64)
    if ids.size and (ids.min() < 0 or ids.max() >= n_nodes):
        raise ValueError("node id out of range")
    key = _splitmix64(_splitmix64(np.uint64(seed)) ^ np.uint64(sub))
    row = _splitmix64(key ^ ids.astype(np.uint64))[:, None]
    j = np.arange(cols, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        b1 = _splitmix64(row + np.uint64(2) * j)
        b2 = _splitmix64(row + np.uint64(2) * j + np.uint64(1))
    u1 = ((b1 >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53   # (0, 1)
    u2 = (b2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.ascontiguousarray(np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))


def poisson_arrivals(n_requests: int, rate: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
