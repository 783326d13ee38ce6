"""Local reduction on one subdomain, in float64 (test infrastructure, see package docstring).

Steps, in the paper's order (Section 6, step 2, built on Sections 3 and 4):
  1. assemble the stiffness A_i^+ on omega_i^+ and split it into the I/B blocks;
  2. solve the zero-boundary load problem (Problem 3.2) for q_0 and the lifting
     problems (Problem 3.3) for every interface basis function: the matrix of the
     lifting operator Z_i = C_i (A_II^+)^{-1} A_IB^+ (Section 4), taken with the
     minus sign of the true harmonic extension (the paper drops it; the sign changes
     neither the singular values nor the spans);
  3. the weights: R_i = Cholesky factor of the H1 matrix on omega_i (Section 4) and
     R_BB = Cholesky factor of the Schur complement of the H1 matrix on omega_i^+
     onto B (Lemmas 4.1 and 4.2);
  4. the SVD  R_i Z_i R_BB^{-1} = U Lambda V^T  (eq. 4.4 of Section 4) and the
     truncation to the leading singular triplets (eq. 4.5);
  5. the basis R_i^{-1} U_k, then D_i restricts it to the interior of omega_i
     (the stitching, Definition 3.1), together with q_0;
  6. the local projected block Q_i^T A_ii Q_i and load Q_i^T f_i (Section 6, step 2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as la
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import decomp, fem

CLUSTER_GAP = 1e-4


@dataclass
class LocalMatrices:
    sets: decomp.LocalSets
    A_plus: sp.csr_matrix   # stiffness (kappa) on [I, B]
    K_plus: sp.csr_matrix   # H1 matrix (unweighted stiffness + mass) on [I, B]
    f_plus: np.ndarray      # load on [I, B]
    K_i: sp.csr_matrix      # H1 matrix on omega_i over V
    nI: int
    nB: int
    C_idx: np.ndarray       # positions of V inside I (the restriction C_i)
    D_idx: np.ndarray       # positions of P inside V (the restriction D_i)


@dataclass
class LocalResult:
    sets: decomp.LocalSets
    sigma: np.ndarray       # singular values of R_i Z_i R_BB^{-1}, descending
    k_eff: int              # number of lifting modes kept
    q0: np.ndarray          # (|V|,) zero-boundary load solution restricted to omega_i
    Phi: np.ndarray         # (|V|, k_eff) = R_i^{-1} U_k: H1(omega_i)-orthonormal lifting modes
    Vloc: np.ndarray        # (|P|, k_eff+1) stitched basis D_i [q0, Phi]
    Aii: np.ndarray         # (k_eff+1, k_eff+1) = Vloc^T A_PP Vloc
    bi: np.ndarray          # (k_eff+1,) = Vloc^T f_P


def local_matrices(mesh, kappa, f_nodal, sets: decomp.LocalSets) -> LocalMatrices:
    L = np.concatenate([sets.I, sets.B])
    lmap = -np.ones(mesh.n_nodes, dtype=np.int64)
    lmap[L] = np.arange(L.size)
    ext = mesh.tets[sets.ext_tets]
    Ke, G, Me = fem.element_matrices(mesh.xyz, ext, kappa[sets.ext_tets])
    A_plus = fem.assemble(Ke, ext, lmap, L.size)
    K_plus = fem.assemble(G + Me, ext, lmap, L.size)
    f_plus = fem.load_vector(Me, ext, f_nodal, mesh.n_nodes, lmap, L.size)
    vmap = -np.ones(mesh.n_nodes, dtype=np.int64)
    vmap[sets.V] = np.arange(sets.V.size)
    core = mesh.tets[sets.core_tets]
    _, Gc, Mc = fem.element_matrices(mesh.xyz, core, kappa[sets.core_tets])
    K_i = fem.assemble(Gc + Mc, core, vmap, sets.V.size)
    C_idx = np.searchsorted(sets.I, sets.V)
    if not np.array_equal(sets.I[C_idx], sets.V):
        raise ValueError("omega_i is not inside the interior of omega_i^+ (need r >= 1)")
    D_idx = np.searchsorted(sets.V, sets.P)
    return LocalMatrices(sets=sets, A_plus=A_plus, K_plus=K_plus, f_plus=f_plus, K_i=K_i,
                         nI=sets.I.size, nB=sets.B.size, C_idx=C_idx, D_idx=D_idx)


def blocks(Mat: sp.csr_matrix, nI: int):
    return Mat[:nI, :nI].tocsc(), Mat[:nI, nI:], Mat[nI:, :nI], Mat[nI:, nI:]


def lifting(lm: LocalMatrices):
    """Solve A_II X = [-A_IB, f_I] (Problems 3.2-3.3): columns 0..M-1 lift the interface
    hat functions, column M is the zero-boundary load solution."""
    A_II, A_IB, _, _ = blocks(lm.A_plus, lm.nI)
    rhs = np.hstack([-A_IB.toarray(), lm.f_plus[:lm.nI, None]])
    lu = spla.splu(A_II)
    return lu.solve(rhs)


def schur_H1(lm: LocalMatrices) -> np.ndarray:
    """Schur complement K_BB - K_BI K_II^{-1} K_IB of the H1 matrix on omega_i^+ (Lemma 4.1)."""
    K_II, K_IB, K_BI, K_BB = blocks(lm.K_plus, lm.nI)
    lu = spla.splu(K_II)
    Y = lu.solve(K_IB.toarray())
    S = K_BB.toarray() - K_BI @ Y
    return 0.5 * (S + S.T)


def truncation_rank(sigma: np.ndarray, rank: int | None, tol: float | None, gap: float = CLUSTER_GAP) -> int:
    """Number of leading singular triplets kept.

    rank > 0: the top-`rank`, widened to the end of a cluster of (numerically)
    equal singular values so that the kept subspace is well defined: the smallest
    k' >= rank with (s_k' - s_{k'+1}) / s_k' > gap.  Otherwise keep s > tol
    (eq. 4.5), widened the same way.
    """
    M = sigma.size
    if rank is not None and rank > 0:
        k = min(rank, M)
    else:
        if tol is None:
            raise ValueError("need rank > 0 or a tolerance")
        k = int(np.count_nonzero(sigma > tol))
    if k == 0:
        return 0
    while k < M:
        if sigma[k - 1] <= 0.0 or (sigma[k - 1] - sigma[k]) / sigma[k - 1] > gap:
            break
        k += 1
    return k


def reduce_local(mesh, kappa, f_nodal, sets: decomp.LocalSets, rank: int | None, tol: float | None = None,
                 keep: bool = False):
    lm = local_matrices(mesh, kappa, f_nodal, sets)
    M = lm.nB
    X = lifting(lm)
    Z = X[lm.C_idx, :M]                     # lifting matrix on V
    q0 = X[lm.C_idx, M]
    S_B = schur_H1(lm)
    R_BB = la.cholesky(S_B, lower=False)    # S_B = R_BB^T R_BB
    R_i = la.cholesky(lm.K_i.toarray(), lower=False)
    # R_i Z R_BB^{-1}:  (Z R_BB^{-1})^T = R_BB^{-T} Z^T
    ZRinv = la.solve_triangular(R_BB, Z.T, trans="T", lower=False).T
    Bw = R_i @ ZRinv
    U, s, _ = la.svd(Bw, full_matrices=False)
    k = truncation_rank(s, rank, tol)
    Phi = la.solve_triangular(R_i, U[:, :k], lower=False)
    res = _stitch_and_project(lm, sets, s, k, q0, Phi)
    if keep:
        return res, dict(lm=lm, X=X, Z=Z, S_B=S_B, R_BB=R_BB, R_i=R_i, Bw=Bw, U=U)
    return res


def reduce_local_implicit(mesh, kappa, f_nodal, sets: decomp.LocalSets, rank: int | None, tol: float | None = None,
                          eig_tol: float = 1e-13, keep: bool = False):
    """The same local reduction as `reduce_local`, for subdomains whose dense matrices do not fit
    (tens of thousands of interior and thousands of interface nodes): nothing of size
    |I| x M_i or |V_i| x |V_i| is formed.

    The leading singular triplets of R_i Z_i R_BB^{-1} (eq. 4.4) are the leading eigenpairs of
    the pencil

        (Z_i^T K_i Z_i) beta = sigma^2 S_B beta,   S_B = R_BB^T R_BB (Lemma 4.1),

    because R_i^T R_i = K_i: with v = R_BB beta, (R_i Z_i R_BB^{-1})^T (R_i Z_i R_BB^{-1}) v =
    sigma^2 v.  For beta normalised to beta^T S_B beta = 1 the basis function is
    q = R_i^{-1} u = Z_i beta / sigma (eq. 4.5 and the end of Section 4).  ARPACK's Lanczos
    iteration (scipy's eigsh, generalised mode) finds the leading eigenpairs from products
    with the pencil's matrices, each made of sparse solves with SuperLU factors:
      Z_i x   = -C_i A_II^{-1} A_IB x                       (the lifting, Problem 3.3)
      Z_i^T y = -A_BI A_II^{-1} C_i^T y                     (A_II is symmetric)
      S_B x   = K_BB x - K_BI K_II^{-1} K_IB x              (the Schur complement)
      S_B^{-1} y = [(K^+)^{-1} (0, y)]_B                    (the inverse of a Schur complement is
                                                             the B block of the inverse)
    More eigenpairs than the truncation reads are computed, doubling until the truncation rule
    (top-`rank` widened over a cluster, or sigma > tol) ends strictly inside the computed set.
    sigma holds the computed leading singular values only."""
    lm = local_matrices(mesh, kappa, f_nodal, sets)
    M = lm.nB
    A_II, A_IB, A_BI, _ = blocks(lm.A_plus, lm.nI)
    K_II, K_IB, K_BI, K_BB = blocks(lm.K_plus, lm.nI)
    luA = spla.splu(A_II)
    luK = spla.splu(K_II)
    luKp = spla.splu(lm.K_plus.tocsc())
    C = lm.C_idx
    K_i = lm.K_i.tocsr()

    def Z(x):                                 # V x (..) from B x (..)
        return -luA.solve(np.asarray(A_IB @ x))[C]

    def Zt(y):
        w = np.zeros((lm.nI,) + y.shape[1:])
        w[C] = y
        return -(A_BI @ luA.solve(w))

    def G(x):                                 # Z^T K_i Z
        return Zt(K_i @ Z(x))

    def SB(x):
        return K_BB @ x - K_BI @ luK.solve(np.asarray(K_IB @ x))

    def SBinv(y):
        w = np.zeros((lm.nI + M,) + y.shape[1:])
        w[lm.nI:] = y
        return luKp.solve(w)[lm.nI:]

    def op(f):
        return spla.LinearOperator((M, M), matvec=lambda x: f(x.reshape(M)), matmat=f, dtype=np.float64)

    want = rank if (rank is not None and rank > 0) else 8
    nev = min(M - 1, want + 8)
    while True:
        lam, beta = spla.eigsh(op(G), k=nev, M=op(SB), Minv=op(SBinv), which="LA", tol=eig_tol,
                               v0=np.ones(M))
        order = np.argsort(lam)[::-1]
        lam, beta = lam[order], beta[:, order]
        s = np.sqrt(np.maximum(lam, 0.0))
        k = truncation_rank(s, rank, tol)
        if k < nev or nev >= M - 1:
            break
        nev = min(M - 1, 2 * nev)
    beta = beta[:, :k] / np.sqrt(np.einsum("ij,ij->j", beta[:, :k], SB(beta[:, :k])))
    Phi = Z(beta) / s[:k]
    q0 = luA.solve(lm.f_plus[:lm.nI])[C]
    res = _stitch_and_project(lm, sets, s, k, q0, Phi)
    if keep:
        return res, dict(lm=lm, beta=beta, lam=lam)
    return res


def _stitch_and_project(lm: LocalMatrices, sets, sigma, k, q0, Phi) -> LocalResult:
    """Steps 5-6: V_i = D_i [q0, Phi] and the local projected block and load."""
    Vfull = np.hstack([q0[:, None], Phi])
    Vloc = Vfull[lm.D_idx]
    # A restricted to P: P lies in I and every star of a P node lies in omega_i^+
    P_in_I = lm.C_idx[lm.D_idx]
    A_PP = lm.A_plus[P_in_I][:, P_in_I]
    Aii = Vloc.T @ (A_PP @ Vloc)
    Aii = 0.5 * (Aii + Aii.T)
    bi = Vloc.T @ lm.f_plus[P_in_I]
    return LocalResult(sets=sets, sigma=sigma, k_eff=k, q0=q0, Phi=Phi, Vloc=Vloc, Aii=Aii, bi=bi)


def basis_update(res: LocalResult, drop: float = 1e-10) -> LocalResult:
    """Section 6, step 2's update that diagonalises the diagonal block Q_i^T A_ii Q_i of the
    reduced system.  The paper leaves the details to its source code; the reading taken here:
    the eigendecomposition Q_i^T A_ii Q_i = U Lambda U^T of the stitched block, eigenvalues
    below drop * lambda_max removed (numerically dependent stitched columns), and the basis
    Q_i U_r Lambda_r^{-1/2}, whose diagonal block is the identity.  The load becomes
    Lambda_r^{-1/2} U_r^T Q_i^T f.  The span changes only by the dropped directions."""
    lam, U = la.eigh(res.Aii)
    order = np.argsort(lam)[::-1]
    lam, U = lam[order], U[:, order]
    keep = lam > drop * lam[0]
    T = U[:, keep] / np.sqrt(lam[keep])
    return LocalResult(sets=res.sets, sigma=res.sigma, k_eff=res.k_eff, q0=res.q0, Phi=res.Phi,
                       Vloc=res.Vloc @ T, Aii=np.eye(T.shape[1]), bi=T.T @ res.bi)


def reduce_local_sketched(mesh, kappa, f_nodal, sets: decomp.LocalSets, rank: int | None, tol: float | None,
                          omega: np.ndarray, keep: bool = False):
    """The randomized variant of step 2 (Section 6, "Randomized numerical linear algebra").

    omega is the random matrix S_i (M_i x l, rows in the order of B); the method's random
    draws are an input here.  In the paper's order:
      1. sketch: Qhat Rhat = R_i C_i A_II^{-1} A_IB R_BB^{-1} S_i (a QR factorisation; the
         lifting carries the minus sign of the harmonic extension, as in the explicit path);
      2. project the image of the weighted Z_i onto Qhat: B = Qhat^T R_i C_i A_II^{-1} A_IB
         R_BB^{-1}, evaluated by the two left solves (transposes) so that the solves have l
         right-hand sides instead of M_i;
      3. the SVD B = Uhat Sigma V^T, truncated as in the explicit path;
      4. the basis R_i^{-1} Qhat Uhat_k, stitched and projected as in the explicit path.
    q_0 comes from the zero-boundary load problem as before.
    """
    lm = local_matrices(mesh, kappa, f_nodal, sets)
    A_II, A_IB, _, _ = blocks(lm.A_plus, lm.nI)
    lu = spla.splu(A_II)
    S_B = schur_H1(lm)
    R_BB = la.cholesky(S_B, lower=False)
    R_i = la.cholesky(lm.K_i.toarray(), lower=False)
    # 1. sketch and its QR
    T = la.solve_triangular(R_BB, omega, lower=False)             # R_BB^{-1} S_i
    Xs = lu.solve(-(A_IB @ T))                                    # A_II^{-1} (-A_IB) R_BB^{-1} S_i
    Qh, _ = la.qr(R_i @ Xs[lm.C_idx], mode="economic")
    # 2. B = Qhat^T R_i C (A_II^{-1} (-A_IB)) R_BB^{-1} by two left solves
    L = np.zeros((lm.nI, Qh.shape[1]))
    L[lm.C_idx] = R_i.T @ Qh                                      # (Qhat^T R_i C)^T
    G = lu.solve(L, trans="T")                                    # A_II^{-T} (Qhat^T R_i C)^T
    Bt = la.solve_triangular(R_BB, -(A_IB.T @ G), trans="T", lower=False)   # R_BB^{-T} (G^T (-A_IB))^T
    # 3. SVD of the small matrix and truncation
    Uh, s, _ = la.svd(Bt.T, full_matrices=False)
    k = truncation_rank(s, rank, tol)
    # 4. basis, stitching, projection
    Phi = la.solve_triangular(R_i, Qh @ Uh[:, :k], lower=False)
    q0 = lu.solve(lm.f_plus[:lm.nI])[lm.C_idx]
    res = _stitch_and_project(lm, sets, s, k, q0, Phi)
    if keep:
        return res, dict(lm=lm, Qh=Qh, B=Bt.T, R_i=R_i, R_BB=R_BB)
    return res


def reduce_local_sketched_solves(mesh, kappa, f_nodal, sets: decomp.LocalSets, rank: int | None,
                                 tol: float | None, omega: np.ndarray, keep: bool = False):
    """The randomized variant of step 2 (Section 6) with the weights applied through sparse
    solves, so that no solve carries M_i right-hand sides and no M_i x M_i matrix is formed.

    The weight R_BB (Lemma 4.1: S_B = R_BB^T R_BB) enters only as R_BB^{-1} on the right of the
    weighted lifting operator, and the inverse of the Schur complement is the B block of the
    inverse of K^+ (Lemma 4.1 with B ordered last), so S_B^{-1} v = [(K^+)^{-1} [0; v]]_B.
    omega is the random matrix (M_i x l, rows in the order of B), an input here.
      1. sketch: T = S_B^{-1} omega (l solves with K^+), and Qhat Rhat = R_i C A_II^{-1}(-A_IB) T;
         this is the paper's sketch with S_i = R_BB^{-T} omega (R_BB^{-1} S_i = S_B^{-1} omega);
      2. W = Qhat^T R_i C A_II^{-1}(-A_IB) by the left solve (l right-hand sides), as in
         reduce_local_sketched;
      3. B = W R_BB^{-1} has B B^T = W S_B^{-1} W^T, with S_B^{-1} W^T from l more solves with
         K^+; its eigenpairs give sigma^2 and the left singular vectors Uhat of B, which do not
         depend on how S_B is factored;
      4. the truncation and the basis R_i^{-1} Qhat Uhat_k, stitched and projected as in the
         explicit path; q_0 from the zero-boundary load problem.
    """
    lm = local_matrices(mesh, kappa, f_nodal, sets)
    A_II, A_IB, A_BI, _ = blocks(lm.A_plus, lm.nI)
    lu = spla.splu(A_II)
    luK = spla.splu(lm.K_plus.tocsc())
    R_i = la.cholesky(lm.K_i.toarray(), lower=False)

    def sb_inv(V):                                               # S_B^{-1} V, V: M x l
        rhs = np.zeros((lm.nI + lm.nB, V.shape[1]))
        rhs[lm.nI:] = V
        return luK.solve(rhs)[lm.nI:]

    # 1. sketch and its QR
    T = sb_inv(omega)
    Xs = lu.solve(-(A_IB @ T))                                    # A_II^{-1} (-A_IB) T
    Qh, _ = la.qr(R_i @ Xs[lm.C_idx], mode="economic")
    # 2. W^T = (-A_IB)^T A_II^{-T} (Qhat^T R_i C)^T by the left solve
    L = np.zeros((lm.nI, Qh.shape[1]))
    L[lm.C_idx] = R_i.T @ Qh
    G = lu.solve(L, trans="T")
    Wt = -(A_BI @ G)                                              # A_IB^T = A_BI (A^+ symmetric)
    # 3. B B^T = W S_B^{-1} W^T and its eigenpairs (descending)
    BBt = Wt.T @ sb_inv(Wt)
    lam, U = la.eigh(0.5 * (BBt + BBt.T))
    order = np.argsort(lam)[::-1]
    lam, U = lam[order], U[:, order]
    s = np.sqrt(np.maximum(lam, 0.0))
    k = truncation_rank(s, rank, tol)
    # 4. basis, stitching, projection
    Phi = la.solve_triangular(R_i, Qh @ U[:, :k], lower=False)
    q0 = lu.solve(lm.f_plus[:lm.nI])[lm.C_idx]
    res = _stitch_and_project(lm, sets, s, k, q0, Phi)
    if keep:
        return res, dict(lm=lm, Qh=Qh, BBt=BBt, T=T)
    return res


# ----------------------------------------------------------------------------------
# whole-problem driver (serial, or a process pool over subdomains)

_G = {}


def _work(i):
    p, sets, rank, tol = _G["p"], _G["sets"], _G["rank"], _G["tol"]
    r = p.ranks[i] if (p.ranks is not None and rank is None) else rank
    r = int(r) if r is not None else None
    if _G.get("sketches") is not None:
        route = reduce_local_sketched_solves if _G.get("sketch_solves") else reduce_local_sketched
        return route(p.mesh, p.kappa, p.f_nodal, sets[i], r, tol, _G["sketches"][i])
    if _G.get("implicit"):
        return reduce_local_implicit(p.mesh, p.kappa, p.f_nodal, sets[i], r, tol)
    return reduce_local(p.mesh, p.kappa, p.f_nodal, sets[i], r, tol)


def reduce_all(problem, rank: int | None = None, tol: float | None = None, workers: int = 1,
               subset=None, sketches=None, implicit: bool = False, order=None,
               sketch_solves: bool = False) -> list[LocalResult]:
    """Every subdomain's local reduction (explicit; through the pencil's sparse factors when
    `implicit`, for subdomains too large for the dense matrices; the randomized variant when
    `sketches` holds one random matrix per subdomain, with the weights applied by K^+ solves
    when `sketch_solves`).  `order`, if given, is the order in which
    a process pool takes the subdomains up (largest first keeps the pool busy to the end); the
    results are always returned in subdomain order."""
    sets = decomp.all_local_sets(problem.mesh, problem.subdomains)
    if rank is None and tol is None and problem.ranks is None:
        rank = problem.rank
    idx = list(range(problem.subdomains.n_sub)) if subset is None else list(subset)
    _G.update(p=problem, sets=sets, rank=rank, tol=tol, sketches=sketches, implicit=implicit,
              sketch_solves=sketch_solves)
    if workers <= 1:
        return [_work(i) for i in idx]
    import multiprocessing as mp
    run = idx if order is None else [i for i in order if i in set(idx)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        out = dict(zip(run, pool.imap(_work, run, chunksize=1)))
    return [out[i] for i in idx]
