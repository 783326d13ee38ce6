"""Pins of the oracle's local reduction (Sections 3 and 4) by independent routes.

  linear reproduction   P1 harmonic extension of linear data reproduces it exactly
  Lemma 4.1             R_BB read off a dense Cholesky of the whole H1 matrix (B last)
  Lemma 4.2             trace norm = minimum H1 energy over extensions, found by an optimizer
  eq. 4.3               ||Z|| = sigma_1, via a generalized symmetric eigenproblem
  invariance            the kept span does not depend on the order of B or on the route
  Lemma 5.1             local relative error bound per subdomain
"""
import numpy as np
import pytest
import scipy.linalg as la
import scipy.optimize as opt

import workloads as w
from oracle import decomp, reduce, solve


def _interior_problem(jitter=0.0, kappa="one"):
    # 12^3 cells, 3^3 boxes of 4 cells, r = 2: the centre box's extension stays off the boundary
    return w.make_problem(12, (3, 3, 3), r=2, rank=6, jitter=jitter, seed=5, kappa=kappa)


def _centre(p):
    return 13  # box (1,1,1) in x-fastest order


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_lifting_reproduces_linear_interface_data(jitter):
    p = _interior_problem(jitter)
    sets = decomp.local_sets(p.mesh, p.subdomains, _centre(p))
    assert not np.any(p.mesh.dirichlet[np.concatenate([sets.I, sets.B])])
    lm = reduce.local_matrices(p.mesh, p.kappa, p.f_nodal, sets)
    X = reduce.lifting(lm)
    Z = X[lm.C_idx, :lm.nB]
    a = np.array([0.7, -0.2, 1.3])
    g = p.mesh.xyz @ a - 0.25
    np.testing.assert_allclose(Z @ g[sets.B], g[sets.V], atol=1e-12)
    # and the full interior lifting, not only on omega_i
    np.testing.assert_allclose(X[:, :lm.nB] @ g[sets.B], g[sets.I], atol=1e-12)


def _keep(p, i, rank=None):
    sets = decomp.local_sets(p.mesh, p.subdomains, i)
    return reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, sets, rank or p.rank, keep=True)


def test_spd_of_local_matrices():
    p = w.make_config("C1")
    res, d = _keep(p, 0)
    lm = d["lm"]
    nI = lm.nI
    for Mat in (lm.A_plus, lm.K_plus):
        la.cholesky(Mat[:nI, :nI].toarray())
    la.cholesky(d["S_B"])
    G1 = d["Z"].T @ (lm.K_i @ d["Z"])
    ev = la.eigvalsh(0.5 * (G1 + G1.T))
    assert ev.min() > -1e-12 * ev.max()


def test_lemma_4_1_schur_equals_cholesky_block():
    p = w.make_config("C1")
    res, d = _keep(p, 3)
    K = d["lm"].K_plus.toarray()                      # ordered [I, B]
    R = la.cholesky(K, lower=False)
    nI = d["lm"].nI
    R_BB_block = R[nI:, nI:]
    # both are upper Cholesky factors with positive diagonals, hence equal
    np.testing.assert_allclose(R_BB_block, d["R_BB"], atol=1e-11)
    np.testing.assert_allclose(R_BB_block.T @ R_BB_block, d["S_B"], atol=1e-11)


def test_lemma_4_2_trace_norm_is_min_extension_energy():
    p = w.make_problem(8, (2, 2, 2), r=1)
    res, d = _keep(p, 0)
    K = d["lm"].K_plus
    nI = d["lm"].nI
    rng = np.random.default_rng(11)
    for _ in range(3):
        bz = rng.standard_normal(d["lm"].nB)

        def fun(bI):
            v = np.concatenate([bI, bz])
            Kv = K @ v
            return v @ Kv, 2 * Kv[:nI]

        r = opt.minimize(fun, np.zeros(nI), jac=True, method="L-BFGS-B",
                         options=dict(maxiter=20000, ftol=1e-15, gtol=1e-11))
        lemma = np.linalg.norm(d["R_BB"] @ bz) ** 2
        assert abs(r.fun - lemma) < 1e-8 * lemma
        # any other extension has more energy
        v = np.concatenate([r.x + 1e-3 * rng.standard_normal(nI), bz])
        assert v @ (K @ v) > lemma


def test_operator_norm_is_sigma1_and_pencil_route_agrees():
    """eq. 4.3: sup ||R_i Z b|| / ||R_BB b|| = ||R_i Z R_BB^{-1}||_2 = sigma_1; the squared
    singular values are the eigenvalues of the pencil (Z^T K_i Z, S_B)."""
    p = w.make_config("C1")
    res, d = _keep(p, 5)
    Z, K_i, S_B = d["Z"], d["lm"].K_i, d["S_B"]
    G1 = Z.T @ (K_i @ Z)
    lam, Vv = la.eigh(0.5 * (G1 + G1.T), S_B)
    lam, Vv = lam[::-1], Vv[:, ::-1]
    np.testing.assert_allclose(np.sqrt(np.maximum(lam[:20], 0)), res.sigma[:20], rtol=1e-9)
    rng = np.random.default_rng(0)
    for _ in range(20):
        b = rng.standard_normal(S_B.shape[0])
        ratio = np.sqrt(b @ G1 @ b) / np.linalg.norm(d["R_BB"] @ b)
        assert ratio <= res.sigma[0] * (1 + 1e-12)
    # same kept span by the pencil route: q_j = Z v_j / sigma_j
    k = res.k_eff
    Qp = Z @ Vv[:, :k] / np.sqrt(lam[:k])
    _assert_same_span(Qp, res.Phi, K_i.toarray(), 1e-8)


def _assert_same_span(Q1, Q2, K, tol):
    """Largest principal angle between spans, in the K inner product (sin theta)."""
    R = la.cholesky(K, lower=False)
    A1, _ = np.linalg.qr(R @ Q1)
    A2, _ = np.linalg.qr(R @ Q2)
    s = np.linalg.norm(A2 - A1 @ (A1.T @ A2), 2)
    assert s < tol, s


def test_basis_invariant_to_interface_ordering():
    p = w.make_config("C1")
    sets = decomp.local_sets(p.mesh, p.subdomains, 2)
    r1 = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, sets, 8)
    perm = np.random.default_rng(1).permutation(sets.B.size)
    sets2 = decomp.LocalSets(ext_tets=sets.ext_tets, core_tets=sets.core_tets, I=sets.I, B=sets.B[perm],
                             V=sets.V, P=sets.P)
    r2 = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, sets2, 8)
    np.testing.assert_allclose(r1.sigma, r2.sigma, rtol=1e-10, atol=1e-14)
    assert r1.k_eff == r2.k_eff
    lm = reduce.local_matrices(p.mesh, p.kappa, p.f_nodal, sets)
    _assert_same_span(r1.Phi, r2.Phi, lm.K_i.toarray(), 1e-9)
    # H1(omega_i)-orthonormal modes (R_i^{-1} U has K_i-orthonormal columns)
    np.testing.assert_allclose(r1.Phi.T @ (lm.K_i @ r1.Phi), np.eye(r1.k_eff), atol=1e-10)


def test_truncation_rank_cluster_rule():
    s = np.array([1.0, 0.5, 0.5 * (1 - 1e-6), 0.5 * (1 - 2e-6), 0.1, 0.01])
    assert reduce.truncation_rank(s, 1, None) == 1
    assert reduce.truncation_rank(s, 2, None) == 4       # cluster of three equal values
    assert reduce.truncation_rank(s, 5, None) == 5
    assert reduce.truncation_rank(s, 50, None) == 6
    assert reduce.truncation_rank(s, None, 0.2) == 4
    assert reduce.truncation_rank(s, None, 2.0) == 0


def test_lemma_5_1_local_bound():
    """||u - v_i||_{1,omega_i} / ||u||_{1,omega_i^+} < eps = sigma_{k+1} (Lemma 5.1), where
    v_i = q_0 + Z~_i(u on B) and Z~_i = R_i^{-1} U_k U_k^T R_i Z_i is the truncated lifting."""
    p = w.make_problem(12, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=3)
    u, *_ = solve.fe_solution(p.mesh, p.kappa, p.f_nodal)
    for i in range(p.subdomains.n_sub):
        res, d = _keep(p, i, rank=6)
        sets, lm = res.sets, d["lm"]
        k = res.k_eff
        Uk = d["U"][:, :k]
        Zt = la.solve_triangular(d["R_i"], Uk @ (Uk.T @ (d["R_i"] @ d["Z"])), lower=False)
        v = res.q0 + Zt @ u[sets.B]
        e = u[sets.V] - v
        num = np.sqrt(e @ (lm.K_i @ e))
        L = np.concatenate([sets.I, sets.B])
        den = np.sqrt(u[L] @ (lm.K_plus @ u[L]))
        eps = res.sigma[k]
        assert num / den < eps, (i, num / den, eps)


# --------------------------------------------------------------------------------------
# randomized variant (Section 6, "Randomized numerical linear algebra")

def _sketch_case():
    p = w.make_problem(10, (2, 2, 2), r=2, rank=5, kappa="lognormal", seed=3, name="sketch")
    s = decomp.local_sets(p.mesh, p.subdomains, 0)
    return p, s


def test_sketched_variant_with_identity_sketch_is_the_explicit_svd():
    """S_i = I: the sketch spans the whole image, so the projected SVD is the explicit one."""
    p, s = _sketch_case()
    ex = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, s, 5)
    sk = reduce.reduce_local_sketched(p.mesh, p.kappa, p.f_nodal, s, 5, None, np.eye(s.B.size))
    n = min(ex.sigma.size, sk.sigma.size)
    np.testing.assert_allclose(sk.sigma[:n], ex.sigma[:n], rtol=1e-10, atol=1e-14 * ex.sigma[0])
    assert sk.k_eff == ex.k_eff
    np.testing.assert_allclose(sk.q0, ex.q0, rtol=0, atol=1e-12 * np.abs(ex.q0).max())
    # same span (the singular vectors agree up to sign for distinct singular values)
    P = sk.Phi @ np.linalg.lstsq(sk.Phi, ex.Phi, rcond=None)[0]
    assert np.linalg.norm(P - ex.Phi) < 1e-9 * np.linalg.norm(ex.Phi)


def test_full_width_gaussian_sketch_is_exact_and_narrow_sketches_interlace():
    """A Gaussian S_i with M_i columns spans R^M almost surely, so the result is exact; with
    fewer columns the singular values of Qhat^T (weighted Z) are lower bounds of the exact
    ones (Qhat has orthonormal columns), and widening the sketch can only raise them."""
    p, s = _sketch_case()
    M = s.B.size
    ex = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, s, 5)
    full = reduce.reduce_local_sketched(p.mesh, p.kappa, p.f_nodal, s, 5, None,
                                         w.sketch_rows(p.mesh.n_nodes, s.B, M, 0))
    np.testing.assert_allclose(full.sigma[:20], ex.sigma[:20], rtol=1e-8)
    prev = None
    for l in (8, 24, 64):
        om = w.sketch_rows(p.mesh.n_nodes, s.B, 64, 0)[:, :l]
        sk = reduce.reduce_local_sketched(p.mesh, p.kappa, p.f_nodal, s, 5, None, om)
        n = sk.sigma.size
        assert n == l
        assert np.all(sk.sigma <= ex.sigma[:n] * (1 + 1e-10))
        if prev is not None:
            assert np.all(sk.sigma[:prev.size] >= prev * (1 - 1e-10))
        prev = sk.sigma


def _span_residual(A, B):
    """How far the columns of B lie outside span(A), relative to |B|."""
    P = A @ np.linalg.lstsq(A, B, rcond=None)[0]
    return np.linalg.norm(P - B) / np.linalg.norm(B)


def test_solve_route_of_the_sketch_is_the_papers_sketch_of_a_correlated_test_matrix():
    """The route with the weights applied by K^+ solves, driven by omega = R_BB^T S_i, is the
    paper's sketched SVD driven by S_i: S_B^{-1} R_BB^T S_i = R_BB^{-1} S_i with R_BB from a dense
    Cholesky of the explicit Schur complement (Lemma 4.1), and B B^T = W S_B^{-1} W^T has the
    squares of the singular values of B = W R_BB^{-1}."""
    p, s = _sketch_case()
    lm = reduce.local_matrices(p.mesh, p.kappa, p.f_nodal, s)
    R_BB = la.cholesky(reduce.schur_H1(lm), lower=False)
    S = w.sketch_rows(p.mesh.n_nodes, s.B, 24, 0)
    old = reduce.reduce_local_sketched(p.mesh, p.kappa, p.f_nodal, s, 5, None, S)
    new = reduce.reduce_local_sketched_solves(p.mesh, p.kappa, p.f_nodal, s, 5, None, R_BB.T @ S)
    np.testing.assert_allclose(new.sigma, old.sigma, rtol=1e-9, atol=1e-12 * old.sigma[0])
    assert new.k_eff == old.k_eff
    np.testing.assert_allclose(new.q0, old.q0, rtol=0, atol=1e-12 * np.abs(old.q0).max())
    assert _span_residual(new.Phi, old.Phi) < 1e-8


def test_solve_route_is_exact_at_full_width_and_interlaces_below():
    """A Gaussian omega with M_i columns makes T = S_B^{-1} omega span R^M, so the result is the
    explicit SVD; narrower sketches give singular values no larger than the exact ones (Qhat has
    orthonormal columns), nondecreasing as the sketch widens."""
    p, s = _sketch_case()
    M = s.B.size
    ex = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, s, 5)
    om = w.sketch_rows(p.mesh.n_nodes, s.B, M, 1)
    full = reduce.reduce_local_sketched_solves(p.mesh, p.kappa, p.f_nodal, s, 5, None, om)
    np.testing.assert_allclose(full.sigma[:20], ex.sigma[:20], rtol=1e-8)
    assert full.k_eff == ex.k_eff
    assert _span_residual(full.Phi, ex.Phi) < 1e-8
    prev = None
    for l in (8, 24, 64):
        sk = reduce.reduce_local_sketched_solves(p.mesh, p.kappa, p.f_nodal, s, 5, None, om[:, :l])
        assert sk.sigma.size == l
        assert np.all(sk.sigma <= ex.sigma[:l] * (1 + 1e-10))
        if prev is not None:
            assert np.all(sk.sigma[:prev.size] >= prev * (1 - 1e-10))
        prev = sk.sigma


@pytest.mark.parametrize("kappa", ["one", "lognormal"])
def test_rank_of_the_lifting_equals_the_boundary_dofs_of_omega_i(kappa):
    """The spectrum of the weighted lifting operator reaches rounding at the number of interface
    degrees of freedom of omega_i: a discrete harmonic function on omega_i is fixed by its
    values on the free nodes of the boundary of omega_i (V_i minus P_i), so rank Z <= |V_i \\ P_i|,
    and the traces of the liftings reach every such value, so the bound is attained.  The
    gap is clean: the same count above 1e-10 and above 1e-13 of sigma_1."""
    p = w.make_problem(10, (2, 2, 2), r=2, kappa=kappa, seed=5)
    for i in (0, 7):
        s = decomp.local_sets(p.mesh, p.subdomains, i)
        r = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, s, 10 ** 6)
        sg = r.sigma / r.sigma[0]
        nb = s.V.size - s.P.size
        assert s.B.size > nb
        assert (sg > 1e-10).sum() == (sg > 1e-13).sum() == nb, (i, nb)


def _kspan_sin(A, B, K):
    """Largest principal angle (sine) between the spans of two K-orthonormal bases."""
    D = B - A @ (A.T @ (K @ B))
    return float(np.sqrt(max(np.linalg.eigvalsh(D.T @ (K @ D)).max(), 0.0)))


@pytest.mark.parametrize("case", ["lognormal-rank", "lognormal-tol", "inclusions-rank"])
def test_implicit_route_equals_the_dense_svd(case):
    """The large-subdomain route (Lanczos on the pencil (Z^T K_i Z, S_B) through sparse factors,
    S_B^-1 as the B block of (K^+)^-1) against the dense SVD of R_i Z R_BB^-1 (eq. 4.4), which the
    other pins of this file fix: the same k_eff, the leading singular values to 1e-9, the same
    q_0, K_i-orthonormal modes spanning the same space (sine of the largest principal angle below
    1e-8), and the same projected block.  The tolerance case keeps more modes than the first
    Lanczos call computes, so the route has to widen its eigenpair count."""
    if case.startswith("inclusions"):
        p = w.make_problem(16, (2, 2, 2), r=3, rank=24, kappa="inclusions", seed=5)
    else:
        p = w.make_problem(16, (2, 2, 2), r=3, rank=10, kappa="lognormal", kappa_sigma=1.0, seed=5)
    for i in (0, 6):
        sets = decomp.local_sets(p.mesh, p.subdomains, i)
        rank, tol = p.rank, None
        if case.endswith("tol"):     # a tolerance between the 22nd and 23rd singular values
            s = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, sets, 40).sigma
            rank, tol = None, 0.5 * (s[21] + s[22])
        rd = reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, sets, rank, tol)
        ri = reduce.reduce_local_implicit(p.mesh, p.kappa, p.f_nodal, sets, rank, tol)
        k = rd.k_eff
        assert ri.k_eff == k and (tol is None or k >= 22)
        np.testing.assert_allclose(ri.sigma[:k + 1], rd.sigma[:k + 1], rtol=1e-9)
        np.testing.assert_allclose(ri.q0, rd.q0, rtol=0, atol=1e-12 * np.abs(rd.q0).max())
        K = reduce.local_matrices(p.mesh, p.kappa, p.f_nodal, sets).K_i.tocsr()
        np.testing.assert_allclose(ri.Phi.T @ (K @ ri.Phi), np.eye(k), atol=1e-9)
        assert _kspan_sin(rd.Phi, ri.Phi, K) < 1e-8
        np.testing.assert_allclose(ri.Aii[0, 0], rd.Aii[0, 0], rtol=1e-12)
        np.testing.assert_allclose(np.linalg.eigvalsh(ri.Aii), np.linalg.eigvalsh(rd.Aii), rtol=1e-8,
                                   atol=1e-12 * np.abs(rd.Aii).max())
