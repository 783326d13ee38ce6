"""Pins of the oracle's global part (Sections 3, 5, 6 and 7.1) against exact statements.

  partition of unity    every free node lies in exactly one P_i; sum_i S_i(v|omega_i) = v
  full rank             with every lifting mode kept, u~ equals the FE solution (Section 3)
  nested spaces         the energy error does not increase with the rank
  projection            the memory-efficient Q^T A Q equals the directly formed product
  Galerkin identity     ||u - u~||_A^2 = u^T b - x^T Q^T b (Section 7.1)
  reduced PCG           the diagonal-preconditioned CG of Section 6 step 3 against exact
                        statements: one step on a diagonal matrix, LAPACK's solution, a
                        monotone A-norm error, recurrence = true residual, invariance under
                        diagonal scaling, and the Cholesky route on a real reduced system;
                        the block-preconditioned variant equals plain CG after the basis update
"""
import numpy as np
import pytest

import workloads as w
from oracle import decomp, fem, project, reduce, solve


def test_partition_of_unity_and_ownership():
    for p in (w.make_config("C1"), w.make_problem(12, (3, 2, 1), r=2)):
        sets = decomp.all_local_sets(p.mesh, p.subdomains)
        owner = decomp.owner_map(p.mesh, sets)
        v = np.random.default_rng(0).standard_normal(p.mesh.n_nodes) * (p.mesh.dirichlet == 0)
        acc = np.zeros_like(v)
        for s in sets:
            acc[s.P] += v[s.P]          # S_i(v|omega_i): keep the interior of omega_i, zero elsewhere
        np.testing.assert_array_equal(acc, v)
        assert np.all(owner[p.mesh.dirichlet == 0] >= 0)
        for s in sets:
            assert np.all(np.isin(s.P, s.V)) and np.all(np.isin(s.V, s.I))


def test_single_layer_overlap():
    """Two cores share either nothing or one element layer (Section 3)."""
    p = w.make_problem(12, (3, 3, 2), r=2)
    sd = p.subdomains
    for i in range(sd.n_sub):
        (ci, _) = sd.boxes[i]
        for j in range(i + 1, sd.n_sub):
            (cj, _) = sd.boxes[j]
            widths = [min(a[1], b[1]) - max(a[0], b[0]) for a, b in zip(ci, cj)]
            if min(widths) > 0:
                assert sorted(widths)[0] == 1


def test_full_rank_reproduces_fe_solution():
    p = w.make_problem(8, (2, 2, 2), r=1, rank=10 ** 6, kappa="lognormal", seed=9)
    out = solve.run(p, rank=10 ** 6, pinv_rtol=1e-13)
    assert all(r.k_eff == r.sets.B.size for r in out["results"])
    rel = out["red_err"] / out["u_energy"]
    assert rel < 1e-9, rel
    np.testing.assert_allclose(out["u_tilde"], out["u_fe"], atol=1e-9 * np.abs(out["u_fe"]).max())


def test_full_rank_reproduces_fe_solution_on_a_general_mesh():
    """The same statement on a non-box region (L-shape with a cavity) with shuffled numbering
    and a graph partition: the method does not depend on boxes."""
    p = w.make_general_problem(n=10, n_parts=4, r=1, seed=41)
    sets = decomp.all_local_sets(p.mesh, p.subdomains)
    decomp.owner_map(p.mesh, sets)                  # the interiors partition the free nodes
    out = solve.run(p, rank=10 ** 6, pinv_rtol=1e-13)
    assert all(r.k_eff == r.sets.B.size for r in out["results"])
    rel = out["red_err"] / out["u_energy"]
    assert rel < 1e-9, rel


def test_error_monotone_in_rank():
    p = w.make_problem(12, (2, 2, 2), r=2, kappa="lognormal", seed=4)
    errs = []
    for k in (1, 2, 4, 8, 16, 32):
        out = solve.run(p, rank=k)
        errs.append(out["red_err"])
    assert all(e2 <= e1 * (1 + 1e-10) for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.05 * errs[0]


@pytest.mark.parametrize("cfg", ["C1", "lognormal-uneven"])
def test_memory_efficient_projection_equals_dense(cfg):
    if cfg == "C1":
        p = w.make_config("C1")
    else:
        rng = np.random.default_rng(3)
        cuts = tuple(w.cuts_random(12, k, 3, rng) for k in (3, 2, 2))
        p = w.make_problem(12, cuts=cuts, r=2, rank=5, kappa="lognormal", seed=2)
    res = reduce.reduce_all(p, workers=1)
    At, bt, off = project.reduced_system(p.mesh, p.kappa, p.subdomains, res)
    D, _ = project.dense_QtAQ(p.mesh, p.kappa, res)
    np.testing.assert_allclose(At, D, atol=1e-12 * np.abs(D).max())
    np.linalg.cholesky(At)                       # SPD when Q has full column rank


def test_galerkin_error_identity():
    p = w.make_problem(12, (2, 2, 2), r=2, rank=4, kappa="lognormal", seed=8, load="poly")
    out = solve.run(p)
    u = out["u_fe"][out["free"]]
    lhs = out["red_err"] ** 2
    rhs = u @ out["b"] - out["x"] @ out["bt"]
    assert abs(lhs - rhs) < 1e-10 * (u @ out["b"])


# --------------------------------------------------------------------------------------
# the basis update of Section 6, step 2 (reading: whitening of the stitched diagonal block)

def _results(p, **kw):
    from oracle import reduce as oreduce
    return oreduce.reduce_all(p, workers=1, **kw)


def test_basis_update_without_drops_keeps_the_galerkin_solution():
    """With nothing dropped the updated basis spans the same space, so the Galerkin solution
    u~ is unchanged, while every diagonal block Q_i^T A_ii Q_i (recomputed here from the
    updated stitched basis and A) is the identity."""
    from oracle import reduce as oreduce
    p = w.make_problem(10, (2, 2, 1), r=2, rank=4, kappa="lognormal", seed=3, name="upd")
    res = _results(p)
    upd = [oreduce.basis_update(r, drop=0.0) for r in res]
    A, b, free, gmap = fem.global_system(p.mesh, p.kappa, p.f_nodal)
    for r in upd:
        P = gmap[r.sets.P]
        Aii = r.Vloc.T @ (A[P][:, P] @ r.Vloc)
        np.testing.assert_allclose(Aii, np.eye(Aii.shape[0]), atol=1e-10)
        np.testing.assert_allclose(r.bi, r.Vloc.T @ b[P], rtol=1e-10, atol=1e-14)
    outs = []
    for rr in (res, upd):
        At, bt, _ = project.reduced_system(p.mesh, p.kappa, p.subdomains, rr)
        outs.append(project.reconstruct(p.mesh, rr, project.solve_reduced(At, bt)))
    np.testing.assert_allclose(outs[1], outs[0], rtol=0, atol=1e-10 * np.abs(outs[0]).max())


def test_basis_update_removes_dependent_columns_of_many_mode_bases():
    """Keeping many modes (tolerance far below the spectrum) makes stitched columns nearly
    dependent: the plain reduced matrix is then numerically singular.  After the update (drop
    1e-10) it is the identity on the diagonal blocks and positive definite, and its solution
    matches the eigenvalue-truncated (pseudo-inverse) solution of the plain system."""
    from oracle import reduce as oreduce
    p = w.make_problem(10, (2, 2, 1), r=2, rank=4, kappa="lognormal", seed=3, name="upd")
    res = _results(p, rank=None, tol=1e-6)
    upd = [oreduce.basis_update(r, drop=1e-10) for r in res]
    assert sum(r.Vloc.shape[1] for r in upd) < sum(r.Vloc.shape[1] for r in res)
    At0, bt0, _ = project.reduced_system(p.mesh, p.kappa, p.subdomains, res)
    At1, bt1, _ = project.reduced_system(p.mesh, p.kappa, p.subdomains, upd)
    np.linalg.cholesky(At1)
    u1 = project.reconstruct(p.mesh, upd, project.solve_reduced(At1, bt1))
    u0 = project.reconstruct(p.mesh, res, project.solve_reduced(At0, bt0, pinv_rtol=1e-12))
    A, _, free, _ = fem.global_system(p.mesh, p.kappa, p.f_nodal)
    d = (u1 - u0)[free]
    assert np.sqrt(d @ (A @ d)) <= 1e-4 * np.sqrt(u0[free] @ (A @ u0[free]))


# --------------------------------------------------------------------------------------
# the reduced solver of Section 6, step 3: conjugate gradients with a diagonal preconditioner

def _spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (U * lam) @ U.T


def test_pcg_solves_a_diagonal_system_in_one_step():
    d = np.array([3.0, 0.5, 7.0, 2.0, 11.0])
    b = np.array([1.0, -2.0, 0.25, 4.0, 3.0])
    x, it, res = project.pcg_diag(np.diag(d), b, rtol=1e-14)
    assert it == 1 and res < 1e-15
    np.testing.assert_allclose(x, b / d, rtol=1e-15)


def test_pcg_matches_lapack_with_monotone_energy_error():
    n = 30
    S = np.diag(np.geomspace(0.1, 10.0, n))           # row scaling: the diagonal matters
    A = S @ _spd(n, 1e3, 5) @ S
    b = np.random.default_rng(6).standard_normal(n)
    xs = np.linalg.solve(A, b)
    errs, gaps = [], []

    def seen(k, x, r):
        e = x - xs
        errs.append(float(e @ A @ e))
        gaps.append(float(np.linalg.norm(r - (b - A @ x)) / np.linalg.norm(b)))

    x, it, res = project.pcg_diag(A, b, rtol=1e-12, on_iter=seen)
    assert res <= 1e-12 and it <= 3 * n
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-8 * np.abs(xs).max())
    assert all(e2 <= e1 * (1 + 1e-9) for e1, e2 in zip(errs, errs[1:])), errs
    assert max(gaps) < 1e-10, max(gaps)


def test_pcg_is_invariant_under_diagonal_scaling():
    """Diagonal preconditioning makes CG on A = S B S (B with unit diagonal) the same
    iteration as plain CG on B: the A-norm errors of the iterates agree step by step."""
    n = 24
    B = _spd(n, 50.0, 7)
    dB = np.sqrt(np.diag(B))
    B = B / np.outer(dB, dB)                            # unit diagonal: its own preconditioner is I
    S = np.diag(np.random.default_rng(8).uniform(0.2, 5.0, n))
    A = S @ B @ S
    c = np.random.default_rng(9).standard_normal(n)
    b = S @ c                                           # A x = b  <=>  B (S x) = c
    xa, xb = np.linalg.solve(A, b), np.linalg.solve(B, c)
    ea, eb = [], []
    project.pcg_diag(A, b, rtol=1e-10, on_iter=lambda k, x, r: ea.append(float((x - xa) @ A @ (x - xa))))
    project.pcg_diag(B, c, rtol=1e-10, on_iter=lambda k, x, r: eb.append(float((x - xb) @ B @ (x - xb))))
    m = min(len(ea), len(eb), 12)
    np.testing.assert_allclose(ea[:m], eb[:m], rtol=1e-6)


def test_pcg_on_a_reduced_system_matches_cholesky():
    p = w.make_problem(10, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=12)
    res = reduce.reduce_all(p, workers=1)
    At, bt, _ = project.reduced_system(p.mesh, p.kappa, p.subdomains, res)
    xc = project.solve_reduced(At, bt)
    x, it, rel = project.pcg_diag(At, bt, rtol=1e-13)
    assert rel <= 1e-13 and 0 < it < At.shape[0] + 50
    np.testing.assert_allclose(x, xc, rtol=0, atol=1e-9 * np.abs(xc).max())
    np.testing.assert_allclose(x @ bt, xc @ bt, rtol=1e-12)


def test_pcg_rejects_an_indefinite_matrix():
    with pytest.raises(np.linalg.LinAlgError):
        project.pcg_diag(np.diag([2.0, -1.0]), np.array([1.0, 1.0]))


def test_block_pcg_solves_a_block_diagonal_system_in_one_step():
    rng = np.random.default_rng(3)
    blocks = [_spd(k, 30.0, 10 + k) for k in (3, 5, 2)]
    A = np.zeros((10, 10))
    off = [0, 3, 8, 10]
    for (a, b), B in zip(zip(off[:-1], off[1:]), blocks):
        A[a:b, a:b] = B
    bvec = rng.standard_normal(10)
    x, it, res = project.pcg_block(A, bvec, off, rtol=1e-13)
    assert it == 1 and res < 1e-13
    np.testing.assert_allclose(x, np.linalg.solve(A, bvec), rtol=1e-12)


def test_block_pcg_equals_plain_cg_after_the_basis_update():
    """Block-inverse PCG on Q^T A Q and plain CG on the reduced system of the updated bases
    (diagonal blocks = I, so the diagonal preconditioner is the identity) are one iteration in
    exact arithmetic: same iteration count (to one) and the same energy x^T b~."""
    drop = 1e-10
    p = w.make_problem(10, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=12)
    res = reduce.reduce_all(p, workers=1)
    At, bt, off = project.reduced_system(p.mesh, p.kappa, p.subdomains, res)
    upd = [reduce.basis_update(r, drop=drop) for r in res]
    Au, bu, _ = project.reduced_system(p.mesh, p.kappa, p.subdomains, upd)
    np.testing.assert_allclose(np.diag(Au), 1.0, rtol=1e-9)
    xb, itb, _ = project.pcg_block(At, bt, off, drop=drop, rtol=1e-12)
    xu, itu, _ = project.pcg_diag(Au, bu, rtol=1e-12)
    assert abs(itb - itu) <= 1, (itb, itu)
    np.testing.assert_allclose(xb @ bt, xu @ bu, rtol=1e-10)
    xc = project.solve_reduced(At, bt)
    np.testing.assert_allclose(xb, xc, rtol=0, atol=1e-9 * np.abs(xc).max())


def test_block_pcg_with_dropped_directions_tracks_the_update_then_loses_conjugacy():
    """With directions dropped (singular block pseudo-inverse) the full-space iteration follows
    plain CG on the updated system step by step while the kept residual is well above rounding
    relative to the dropped part, and then loses conjugacy: why the library's block preconditioner
    keeps every positive eigenvalue and dropping is left to the basis update."""
    p = w.make_problem(10, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=12)
    res = reduce.reduce_all(p, workers=1)
    At, bt, off = project.reduced_system(p.mesh, p.kappa, p.subdomains, res)
    upd = [reduce.basis_update(r, drop=1e-3) for r in res]
    Au, bu, _ = project.reduced_system(p.mesh, p.kappa, p.subdomains, upd)
    assert Au.shape[0] < At.shape[0]                 # directions were dropped
    hb, hu = [], []
    project.pcg_block(At, bt, off, drop=1e-3, rtol=1e-9, on_iter=lambda k, x, r: hb.append(x @ bt))
    project.pcg_diag(Au, bu, rtol=1e-9, on_iter=lambda k, x, r: hu.append(x @ bu))
    m = min(len(hb), len(hu))
    np.testing.assert_allclose(hb[:m], hu[:m], rtol=1e-9)
