"""The randomized local reduction (Section 6, two left solves, with the weights applied by K^+
solves: the sketch S_B^-1 S_i and B B^T = W S_B^-1 W^T) on the GPU against the oracle's route of
the same reading with the same random matrices S_i (seeded, from the input generators): k_eff
exact, singular values, q_0, the span of the modes in the K_i inner product, and the reduced
solution in the global energy norm.  Every solve carries l or l + 1 right-hand sides."""
import sys

import numpy as np
import pytest

import workloads as w
from oracle import decomp as odecomp
from oracle import project as oproj
from oracle import reduce as oreduce

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(sigma=1e-9, angle=1e-7, energy=1e-9), "fp32_refine": dict(sigma=1e-7, angle=1e-5, energy=1e-6)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sin_angle(Q1, Q2, K):
    import scipy.linalg as la
    KQ2 = K @ Q2
    L1 = np.linalg.cholesky(Q1.T @ (K @ Q1))
    L2 = np.linalg.cholesky(Q2.T @ KQ2)
    M = la.solve_triangular(L1, la.solve_triangular(L2, (Q1.T @ KQ2).T, lower=True).T, lower=True)
    c = np.linalg.svd(M, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(c.min(), 1.0) ** 2)))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("l", [24, 64])
def test_sketched_matches_oracle(precision, l):
    import torch
    from paper_2404_06260_amd import mor
    p = w.make_problem(12, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=3, name="sketch")
    n = p.subdomains.n_sub
    sets = [odecomp.local_sets(p.mesh, p.subdomains, i) for i in range(n)]
    oms = [w.sketch_rows(p.mesh.n_nodes, s.B, l, i) for i, s in enumerate(sets)]
    res = oreduce.reduce_all(p, rank=p.rank, workers=4, sketches=oms, sketch_solves=True)
    At, bt, _ = oproj.reduced_system(p.mesh, p.kappa, p.subdomains, res)
    x = oproj.solve_reduced(At, bt)
    ut = oproj.reconstruct(p.mesh, res, x)
    torch.cuda.set_device(0)
    tol = TOL[precision]
    kw = dict(refine_rtol=1e-11) if precision == "fp64" else {}
    m = mor.Mor(p, precision=precision, **kw)
    try:
        for i in range(n):   # the library's interface order is the oracle's (ascending global id)
            nP, nV, nI, nB = mor.mor_get_sizes(m.ctx, i)
            np.testing.assert_array_equal(mor.mor_get_nodes(m.ctx, i)[nI:nI + nB], sets[i].B)
        _say(f"[gpu] sketched l={l} {precision}")
        k = mor.mor_local_basis_sketched(m.ctx, np.arange(n), np.full(n, p.rank), oms)
        np.testing.assert_array_equal(k, [r.k_eff for r in res])
        for i, r in enumerate(res):
            sig = mor.mor_get_sigma(m.ctx, i)
            ns = min(sig.size, r.k_eff + 1)
            np.testing.assert_allclose(sig[:ns], r.sigma[:ns], rtol=tol["sigma"], err_msg=f"subdomain {i}")
            nP, nV, nI, nB = mor.mor_get_sizes(m.ctx, i)
            Vs = mor.mor_get_basis(m.ctx, i)[np.argsort(mor.mor_get_nodes(m.ctx, i)[:nV])]
            np.testing.assert_allclose(Vs[:, 0], r.q0, rtol=0, atol=10 * tol["angle"] * np.abs(r.q0).max())
            lm = oreduce.local_matrices(p.mesh, p.kappa, p.f_nodal, r.sets)
            ang = _sin_angle(Vs[:, 1:], r.Phi, lm.K_i.tocsr())
            assert ang < tol["angle"], (i, ang)
        m.project()
        u, nred = m.solve()
        from oracle import fem
        A, _, free, _ = fem.global_system(p.mesh, p.kappa, p.f_nodal)
        d = (u - ut)[free]
        rel = np.sqrt(d @ (A @ d)) / np.sqrt(ut[free] @ (A @ ut[free]))
        _say(f"[gpu] sketched l={l} {precision}: k_eff {k.tolist()}, energy rel {rel:.3e}")
        assert rel < tol["energy"], rel
    finally:
        m.close()


def test_sketched_rejects_plain_fp32_and_wide_sketches():
    from paper_2404_06260_amd import mor
    p = w.make_problem(8, (2, 1, 1), r=1, rank=3, name="tiny")
    m = mor.Mor(p, precision="fp32")
    try:
        nB = mor.mor_get_sizes(m.ctx, 0)[3]
        with pytest.raises(mor.MorError):
            mor.mor_local_basis_sketched(m.ctx, [0], [3], [np.zeros((nB, 8))])
    finally:
        m.close()
    m = mor.Mor(p, precision="fp32_refine")
    try:
        nB = mor.mor_get_sizes(m.ctx, 0)[3]
        with pytest.raises(mor.MorError):
            mor.mor_local_basis_sketched(m.ctx, [0], [3], [np.zeros((nB, 65))])
    finally:
        m.close()


def test_sketched_at_the_papers_sketch_size():
    """Each subdomain with its own sketch of l_i = floor(M_i / 8) columns (the size the paper's
    scaling runs use), requests grouped by l_i, FP32 CG with FP64 refinement, against the
    oracle's route with the same S_i."""
    import torch
    from paper_2404_06260_amd import mor
    p = w.make_problem(12, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=3, name="sketch")
    n = p.subdomains.n_sub
    sets = [odecomp.local_sets(p.mesh, p.subdomains, i) for i in range(n)]
    ls = [s.B.size // 8 for s in sets]
    assert min(ls) >= 16 and max(ls) <= 64, ls
    torch.cuda.set_device(0)
    tol = TOL["fp32_refine"]
    m = mor.Mor(p, precision="fp32_refine")
    try:
        for l in sorted(set(ls)):
            ids = [i for i in range(n) if ls[i] == l]
            oms = [w.sketch_rows(p.mesh.n_nodes, sets[i].B, l, i) for i in ids]
            k = mor.mor_local_basis_sketched(m.ctx, np.array(ids), np.full(len(ids), p.rank), oms)
            for j, i in enumerate(ids):
                r = oreduce.reduce_local_sketched_solves(p.mesh, p.kappa, p.f_nodal, sets[i], p.rank, None, oms[j])
                assert k[j] == r.k_eff, (i, k[j], r.k_eff)
                sig = mor.mor_get_sigma(m.ctx, i)
                ns = min(sig.size, r.k_eff + 1)
                np.testing.assert_allclose(sig[:ns], r.sigma[:ns], rtol=tol["sigma"], err_msg=f"subdomain {i}")
                nV = mor.mor_get_sizes(m.ctx, i)[1]
                Vs = mor.mor_get_basis(m.ctx, i)[np.argsort(mor.mor_get_nodes(m.ctx, i)[:nV])]
                lm = oreduce.local_matrices(p.mesh, p.kappa, p.f_nodal, r.sets)
                ang = _sin_angle(Vs[:, 1:], r.Phi, lm.K_i.tocsr())
                _say(f"[gpu] sketched subdomain {i}: M {sets[i].B.size}, l {l}, k_eff {r.k_eff}, span angle {ang:.2e}")
                assert ang < tol["angle"], (i, ang)
    finally:
        m.close()
