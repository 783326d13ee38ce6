"""Full-size parity on the 48^3 lognormal workload (64 box subdomains, r = 6, rank 16), in the
launch configuration the benchmark times (FP32 block CG with FP64 refinement, autotuned tiles).

The FP64 oracle's whole-path result for this workload is stored in tests/golden/C2_oracle.npz,
written by tests/golden/make_oracle_reference.py (which calls only the oracle; about an hour on
8 cores).  Compared here:
  - k_eff of every subdomain (exact) and the reduced dimension,
  - the leading singular values of every subdomain (rtol 1e-7),
  - the reduced solution in the global energy norm (relative, 1e-6),
  - the Galerkin identity A~ x = b~ on the GPU's reduced system, and x.b~ against the oracle,
  - two sampled subdomains (a corner and an interior box) recomputed by the oracle one by one:
    q_0 and the span of the lifting modes in the K_i inner product;
  - with the benchmark's reduced solver (conjugate gradients with the diagonal preconditioner
    on the block-sparse reduced matrix): the requested residual 1e-12, an iteration count
    within 10% of the oracle's on its own reduced system (stored beside its result), and the
    oracle's u~ (energy norm, 1e-6) and x.b~.
"""
import os
import sys

import numpy as np
import pytest
import scipy.linalg as la

import workloads as w
from oracle import decomp as odecomp
from oracle import fem as ofem
from oracle import reduce as oreduce

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "C2_oracle.npz")
TOL_ENERGY = 1e-6
TOL_SIGMA = 1e-7
TOL_ANGLE = 1e-5
SAMPLED = (0, 21)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sin_angle(Q1, Q2, K):
    """Largest principal angle between span(Q1) and span(Q2) in the inner product of the sparse
    SPD matrix K, from the K-Gram matrices (no dense factorisation of K)."""
    KQ2 = K @ Q2
    G11 = Q1.T @ (K @ Q1)
    G22 = Q2.T @ KQ2
    G12 = Q1.T @ KQ2
    L1 = np.linalg.cholesky(G11)
    L2 = np.linalg.cholesky(G22)
    M = la.solve_triangular(L1, la.solve_triangular(L2, G12.T, lower=True).T, lower=True)
    c = np.linalg.svd(M, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(c.min(), 1.0) ** 2)))


def test_c2_full_size_parity():
    import torch
    from paper_2404_06260_amd import autotune, mor
    ref = np.load(GOLDEN)
    p = w.make_config("C2")
    torch.cuda.set_device(0)
    tile = autotune.best(p, "fp32_refine") or {}
    _say(f"[gpu] C2 fp32_refine tiles {tile}: local bases")
    m = mor.Mor(p, precision="fp32_refine", **tile)
    try:
        k = m.local_basis_all()
        _say("[gpu] C2: project + solve")
        m.project()
        u, nred = m.solve()
        np.testing.assert_array_equal(k, ref["k_eff"])
        assert nred == ref["x"].size
        for i in range(p.subdomains.n_sub):
            sig = mor.mor_get_sigma(m.ctx, i)
            ns = min(sig.size, int(ref["k_eff"][i]) + 1)
            np.testing.assert_allclose(sig[:ns], ref["sigma"][i, :ns], rtol=TOL_SIGMA, err_msg=f"subdomain {i}")
        At, bt = mor.mor_get_reduced(m.ctx)
        x = mor.mor_get_reduced_solution(m.ctx, nred)
        np.testing.assert_allclose(At @ x, bt, rtol=0, atol=1e-10 * np.abs(bt).max())
        np.testing.assert_allclose(x @ bt, ref["x"] @ ref["bt"], rtol=1e-7)
        A, _, free, _ = ofem.global_system(p.mesh, p.kappa, p.f_nodal)
        d = (u - ref["u_tilde"])[free]
        uo = ref["u_tilde"][free]
        rel = np.sqrt(max(d @ (A @ d), 0.0)) / np.sqrt(uo @ (A @ uo))
        _say(f"[gpu] C2: energy rel {rel:.3e}")
        assert rel < TOL_ENERGY, rel
        for i in SAMPLED:
            s = odecomp.local_sets(p.mesh, p.subdomains, i)
            r = oreduce.reduce_local(p.mesh, p.kappa, p.f_nodal, s, p.rank)
            nP, nV, nI, nB = mor.mor_get_sizes(m.ctx, i)
            nodes = mor.mor_get_nodes(m.ctx, i)[:nV]
            Vs = mor.mor_get_basis(m.ctx, i)[np.argsort(nodes)]
            np.testing.assert_allclose(Vs[:, 0], r.q0, rtol=0, atol=10 * TOL_ANGLE * np.abs(r.q0).max())
            lm = oreduce.local_matrices(p.mesh, p.kappa, p.f_nodal, r.sets)
            ang = _sin_angle(Vs[:, 1:], r.Phi, lm.K_i.tocsr())
            _say(f"[gpu] C2 subdomain {i}: span angle {ang:.2e}")
            assert ang < TOL_ANGLE, (i, ang)
    finally:
        m.close()


def test_c2_full_size_reduced_pcg():
    import torch
    from paper_2404_06260_amd import autotune, mor
    ref = np.load(GOLDEN)
    p = w.make_config("C2")
    torch.cuda.set_device(0)
    tile = autotune.best(p, "fp32_refine") or {}
    _say("[gpu] C2 fp32_refine, reduced CG: local bases")
    m = mor.Mor(p, precision="fp32_refine", reduced_solver=1, reduced_rtol=float(ref["pcg_rtol"]), **tile)
    try:
        m.local_basis_all()
        m.project()
        u, nred = m.solve()
        solver, it, rel = mor.mor_get_solve_info(m.ctx)
        it_o = int(ref["pcg_iters"])
        _say(f"[gpu] C2 reduced CG: {it} iterations (oracle {it_o}), ||r||/||b|| {rel:.2e}")
        assert solver == 1 and 0 < rel <= float(ref["pcg_rtol"])
        assert abs(it - it_o) <= max(3, 0.1 * it_o), (it, it_o)
        At, bt = mor.mor_get_reduced(m.ctx)
        x = mor.mor_get_reduced_solution(m.ctx, nred)
        assert np.linalg.norm(bt - At @ x) <= 1e-10 * np.linalg.norm(bt)
        np.testing.assert_allclose(x @ bt, ref["x"] @ ref["bt"], rtol=1e-7)
        A, _, free, _ = ofem.global_system(p.mesh, p.kappa, p.f_nodal)
        d = (u - ref["u_tilde"])[free]
        uo = ref["u_tilde"][free]
        e = np.sqrt(max(d @ (A @ d), 0.0)) / np.sqrt(uo @ (A @ uo))
        _say(f"[gpu] C2 reduced CG: energy rel {e:.3e}")
        assert e < TOL_ENERGY, e
    finally:
        m.close()
