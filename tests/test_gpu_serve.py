"""Serving on the GPU: continuous batching gives each request the same result as running it
alone, admission keeps the device bytes of admitted requests within the HBM budget, and mixed
precisions in one stream each match their own solo run.

"Same" is judged at the FP32 paths' tolerance: singular values within 1e-7 relative, k_eff
exact, and the largest principal angle between the two bases below 1e-5 (the batched CG sums
p'Ap with atomics in a different order, so results agree to rounding, not bit for bit).
"""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

TOL_SIGMA = 1e-7
TOL_ANGLE = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem():
    rng = np.random.default_rng(21)
    cuts = tuple(w.cuts_random(14, k, 3, rng) for k in (3, 2, 2))
    p = w.make_problem(14, cuts=cuts, r=2, rank=6, kappa="lognormal", kappa_sigma=1.0, seed=22,
                       name="serve-uneven")
    p.ranks = np.random.default_rng(23).integers(3, 9, size=p.subdomains.n_sub)
    return p


def _sin_angle(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    return np.linalg.norm(qb - qa @ (qa.T @ qb), 2)


def _result(mor, ctx, sd):
    return dict(sigma=mor.mor_get_sigma(ctx, sd), V=mor.mor_get_basis(ctx, sd))


def _solo(p, sd, rank, precision):
    from paper_2404_06260_amd import mor
    m = mor.Mor(p, precision=precision)
    try:
        k, _ = mor.mor_local_basis(m.ctx, sd, int(rank))
        r = _result(mor, m.ctx, sd)
        r["k"] = k
        return r
    finally:
        m.close()


def _compare(a, b, k, tag):
    ns = min(a["sigma"].size, b["sigma"].size, k + 1)
    np.testing.assert_allclose(b["sigma"][:ns], a["sigma"][:ns], rtol=TOL_SIGMA, err_msg=tag)
    assert a["V"].shape == b["V"].shape, tag
    np.testing.assert_allclose(b["V"][:, 0], a["V"][:, 0], rtol=0, atol=1e-6 * np.abs(a["V"][:, 0]).max(),
                               err_msg=tag)
    s = _sin_angle(a["V"][:, 1:], b["V"][:, 1:])
    assert s < TOL_ANGLE, (tag, s)


def _run_mix(p, stream, **opts):
    import torch
    from paper_2404_06260_amd import mor, serve
    torch.cuda.set_device(0)
    m = mor.Mor(p, precision="fp32_refine", **opts)
    try:
        res = serve.run_stream(m.ctx, stream)
        assert (res.status == 0).all(), res.status
        out = {}
        for j in range(len(stream)):
            out[j] = _result(mor, m.ctx, int(stream.sds[j]))
        return res, out
    finally:
        m.close()


def test_results_same_alone_and_in_the_mix():
    from paper_2404_06260_amd import serve
    p = _problem()
    n = p.subdomains.n_sub
    # arrivals spread over a few CG chunks so that requests join while others run
    stream = serve.make_stream(p, n, rate=400.0, seed_arrivals=31, seed_order=32)
    _say(f"[serve] mix of {n} requests")
    res, mix = _run_mix(p, stream, cg_chunk=4)
    assert (res.status == 0).all()
    assert res.max_live >= 2, "requests never overlapped on the device"
    _say(f"[serve] p50 {res.percentiles()['p50'] * 1e3:.1f} ms, max live {res.max_live}")
    for j in range(n):
        sd = int(stream.sds[j])
        solo = _solo(p, sd, stream.ranks[j], "fp32_refine")
        _compare(solo, mix[j], solo["k"], f"subdomain {sd}")


def test_admission_respects_the_hbm_budget():
    from paper_2404_06260_amd import mor, serve
    p = _problem()
    n = p.subdomains.n_sub
    # a budget that holds about two of the largest requests at once
    big = int(np.argmax(np.diff(p.subdomains.ext_tet_ptr)))
    m = mor.Mor(p, precision="fp32_refine")
    try:
        mor.mor_local_basis(m.ctx, big, int(p.ranks[big]))
        one = mor.mor_engine_stats(m.ctx)["peak_bytes"]
    finally:
        m.close()
    budget = int(2.5 * one)
    stream = serve.make_stream(p, n, rate=float("inf"), seed_order=41)
    res, mix = _run_mix(p, stream, hbm_budget_bytes=budget)
    _say(f"[serve] budget {budget} B, peak {res.peak_bytes} B, max live {res.max_live}")
    assert (res.status == 0).all()
    assert res.budget_bytes == budget
    assert 0 < res.peak_bytes <= budget
    assert res.max_live < n
    for j in (0, n - 1):
        sd = int(stream.sds[j])
        solo = _solo(p, sd, stream.ranks[j], "fp32_refine")
        _compare(solo, mix[j], solo["k"], f"subdomain {sd}")


def test_mixed_precisions_each_match_their_solo_run():
    from paper_2404_06260_amd import serve
    p = _problem()
    n = p.subdomains.n_sub
    stream = serve.make_stream(p, n, rate=400.0, seed_arrivals=51, seed_order=52,
                               precisions=("fp32_refine", "fp64"), precision_p=(0.5, 0.5))
    assert len(set(stream.precisions)) == 2
    res, mix = _run_mix(p, stream, cg_chunk=4)
    assert (res.status == 0).all()
    for j in range(n):
        sd = int(stream.sds[j])
        solo = _solo(p, sd, stream.ranks[j], stream.precisions[j])
        _compare(solo, mix[j], solo["k"], f"subdomain {sd} {stream.precisions[j]}")
