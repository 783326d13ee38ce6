"""Failure handling on the GPU, every condition forced from the host so that every kernel
exits normally: an iteration cap the block CG cannot meet, an FP64 refinement target the allowed
corrections cannot reach, an eigensolver cap, an iteration cap of the reduced conjugate
gradients, a request larger than the HBM budget, and calls out of order.  Each failure comes
back as its error code with a message, the engine is left idle with its memory released, and the
context keeps working."""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem():
    return w.make_problem(10, (2, 2, 1), r=2, rank=5, kappa="lognormal", seed=7, name="fail")


def _idle(mor, ctx):
    st = mor.mor_engine_stats(ctx)
    assert st["live"] == 0 and st["pending"] == 0 and st["live_bytes"] == 0, st


def test_cg_iteration_cap_reports_enotconv():
    from paper_2404_06260_amd import mor
    p = _problem()
    m = mor.Mor(p, precision="fp32_refine", max_iter=8, cg_chunk=4)
    try:
        with pytest.raises(mor.MorError) as ei:
            m.local_basis_all()
        _say(f"[gpu] {ei.value}")
        assert ei.value.code == mor.MOR_ENOTCONV
        _idle(mor, m.ctx)
    finally:
        m.close()


def test_refinement_target_out_of_reach_reports_enotconv():
    """FP32 block CG with FP64 residual refinement: with no correction allowed (refine_steps = 0),
    a refinement target far below what one FP32 solve to cg_rtol reaches must fail the request
    instead of returning the unrefined solution; the same context with corrections allowed
    reaches it."""
    from paper_2404_06260_amd import mor
    p = _problem()
    for prec in ("fp32_refine", "bf16_split"):
        m = mor.Mor(p, precision=prec, refine_steps=0, refine_rtol=1e-12)
        try:
            with pytest.raises(mor.MorError) as ei:
                mor.mor_local_basis(m.ctx, 0, p.rank)
            _say(f"[gpu] {prec}: {ei.value}")
            assert ei.value.code == mor.MOR_ENOTCONV
            assert "refine" in str(ei.value)
            _idle(mor, m.ctx)
        finally:
            m.close()
    m = mor.Mor(p, precision="fp32_refine", refine_steps=4, refine_rtol=1e-12)
    try:
        k, _ = mor.mor_local_basis(m.ctx, 0, p.rank)
        assert k >= p.rank
        assert 1 <= mor.mor_get_stats(m.ctx, 0)["refine"] <= 4
    finally:
        m.close()


def test_eigensolver_cap_reports_enotconv_then_context_recovers():
    from paper_2404_06260_amd import mor
    p = _problem()
    m = mor.Mor(p, precision="fp64", eig_max_iter=1)
    try:
        with pytest.raises(mor.MorError) as ei:
            mor.mor_local_basis(m.ctx, 0, p.rank)
        assert ei.value.code == mor.MOR_ENOTCONV
        _idle(mor, m.ctx)
    finally:
        m.close()
    m = mor.Mor(p, precision="fp64")
    try:
        k, _ = mor.mor_local_basis(m.ctx, 0, p.rank)
        assert k >= p.rank
    finally:
        m.close()


def test_request_above_the_budget_fails_alone():
    from paper_2404_06260_amd import mor
    p = _problem()
    m = mor.Mor(p, precision="fp32_refine", hbm_budget_bytes=1 << 20)
    try:
        with pytest.raises(mor.MorError) as ei:
            mor.mor_local_basis(m.ctx, 0, p.rank)
        assert ei.value.code == mor.MOR_ENOMEM
        _idle(mor, m.ctx)
        t = mor.mor_submit(m.ctx, 1, p.rank, 0.0, mor.MOR_FP32_REFINE)
        mor.mor_drain(m.ctx)
        done, status = mor.mor_poll(m.ctx, t)
        assert done == 1 and status == mor.MOR_ENOMEM
        _idle(mor, m.ctx)
    finally:
        m.close()


def test_calls_out_of_order_report_estate():
    from paper_2404_06260_amd import mor
    p = _problem()
    m = mor.Mor(p, precision="fp32_refine")
    try:
        with pytest.raises(mor.MorError) as ei:
            m.project()
        assert ei.value.code == mor.MOR_ESTATE
        with pytest.raises(mor.MorError) as ei:
            m.solve()
        assert ei.value.code == mor.MOR_ESTATE
        m.local_basis_all()
        m.project()
        u, n = m.solve()
        assert np.isfinite(u).all() and n == (p.rank + 1) * p.subdomains.n_sub
    finally:
        m.close()


def test_reduced_pcg_iteration_cap_reports_enotconv():
    from paper_2404_06260_amd import mor
    p = _problem()
    m = mor.Mor(p, precision="fp64", reduced_solver=1, reduced_max_iter=2)
    try:
        m.local_basis_all()
        m.project()
        with pytest.raises(mor.MorError) as ei:
            m.solve()
        _say(f"[gpu] {ei.value}")
        assert ei.value.code == mor.MOR_ENOTCONV
        with pytest.raises(mor.MorError) as ei:
            mor.mor_get_reduced_solution(m.ctx, 1)
        assert ei.value.code == mor.MOR_ESTATE
    finally:
        m.close()
