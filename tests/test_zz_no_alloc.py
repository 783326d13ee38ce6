"""The allocation-free reduced solve (mor_solve_noalloc) against mor_solve on the same context,
through the C-ABI: two calls in a row on different problems, the second with a smaller reduced
system (the shared static array keeps the first call's contents), each equal to mor_solve's
result to rounding, and no device allocation through the library's allocation callback during
either call."""
import sys

import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _prepare(p, solver):
    from paper_2404_06260_amd import mor
    m = mor.Mor(p, precision="fp64", reduced_solver=solver, refine_rtol=1e-11)
    m.local_basis_all()
    m.project()
    u_ref, n = m.solve()
    x_ref = mor.mor_get_reduced_solution(m.ctx, n)
    return m, u_ref, x_ref, n


def _noalloc(m, n_nodes):
    import torch
    from paper_2404_06260_amd import mor
    u_dev = torch.full((n_nodes,), 7.0, dtype=torch.float64, device="cuda")   # stale contents on purpose
    torch.cuda.synchronize()
    a0, f0 = m._alloc.n_alloc, m._alloc.n_free
    n = mor.mor_solve_noalloc(m.ctx, u_dev.data_ptr())
    assert (m._alloc.n_alloc, m._alloc.n_free) == (a0, f0), "the call went through the allocation callbacks"
    torch.cuda.synchronize()
    return u_dev.cpu().numpy(), n


def test_noalloc_solve_matches_mor_solve_twice_second_smaller():
    import torch
    from paper_2404_06260_amd import mor
    torch.cuda.set_device(0)
    big = w.make_problem(12, (2, 2, 2), r=2, rank=6, kappa="lognormal", seed=3, name="noalloc-big")
    small = w.make_problem(10, (2, 1, 1), r=2, rank=3, kappa="lognormal", seed=4, name="noalloc-small")
    runs = []
    for p, solver in ((big, 1), (small, 2)):
        m, u_ref, x_ref, n = _prepare(p, solver)
        runs.append((p, m, u_ref, x_ref, n))
    assert runs[1][4] < runs[0][4]
    try:
        for p, m, u_ref, x_ref, n in runs:
            u, n2 = _noalloc(m, p.mesh.n_nodes)
            x = mor.mor_get_reduced_solution(m.ctx, n)
            _say(f"[gpu] {p.name}: reduced dim {n2}, max |u - u_ref| {np.abs(u - u_ref).max():.2e}")
            assert n2 == n
            np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-11 * np.abs(x_ref).max())
            np.testing.assert_allclose(u, u_ref, rtol=0, atol=1e-11 * np.abs(u_ref).max())
            assert np.all(u[p.mesh.dirichlet != 0] == 0.0)
    finally:
        for r in runs:
            r[1].close()


def test_noalloc_solve_rejects_the_cholesky_path_and_calls_out_of_order():
    import torch
    from paper_2404_06260_amd import mor
    torch.cuda.set_device(0)
    p = w.make_problem(8, (2, 1, 1), r=1, rank=3, name="noalloc-errors")
    u_dev = torch.zeros(p.mesh.n_nodes, dtype=torch.float64, device="cuda")
    m = mor.Mor(p, precision="fp64", reduced_solver=0)
    try:
        with pytest.raises(mor.MorError) as ei:
            mor.mor_solve_noalloc(m.ctx, u_dev.data_ptr())
        assert ei.value.code == mor.MOR_ESTATE
        m.local_basis_all()
        m.project()
        with pytest.raises(mor.MorError) as ei:
            mor.mor_solve_noalloc(m.ctx, u_dev.data_ptr())
        assert ei.value.code == mor.MOR_EINVAL
    finally:
        m.close()
