"""Pins of the oracle's P1 discretisation against closed forms and convergence.

Nothing here re-types the oracle's formulas: each check compares against a value
that the mathematics fixes independently (a hand-computed element matrix, exact
integrals of polynomials, the O(h) energy convergence of P1 elements for the
manufactured solution of Section 7.1's kind).
"""
import numpy as np
import pytest

import workloads as w
from oracle import fem, solve

# 4-point degree-2 quadrature on a tet (barycentric (a,b,b,b) and permutations)
_QA, _QB = 0.5854101966249685, 0.1381966011250105
_QBARY = np.array([[_QA, _QB, _QB, _QB], [_QB, _QA, _QB, _QB], [_QB, _QB, _QA, _QB], [_QB, _QB, _QB, _QA]])


def test_reference_tet_closed_form():
    """Unit right tet: stiffness = (1/6) [[3,-1,-1,-1],[-1,1,0,0],[-1,0,1,0],[-1,0,0,1]],
    mass = (1/120)(1 + delta_ab)."""
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    tets = np.array([[0, 1, 2, 3]])
    Ke, G, Me = fem.element_matrices(xyz, tets, np.array([2.0]))
    K_ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    np.testing.assert_allclose(G[0], K_ref, atol=1e-15)
    np.testing.assert_allclose(Ke[0], 2.0 * K_ref, atol=1e-15)
    np.testing.assert_allclose(Me[0], (np.ones((4, 4)) + np.eye(4)) / 120.0, atol=1e-16)


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_mesh_volume_orientation(jitter):
    m = w.kuhn_cube(6, jitter=jitter, seed=2)
    vol, det, _ = fem.tet_geometry(m.xyz, m.tets)
    assert np.all(det > 0)
    assert abs(vol.sum() - 1.0) < 1e-13
    assert m.n_nodes == 7 ** 3 and m.n_tets == 6 * 6 ** 3


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_stiffness_kernel_and_linear_energy(jitter):
    """Without Dirichlet rows: A 1 = 0; g^T A g = |a|^2 |Omega| for linear g = a.x + c;
    1^T M 1 = |Omega|; g^T M g = exact integral of g^2."""
    m = w.kuhn_cube(5, jitter=jitter, seed=3)
    allmap = np.arange(m.n_nodes)
    Ke, G, Me = fem.element_matrices(m.xyz, m.tets, np.ones(m.n_tets))
    A = fem.assemble(G, m.tets, allmap, m.n_nodes)
    M = fem.assemble(Me, m.tets, allmap, m.n_nodes)
    one = np.ones(m.n_nodes)
    assert np.abs(A @ one).max() < 1e-13
    a = np.array([0.3, -1.2, 0.7])
    g = m.xyz @ a + 0.4
    assert abs(g @ (A @ g) - a @ a) < 1e-12
    assert abs(one @ (M @ one) - 1.0) < 1e-14
    # int_[0,1]^3 (a.x + c)^2 dx = sum_i a_i^2/3 + sum_{i<j} a_i a_j/2 + c*sum a_i + c^2
    c = 0.4
    exact = (a ** 2).sum() / 3 + (a[0] * a[1] + a[0] * a[2] + a[1] * a[2]) / 2 + c * a.sum() + c ** 2
    assert abs(g @ (M @ g) - exact) < 1e-13


def _h1_seminorm_error(mesh, u, grad_exact):
    vol, _, grads = fem.tet_geometry(mesh.xyz, mesh.tets)
    gu = np.einsum("tai,ta->ti", grads, u[mesh.tets])          # constant gradient per tet
    X = mesh.xyz[mesh.tets]                                     # (t, 4, 3)
    err = 0.0
    for q in range(4):
        xq = np.einsum("a,tai->ti", _QBARY[q], X)
        d = grad_exact(xq) - gu
        err += 0.25 * np.sum(vol * np.sum(d * d, axis=1))
    return np.sqrt(err)


def _grad_sine(x):
    s = np.sin(np.pi * x)
    c = np.cos(np.pi * x)
    return np.pi * np.stack([c[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * c[:, 1] * s[:, 2], s[:, 0] * s[:, 1] * c[:, 2]], 1)


def test_manufactured_sine_converges_at_order_one():
    """phi = sin(pi x) sin(pi y) sin(pi z), f = 3 pi^2 phi: ||grad(phi - u_h)|| = O(h)."""
    errs = []
    for n in (4, 8, 16):
        p = w.make_problem(n, (1, 1, 1), r=0, load="sine")
        u, *_ = solve.fe_solution(p.mesh, p.kappa, p.f_nodal)
        errs.append(_h1_seminorm_error(p.mesh, u, _grad_sine))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 1.0) < 0.15), (errs, rates)
    # the energy of phi is 3 pi^2 / 8; the discrete energy approaches it from below
    assert errs[-1] / np.sqrt(3 * np.pi ** 2 / 8) < 0.2


def test_polynomial_load_has_unit_energy_and_error_near_table2():
    """Section 7.1: f = 2 sqrt(900)(...) has phi = 30 x(1-x) y(1-y) z(1-z) with ||grad phi|| = 1.
    The FE error is about 1.2 h with h = sqrt(3)/n (Table 2, cases 7-11); loose soft check."""
    n = 12
    p = w.make_problem(n, (1, 1, 1), r=0, load="poly")

    def grad_phi(x):
        g = x * (1 - x)
        dg = 1 - 2 * x
        return 30 * np.stack([dg[:, 0] * g[:, 1] * g[:, 2], g[:, 0] * dg[:, 1] * g[:, 2], g[:, 0] * g[:, 1] * dg[:, 2]], 1)

    zero = np.zeros(p.mesh.n_nodes)
    e_phi = _h1_seminorm_error(p.mesh, zero, grad_phi)      # = ||grad phi|| by quadrature
    assert abs(e_phi - 1.0) < 5e-3
    u, *_ = solve.fe_solution(p.mesh, p.kappa, p.f_nodal)
    err = _h1_seminorm_error(p.mesh, u, grad_phi)
    h = np.sqrt(3) / n
    assert 0.4 * h < err < 2.0 * h, (err, h)


def test_error_to_h_ratio_within_table2_band():
    """Table 2 (Section 7.1) prints error/h between about 0.8 and 1.25 for cases 4-11;
    the Kuhn-cube FE error of the polynomial load lands in a generous band around it."""
    import os
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "table2_scaling.txt"))
            if l.strip() and not l.startswith("#")]
    ratios = np.array([float(r[5]) / float(r[4]) for r in rows])
    assert 0.8 < ratios.min() and ratios.max() < 1.25
    n = 12
    p = w.make_problem(n, (1, 1, 1), r=0, load="poly")

    def grad_phi(x):
        g = x * (1 - x)
        dg = 1 - 2 * x
        return 30 * np.stack([dg[:, 0] * g[:, 1] * g[:, 2], g[:, 0] * dg[:, 1] * g[:, 2], g[:, 0] * g[:, 1] * dg[:, 2]], 1)

    u, *_ = solve.fe_solution(p.mesh, p.kappa, p.f_nodal)
    ratio = _h1_seminorm_error(p.mesh, u, grad_phi) / (np.sqrt(3) / n)
    assert 0.5 * ratios.min() < ratio < 2.0 * ratios.max(), ratio
