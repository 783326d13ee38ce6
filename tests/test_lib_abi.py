"""CPU checks of the C-ABI library: it loads, exports every declared entry point, and its
host-side decomposition (index sets I, B, V_i, P_i and the neighbour pairs) equals the
oracle's independent derivation (bit-exact integer work)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as w
from oracle import decomp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    h = open(os.path.join(ROOT, "include", "mor.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(mor_\w+)\s*\(", h, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2404_06260_amd import mor
    lib = ctypes.CDLL(mor.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(mor.EXPORTED)


def _host_ctx(p):
    from paper_2404_06260_amd import mor
    o = mor.mor_default_opts()
    o.host_only = 1
    m, sd = p.mesh, p.subdomains
    return mor.mor_create(m.xyz, m.tets, m.dirichlet, p.kappa, p.f_nodal, sd.ext_tet_ptr, sd.ext_tets, sd.in_core, o)


@pytest.mark.parametrize("case", ["C1", "uneven", "jitter", "general"])
def test_host_decomposition_matches_oracle(case):
    from paper_2404_06260_amd import mor
    if case == "general":          # L-shape with a cavity, shuffled numbering, BFS graph partition
        p = w.make_general_problem()
    elif case == "C1":
        p = w.make_config("C1")
    elif case == "uneven":
        rng = np.random.default_rng(3)
        cuts = tuple(w.cuts_random(14, k, 3, rng) for k in (3, 2, 2))
        p = w.make_problem(14, cuts=cuts, r=2)
    else:
        p = w.make_problem(10, (2, 2, 1), r=2, jitter=0.2, seed=1)
    ctx = _host_ctx(p)
    try:
        sets = decomp.all_local_sets(p.mesh, p.subdomains)
        for i, s in enumerate(sets):
            nP, nV, nI, nB = mor.mor_get_sizes(ctx, i)
            nodes = mor.mor_get_nodes(ctx, i)
            assert (nP, nV, nI, nB) == (s.P.size, s.V.size, s.I.size, s.B.size)
            np.testing.assert_array_equal(np.sort(nodes[:nP]), s.P)
            np.testing.assert_array_equal(np.sort(nodes[:nV]), s.V)
            np.testing.assert_array_equal(np.sort(nodes[:nI]), s.I)
            np.testing.assert_array_equal(nodes[nI:], s.B)
        # neighbour pairs coupled through A_0 on omega_0
        owner = decomp.owner_map(p.mesh, sets)
        from oracle import project
        A0, free, _ = project.omega0_stiffness(p.mesh, p.kappa, p.subdomains)
        coo = A0.tocoo()
        oi, oj = owner[free[coo.row]], owner[free[coo.col]]
        ref = {(int(a), int(b)) for a, b in zip(oi, oj) if a < b}
        got = {tuple(x) for x in mor.mor_get_pairs(ctx).tolist()}
        assert got == ref
    finally:
        mor.mor_destroy(ctx)


def test_invalid_inputs_are_rejected():
    from paper_2404_06260_amd import mor
    p = w.make_config("C1")
    o = mor.mor_default_opts()
    o.host_only = 1
    m, sd = p.mesh, p.subdomains
    bad = m.tets.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]            # inverted tet
    with pytest.raises(mor.MorError) as e:
        mor.mor_create(m.xyz, bad, m.dirichlet, p.kappa, None, sd.ext_tet_ptr, sd.ext_tets, sd.in_core, o)
    assert e.value.code == mor.MOR_EINVAL
    # cores overlapping by two layers: not a partition of the free nodes
    p2 = w.make_problem(8, (2, 1, 1), r=1)
    core = p2.subdomains.in_core.copy()
    core[:] = 1
    with pytest.raises(mor.MorError):
        mor.mor_create(p2.mesh.xyz, p2.mesh.tets, p2.mesh.dirichlet, p2.kappa, None, p2.subdomains.ext_tet_ptr,
                       p2.subdomains.ext_tets, core, o)
    # extension r = 0: omega_i reaches the boundary of omega_i^+
    p3 = w.make_problem(8, (2, 1, 1), r=0)
    with pytest.raises(mor.MorError):
        mor.mor_create(p3.mesh.xyz, p3.mesh.tets, p3.mesh.dirichlet, p3.kappa, None, p3.subdomains.ext_tet_ptr,
                       p3.subdomains.ext_tets, p3.subdomains.in_core, o)


def test_default_options_and_option_checks():
    """mor_default_opts fills the defaults include/mor.h documents, the binding's struct has the
    header's size (a field added on one side only would shift every later field), and
    mor_create rejects out-of-range reduced-solver options before touching a device."""
    from paper_2404_06260_amd import mor
    o = mor.mor_default_opts()
    assert o.precision == mor.PRECISIONS["fp32_refine"]
    assert (o.cg_rtol, o.refine_rtol, o.max_iter, o.refine_steps) == (1e-5, 1e-8, 4000, 3)
    assert (o.reduced_solver, o.reduced_rtol, o.reduced_max_iter) == (0, 1e-12, 20000)
    assert o.coarse == 1 and o.basis_update == 0 and o.update_drop == 0.0
    h = open(os.path.join(ROOT, "include", "mor.h")).read()
    body = h[h.index("typedef struct {\n  int32_t precision;"):h.index("} mor_opts;")]
    fields = re.findall(r"^\s*(?:int32_t|double|size_t|mor_alloc_fn|mor_free_fn|void\*)\s+(\w+);", body, re.M)
    assert fields == [f[0] for f in mor.MorOpts._fields_]
    p = w.make_config("C1")
    m, sd = p.mesh, p.subdomains
    for bad in (dict(reduced_solver=3), dict(reduced_solver=-1), dict(reduced_rtol=-1.0), dict(reduced_max_iter=-2)):
        o = mor.mor_default_opts()
        o.host_only = 1
        for k, v in bad.items():
            setattr(o, k, v)
        with pytest.raises(mor.MorError) as e:
            mor.mor_create(m.xyz, m.tets, m.dirichlet, p.kappa, None, sd.ext_tet_ptr, sd.ext_tets, sd.in_core, o)
        assert e.value.code == mor.MOR_EINVAL, bad


_ENOMEM_CHILD = r"""
import resource, sys
sys.path.insert(0, sys.argv[1])
import workloads as w
from paper_2404_06260_amd import mor
p = w.make_problem(40, (2, 2, 2), r=2)
o = mor.mor_default_opts()
o.host_only = 1
m, sd = p.mesh, p.subdomains
mor.lib()
vm = int([l.split()[1] for l in open("/proc/self/status") if l.startswith("VmSize:")][0]) * 1024
resource.setrlimit(resource.RLIMIT_AS, (vm + (1 << 20), resource.RLIM_INFINITY))
try:
    ctx = mor.mor_create(m.xyz, m.tets, m.dirichlet, p.kappa, None, sd.ext_tet_ptr, sd.ext_tets, sd.in_core, o)
    print("CODE 0")
except mor.MorError as e:
    print("CODE", e.code, str(e))
"""


def test_host_allocation_failure_is_an_error_code():
    """A host allocation that fails inside an entry point comes back as MOR_ENOMEM with a message,
    not as a C++ exception through the C-ABI (which would abort the process): a child process
    caps its address space just above its current size, then builds a context (host-only, no
    device) for a 40^3 mesh whose copies alone exceed the cap."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-c", _ENOMEM_CHILD, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("CODE")][-1]
    from paper_2404_06260_amd import mor
    assert int(line.split()[1]) == mor.MOR_ENOMEM, line
    assert "host memory allocation failed" in line
