"""ctypes binding of libmor.so (include/mor.h): argument marshalling only.

Every step of the local reduction, the projection and the reduced solve runs in the
library's HIP kernels.  PyTorch supplies device memory (its caching allocator, through the
allocation callbacks of mor_opts) and the HIP stream the library orders its work on.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmor.so")

MOR_OK, MOR_EINVAL, MOR_ENOMEM, MOR_ENOTCONV, MOR_ESTATE, MOR_EDEVICE = 0, -1, -2, -3, -4, -5
MOR_FP64, MOR_FP32_REFINE, MOR_FP32, MOR_BF16_SPLIT = 0, 1, 2, 3
PRECISIONS = {"fp64": MOR_FP64, "fp32_refine": MOR_FP32_REFINE, "fp32": MOR_FP32, "bf16_split": MOR_BF16_SPLIT}

EXPORTED = ("mor_default_opts", "mor_create", "mor_local_basis", "mor_local_basis_batch", "mor_local_basis_sketched",
            "mor_project",
            "mor_solve", "mor_solve_noalloc", "mor_submit", "mor_poll", "mor_drain", "mor_step", "mor_engine_stats", "mor_get_sizes", "mor_get_nodes",
            "mor_get_pairs", "mor_get_basis", "mor_get_rank", "mor_get_sigma", "mor_get_local_block", "mor_get_reduced",
            "mor_get_reduced_solution", "mor_get_solve_info", "mor_get_stats", "mor_timing_enable", "mor_timing_get",
            "mor_timing_reset", "mor_destroy", "mor_last_error")


class MorError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mor error {code}: {msg}")
        self.code = code


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class MorMesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_tets", ctypes.c_int64), ("xyz", ctypes.c_void_p),
                ("tets", ctypes.c_void_p), ("dirichlet", ctypes.c_void_p)]


class MorCoeff(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_void_p), ("f_nodal", ctypes.c_void_p)]


class MorSubdomains(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("ext_tet_ptr", ctypes.c_void_p), ("ext_tets", ctypes.c_void_p),
                ("in_core", ctypes.c_void_p)]


class MorOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("cg_rtol", ctypes.c_double), ("refine_rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("oversample", ctypes.c_int32),
                ("eig_rtol", ctypes.c_double), ("eig_max_iter", ctypes.c_int32), ("cg_chunk", ctypes.c_int32),
                ("spmm_rows", ctypes.c_int32), ("spmm_vec", ctypes.c_int32), ("spmm_kind", ctypes.c_int32), ("stream_vec", ctypes.c_int32),
                ("stream_blocks", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("dense_batch", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_size_t),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_user", ctypes.c_void_p),
                ("hip_stream", ctypes.c_void_p), ("host_only", ctypes.c_int32), ("basis_update", ctypes.c_int32), ("update_drop", ctypes.c_double),
                ("reduced_solver", ctypes.c_int32), ("reduced_rtol", ctypes.c_double),
                ("reduced_max_iter", ctypes.c_int32), ("coarse", ctypes.c_int32), ("box_spmm", ctypes.c_int32)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # torch (when present) brings its own HIP/HSA runtime libraries; load them first so that
    # the library's runtime binds to the already-loaded HSA runtime in the same order every time
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mor_default_opts": (None, [P]),
        "mor_create": (I32, [P, P, P, P, P]),
        "mor_local_basis": (I32, [P, I32, I32, D, P, P, I32]),
        "mor_local_basis_batch": (I32, [P, I32, P, P, P, P]),
        "mor_local_basis_sketched": (I32, [P, I32, P, P, P, I32, P, P]),
        "mor_project": (I32, [P]),
        "mor_solve": (I32, [P, P, P]),
        "mor_solve_noalloc": (I32, [P, P, P]),
        "mor_submit": (I32, [P, I32, I32, D, I32, P]),
        "mor_poll": (I32, [P, ctypes.c_uint64, P, P]),
        "mor_drain": (I32, [P]),
        "mor_step": (I32, [P]),
        "mor_engine_stats": (I32, [P, P, P, P, P, P]),
        "mor_get_sizes": (I32, [P, I32, P, P, P, P]),
        "mor_get_nodes": (I32, [P, I32, P, I64]),
        "mor_get_pairs": (I32, [P, P, I64, P]),
        "mor_get_basis": (I32, [P, I32, P, I64, P]),
        "mor_get_rank": (I32, [P, I32, P, P]),
        "mor_get_sigma": (I32, [P, I32, P, I32, P]),
        "mor_get_local_block": (I32, [P, I32, P, P, I64]),
        "mor_get_reduced": (I32, [P, P, P, I64, P]),
        "mor_get_reduced_solution": (I32, [P, P, I64]),
        "mor_get_solve_info": (I32, [P, P, P, P]),
        "mor_get_stats": (I32, [P, I32, P, P, P, P]),
        "mor_timing_enable": (I32, [P, I32]),
        "mor_timing_get": (I32, [P, ctypes.c_char_p, P, P, P]),
        "mor_timing_reset": (I32, [P]),
        "mor_destroy": (None, [P]),
        "mor_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(rc):
    if rc != MOR_OK:
        raise MorError(rc, lib().mor_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


class _TorchAllocator:
    """Device memory from torch's caching allocator, handed to the library as callbacks."""

    def __init__(self, stream_handle: int):
        import torch
        self.torch = torch
        self.stream = stream_handle
        self.live = {}
        self.n_alloc = 0     # allocation and release callbacks seen
        self.n_free = 0

        def _alloc(nbytes, user):
            self.n_alloc += 1
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:
                return None
            self.live[p] = nbytes
            return p

        def _free(ptr, user):
            self.n_free += 1
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self.alloc_cb = ALLOC_FN(_alloc)
        self.free_cb = FREE_FN(_free)


def mor_default_opts() -> MorOpts:
    o = MorOpts()
    lib().mor_default_opts(ctypes.byref(o))
    return o


def mor_create(xyz, tets, dirichlet, kappa, f_nodal, ext_tet_ptr, ext_tets, in_core, opts: MorOpts | None = None):
    """Create a context (see include/mor.h).  Arrays are host numpy arrays."""
    keep = dict(
        xyz=np.ascontiguousarray(xyz, dtype=np.float64), tets=np.ascontiguousarray(tets, dtype=np.int32),
        dirichlet=np.ascontiguousarray(dirichlet, dtype=np.uint8), kappa=np.ascontiguousarray(kappa, dtype=np.float64),
        f=None if f_nodal is None else np.ascontiguousarray(f_nodal, dtype=np.float64),
        ptr=np.ascontiguousarray(ext_tet_ptr, dtype=np.int64), ext=np.ascontiguousarray(ext_tets, dtype=np.int32),
        core=np.ascontiguousarray(in_core, dtype=np.uint8))
    mesh = MorMesh(keep["xyz"].shape[0], keep["tets"].shape[0], _ptr(keep["xyz"]), _ptr(keep["tets"]),
                   _ptr(keep["dirichlet"]))
    coeff = MorCoeff(_ptr(keep["kappa"]), _ptr(keep["f"]))
    sub = MorSubdomains(keep["ptr"].shape[0] - 1, _ptr(keep["ptr"]), _ptr(keep["ext"]), _ptr(keep["core"]))
    if opts is None:
        opts = mor_default_opts()
    ctx = ctypes.c_void_p()
    _check(lib().mor_create(ctypes.byref(mesh), ctypes.byref(coeff), ctypes.byref(sub), ctypes.byref(opts),
                            ctypes.byref(ctx)))
    return ctx


def mor_local_basis(ctx, sd: int, rank: int, tol: float = 0.0, sigma_cap: int = 64):
    k = ctypes.c_int32()
    sig = np.zeros(sigma_cap)
    _check(lib().mor_local_basis(ctx, sd, rank, tol, ctypes.byref(k), _ptr(sig), sigma_cap))
    return k.value, sig


def mor_local_basis_batch(ctx, sds, ranks, tols=None):
    sds = np.ascontiguousarray(sds, dtype=np.int32)
    ranks = np.ascontiguousarray(ranks, dtype=np.int32)
    tl = None if tols is None else np.ascontiguousarray(tols, dtype=np.float64)
    k = np.zeros(sds.size, dtype=np.int32)
    _check(lib().mor_local_basis_batch(ctx, sds.size, _ptr(sds), _ptr(ranks), _ptr(tl), _ptr(k)))
    return k


def mor_local_basis_sketched(ctx, sds, ranks, omegas, tols=None):
    """Randomized local reduction (the C entry point of the same name).  omegas[i]: the
    random matrix of subdomain sds[i], (M_i, l) float64, rows in the subdomain's interface
    node order; the same l for every subdomain."""
    sds = np.ascontiguousarray(sds, dtype=np.int32)
    ranks = np.ascontiguousarray(ranks, dtype=np.int32)
    tl = None if tols is None else np.ascontiguousarray(tols, dtype=np.float64)
    oms = [np.ascontiguousarray(o, dtype=np.float64) for o in omegas]
    if len(oms) != sds.size or len({o.shape[1] for o in oms}) != 1:
        raise ValueError("one (M_i, l) sketch per subdomain, same l")
    ptrs = (ctypes.c_void_p * len(oms))(*[o.ctypes.data for o in oms])
    k = np.zeros(sds.size, dtype=np.int32)
    _check(lib().mor_local_basis_sketched(ctx, sds.size, _ptr(sds), _ptr(ranks), _ptr(tl), oms[0].shape[1],
                                          ctypes.cast(ptrs, ctypes.c_void_p), _ptr(k)))
    return k


def mor_project(ctx):
    _check(lib().mor_project(ctx))


def mor_solve(ctx, n_nodes: int):
    u = np.zeros(n_nodes)
    n = ctypes.c_int64()
    _check(lib().mor_solve(ctx, _ptr(u), ctypes.byref(n)))
    return u, n.value


def mor_solve_noalloc(ctx, u_dev_ptr: int):
    """The allocation-free reduced solve: u~ is written to the caller's device buffer at
    u_dev_ptr (n_nodes doubles); returns the reduced dimension."""
    n = ctypes.c_int64()
    _check(lib().mor_solve_noalloc(ctx, ctypes.c_void_p(u_dev_ptr), ctypes.byref(n)))
    return n.value


def mor_submit(ctx, sd, rank, tol, precision):
    t = ctypes.c_uint64()
    _check(lib().mor_submit(ctx, sd, rank, tol, precision, ctypes.byref(t)))
    return t.value


def mor_poll(ctx, ticket):
    d, s = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mor_poll(ctx, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(s)))
    return d.value, s.value


def mor_drain(ctx):
    _check(lib().mor_drain(ctx))


def mor_step(ctx):
    _check(lib().mor_step(ctx))


def mor_engine_stats(ctx):
    l, p = ctypes.c_int32(), ctypes.c_int32()
    lb, pb, bu = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mor_engine_stats(ctx, ctypes.byref(l), ctypes.byref(p), ctypes.byref(lb), ctypes.byref(pb),
                                  ctypes.byref(bu)))
    return dict(live=l.value, pending=p.value, live_bytes=lb.value, peak_bytes=pb.value, budget=bu.value)


def mor_get_sizes(ctx, sd):
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().mor_get_sizes(ctx, sd, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def mor_get_nodes(ctx, sd):
    nP, nV, nI, nB = mor_get_sizes(ctx, sd)
    out = np.zeros(nI + nB, dtype=np.int32)
    _check(lib().mor_get_nodes(ctx, sd, _ptr(out), out.size))
    return out


def mor_get_pairs(ctx):
    n = ctypes.c_int64()
    _check(lib().mor_get_pairs(ctx, None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, 2), dtype=np.int32)
    _check(lib().mor_get_pairs(ctx, _ptr(out), n.value, ctypes.byref(n)))
    return out


def mor_get_basis(ctx, sd):
    k = ctypes.c_int32()
    _check(lib().mor_get_basis(ctx, sd, None, 0, ctypes.byref(k)))
    nP, nV, nI, nB = mor_get_sizes(ctx, sd)
    out = np.zeros((nV, k.value + 1))
    _check(lib().mor_get_basis(ctx, sd, _ptr(out), out.size, ctypes.byref(k)))
    return out


def mor_get_rank(ctx, sd):
    """(k_eff, dim): lifting modes kept and basis columns after the optional basis update."""
    k, d = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mor_get_rank(ctx, sd, ctypes.byref(k), ctypes.byref(d)))
    return k.value, d.value


def mor_get_sigma(ctx, sd, cap=64):
    n = ctypes.c_int32()
    out = np.zeros(cap)
    _check(lib().mor_get_sigma(ctx, sd, _ptr(out), cap, ctypes.byref(n)))
    return out[:min(cap, n.value)]


def mor_get_local_block(ctx, sd):
    k = ctypes.c_int32()
    _check(lib().mor_get_basis(ctx, sd, None, 0, ctypes.byref(k)))
    k1 = k.value + 1
    A = np.zeros((k1, k1))
    b = np.zeros(k1)
    _check(lib().mor_get_local_block(ctx, sd, _ptr(A), _ptr(b), A.size))
    return A, b


def mor_get_reduced(ctx):
    n = ctypes.c_int64()
    _check(lib().mor_get_reduced(ctx, None, None, 0, ctypes.byref(n)))
    A = np.zeros((n.value, n.value))
    b = np.zeros(n.value)
    _check(lib().mor_get_reduced(ctx, _ptr(A), _ptr(b), A.size, ctypes.byref(n)))
    return A, b


def mor_get_reduced_load(ctx):
    """The reduced load b~ alone (no n x n matrix)."""
    n = ctypes.c_int64()
    _check(lib().mor_get_reduced(ctx, None, None, 0, ctypes.byref(n)))
    b = np.zeros(n.value)
    _check(lib().mor_get_reduced(ctx, None, _ptr(b), 0, ctypes.byref(n)))
    return b


def mor_get_reduced_solution(ctx, n):
    x = np.zeros(n)
    _check(lib().mor_get_reduced_solution(ctx, _ptr(x), n))
    return x


def mor_get_solve_info(ctx):
    """(solver, iterations, relative recurrence residual) of the last reduced solve."""
    s, it, rr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().mor_get_solve_info(ctx, ctypes.byref(s), ctypes.byref(it), ctypes.byref(rr)))
    return s.value, it.value, rr.value


def mor_get_stats(ctx, sd):
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().mor_get_stats(ctx, sd, *[ctypes.byref(x) for x in v]))
    return dict(cg_iter_a=v[0].value, cg_iter_k=v[1].value, refine=v[2].value, eig_iter=v[3].value)


def mor_timing_enable(ctx, on=True):
    _check(lib().mor_timing_enable(ctx, 1 if on else 0))


def mor_timing_get(ctx, name):
    n, ms, w = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(lib().mor_timing_get(ctx, name.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)))
    return n.value, ms.value, w.value


def mor_timing_reset(ctx):
    _check(lib().mor_timing_reset(ctx))


def mor_destroy(ctx):
    lib().mor_destroy(ctx)


class Mor:
    """A context on one problem (the `workloads.Problem` layout), with torch-managed memory."""

    def __init__(self, problem, precision="fp32_refine", use_torch=True, **opt_overrides):
        self.problem = problem
        self.opts = mor_default_opts()
        self.opts.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        for k, v in opt_overrides.items():
            setattr(self.opts, k, v)
        self._alloc = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible to torch")
            # memory from torch's caching allocator; the library orders its work on its own null
            # stream and synchronizes before it returns or releases memory.  Blocks that earlier
            # contexts released stay in torch's cache, where the library's default HBM budget
            # (3/4 of the device's free memory) would not see them: hand them back first.
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            self._alloc = _TorchAllocator(None)
            self.opts.dev_alloc = self._alloc.alloc_cb
            self.opts.dev_free = self._alloc.free_cb
            self.opts.hip_stream = None
        m, sd = problem.mesh, problem.subdomains
        self.ctx = mor_create(m.xyz, m.tets, m.dirichlet, problem.kappa, problem.f_nodal, sd.ext_tet_ptr,
                              sd.ext_tets, sd.in_core, self.opts)
        self.n_sub = sd.n_sub

    def local_basis_all(self, rank=None, tols=None):
        ranks = np.full(self.n_sub, self.problem.rank if rank is None else rank, dtype=np.int32)
        if self.problem.ranks is not None and rank is None:
            ranks = self.problem.ranks.astype(np.int32)
        return mor_local_basis_batch(self.ctx, np.arange(self.n_sub), ranks, tols)

    def project(self):
        mor_project(self.ctx)

    def solve(self):
        return mor_solve(self.ctx, self.problem.mesh.n_nodes)

    def close(self):
        if self.ctx is not None:
            mor_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
