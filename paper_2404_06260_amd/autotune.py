"""Autotuner for the block-CG tiles.

Two sweeps on the real workload, each candidate running the batched local reduction with a
loose CG tolerance (a few dozen iterations of the real kernels on the real matrices), timed
with the library's HIP-event timers on its stream:
  1. the SpMM: LDS-halo tiles (halo cap x 256-byte column slices per workgroup) or row tiles
     (rows x width), best algorithmic GB/s;
  2. the streaming (update / direction) tile: width x row aggregates per tile, least time.
The winner is cached per workload in a JSON file next to this module, with a hash of the
source text of the kernels it tuned; `best()` returns the cached options, or None when there is
no entry or those kernels have changed since it was measured.
"""
from __future__ import annotations

import json
import os

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
# (kind, spmm_vec, spmm_rows): kind 1 / 3 = LDS halo tiles with 256- / 128-byte column slices
# (slices per workgroup, halo cap), kind 2 = row tiles (width in 64 columns, rows)
CANDIDATES = [(3, 16, 96), (3, 16, 64), (3, 32, 96), (3, 16, 128), (3, 8, 96), (1, 16, 64), (1, 8, 64), (2, 4, 8)]
# (stream_vec, stream_blocks); the block counts divide the 8-aggregate coarse blocks of the
# two-level preconditioner (a tile never straddles two blocks), so none is overridden
STREAM_CANDIDATES = [(2, 4), (2, 8), (1, 4), (1, 8), (4, 4), (4, 8)]


# the kernels whose launch shapes the cached options choose
TUNED_KERNELS = ("k_cg_spmm_halo", "k_cg_spmm", "k_cg_update", "k_cg_direction")


def kernel_hash() -> str:
    """sha256 (16 hex digits) of the tuned kernels' source text in csrc/mor_kernels.hip, each
    from its `template` line (if any) to the closing brace at column 0."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "mor_kernels.hip")
    lines = open(path).read().split("\n")
    h = hashlib.sha256()
    for name in TUNED_KERNELS:
        for i, ln in enumerate(lines):
            if "__global__" in ln and f"void {name}(" in ln:
                b = i - 1 if i > 0 and lines[i - 1].startswith("template") else i
                e = next(j for j in range(i, len(lines)) if lines[j] == "}")
                h.update("\n".join(lines[b:e + 1]).encode())
                break
    return h.hexdigest()[:16]


def _key(problem, precision):
    # one target (gfx950): the key is the workload, not the device name the runtime reports
    return f"{problem.name}|{problem.subdomains.n_sub}|{precision}"


def best(problem, precision):
    """Cached options dict (spmm_vec, spmm_rows, stream_vec, stream_blocks) or None."""
    if not os.path.exists(CACHE):
        return None
    try:
        d = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    r = d.get(_key(problem, precision))
    if r is None or r.get("src") != kernel_hash():
        return None
    return {k: int(r[k]) for k in ("spmm_kind", "spmm_vec", "spmm_rows", "stream_vec", "stream_blocks") if k in r}


def _run(problem, ids, cg_prec, opts):
    import numpy as np
    from . import mor
    m = mor.Mor(problem, precision=cg_prec, cg_rtol=1e-2, refine_rtol=1e-2, **opts)
    try:
        mor.mor_timing_enable(m.ctx, True)
        ranks = np.full(ids.size, problem.rank, dtype=np.int32)
        mor.mor_local_basis_batch(m.ctx, ids, ranks)
        return {k: mor.mor_timing_get(m.ctx, k) for k in ("spmm", "cg_update", "cg_direction")}
    finally:
        m.close()


def tune(problem, precision="fp32_refine", sub_ids=None, verbose=True, save=True):
    import numpy as np
    cg_prec = "fp64" if precision == "fp64" else "fp32"
    ids = np.arange(problem.subdomains.n_sub) if sub_ids is None else np.asarray(sub_ids)
    sp_res = []
    _run(problem, ids, cg_prec, {})   # warm-up: module load and first-touch allocations
    for kind, v, rb in CANDIDATES:
        if cg_prec == "fp64" and kind == 2 and v > 2:
            continue
        t = _run(problem, ids, cg_prec, dict(spmm_kind=kind, spmm_vec=v, spmm_rows=rb))
        n, ms, by = t["spmm"]
        gbs = (by / n) / (ms / n * 1e-3) / 1e9 if n and ms > 0 else 0.0
        sp_res.append(dict(spmm_kind=kind, spmm_vec=v, spmm_rows=rb, launches=n, avg_ms=ms / max(n, 1), gbs=gbs))
        if verbose:
            print(f"[autotune] spmm kind={kind} v={v} rows={rb}: {n} launches, {ms / max(n, 1):.3f} ms avg, "
                  f"{gbs:.0f} GB/s", flush=True)
    sp = max(sp_res, key=lambda r: r["gbs"])
    st_res = []
    for v, nb in STREAM_CANDIDATES:
        if cg_prec == "fp64" and v > 2:
            continue
        t = _run(problem, ids, cg_prec, dict(spmm_kind=sp["spmm_kind"], spmm_vec=sp["spmm_vec"],
                                             spmm_rows=sp["spmm_rows"], stream_vec=v, stream_blocks=nb))
        ms = t["cg_update"][1] + t["cg_direction"][1]
        n = t["cg_update"][0]
        st_res.append(dict(stream_vec=v, stream_blocks=nb, launches=n, ms=ms))
        if verbose:
            print(f"[autotune] stream v={v} blocks={nb}: {n} iterations, update+direction {ms / max(n, 1):.3f} ms/iter",
                  flush=True)
    st = min(st_res, key=lambda r: r["ms"] / max(r["launches"], 1))
    win = dict(spmm_kind=sp["spmm_kind"], spmm_vec=sp["spmm_vec"], spmm_rows=sp["spmm_rows"], spmm_gbs=sp["gbs"],
               stream_vec=st["stream_vec"], stream_blocks=st["stream_blocks"])
    if save:
        d = {}
        if os.path.exists(CACHE):
            try:
                d = json.load(open(CACHE))
            except (OSError, ValueError):
                d = {}
        d[_key(problem, precision)] = dict(win, src=kernel_hash(), spmm_all=sp_res, stream_all=st_res)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    return win


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as w
    name = sys.argv[1] if len(sys.argv) > 1 else "C2"
    prec = sys.argv[2] if len(sys.argv) > 2 else "fp32_refine"
    print(json.dumps(tune(w.make_config(name), prec)))
