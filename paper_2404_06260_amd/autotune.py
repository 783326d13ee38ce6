"""Autotuner for the block-CG SpMM tile: width (64, 128 or 256 columns) and rows per tile.

Each candidate runs the batched local reduction of a workload with a loose CG tolerance (a
few dozen iterations of the real kernels on the real matrices) and is timed with the
library's HIP-event timer on its stream; the candidate with the highest algorithmic SpMM
bandwidth wins.  Results are cached per device name and workload in a JSON file next to
this module, and `best()` returns the cached choice (or None).
"""
from __future__ import annotations

import json
import os

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
CANDIDATES = [(4, 4), (4, 8), (4, 16), (2, 8), (2, 16)]


def _key(problem, precision):
    import torch
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{problem.name}|{problem.subdomains.n_sub}|{precision}"


def best(problem, precision):
    if not os.path.exists(CACHE):
        return None
    try:
        d = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    r = d.get(_key(problem, precision))
    return None if r is None else (int(r["spmm_vec"]), int(r["spmm_rows"]))


def tune(problem, precision="fp32_refine", candidates=CANDIDATES, sub_ids=None, verbose=True, save=True):
    import numpy as np
    from . import mor
    cg_prec = "fp64" if precision == "fp64" else "fp32"
    results = []
    ids = np.arange(problem.subdomains.n_sub) if sub_ids is None else np.asarray(sub_ids)
    for v, rb in candidates:
        if cg_prec == "fp64" and v > 2:
            continue
        m = mor.Mor(problem, precision=cg_prec, spmm_vec=v, spmm_rows=rb, cg_rtol=1e-2, refine_rtol=1e-2)
        try:
            mor.mor_timing_enable(m.ctx, True)
            ranks = np.full(ids.size, problem.rank, dtype=np.int32)
            mor.mor_local_basis_batch(m.ctx, ids, ranks)
            n, ms, by = mor.mor_timing_get(m.ctx, "spmm")
        finally:
            m.close()
        gbs = (by / n) / (ms / n * 1e-3) / 1e9 if n and ms > 0 else 0.0
        results.append(dict(spmm_vec=v, spmm_rows=rb, launches=n, avg_ms=ms / max(n, 1), gbs=gbs))
        if verbose:
            print(f"[autotune] v={v} rows={rb}: {n} launches, {ms / max(n, 1):.3f} ms avg, {gbs:.0f} GB/s", flush=True)
    win = max(results, key=lambda r: r["gbs"])
    if save:
        d = {}
        if os.path.exists(CACHE):
            try:
                d = json.load(open(CACHE))
            except (OSError, ValueError):
                d = {}
        d[_key(problem, precision)] = dict(win, all=results)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    return win, results


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as w
    name = sys.argv[1] if len(sys.argv) > 1 else "C2"
    prec = sys.argv[2] if len(sys.argv) > 2 else "fp32_refine"
    win, _ = tune(w.make_config(name), prec)
    print(json.dumps(win))
