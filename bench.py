"""Benchmark of the local model-order-reduction hot path on one MI355X.

Default workload (the serving configuration the metric is quoted on): the 128^3 Kuhn cube with
kappa = 1 and twenty spherical inclusions of kappa = 1e4, cut into 100 boxes of widths 10-40
cells (r = 6), each local reduction one request with a rank in 8..48 and FP32 (+ FP64
refinement) or BF16-split Gram precision drawn with p = 1/2 each.

Setup (untimed): one full epoch of the request stream, so that every subdomain has a basis and
the global projection is defined.  One step = a fixed slice of the request stream (default 4
requests, cycling through a seeded order of the subdomains) submitted at once to the
continuous-batching engine and served to completion (assembly, FP32 block CG with FP64
refinement lifting every interface hat function, Gram/Schur, Cholesky, top-k eigensolve,
stitching, local projection, the basis update), then the memory-efficient projection over all
neighbour pairs and the reduced solve (diagonal-preconditioned CG) with the new bases.
Inputs (mesh, coefficients, decomposition) are resident on the device before timing starts.

The other workloads (--config C1..C4, C6) time the whole batched path per step.

Prints one JSON line: subdomain reductions/s, the SpMM roofline (algorithmic HBM bytes per
launch / average launch time from HIP events on the library's stream), p50/p99 latency of a
Poisson stream, the MFMA roofline of the Gram contraction, the plain FP64 one-at-a-time
comparator on a sample, and the FP64 CPU oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

CONFIG_DEFAULT = "C5"
PRECISION_OF = {"C1": "fp64", "C2": "fp32_refine", "C3": "fp32_refine", "C4": "bf16_split", "C5": "fp32_refine",
                "C6": "fp32_refine"}
WORKLOAD_OF = {
    "C1": "16^3 Kuhn cube, kappa=1, 2x2x2 boxes, r=1, k=8",
    "C2": "48^3 Kuhn cube (117,649 nodes), lognormal kappa sigma=1, 4x4x4 boxes, r=6, k=16",
    "C3": "64^3 jittered Kuhn cube, 6x5x4 random boxes, r=6, k=24",
    "C4": "96^3 Kuhn cube, lognormal kappa sigma=2, 8x8x8 boxes, r=6, k=32",
    "C5": "128^3 Kuhn cube (2,146,689 nodes), kappa=1 with 20 spheres of kappa=1e4, 100 boxes of widths "
          "10-40 cells, r=6, request stream with ranks 8-48, FP32+refinement / BF16-split Gram mixed",
    "C6": "216^3 Kuhn cube (10,218,313 nodes, 9.9M free DOFs), lognormal kappa sigma=1, 18x18x18 boxes, r=6, k=16",
}
STREAM_PRECISIONS = ("fp32_refine", "bf16_split")


def _oracle_box(i):
    """One local reduction by the FP64 oracle (a process-pool task, one BLAS thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import decomp, reduce
    threadpool_limits(1)
    p = _POOL["p"]
    s = decomp.local_sets(p.mesh, p.subdomains, i)
    r = int(p.ranks[i]) if p.ranks is not None else p.rank
    t0 = time.perf_counter()
    if _POOL["implicit"]:
        reduce.reduce_local_implicit(p.mesh, p.kappa, p.f_nodal, s, r)
    else:
        reduce.reduce_local(p.mesh, p.kappa, p.f_nodal, s, r)
    return time.perf_counter() - t0


_POOL = {}


def cpu_baseline(problem, workers: int, implicit: bool):
    """The FP64 oracle's local reduction as a process pool on the host cores, one BLAS thread per
    process, one subdomain per process: the `workers` smallest subdomains (their extended boxes
    by tet count), all started at once.  Must run before the process touches the GPU (the pool
    forks it).  Rate = subdomains / wall time."""
    import multiprocessing as mp

    import numpy as np
    sizes = np.diff(problem.subdomains.ext_tet_ptr)
    ids = [int(i) for i in np.argsort(sizes, kind="stable")[:workers]]
    _POOL.update(p=problem, implicit=implicit)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(ids)) as pool:
        per = pool.map(_oracle_box, ids, chunksize=1)
    el = time.perf_counter() - t0
    route = "sparse-factor pencil route (Lanczos)" if implicit else "dense SVD route"
    return dict(value=round(len(ids) / el, 5), unit="subdomain reductions/s", cores=len(ids), kind="oracle",
                sample=f"process pool of {len(ids)} processes x 1 BLAS thread, one subdomain each: the {len(ids)} "
                       f"smallest subdomains {ids} of {problem.name} (extended-box tets "
                       f"{int(sizes[ids].min())}-{int(sizes[ids].max())}), full FP64 local reduction each "
                       f"({route}), {el:.1f} s wall, per-subdomain {min(per):.1f}-{max(per):.1f} s")


PROFILE_OF = {
    "C2": os.path.join(ROOT, "profiles", "k_cg_spmm_halo_cap96_slice128_48cube_lognormal_fp32refine.md"),
    "C5": os.path.join(ROOT, "profiles", "k_cg_spmm_box_128cube_inclusions_stream.md"),
}


def kernel_source_hash(name: str) -> str:
    """sha256 (16 hex digits) of one kernel's source text in mor_kernels.hip: from its
    `template` line to the closing brace at column 0."""
    import hashlib
    lines = open(os.path.join(ROOT, "paper_2404_06260_amd", "csrc", "mor_kernels.hip")).read().split("\n")
    for i, ln in enumerate(lines):
        if f"void {name}(" in ln and "__global__" in ln:
            b = i - 1 if i > 0 and lines[i - 1].startswith("template") else i
            e = next(j for j in range(i, len(lines)) if lines[j] == "}")
            return hashlib.sha256("\n".join(lines[b:e + 1]).encode()).hexdigest()[:16]
    return ""


def profiled_traffic(kernel: str, config: str, algorithmic_bytes: float):
    """HBM bytes per launch of `kernel`: the committed rocprofv3 summary of this workload gives its
    calibrated FETCH_SIZE + WRITE_SIZE per algorithmic byte over the launches it profiled, applied
    here to this run's algorithmic bytes per launch.  None when there is no summary or the
    kernel's source has changed since the counters were taken."""
    import re
    path = PROFILE_OF.get(config)
    if path is None or not os.path.exists(path):
        return None
    txt = open(path).read()
    base = kernel.split("<")[0]
    m = re.search(base + r" source sha256 ([0-9a-f]{16})", txt)
    if not m or kernel_source_hash(base) != m.group(1):
        return None
    row = re.search(base + r" traffic per algorithmic byte ([0-9.]+)", txt)
    if not row:
        return None
    return round(float(row.group(1)) * algorithmic_bytes)


def comparator_leg(problem, steps: int, reduced_solver: int = 0):
    """The plain FP64 per-subdomain GPU path: FP64 block CG (to the refined path's residual
    target), FP64 Gram and eigensolve, one subdomain per call, no batching; same projection and
    reduced solve.  Returns its reductions/s and the reduced energy x.b~ for comparison."""
    import numpy as np
    import torch
    from paper_2404_06260_amd import mor
    m = mor.Mor(problem, precision="fp64", reduced_solver=reduced_solver)
    n = problem.subdomains.n_sub
    ranks = problem.ranks if problem.ranks is not None else np.full(n, problem.rank)
    try:
        for i in range(n):                      # warm-up: one subdomain
            mor.mor_local_basis(m.ctx, i, int(ranks[i]))
            break
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for i in range(n):
                mor.mor_local_basis(m.ctx, i, int(ranks[i]))
            m.project()
            m.solve()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        bt = mor.mor_get_reduced_load(m.ctx)
        x = mor.mor_get_reduced_solution(m.ctx, bt.size)
        return dict(value=round(n * steps / el, 4), unit="subdomain reductions/s", ms_per_step=round(1e3 * el / steps, 2),
                    path="plain FP64 block CG (residual 1e-8) + FP64 Gram/eigen, one subdomain per call",
                    energy=float(x @ bt))
    finally:
        m.close()


def comparator_sample(problem, sds, ranks, batched_s: float, batched_sigma: dict):
    """The plain FP64 per-subdomain path on a sample of requests (the first timed step's): each
    subdomain alone, FP64 block CG to the refined path's residual target, FP64 Gram and eigensolve.
    Compared with the batched mixed-precision time of the same requests, at equal accuracy: the
    largest relative difference of the kept singular values."""
    import numpy as np
    import torch
    from paper_2404_06260_amd import mor
    m = mor.Mor(problem, precision="fp64")
    try:
        mor.mor_local_basis(m.ctx, int(sds[0]), int(ranks[0]))     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sd, r in zip(sds, ranks):
            mor.mor_local_basis(m.ctx, int(sd), int(r))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        dev = 0.0
        for sd in sds:   # the singular values the truncation read: the kept ones and the next
            s64 = mor.mor_get_sigma(m.ctx, int(sd))
            k = min(mor.mor_get_rank(m.ctx, int(sd))[0] + 1, s64.size)
            sb = batched_sigma[int(sd)][:k]
            dev = max(dev, float(np.max(np.abs(sb - s64[:k]) / s64[:k])))
    finally:
        m.close()
    return dict(value=round(len(sds) / el, 4), unit="subdomain reductions/s",
                path="plain FP64 block CG (residual 1e-8) + FP64 Gram/eigen, one subdomain per call",
                sample=f"the first timed step's requests, subdomains {list(map(int, sds))}",
                batched_value=round(len(sds) / batched_s, 4), speedup_of_batched=round(el / batched_s, 3),
                sigma_max_rel_diff=dev)


def serving_leg(m, problem, n_req: int, load: float, rate: float = 0.0, precisions=("fp32_refine",),
                on_done=None, saturation=None):
    """Continuous-batching serving on the same context: the saturation rate (all requests
    queued at t = 0), then a Poisson stream at `load` times that rate (or at `rate` req/s when
    given, without the saturation run); latency = completion seen - arrival."""
    from paper_2404_06260_amd import serve
    pp = tuple(1.0 / len(precisions) for _ in precisions)
    sat_tp = None
    if rate <= 0:
        sat = serve.run_stream(m.ctx, serve.make_stream(problem, n_req, float("inf"), seed_order=12,
                                                       precisions=precisions, precision_p=pp), on_done=on_done)
        sat_tp = sat.throughput
        rate = load * sat_tp
        print(f"[bench] serving: saturation {sat_tp:.2f} req/s, stream at {rate:.2f} req/s", file=sys.stderr,
              flush=True)
    else:
        sat_tp = saturation
    res = serve.run_stream(m.ctx, serve.make_stream(problem, n_req, rate, seed_arrivals=7, seed_order=11,
                                                    precisions=precisions, precision_p=pp), on_done=on_done)
    pc = res.percentiles((50, 99))
    return {"requests": n_req, "arrivals": "poisson", "rate_per_s": round(rate, 3),
            "precisions": list(precisions),
            "load_vs_saturation": round(rate / sat_tp, 3) if sat_tp else None,
            "saturation_per_s": round(sat_tp, 3) if sat_tp else None,
            "throughput_per_s": round(res.throughput, 3), "p50_ms": round(pc["p50"] * 1e3, 1),
            "p99_ms": round(pc["p99"] * 1e3, 1), "max_live": res.max_live, "peak_bytes": res.peak_bytes,
            "budget_bytes": res.budget_bytes, "failed": int((res.status != 0).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default=CONFIG_DEFAULT)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--spmm-rows", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the CPU-baseline pool (0: min(8, host cores))")
    ap.add_argument("--sketch", type=int, default=0,
                    help="randomized local reduction with this many sketch columns (1..64); 0: explicit SVD")
    ap.add_argument("--graph", type=int, default=-1,
                    help="capture each CG chunk in a HIP graph (1) or launch eagerly (0); -1: graphs for C3")
    ap.add_argument("--no-comparator", action="store_true",
                    help="skip the plain FP64 one-subdomain-at-a-time comparator leg")
    ap.add_argument("--step-requests", type=int, default=4,
                    help="request-stream workload: requests per timed step")
    ap.add_argument("--serve-requests", type=int, default=-1,
                    help="requests in the Poisson serving leg (-1: 40 on the request-stream workload, one per "
                         "subdomain otherwise; 0: no serving leg)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="absolute Poisson arrival rate (req/s) of the serving leg; 0: a fraction of saturation")
    ap.add_argument("--serve-load", type=float, default=0.9,
                    help="Poisson arrival rate of the serving leg as a fraction of the measured saturation rate")
    ap.add_argument("--cg-rtol", type=float, default=0.0,
                    help="inner block-CG tolerance (0: the library default); FP32 paths refine to the same FP64 target")
    ap.add_argument("--box-spmm", type=int, default=0,
                    help="0: the plane-streaming SpMM for box interiors (FP32 systems), -1: the general SpMM only")
    ap.add_argument("--coarse", type=int, default=1,
                    help="block-CG preconditioner: 1 two-level (block Jacobi + coarse correction), 0 block Jacobi")
    ap.add_argument("--reduced-solver", choices=("pcg", "pcg-block", "cholesky"), default="pcg",
                    help="reduced system: the paper's diagonal-preconditioned conjugate gradients on the "
                         "block-sparse matrix, the same with block-Jacobi preconditioning, or a dense FP64 "
                         "Cholesky factorization")
    ap.add_argument("--basis-update", type=int, default=-1,
                    help="1: the basis update of Section 6 step 2 (whitened diagonal blocks, dependent directions "
                         "dropped); -1: on for the inclusions stream (high-contrast coefficient, ranks up to 48, "
                         "whose stitched columns are nearly dependent), off otherwise")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB copied by one plain device copy before the steps (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU sharding of the subdomains is a "
                                   "design note only", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np

    import workloads as w

    stream_wl = args.config == "C5"    # the request-stream workload
    prec = args.precision or PRECISION_OF[args.config]
    p = w.make_config(args.config)
    n_sub = p.subdomains.n_sub
    print(f"[bench] {args.config}: {n_sub} subdomains, precision {prec}", file=sys.stderr, flush=True)
    # the CPU baseline forks a process pool: run it before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(8, os.cpu_count() or 1)
        print(f"[bench] cpu baseline (oracle, {workers} processes)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(p, workers, implicit=stream_wl)
        print(f"[bench] cpu baseline done: {cpu['value']} /s", file=sys.stderr, flush=True)

    import torch
    from paper_2404_06260_amd import mor, serve
    torch.cuda.set_device(0)
    tile = {}
    if not args.spmm_rows:
        from paper_2404_06260_amd import autotune
        tile = autotune.best(p, prec) or {}
        if tile:
            print(f"[bench] autotuned tiles: {tile}", file=sys.stderr, flush=True)
    else:
        tile = dict(spmm_rows=args.spmm_rows)
    use_graph = (args.config == "C3") if args.graph < 0 else bool(args.graph)
    red_solver = {"cholesky": 0, "pcg": 1, "pcg-block": 2}[args.reduced_solver]
    t_create = time.perf_counter()
    extra = {"cg_rtol": args.cg_rtol} if args.cg_rtol > 0 else {}
    extra["coarse"] = args.coarse
    extra["box_spmm"] = args.box_spmm
    basis_update = stream_wl if args.basis_update < 0 else bool(args.basis_update)
    if basis_update:
        extra["basis_update"] = 1
    m = mor.Mor(p, precision=prec, use_graph=int(use_graph), reduced_solver=red_solver, **tile, **extra)
    print(f"[bench] context created ({time.perf_counter() - t_create:.0f} s)", file=sys.stderr, flush=True)
    halo = tile.get("spmm_kind", 0) != 2
    spmm_cap = max([c for c in (48, 64, 96, 128, 176) if c <= tile.get("spmm_rows", 0)] or [96]) if halo else 0
    spmm_cwb = 256 if tile.get("spmm_kind", 0) == 1 else 128   # bytes of a row per column slice
    elt = "double" if prec == "fp64" else "float"
    spmm_kernel = (f"k_cg_spmm_halo<{elt}, {spmm_cap}, {spmm_cwb}>" if halo else
                   f"k_cg_spmm<{elt}, {tile.get('spmm_vec', 4)}>")

    def progress(j, n_done, t):
        print(f"[bench] {n_done} requests served ({t:.0f} s)", file=sys.stderr, flush=True)

    sketches = None
    if args.sketch > 0:   # seeded Gaussian S_i per subdomain, rows in the library's interface order
        sketches = []
        for i in range(n_sub):
            nP, nV, nI, nB = mor.mor_get_sizes(m.ctx, i)
            sketches.append(w.sketch_rows(p.mesh.n_nodes, mor.mor_get_nodes(m.ctx, i)[nI:nI + nB], args.sketch, i))
        sk_ranks = p.ranks if p.ranks is not None else np.full(n_sub, p.rank)

    setup = None
    slices = None
    if stream_wl:
        # setup: one full epoch of the stream (every subdomain reduced once), untimed
        t0 = time.perf_counter()
        ep = serve.run_stream(m.ctx, serve.make_stream(p, n_sub, float("inf"), seed_order=12,
                                                       precisions=STREAM_PRECISIONS, precision_p=(0.5, 0.5)),
                              on_done=lambda j, n, t: n % 10 == 0 and progress(j, n, t))
        if (ep.status != 0).any():
            raise RuntimeError(f"{int((ep.status != 0).sum())} requests of the setup epoch failed")
        m.project()
        m.solve()
        torch.cuda.synchronize()
        setup = {"epoch_requests": n_sub, "epoch_s": round(time.perf_counter() - t0, 2),
                 "epoch_throughput_per_s": round(ep.throughput, 4)}
        print(f"[bench] setup epoch {setup['epoch_s']} s", file=sys.stderr, flush=True)
        # the steps' request slices: a second seeded order of the subdomains, cycling
        S = args.step_requests
        n_req = S * (args.warmup + args.steps)
        full = serve.make_stream(p, n_req, float("inf"), seed_order=13, seed_precision=14,
                                 precisions=STREAM_PRECISIONS, precision_p=(0.5, 0.5))
        slices = [serve.Stream(arrivals=full.arrivals[a:a + S], sds=full.sds[a:a + S], ranks=full.ranks[a:a + S],
                               precisions=full.precisions[a:a + S]) for a in range(0, n_req, S)]
    step_no = [0]

    def step():
        if sketches is not None:
            mor.mor_local_basis_sketched(m.ctx, np.arange(n_sub), sk_ranks, sketches)
        elif stream_wl:
            res = serve.run_stream(m.ctx, slices[step_no[0]])
            if (res.status != 0).any():
                raise RuntimeError(f"{int((res.status != 0).sum())} requests failed")
        elif n_sub > 1000:   # thousands of subdomains: batches of 729 with a progress line after each
            ranks = p.ranks if p.ranks is not None else np.full(n_sub, p.rank)
            t0s = time.perf_counter()
            for a in range(0, n_sub, 729):
                ids = np.arange(a, min(a + 729, n_sub))
                mor.mor_local_basis_batch(m.ctx, ids, ranks[ids].astype(np.int32))
                progress(None, int(ids[-1]) + 1, time.perf_counter() - t0s)
        else:
            m.local_basis_all()
        step_no[0] += 1
        m.project()
        return m.solve()

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    mor.mor_timing_reset(m.ctx)
    mor.mor_timing_enable(m.ctx, True)
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        u, nred = step()
        step_s.append(time.perf_counter() - ts)
        print(f"[bench] step {i} done ({step_s[-1]:.2f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mor.mor_timing_enable(m.ctx, False)
    el = t1 - t0
    ms_per_step = 1e3 * el / args.steps
    per_step = args.step_requests if stream_wl else n_sub
    value = per_step * args.steps / el
    n_launch, spmm_ms, spmm_bytes = mor.mor_timing_get(m.ctx, "spmm")
    nb_l, nb_ms, nb_bytes = mor.mor_timing_get(m.ctx, "spmm_box")
    if nb_l and nb_ms > 0 and nb_bytes >= spmm_bytes:   # the box kernel carried most of the SpMM bytes
        n_launch, spmm_ms, spmm_bytes = nb_l, nb_ms, nb_bytes
        spmm_kernel = "k_cg_spmm_box"
    if use_graph:   # per-kernel events do not exist inside a graph: the whole chunk is the unit
        n_launch, spmm_ms, spmm_bytes = mor.mor_timing_get(m.ctx, "cg_graph")
        spmm_kernel = "CG chunk graph: SpMM + alpha + update + beta + direction"
    avg_ms = spmm_ms / max(n_launch, 1)
    bytes_per_launch = spmm_bytes / max(n_launch, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    kernels = {}
    for name in ("spmm", "spmm_box", "cg_update", "cg_direction", "cg_coarse", "coarse_setup", "cg_graph", "residual64", "assemble", "gram", "gram_split", "gram_bf16",
                 "schur", "potrf", "trsm", "trsm_basis", "eig", "basis", "project_local", "project", "solve",
                 "host_admit", "host_chunk", "host_stage", "host_dense"):
        n, ms, wk = mor.mor_timing_get(m.ctx, name)
        if n:
            kernels[name] = dict(launches=n, ms_per_step=round(ms / args.steps, 3))
            if wk > 0:   # the timer's work: bytes for the streaming kernels, flops for the dense ones
                kernels[name]["work_per_step"] = wk / args.steps
    timed_sds = sorted({int(s) for sl in slices[args.warmup:] for s in sl.sds}) if stream_wl else range(n_sub)
    stats = [mor.mor_get_stats(m.ctx, i) for i in timed_sds]
    _, red_iters, red_rel = mor.mor_get_solve_info(m.ctx)
    n_s, ms_s, _ = mor.mor_timing_get(m.ctx, "solve")
    reduced_solve = {"solver": {0: "dense FP64 Cholesky", 1: "diagonal-preconditioned CG, block-sparse",
                                2: "CG with block-inverse preconditioner, block-sparse"}[red_solver],
                     "iterations": red_iters, "rel_residual": red_rel,
                     "ms": round(ms_s / max(n_s, 1), 3)}
    bt_b = mor.mor_get_reduced_load(m.ctx)
    energy_b = float(mor.mor_get_reduced_solution(m.ctx, bt_b.size) @ bt_b)
    # the dense contraction of the Gram G1 = X_C^T K_i X_C on the matrix cores
    mfma = None
    n_g, ms_g, fl_g = mor.mor_timing_get(m.ctx, "gram_bf16")
    peak, kname = 2500.0, "k_gram_bf16 (BF16 hi/lo split, 3 products)"
    if not n_g:
        n_g, ms_g, fl_g = mor.mor_timing_get(m.ctx, "gram")
        peak, kname = 78.6, "k_gemm (FP64 MFMA)"
    if n_g and ms_g > 0:
        tf = fl_g / (ms_g * 1e-3) / 1e12
        mfma = {"bound": "mfma", "kernel": kname, "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tf / peak, 4), "flops_per_step": fl_g / args.steps}
    # the comparator sample (request-stream workload): the first timed step's requests
    cmp_sample = None
    if stream_wl and not args.no_comparator:
        sl = slices[args.warmup]
        cmp_sample = (sl.sds, sl.ranks, step_s[0], {int(s): mor.mor_get_sigma(m.ctx, int(s)) for s in sl.sds})
    serving = None
    if args.serve_requests != 0:
        n_serve = args.serve_requests if args.serve_requests > 0 else (40 if stream_wl else n_sub)
        rate, sat = args.serve_rate, None
        if stream_wl and rate <= 0:   # the timed steps measured the saturated rate already
            sat = value
            rate = args.serve_load * sat
        serving = serving_leg(m, p, n_serve, args.serve_load, rate=rate,
                              precisions=STREAM_PRECISIONS if stream_wl else ("fp32_refine",),
                              on_done=(lambda j, n, t: n % 10 == 0 and progress(j, n, t)) if stream_wl else None,
                              saturation=sat)
    m.close()
    torch.cuda.empty_cache()   # the context's memory back to the device for the comparator's budget
    comparator = None
    if not args.no_comparator and prec != "fp64":
        print("[bench] comparator: plain FP64 per-subdomain path", file=sys.stderr, flush=True)
        if stream_wl:
            comparator = comparator_sample(p, *cmp_sample)
        else:
            comparator = comparator_leg(p, 1, red_solver)
            comparator["speedup_of_value"] = round(value / comparator["value"], 3)
            comparator["energy_rel_diff"] = abs(comparator.pop("energy") - energy_b) / abs(energy_b)
    cfg = {"workload": WORKLOAD_OF[args.config], "name": args.config, "subdomains": n_sub,
           "precision": "fp32_refine | bf16_split, p = 1/2 each" if stream_wl else prec,
           "reduced_dim": int(nred), "hip_graph": use_graph,
           "cg_preconditioner": "block Jacobi + coarse correction" if args.coarse else "block Jacobi",
           "basis_update": basis_update,
           "local_svd": f"randomized, {args.sketch} sketch columns" if sketches is not None else "explicit",
           "tiles": tile or "library defaults"}
    if stream_wl:
        cfg["step"] = (f"{args.step_requests} requests of the stream served to completion by the continuous-batching "
                       f"engine, then projection over all {n_sub} subdomains and the reduced solve")
        cfg["setup"] = setup
    out = {
        "metric": "subdomain reductions/s",
        "value": round(value, 4),
        "unit": "subdomain reductions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64+bf16" if stream_wl else {"fp64": "f64", "fp32_refine": "f32+f64", "fp32": "f32",
                                                   "bf16_split": "f32+f64+bf16"}[prec],
        "data": "synthetic",
        "config": cfg,
        "roofline": {"bound": "hbm",
                     "kernel": spmm_kernel if use_graph else f"{spmm_kernel} (block-CG SpMM Q = A_II P)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(spmm_kernel, args.config, bytes_per_launch) if not use_graph else None,
                     "traffic_unit": "bytes per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE (calibrated) per algorithmic "
                                     "byte of the profiled launches, times this run's algorithmic bytes per launch",
                     "avg_launch_ms": round(avg_ms, 4), "launches": n_launch,
                     "algorithmic_bytes_per_launch": round(bytes_per_launch)},
        "cpu_baseline": cpu,
        "serving": serving,
        "comparator": comparator,
        "mfma": mfma,
        "kernels": kernels,
        "reduced_energy": energy_b,   # x^T b~ = ||u~||_A^2 (larger = closer to the FE solution)
        "reduced_solve": reduced_solve,
        "cg_iters_max": [max(s["cg_iter_a"] for s in stats), max(s["cg_iter_k"] for s in stats)],
        "eig_iters_max": max(s["eig_iter"] for s in stats),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
