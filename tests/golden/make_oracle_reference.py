"""Write the FP64 oracle's results for a named workload to tests/golden/<name>_oracle.npz.

Calls only `oracle/` (and the seeded input generators); the GPU tests compare the HIP path's
full-size output with this file.  Usage:
    python tests/golden/make_oracle_reference.py C2 [workers] [options]
Options:
  --no-fe          skip the full FE solve (a sparse direct factorisation of the global matrix,
                   out of reach for the larger meshes); the file then holds the reduced solution
  --implicit       local reductions through the sparse factors of the pencil (Z^T K_i Z, S_B)
                   instead of dense matrices (subdomains with tens of thousands of nodes)
  --update-drop=D  the basis update of Section 6, step 2 on every local basis, relative drop D
  --pcg            reduced solve by the paper's diagonal-preconditioned conjugate gradients (to
                   the relative residual below) instead of a Cholesky factorization
  --u32            store u~ in float32 (its rounding, 6e-8 relative per entry, stays far below
                   the tolerances the tests apply; keeps the file small at 2 million nodes)
The file also records the iterations the oracle's reduced conjugate gradients (diagonal
preconditioner, Section 6 step 3) take to a relative residual of 1e-12 on the oracle's reduced
system, and each subdomain's basis dimension after the optional update.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from oracle import project, solve  # noqa: E402

PCG_RTOL = 1e-12


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    flags = [a for a in sys.argv[1:] if a.startswith("--")]
    with_fe = "--no-fe" not in flags
    implicit = "--implicit" in flags
    use_pcg = "--pcg" in flags
    u32 = "--u32" in flags
    drop = next((float(f.split("=", 1)[1]) for f in flags if f.startswith("--update-drop=")), None)
    name = args[0] if args else "C2"
    workers = int(args[1]) if len(args) > 1 else (os.cpu_count() or 1)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    p = w.make_config(name)
    t0 = time.time()
    sizes = np.diff(p.subdomains.ext_tet_ptr)
    out = solve.run(p, workers=workers, with_fe=with_fe, implicit=implicit, update_drop=drop,
                    pcg_rtol=PCG_RTOL if use_pcg else None, order=list(np.argsort(-sizes)))
    res = out["local"]
    kmax = max(r.k_eff for r in res) + 1
    sig = np.zeros((len(res), kmax + 8))
    for i, r in enumerate(res):
        n = min(sig.shape[1], r.sigma.size)
        sig[i, :n] = r.sigma[:n]
    if out["pcg_iters"] is not None:
        pcg_iters = out["pcg_iters"]
    else:
        _, pcg_iters, _ = project.pcg_diag(out["At"], out["bt"], rtol=PCG_RTOL)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.npz")
    extra = dict(u_fe=out["u_fe"], red_err=out["red_err"], u_energy=out["u_energy"]) if with_fe else {}
    ut = out["u_tilde"].astype(np.float32) if u32 else out["u_tilde"]
    np.savez_compressed(path, u_tilde=ut, x=out["x"], bt=out["bt"],
                        k_eff=np.array([r.k_eff for r in res]), sigma=sig, pcg_iters=pcg_iters,
                        pcg_rtol=PCG_RTOL, dim=np.array([r.Vloc.shape[1] for r in out["results"]]),
                        update_drop=-1.0 if drop is None else drop, reduced_pcg=int(use_pcg),
                        implicit=int(implicit), **extra)
    msg = f", relative reduction error {out['red_err'] / out['u_energy']:.3e}" if with_fe else ""
    print(f"{name}: {len(res)} subdomains, reduced dim {out['x'].size}{msg}, reduced PCG {pcg_iters} iterations, "
          f"{time.time() - t0:.0f} s -> {path}")


if __name__ == "__main__":
    main()
