"""Benchmark: Trotter steps/s of the MPO-TEBD Lindblad step on one MI355X.

Workload (the configuration the headline metric is quoted on): an N=30 open
chain of driven, dissipative qubits with alternating detunings 0/5 plus
N(0, 0.1^2) jitter and couplings J ~ U[0.8, 1.2] (seed 0), edge drive
Omega=1, g0=0.1, g2=0.05; tau=0.05, chi_max=256, cutoff 1e-10, second-order
Trotter, from the all-"+x" product state.  A step is one full Trotter step of
the hot path (centre hops, contraction + gate, truncated SVD, canonical
update, trace renormalisation).  `value` is steps/s of the FP32-contraction
form over the timed steps (inputs resident in HBM); the FP64 form is timed
the same way beside it, and the maximum observable difference between the
two is reported.

Warm-up runs W steps on a separate chain; the timed run starts a fresh chain
at t=0 and times exactly K steps (default 50 = the whole configured run).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Trotter steps/s at N=30 χ=256 (FP32-MFMA vs FP64) at ≤1e-5 obs error"
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 (matrix and vector)


def zz(ch):
    import numpy as np

    z1, z2 = ch.zz_observables()
    return np.concatenate([z1, z2])


def timed_run(model, run, precision, steps, warmup):
    import numpy as np
    import torch

    from paper_2203_05871_amd import Chain

    if warmup > 0:
        w = Chain(model, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
        w.evolve(warmup)
        w.sync()
        w.close()
    ch = Chain(model, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
    torch.cuda.synchronize()
    ch.profile_begin(200 * steps)
    t0 = time.perf_counter()
    ch.evolve(steps)
    ch.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, svd_ms, svd_flops = ch.profile_end()
    obs = zz(ch)
    dims = ch.bond_dims()
    stats = ch.svd_stats()
    tr = ch.trace()
    ch.close()
    return {"seconds": dt, "launches": launches, "svd_ms": svd_ms, "svd_flops": svd_flops, "obs": obs,
            "dims": dims, "sweeps": stats[2], "svds": stats[3], "trace": tr}


def cpu_baseline(model, run, steps, budget_s):
    """The FP64 oracle on the host cores: as many of the same steps as fit in
    the time budget (a bounded sample of the same trajectory)."""
    import numpy as np

    from oracle import tebd

    mps = tebd.MPS.product(run["init"], model["N"])
    gates = tebd.gate_tables(model, run["tau"])
    t0 = time.perf_counter()
    done = 0
    for n in range(steps):
        tebd.evolve(mps, model, run["tau"], 1, run["chi_max"], run["cutoff"], gates=gates, first_step=n)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    obs = None
    if done == steps:
        z1, z2 = tebd.zz_observables(mps)
        obs = np.concatenate([z1, z2])
    return done, dt, obs


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--cpu-budget", type=float, default=25.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--init", default="+x")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): a single chain's Trotter step is a "
              "strictly sequential chain of gates; multi-GPU sharding is described in DESIGN.md, not run.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    model, run = workloads.c3(args.init)
    K, W = args.steps, args.warmup
    res = {}
    for prec in (["fp32", "fp64"] if args.precision == "both" else [args.precision]):
        res[prec] = timed_run(model, run, prec, K, W)
        r = res[prec]
        print(f"# {prec}: {K} steps in {r['seconds']:.2f} s, SVD launches {r['launches']}, "
              f"kernel {r['svd_ms']:.0f} ms, max chi {max(r['dims'])}, sweeps/svd {r['sweeps'] / max(1, r['svds']):.1f}",
              file=sys.stderr, flush=True)
    head = "fp32" if "fp32" in res else "fp64"
    h = res[head]
    value = K / h["seconds"]
    # roofline of the dominant kernel (the persistent truncated SVD)
    achieved = h["svd_flops"] / (h["svd_ms"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": "svd_persistent_kernel", "achieved": achieved,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": None, "launches": h["launches"],
                "avg_launch_ms": h["svd_ms"] / max(1, h["launches"]),
                "flops_per_launch": h["svd_flops"] / max(1, h["launches"]),
                "kernel_share_of_step": h["svd_ms"] * 1e-3 / h["seconds"]}
    line = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * h["seconds"] / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 contraction + fp64 svd" if head == "fp32" else "fp64",
        "data": "synthetic (seeded driven-dissipative chain, no dataset)",
        "config": {"workload": f"N=30 jittered XY chain, chi_max=256, cutoff=1e-10, tau=0.05, "
                               f"{K} steps from {args.init}", "N": 30, "chi_max": 256, "cutoff": 1e-10,
                   "tau": 0.05, "init": args.init, "max_chi_reached": int(max(h["dims"]))},
        "roofline": roofline,
    }
    if "fp32" in res and "fp64" in res:
        line["fp64_steps_per_s"] = K / res["fp64"]["seconds"]
        line["obs_err_fp32_vs_fp64"] = float(np.abs(res["fp32"]["obs"] - res["fp64"]["obs"]).max())
    if not args.no_cpu:
        done, dt, obs = cpu_baseline(model, run, K, args.cpu_budget)
        line["cpu_baseline"] = {"value": done / dt, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                                "sample": f"first {done} of the {K} timed steps (FP64 NumPy/LAPACK oracle)"}
        if obs is not None:
            ref = res["fp64"]["obs"] if "fp64" in res else h["obs"]
            line["obs_err_fp64_vs_oracle"] = float(np.abs(ref - obs).max())
            if "fp32" in res:
                line["obs_err_fp32_vs_oracle"] = float(np.abs(res["fp32"]["obs"] - obs).max())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
