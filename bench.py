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
Under the 1e-10 cutoff chi stays well below 256 on this trajectory, so the
line also carries `saturated`: the same chain with cutoff 0, whose interior
bonds sit at chi_max = 256 after two steps, timed over two steps once settled
(FP32-contraction form), with the SVD kernel's roofline at that shape.  The
real-arithmetic Pauli-basis form (opt-in, exact because every propagator is
real in that basis) is timed the same way and reported on its own
(`real_steps_per_s`, with its observable difference to the complex FP64 run).
`gradient` times the adjoint parameter gradients of one observable on the
2 x 8 ladder against that ladder's forward run (gradient_leg).
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


def chi_per_step(model, run, precision, steps):
    """Largest bond dimension after every step (an untimed pass: it reads the
    bond dims after each step)."""
    from paper_2203_05871_amd import Chain

    ch = Chain(model, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
    out = []
    for _ in range(steps):
        ch.evolve(1)
        out.append(int(max(ch.bond_dims())))
    ch.close()
    return out


def saturated_run(model, run, precision, settle, steps):
    """The chain with cutoff 0 (chi_max binds in the bulk): `settle` untimed
    steps, then `steps` timed ones."""
    import torch

    from paper_2203_05871_amd import Chain

    ch = Chain(model, run["tau"], run["chi_max"], 0.0, precision, run["init"])
    ch.evolve(settle)
    ch.sync()
    torch.cuda.synchronize()
    ch.profile_begin(200 * steps)
    t0 = time.perf_counter()
    ch.evolve(steps)
    ch.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, svd_ms, svd_flops = ch.profile_end()
    dims = ch.bond_dims()
    ch.close()
    return {"seconds": dt, "launches": launches, "svd_ms": svd_ms, "svd_flops": svd_flops, "dims": dims}


def timed_batch(models, run, steps, warmup, sequential):
    """The 64-chain workload in the batched form (one launch per Trotter layer over all chains), and
    optionally the same chains run one after another through the single-chain
    path (the plain FP64 GPU path) for comparison."""
    import torch

    from paper_2203_05871_amd import Batch, Chain

    def make():
        return [Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"]) for m in models]

    if warmup > 0:
        # the warm-up batch runs the whole trajectory with the online autotuner on,
        # so every block-size bucket the timed run meets is already tuned
        w = make()
        wb = Batch(w)
        wb.set_autotune(True)
        wb.evolve(max(warmup, steps))
        wb.sync()
        wb.close()
        for c in w:
            c.close()
    chains = make()
    b = Batch(chains)
    torch.cuda.synchronize()
    b.profile_begin(3 * steps + 3)
    t0 = time.perf_counter()
    b.evolve(steps)
    b.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, ms, flops = b.profile_end()
    plan = b.plan()
    out = {"seconds": dt, "launches": launches, "kernel_ms": ms, "flops": flops, "plan": plan,
           "tuning": Batch.tuning_table(),
           "obs": [zz(c) for c in chains], "max_chi": max(max(c.bond_dims()) for c in chains)}
    b.close()
    for c in chains:
        c.close()
    if sequential:
        chains = make()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in chains:
            c.evolve(steps)
        for c in chains:
            c.sync()
        torch.cuda.synchronize()
        out["sequential_seconds"] = time.perf_counter() - t0
        out["sequential_obs"] = [zz(c) for c in chains]
        for c in chains:
            c.close()
    return out


def bench_batch(args):
    """Batched form on the 64-chain workload (a separate line from the
    headline, printed with --workload chains64)."""
    import numpy as np

    import workloads

    models, run = workloads.chains64_uneven()
    K, W = args.steps, args.warmup
    r = timed_batch(models, run, K, W, sequential=not args.no_sequential)
    value = K / r["seconds"]
    achieved = r["flops"] / (r["kernel_ms"] * 1e-3) / 1e12
    line = {
        "metric": "Trotter steps/s of the whole 64-chain batch (batched form, FP64)", "value": value,
        "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": 1e3 * r["seconds"] / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded uneven chains, no dataset)",
        "config": {"workload": f"64 chains, N~U{{8..24}}, Omega~U[0.5,2], Delta~U[2,8], chi_max=64, cutoff=1e-12, "
                               f"tau=0.05, {K} steps from {run['init']}", "chains": len(models),
                   "max_chi_reached": int(r["max_chi"]), "workgroups": int(r["plan"].sum()),
                   "autotuned_caps": {f"C<=2^{b}": cap for b, _, cap, _ in r["tuning"]}},
        "roofline": {"bound": "mfma", "kernel": "batch_layer_kernel", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": None, "launches": r["launches"],
                     "avg_launch_ms": r["kernel_ms"] / max(1, r["launches"]),
                     "flops_per_launch": r["flops"] / max(1, r["launches"])},
    }
    if "sequential_seconds" in r:
        line["sequential_single_chain_steps_per_s"] = K / r["sequential_seconds"]
        line["speedup_vs_sequential"] = r["sequential_seconds"] / r["seconds"]
        line["batch_vs_sequential_max_obs_diff"] = float(max(np.abs(a - b).max() for a, b in
                                                             zip(r["obs"], r["sequential_obs"])))
    if not args.no_cpu:
        # oracle on a bounded sample: the first chains, all K steps each, until the budget is spent
        from oracle import tebd

        t0 = time.perf_counter()
        done_chains = 0
        worst = 0.0
        for c, m in enumerate(models):
            mps = tebd.MPS.product(run["init"], m["N"])
            gates = tebd.gate_tables(m, run["tau"])
            tebd.evolve(mps, m, run["tau"], K, run["chi_max"], run["cutoff"], gates=gates)
            z1, z2 = tebd.zz_observables(mps)
            worst = max(worst, float(np.abs(np.concatenate([z1, z2]) - r["obs"][c]).max()))
            done_chains += 1
            if time.perf_counter() - t0 > args.cpu_budget:
                break
        dt = time.perf_counter() - t0
        # steps/s of the whole batch, extrapolated from the sampled chains' share of the sites
        frac = sum(m["N"] for m in models[:done_chains]) / sum(m["N"] for m in models)
        line["cpu_baseline"] = {"value": K * frac / dt, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                                "sample": f"first {done_chains} of {len(models)} chains, all {K} steps; "
                                          f"batch rate scaled by their share of the sites"}
        line["obs_err_vs_oracle_sampled"] = worst
    print(json.dumps(line), flush=True)


def gradient_leg(cpu_budget, no_cpu, connected=False):
    """Adjoint parameter gradients on the 2 x 8 ladder (N=16, 22 bonds: 8 rungs
    and 14 legs through the SWAP network), chi_max 128, cutoff 1e-12, tau 0.05,
    40 steps from +z: F = <sigma^z_15>(T), the far corner from the drive, and
    all 6N + 2 n_bonds = 140 derivatives in one lmpo_grad_run (state forward,
    replay, co-state backward), against the forward run alone; central
    differences of the GPU forward (h = 1e-5) on a few parameters as a check.
    With `connected`, also the connected correlator <Z_0 Z_15> - <Z_0><Z_15>
    (one more backward pass from its four-term co-state) and the second Renyi
    entropy S_2(T) (real-arithmetic form; its co-state starts from the state)."""
    import numpy as np
    import torch

    import workloads
    from paper_2203_05871_amd import Chain, Gradient

    m, run = workloads.ladder2x8()
    tau, steps, chi, cut, init = run["tau"], run["steps"], run["chi_max"], run["cutoff"], run["init"]
    site, pauli = 15, "Z"

    def forward(model):
        c = Chain(model, tau, chi, cut, "fp64", init, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.evolve(steps)
        c.sync()
        dt = time.perf_counter() - t0
        v = c.measure_1q([site], pauli)[0].real
        c.close()
        return v, dt

    forward(m)  # warm-up (module load, first launches)
    F0, tf = forward(m)
    c = Chain(m, tau, chi, cut, "fp64", init, device="cuda:0")
    G = Gradient(c, steps)
    G.costate_profile_begin(40000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, g = G.run(site, pauli)
    tg = time.perf_counter() - t0
    launches, co_ms, co_flops = G.costate_profile_end()
    co_dims, st_dims = G.costate_dims(), c.bond_dims()
    G.close()
    c.close()
    fd = {}
    # the drive and parameters acting on the observed qubit (far ones give derivatives
    # near 1e-7 at T = 2, below what differences of the truncated forward resolve)
    near = [b for b, (i, j) in enumerate(np.asarray(m["bonds"])) if site in (i, j)]
    for key, idx in (("hx", 0), ("hz", site), ("g0", site), ("J", near[0])):
        vals = []
        for sgn in (1.0, -1.0):
            mm = {k: (np.array(v, dtype=float) if k != "bonds" and isinstance(v, np.ndarray) else v)
                  for k, v in m.items()}
            mm[key][idx] += sgn * 1e-5
            vals.append(forward(mm)[0])
        fd[f"{key}[{idx}]"] = {"adjoint": float(g[key][idx]), "central_difference": (vals[0] - vals[1]) / 2e-5}
    gmax = max(float(np.abs(v).max()) for v in g.values())

    def forty(gr):
        # the 40 numbers of the ladder case: 16 h_z, 22 J, Omega = h_x[0], one g0 shared by all qubits
        return {"hz": [float(x) for x in gr["hz"]], "J": [float(x) for x in gr["J"]], "Omega": float(gr["hx"][0]),
                "g0_uniform": float(np.sum(gr["g0"]))}

    out = {"workload": "2x8 ladder (N=16, 8 rungs + 14 legs via SWAP gates), chi_max=128, cutoff=1e-12, tau=0.05, "
                       "40 steps from +z; F = <sigma^z_15>(T); co-state with the same chi_max and cutoff",
           "parameters": int(sum(len(v) for k, v in g.items() if k != "tau")), "dF_dtau": float(g["tau"][0]),
           "scaling_identity": {"sum_theta_dF": float(sum(np.dot(np.asarray(m[k], dtype=float), g[k])
                                                          for k in g if k != "tau")),
                                "tau_dF_dtau": float(tau * g["tau"][0])},
           "seconds": tg, "forward_seconds": tf,
           "gradient_over_forward": tg / tf, "F": F.real, "F_forward_only": F0, "max_abs_gradient": gmax,
           "state_bond_dims_T": st_dims, "costate_bond_dims_t0": co_dims,
           "roofline": {"bound": "mfma", "kernel": "svd_persistent_kernel (co-state, real form)",
                        "achieved": co_flops / (co_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": co_flops / (co_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "traffic": None, "launches": launches, "avg_launch_ms": co_ms / max(1, launches),
                        "flops_per_launch": co_flops / max(1, launches), "kernel_share_of_gradient":
                            co_ms * 1e-3 / tg},
           "fd_check_h1e-5": fd, "derivatives": forty(g),
           "fd_max_abs_diff": max(abs(v["adjoint"] - v["central_difference"]) for v in fd.values())}
    print(f"# gradient: {tg:.1f} s vs forward {tf:.2f} s", file=sys.stderr, flush=True)
    if connected:
        # the same gradient with every step's gate snapshots kept from the forward run (no replay)
        c = Chain(m, tau, chi, cut, "fp64", init, device="cuda:0")
        G = Gradient(c, steps, keep_gates=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fk, gk = G.run(site, pauli)
        out["keep_gates"] = {"seconds": time.perf_counter() - t0,
                             "arena_GB": G.arena.numel() / 1e9,
                             "same_result": bool(Fk == F and all(np.array_equal(gk[k], g[k]) for k in g))}
        G.close()
        c.close()
        c = Chain(m, tau, chi, cut, "fp64", init, device="cuda:0")
        G = Gradient(c, steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, gc = G.run_connected(0, 15, "ZZ")
        out["connected_zz_0_15"] = {"C": C.real, "seconds": time.perf_counter() - t0,
                                    "max_abs_gradient": max(float(np.abs(v).max()) for v in gc.values()),
                                    "costate_bond_dims_t0": G.costate_dims(), "derivatives": forty(gc)}
        G.close()
        c.close()
        # the second Renyi entropy S_2(T): its co-state starts as the state itself
        # (real-arithmetic form, so the copy is exact), checked against central
        # differences of the real-form forward on the drive and one decay rate
        def renyi_forward(model):
            cr = Chain(model, tau, chi, cut, "real", init, device="cuda:0")
            cr.evolve(steps)
            v = cr.renyi2()
            cr.close()
            return v

        c = Chain(m, tau, chi, cut, "real", init, device="cuda:0")
        G = Gradient(c, steps, series=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S2, gs = G.run_renyi2()
        ts = time.perf_counter() - t0
        fd2 = {}
        for key, idx in (("hx", 0), ("g0", 0)):
            vals = []
            for sgn in (1.0, -1.0):
                mm = {k: (np.array(v, dtype=float) if k != "bonds" and isinstance(v, np.ndarray) else v)
                      for k, v in m.items()}
                mm[key][idx] += sgn * 1e-5
                vals.append(renyi_forward(mm))
            fd2[f"{key}[{idx}]"] = {"adjoint": float(gs[key][idx]), "central_difference": (vals[0] - vals[1]) / 2e-5}
        out["renyi2"] = {"S2": S2, "seconds": ts, "arena_GB": G.arena.numel() / 1e9,
                         "state_bond_dims_T": c.bond_dims(), "costate_bond_dims_t0": G.costate_dims(),
                         "max_abs_gradient": max(float(np.abs(v).max()) for v in gs.values()),
                         "scaling_identity": {"sum_theta_dS2": float(sum(np.dot(np.asarray(m[k], dtype=float), gs[k])
                                                                        for k in gs if k != "tau")),
                                              "tau_dS2_dtau": float(tau * gs["tau"][0])},
                         "fd_check_h1e-5": fd2, "derivatives": forty(gs)}
        G.close()
        c.close()
        print(f"# Renyi-2 gradient: {ts:.1f} s", file=sys.stderr, flush=True)
    if not no_cpu:
        # oracle on a bounded sample: the whole gradient after the first n
        # steps, n doubling while the budget lasts; the GPU runs the same n
        from oracle import adjoint

        n, dt, t_all = 0, 0.0, time.perf_counter()
        while n < steps and time.perf_counter() - t_all < cpu_budget:
            nn = 1 if n == 0 else min(2 * n, steps)
            t0 = time.perf_counter()
            adjoint.gradient(m, tau, nn, chi, cut, init, site, pauli)
            n, dt = nn, time.perf_counter() - t0
        c = Chain(m, tau, chi, cut, "fp64", init, device="cuda:0")
        G = Gradient(c, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.run(site, pauli)
        tgn = time.perf_counter() - t0
        G.close()
        c.close()
        out["cpu_baseline"] = {"value": n / dt, "unit": "gradient steps/s (forward + backward)",
                               "cores": blas_threads(), "kind": "oracle",
                               "sample": f"the gradient after the first {n} of the 40 steps"}
        out["gpu_same_sample"] = {"value": n / tgn, "unit": "gradient steps/s (forward + backward)",
                                  "seconds": tgn}
        out["gpu_steps_per_s"] = steps / tg
    return out


def cpu_baseline(model, run, steps, budget_s, threads=None):
    """The FP64 oracle on the host cores: as many of the same steps as fit in
    the time budget (a bounded sample of the same trajectory); `threads`
    limits the BLAS threads."""
    if threads is not None:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=threads):
            return cpu_baseline(model, run, steps, budget_s)
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "svd_persistent_chain30_traffic.json")


def measured_traffic():
    """HBM bytes per SVD launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (scaled by a plain copy of known size), or None once the kernel
    sources differ from the ones the counters were taken on."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for rel in rec["sources"]:
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return rec
    except (OSError, KeyError, ValueError):
        return None


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
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's run, 50 or 40)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--cpu-budget", type=float, default=25.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--init", default="+x")
    ap.add_argument("--workload", choices=["chain30", "chains64", "ladder_grad"], default="chain30",
                    help="chain30: N=30 chain at chi_max=256 (headline); chains64: 64 uneven chains, batched form")
    ap.add_argument("--no-sequential", action="store_true", help="chains64: skip the sequential single-chain run")
    ap.add_argument("--no-saturated", action="store_true", help="chain30: skip the cutoff-0 run at chi = 256")
    ap.add_argument("--no-real", action="store_true", help="chain30: skip the real-arithmetic form")
    ap.add_argument("--no-variants", action="store_true",
                    help="chain30: skip the +z variant and the per-step chi profiles")
    ap.add_argument("--no-gradient", action="store_true", help="chain30: skip the adjoint-gradient leg (2x8 ladder)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (the calibration kernel of "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): a single chain's Trotter step is a "
              "strictly sequential chain of gates; sharding over several GPUs is not run.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {args.copy_probe} MiB read + written", file=sys.stderr, flush=True)
        del src, dst
    # context for the HBM roofline: a plain 1 GiB device copy (read + write);
    # skipped in counter runs, whose calibration is the probe copy above
    copy_gbps = None
    if args.copy_probe == 0:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        copy_gbps = 5 * 2 * (1 << 30) / (time.perf_counter() - t0) / 1e9
        del src, dst
    # and of the FP64 matrix-core peak: the library's MFMA throughput probe
    from paper_2203_05871_amd.lmpo import measured_fp64_mfma_peak

    mfma_tflops = measured_fp64_mfma_peak() if args.copy_probe == 0 else None
    if args.workload == "chains64":
        if args.steps is None:
            args.steps = 40
        return bench_batch(args)
    if args.workload == "ladder_grad":
        g = gradient_leg(args.cpu_budget, args.no_cpu, connected=True)
        line = {"metric": "adjoint gradients (140 parameters) per second, 2x8 ladder", "value": 1.0 / g["seconds"],
                "unit": "gradients/s", "n_gpus": 1, "steps": 40, "warmup": 1,
                "ms_per_step": 1e3 * g["seconds"] / 40, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64", "data": "synthetic (the 2x8 ladder model, no dataset)",
                "config": {"workload": g["workload"]}, "roofline": g["roofline"], "gradient": g}
        if "cpu_baseline" in g:
            line["cpu_baseline"] = g["cpu_baseline"]
        print(json.dumps(line), flush=True)
        return
    if args.steps is None:
        args.steps = 50
    model, run = workloads.chain30_jittered(args.init)
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
    tr = measured_traffic()
    roofline = {"bound": "mfma", "kernel": "svd_persistent_kernel", "achieved": achieved,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": tr["hbm_bytes_per_launch"] if tr else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                "launches": h["launches"],
                "avg_launch_ms": h["svd_ms"] / max(1, h["launches"]),
                "flops_per_launch": h["svd_flops"] / max(1, h["launches"]),
                "kernel_share_of_step": h["svd_ms"] * 1e-3 / h["seconds"],
                "measured_copy_GBps": copy_gbps, "measured_fp64_mfma_TFLOPs": mfma_tflops}
    line = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * h["seconds"] / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 contraction + fp64 svd" if head == "fp32" else "fp64",
        "data": "synthetic (seeded driven-dissipative chain, no dataset)",
        "config": {"workload": f"N=30 jittered XY chain, chi_max=256, cutoff=1e-10, tau=0.05, "
                               f"{K} steps from {args.init}", "N": 30, "chi_max": 256, "cutoff": 1e-10,
                   "tau": 0.05, "init": args.init, "max_chi_reached": int(max(h["dims"])),
                   "bond_dims_final": [int(d) for d in h["dims"]]},
        "roofline": roofline,
    }
    if "fp32" in res and "fp64" in res:
        line["fp64_steps_per_s"] = K / res["fp64"]["seconds"]
        line["obs_err_fp32_vs_fp64"] = float(np.abs(res["fp32"]["obs"] - res["fp64"]["obs"]).max())
    if not args.no_real and "fp64" in res:
        rr = timed_run(model, run, "real", K, W)
        line["real_steps_per_s"] = K / rr["seconds"]
        line["obs_err_real_vs_fp64"] = float(np.abs(rr["obs"] - res["fp64"]["obs"]).max())
        print(f"# real: {K} steps in {rr['seconds']:.2f} s", file=sys.stderr, flush=True)
    if not args.no_variants:
        # the edge-driven variant (+z) beside the global quench (+x), and the
        # largest bond dimension after every step of both
        _, run_z = workloads.chain30_jittered("+z")
        rz = timed_run(model, run_z, head, K, 0)
        line["plus_z"] = {"steps_per_s": K / rz["seconds"], "max_chi_reached": int(max(rz["dims"])),
                          "bond_dims_final": [int(d) for d in rz["dims"]]}
        line["max_chi_per_step"] = {args.init: chi_per_step(model, run, head, K),
                                    "+z": chi_per_step(model, run_z, head, K)}
    if not args.no_saturated:
        settle, ks = 4, 2
        sat = saturated_run(model, run, head, settle, ks)
        sa = sat["svd_flops"] / (sat["svd_ms"] * 1e-3) / 1e12
        line["saturated"] = {
            "workload": f"the same chain and run with cutoff 0: interior bonds at chi_max=256; steps {settle + 1}-"
                        f"{settle + ks} timed after {settle} untimed", "steps_per_s": ks / sat["seconds"],
            "ms_per_step": 1e3 * sat["seconds"] / ks, "bond_dims": [int(d) for d in sat["dims"]],
            "roofline": {"bound": "mfma", "kernel": "svd_persistent_kernel", "achieved": sa,
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": sa / FP64_PEAK_TFLOPS,
                         "launches": sat["launches"], "avg_launch_ms": sat["svd_ms"] / max(1, sat["launches"]),
                         "flops_per_launch": sat["svd_flops"] / max(1, sat["launches"])}}
        print(f"# saturated ({head}): {ks} steps in {sat['seconds']:.2f} s, max chi {max(sat['dims'])}",
              file=sys.stderr, flush=True)
    if not args.no_cpu:
        done, dt, obs = cpu_baseline(model, run, K, args.cpu_budget)
        line["cpu_baseline"] = {"value": done / dt, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                                "sample": f"first {done} of the {K} timed steps (FP64 NumPy/LAPACK oracle)"}
        d1, t1, _ = cpu_baseline(model, run, K, args.cpu_budget / 2, threads=1)
        line["cpu_baseline_1thread"] = {"value": d1 / t1, "unit": "steps/s", "cores": 1, "kind": "oracle",
                                        "sample": f"first {d1} of the {K} timed steps, one BLAS thread"}
        if obs is not None:
            ref = res["fp64"]["obs"] if "fp64" in res else h["obs"]
            line["obs_err_fp64_vs_oracle"] = float(np.abs(ref - obs).max())
            if "fp32" in res:
                line["obs_err_fp32_vs_oracle"] = float(np.abs(res["fp32"]["obs"] - obs).max())
    if not args.no_gradient:
        line["gradient"] = gradient_leg(args.cpu_budget, args.no_cpu)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
