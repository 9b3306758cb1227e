"""Benchmark: Trotter steps/s of the MPO-TEBD Lindblad step on one MI355X.

Headline workload: the N=30 open chain of driven, dissipative qubits
(alternating detunings 0/5 plus N(0, 0.1^2) jitter, couplings J ~ U[0.8, 1.2],
seed 0; edge drive Omega=1, g0=0.1, g2=0.05) at chi_max=256, cutoff 1e-10,
tau=0.05, second-order Trotter, in the regime where chi_max binds: the global
quench from all-"+x" is first evolved untimed, in FP64, to t = 6.5 (the
settling run, with a coarser step tau=0.1 to halve its cost), where the
interior bonds sit at 256.  From copies of that one state the FP32-contraction
form and the plain FP64 form then each run exactly K timed steps of tau=0.05
(inputs resident in HBM).  `value` is the FP32 form's steps/s; the FP64 form's
steps/s and the largest difference of all <s^z_i>, <s^z_i s^z_j> between the
two after the K steps sit beside it.

A step is one whole Trotter step of the hot path: centre hops, contraction +
gate, truncated SVD, canonical update, trace renormalisation.  Gate blocks of
512 columns or more (the 1024 x 1024 blocks between two chi=256 bonds) take
the subspace-iteration truncated SVD, accepted per block by its Ritz
residuals, the rest the full Jacobi SVD; `subspace_svd` counts both.  Warm-up
runs W steps of each form from t=0 (first launches), untimed.

Also on the line: the configured 50-step run from +x (where chi stays below
256) in the FP32, FP64 and real-arithmetic forms with the oracle's observables
beside it; the oracle timed on the host at the headline's block shapes
(`cpu_baseline`); the batched form on 64 uneven chains (`batched`); the adjoint
gradients on the 2 x 8 ladder with their gap to the oracle's (`gradient`).
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
SETTLE_TAU, SETTLE_T = 0.1, 6.5


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def zz(ch):
    import numpy as np

    z1, z2 = ch.zz_observables()
    return np.concatenate([z1, z2])


def settle(model, run, tau, t_end):
    """The headline's starting state: the +x quench evolved (FP64, chi_max and
    cutoff as configured) to t_end with step tau.  Returns the site tensors,
    the orthogonality centre, the largest bond dimension every 5 steps and the
    wall time."""
    from paper_2203_05871_amd import Chain

    ch = Chain(model, tau, run["chi_max"], run["cutoff"], "fp64", run["init"])
    n = int(round(t_end / tau))
    t0 = time.perf_counter()
    maxchi = []
    for i in range(n):
        ch.evolve(1)
        if i % 5 == 4 or i == n - 1:
            maxchi.append(int(max(ch.bond_dims())))
    ch.sync()
    dt = time.perf_counter() - t0
    sites = [ch.get_site(k) for k in range(model["N"])]
    centre = ch.centre()
    dims = ch.bond_dims()
    ch.close()
    return {"sites": sites, "centre": centre, "dims": dims, "steps": n, "seconds": dt, "max_chi_every5": maxchi}


def chain_from(model, run, precision, state):
    from paper_2203_05871_amd import Chain

    ch = Chain(model, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
    for k, A in enumerate(state["sites"]):
        ch.set_site(k, A)
    ch.set_centre(state["centre"])
    return ch


# phase timers of the SVD kernel's first workgroup (lmpo_svd_profile), reported per step
PHASES = ("pairs", "wait", "sub_iterations", "sub_final_cholqr", "sub_vectors", "hop_cholqr", "cholqr_gram",
          "cholqr_cholesky", "cholqr_solve", "chol_diag_lookahead", "chol_last_step", "chol_rows")


def timed(ch, steps):
    """Exactly `steps` steps between stream synchronisations, HIP events around
    every SVD launch; returns time, kernel figures and the final observables."""
    import torch

    torch.cuda.synchronize()
    ch.profile_begin(200 * steps)
    t0 = time.perf_counter()
    ch.evolve(steps)
    ch.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, svd_ms, svd_flops = ch.profile_end()
    stats = ch.svd_stats()
    acc, fell, iters = ch.svd_subspace_stats()
    prof = ch.svd_profile()
    phases = {k: round(prof[k] / 1e3 / steps, 2) for k in PHASES}
    phases["cholqr_passes_per_step"] = prof["cholqr_passes"] / steps
    return {"seconds": dt, "launches": launches, "svd_ms": svd_ms, "svd_flops": svd_flops, "obs": zz(ch),
            "phases_ms_per_step": phases,
            "dims": ch.bond_dims(), "sweeps": stats[2], "svds": stats[3],
            "subspace": {"accepted": acc, "to_full_svd": fell, "iterations_per_accepted": iters / max(1, acc)}}


def warm(model, run, precision, steps):
    from paper_2203_05871_amd import Chain

    if steps > 0:
        w = Chain(model, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
        w.evolve(steps)
        w.sync()
        w.close()


def fresh_run(model, run, precision, steps):
    from paper_2203_05871_amd import Chain

    ch = Chain(model, run["tau"], run["chi_max"], run["cutoff"], precision, run["init"])
    r = timed(ch, steps)
    ch.close()
    return r


def roofline_of(r, traffic=None):
    achieved = r["svd_flops"] / (r["svd_ms"] * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": "svd_persistent_kernel", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
            "launches": r["launches"], "avg_launch_ms": r["svd_ms"] / max(1, r["launches"]),
            "flops_per_launch": r["svd_flops"] / max(1, r["launches"]),
            "kernel_share_of_step": r["svd_ms"] * 1e-3 / r["seconds"]}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def oracle_steps(model, run, steps, budget_s, cutoff=None, threads=None, first_timed=0):
    """The FP64 oracle on the host cores: its own run of the same chain, steps
    before `first_timed` untimed, then timed steps until `steps` are done or the
    budget is spent.  Returns (timed steps, seconds, final observables or None)."""
    if threads is not None:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=threads):
            return oracle_steps(model, run, steps, budget_s, cutoff, None, first_timed)
    import numpy as np

    from oracle import tebd

    cut = run["cutoff"] if cutoff is None else cutoff
    mps = tebd.MPS.product(run["init"], model["N"])
    gates = tebd.gate_tables(model, run["tau"])
    for n in range(first_timed):
        tebd.evolve(mps, model, run["tau"], 1, run["chi_max"], cut, gates=gates, first_step=n)
    t0 = time.perf_counter()
    done = 0
    for n in range(first_timed, steps):
        tebd.evolve(mps, model, run["tau"], 1, run["chi_max"], cut, gates=gates, first_step=n)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    obs = None
    if first_timed + done == steps:
        z1, z2 = tebd.zz_observables(mps)
        obs = np.concatenate([z1, z2])
    return done, dt, obs, [int(d) for d in mps.bond_dims()] if hasattr(mps, "bond_dims") else None


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


# ---------------------------------------------------------------- batched form
def batched_leg(args):
    """64 uneven chains (N ~ U{8..24}), chi_max 64, cutoff 1e-12, 40 steps:
    the batched form (one launch per Trotter layer for all chains; the warm-up
    batch runs the whole trajectory with the autotuner on), the same chains one
    after another on the single-chain path, and the oracle on the first chains
    within the budget."""
    import numpy as np
    import torch

    import workloads
    from paper_2203_05871_amd import Batch, Chain

    models, run = workloads.chains64_uneven()
    K = run["steps"]

    def make():
        return [Chain(m, run["tau"], run["chi_max"], run["cutoff"], "fp64", run["init"]) for m in models]

    w = make()
    wb = Batch(w)
    wb.set_autotune(True)
    wb.evolve(K)
    wb.sync()
    wb.close()
    for c in w:
        c.close()
    chains = make()
    b = Batch(chains)
    torch.cuda.synchronize()
    b.profile_begin(3 * K + 3)
    t0 = time.perf_counter()
    b.evolve(K)
    b.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, ms, flops = b.profile_end()
    plan = b.plan()
    obs = [zz(c) for c in chains]
    max_chi = max(max(c.bond_dims()) for c in chains)
    b.close()
    for c in chains:
        c.close()
    achieved = flops / (ms * 1e-3) / 1e12
    out = {"workload": f"64 chains, N~U{{8..24}}, Omega~U[0.5,2], Delta~U[2,8], chi_max=64, cutoff=1e-12, "
                       f"tau=0.05, {K} steps from {run['init']} (FP64)",
           "steps_per_s": K / dt, "seconds": dt, "max_chi_reached": int(max_chi), "workgroups": int(plan.sum())}
    if not getattr(args, "no_sequential", False):
        chains = make()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in chains:
            c.evolve(K)
        for c in chains:
            c.sync()
        torch.cuda.synchronize()
        dseq = time.perf_counter() - t0
        seq_obs = [zz(c) for c in chains]
        for c in chains:
            c.close()
        out.update({"sequential_single_chain_steps_per_s": K / dseq, "speedup_vs_sequential": dseq / dt,
                    "batch_vs_sequential_max_obs_diff": float(max(np.abs(x - y).max()
                                                                  for x, y in zip(obs, seq_obs)))})
        log(f"batched: {K} steps in {dt:.2f} s (sequential {dseq:.1f} s)")
    else:
        log(f"batched: {K} steps in {dt:.2f} s")
    out.update({
           "roofline": {"bound": "mfma", "kernel": "batch_layer_kernel", "achieved": achieved,
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                        "traffic": None, "launches": launches, "avg_launch_ms": ms / max(1, launches),
                        "flops_per_launch": flops / max(1, launches)}})
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import tebd

        def oracle_chains(budget):
            t0 = time.perf_counter()
            done, worst = 0, 0.0
            for c, m in enumerate(models):
                mps = tebd.MPS.product(run["init"], m["N"])
                gates = tebd.gate_tables(m, run["tau"])
                tebd.evolve(mps, m, run["tau"], K, run["chi_max"], run["cutoff"], gates=gates)
                z1, z2 = tebd.zz_observables(mps)
                worst = max(worst, float(np.abs(np.concatenate([z1, z2]) - obs[c]).max()))
                done += 1
                if time.perf_counter() - t0 > budget:
                    break
            dto = time.perf_counter() - t0
            frac = sum(m["N"] for m in models[:done]) / sum(m["N"] for m in models)
            return done, K * frac / dto, worst

        done, rate, worst = oracle_chains(args.cpu_budget / 2)
        out["cpu_baseline"] = {"value": rate, "unit": "steps/s", "cores": blas_threads(),
                               "kind": "oracle", "sample": f"first {done} of {len(models)} chains, all {K} steps; "
                                                           f"batch rate scaled by their share of the sites"}
        out["obs_err_vs_oracle_sampled"] = worst
        with threadpool_limits(limits=1):
            done1, rate1, _ = oracle_chains(args.cpu_budget / 4)
        out["cpu_baseline_1thread"] = {"value": rate1, "unit": "steps/s", "cores": 1, "kind": "oracle",
                                       "sample": f"first {done1} chains, all {K} steps, one BLAS thread"}
    return out


# ------------------------------------------------------------ gradient form
def forty(m, gr):
    """The 40 numbers of the ladder case: 16 h_z, 22 J, Omega = h_x[0], and one
    g0 shared by all qubits (the sum of the per-qubit derivatives)."""
    import numpy as np

    return np.concatenate([np.asarray(gr["hz"]).real, np.asarray(gr["J"]).real, [np.real(gr["hx"][0])],
                           [np.real(np.sum(gr["g0"]))]])


def costate_convergence(m, run, chis=(64, 128, 256)):
    """How far the co-state's truncation moves the gradient: both ladder
    objectives with the co-state's chi_max at 64, 128 (the configured value)
    and 256, the largest change of any of the 140 derivatives between
    successive co-state chi_max, absolute and relative to the largest."""
    import numpy as np

    from paper_2203_05871_amd import Chain, Gradient

    tau, steps, chi, cut, init = run["tau"], run["steps"], run["chi_max"], run["cutoff"], run["init"]
    out, prev = {}, {}
    for cchi in chis:
        for name in ("z15", "connected_z0_z15"):
            c = Chain(m, tau, chi, cut, "fp64", init)
            G = Gradient(c, steps, costate_chi_max=cchi)
            t0 = time.perf_counter()
            F, g = G.run(15, "Z") if name == "z15" else G.run_connected(0, 15, "ZZ")
            dt = time.perf_counter() - t0
            dims = G.costate_dims()
            G.close()
            c.close()
            v = np.concatenate([np.real(g[k]) for k in g if k != "tau"])
            rec = {"seconds": dt, "max_abs_derivative": float(np.abs(v).max()),
                   "costate_bond_dims_t0": [int(x) for x in dims]}
            if name in prev:
                d = float(np.abs(v - prev[name]).max())
                rec["max_abs_change_from_previous_chi"] = d
                rec["change_over_largest"] = d / float(np.abs(v).max())
            prev[name] = v
            out.setdefault(name, {})[str(cchi)] = rec
            log(f"co-state chi {cchi}, {name}: {dt:.1f} s")
    return out


def gradient_leg(args):
    """Adjoint gradients on the 2 x 8 ladder (N=16, 8 rungs and 14 legs through
    the SWAP network), chi_max 128, cutoff 1e-12, tau 0.05, 40 steps from +z:
    F = <s^z_15>(T), the far corner from the drive, with all 6N + 2 n_bonds =
    140 derivatives in one backward pass, timed against the forward run alone;
    then both objectives of the configuration (<s^z_15> and the connected
    <s^z_0 s^z_15>_c) after the first n steps on the GPU and in the oracle,
    compared derivative by derivative."""
    import numpy as np
    import torch

    import workloads
    from paper_2203_05871_amd import Chain, Gradient

    m, run = workloads.ladder2x8()
    tau, steps, chi, cut, init = run["tau"], run["steps"], run["chi_max"], run["cutoff"], run["init"]

    def forward():
        c = Chain(m, tau, chi, cut, "fp64", init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.evolve(steps)
        c.sync()
        dt = time.perf_counter() - t0
        c.close()
        return dt

    forward()
    tf = forward()
    c = Chain(m, tau, chi, cut, "fp64", init)
    G = Gradient(c, steps)
    G.costate_profile_begin(40000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, g = G.run(15, "Z")
    tg = time.perf_counter() - t0
    launches, co_ms, co_flops = G.costate_profile_end()
    co_dims, st_dims = G.costate_dims(), c.bond_dims()
    G.close()
    c.close()
    log(f"gradient: {tg:.1f} s vs forward {tf:.2f} s")
    conv = costate_convergence(m, run) if args.costate_convergence else None
    out = {"workload": "2x8 ladder (N=16, 8 rungs + 14 legs via SWAP gates), chi_max=128, cutoff=1e-12, tau=0.05, "
                       "40 steps from +z; F = <sigma^z_15>(T); co-state with the same chi_max and cutoff",
           "parameters": int(sum(len(v) for k, v in g.items() if k != "tau")), "F": F.real,
           "seconds": tg, "forward_seconds": tf, "gradient_over_forward": tg / tf,
           "max_abs_gradient": max(float(np.abs(v).max()) for v in g.values()),
           "state_bond_dims_T": st_dims, "costate_bond_dims_t0": co_dims,
           "scaling_identity": {"sum_theta_dF": float(sum(np.dot(np.asarray(m[k], dtype=float), g[k])
                                                          for k in g if k != "tau")),
                                "tau_dF_dtau": float(tau * g["tau"][0])},
           "roofline": {"bound": "mfma", "kernel": "svd_persistent_kernel (co-state, real form)",
                        "achieved": co_flops / (co_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": co_flops / (co_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                        "traffic": None, "launches": launches, "avg_launch_ms": co_ms / max(1, launches),
                        "flops_per_launch": co_flops / max(1, launches), "kernel_share_of_gradient": co_ms * 1e-3 / tg},
           "derivatives_40": [float(x) for x in forty(m, g)]}
    if conv is not None:
        out["costate_chi_convergence"] = conv
    if not args.no_cpu:
        from oracle import adjoint

        n = args.grad_oracle_steps
        gp = {}
        c = Chain(m, tau, chi, cut, "fp64", init)
        G = Gradient(c, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F1, g1 = G.run(15, "Z")
        tg1 = time.perf_counter() - t0
        G.close()
        c.close()
        c = Chain(m, tau, chi, cut, "fp64", init)
        G = Gradient(c, n)
        C2, g2 = G.run_connected(0, 15, "ZZ")
        G.close()
        c.close()
        t0 = time.perf_counter()
        Fo, go, _ = adjoint.gradient(m, tau, n, chi, cut, init, 15, "Z")
        to = time.perf_counter() - t0
        Co, gco, _ = adjoint.gradient_connected(m, tau, n, chi, cut, init, 0, 15, "ZZ")
        for name, (gg, oo, val, vo) in {"z15": (g1, go, F1, Fo), "connected_z0_z15": (g2, gco, C2, Co)}.items():
            keys = [k for k in gg if k != "tau"]
            gpu = np.concatenate([np.real(gg[k]) for k in keys])
            ora = np.concatenate([np.real(oo[k]) for k in keys])
            scale = float(np.abs(ora).max())
            gp[name] = {"value_gpu": float(np.real(val)), "value_oracle": float(np.real(vo)),
                        "max_abs_derivative": scale, "max_abs_diff": float(np.abs(gpu - ora).max()),
                        "max_rel_diff_of_largest": float(np.abs(gpu - ora).max() / scale)}
        out["oracle_parity"] = {"steps": n, "parameters": 140, **gp}
        out["cpu_baseline"] = {"value": n / to, "unit": "gradient steps/s (forward + backward)",
                               "cores": blas_threads(), "kind": "oracle",
                               "sample": f"the gradient of <s^z_15> after the first {n} of the 40 steps"}
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            adjoint.gradient(m, tau, n, chi, cut, init, 15, "Z")
            to1 = time.perf_counter() - t0
        out["cpu_baseline_1thread"] = {"value": n / to1, "unit": "gradient steps/s (forward + backward)",
                                       "cores": 1, "kind": "oracle",
                                       "sample": f"the same gradient, one BLAS thread"}
        out["gpu_same_sample"] = {"value": n / tg1, "unit": "gradient steps/s (forward + backward)",
                                  "seconds": tg1}
        log(f"gradient vs oracle at {n} steps: {gp}")
    return out


# ------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps at chi=256 (default 20)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-t", type=float, default=SETTLE_T, help="time the +x quench is settled to, untimed")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle time per oracle sample")
    ap.add_argument("--grad-oracle-steps", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configured", action="store_true", help="skip the configured 50-step run from +x")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--costate-convergence", action="store_true",
                    help="add to the gradient object both ladder objectives at co-state chi_max 64, 128, 256 "
                         "(about 5 minutes)")
    ap.add_argument("--headline-only", action="store_true", help="only the settle and the timed chi=256 steps")
    ap.add_argument("--workload", choices=("chain30", "chains64", "ladder_grad"), default="chain30",
                    help="chain30: the line above (default); chains64: only the batched form's object; "
                         "ladder_grad: only the adjoint gradients' object")
    ap.add_argument("--no-sequential", action="store_true",
                    help="chains64: skip the same chains run one after another")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (the calibration kernel of "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): a single chain's Trotter step is a "
              "strictly sequential chain of gates; sharding over several GPUs is not run.",
              file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_configured = args.no_batched = args.no_gradient = args.no_cpu = True
    if args.workload != "chain30":
        import torch

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        if args.workload == "chains64":
            b = batched_leg(args)
            line = {"metric": "Trotter steps/s of a 64-chain batch (batched form)", "value": b["steps_per_s"],
                    "unit": "steps/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
                    "data": "synthetic (seeded chains, no dataset)", "config": {"workload": b["workload"]}, **b}
        else:
            g = gradient_leg(args)
            line = {"metric": "adjoint gradients/s on the 2x8 ladder (140 derivatives each)",
                    "value": 1.0 / g["seconds"], "unit": "gradients/s", "n_gpus": 1, "higher_is_better": True,
                    "dtype": "f64", "data": "synthetic (seeded ladder, no dataset)",
                    "config": {"workload": g["workload"]}, **g}
        print(json.dumps(line), flush=True)
        return

    import numpy as np
    import torch

    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_start = time.perf_counter()
    if args.copy_probe > 0:
        src = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read + written")
        del src, dst
    copy_gbps = mfma_tflops = None
    if args.copy_probe == 0:
        # context for the peaks: a plain 1 GiB device copy (read + write) and the
        # library's FP64 matrix-core throughput probe
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
        from paper_2203_05871_amd.lmpo import measured_fp64_mfma_peak

        mfma_tflops = measured_fp64_mfma_peak()

    model, run = workloads.chain30_jittered("+x")
    K, W = args.steps, args.warmup
    for prec in ("fp32", "fp64"):
        warm(model, run, prec, W)
    st = settle(model, run, SETTLE_TAU, args.settle_t)
    log(f"settled: {st['steps']} steps of tau={SETTLE_TAU} in {st['seconds']:.1f} s, dims {st['dims']}")
    res = {}
    for prec in ("fp32", "fp64"):
        ch = chain_from(model, run, prec, st)
        res[prec] = timed(ch, K)
        ch.close()
        r = res[prec]
        log(f"{prec}: {K} steps at chi=256 in {r['seconds']:.2f} s, SVD launches {r['launches']}, "
            f"kernel {r['svd_ms']:.0f} ms, sweeps/svd {r['sweeps'] / max(1, r['svds']):.2f}")
    h, d = res["fp32"], res["fp64"]
    interior = st["dims"][2:-2]
    tr = measured_traffic()
    roofline = roofline_of(h, tr["hbm_bytes_per_launch"] if tr else None)
    roofline.update({"traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                     "measured_copy_GBps": copy_gbps, "measured_fp64_mfma_TFLOPs": mfma_tflops,
                     "counters_mfma_busy_frac": tr.get("mfma_busy_frac") if tr else None,
                     "counters_mfma_f64_flops_executed_per_launch":
                         tr.get("mfma_f64_flops_per_launch_executed") if tr else None})
    line = {
        "metric": METRIC, "value": K / h["seconds"], "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": 1e3 * h["seconds"] / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32 contraction + fp64 svd",
        "data": "synthetic (seeded driven-dissipative chain, no dataset)",
        "config": {"workload": f"N=30 jittered XY chain, chi_max=256 binding: the +x quench settled untimed to "
                               f"t={args.settle_t} ({st['steps']} FP64 steps of tau={SETTLE_TAU}), then {K} steps "
                               f"of tau=0.05, cutoff 1e-10 timed from that state in each form",
                   "N": 30, "chi_max": 256, "cutoff": 1e-10, "tau": 0.05, "init": "+x",
                   "chi256_binds": bool(max(st["dims"]) == 256),
                   "interior_bonds_at_256_start": int(sum(1 for x in interior if x == 256)),
                   "interior_bonds": len(interior), "min_interior_chi_start": int(min(interior)),
                   "bond_dims_start": [int(x) for x in st["dims"]], "bond_dims_final": [int(x) for x in h["dims"]],
                   "settle_seconds": st["seconds"], "settle_max_chi_every5": st["max_chi_every5"]},
        "roofline": roofline,
        "fp64_steps_per_s": K / d["seconds"],
        "fp32_over_fp64": d["seconds"] / h["seconds"],
        "obs_err_fp32_vs_fp64": float(np.abs(h["obs"] - d["obs"]).max()),
        "fp64_roofline": roofline_of(d),
        "sweeps_per_svd": {"fp32": h["sweeps"] / max(1, h["svds"]), "fp64": d["sweeps"] / max(1, d["svds"])},
        "subspace_svd": {"fp32": h["subspace"], "fp64": d["subspace"]},
        "svd_phases_ms_per_step": {"fp32": h["phases_ms_per_step"], "fp64": d["phases_ms_per_step"]},
    }
    if not args.no_cpu:
        # the oracle at the headline's block shapes: its own +x run with cutoff 0,
        # whose interior bonds sit at chi=256 from its second step on; step 3 timed
        done, dt, _, _ = oracle_steps(model, run, 3, args.cpu_budget, cutoff=0.0, first_timed=2)
        line["cpu_baseline"] = {"value": done / dt, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                                "sample": "one oracle step whose interior bonds sit at chi=256 (its own +x run with "
                                          "cutoff 0: step 3 timed after 2 untimed), FP64 NumPy/LAPACK"}
        d1, t1, _, _ = oracle_steps(model, run, 3, args.cpu_budget, cutoff=0.0, first_timed=2, threads=1)
        line["cpu_baseline_1thread"] = {"value": d1 / t1, "unit": "steps/s", "cores": 1, "kind": "oracle",
                                        "sample": "the same oracle step, one BLAS thread"}
        log(f"oracle at chi=256: {done} step in {dt:.1f} s ({t1:.1f} s on one thread)")
    if not args.no_configured:
        # the configured trajectory: 50 steps from +x at tau 0.05 (chi stays below 256)
        ks = run["steps"]
        cfg = {}
        for prec in ("fp32", "fp64", "real"):
            cfg[prec] = fresh_run(model, run, prec, ks)
        c = {"workload": f"the configured run: {ks} steps of tau=0.05 from +x, chi_max=256, cutoff 1e-10 "
                         f"(chi stays below 256)", "max_chi_reached": int(max(cfg["fp64"]["dims"])),
             "bond_dims_final": [int(x) for x in cfg["fp64"]["dims"]],
             "fp32_steps_per_s": ks / cfg["fp32"]["seconds"], "fp64_steps_per_s": ks / cfg["fp64"]["seconds"],
             "real_steps_per_s": ks / cfg["real"]["seconds"],
             "obs_err_fp32_vs_fp64": float(np.abs(cfg["fp32"]["obs"] - cfg["fp64"]["obs"]).max()),
             "obs_err_real_vs_fp64": float(np.abs(cfg["real"]["obs"] - cfg["fp64"]["obs"]).max()),
             "roofline_fp64": roofline_of(cfg["fp64"])}
        if not args.no_cpu:
            # (1.5 budgets: the 16-thread oracle needs 20-22 s for all 50 steps, and the
            # oracle's observables are compared only when it finishes them)
            done, dt, obs, _ = oracle_steps(model, run, ks, 1.5 * args.cpu_budget)
            c["cpu_baseline"] = {"value": done / dt, "unit": "steps/s", "cores": blas_threads(), "kind": "oracle",
                                 "sample": f"first {done} of the {ks} steps"}
            d1, t1, _, _ = oracle_steps(model, run, ks, args.cpu_budget / 2, threads=1)
            c["cpu_baseline_1thread"] = {"value": d1 / t1, "unit": "steps/s", "cores": 1, "kind": "oracle",
                                         "sample": f"first {d1} of the {ks} steps, one BLAS thread"}
            if obs is not None:
                c["obs_err_fp64_vs_oracle"] = float(np.abs(cfg["fp64"]["obs"] - obs).max())
                c["obs_err_fp32_vs_oracle"] = float(np.abs(cfg["fp32"]["obs"] - obs).max())
                c["obs_err_real_vs_oracle"] = float(np.abs(cfg["real"]["obs"] - obs).max())
        line["configured_run"] = c
        log(f"configured run: fp32 {c['fp32_steps_per_s']:.2f} fp64 {c['fp64_steps_per_s']:.2f} steps/s")
    if not args.no_batched:
        line["batched"] = batched_leg(args)
    if not args.no_gradient:
        line["gradient"] = gradient_leg(args)
    line["bench_seconds"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
