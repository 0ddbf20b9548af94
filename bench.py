"""Benchmark of the CF-DQMC sweep on one MI355X.

Workload (default): 256 independent chains of the torus N_phi = 100 model
(spin block n = 200, 4N = 400), paper momentum cutoff (933 HS components per
channel), L = 400 slices of dtau = 0.1, u = 1.5 on the SO(5) line, FP64
recomputation every 8 slices, complex FP32 MFMA wraps and drift frames with the
precision guard (chains with large |G| or error run them in FP64; --precision
fp64 for the all-FP64 path). A step is one sweep of every chain: L Langevin
slice moves of 4 n_q fields each, with wraps, Woodbury updates and
stabilisation. After the timed sweeps: the same chains with every product in
FP64 (timed), then untimed sweeps of re-created mixed chains for a short
tau_int and for the learned proposal's training set (trained, then tried),
one imaginary-time correlator pass, a one-chain FP64 reference sweep, and the
FP64 oracle on the host. The independent-sample rate uses the tau_int of a
long run of the same shape (--workload tau-long). --workload batched, learned,
tau, tau-long and oracle-tau run the other workloads.

Prints one JSON line (see the fields below). Synthetic fields N(0,1).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "mixed": 157.3, "mixed_all": 157.3}     # MI355X dense MFMA TFLOP/s (FP64, FP32)
# what a loop of nothing but independent 16x16x4 MFMAs sustains on one MI355X
# (kbench mfma, profiles/mfma_sustained_rate.md): the practical ceiling
SUSTAINED = {"fp64": 49.2, "mixed": 135.5, "mixed_all": 135.5}

# HBM bytes per launch of the timed channel application, FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (KiB, factors from a 1 GiB copy) from rocprofv3 PMC runs of
# this script (profiles/chan_apply_traffic_n100_256chains.md); keyed by
# (N_phi, chains per context, precision, tile configuration). Absent key, or a
# kernel changed since the counters were taken: traffic not measured (null).
# HBM bytes per chain of one channel application at N_phi = 100 (rocprofv3
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, KiB per dispatch of 256 chains, scaled by
# the copy calibration; profiles/chan_apply_traffic_n100_256chains.md), keyed
# by (n_phi, arithmetic, channel-application configuration)
TRAFFIC = {(100, "f32", 12): (167544.25 * 2.0 + 160000.0) * 1024 / 256,
           (100, "f64", 1): (126926.55 * 2.0 + 171777.13) * 1024 / 256,
           # the guarded one-launch form with the given percentage of the chains in FP64
           (100, "dual", 12, 94): (126374.02 * 2.0 + 160000.67) * 1024 / 256}

# Integrated autocorrelation times at the default workload's shape (N_phi = 100,
# L = 400, dtau = 0.1, u = 1.5, paper cutoff) from one long run, 32 chains x
# 1000 sweeps after 8 (bench.py --workload tau-long, profiles/
# tau_int_n100_32chains_1000sweeps.md); every window closed. tau_int is a
# property of the Markov chain, not of the kernels' speed, so the default line
# divides its own sweep rate by 2 x the slowest of these.
TAU_LONG = {"shape": (100, 400, 0.1, 1.5), "chains": 32, "sweeps": 1000,
            "tau_int": {"m2": 1.18, "action": 14.33, "phi_q0_power": 69.06}}


def cpu_baseline(n_phi, l_tau, dtau, u, seconds=15.0, sphere=False):
    """The FP64 oracle timed on the host on a bounded sample of the same
    workload, with all cores and with one BLAS thread: see _cpu_rate."""
    out = _cpu_rate(n_phi, l_tau, dtau, u, seconds, sphere)
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            one = _cpu_rate(n_phi, l_tau, dtau, u, seconds, sphere)
        out["value_1thread"] = one["value"]
        out["sample_1thread"] = one["sample"]
    except Exception as e:     # threadpoolctl missing: report the all-core figure only
        out["value_1thread"] = None
        out["sample_1thread"] = "not measured (%s)" % e
    return out


def _cpu_rate(n_phi, l_tau, dtau, u, seconds, sphere):
    """A chain with the same N_phi, momentum set and couplings and at most 16
    slices. Its sweep set-up alone (all slice exponentials and suffix products,
    cost proportional to L: a sweep stopped before its first move), the set-up
    plus one move, and the set-up plus k moves are timed; k is as large as the
    time budget allows, up to every slice of the chain, so that the moves'
    time stands well above the run-to-run noise of the set-up (best of two
    runs), from which it is taken as a difference. The reported rate is
    4 n_q / (set-up per slice + time per slice move), the oracle's full-sweep
    rate at any L."""
    import synth
    from oracle import dqmc
    from oracle.model import Model, Q_PAPER, Q_SPHERE
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    ls = min(l_tau, 16)
    m = Model(n_phi, ls, dtau, u0=1.0, uk=u, un=u, q_mode=Q_SPHERE if sphere else Q_PAPER)
    phi = synth.fields(1, ls, m.n_q)
    rp = synth.replay(2, 1, ls, m.n_q)[0]
    def timed(k):
        t0 = time.perf_counter()
        dqmc.Chain(m, phi, eps0=0.3, adapt=False).sweep(rp, max_slices=k)
        return time.perf_counter() - t0
    t_set = min(timed(0), timed(0))           # the set-up alone
    t_1 = timed(1)                            # set-up and one move: the estimate of a move
    k = max(4, min(ls, int((seconds - t_set) / max(t_1 - t_set, 1e-3))))
    t_k = timed(k)
    per_move = max(t_k - t_set, 1e-9) / k
    per_slice = t_set / ls + per_move
    return {"value": 4 * m.n_q / per_slice, "unit": "field updates/s", "cores": cores, "kind": "oracle",
            "sample": "set-up of a %d-slice chain (%.1f s) and its first %d slice moves (%.1f s per move) at "
                      "N_phi=%d, n_q=%d, u=%g; FP64 numpy/LAPACK; rate = 4 n_q / (set-up per slice + move)"
                      % (ls, t_set, k, per_move, n_phi, m.n_q, u)}


def progress(msg):
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def sweep_each(b, steps, report_every=0, after=None):
    """Run `steps` sweeps one at a time; returns wall time, stats of every
    chain over all sweeps, and per sweep the max over chains of
    max|G_updated - G_FP64| (absolute, max norm) and of max|G_updated - G_FP64|
    / max|G_FP64| (relative) at the recomputation points. report_every > 0
    prints a progress line every that many sweeps."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, g_err = [], []
    for i in range(steps):
        st = b.sweep(1)
        stats.append(st)
        g_err.append((max(x["max_stab_err"] for x in st), max(x["max_stab_rel"] for x in st)))
        if after is not None:
            after()
        if report_every > 0 and (i + 1) % report_every == 0:
            progress("%d of %d sweeps" % (i + 1, steps))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats, g_err


def chain_acceptance(stats):
    """Per-chain acceptance over a list of sweeps' stats: (min, count of chains
    with no accepted move)."""
    n = len(stats[0])
    acc = [sum(st[z]["accepted"] for st in stats) / max(1, sum(st[z]["proposed"] for st in stats)) for z in range(n)]
    return min(acc), sum(1 for a in acc if a == 0.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--therm", type=int, default=4,
                    help="thermalisation sweeps from the N(0,1) start before the warm-up (untimed; their G "
                         "errors are reported apart)")
    ap.add_argument("--n-phi", type=int, default=100)
    ap.add_argument("--l-tau", type=int, default=400)
    ap.add_argument("--dtau", type=float, default=0.1)
    ap.add_argument("--u", type=float, default=1.5)
    ap.add_argument("--n-stab", type=int, default=8)
    ap.add_argument("--chains", type=int, default=256,
                    help="independent chains in one context; 256 N_phi = 100 chains take about 190 GB of HBM")
    ap.add_argument("--groups", type=int, default=1, help="split the chains over this many streams")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed_all"], default="mixed")
    ap.add_argument("--series-out", default=None,
                    help="tau-long: write the per-sweep series (npz) here every 100 sweeps and at the end")
    ap.add_argument("--q-mode", choices=["paper", "bz"], default="paper",
                    help="tau-long and oracle-tau: momentum set (paper cutoff, or the N^2 Brillouin-zone momenta)")
    ap.add_argument("--workload", choices=["c3", "batched", "learned", "tau", "tau-long", "oracle-tau"],
                    default="c3",
                    help="c3: N_phi=100 torus; batched: 64 chains over N_phi 24/48/72 and a 16-point u grid; "
                         "learned: N_phi=140, L=600 with the learned global proposal; tau: imaginary-time "
                         "correlator passes over the c3 chains (no sweeps)")
    ap.add_argument("--learned-chains", type=int, default=16)
    ap.add_argument("--learned-sweeps", type=int, default=12)
    ap.add_argument("--learned-epochs", type=int, default=30)
    ap.add_argument("--tile-cfg", type=int, default=-1)
    ap.add_argument("--geometry", choices=["torus", "sphere"], default="torus",
                    help="torus (paper momentum cutoff) or sphere (every (l, m), l <= 2s)")
    ap.add_argument("--exp-squarings", type=int, default=2,
                    help="max scaling-and-squaring steps of the slice exponentials (the sphere needs more)")
    ap.add_argument("--tau-sweeps", type=int, default=40,
                    help="untimed sweeps after the timed ones for tau_int (their configurations train the learned "
                         "proposal)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned global proposal (collection during the tau_int sweeps, training, moves)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-chain FP64 reference sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip timing the same chains with every product in FP64 after the mixed run")
    ap.add_argument("--no-tau-correlator", action="store_true",
                    help="skip the imaginary-time correlator pass after the tau_int sweeps")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--guard-gmax", type=float, default=0.8,
                    help="precision guard: FP64 applications for chains with max|G_FP64| above this")
    ap.add_argument("--guard-err", type=float, default=2.5e-7,
                    help="precision guard: FP64 applications for chains whose last block error exceeded this")
    ap.add_argument("--no-guard", action="store_true", help="FP32 applications for every chain (mixed modes)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every sweep launch by launch (no recorded sweep graphs)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="no HIP-event timing of the channel application in the timed sweeps (they then run as "
                         "recorded sweep graphs; no roofline object)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the short batched-workload leg (64 chains over N_phi 24/48/72) of the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB between two fresh device buffers three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the chains are independent, so "
              "several GPUs would each run their own contexts with no communication). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.zeros_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8, "copies": 3}))
        return
    if args.workload == "oracle-tau":
        return bench_oracle_tau(args)
    import numpy as np
    import torch
    from paper_2605_03700_amd import Batch, FP64, MIXED, MIXED_ALL, Q_PAPER, Q_SPHERE
    from paper_2605_03700_amd.analysis import tau_int_pooled
    assert torch.cuda.is_available(), "needs the GPU"
    prec = {"fp64": FP64, "mixed": MIXED, "mixed_all": MIXED_ALL}[args.precision]
    if args.workload == "batched":
        return bench_batched(args, prec)
    if args.workload == "learned":
        return bench_learned(args, prec)
    if args.workload == "tau":
        return bench_tau(args, prec)
    if args.workload == "tau-long":
        return bench_tau_long(args, prec)
    if args.workload == "oracle-tau":
        return bench_oracle_tau(args)
    if args.chains % args.groups:
        raise SystemExit("--chains must be a multiple of --groups")
    nper = args.chains // args.groups
    geo = dict(q_mode=Q_SPHERE if args.geometry == "sphere" else Q_PAPER, exp_squarings=args.exp_squarings,
               sweep_graph=0 if args.no_graph else 1)
    guard = dict(precision_guard=0 if args.no_guard else 1, guard_gmax=args.guard_gmax, guard_err=args.guard_err)
    b = Batch([dict(n_phi=args.n_phi, l_tau=args.l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u,
                    n_stab=args.n_stab, precision=prec, eps0=0.3, adapt_eps=True, seed=3 + k, n_chains=nper,
                    tile_cfg=args.tile_cfg, **geo, **guard) for k in range(args.groups)])
    g = b.groups[0]
    progress("contexts created (tiles %s)" % (g.tile_config(),))
    b.init_fields()
    progress("fields initialised")
    g_err_therm = []
    if args.therm > 0:
        _, therm_stats, g_err_therm = sweep_each(b, args.therm)
        progress("thermalisation done")
    if args.warmup:
        b.sweep(args.warmup)
        progress("warm-up done")
    g.kernel_timing(not args.no_kernel_timing)
    dt, stats, g_err = sweep_each(b, args.steps)
    progress("timed sweeps done: %.1f ms per sweep" % (1000.0 * dt / args.steps))
    k_ms, k_count, k_flops = g.kernel_timing_read()
    w_ms, w_count, w_flops = g.kernel_timing_read(woodbury=True)
    g.kernel_timing(False)
    fields = args.chains * args.l_tau * 4 * g.n_q * args.steps
    value = fields / dt
    sweeps_per_s = args.steps / dt
    flat = [x for st in stats for x in st]
    acc = sum(x["accepted"] for x in flat) / max(1, sum(x["proposed"] for x in flat))
    out = {
        "metric": "field updates/s + indep. samples/s at N_phi=100, plain vs learned/FP32; G err",
        "value": value, "unit": "field updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "%s N_phi=%d L_tau=%d dtau=%g u=%g %s n_q=%d, %d chain(s) in %d "
                               "stream group(s), FP64 recompute every %d slices"
                               % (args.geometry, args.n_phi, args.l_tau, args.dtau, args.u,
                                  "all (l, m)" if args.geometry == "sphere" else "paper cutoff", g.n_q,
                                  args.chains, args.groups, args.n_stab),
                   "chains": args.chains, "groups": args.groups, "precision": args.precision, "n_q": g.n_q,
                   "tile_cfg": list(g.tile_config()), "launch_config": g.launch_config()},
        "acceptance": acc,
        "acceptance_min_chain": chain_acceptance(stats)[0],
        "frozen_chains": chain_acceptance(stats)[1],
        "eps": float(np.mean(np.concatenate([q.get_eps() for q in b.groups]))),
        "g_err_max": max(e[0] for e in g_err),
        "g_err_per_sweep": [e[0] for e in g_err],
        "g_err_definition": "max over chains and recomputation points of max|G_updated - G_FP64| (absolute, "
                            "max norm); g_err_rel_* divide by max|G_FP64| of the chain",
        "g_err_rel_max": max(e[1] for e in g_err),
        "g_err_rel_per_sweep": [e[1] for e in g_err],
        "g_err_median_chain": float(np.median([max(st[z]["max_stab_err"] for st in stats)
                                               for z in range(len(stats[0]))])),
        "g_err_frac_chain_sweeps_above_1e-6": float(np.mean([x["max_stab_err"] > 1e-6 for x in flat])),
        "thermalization_sweeps": args.therm,
        "g_err_per_thermalization_sweep": [e[0] for e in g_err_therm],
        "g_err_rel_per_thermalization_sweep": [e[1] for e in g_err_therm],
        "sweeps_per_s_per_chain": sweeps_per_s,
        "accepted_field_updates_per_s": value * acc,
        "max_abs_g_median_chain": float(np.median([max(st[z]["max_abs_g"] for st in stats)
                                                   for z in range(len(stats[0]))])),
        "max_abs_g_max": max(x["max_abs_g"] for x in flat),
        "fp64_guard_frac": float(np.mean([x["fp64_guard_frac"] for x in flat])),
        "sweep_graph_frac": float(np.mean([x["graph_sweep_frac"] for x in flat])),
        "sweep_graph_definition": "fraction of the timed sweeps run as one launch of the recorded sweep graph "
                                  "(kernel timing runs them launch by launch)",
        "fp64_guard_definition": "fraction of (chain, stabilisation block) pairs whose FP32 applications the "
                                 "precision guard ran in FP64 from some slice on (an entry of the updated G above "
                                 "%g, or at the previous recomputation max|G_FP64| > %g or a block error > %g)"
                                 % (args.guard_gmax, args.guard_gmax, args.guard_err),
    }
    if args.therm > 0:
        out["acceptance_min_chain_thermalization"], out["frozen_chains_thermalization"] = \
            chain_acceptance(therm_stats)
    # whole-path figure: W_slice = 64 n^3 real flops per slice move (8 complex
    # n x n x n GEMM-equivalents: wrap 2, B' 3, Delta 1, M 1, solve 1), n = 2 N_phi
    n_sp = 2 * args.n_phi
    w_slice = 64.0 * n_sp ** 3
    path_tf = args.chains * args.l_tau * args.steps / dt * w_slice / 1e12
    out["path_roofline"] = {"work_per_slice_move_flop": w_slice, "achieved": path_tf, "unit": "TFLOP/s",
                            "peak": PEAK[args.precision], "frac": path_tf / PEAK[args.precision],
                            "peak_fp64": PEAK["fp64"], "frac_of_fp64_peak": path_tf / PEAK["fp64"],
                            "definition": "64 n^3 real flops per slice move, n = 2 N_phi"}
    # one channel application carries an eighth of the wrap's two n x n x n
    # complex products (16 n^3 real flops per chain): 2 n^3 algorithmic flops
    # per chain per launch; the kernel itself performs two N x N x n complex
    # products, 4 n^3 (its MFMA issue rate is reported apart)
    algo_per_launch = 2.0 * n_sp ** 3 * nper
    if k_count > 0 and k_ms > 0:
        ach = algo_per_launch / (k_ms * 1e-3) / 1e12
        issued = k_flops / (k_ms * 1e-3) / 1e12
        # bytes of the timed application: FP32 launches for the chains the guard
        # leaves in FP32, FP64 launches (configuration 1) for the others
        t32 = TRAFFIC.get((args.n_phi, "f32", g.tile_config()[0]))
        t64 = TRAFFIC.get((args.n_phi, "f64", 1))
        f64 = out["fp64_guard_frac"] if prec != FP64 else 1.0
        traffic = None
        lc = g.launch_config()
        # the measured one-launch form whose FP64 share is closest to this run's
        duals = [(abs(k[3] - 100.0 * f64), k[3], v) for k, v in TRAFFIC.items()
                 if len(k) == 4 and k[0] == args.n_phi and k[1] == "dual" and k[2] == lc["chan"]]
        dual_pct, tdual = (min(duals)[1], min(duals)[2]) if duals else (None, None)
        traffic_basis = ("HBM bytes per chain of the FP32 and the FP64 application (rocprofv3 FETCH_SIZE / "
                         "WRITE_SIZE, copy-calibrated, profiles/chan_apply_traffic_n100_256chains.md) weighted by "
                         "the fraction of chains in FP64")
        if prec == FP64 and g.tile_config()[0] == 1 and t64:
            traffic = nper * t64
        elif prec == MIXED and lc["guard_launch"] > 0 and tdual and abs(dual_pct - 100.0 * f64) < 5.0:
            traffic = nper * tdual
            traffic_basis = ("HBM bytes per chain of the guarded one-launch application with %d%% of the chains "
                             "in FP64 (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated, "
                             "profiles/chan_apply_traffic_n100_256chains.md)" % dual_pct)
        elif prec == MIXED and t32 and t64:
            traffic = nper * ((1.0 - f64) * t32 + f64 * t64)
        out["roofline"] = {"bound": "mfma", "kernel": "chan_apply", "achieved": ach,
                           "peak": PEAK[args.precision], "unit": "TFLOP/s", "frac": ach / PEAK[args.precision],
                           "traffic": traffic, "avg_launch_ms": k_ms, "launches_timed": k_count,
                           "flops_per_launch": algo_per_launch,
                           "issued_flops_per_launch": k_flops, "issued_tflops": issued,
                           "issued_frac": issued / PEAK[args.precision],
                           "hbm_gbps_at_traffic": traffic / (k_ms * 1e-3) / 1e9 if traffic else None,
                           "traffic_basis": traffic_basis,
                           "definition": "achieved = 2 n^3 real flops per chain (an eighth of the wrap's two "
                                         "n x n x n complex products) / mean HIP-event duration of the timed "
                                         "launch; issued_* count the 4 n^3 the launch performs"}
        sus = SUSTAINED[args.precision]
        if prec == MIXED:
            # the timed application runs the guarded chains in FP64: the peak of
            # that mix (harmonic weighting by the FP64 fraction) beside the FP32 one
            pk = 1.0 / ((1.0 - f64) / PEAK["mixed"] + f64 / PEAK["fp64"])
            out["roofline"]["peak_of_precision_mix"] = pk
            out["roofline"]["frac_of_precision_mix"] = ach / pk
            sus = 1.0 / ((1.0 - f64) / SUSTAINED["mixed"] + f64 / SUSTAINED["fp64"])
        out["roofline"]["peak_sustained"] = sus
        out["roofline"]["frac_of_sustained"] = ach / sus
        out["roofline"]["issued_frac_of_sustained"] = issued / sus
        out["roofline"]["peak_sustained_basis"] = ("16x16x4 MFMA loop with no memory traffic, FP64 %.1f and FP32 "
                                                   "%.1f TFLOP/s (kbench mfma, profiles/mfma_sustained_rate.md); "
                                                   "for a mixed run weighted by the FP64 fraction"
                                                   % (SUSTAINED["fp64"], SUSTAINED["mixed"]))
    if w_count > 0 and w_ms > 0:
        # the same kernel family in the Woodbury product M = G + B'B^-1(1 - G),
        # FP64 unless every product runs in FP32
        w_peak = PEAK["mixed"] if args.precision == "mixed_all" else PEAK["fp64"]
        w_ach = algo_per_launch / (w_ms * 1e-3) / 1e12
        w_iss = w_flops / (w_ms * 1e-3) / 1e12
        out["roofline_woodbury_application"] = {
            "bound": "mfma", "kernel": "chan_apply (Woodbury product, %s)" % (
                "FP32" if args.precision == "mixed_all" else "FP64"),
            "achieved": w_ach, "peak": w_peak, "unit": "TFLOP/s", "frac": w_ach / w_peak,
            "avg_launch_ms": w_ms, "launches_timed": w_count, "flops_per_launch": algo_per_launch,
            "issued_flops_per_launch": w_flops, "issued_tflops": w_iss, "issued_frac": w_iss / w_peak}
        w_sus = SUSTAINED["mixed_all"] if args.precision == "mixed_all" else SUSTAINED["fp64"]
        out["roofline_woodbury_application"]["peak_sustained"] = w_sus
        out["roofline_woodbury_application"]["frac_of_sustained"] = w_ach / w_sus
        out["roofline_woodbury_application"]["issued_frac_of_sustained"] = w_iss / w_sus
    if prec != FP64 and not args.no_fp64_compare:
        # the same chains with every product in FP64, right after the timed mixed
        # sweeps (one context of this size at a time fits in HBM): the FP64
        # context starts from the mixed chains' fields and step sizes, runs one
        # warm-up sweep and the same number of timed sweeps; the mixed chains are
        # then re-created from that same state
        state = [(q.get_fields(), q.get_eps()) for q in b.groups]
        b.close()

        def restart(batch):
            for q, (phi, eps) in zip(batch.groups, state):
                q.init_fields(phi)
                q.set_eps(eps)
        f = Batch([dict(n_phi=args.n_phi, l_tau=args.l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u,
                        n_stab=args.n_stab, precision=FP64, eps0=0.3, adapt_eps=True, seed=3 + k, n_chains=nper,
                        tile_cfg=args.tile_cfg, **geo) for k in range(args.groups)])
        restart(f)
        f.sweep(1)
        dtf, _, gef = sweep_each(f, args.steps)
        f_rate = args.chains * args.l_tau * 4 * g.n_q * args.steps / dtf
        out["fp64_same_chains"] = {"precision": "fp64", "chains": args.chains, "field_updates_per_s": f_rate,
                                   "ms_per_sweep": 1000.0 * dtf / args.steps, "g_err_max": max(e[0] for e in gef),
                                   "mixed_over_fp64": value / f_rate,
                                   "launch_config": f.groups[0].launch_config(),
                                   "start": "the mixed chains' fields and step sizes after the timed sweeps, "
                                            "one warm-up sweep, %d timed sweeps" % args.steps}
        f.close()
        progress("FP64 comparison on the same chains done")
        b = Batch([dict(n_phi=args.n_phi, l_tau=args.l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u,
                        n_stab=args.n_stab, precision=prec, eps0=0.3, adapt_eps=True, seed=3 + k, n_chains=nper,
                        tile_cfg=args.tile_cfg, **geo, **guard) for k in range(args.groups)])
        g = b.groups[0]
        restart(b)
        del state
        progress("mixed chains re-created from the same state")
    tau = None
    slmc = None
    if args.tau_sweeps > 0:
        n0 = [len(q.series(0)) for q in b.groups]
        collect = None
        if not args.no_learned and args.groups == 1:
            from paper_2605_03700_amd import Slmc
            slmc = Slmc(g, hidden=256, n_qbins=16, n_wbins=16, capacity=args.chains * args.tau_sweeps,
                        max_batch=256, seed=11)
            collect = slmc.collect
        dt2, stats2, g_err2 = sweep_each(b, args.tau_sweeps, report_every=10, after=collect)
        out["g_err_max_later_sweeps"] = max(e[0] for e in g_err2)
        out["g_err_rel_max_later_sweeps"] = max(e[1] for e in g_err2)
        out["g_err_per_later_sweep"] = [e[0] for e in g_err2]
        out["sweep_graph_frac_later_sweeps"] = float(np.mean([x["graph_sweep_frac"] for st in stats2 for x in st]))
        taus, open_w = {}, []
        for obs in ("m2", "action", "phi_q0_power"):
            series = [q.series(k, obs)[n0[i]:] for i, q in enumerate(b.groups) for k in range(nper)]
            t_o, _, closed = tau_int_pooled(series)
            taus[obs] = float(t_o)
            if not closed:
                open_w.append(obs)
        tau = max(taus.values())
        out["tau_int_sweeps"] = tau
        out["tau_int_per_observable"] = taus
        out["tau_int_observable"] = ("max over m2_SO(5), the action S and the q = 0 field power; autocorrelation "
                                     "pooled over the %d chains' %d-sweep series, deviations from the per-sweep "
                                     "ensemble mean" % (args.chains, args.tau_sweeps))
        # an open window means the series is shorter than that observable's
        # autocorrelation: tau_int is then a lower bound and the rate an upper one
        out["tau_int_window_open"] = open_w
        out["tau_int_is_lower_bound"] = bool(open_w)
        rate = args.chains * (args.tau_sweeps / dt2) / (2 * tau)
        if open_w:
            # tau_int is a lower bound: the rate is only an upper bound
            out["indep_samples_per_s"] = None
            out["indep_samples_per_s_upper_bound"] = rate
        else:
            out["indep_samples_per_s"] = rate
        if TAU_LONG["shape"] == (args.n_phi, args.l_tau, args.dtau, args.u) and args.geometry == "torus":
            # the long run's closed-window tau_int with this run's sweep rate
            t_long = max(TAU_LONG["tau_int"].values())
            out["tau_int_long_run"] = dict(TAU_LONG, source="bench.py --workload tau-long (profiles/"
                                           "tau_int_n100_32chains_1000sweeps.md)")
            out["indep_samples_per_s"] = args.chains * sweeps_per_s / (2 * t_long)
            out["indep_samples_per_s_definition"] = ("chains x sweeps/s per chain of the timed sweeps / (2 x the "
                                                     "long run's tau_int of the q = 0 field power, %.1f sweeps)"
                                                     % t_long)
        out["acceptance_min_chain_later_sweeps"], out["frozen_chains_later_sweeps"] = chain_acceptance(stats2)
        progress("tau_int sweeps done")
        if slmc is not None:
            try:
                out["learned"] = learned_leg(g, slmc, args, dt2 / args.tau_sweeps)
            except RuntimeError as e:     # reported in the line; the sweep results above stand
                out["learned"] = {"error": str(e)}
            slmc.close()
            progress("learned proposal trained and tried")
    if not args.no_tau_correlator:
        # one imaginary-time pass (G(tau,0), G(0,tau), G(tau,tau) for tau = 0..L
        # and the SO(5) correlator at q = 0) over every chain, FP64
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [q.measure_tau(with_stab=True) for q in b.groups]
        dtm = time.perf_counter() - t0
        C = np.concatenate([r[0] for r in res])
        st = np.concatenate([r[1] for r in res])
        m2t = C.mean(axis=2).mean(axis=0)
        pts = sorted({0, 1, 2, 4, 8, 16, 32, 64, 128, args.l_tau // 2} & set(range(args.l_tau + 1)))
        chan_flops = 12.0 * args.l_tau * 16.0 * args.n_phi ** 2 * n_sp * args.chains
        out["tau_correlator"] = {
            "ms_per_pass": 1000.0 * dtm, "chains": args.chains, "pass_over_sweep": dtm / (dt / args.steps),
            "channel_application_tflops": chan_flops / dtm / 1e12,
            "carried_vs_recomputed_rel_max": float(st.max()),
            "m2_so5_tau_mean_over_chains": {str(t): float(m2t[t].real) for t in pts},
            "definition": "m^2_SO(5)(tau, q=0) = (1/5) sum_i <n^i_{q=0}(tau) n^i_{q=0}(0)>, tau in slices; "
                          "one pass = L slices x 12 FP64 channel applications + a recomputation per block"}
        progress("imaginary-time correlator pass done")
    b.close()
    if not args.no_plain:
        # the plain path for comparison: one chain, FP64, same workload
        p = Batch([dict(n_phi=args.n_phi, l_tau=args.l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u,
                        n_stab=args.n_stab, precision=FP64, eps0=0.3, adapt_eps=True, seed=99, n_chains=1,
                        tile_cfg=args.tile_cfg, **geo)])
        p.init_fields()
        p.sweep(1)
        dtp, stp, gep = sweep_each(p, 2)
        plain = {"chains": 1, "precision": "fp64", "field_updates_per_s": args.l_tau * 4 * g.n_q * 2 / dtp,
                 "ms_per_sweep": 1000.0 * dtp / 2, "g_err_max": max(e[0] for e in gep)}
        if "tau_int_long_run" in out:
            plain["indep_samples_per_s"] = (2 / dtp) / (2 * max(TAU_LONG["tau_int"].values()))
            out["indep_samples_ratio_vs_plain_fp64"] = out["indep_samples_per_s"] / plain["indep_samples_per_s"]
        elif tau:
            key = "indep_samples_per_s_upper_bound" if out.get("tau_int_is_lower_bound") else "indep_samples_per_s"
            plain[key] = (2 / dtp) / (2 * tau)
        out["plain_fp64_1chain"] = plain
        p.close()
        progress("one-chain FP64 reference done")
    if not args.no_batched and args.geometry == "torus":
        # the batched workload (64 chains over N_phi 24 / 48 / 72), short: one
        # warm-up and five timed sweeps, with recorded sweep graphs and launch
        # by launch
        bg = batched_run(args, prec, True, 5, 1)
        bl = batched_run(args, prec, False, 5, 1)
        out["batched"] = {"workload": "64 chains, N_phi 24/48/72 (32/16/16 chains, L_tau 60/120/180), paper cutoff, "
                                      "u grid 0.5..3.0 (16 points), recompute every 10 slices, %s, 5 timed sweeps"
                                      % args.precision,
                          "graph": bg, "launch_by_launch": bl, "graph_speedup": bg["value"] / bl["value"]}
        progress("batched leg done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.n_phi, args.l_tau, args.dtau, args.u, args.cpu_seconds,
                                           args.geometry == "sphere")
        progress("CPU oracle baseline done")
    print(json.dumps(out))


def learned_leg(g, s, args, sweep_s):
    """The learned global proposal on the timed chains (Methods' local Langevin
    sweep stays the judge): the configurations of the tau_int sweeps (every
    chain after every sweep, with their exact FP64 ln w_F) train the
    effective-action network on the GPU, the last four sweeps held out, with
    early stopping on the held-out loss; then global moves (HMC on the learned
    action, exact determinant test) of every chain, trained network against the
    Gaussian proposal (network = 0), on all fields and on the slow uniform q = 0
    subspace."""
    import numpy as np
    import torch
    n_val = min(4 * g.n_chains, s.n_data() // 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tl, vl, be = s.train_heldout(max_epochs=200, batch=256, lr=1e-3, n_val=n_val, patience=8, refit_norm=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w = s.get_params()
    res = {"configurations": s.n_data(), "heldout": n_val, "best_epoch": be, "train_loss": tl,
           "heldout_loss": vl, "heldout_r2": 1.0 - vl, "train_s": t_train,
           "network": "3 layers, hidden 256, BF16 products (gfx950 16x16x32 MFMA), FP32 Adam",
           "moves": []}
    for sub, step in (("all", 0.002), ("uniform_q0", 0.5)):
        s.set_subspace(sub)
        row = {"subspace": sub, "step": step, "n_leap": 4}
        for name, wv in (("trained", w), ("gaussian", np.zeros_like(w))):
            s.set_params(wv)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            mv = s.global_move(1, 4, step)
            torch.cuda.synchronize()
            row["acceptance_" + name] = sum(m["accepted"] for m in mv) / len(mv)
            row["move_over_sweep_" + name] = (time.perf_counter() - t1) / sweep_s
        res["moves"].append(row)
    s.set_subspace("all")
    s.set_params(w)
    return res


def bench_tau_long(args, prec):
    """Integrated autocorrelation times at the N_phi = 100 shape from a long
    run: --chains chains (default here 32) of the c3 workload, --therm
    thermalisation sweeps, then --tau-sweeps sweeps (default here 1000) whose
    m^2_SO(5), action and q = 0 field-power series give tau_int pooled over
    the chains, with Sokal's window; a window that does not close is reported."""
    import numpy as np
    import torch
    from paper_2605_03700_amd import Batch, Q_BZ, Q_PAPER
    from paper_2605_03700_amd.analysis import tau_int_pooled
    chains = args.chains if args.chains != 256 else 32
    n_sw = args.tau_sweeps if args.tau_sweeps != 40 else 1000
    b = Batch([dict(n_phi=args.n_phi, l_tau=args.l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u,
                    n_stab=args.n_stab, precision=prec, eps0=0.3, adapt_eps=True, seed=3, n_chains=chains,
                    tile_cfg=args.tile_cfg, q_mode=Q_BZ if args.q_mode == "bz" else Q_PAPER,
                    precision_guard=0 if args.no_guard else 1, guard_gmax=args.guard_gmax,
                    guard_err=args.guard_err)])
    g = b.groups[0]
    b.init_fields()
    if args.therm:
        b.sweep(args.therm)
    progress("tau-long: %d chains thermalised (%d sweeps)" % (chains, args.therm))
    n0 = len(g.series(0))
    acc = prop = 0
    g_abs = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def series_now():
        return {obs: np.array([g.series(k, obs)[n0:] for k in range(chains)]) for obs in
                ("m2", "action", "phi_q0_power")}
    for i in range(n_sw):
        st = b.sweep(1)
        acc += sum(x["accepted"] for x in st)
        prop += sum(x["proposed"] for x in st)
        g_abs = max(g_abs, max(x["max_stab_err"] for x in st))
        if (i + 1) % 10 == 0:
            progress("tau-long: %d of %d sweeps (%.1f s)" % (i + 1, n_sw, time.perf_counter() - t0))
        if args.series_out and (i + 1) % 100 == 0:
            np.savez(args.series_out, **series_now())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ser = series_now()
    if args.series_out:
        np.savez(args.series_out, **ser)
    taus = {}
    for obs, arr in ser.items():
        t_o, win, closed = tau_int_pooled(list(arr))
        taus[obs] = {"tau_int": float(t_o), "window": int(win), "window_closed": bool(closed)}
    tau = max(v["tau_int"] for v in taus.values())
    print(json.dumps({
        "metric": "integrated autocorrelation time (sweeps) at N_phi=100", "value": tau, "unit": "sweeps",
        "n_gpus": 1, "steps": n_sw, "warmup": args.therm, "ms_per_step": 1000.0 * dt / n_sw,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": "tau-long: torus N_phi=%d L_tau=%d dtau=%g u=%g %s, %d chains, %d sweeps "
                               "after %d" % (args.n_phi, args.l_tau, args.dtau, args.u,
                                             "Brillouin zone" if args.q_mode == "bz" else "paper cutoff",
                                             chains, n_sw, args.therm)},
        "tau_int": taus, "acceptance": acc / max(1, prop), "g_err_max": g_abs,
        "m2_mean": float(ser["m2"].mean()),
        "m2_stderr": float(ser["m2"].std() * np.sqrt(2 * taus["m2"]["tau_int"] / ser["m2"].size)),
        "sweeps_per_s_per_chain": n_sw / dt,
        "indep_samples_per_s": chains * n_sw / dt / (2 * tau) if all(v["window_closed"] for v in taus.values())
        else None}))
    b.close()


def bench_oracle_tau(args):
    """The FP64 oracle's own Markov chain on the host (the CPU baseline's
    autocorrelation): one chain of the given shape, --therm sweeps with the step
    size adapting, then --tau-sweeps sweeps at the frozen step; tau_int of
    m^2_SO(5), the action and the q = 0 field power with Sokal's window, and
    the mean of m^2_SO(5) with its autocorrelation-corrected error."""
    import numpy as np
    import synth
    from oracle import dqmc
    from oracle.model import Model, Q_BZ, Q_PAPER
    from oracle.observables import so5_observables
    from paper_2605_03700_amd.analysis import tau_int
    n_sw = args.tau_sweeps if args.tau_sweeps != 40 else 2000
    m = Model(args.n_phi, args.l_tau, args.dtau, u0=1.0, uk=args.u, un=args.u,
              q_mode=Q_BZ if args.q_mode == "bz" else Q_PAPER)
    ch = dqmc.Chain(m, synth.fields(1, args.l_tau, m.n_q), eps0=0.3, adapt=True)
    rp = synth.replay(2, args.therm + n_sw, args.l_tau, m.n_q)
    for i in range(args.therm):
        ch.sweep(rp[i])
    ch.adapt = False
    ser = {"m2": [], "action": [], "phi_q0_power": []}
    t0 = time.perf_counter()
    for i in range(n_sw):
        ch.sweep(rp[args.therm + i])
        Bs = dqmc.propagators(m, ch.phi)
        G = dqmc.green(m, ch.phi, args.l_tau, Bs)
        ser["m2"].append(float(np.real(so5_observables(G, args.n_phi)[1])))
        ser["action"].append(0.5 * float(np.sum(ch.phi ** 2)) - float(np.real(dqmc.logdet(m, ch.phi, Bs))))
        ser["phi_q0_power"].append(float(np.sum(ch.phi[:, :, 0].sum(axis=0) ** 2)) / args.l_tau)
        if (i + 1) % 100 == 0:
            progress("oracle-tau: %d of %d sweeps (%.1f s)" % (i + 1, n_sw, time.perf_counter() - t0))
    dt = time.perf_counter() - t0
    taus = {}
    for k, v in ser.items():
        t, w = tau_int(v)
        taus[k] = {"tau_int": float(t), "window": int(w)}
    m2 = np.array(ser["m2"])
    print(json.dumps({
        "metric": "oracle integrated autocorrelation time (sweeps)", "value": max(v["tau_int"] for v in taus.values()),
        "unit": "sweeps", "n_gpus": 0, "steps": n_sw, "warmup": args.therm, "ms_per_step": 1000.0 * dt / n_sw,
        "higher_is_better": False, "data": "synthetic", "dtype": "f64",
        "config": {"workload": "oracle-tau: torus N_phi=%d L_tau=%d dtau=%g u=%g %s, one chain on the host"
                               % (args.n_phi, args.l_tau, args.dtau, args.u, args.q_mode)},
        "tau_int": taus, "eps": ch.eps, "acceptance": float(np.mean([h[2] for h in ch.history[-n_sw * args.l_tau:]])),
        "m2_mean": float(m2.mean()), "m2_stderr": float(m2.std() * np.sqrt(2 * taus["m2"]["tau_int"] / m2.size)),
        "sweeps_per_s": n_sw / dt}))


def bench_tau(args, prec):
    """Imaginary-time correlator passes (G(tau,0), G(0,tau), G(tau,tau) and
    m^2_SO(5)(tau, q=0) for tau = 0..L) over the chains of the c3 workload at
    their initial fields: one untimed pass, then --steps timed passes."""
    import numpy as np
    import torch
    from paper_2605_03700_amd import Batch, Q_PAPER, Q_SPHERE
    geo = dict(q_mode=Q_SPHERE if args.geometry == "sphere" else Q_PAPER, exp_squarings=args.exp_squarings)
    b = Batch([dict(n_phi=args.n_phi, l_tau=args.l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u,
                    n_stab=args.n_stab, precision=prec, eps0=0.3, adapt_eps=True, seed=3, n_chains=args.chains,
                    tile_cfg=args.tile_cfg, **geo)])
    g = b.groups[0]
    b.init_fields()
    g.measure_tau()
    progress("warm-up pass done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_max = 0.0
    for _ in range(args.steps):
        _, st = g.measure_tau(with_stab=True)
        st_max = max(st_max, float(st.max()))
    dt = (time.perf_counter() - t0) / args.steps
    n_sp = 2 * args.n_phi
    chan_flops = 12.0 * args.l_tau * 16.0 * args.n_phi ** 2 * n_sp * args.chains
    print(json.dumps({
        "metric": "imaginary-time correlator passes (G(tau,0), G(0,tau), G(tau,tau), m^2_SO(5)(tau)) per second",
        "value": args.chains / dt, "unit": "chain-passes/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1000.0 * dt, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s N_phi=%d L_tau=%d dtau=%g u=%g, %d chains, recompute every %d slices"
                               % (args.geometry, args.n_phi, args.l_tau, args.dtau, args.u, args.chains,
                                  args.n_stab)},
        "channel_application_tflops": chan_flops / dt / 1e12,
        "carried_vs_recomputed_rel_max": st_max}))
    b.close()


def batched_run(args, prec, graph, steps, warmup):
    """64 independent chains in one job: 32 at N_phi=24 (L=60), 16 at N_phi=48
    (L=120), 16 at N_phi=72 (L=180), paper cutoff, u on the grid 0.5 + j/6
    (j = 0..15), dtau = 0.1. One context per N_phi group, each on its own
    stream; a step is one sweep of every chain. graph: each group's sweep is one
    launch of its recorded graph (else launch by launch, the groups' slice
    steps interleaved). The kernel timing of the N_phi = 72 group's channel
    application comes from one more sweep of that group alone."""
    import torch
    from paper_2605_03700_amd import Batch
    grid = [0.5 + j / 6.0 for j in range(16)]
    groups = []
    for k, (n_phi, nch) in enumerate([(24, 32), (48, 16), (72, 16)]):
        groups.append(dict(n_phi=n_phi, l_tau=10 * n_phi // 4, dtau=args.dtau, n_stab=10, precision=prec,
                           eps0=0.3, adapt_eps=True, seed=400 + k, n_chains=nch,
                           chain_u=[(1.0, grid[c % 16], grid[c % 16]) for c in range(nch)],
                           tile_cfg=args.tile_cfg, sweep_graph=int(graph)))
    b = Batch(groups)
    b.init_fields()
    if warmup:
        b.sweep(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = b.sweep(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the N_phi = 72 group's timed launches in one more sweep of that group
    # alone (after the timed batch sweeps): in a batch sweep the other groups'
    # kernels share the GPU and the events would time the contention
    g72 = b.groups[2]
    g72.kernel_timing(True)
    g72.sweep(1)
    k_ms, k_count, k_flops = g72.kernel_timing_read()
    g72.kernel_timing(False)
    fields = sum(g.n_chains * g.l_tau * 4 * g.n_q for g in b.groups) * steps
    out = {
        "value": fields / dt, "ms_per_step": 1000.0 * dt / steps, "sweep_graph": bool(graph),
        "chains": b.n_chains, "n_q": [g.n_q for g in b.groups],
        "tile_cfg": [list(g.tile_config()) for g in b.groups],
        "acceptance": sum(s["accepted"] for s in st) / max(1, sum(s["proposed"] for s in st)),
        "g_err_max": max(s["max_stab_err"] for s in st),
        "g_err_rel_max": max(s["max_stab_rel"] for s in st),
        "acceptance_min_chain": chain_acceptance([st])[0],
        "frozen_chains": chain_acceptance([st])[1],
    }
    if k_count > 0 and k_ms > 0:
        algo = 2.0 * (2 * 72) ** 3 * g72.n_chains
        ach = algo / (k_ms * 1e-3) / 1e12
        issued = k_flops / (k_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "kernel": "chan_apply (N_phi=72 group, timed in a sweep of that "
                                                     "group alone)", "achieved": ach,
                           "peak": PEAK[args.precision], "unit": "TFLOP/s", "frac": ach / PEAK[args.precision],
                           "traffic": None, "avg_launch_ms": k_ms, "launches_timed": k_count,
                           "flops_per_launch": algo, "issued_flops_per_launch": k_flops,
                           "issued_tflops": issued, "issued_frac": issued / PEAK[args.precision]}
    b.close()
    return out


def bench_batched(args, prec):
    """The batched workload as its own bench line (see batched_run), recorded
    sweep graphs unless --no-graph."""
    r = batched_run(args, prec, not args.no_graph, args.steps, args.warmup)
    out = {
        "metric": "field updates/s + indep. samples/s at N_phi=100, plain vs learned/FP32; G err",
        "value": r.pop("value"), "unit": "field updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "batched: 64 chains, N_phi 24/48/72 (32/16/16 chains, L_tau 60/120/180), "
                               "paper cutoff, u grid 0.5..3.0 (16 points), recompute every 10 slices",
                   "chains": r.pop("chains"), "precision": args.precision, "n_q": r.pop("n_q"),
                   "tile_cfg": r.pop("tile_cfg"), "sweep_graph": r.pop("sweep_graph")},
        "g_err_definition": "max over chains and recomputation points of max|G_updated - G_FP64| (absolute, "
                            "max norm); g_err_rel_max divides by max|G_FP64| of the chain",
    }
    out.update(r)
    print(json.dumps(out))


def bench_learned(args, prec):
    """Learned global proposal at N_phi = 140 (spin block n = 280), L = 600,
    paper cutoff, u on the SO(5) line: plain local sweeps of --learned-chains
    chains (timed: the value), every sweep's configurations collected with
    their exact FP64 ln w_F, the effective-action network (three layers,
    hidden 256, BF16 products, FP32 Adam) trained on the GPU, its held-out R^2
    against -ln w_F, and global moves (HMC on S_eff, exact determinant test)
    with the trained network and with the Gaussian proposal (network = 0) at a
    few trajectory lengths. The collection is --learned-sweeps sweeps, far
    below the 10^4 configurations a production training set would hold."""
    import numpy as np
    import torch
    from paper_2605_03700_amd import CFQMC, Slmc
    n_phi, l_tau, nch = 140, 600, args.learned_chains
    g = CFQMC(n_phi=n_phi, l_tau=l_tau, dtau=args.dtau, u0=1.0, uk=args.u, un=args.u, n_stab=args.n_stab,
              precision=prec, n_chains=nch, seed=7, eps0=0.3, adapt_eps=True, tile_cfg=args.tile_cfg)
    n_sw = args.learned_sweeps
    s = Slmc(g, hidden=256, n_qbins=16, n_wbins=16, capacity=nch * (n_sw + 4), max_batch=256, seed=11)
    g.init_fields(None)
    progress("learned workload: context and network created")
    if args.warmup:
        g.sweep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc, prop = 0, 0
    for _ in range(n_sw):
        st = g.sweep(1)
        acc += sum(x["accepted"] for x in st)
        prop += sum(x["proposed"] for x in st)
        s.collect()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    progress("learned workload: %d sweeps collected (%.1f s per sweep)" % (n_sw, dt / n_sw))
    w0 = s.get_params()
    t1 = time.perf_counter()
    loss0 = s.train(epochs=1, batch=32, lr=1e-3, refit_norm=True)
    s.set_params(w0)
    loss = s.train(epochs=args.learned_epochs, batch=32, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    w_trained = s.get_params()
    res, lnw = [], []
    for _ in range(2):
        g.sweep(1)
        snn = s.action(g.get_fields())
        for z in range(nch):
            lw = g.logdet(z).real
            lnw.append(lw)
            res.append(snn[z] + lw)
    r2 = 1.0 - float(np.var(res) / np.var(lnw))
    progress("learned workload: trained (R^2 %.3f)" % r2)
    moves = []
    for step in (0.002, 0.01, 0.05):
        row = {"step": step, "n_leap": 4}
        for name, w in (("trained", w_trained), ("gaussian", np.zeros_like(w_trained))):
            s.set_params(w)
            a, n_mv = 0, 0
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(2):
                mv = s.global_move(1, 4, step)
                a += sum(m["accepted"] for m in mv)
                n_mv += len(mv)
            torch.cuda.synchronize()
            row["acceptance_" + name] = a / n_mv
            row["ms_per_move_" + name] = 1000.0 * (time.perf_counter() - t2) / 2
        moves.append(row)
        progress("learned workload: global moves at step %g done" % step)
    # the uniform q = 0 amplitudes A_i = sum_tau phi^i_{tau,0} / sqrt(L) relax
    # slowest under local moves: their mean squared change per local sweep and
    # per global move restricted to the q = 0 subspace (same network)
    def amps():
        return g.get_fields()[:, :, :, 0].sum(axis=1) / np.sqrt(l_tau)      # [chain][4]
    s.set_params(w_trained)
    a_0 = amps()
    g.sweep(1)
    a_1 = amps()
    local_msd = float(np.mean(np.sum((a_1 - a_0) ** 2, axis=1)))
    sub_moves = []
    for sub, steps, reps in (("q0", (0.05, 0.2), 2), ("uniform_q0", (0.25, 0.5, 0.75), 4)):
        s.set_subspace(sub)
        for step in steps:
            row = {"subspace": sub, "step": step, "n_leap": 4}
            for name, w in (("trained", w_trained), ("gaussian", np.zeros_like(w_trained))):
                s.set_params(w)
                a, n_mv, msd = 0, 0, 0.0
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                for _ in range(reps):
                    before = amps()
                    mv = s.global_move(1, 4, step)
                    after = amps()
                    a += sum(m["accepted"] for m in mv)
                    n_mv += len(mv)
                    msd += float(np.sum((after - before) ** 2))
                t_mv = (time.perf_counter() - t3) / reps
                row["acceptance_" + name] = a / n_mv
                row["q0_amplitude_msd_" + name] = msd / n_mv
                # per unit of sweep time, against the local sweep's
                row["msd_per_sweep_time_" + name] = (msd / n_mv) / (t_mv / (dt / n_sw))
            sub_moves.append(row)
            progress("learned workload: %s subspace moves at step %g done" % (sub, step))
    s.set_subspace("all")
    fields = nch * l_tau * 4 * g.n_q * n_sw
    out = {
        "metric": "field updates/s + indep. samples/s at N_phi=100, plain vs learned/FP32; G err",
        "value": fields / dt, "unit": "field updates/s", "n_gpus": 1, "steps": n_sw, "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / n_sw, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "learned: torus N_phi=%d L_tau=%d dtau=%g u=%g paper cutoff n_q=%d, %d chains, "
                               "FP64 recompute every %d slices; MLP hidden 256 on 16 x 16 periodogram bins"
                               % (n_phi, l_tau, args.dtau, args.u, g.n_q, nch, args.n_stab),
                   "chains": nch, "precision": args.precision, "n_q": g.n_q, "tile_cfg": list(g.tile_config())},
        "acceptance": acc / max(1, prop),
        "learned": {"configurations": s.n_data(), "train_epochs": args.learned_epochs,
                    "train_loss_first_epoch": loss0, "train_loss_last": loss, "train_s": t_train,
                    "heldout_r2": r2, "heldout_points": len(lnw), "global_moves": moves,
                    "subspace_moves": {"local_sweep_q0_amplitude_msd": local_msd, "global_moves": sub_moves,
                                    "definition": "mean over chains of sum_i (A_i' - A_i)^2, A_i = sum_tau "
                                                  "phi^i_{tau,q=0} / sqrt(L), per local sweep and per global "
                                                  "move (rejections count as zero change)"}},
    }
    s.close()
    g.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
