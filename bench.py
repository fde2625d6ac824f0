#!/usr/bin/env python3
"""Benchmark one Henon Monte Carlo step (sort + potential + relax + orbit) on
one MI355X: star-updates per second, per-phase times from HIP events recorded
on the stream the kernels run on, the roofline of the dominant phase, and the
FP64 oracle timed on the host for reference.

python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64|mixed]

The other precision form runs on the same initial model right after the
timed run and is reported beside it ("other_precision").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "star-updates/s (sort+Φ+relax+orbit) at N=1e6/1e7, mixed vs FP64, % HBM roofline"

# Seeded synthetic Plummer workloads, each with the precision it is quoted in.
WORKLOADS = {
    # headline: 10^7 stars, broken power-law masses stored as f32, ln(0.01 N)
    "plummer_n1e7_broken_power_law": dict(n=10_000_000, mass_spectrum=1, m_f32=True,
                                          gamma=0.01, seed=1, precision="mixed"),
    "plummer_n1e6_equal_mass": dict(n=1_000_000, mass_spectrum=0, m_f32=False, gamma=0.11,
                                    seed=1, precision="mixed"),
    "plummer_n1e5_equal_mass": dict(n=100_000, mass_spectrum=0, m_f32=False, gamma=0.11,
                                    seed=1, precision="fp64"),
    # 64 independent clusters, N log-uniform in [1e4, 1e6], even clusters
    # Plummer and odd ones King W0 = 6, advanced together by one captured graph
    "ensemble_64_plummer_king_w6": dict(clusters=64, seed=1, gamma=0.11, w0=6.0, m_f32=False,
                                        precision="mixed"),
    # the paper's validation runs (Sec. 4): equal-mass Plummer spheres of 1e5,
    # 1e6 and 1e7 stars evolved to core collapse; --steps / --warmup unused
    "core_collapse_plummer_n1e5_1e6_1e7": dict(core_collapse=(100_000, 1_000_000, 10_000_000),
                                               seed=1, gamma=0.11, precision="mixed"),
}
DEFAULT_WORKLOAD = "plummer_n1e7_broken_power_law"

PHASES = ("potential", "timestep", "relax", "orbit", "sort")
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def alg_bytes(m_bytes: int) -> dict:
    """Minimum HBM bytes per star-update of each step: every array the step
    must read once and write once (table probes that hit cache excluded)."""
    return {
        # read r, m; write phi
        "potential": 8 + m_bytes + 8,
        # read m, vr, vt, half an id, two bin-edge radii per 20 stars; write vr, vt
        "relax": m_bytes + 8 + 8 + 2 + 0.8 + 16,
        # read r, phi, vr, vt, id; write r_new, vr, vt
        "orbit": 8 + 8 + 8 + 8 + 4 + 24,
        # read and write the record r, vr, vt, m, id
        "sort": 2 * (8 + 8 + 8 + m_bytes + 4),
    }


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_SAMPLE_N = 3_000_000  # oracle sample: about 5 s per serial step on the GPU machine's host


def cpu_baseline(wl: dict) -> dict:
    """The oracle as it stands: one step of a sample of the same workload
    (same generator, mass spectrum and Coulomb logarithm) timed on the host,
    serial (the parity reference, one core) and in its OpenMP build on every
    core (same results bit for bit: per-star and per-pair loops in parallel,
    the scan, the sort and every sum serial)."""
    import numpy as np
    import oracle

    n = min(wl["n"], CPU_SAMPLE_N)
    st = oracle.plummer(n, wl["seed"], wl["mass_spectrum"])
    if wl["m_f32"]:
        st.m = st.m.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    ser, _ = oracle.step(st, wl["seed"], 0, wl["gamma"])
    el = time.perf_counter() - t0
    with oracle.threads() as L:
        threads = int(L.ora_threads())
        t0 = time.perf_counter()
        par, _ = oracle.step(st, wl["seed"], 0, wl["gamma"])
        el_p = time.perf_counter() - t0
    same = bool(np.array_equal(ser.r, par.r) and np.array_equal(ser.id, par.id))
    return {"value": n / el, "unit": "star-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of a {n}-star sample of the workload, serial FP64 C oracle, "
                      f"{el:.2f} s",
            "cpu": cpu_model(),
            "all_cores": {"value": n / el_p, "cores": threads, "seconds": el_p,
                          "same_result_as_serial": same,
                          "note": "OpenMP build of the oracle: the per-star and per-pair "
                                  "loops on every core; potential scan, sort and sums serial"}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: the precision the workload is quoted in")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the run of the other precision form")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the N = 1e6 and ensemble legs of the default run")
    ap.add_argument("--uncorrected", action="store_true",
                    help="core-collapse workload: run without the energy correction")
    ap.add_argument("--energy-corr", action="store_true",
                    help="with --plain: steps with the potential-change energy correction")
    ap.add_argument("--lfsr113", action="store_true",
                    help="with --plain: steps drawing from per-star LFSR113 streams")
    ap.add_argument("--plain", action="store_true",
                    help="time plain cmc_step calls only (no per-phase events); for profilers")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB, --steps times "
                         "(checks the byte formula of the L2 request counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "step over several GPUs is not built", file=sys.stderr)
        return 2

    import torch

    import paper_1206_5878_amd as P
    from paper_1206_5878_amd.hipevents import EventSet

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_mib:
        nb = args.copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        el = e0.elapsed_time(e1) * 1e-3
        print(json.dumps({"mode": "copy", "bytes_per_copy": nb, "copies": args.steps,
                          "GBs_read_plus_write": 2 * nb * args.steps / el / 1e9}), flush=True)
        return 0
    wl = WORKLOADS[args.workload]
    precision = args.precision or wl["precision"]
    K = args.steps
    if "clusters" in wl:
        return ensemble_bench(P, args, wl, precision)
    if "core_collapse" in wl:
        return core_collapse_bench(P, args, wl, precision)
    if args.plain:
        prec = P.CMC_FP64 if precision == "fp64" else P.CMC_MIXED
        cl, params = setup(P, wl, prec, args.warmup, lfsr=args.lfsr113)
        params.energy_corr = 1 if args.energy_corr else 0
        n_start = cl.n
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            params.step = args.warmup + k
            P.cmc_step(cl, params)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"metric": METRIC, "value": n_start * K / el, "unit": "star-updates/s",
                          "n_gpus": 1, "steps": K, "warmup": args.warmup,
                          "ms_per_step": el / K * 1e3, "mode": "plain", "n_start": n_start,
                          "n_end": cl.n, "workload": args.workload, "precision": precision,
                          "energy_corr": bool(args.energy_corr), "lfsr113": bool(args.lfsr113)}),
              flush=True)
        return 0

    run = timed_run(P, EventSet, wl, precision, K, args.warmup, corr_too=True)
    other = "fp64" if precision == "mixed" else "mixed"
    run_o = None if args.no_other else timed_run(P, EventSet, wl, other, K, args.warmup)

    m_bytes = 4 if wl["m_f32"] else 8
    ab = alg_bytes(m_bytes)
    phase_ms, n_mean = run["phases_ms"], run["n_mean"]
    # timestep + relax are the relaxation unit of the algorithmic-byte table
    unit_ms = {"potential": phase_ms["potential"],
               "relax": phase_ms["timestep"] + phase_ms["relax"],
               "orbit": phase_ms["orbit"], "sort": phase_ms["sort"]}
    dom = max(unit_ms, key=unit_ms.get)
    dom_gbs = ab[dom] * n_mean / (unit_ms[dom] * 1e-3) / 1e9
    step_bytes = sum(ab.values())
    value = run["value"]
    traffic = measured_traffic(args.workload, precision, dom)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "star-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": wl["n"], "precision": precision,
                   "mass_spectrum": wl["mass_spectrum"], "m_f32": wl["m_f32"],
                   "gamma": wl["gamma"], "seed": wl["seed"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dom_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     # the measured HBM bytes per launch over the same mean duration
                     "traffic_GBs": (traffic / (unit_ms[dom] * 1e-3) / 1e9
                                     if traffic is not None else None),
                     "alg_bytes_per_star": ab[dom],
                     "launch_ms": unit_ms[dom], "stars_per_launch": n_mean},
        "step_roofline": {"alg_bytes_per_star": step_bytes,
                          "achieved_GBs": value * step_bytes / 1e9,
                          "frac": value * step_bytes / 1e9 / HBM_PEAK_GBS},
        "phases_ms": phase_ms,
        "timing": "hipGraph replays of one captured step (dt_iters = %d: warm-started dt "
                  "solves converge in 2-3 Newton iterations, checked through "
                  "CMC_ST_DT_NOCONV); 'calls' times the same number of plain cmc_step_timed "
                  "calls first (default 10 iterations), which also give the per-phase split"
                  % GRAPH_DT_ITERS,
        "gpu_ms_per_step": run["gpu_ms_per_step"],
        "calls": run["calls"],
        # the same step with the potential-change energy correction (Sec. 2.1
        # item 6), which the headline metric's step list leaves out
        "with_energy_correction": run["with_energy_correction"],
        # the same step drawing from per-star LFSR113 streams (Sec. 3.6)
        "with_lfsr113": lfsr_rate(P, wl, precision, K, args.warmup),
        "final": run["final"],
    }
    if run_o is not None:
        out["other_precision"] = {"precision": other, "value": run_o["value"],
                                  "ms_per_step": run_o["ms_per_step"],
                                  "calls": run_o["calls"],
                                  "phases_ms": run_o["phases_ms"], "final": run_o["final"]}
    out["launch_table"] = tune_entry(P, wl["n"])
    if not args.no_legs:
        # the other metric point (N = 1e6) and the batched ensemble
        out["legs"] = {
            "plummer_n1e6_equal_mass": point_leg(P, EventSet, "plummer_n1e6_equal_mass", K,
                                                 args.warmup),
            "ensemble_64_plummer_king_w6": ensemble_leg(
                P, WORKLOADS["ensemble_64_plummer_king_w6"],
                WORKLOADS["ensemble_64_plummer_king_w6"]["precision"], K, args.warmup),
        }
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    return 0


def ensemble_specs(P, wl) -> list:
    """Cluster c: N = floor(10^(4 + 2u)) with u the uniform of Philox word
    pair (w1:w0) at key = seed, counter (c, 0, 0x40, 0); seed c + 1; Plummer
    for even c, King W0 for odd c."""
    import numpy as np
    k = wl["clusters"]
    ctr = np.zeros((k, 4), np.uint32)
    ctr[:, 0] = np.arange(k)
    ctr[:, 2] = 0x40
    w = P.cmc_philox(wl["seed"], ctr).astype(np.uint64)
    x = ((w[:, 1] << np.uint64(32)) | w[:, 0]) >> np.uint64(12)
    u = (2.0 * x.astype(np.float64) + 1.0) * 2.0 ** -53
    n = np.floor(10.0 ** (4.0 + 2.0 * u)).astype(np.int64)
    return [dict(n=int(n[c]), seed=c + 1, gamma=wl["gamma"], model=c % 2, w0=wl["w0"])
            for c in range(k)]


def ensemble_leg(P, wl, precision, K, warmup, drift_steps=50) -> dict:
    """The ensemble advanced by one captured graph per step (device step
    counter), against the same clusters stepped one by one with the
    single-cluster call in FP64; then drift_steps corrected steps of each
    form from the same initial models, with each cluster's relative energy
    change (T + W after the last pending correction) in both forms."""
    import numpy as np
    import torch
    prec = P.CMC_FP64 if precision == "fp64" else P.CMC_MIXED
    specs = ensemble_specs(P, wl)
    ens = P.Ensemble(specs, m_f32=wl["m_f32"])
    ens.init()
    params = P.Params(precision=prec)
    g = ens.capture(params)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    n0 = sum(cl.n for cl in ens.clusters)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(K):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1) / K
    n1 = sum(cl.n for cl in ens.clusters)
    updates = K * 0.5 * (n0 + n1)  # escapers leave a few stars per step
    stats = [cl.scalars() for cl in ens.clusters]
    del g
    print(f"# ensemble {precision}: {el / K * 1e3:.3f} ms/step (graph replays)",
          file=sys.stderr, flush=True)

    def loop(prec_loop, steps, first, corr=0):
        for k in range(first, first + steps):
            for cl, sp in zip(ens.clusters, specs):
                P.cmc_step(cl, P.Params(seed=sp["seed"], gamma=sp["gamma"], step=k,
                                        precision=prec_loop, energy_corr=corr))

    # the same clusters, one single-cluster FP64 call each per step
    ens.init()
    loop(P.CMC_FP64, warmup, 0)
    torch.cuda.synchronize()
    m0 = sum(cl.n for cl in ens.clusters)
    t1 = time.perf_counter()
    loop(P.CMC_FP64, K, warmup)
    torch.cuda.synchronize()
    el_loop = time.perf_counter() - t1
    m1 = sum(cl.n for cl in ens.clusters)
    print(f"# per-cluster FP64 loop: {el_loop / K * 1e3:.3f} ms/step",
          file=sys.stderr, flush=True)

    def energies():
        ens.potential(P.CMC_FP64)
        ens.energy_correction()
        return np.array([d["E"] for d in ens.diagnostics()])

    # drift: the batched form in its precision against the FP64 loop
    ens.init()
    E0 = energies()
    gc = ens.capture(P.Params(precision=prec, energy_corr=1))
    for _ in range(drift_steps):
        gc.replay()
    torch.cuda.synchronize()
    del gc
    d_b = (energies() - E0) / np.abs(E0)
    ens.init()
    loop(P.CMC_FP64, drift_steps, 0, corr=1)
    d_f = (energies() - E0) / np.abs(E0)
    diff = np.abs(d_b - d_f)
    return {
        "value": updates / el,
        "ms_per_step": el / K * 1e3,
        "gpu_ms_per_step": gpu_ms,
        "stars": n0,
        "clusters": len(specs),
        "n_min": min(sp["n"] for sp in specs), "n_max": max(sp["n"] for sp in specs),
        "precision": precision,
        "launch_table": tune_entry(P, max(cl.cap for cl in ens.clusters)),
        "per_cluster_fp64_calls": {"value": K * 0.5 * (m0 + m1) / el_loop,
                                   "ms_per_step": el_loop / K * 1e3},
        "drift": {"steps": drift_steps, "energy_corr": True,
                  "batched_rel_dE_max": float(np.abs(d_b).max()),
                  "fp64_loop_rel_dE_max": float(np.abs(d_f).max()),
                  "abs_difference_max": float(diff.max()),
                  "abs_difference_median": float(np.median(diff))},
        "final": {"n": n1, "status_or": int(np.bitwise_or.reduce([s["status"] for s in stats])),
                  "dt_min": min(s["dt"] for s in stats), "dt_max": max(s["dt"] for s in stats)},
    }


def ensemble_bench(P, args, wl, precision) -> int:
    leg = ensemble_leg(P, wl, precision, args.steps, args.warmup)
    out = {
        "metric": METRIC,
        "value": leg["value"],
        "unit": "star-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "clusters": wl["clusters"], "stars": leg["stars"],
                   "n_min": leg["n_min"], "n_max": leg["n_max"], "precision": precision,
                   "w0": wl["w0"], "gamma": wl["gamma"], "seed": wl["seed"], "graph": True},
        **{k: leg[k] for k in ("gpu_ms_per_step", "launch_table", "per_cluster_fp64_calls",
                               "drift", "final")},
    }
    print(json.dumps(out), flush=True)
    return 0


def tune_entry(P, cap: int) -> dict:
    """The launch-table entry the library uses for a capacity."""
    from paper_1206_5878_amd import tune
    return tune.get(cap)


def point_leg(P, EventSet, name: str, K: int, warmup: int) -> dict:
    """One more single-cluster workload: its precision and the other, each as
    plain calls (with phases) and graph replays, with the phase roofline."""
    wl = WORKLOADS[name]
    precision = wl["precision"]
    other = "fp64" if precision == "mixed" else "mixed"
    run = timed_run(P, EventSet, wl, precision, K, warmup)
    run_o = timed_run(P, EventSet, wl, other, K, warmup)
    ab = alg_bytes(4 if wl["m_f32"] else 8)
    step_bytes = sum(ab.values())
    return {"workload": name, "n": wl["n"], "precision": precision,
            "value": run["value"], "ms_per_step": run["ms_per_step"],
            "calls": run["calls"], "phases_ms": run["phases_ms"],
            "launch_table": tune_entry(P, wl["n"]),
            "step_roofline": {"alg_bytes_per_star": step_bytes,
                              "achieved_GBs": run["value"] * step_bytes / 1e9,
                              "frac": run["value"] * step_bytes / 1e9 / HBM_PEAK_GBS},
            "other_precision": {"precision": other, "value": run_o["value"],
                                "ms_per_step": run_o["ms_per_step"],
                                "phases_ms": run_o["phases_ms"]},
            "final": run["final"]}


LFSR_SEED = [0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321]
# Newton iterations enqueued in a captured step.  Every captured step here
# follows eager warm-up steps, so its dt solve starts from the last dt and
# converges in 2-3 iterations; an iteration after convergence is a no-op
# launch pair (~9 us).  A solve that ran out would raise CMC_ST_DT_NOCONV,
# which the runs below check.
GRAPH_DT_ITERS = 5


def graph_params(P, params):
    return P.Params(**{**params.__dict__, "dt_iters": GRAPH_DT_ITERS})


def check_dt(P, cl, what):
    st = int(cl.scalars()["status"])
    if st & P.ST_DT_NOCONV:
        raise RuntimeError(f"{what}: the dt solve ran out of iterations (status {st:#x})")


def setup(P, wl, prec, warmup, lfsr=False):
    import torch
    n0 = wl["n"]
    cl = P.Cluster(n0, m_f32=wl["m_f32"], rng=lfsr)
    P.cmc_init_plummer(cl, n0, wl["seed"], wl["mass_spectrum"])
    params = P.Params(seed=wl["seed"], gamma=wl["gamma"], precision=prec)
    if lfsr:
        P.cmc_rng_seed_lfsr113(cl, LFSR_SEED, 0)
        params.rng = P.CMC_RNG_LFSR113
    for k in range(warmup):
        params.step = k
        P.cmc_step(cl, params)
    torch.cuda.synchronize()
    print(f"# warmup done: {warmup} steps, n={cl.n}", file=sys.stderr, flush=True)
    return cl, params


def timed_run(P, EventSet, wl, precision, K, warmup, corr_too=False) -> dict:
    """K whole steps after the warm-up as plain calls, with inputs resident in
    HBM and per-phase times from HIP events on the library's stream; then K
    more as replays of one captured step (the headline rate); with corr_too,
    K more replays of the step with the potential-change energy correction."""
    import torch
    prec = P.CMC_FP64 if precision == "fp64" else P.CMC_MIXED
    cl, params = setup(P, wl, prec, warmup)
    ev = [EventSet(6) for _ in range(K)]
    nlog = torch.zeros(K + 1, dtype=torch.int64, device="cuda")
    nlog[0].copy_(cl.sc[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        params.step = warmup + k
        P.cmc_step_timed(cl, params, ev[k].h)
        nlog[k + 1].copy_(cl.sc[0])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    counts = nlog.cpu().tolist()
    updates = float(sum(counts[:K]))  # stars entering each timed step
    phase_ms = {ph: 0.0 for ph in PHASES}
    for k in range(K):
        for i, ph in enumerate(PHASES):
            phase_ms[ph] += ev[k].elapsed(i, i + 1)
    for e in ev:
        e.close()
    sc = cl.scalars()
    n_mean = updates / K
    print(f"# {precision}: {el / K * 1e3:.3f} ms/step (calls)", file=sys.stderr, flush=True)
    # The same cluster continues with K replays of one captured step (the step
    # index comes from the device counter, set to carry on from the calls).
    cl.set_scalar("step", warmup + K)
    g = cl.capture(graph_params(P, params))
    g.replay()  # steps warmup + K: not timed
    glog = torch.zeros(K + 1, dtype=torch.int64, device="cuda")
    glog[0].copy_(cl.sc[0])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(K):
        g.replay()
        glog[k + 1].copy_(cl.sc[0])
    e1.record()
    torch.cuda.synchronize()
    gel = time.perf_counter() - t0
    gupdates = float(sum(glog.cpu().tolist()[:K]))
    check_dt(P, cl, "graph replays")
    print(f"# {precision}: {gel / K * 1e3:.3f} ms/step (graph replays)", file=sys.stderr,
          flush=True)
    corr = None
    if corr_too:
        del g
        q = P.Params(**{**graph_params(P, params).__dict__, "energy_corr": 1})
        gc = cl.capture(q)
        gc.replay()  # leaves the first correction pending: not timed
        glog[0].copy_(cl.sc[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            gc.replay()
            glog[k + 1].copy_(cl.sc[0])
        torch.cuda.synchronize()
        cel = time.perf_counter() - t0
        check_dt(P, cl, "graph replays with the energy correction")
        corr = {"value": float(sum(glog.cpu().tolist()[:K])) / cel, "ms_per_step": cel / K * 1e3,
                "corr_skipped_last": int(cl.scalars()["corr_skipped"])}
        print(f"# {precision}: {cel / K * 1e3:.3f} ms/step (graph replays, energy correction)",
              file=sys.stderr, flush=True)
    return {"value": gupdates / gel, "ms_per_step": gel / K * 1e3, "with_energy_correction": corr,
            "gpu_ms_per_step": e0.elapsed_time(e1) / K,
            "calls": {"value": updates / el, "ms_per_step": el / K * 1e3},
            "n_mean": n_mean,
            "phases_ms": {ph: v / K for ph, v in phase_ms.items()},
            "final": {"n": sc["n"], "dt": sc["dt"], "status": sc["status"],
                      "trials_per_star": sc["trials"] / max(n_mean, 1),
                      "dt_iters": sc["dt_iters"]}}


def lfsr_rate(P, wl, precision, K, warmup) -> dict:
    """The same workload with every draw from the stars' LFSR113 streams (the
    generator of Sec. 3.6), timed as K replays of one captured step."""
    import torch
    prec = P.CMC_FP64 if precision == "fp64" else P.CMC_MIXED
    cl, params = setup(P, wl, prec, warmup, lfsr=True)
    cl.set_scalar("step", warmup)
    g = cl.capture(graph_params(P, params))
    glog = torch.zeros(K + 1, dtype=torch.int64, device="cuda")
    glog[0].copy_(cl.sc[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        g.replay()
        glog[k + 1].copy_(cl.sc[0])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    check_dt(P, cl, "LFSR113 graph replays")
    print(f"# {precision}: {el / K * 1e3:.3f} ms/step (graph replays, LFSR113 streams)",
          file=sys.stderr, flush=True)
    return {"value": float(sum(glog.cpu().tolist()[:K])) / el, "ms_per_step": el / K * 1e3}


def core_collapse_bench(P, args, wl, precision) -> int:
    """Wall-clock to core collapse (Sec. 4 validation runs), with the collapse
    time in initial half-mass relaxation times next to the paper's."""
    from paper_1206_5878_amd.evolve import core_collapse_run
    prec = P.CMC_FP64 if precision == "fp64" else P.CMC_MIXED
    runs = []
    for n in wl["core_collapse"]:
        res = core_collapse_run(n, wl["seed"], gamma=wl["gamma"], precision=prec,
                                energy_corr=not args.uncorrected)
        res.pop("series")
        runs.append(res)
        cc = res["collapse"] or {}
        print(f"# N={n}: t_cc = {cc.get('t_over_t_rh')} t_rh after {cc.get('steps')} steps, "
              f"{cc.get('wall_s')} s, energy drift {cc.get('energy_drift')}, budget "
              f"{cc.get('energy_budget')}", file=sys.stderr, flush=True)
    big = runs[-1]["collapse"] or {}
    out = {
        "metric": "wall-clock seconds to core collapse of an equal-mass Plummer sphere",
        "value": big.get("wall_s"),
        "unit": "s",
        "n_gpus": 1,
        "steps": big.get("steps"),
        "warmup": 0,
        "ms_per_step": (big["wall_s"] / big["steps"] * 1e3) if big else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": list(wl["core_collapse"]),
                   "precision": precision, "gamma": wl["gamma"], "seed": wl["seed"],
                   "energy_corr": not args.uncorrected},
        "runs": runs,
        "paper": {"t_cc_over_t_rh": [17.4, 16.7, 16.6],
                  "wall": ["11.4 min, 128 processors", "1.17 h, 256 processors",
                           "12.8 h, 1024 processors"]},
    }
    print(json.dumps(out), flush=True)
    return 0


def sources_sha256() -> str:
    """Hash of the kernel sources, to tell whether recorded counters still
    describe the library being timed."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1206_5878_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, phase: str):
    """HBM-side bytes per launch of the phase's kernels from the L2 request
    counter runs recorded under profiles/ (request counts by size, checked
    on a plain copy there), or None when they were taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != sources_sha256():
        return None
    v = kv.get(f"{phase}_bytes_per_launch")
    return float(v) if v else None


if __name__ == "__main__":
    sys.exit(main())
