#!/usr/bin/env python3
"""Benchmark one Henon Monte Carlo step (sort + potential + relax + orbit) on
one MI355X: star-updates per second, per-phase times from HIP events recorded
on the stream the kernels run on, the roofline of the dominant phase, and the
FP64 oracle timed on the host for reference.

python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64]
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

# Seeded synthetic workloads (Plummer models; see the design doc for the recipe).
WORKLOADS = {
    # headline: 10^7 stars, broken power-law masses stored as f32, ln(0.01 N)
    "plummer_n1e7_broken_power_law": dict(n=10_000_000, mass_spectrum=1, m_f32=True,
                                          gamma=0.01, seed=1),
    "plummer_n1e6_equal_mass": dict(n=1_000_000, mass_spectrum=0, m_f32=False, gamma=0.11,
                                    seed=1),
    "plummer_n1e5_equal_mass": dict(n=100_000, mass_spectrum=0, m_f32=False, gamma=0.11,
                                    seed=1),
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


def cpu_baseline(wl: dict) -> dict:
    """The oracle as it stands, one step of a 10^6-star sample of the same
    workload (same generator, mass spectrum and Coulomb logarithm), serial."""
    import oracle

    n = min(wl["n"], 1_000_000)
    st = oracle.plummer(n, wl["seed"], wl["mass_spectrum"])
    if wl["m_f32"]:
        import numpy as np
        st.m = st.m.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    new, info = oracle.step(st, wl["seed"], 0, wl["gamma"])
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "star-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of a {n}-star sample of the workload, serial FP64 C oracle, "
                      f"{el:.2f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain", action="store_true",
                    help="time plain cmc_step calls only (no per-phase events); for profilers")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB, --steps times "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this step is a design, not a build: see DESIGN.md", file=sys.stderr)
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
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"mode": "copy", "bytes_per_copy": nb, "copies": args.steps,
                          "GBs_read_plus_write": 2 * nb * args.steps / el / 1e9}), flush=True)
        return 0
    wl = WORKLOADS[args.workload]
    prec = P.CMC_FP64 if args.precision == "fp64" else P.CMC_MIXED
    n0 = wl["n"]
    cl = P.Cluster(n0, m_f32=wl["m_f32"])
    P.cmc_init_plummer(cl, n0, wl["seed"], wl["mass_spectrum"])
    params = P.Params(seed=wl["seed"], gamma=wl["gamma"], precision=prec)

    for k in range(args.warmup):
        params.step = k
        P.cmc_step(cl, params)
    torch.cuda.synchronize()
    print(f"# warmup done: {args.warmup} steps, n={cl.n}", file=sys.stderr, flush=True)

    K = args.steps
    if args.plain:
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
                          "n_end": cl.n, "workload": args.workload}), flush=True)
        return 0
    ev = [EventSet(6) for _ in range(K)]
    nlog = torch.zeros(K + 1, dtype=torch.int64, device="cuda")
    nlog[0].copy_(cl.sc[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        params.step = args.warmup + k
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
    phase_ms = {ph: v / K for ph, v in phase_ms.items()}
    sc = cl.scalars()

    m_bytes = 4 if wl["m_f32"] else 8
    ab = alg_bytes(m_bytes)
    n_mean = updates / K
    # timestep + relax are the relaxation unit of the algorithmic-byte table
    unit_ms = {"potential": phase_ms["potential"],
               "relax": phase_ms["timestep"] + phase_ms["relax"],
               "orbit": phase_ms["orbit"], "sort": phase_ms["sort"]}
    dom = max(unit_ms, key=unit_ms.get)
    dom_gbs = ab[dom] * n_mean / (unit_ms[dom] * 1e-3) / 1e9
    step_bytes = sum(ab.values())
    value = updates / el
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "star-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n0, "precision": args.precision,
                   "mass_spectrum": wl["mass_spectrum"], "m_f32": wl["m_f32"],
                   "gamma": wl["gamma"], "seed": wl["seed"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dom_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_star": ab[dom]},
        "step_roofline": {"alg_bytes_per_star": step_bytes,
                          "achieved_GBs": value * step_bytes / 1e9,
                          "frac": value * step_bytes / 1e9 / HBM_PEAK_GBS},
        "phases_ms": phase_ms,
        "final": {"n": sc["n"], "dt": sc["dt"], "status": sc["status"],
                  "trials_per_star": sc["trials"] / max(n_mean, 1), "dt_iters": sc["dt_iters"]},
    }
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
