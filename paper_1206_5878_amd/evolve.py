"""Long runs of the step: a Plummer sphere evolved towards core collapse, as in
the paper's validation runs (arXiv:1206.5878, Sec. 4), with the core sampled
along the way.

Time is the sum of the steps' Delta t, in units of the initial half-mass
relaxation time of Sec. 4, t_rh = 0.138 N / ln(0.1 N) (r_h^3 / G M)^(1/2)
(G = M = 1).  Steps are replays of one captured step (the step index comes
from the device counter).  Each step's Delta t, escaper energy and count of
stars the energy correction skipped are copied on the device, so the host
waits only when it samples the diagnostics.
"""
from __future__ import annotations

import math
import time

import torch

from . import _capi as A
from .cluster import (Cluster, Params, cmc_diagnostics, cmc_energy_correction, cmc_init_plummer,
                      cmc_potential)


def half_mass_relaxation_time(n: int, r_h: float, gamma: float = 0.1) -> float:
    """t_rh of Sec. 4 in Henon units (G = M = 1); gamma = 0.1 as there."""
    return 0.138 * n / math.log(gamma * n) * math.sqrt(r_h ** 3)


def density_slope(r, m, r_lo: float, r_hi: float, bins: int = 12) -> float:
    """Power-law index beta of rho ~ r^-beta between r_lo and r_hi: shell
    densities (mass over volume) in log-spaced shells, fitted by least
    squares in log-log."""
    import numpy as np
    edges = np.geomspace(r_lo, r_hi, bins + 1)
    mass, _ = np.histogram(r, bins=edges, weights=m)
    vol = 4.0 * np.pi / 3.0 * (edges[1:] ** 3 - edges[:-1] ** 3)
    mid = np.sqrt(edges[1:] * edges[:-1])
    ok = mass > 0
    if ok.sum() < 3:
        return float("nan")
    slope = np.polyfit(np.log(mid[ok]), np.log(mass[ok] / vol[ok]), 1)[0]
    return float(-slope)


def core_density_slope(series, rho_c0: float, lo: float = 1e2, hi: float = 1e5) -> float:
    """Power-law index of rho_c against r_c along the collapse: least squares in
    log-log over the samples with lo <= rho_c / rho_c(0) <= hi (the paper fits
    the same relation in its core-collapse runs, Sec. 4)."""
    import numpy as np
    rows = np.array([(r[2], r[7]) for r in series])
    sel = (rows[:, 0] >= lo * rho_c0) & (rows[:, 0] <= hi * rho_c0)
    if sel.sum() < 4:
        return float("nan")
    return float(np.polyfit(np.log(rows[sel, 1]), np.log(rows[sel, 0]), 1)[0])


def core_collapse_run(n: int, seed: int = 1, *, gamma: float = 0.11,
                      precision: int = A.CMC_MIXED, energy_corr: bool = True,
                      t_end: float = 30.0, every: int = 10, collapse: float = 1e4,
                      stop: float = 1e6, max_steps: int = 50_000,
                      target: float = 0.03) -> dict:
    """Evolve an equal-mass Plummer sphere of n stars towards core collapse.

    energy_corr: each step applies the potential-change energy correction of
    Sec. 2.1 item 6, which the paper's code applies.  target: the mean
    sin^2(beta/2) over pairs that fixes each step's Delta t.  Every `every` steps,
    the potential, the pending correction and the diagnostics are taken:
    t / t_rh, r_c / r_h (r_h the current half-mass radius), rho_c, E, N, the
    step count, the energy budget (E - E0 + the energy escapers took) / |E0|,
    and r_c (in units of the virial radius, 1 in Henon units).  The
    collapse
    time t_cc is the first sample with rho_c >= collapse * rho_c(0), where the
    density profile's power-law index between 10 r_c and r_h / 2 is also
    taken (the host copies the state once; not counted in wall_s): without
    binaries nothing halts the collapse, and rho_c climbs by orders of
    magnitude within a small fraction of t_rh.  The run stops once rho_c >=
    stop * rho_c(0), at t = t_end t_rh or after max_steps steps."""
    cl = Cluster(n)
    cmc_init_plummer(cl, n, seed, 0)
    cmc_potential(cl)
    d0 = cmc_diagnostics(cl)
    trh = half_mass_relaxation_time(n, float(d0["r50"]))
    rho0 = float(d0["rho_c"])
    g = cl.capture(Params(seed=seed, gamma=gamma, precision=precision, target=target,
                          energy_corr=1 if energy_corr else 0))
    dev = cl.sc.device
    # scalars copied after each step: dt, e_esc (f64 bits), corr_skipped
    pick = torch.tensor([1, 7, 11], dtype=torch.int64, device=dev)
    rec = torch.zeros((every, 3), dtype=torch.int64, device=dev)
    E0 = float(d0["E"])
    rows = [(0.0, float(d0["rc"] / d0["r50"]), rho0, E0, int(cl.n), 0, 0.0, float(d0["rc"]))]
    t = 0.0
    e_esc = 0.0
    skipped = 0
    steps = 0
    cc = None
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    while t < t_end * trh and steps < max_steps:
        for k in range(every):
            g.replay()
            rec[k].copy_(cl.sc.index_select(0, pick))
        steps += every
        h = rec.cpu()
        t += float(h[:, 0].clone().view(torch.float64).sum())
        e_esc += float(h[:, 1].clone().view(torch.float64).sum())
        skipped += int(h[:, 2].sum()) if energy_corr else 0
        cmc_potential(cl)
        cmc_energy_correction(cl)  # the last step's, so that E is the corrected one
        skipped += int(cl.scalars()["corr_skipped"]) if energy_corr else 0
        d = cmc_diagnostics(cl)
        E = float(d["E"])
        rows.append((t / trh, float(d["rc"] / d["r50"]), float(d["rho_c"]), E,
                     int(cl.n), steps, (E - E0 + e_esc) / abs(E0), float(d["rc"])))
        if cc is None and rows[-1][2] >= collapse * rho0:
            wall = time.perf_counter() - wall0
            h = cl.host()
            rh = float(d["r50"])
            cc = dict(t_over_t_rh=rows[-1][0], steps=steps, wall_s=wall,
                      rc_over_rh=rows[-1][1], rho_c=rows[-1][2],
                      energy_drift=rows[-1][3] / rows[0][3] - 1.0, n=rows[-1][4],
                      energy_budget=rows[-1][6], corr_skipped=skipped, e_esc=e_esc,
                      # outside the core, inside the half-mass radius
                      density_slope=density_slope(h["r"], h["m"], 10.0 * float(d["rc"]),
                                                  0.5 * rh))
        if rows[-1][2] >= stop * rho0:
            break
    torch.cuda.synchronize()
    return {"n": n, "seed": seed, "precision": "mixed" if precision == A.CMC_MIXED else "fp64",
            "energy_corr": bool(energy_corr), "t_rh": trh,
            "core_slope": core_density_slope(rows, rho0), "rho_c0": rho0, "collapse": cc, "steps": steps,
            "wall_s": time.perf_counter() - wall0, "status": int(cl.scalars()["status"]),
            "series": rows}
