"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds none of the method's arithmetic: it only draws generic
sorted star states (log-normal radii, Gaussian velocities, positive masses)
and builds special configurations (ties, massless stars, a central point mass)
from numpy's seeded generator.  Plummer models come from each side's own
initial-model code instead.
"""
from __future__ import annotations

import numpy as np


def generic_state(n: int, seed: int, *, ties: int = 0, massless: float = 0.0,
                  jzero: float = 0.0, mass_f32: bool = False):
    """Sorted generic state: radii ~ lognormal, vr ~ N(0, s), vt ~ |N(0, s)|*sqrt2
    with s chosen so most stars are bound in their own potential.  ``ties`` copies
    that many radii onto their neighbour; ``massless`` / ``jzero`` set that
    fraction of masses / transverse speeds to zero."""
    g = np.random.default_rng(seed)
    r = np.sort(np.exp(g.normal(-0.3, 0.9, size=n)))
    if ties and n > 1:
        idx = g.choice(n - 1, size=min(ties, n - 1), replace=False)
        r[idx + 1] = r[idx]
        r = np.sort(r)
    m = g.uniform(0.5, 1.5, size=n)
    if massless:
        m[g.random(n) < massless] = 0.0
    if m.sum() == 0:
        m[:] = 1.0
    m = m / m.sum()
    if mass_f32:
        m = m.astype(np.float32).astype(np.float64)
    s = 0.35
    vr = g.normal(0.0, s, size=n)
    vt = np.abs(g.normal(0.0, s, size=n)) * np.sqrt(2.0)
    if jzero:
        vt[g.random(n) < jzero] = 0.0
    id_ = g.permutation(n).astype(np.uint32)
    return r, vr, vt, m, id_


def kepler_probes(n_probe: int, E: float, J: float, seed: int, r_core: float = 1e-6):
    """A unit point mass at ``r_core`` plus ``n_probe`` massless stars inside the
    Kepler orbit (E, J) of G M = 1, sorted by radius.  Returns
    (r, vr, vt, m, id) with every probe on that orbit (up to rounding)."""
    g = np.random.default_rng(seed)
    a = -1.0 / (2.0 * E)
    e = np.sqrt(max(0.0, 1.0 + 2.0 * E * J * J))
    rmin, rmax = a * (1.0 - e), a * (1.0 + e)
    lo = rmin + 1e-3 * (rmax - rmin)
    hi = rmax - 1e-3 * (rmax - rmin)
    rp = np.sort(g.uniform(lo, hi, size=n_probe))
    vt = np.where(rp > 0, J / rp, 0.0)
    q = 2.0 * E + 2.0 / rp - (J * J) / (rp * rp)
    vr = np.sqrt(np.maximum(q, 0.0)) * np.where(g.random(n_probe) < 0.5, -1.0, 1.0)
    r = np.concatenate([[r_core], rp])
    vr = np.concatenate([[1.0], vr])  # the point mass itself moves inside ~r_core
    vt = np.concatenate([[0.0], vt])
    m = np.concatenate([[1.0], np.zeros(n_probe)])
    id_ = np.arange(n_probe + 1, dtype=np.uint32)
    return r, vr, vt, m, id_


def uniform_sphere(n: int, radius: float = 1.0):
    """Radii r_k = R (k/n)^(1/3), k = 1..n: a sphere of exactly uniform number
    density n / (4/3 pi R^3) between consecutive stars."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return radius * np.cbrt(k / n)


def random_keys(n: int, seed: int, *, ties: int = 0, n_inf: int = 0):
    """Positive radii with optional exact duplicates and +inf (escaper) keys."""
    g = np.random.default_rng(seed)
    x = np.exp(g.normal(0.0, 2.0, size=n))
    if ties and n > 1:
        src = g.integers(0, n, size=ties)
        dst = g.integers(0, n, size=ties)
        x[dst] = x[src]
    if n_inf:
        x[g.choice(n, size=min(n_inf, n), replace=False)] = np.inf
    return x
