"""Pins of the FP64 oracle against facts fixed outside its own code.

Each test checks one oracle function against a closed form, a brute-force
definition, a textbook limit, a third-party library routine, or an exact
special case, chosen so a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them.  No GPU is needed.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import inputs

A_PLUMMER = 3.0 * np.pi / 16.0  # Plummer scale radius in Henon units


# ------------------------------------------------------------------ Philox
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    src = os.path.join(os.path.dirname(__file__), "golden", "philox_rocrand_ref.cpp")
    exe = str(tmp_path_factory.mktemp("px") / "ref")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe, src],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(ora, rocrand_ref):
    g = np.random.default_rng(7)
    keys = [0, 1, 2**32 - 1, 2**64 - 1, 0x123456789ABCDEF0] + list(
        g.integers(0, 2**63, size=20))
    lines, cases = [], []
    for k in keys:
        for _ in range(25):
            c = g.integers(0, 2**32, size=4, dtype=np.uint64)
            cases.append((int(k), c.astype(np.uint32)))
            lines.append(f"{int(k)} {c[0]} {c[1]} {c[2]} {c[3]}")
    for k in (0, 5):  # the all-zero and all-ones counters
        for c in ([0, 0, 0, 0], [2**32 - 1] * 4):
            cases.append((k, np.array(c, np.uint32)))
            lines.append(f"{k} {c[0]} {c[1]} {c[2]} {c[3]}")
    out = subprocess.run([rocrand_ref], input="\n".join(lines) + "\n", text=True,
                         capture_output=True, check=True).stdout.split("\n")
    for (k, c), line in zip(cases, out):
        want = np.array([int(x) for x in line.split()], np.uint32)
        got = ora.philox(k, c[None, :])[0]
        assert np.array_equal(got, want), (k, c, got, want)


def test_uniform_conversions(ora):
    # exact endpoints of the (2x+1) 2^-53 map
    assert ora.u01(0, 0) == 2.0**-53
    assert ora.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert ora.u01(0x80000000, 0) == 0.5 + 2.0**-53
    assert ora.u01f(0) == np.float32(2.0**-24)
    assert ora.u01f(0xFFFFFFFF) == np.float32(1.0 - 2.0**-24)
    g = np.random.default_rng(3)
    for hi, lo in g.integers(0, 2**32, size=(200, 2)):
        d, f = ora.u01(hi, lo), ora.u01f(hi)
        assert 0.0 < d < 1.0 and abs(d - float(f)) <= 2.0**-23


def test_philox_statistics(ora):
    n = 200_000
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 3
    ctr[:, 2] = 0x30
    w = ora.philox(42, ctr).astype(np.uint64)
    u = (((w[:, 1] << 32) | w[:, 0]) >> 12).astype(np.float64) * 2.0**-52
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # 16x16 equidistribution of consecutive pairs
    h, _, _ = np.histogram2d(u[:-1], u[1:], bins=16, range=[[0, 1], [0, 1]])
    assert stats.chisquare(h.ravel()).pvalue > 1e-4
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5.0 / np.sqrt(n)
    # avalanche: one counter bit flipped changes about half the output bits
    c2 = ctr.copy()
    c2[:, 3] ^= 1
    w2 = ora.philox(42, c2).astype(np.uint64)
    flips = np.unpackbits((w ^ w2).astype(np.uint32).view(np.uint8)).mean()
    assert abs(flips - 0.5) < 0.01


# ------------------------------------------------------------------ initial model
def test_plummer_radii_and_velocities(ora):
    n = 100_000
    st = ora.plummer(n, 11)
    assert np.all(np.diff(st.r) >= 0)
    assert np.array_equal(np.sort(st.id), np.arange(n, dtype=np.uint32))
    # enclosed-mass closed form M(r) = r^3 / (r^2 + a^2)^(3/2)
    cdf = lambda x: x**3 / (x * x + A_PLUMMER**2) ** 1.5
    assert stats.kstest(st.r, cdf).pvalue > 1e-3
    for f in (0.01, 0.1, 0.5, 0.9):
        want = A_PLUMMER / np.sqrt(f ** (-2.0 / 3.0) - 1.0)
        got = st.r[int(np.ceil(f * n)) - 1]
        # order-statistic error ~ sqrt(f(1-f)/n) / (dM/dr)
        dm = 3 * want**2 * A_PLUMMER**2 / (want**2 + A_PLUMMER**2) ** 2.5
        assert abs(got - want) < 5 * np.sqrt(f * (1 - f) / n) / dm
    # q = v / v_esc(r) with q^2 ~ Beta(3/2, 9/2); isotropic directions
    v = np.hypot(st.vr, st.vt)
    vesc = np.sqrt(2.0 / np.sqrt(st.r**2 + A_PLUMMER**2))
    assert stats.kstest((v / vesc) ** 2, stats.beta(1.5, 4.5).cdf).pvalue > 1e-3
    assert stats.kstest(st.vr / v, stats.uniform(-1, 2).cdf).pvalue > 1e-3
    assert np.all(st.vt >= 0)
    assert np.allclose(st.m, 1.0 / n, rtol=0, atol=0)


def test_plummer_energy_and_virial(ora):
    n = 100_000
    st = ora.plummer(n, 5)
    d = ora.diagnostics(st)
    assert abs(d["virial"] - 1.0) < 5.0 / np.sqrt(n) * 3
    assert abs(d["E"] + 0.25) < 0.25 * 10.0 / np.sqrt(n)
    assert abs(d["M"] - 1.0) < 1e-14
    # Plummer closed-form potential -1/sqrt(r^2 + a^2) at the star radii
    phi, _, _ = ora.potential(st.r, st.m)
    exact = -1.0 / np.sqrt(st.r**2 + A_PLUMMER**2)
    assert np.max(np.abs(phi - exact)) < 20.0 / np.sqrt(n)


def test_broken_power_law_masses(ora):
    n = 100_000
    st = ora.plummer(n, 9, mass_spectrum=1)
    assert abs(st.m.sum() - 1.0) < 1e-13
    s = 0.1 / st.m.min()  # total raw mass, since the lightest draw sits at 0.1
    raw = st.m * s
    assert raw.max() <= 100.0 * (1 + 1e-3)
    # analytic segment weights: C m^-1.3 on [0.1, 0.5], C/2 m^-2.3 on [0.5, 100]
    i1 = (0.1**-0.3 - 0.5**-0.3) / 0.3
    i2 = 0.5 * (0.5**-1.3 - 100**-1.3) / 1.3
    f1 = i1 / (i1 + i2)
    assert abs(f1 - 0.7292) < 5e-5
    frac = np.mean(raw < 0.5)
    assert abs(frac - f1) < 5 * np.sqrt(f1 * (1 - f1) / n)
    mean = ((0.5**0.7 - 0.1**0.7) / 0.7 + 0.5 * (0.5**-0.3 - 100**-0.3) / 0.3) / (i1 + i2)
    assert abs(mean - 0.6377) < 5e-4
    assert abs(s / n - mean) < 5 * 2.16 / np.sqrt(n)
    # shape inside segment 2: KS against its own truncated power law
    seg2 = raw[raw >= 0.5]
    cdf2 = lambda x: (0.5**-1.3 - x**-1.3) / (0.5**-1.3 - 100**-1.3)
    assert stats.kstest(seg2, cdf2).pvalue > 1e-3


# ------------------------------------------------------------------ sort
def test_sort_perm_matches_lexsort(ora):
    for seed, n in ((1, 1), (2, 2), (3, 1000), (4, 50_000)):
        x = inputs.random_keys(n, seed, ties=n // 10, n_inf=n // 50)
        x[::97] = -0.0 if n > 97 else x[::97]
        perm = ora.sort_perm(x)
        bits = (x + 0.0).view(np.uint64)
        want = np.lexsort((np.arange(n), bits))
        assert np.array_equal(perm, want)


# ------------------------------------------------------------------ potential
def _brute_phi(r, m):
    # shell theorem: Phi_k = -sum_j m_j / max(r_j, r_k)
    return -np.array([np.sum(m / np.maximum(r, rk)) for rk in r])


@pytest.mark.parametrize("ties", [0, 40])
def test_potential_brute_force(ora, ties):
    r, vr, vt, m, id_ = inputs.generic_state(800, 17 + ties, ties=ties, massless=0.1)
    phi, mcum, ssuf = ora.potential(r, m)
    bf = _brute_phi(r, m)
    assert np.max(np.abs(phi - bf) / np.abs(bf)) < 1e-14
    assert np.max(np.abs(mcum - np.cumsum(m))) < 1e-15
    assert np.max(np.abs(ssuf - (np.sum(m / r) - np.cumsum(m / r)))) < 1e-13
    # energy of the shell system: 1/2 sum_k m_k Phi_k = 1/2 double sum incl. self term
    W2 = 0.5 * np.sum(np.outer(m, m) / np.maximum.outer(r, r))
    assert abs(0.5 * np.sum(m * phi) + W2) < 1e-14 * W2


def test_potential_matches_paper_recursion(ora):
    r, vr, vt, m, id_ = inputs.generic_state(5000, 3)
    phi, mcum, _ = ora.potential(r, m)
    # Phi_{N+1} = 0, M_N = sum m, Phi_k = Phi_{k+1} - M_k (1/r_k - 1/r_{k+1}),
    # M_{k-1} = M_k - m_k   (r_{N+1} = inf)
    n = len(r)
    rec = np.empty(n)
    Mk = np.sum(m)
    nxt_phi, nxt_inv = 0.0, 0.0
    for k in range(n - 1, -1, -1):
        rec[k] = nxt_phi - Mk * (1.0 / r[k] - nxt_inv)
        nxt_phi, nxt_inv = rec[k], 1.0 / r[k]
        Mk -= m[k]
    assert np.max(np.abs(phi - rec) / np.abs(rec)) < 1e-12


def test_potential_kepler_and_interpolation(ora):
    r, vr, vt, m, id_ = inputs.kepler_probes(2000, -0.7, 0.5, 1)
    tab = ora.potential(r, m)
    phi = tab[0]
    assert np.array_equal(phi[1:], -1.0 / r[1:])
    g = np.random.default_rng(0)
    for x in g.uniform(r[0], r[-1] * 2, size=200):
        assert ora.phi_at(r, tab, x) == -1.0 / x
    # inside the innermost star the potential is flat
    assert ora.phi_at(r, tab, r[0] * 0.5) == phi[0]
    # generic table: brute-force shell sum at arbitrary radii
    r, vr, vt, m, id_ = inputs.generic_state(500, 6, ties=20)
    tab = ora.potential(r, m)
    for x in g.uniform(r[0] * 0.5, r[-1] * 1.5, size=300):
        bf = -np.sum(m / np.maximum(r, x))
        assert abs(ora.phi_at(r, tab, x) / bf - 1) < 1e-14


# ------------------------------------------------------------------ density, pairs
def test_density_uniform_sphere(ora):
    n = 2000
    r = inputs.uniform_sphere(n, 2.0)
    st = ora.State(r, np.full(n, 0.3), np.full(n, 0.2), np.full(n, 1.0 / n),
                   np.arange(n, dtype=np.uint32))
    w, tp, nb = ora.pair_terms(st, 1, 0, 0.11)
    n0 = n / (4.0 / 3.0 * np.pi * 8.0)
    assert np.max(np.abs(nb / n0 - 1.0)) < 1e-12


def test_relative_speed_law_of_cosines(ora):
    r, vr, vt, m, id_ = inputs.generic_state(3001, 8)
    st = ora.State(r, vr, vt, m, id_)
    seed, step = 99, 4
    w, tp, nb = ora.pair_terms(st, seed, step, 0.11)
    a = np.arange(0, 3000, 2)
    ctr = np.zeros((len(a), 4), np.uint32)
    ctr[:, 0] = id_[a]
    ctr[:, 1] = step
    ctr[:, 2] = 0x20
    blk = ora.philox(seed, ctr).astype(np.uint64)
    u1 = ((((blk[:, 1] << 32) | blk[:, 0]) >> 12) * 2 + 1).astype(np.float64) * 2.0**-53
    psi = 2 * np.pi * u1
    w2 = (vr[a] - vr[a + 1]) ** 2 + vt[a] ** 2 + vt[a + 1] ** 2 \
        - 2 * vt[a] * vt[a + 1] * np.cos(psi)
    assert np.max(np.abs(w**2 - w2) / w2) < 1e-12
    assert len(w) == 1500


def test_relaxation_diffusion_coefficient(ora):
    """Small-angle limit: a star of mass m1 meeting field stars of mass m2 at
    relative speed w gains <dv_perp^2> = 8 pi G^2 n m2^2 lnL dt / w (Spitzer;
    Binney & Tremaine).  The kick direction is uniform in azimuth about w, so
    the radial component carries 1/2 (1 - e1x^2) of it."""
    n = 200_000
    g = np.random.default_rng(4)
    r = inputs.uniform_sphere(n, 1.0)
    m = g.uniform(0.5, 1.5, size=n)
    m /= m.sum()
    vr = g.normal(0, 0.5, n)
    vt = np.abs(g.normal(0, 0.5, n)) * np.sqrt(2)
    id_ = np.arange(n, dtype=np.uint32)
    st = ora.State(r, vr, vt, m, id_)
    gamma = 0.11
    w, tp, nb = ora.pair_terms(st, 5, 0, gamma)
    dt = 1e-8 * np.median(tp)
    out = ora.relax(st, 5, 0, gamma, dt)
    a = np.arange(0, n, 2)
    b = a + 1
    lnL = np.log(gamma * n)
    # 3-D relative velocity direction before the kick
    ctr = np.zeros((len(a), 4), np.uint32)
    ctr[:, 0] = id_[a]
    ctr[:, 2] = 0x20
    blk = ora.philox(5, ctr).astype(np.uint64)
    u1 = ((((blk[:, 1] << 32) | blk[:, 0]) >> 12) * 2 + 1).astype(np.float64) * 2.0**-53
    wx = vr[a] - vr[b]
    e1x = wx / w
    pred = 8 * np.pi * nb * m[b] ** 2 * lnL * dt / w * 0.5 * (1 - e1x**2)
    got = (out.vr[a] - vr[a]) ** 2
    ratio = got.sum() / pred.sum()
    assert abs(ratio - 1.0) < 0.02, ratio
    del u1


def test_relax_conservation_and_special_angles(ora):
    r, vr, vt, m, id_ = inputs.generic_state(4001, 12)
    st = ora.State(r, vr, vt, m, id_)
    w, tp, nb = ora.pair_terms(st, 3, 1, 0.11)
    dt, status = ora.solve_dt(w, tp, 0.03)
    assert status == 0
    out = ora.relax(st, 3, 1, 0.11, dt)
    a = np.arange(0, 4000, 2)
    b = a + 1
    p0 = m[a] * vr[a] + m[b] * vr[b]
    p1 = m[a] * out.vr[a] + m[b] * out.vr[b]
    scale = m[a] * np.abs(vr[a]) + m[b] * np.abs(vr[b]) + (m[a] + m[b]) * w
    assert np.max(np.abs(p1 - p0) / scale) < 1e-14
    k0 = m[a] * (vr[a] ** 2 + vt[a] ** 2) + m[b] * (vr[b] ** 2 + vt[b] ** 2)
    k1 = m[a] * (out.vr[a] ** 2 + out.vt[a] ** 2) + m[b] * (out.vr[b] ** 2 + out.vt[b] ** 2)
    assert np.max(np.abs(k1 - k0) / k0) < 1e-14
    assert out.vr[-1] == vr[-1] and out.vt[-1] == vt[-1]  # odd N: last star unpaired
    assert np.any(out.vr[:-1] != vr[:-1])
    # beta = 0 (dt = 0): nothing moves
    same = ora.relax(st, 3, 1, 0.11, 0.0)
    assert np.array_equal(same.vr, vr) and np.array_equal(same.vt, vt)
    # beta = pi with equal masses: the two 3-D velocities swap, so each star
    # takes its partner's (vr, vt)
    eq = ora.State(r, vr, vt, np.full(len(r), 1.0 / len(r)), id_)
    sw = ora.relax(eq, 3, 1, 0.11, 1e30)
    assert np.max(np.abs(sw.vr[a] - vr[b])) < 1e-14
    assert np.max(np.abs(sw.vr[b] - vr[a])) < 1e-14
    assert np.max(np.abs(sw.vt[a] - vt[b])) < 1e-14
    assert np.max(np.abs(sw.vt[b] - vt[a])) < 1e-14


def test_dt_rule(ora):
    st = ora.plummer(20_000, 2)
    for target in (0.03, 0.001, 0.3):
        w, tp, nb = ora.pair_terms(st, 1, 0, 0.11)
        dt, status = ora.solve_dt(w, tp, target)
        assert status == 0 and dt > 0
        assert abs(ora.mean_sin2(w, tp, dt) / target - 1.0) < 1e-12
        # direct check of the mean with beta = min(pi, pi/2 sqrt(dt/t_p))
        beta = np.minimum(np.pi, 0.5 * np.pi * np.sqrt(dt / tp))
        assert abs(np.mean(np.sin(beta / 2) ** 2) / target - 1.0) < 1e-12
    # smaller target, smaller step
    d1, _ = ora.solve_dt(w, tp, 0.01)
    d2, _ = ora.solve_dt(w, tp, 0.02)
    assert d1 < d2
    # degenerate: no pair can be deflected
    dt, status = ora.solve_dt(np.zeros(10), np.ones(10), 0.03)
    assert dt == 0.0 and status == ora.ST_DT_DEGEN


# ------------------------------------------------------------------ orbits
@pytest.mark.parametrize("E,J", [(-0.5, 0.95), (-0.5, 0.7), (-0.3, 0.5), (-1.0, 0.1),
                                 (-0.5, 0.14)])
def test_kepler_turning_points_and_time_fraction(ora, E, J):
    r, vr, vt, m, id_ = inputs.kepler_probes(60_000, E, J, 2)
    st = ora.State(r, vr, vt, m, id_)
    tab = ora.potential(r, m)
    rn, vrn, vtn, s, d = ora.orbit(st, tab, 77, 3, details=True)
    a = -1.0 / (2.0 * E)
    e = np.sqrt(1.0 + 2.0 * E * J * J)
    p = slice(1, None)
    Ep = d["E"][p]
    ap = -1.0 / (2.0 * Ep)
    ep = np.sqrt(1.0 + 2.0 * Ep * d["J"][p] ** 2)
    assert np.max(np.abs(d["rmin"][p] / (ap * (1 - ep)) - 1)) < 1e-9
    assert np.max(np.abs(d["rmax"][p] / (ap * (1 + ep)) - 1)) < 1e-13
    # g(s) is monotone in r on a Kepler orbit, so the endpoint bound holds
    assert np.all(d["flags"][p] == 0) and s["n_esc"] == 0
    # time fraction: r = a (1 - e cos eta), t ~ eta - e sin eta
    eta = np.arccos(np.clip((1.0 - np.sort(rn[p]) / a) / e, -1, 1))
    cdf = (eta - e * np.sin(eta)) / np.pi
    ks = stats.kstest(cdf, "uniform")
    assert ks.pvalue > 1e-3, ks
    # inward and outward motion equally likely
    npos = np.sum(vrn[p] > 0)
    assert abs(npos / len(vrn[p]) - 0.5) < 5 * 0.5 / np.sqrt(len(vrn[p]))
    # conservation in the old potential
    assert np.max(np.abs(rn[p] * vtn[p] - d["J"][p])) < 1e-14 * J
    Enew = -1.0 / rn[p] + 0.5 * (vrn[p] ** 2 + vtn[p] ** 2)
    assert np.max(np.abs(Enew - d["E"][p])) < 1e-13 * (np.abs(E) + 1.0 / rn[p]).max()


def test_radial_orbit_j_zero(ora):
    E = -0.5
    r, vr, vt, m, id_ = inputs.kepler_probes(40_000, E, 0.0, 5)
    st = ora.State(r, vr, vt, m, id_)
    tab = ora.potential(r, m)
    rn, vrn, vtn, s, d = ora.orbit(st, tab, 7, 0, details=True)
    assert np.all(d["rmin"][1:] == 0.0)
    assert np.all(vtn[1:] == 0.0)
    a = 1.0
    eta = np.arccos(np.clip(1.0 - np.sort(rn[1:]) / a, -1, 1))
    cdf = (eta - np.sin(eta)) / np.pi
    # the central point mass shields r < 1e-6: negligible for the KS test
    assert stats.kstest(cdf, "uniform").pvalue > 1e-3


def test_orbit_star_at_centre_is_the_limit(ora):
    """A star exactly at r = 0 (its own m/r makes Phi_0 = -inf) gives every
    other star the orbit it gets when that star sits at a radius so small
    that J^2/r^2 overflows: Q at r -> 0 is the limit of Q(r)."""
    rng = np.random.default_rng(4)
    n = 3001
    r = np.sort(np.concatenate([[0.0], rng.lognormal(0, 1, n - 1)]))
    v = 0.5 * rng.standard_normal((n, 2))
    m = np.full(n, 1.0 / n)
    ids = np.arange(n, dtype=np.uint32)
    out = []
    for r0 in (0.0, 1e-300):
        rr = r.copy()
        rr[0] = r0
        st = ora.State(rr, v[:, 0].copy(), np.abs(v[:, 1]), m, ids)
        tab = ora.potential(st.r, st.m)
        out.append(ora.orbit(st, tab, 3, 2, details=True))
    assert np.isneginf(ora.potential(r, m)[0][0])
    (a, _, _, _, da), (b, _, _, _, db) = out
    assert np.array_equal(a[1:], b[1:])
    assert np.array_equal(da["kmin"][1:], db["kmin"][1:])
    assert np.sum(da["kmin"][1:] >= 0) > 0.5 * n


def test_orbit_brackets_on_plummer(ora):
    st = ora.plummer(20_000, 3)
    tab = ora.potential(st.r, st.m)
    phi = tab[0]
    rn, vrn, vtn, s, d = ora.orbit(st, tab, 1, 0, details=True)
    bound = np.isfinite(rn)
    assert s["n_esc"] == np.sum(~bound)
    i = np.nonzero(bound)[0]
    E, J = d["E"][i], d["J"][i]
    # turning points are roots of Q and enclose the star's present radius
    for which in ("rmin", "rmax"):
        x = d[which][i]
        ok = x > 0
        # potential at the root by the brute-force shell sum
        pr = np.array([-np.sum(st.m / np.maximum(st.r, xx)) for xx in x[ok]])
        q = 2 * E[ok] - 2 * pr - J[ok] ** 2 / x[ok] ** 2
        sc = 2 * np.abs(E[ok]) + 2 * np.abs(pr) + J[ok] ** 2 / x[ok] ** 2
        assert np.max(np.abs(q) / sc) < 1e-12
    assert np.all(d["rmin"][i] <= st.r[i] * (1 + 1e-12))
    assert np.all(d["rmax"][i] >= st.r[i] * (1 - 1e-12))
    assert np.all((rn[i] >= d["rmin"][i] * (1 - 1e-12)) & (rn[i] <= d["rmax"][i] * (1 + 1e-12)))
    # brackets are the unique sign changes of Q over the table
    for k in np.random.default_rng(0).choice(i, 300, replace=False):
        q = 2 * d["E"][k] - 2 * phi - d["J"][k] ** 2 / st.r**2
        q[k] = max(q[k], 0)
        sgn = q >= 0
        lo = np.nonzero(sgn[: k + 1])[0][0] - 1
        assert d["kmin"][k] == lo
        hi = k + np.nonzero(~sgn[k:])[0][0] - 1 if np.any(~sgn[k:]) else len(q) - 1
        assert d["kmax"][k] == hi
    # energy and angular momentum conserved in the old potential
    pn = np.array([-np.sum(st.m / np.maximum(st.r, x)) for x in rn[i[::7]]])
    En = pn + 0.5 * (vrn[i[::7]] ** 2 + vtn[i[::7]] ** 2)
    E, i = E[::7], i[::7]
    assert np.max(np.abs(En - E) / (np.abs(E) + np.abs(phi[i]))) < 1e-13
    assert np.max(np.abs(rn[i] * vtn[i] - d["J"][i]) / np.maximum(d["J"][i], 1e-300)) < 1e-14
    # sampler efficiency and the bound: few violations, modest trials
    assert s["trials"] / np.sum(bound) < 3.0
    assert s["violations"] < 1e-3 * s["trials"]


def test_star_at_rest_in_flat_core(ora):
    """Q = 0 on the whole allowed range (a star at rest inside the innermost
    shell): no trial can succeed; the sampler stops at the cap, flags it and
    leaves the star inside its range with zero radial speed."""
    r, vr, vt, m, id_ = inputs.generic_state(50, 1)
    vr[0] = 0.0
    vt[0] = 0.0
    st = ora.State(r, vr, vt, m, id_)
    tab = ora.potential(r, m)
    rn, vrn, vtn, s, d = ora.orbit(st, tab, 1, 0, trial_cap=64, details=True)
    assert d["trials"][0] == 64 and s["capped"] >= 1 and s["status"] & ora.ST_TRIAL_CAP
    assert 0.0 <= rn[0] <= r[0] and vrn[0] == 0.0 and vtn[0] == 0.0


def test_escapers_flagged(ora):
    st = ora.plummer(2000, 4)
    st.vr[100] = 5.0  # far above escape speed
    tab = ora.potential(st.r, st.m)
    phi = tab[0]
    rn, vrn, vtn, s = ora.orbit(st, tab, 1, 0)
    assert np.isinf(rn[100]) and s["n_esc"] >= 1 and s["status"] & ora.ST_ESCAPER
    E = phi[100] + 0.5 * (st.vr[100] ** 2 + st.vt[100] ** 2)
    assert s["e_esc"] >= st.m[100] * E * (1 - 1e-12)


# ------------------------------------------------------------------ whole step
def test_step_energy_drift_and_determinism(ora):
    n = 10_000
    st = ora.plummer(n, 1)
    d0 = ora.diagnostics(st)
    cur = st
    for k in range(5):
        cur, info = ora.step(cur, 1, k, 0.11)
        assert info["status"] & ~ora.ST_BOUND == 0
        assert np.all(np.diff(cur.r) >= 0)
    d1 = ora.diagnostics(cur)
    drift = (d1["E"] - d0["E"]) / abs(d0["E"])
    assert abs(drift) < 5 * 5 / n  # O(1/N) per step, uncorrected Henon step
    assert abs(d1["virial"] - 1) < 0.05
    again = st
    for k in range(5):
        again, _ = ora.step(again, 1, k, 0.11)
    assert np.array_equal(again.r, cur.r) and np.array_equal(again.id, cur.id)


# ---------------------------------------------------------------- King models
def test_king_density_is_the_lowered_isothermal_df(ora):
    """rho(W) is, up to a constant, the integral over speeds of King's
    distribution function f = e^(W - v^2/2) - 1 (v < sqrt(2W)); checked by
    quadrature, also in the small-W series branch."""
    from scipy.integrate import quad

    def by_df(W):
        return quad(lambda v: (np.expm1(W - 0.5 * v * v)) * v * v, 0.0, np.sqrt(2 * W),
                    epsabs=0, epsrel=1e-13)[0]

    ref = by_df(6.0) / ora.king_density(6.0)
    for W in (1e-4, 0.03, 0.0999, 0.1001, 0.5, 2.0, 9.0):
        assert abs(by_df(W) / ora.king_density(W) / ref - 1) < 1e-9, W
    assert ora.king_density(0.0) == 0.0 and ora.king_density(-1.0) == 0.0


@pytest.mark.parametrize("w0,c", [(3, 0.67), (5, 1.03), (6, 1.26), (7, 1.53), (9, 2.12),
                                  (12, 2.74)])
def test_king_concentration(ora, w0, c):
    """Concentration log10(r_t / r_K) against King's (1966) tabulation."""
    r, W, M, (rt, Mt, wpot) = ora.king_profile(w0)
    assert abs(np.log10(rt) - c) < 0.01
    assert np.all(np.diff(r) > 0) and np.all(np.diff(M) > 0) and np.all(np.diff(W) < 0)


def test_king_profile_against_independent_integration(ora):
    """The RK4 profile against scipy's adaptive DOP853 on the same Poisson
    equation with the density taken from the distribution-function
    quadrature: tidal radius, total mass and W at the nodes."""
    from scipy.integrate import quad, solve_ivp

    w0 = 6.0

    def rho(W):
        if W <= 0:
            return 0.0
        return quad(lambda v: np.expm1(W - 0.5 * v * v) * v * v, 0.0, np.sqrt(2 * W),
                    epsabs=0, epsrel=1e-13)[0]

    rho0 = rho(w0)

    def rhs(r, y):
        W, U = y
        return [U / (r * r), -9.0 * r * r * rho(W) / rho0]

    def edge(r, y):
        return y[0]
    edge.terminal = True
    r0 = 1e-5
    sol = solve_ivp(rhs, (r0, 100.0), [w0 - 1.5 * r0 * r0, -3.0 * r0 ** 3], method="DOP853",
                    rtol=1e-11, atol=1e-14, events=edge, dense_output=True)
    rt_ref = sol.t_events[0][0]
    mt_ref = -sol.y_events[0][0][1]
    r, W, M, (rt, Mt, wpot) = ora.king_profile(w0)
    assert abs(rt / rt_ref - 1) < 1e-5 and abs(Mt / mt_ref - 1) < 1e-6
    sel = r[1:-1][:: 97]
    assert np.max(np.abs(W[1:-1][:: 97] - sol.sol(sel)[0])) < 1e-7
    # W_pot of the trapezoid rule against the dense solution
    rr = np.linspace(r[1], rt_ref, 200_001)
    Mr = -sol.sol(rr)[1]
    wp_ref = -np.trapezoid(Mr * np.gradient(Mr, rr) / rr, rr)
    assert abs(wpot / wp_ref - 1) < 1e-4


def test_king_sample(ora):
    """A sampled King W0 = 6 model: Henon units (virial ratio 1, E = -1/4
    within the sampling noise), radii distributed as the profile's M(r)."""
    from scipy import stats
    n = 60_000
    st = ora.king(n, 5, 6.0)
    d = ora.diagnostics(st)
    assert abs(d["virial"] - 1) < 5 / np.sqrt(n)
    assert abs(d["E"] + 0.25) < 0.02
    assert abs(d["M"] - 1) < 1e-12
    r, W, M, (rt, Mt, wpot) = ora.king_profile(6.0)
    s = -4.0 * (0.5 * wpot) / Mt ** 2
    cdf = lambda x: np.interp(x / s, r, M / Mt)
    assert stats.kstest(st.r, cdf).pvalue > 1e-3
    assert st.r.max() <= rt * s * (1 + 1e-12)
    # the speeds stay below the local escape speed of the model
    Wr = np.interp(st.r / s, r, W)
    vmod = np.hypot(st.vr, st.vt) * np.sqrt(Mt * s)
    assert np.all(vmod <= np.sqrt(2 * Wr) * (1 + 1e-9) + 1e-12)


# ---------------------------------------------------------------- core diagnostics
# The density estimator of the core diagnostics takes the 5 stars strictly
# inside a window of 7 consecutive radii over the shell volume between the
# window's ends.  For a locally uniform (Poisson) population that volume is
# Gamma(6) distributed in units of 1/(number density), so E[rho_i] = rho and
# E[rho_i^2] = 25/20 rho^2: the core density sum rho_i^2 / sum rho_i is 1.25
# times the mass-weighted mean density, and the density-weighted radius
# sum rho_i r_i / sum rho_i is the mass-weighted mean of r weighted by rho.

def _core_state(ora, r, m):
    order = np.argsort(r, kind="stable")
    r = np.ascontiguousarray(r[order])
    n = r.size
    z = np.zeros(n)
    return ora.State(r, z.copy(), z.copy(), np.ascontiguousarray(m[order]),
                     np.arange(n, dtype=np.uint32))


def test_core_uniform_sphere(ora):
    rng = np.random.default_rng(21)
    n, R = 200_000, 2.0
    r = R * rng.random(n) ** (1.0 / 3.0)
    st = _core_state(ora, r, np.full(n, 1.0 / n))
    d = ora.diagnostics(st)
    rho0 = 1.0 / (4.0 * np.pi / 3.0 * R**3)
    assert d["rho_c"] / rho0 == pytest.approx(1.25, rel=0.02)
    assert d["rc"] == pytest.approx(0.75 * R, rel=0.01)


def test_core_plummer_closed_form(ora):
    from scipy.special import beta
    st = ora.plummer(200_000, 5)
    d = ora.diagnostics(st)
    a = 3.0 * np.pi / 16.0  # Henon-unit Plummer scale
    rho0 = 3.0 / (4.0 * np.pi * a**3)
    # int rho^3 dV / int rho^2 dV and int rho^2 r dV / int rho^2 dV for
    # rho = rho0 (1 + x^2)^(-5/2), x = r/a, through Beta functions
    mean_rho = rho0 * beta(1.5, 6.0) / beta(1.5, 3.5)
    mean_r = a * beta(2.0, 3.0) / beta(1.5, 3.5)
    assert d["rho_c"] == pytest.approx(1.25 * mean_rho, rel=0.02)
    assert d["rc"] == pytest.approx(mean_r, rel=0.01)


def test_core_scaling(ora):
    """Masses x c scale rho_c by c; radii x s scale rho_c by s^-3 and r_c by s."""
    st = ora.plummer(20_000, 6)
    d = ora.diagnostics(st)
    st2 = _core_state(ora, st.r * 3.0, st.m * 0.5)
    d2 = ora.diagnostics(st2)
    assert d2["rho_c"] == pytest.approx(d["rho_c"] * 0.5 / 27.0, rel=1e-12)
    assert d2["rc"] == pytest.approx(d["rc"] * 3.0, rel=1e-12)


def test_core_degenerate(ora):
    st = _core_state(ora, np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6]), np.full(6, 1 / 6))
    d = ora.diagnostics(st)
    assert np.isnan(d["rc"]) and np.isnan(d["rho_c"])  # fewer than 7 stars
    st = _core_state(ora, np.full(50, 0.7), np.full(50, 0.02))
    d = ora.diagnostics(st)
    assert np.isnan(d["rc"]) and np.isnan(d["rho_c"])  # every window has zero volume


def test_orbit_subset_is_the_orbit_pass_restricted():
    """The sampled orbit entry gives, at each listed star, exactly what the
    whole pass gives there (each orbit depends on the table and the star)."""
    import numpy as np
    import oracle as O
    st = O.plummer(4000, 8)
    tab = O.potential(st.r, st.m)
    rn, vr, vt, _ = O.orbit(st, tab, 8, 2)
    idx = np.array([0, 1, 17, 2048, 3998, 3999])
    a, b, c = O.orbit_subset(st, tab, 8, 2, idx)
    assert np.array_equal(a, rn[idx]) and np.array_equal(b, vr[idx]) and np.array_equal(c, vt[idx])


def test_resume_is_bit_identical(tmp_path):
    """The oracle's step keys every draw by (id, step) and keeps no state of its
    own, so a run saved after 2 steps and resumed equals the uninterrupted run."""
    import numpy as np
    import oracle as O
    a = O.plummer(3000, 2)
    for k in range(4):
        a, _ = O.step(a, 2, k, 0.11)
    b = O.plummer(3000, 2)
    for k in range(2):
        b, _ = O.step(b, 2, k, 0.11)
    path = str(tmp_path / "ck.npz")
    np.savez(path, r=b.r, vr=b.vr, vt=b.vt, m=b.m, id=b.id)
    with np.load(path, allow_pickle=False) as f:
        c = O.State(f["r"], f["vr"], f["vt"], f["m"], f["id"])
    for k in range(2, 4):
        c, _ = O.step(c, 2, k, 0.11)
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(getattr(a, key), getattr(c, key)), key
