"""Mixed precision (CMC_MIXED) against the FP64 oracle.

The mixed form computes pair terms, kicks and rejection trials in FP32, so it
agrees with the FP64 oracle to ~1e-7 relative; the bar here is 1e-5 relative
on Phi, dt, velocities, E and J.  An accept/reject decision whose FP32 and
FP64 evaluations straddle the threshold flips the drawn radius; such flips are
counted and bounded (expected ~1e-7 per trial)."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

MTOL = 1e-5


@pytest.fixture(scope="module")
def cmc():
    import torch
    assert torch.cuda.is_available()
    import paper_1206_5878_amd as P
    P.lib()
    return P


def rel(a, b, scale=0.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.maximum(np.abs(b), scale)
    den = np.where(den > 0, den, 1.0)
    return np.max(np.abs(a - b) / den) if a.size else 0.0


def upload(cmc, st, m_f32=False):
    cl = cmc.Cluster(max(st.n, 1), m_f32=m_f32)
    cl.load(st.r, st.vr, st.vt, st.m, st.id)
    return cl


@pytest.mark.parametrize("n,seed,kw", [(3, 1, {}), (2049, 2, {"ties": 50}),
                                       (100_003, 3, {"massless": 0.05})])
def test_potential_mixed(cmc, ora, n, seed, kw):
    st = ora.State(*inputs.generic_state(n, seed, **kw))
    cl = upload(cmc, st)
    cmc.cmc_potential(cl, cmc.CMC_MIXED)
    h = cl.host()
    phi, mcum, ssuf = ora.potential(st.r, st.m)
    assert rel(h["phi"], phi) < MTOL
    assert rel(h["mcum"], mcum, 1e-300) < MTOL
    assert rel(h["ssuf"], ssuf, np.abs(phi).max() * 1e-3) < MTOL


def test_potential_mixed_plummer_1e6(cmc, ora):
    st = ora.plummer(1_000_000, 1, 1)
    st.m = st.m.astype(np.float32).astype(np.float64)
    cl = upload(cmc, st, m_f32=True)
    cmc.cmc_potential(cl, cmc.CMC_MIXED)
    phi, _, _ = ora.potential(st.r, st.m)
    err = rel(cl.host()["phi"], phi)
    assert err < MTOL
    assert err > 0  # FP32 terms really were used


def test_timestep_and_relax_mixed(cmc, ora):
    st = ora.plummer(100_000, 4)
    cl = upload(cmc, st)
    p = cmc.Params(seed=3, step=2, precision=cmc.CMC_MIXED)
    cmc.cmc_timestep(cl, p)
    s = cl.scalars()
    dt, _ = ora.timestep(st, 3, 2, 0.11, 0.03)
    assert rel(s["dt"], dt) < MTOL and s["status"] == 0
    cl.set_scalar("dt", dt)
    cmc.cmc_relax(cl, p)
    h = cl.host()
    ref = ora.relax(st, 3, 2, 0.11, dt)
    sp = np.hypot(st.vr, st.vt)
    pair = np.repeat(np.maximum(sp[0::2], sp[1::2]), 2)
    for k in ("vr", "vt"):
        d = np.abs(h[k] - getattr(ref, k)) / np.maximum(np.abs(getattr(ref, k)), pair)
        assert d.max() < MTOL, k
    # pair energy and radial momentum still conserved to FP32 accuracy
    a = np.arange(0, st.n, 2)
    k0 = st.m[a] * (st.vr[a] ** 2 + st.vt[a] ** 2) + st.m[a + 1] * (st.vr[a + 1] ** 2 + st.vt[a + 1] ** 2)
    k1 = st.m[a] * (h["vr"][a] ** 2 + h["vt"][a] ** 2) + st.m[a + 1] * (h["vr"][a + 1] ** 2 + h["vt"][a + 1] ** 2)
    assert np.max(np.abs(k1 - k0) / k0) < 1e-6


def test_orbit_mixed(cmc, ora):
    import torch
    n = 100_000
    st = ora.plummer(n, 5)
    tab = ora.potential(st.r, st.m)
    cl = upload(cmc, st)
    for k, v in zip(("phi", "mcum", "ssuf"), tab):
        getattr(cl, k)[:n] = torch.as_tensor(v, device="cuda")
    cmc.cmc_orbit(cl, cmc.Params(seed=5, step=1, precision=cmc.CMC_MIXED))
    h = cl.host(n)
    rn, vrn, vtn, so, d = ora.orbit(st, tab, 5, 1, details=True)
    fin = np.isfinite(rn)
    assert np.array_equal(np.isfinite(h["r_new"]), fin)
    # an FP32 trial angle moves r by ~1e-7 of the orbit's half-width r_a,
    # which near a turning point is large relative to r itself
    ra = np.nan_to_num(0.5 * (d["rmax"] - d["rmin"]))[fin]
    e = np.abs(h["r_new"][fin] - rn[fin]) / np.maximum(rn[fin], ra)
    flips = int(np.sum(e > MTOL))
    print("orbit mixed: max scaled r error", e[e <= MTOL].max(), "flips", flips)
    assert flips <= max(3, 2e-5 * n), flips
    ok = e <= MTOL
    J = d["J"][fin][ok]
    # J conserved by construction; E through Q at the new radius, in the old
    # potential
    assert rel(h["r_new"][fin][ok] * h["vt"][fin][ok], J, np.abs(J).max() * 1e-9) < MTOL
    idx = np.nonzero(fin)[0][ok][:: 20]
    e_new = np.array([ora.phi_at(st.r, tab, h["r_new"][i]) for i in idx]) + \
        0.5 * (h["vr"][idx] ** 2 + h["vt"][idx] ** 2)
    assert rel(e_new, d["E"][idx]) < MTOL
    assert abs(cl.scalars()["trials"] / so["trials"] - 1) < 1e-3


@pytest.mark.parametrize("n,gamma,ms", [(10_000, 0.11, 0), (20_000, 0.01, 1)])
def test_step_mixed_lockstep(cmc, ora, n, gamma, ms):
    st = ora.plummer(n, 2, ms)
    m_f32 = bool(ms)
    if m_f32:
        st.m = st.m.astype(np.float32).astype(np.float64)
    cl = cmc.Cluster(n, m_f32=m_f32)
    for k in range(4):
        cl.load(st.r, st.vr, st.vt, st.m, st.id)
        cl.set_scalar("dt", 0.0)
        cmc.cmc_step(cl, cmc.Params(seed=2, step=k, gamma=gamma, precision=cmc.CMC_MIXED))
        s = cl.scalars()
        h = cl.host()
        new, info = ora.step(st, 2, k, gamma)
        assert rel(s["dt"], info["dt"]) < MTOL
        assert s["n"] == new.n
        # match stars by id: positions in the sorted order may swap where two
        # new radii agree to ~1e-7
        og = np.argsort(h["id"])
        oo = np.argsort(new.id)
        assert np.array_equal(h["id"][og], new.id[oo])
        rg, ro = h["r"][og], new.r[oo]
        # scale: the larger of the new radius and the radius before the step
        # (a bound on the orbit's size; see test_orbit_mixed)
        rold = np.zeros(ro.size)
        io = np.argsort(st.id)
        pos = np.searchsorted(st.id[io], new.id[oo])
        rold = st.r[io][pos]
        e = np.abs(rg - ro) / np.maximum(ro, rold)
        flips = int(np.sum(e > MTOL))
        assert flips <= max(3, 2e-5 * n), (k, flips)
        ok = e <= MTOL
        # J = r vt is what the orbit conserves.  The FP32 kick leaves an
        # error of ~1e-7 of the pair's relative speed in vt, so J is compared
        # on the scale r max(|v|, v_rms)
        jg = h["r"][og][ok] * h["vt"][og][ok]
        jo = new.r[oo][ok] * new.vt[oo][ok]
        sp = np.hypot(new.vr, new.vt)[oo][ok]
        vrms = np.sqrt(np.mean(new.vr ** 2 + new.vt ** 2))
        dj = np.abs(jg - jo) / (new.r[oo][ok] * np.maximum(sp, vrms))
        assert dj.max() < MTOL, dj.max()
        st = new


def test_energy_per_step_mixed_vs_oracle(cmc, ora):
    """Precision's share of the energy error: from the same sorted state, one
    mixed step and one oracle step must end at total energies within 1e-6 of
    |E| (so within 1e-4 over 100 steps even if every step's error added up).
    The method's own drift (about 1e-3 per 100 steps at this N in FP64) is
    the same on both sides and cancels."""
    n = 100_000
    st = ora.plummer(n, 1)
    cl = cmc.Cluster(n)
    for k in range(3):
        cl.load(st.r, st.vr, st.vt, st.m, st.id)
        cl.set_scalar("dt", 0.0)
        cmc.cmc_step(cl, cmc.Params(seed=1, step=k, precision=cmc.CMC_MIXED))
        cmc.cmc_potential(cl)
        eg = cmc.cmc_diagnostics(cl)["E"]
        new, info = ora.step(st, 1, k, 0.11)
        eo = ora.diagnostics(new)["E"]
        assert cl.n == new.n
        assert abs(eg - eo) / abs(eo) < 1e-6, (k, eg, eo)
        st = new


def test_energy_drift_mixed_vs_fp64(cmc, ora):
    """Ten GPU steps in each precision from the same initial model.  The two
    runs decorrelate (radii that differ by 1e-7 can swap neighbours and hence
    relaxation partners), so their drifts are compared against the spread the
    oracle itself shows under a 1e-7 perturbation (3e-5 over 10 steps)."""
    n = 100_000
    drifts = {}
    for prec in (cmc.CMC_FP64, cmc.CMC_MIXED):
        cl = cmc.Cluster(n)
        cmc.cmc_init_plummer(cl, n, 1, 0)
        cmc.cmc_potential(cl)
        e0 = cmc.cmc_diagnostics(cl)["E"]
        for k in range(10):
            cmc.cmc_step(cl, cmc.Params(seed=1, step=k, precision=prec))
            assert (cl.scalars()["status"] & ~(cmc.ST_ESCAPER | cmc.ST_BOUND)) == 0
        cmc.cmc_potential(cl)
        d = cmc.cmc_diagnostics(cl)
        drifts[prec] = (d["E"] - e0) / abs(e0)
    print("energy drift over 10 steps, fp64 / mixed:", drifts)
    assert abs(drifts[cmc.CMC_FP64]) < 3e-4
    assert abs(drifts[cmc.CMC_MIXED] - drifts[cmc.CMC_FP64]) < 1e-4, drifts
