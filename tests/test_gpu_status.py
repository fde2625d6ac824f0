"""Every device status bit forced from the host, with the same outcome as the
oracle's.  Each case only changes inputs or parameters: every kernel still
runs to its normal end.
- CMC_ST_TRIAL_CAP: trial_cap = 1 (a star keeps its one trial radius);
- CMC_ST_NUMERIC: an infinite bound factor (no finite rejection bound: the
  star goes to the middle of its orbit);
- CMC_ST_NONFINITE: a star with a NaN velocity (it leaves as an escaper)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def cmc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1206_5878_amd as P
    P.lib()
    return P


def rel(a, b, scale=0.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.maximum(np.abs(b), scale)
    den = np.where(den > 0, den, 1.0)
    return np.max(np.abs(a - b) / den) if a.size else 0.0


def orbit_both(cmc, ora, st, **kw):
    """cmc_orbit on the GPU and the oracle's orbit pass, same table."""
    import torch
    tab = ora.potential(st.r, st.m)
    cl = cmc.Cluster(max(st.n, 1))
    cl.load(st.r, st.vr, st.vt, st.m, st.id)
    for k, v in zip(("phi", "mcum", "ssuf"), tab):
        getattr(cl, k)[:st.n] = torch.as_tensor(v, device="cuda")
    cmc.cmc_orbit(cl, cmc.Params(seed=3, step=2, **kw))
    rn, vrn, vtn, so, d = ora.orbit(st, tab, 3, 2, trial_cap=kw.get("trial_cap", 10000),
                                    bound_factor=kw.get("bound_factor", 1.2), details=True)
    return cl.host(st.n), cl.scalars(), rn, so, d


def test_trial_cap(cmc, ora):
    st = ora.plummer(20_000, 6)
    h, s, rn, so, d = orbit_both(cmc, ora, st, trial_cap=1)
    assert s["status"] & cmc.ST_TRIAL_CAP and so["status"] & ora.ST_TRIAL_CAP
    assert s["capped"] == so["capped"] > 0.2 * st.n
    assert s["trials"] == so["trials"] == st.n - so["n_esc"] - np.sum(d["trials"] == 0)
    fin = np.isfinite(rn)
    assert rel(h["r_new"][fin], rn[fin]) < TOL


def test_numeric(cmc, ora):
    st = ora.plummer(5_000, 7)
    h, s, rn, so, d = orbit_both(cmc, ora, st, bound_factor=float("inf"))
    assert s["status"] & cmc.ST_NUMERIC and so["status"] & ora.ST_NUMERIC
    assert s["trials"] == so["trials"] == 0
    fin = np.isfinite(rn)
    # every bound star sits at the middle of its orbit
    mid = 0.5 * (d["rmin"] + d["rmax"])
    assert rel(rn[fin], mid[fin]) < TOL
    assert rel(h["r_new"][fin], rn[fin]) < TOL


def test_nonfinite(cmc, ora):
    st = ora.plummer(5_000, 8)
    st.vr[1234] = np.nan
    h, s, rn, so, d = orbit_both(cmc, ora, st)
    assert s["status"] & cmc.ST_NONFINITE and so["status"] & ora.ST_NONFINITE
    assert s["status"] & cmc.ST_ESCAPER
    assert np.isinf(h["r_new"][1234]) and np.isinf(rn[1234])
    assert s["n_esc"] == so["n_esc"]
    fin = np.isfinite(rn)
    assert rel(h["r_new"][fin], rn[fin]) < TOL
    # and a whole step drops the star and goes on
    cl = cmc.Cluster(st.n)
    cl.load(st.r, st.vr, st.vt, st.m, st.id)
    cmc.cmc_step(cl, cmc.Params(seed=3, step=0))
    s = cl.scalars()
    assert s["status"] & cmc.ST_NONFINITE
    assert st.id[1234] not in set(cl.host()["id"].tolist())
    assert np.all(np.isfinite(cl.host()["r"]))
