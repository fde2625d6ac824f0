"""The launch table: every entry gives the same results, bit for bit.

Both forms of the turning-point searches (direct, and grouped by the LDS
top's sample: "sorted"), with different resident blocks and trial chunks,
must leave the same state.  The sorted form is also compared with the FP64
oracle on the orbit cases of the parity tests, since the built-in table
gives it only to capacities of 2^22 stars and more, above the sizes most
parity cases use.  Those cases include J = 0 stars, whose lower turning
point the LDS levels already finish (the grouped form's extra group)."""
import numpy as np
import pytest

import inputs
from test_gpu_parity import TOL, _orbit_case, _radii_state, gstate, rel

pytestmark = pytest.mark.gpu

DIRECT = dict(min_cap=0, sorted=0, bracket_blocks=1024, trial_chunk=128)
TABLES = {
    "direct": [DIRECT],
    "direct_512_64": [dict(DIRECT, bracket_blocks=512, trial_chunk=64)],
    "direct_2048_256": [dict(DIRECT, bracket_blocks=2048, trial_chunk=256)],
    "sorted_128": [dict(DIRECT, sorted=1)],
    "sorted_64": [dict(DIRECT, sorted=1, trial_chunk=64)],
    # a table of two bands: small clusters direct, large ones sorted
    "bands": [DIRECT, dict(DIRECT, min_cap=50_000, sorted=1, trial_chunk=256)],
}


@pytest.fixture(scope="module")
def cmc():
    import torch
    assert torch.cuda.is_available()
    import paper_1206_5878_amd as P
    P.lib()
    return P


@pytest.fixture
def table():
    """Install a table for one test, then restore the one lib() installed."""
    from paper_1206_5878_amd import _capi as A
    from paper_1206_5878_amd import tune

    def use(name):
        tune.set_table(TABLES[name])
    yield use
    tune.set_table([])
    A._install_tuning(A.lib())


SORTED_ORBIT_CASES = [("plummer", 100_000), ("plummer", 2_500), ("generic", 20_001),
                      ("wide_range", 6000), ("centre_star", 3001), ("kepler", 30_000)]


def _one_orbit_state(ora, n, seed):
    """Seven in ten stars on one orbit (the same E and J, turning points at
    r = 0.8 and 1.5), the rest on random bound orbits from r = 0.3 to 3: the
    lower and the upper searches crowd into the two groups that hold the
    turning points, each group taking several search blocks."""
    rng = np.random.default_rng(seed)
    k = (7 * n) // 10
    r = np.sort(np.concatenate([np.exp(rng.uniform(np.log(0.8), np.log(1.5), k)),
                                np.exp(rng.uniform(np.log(0.3), np.log(3.0), n - k))]))
    m = np.full(n, 1.0 / n)
    tab = ora.potential(r, m)
    rp, ra = 0.8, 1.5
    pp, pa = ora.phi_at(r, tab, rp), ora.phi_at(r, tab, ra)
    # Q = 2 (E - Phi) - J^2 / r^2 vanishes at r_p and r_a
    J2 = 2.0 * (pa - pp) / (1.0 / rp ** 2 - 1.0 / ra ** 2)
    E = pp + 0.5 * J2 / rp ** 2
    q = 2.0 * (E - tab[0]) - J2 / r ** 2
    on = (r > rp) & (r < ra) & (q > 0.0)
    vr = 0.3 * rng.standard_normal(n)
    vt = np.abs(0.3 * rng.standard_normal(n))
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    vr[on] = sign[on] * np.sqrt(q[on])
    vt[on] = np.sqrt(J2) / r[on]
    assert on.sum() > n // 2
    return ora.State(r, vr, vt, m, np.arange(n, dtype=np.uint32) * 5 + 1)


def _sorted_orbit_check(cmc, ora, st, cap=None):
    h, s, (rn, vrn, vtn, so, d), tab = _orbit_case(cmc, ora, st, seed=3, step=2, cap=cap)
    fin = np.isfinite(rn)
    assert np.array_equal(np.isfinite(h["r_new"]), fin)
    assert rel(h["r_new"][fin], rn[fin]) < TOL
    E, J = d["E"][fin], d["J"][fin]
    qscale = 2 * np.abs(E) + 2 * np.abs(tab[0][fin]) + (J / np.maximum(rn[fin], 1e-300)) ** 2
    assert np.max(np.abs(h["vr"][fin] ** 2 - vrn[fin] ** 2) / qscale, initial=0.0) < TOL
    assert s["n_esc"] == so["n_esc"] and s["trials"] == so["trials"]
    assert s["violations"] == so["violations"] and s["capped"] == so["capped"]
    assert rel(s["e_esc"], so["e_esc"], 1e-300) < 1e-10


@pytest.mark.parametrize("case,n", SORTED_ORBIT_CASES)
def test_sorted_orbit_against_oracle(cmc, ora, table, case, n):
    """cmc_orbit with grouped searches against the oracle (a 2500-star table
    fits the LDS whole: its star pass searches there to the bottom)."""
    table("sorted_64")
    rng = np.random.default_rng(5)
    if case == "plummer":
        st = ora.plummer(n, 5)
        st.vr[n // 3] = 3.0  # an escaper
    elif case == "generic":
        st = gstate(ora, n, 8, ties=300, massless=0.05, jzero=0.05)
    elif case == "wide_range":
        st = _radii_state(ora, np.sort(10.0 ** rng.uniform(-8, 8, n)), 12)
    elif case == "centre_star":
        st = _radii_state(ora, np.sort(np.concatenate([[0.0], rng.lognormal(0, 1, n - 1)])), 12)
    else:
        st = ora.State(*inputs.kepler_probes(n, -0.2, 0.3, 3))
    _sorted_orbit_check(cmc, ora, st)


@pytest.mark.parametrize("cap", [2_000_000, 12_000_000])
@pytest.mark.parametrize("case", ["plummer", "one_orbit"])
def test_sorted_orbit_group_depths(cmc, ora, table, case, cap):
    """The capacity sets the depth of the groups' subtrees below the LDS top:
    4 levels (4096 stars) at 2e6, where a search block stages its group's
    whole subtree in LDS, and 5 at 1.2e7, where the searches read the levels
    below the LDS from the table.  100k stars, grouped searches, against the
    oracle; in the one-orbit state a group holds more searches than one block
    runs."""
    table("sorted_64")
    n = 100_000
    if case == "plummer":
        st = ora.plummer(n, 9)
        st.vr[::4999] = 3.0  # escapers
    else:
        st = _one_orbit_state(ora, n, 4)
    _sorted_orbit_check(cmc, ora, st, cap=cap)


def run_steps(cmc, name, table, n, precision, m_f32, ms, steps=2, **kw):
    table(name)
    cl = cmc.Cluster(n, m_f32=m_f32, rng=kw.get("rng") == cmc.CMC_RNG_LFSR113)
    cmc.cmc_init_plummer(cl, n, 7, ms)
    if kw.get("rng") == cmc.CMC_RNG_LFSR113:
        cmc.cmc_rng_seed_lfsr113(cl, [0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321])
    for k in range(steps):
        cmc.cmc_step(cl, cmc.Params(seed=7, step=k, gamma=0.11, precision=precision, **kw))
    if kw.get("energy_corr"):
        cmc.cmc_potential(cl, precision)
        cmc.cmc_energy_correction(cl)
    return cl.host(), cl.scalars()


@pytest.mark.parametrize("n,precision,m_f32,ms,kw", [
    (200_003, 1, True, 1, {}),
    (100_001, 0, False, 0, {"energy_corr": 1}),
    (60_000, 1, False, 0, {"rng": 1}),
    (2_500, 0, False, 0, {}),
])
def test_tables_give_identical_steps(cmc, table, n, precision, m_f32, ms, kw):
    ref_h, ref_s = run_steps(cmc, "direct", table, n, precision, m_f32, ms, **kw)
    for name in ("direct_512_64", "direct_2048_256", "sorted_128", "sorted_64", "bands"):
        h, s = run_steps(cmc, name, table, n, precision, m_f32, ms, **kw)
        for key in ("r", "vr", "vt", "m", "id"):
            assert np.array_equal(h[key], ref_h[key]), (name, key)
        if "rng" in ref_h:
            assert np.array_equal(h["rng"], ref_h["rng"]), name
        for key in ("n", "dt", "status", "dt_iters", "n_esc", "trials", "violations",
                    "capped", "e_esc", "corr_n", "corr_skipped"):
            assert s[key] == ref_s[key], (name, key)


def test_tables_give_identical_ensembles(cmc, table):
    """Ensembles under each form; the last cluster's capacity (1.2e7) puts its
    groups below the LDS, the others' groups fit it whole, so the grouped
    form runs both search kernels in one step."""
    from test_gpu_batch import SPECS
    specs = SPECS + [dict(n=80_000, seed=21, gamma=0.11, model=0),
                     dict(n=50_000, seed=22, gamma=0.11, model=1, w0=6.0, cap=12_000_000)]
    out = {}
    for name in ("direct", "sorted_128", "direct_512_64"):
        table(name)
        ens = cmc.Ensemble(specs)
        assert ens.handle.sorted_searches == (1 if name.startswith("sorted") else 0)
        ens.init()
        for k in range(2):
            ens.step(cmc.Params(step=k, precision=1))
        out[name] = [(c.host(), c.scalars()) for c in ens.clusters]
    for name in ("sorted_128", "direct_512_64"):
        for (ha, sa), (hb, sb) in zip(out["direct"], out[name]):
            for key in ("r", "vr", "vt", "m", "id"):
                assert np.array_equal(ha[key], hb[key]), (name, key)
            for key in ("n", "dt", "n_esc", "trials", "e_esc"):
                assert sa[key] == sb[key], (name, key)
