"""GPU parity of the potential-change energy correction (arXiv:1206.5878,
Sec. 2.1 item 6): a cmc_step with energy_corr = 1, then cmc_potential and
cmc_energy_correction, against the oracle's step, potential and correction
on the same state.  The step's own outputs are compared as in the step's
parity tests.  The corrected speeds are compared through v^2: the
correction adds 2 dT to v^2, and dT is a difference of potentials of order
one, so its rounding is absolute, about 1e-15.  Skip decisions and the
permutation are compared exactly."""
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


def same_corrected(cl, st, skipped):
    s = cl.scalars()
    h = cl.host()
    assert s["n"] == st.n
    assert np.array_equal(h["id"], st.id)
    assert rel(h["r"], st.r) < TOL
    assert rel(h["m"], st.m) < TOL
    vs = np.hypot(st.vr, st.vt).max() if st.n else 1.0
    for k in ("vr", "vt"):
        want = getattr(st, k)
        assert np.max(np.abs(h[k] ** 2 - want ** 2), initial=0.0) < TOL * 4 * vs ** 2, k
        big = np.abs(want) > 1e-6 * vs
        assert np.array_equal(np.sign(h[k][big]), np.sign(want[big])), k
    assert s["corr_skipped"] == skipped
    assert s["corr_n"] == 0


def oracle_corrected_step(ora, st, seed, k, gamma):
    new, info = ora.step(st, seed, k, gamma, moves=True)
    phi, _, _ = ora.potential(new.r, new.m)
    cor, skipped = ora.energy_correction(new, phi, info["moves"])
    return cor, skipped, info


@pytest.mark.parametrize("n,gamma,ms,steps,big", [(20_000, 0.11, 0, 3, False),
                                                  (4_001, 0.01, 1, 3, False),
                                                  (3_000, 0.11, 0, 2, True)])
def test_corrected_step_lockstep(cmc, ora, n, gamma, ms, steps, big):
    """Each step starts both sides from the same (oracle) state.  big: a
    capacity above CMC_BUCKET_CAP_MAX, where the step's radix sort writes the
    permutation."""
    st = ora.plummer(n, 2, ms)
    cl = cmc.Cluster(cmc.CMC_BUCKET_CAP_MAX + 1 if big else n)
    skipped_any = 0
    for k in range(steps):
        cl.load(st.r, st.vr, st.vt, st.m, st.id)
        cl.set_scalar("dt", 0.0)
        cmc.cmc_step(cl, cmc.Params(seed=2, step=k, gamma=gamma, energy_corr=1))
        assert cl.scalars()["corr_n"] == st.n  # every staged star, escapers too
        cmc.cmc_potential(cl)
        cmc.cmc_energy_correction(cl)
        cor, skipped, info = oracle_corrected_step(ora, st, 2, k, gamma)
        assert rel(cl.scalars()["dt"], info["dt"]) < TOL
        same_corrected(cl, cor, skipped)
        skipped_any += skipped
        st = cor
    del cl


@pytest.mark.parametrize("precision", [0, 1])
def test_step_applies_pending_correction(cmc, precision):
    """A corrected step applies the correction the step before left pending,
    right after its potential: the same, bit for bit, as applying it with
    cmc_potential and cmc_energy_correction between the two steps."""
    n = 30_000
    a = cmc.Cluster(n, m_f32=True)
    b = cmc.Cluster(n, m_f32=True)
    for cl in (a, b):
        cmc.cmc_init_model(cl, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)

    def p(k):
        return cmc.Params(seed=9, step=k, gamma=0.01, precision=precision, energy_corr=1)

    cmc.cmc_step(a, p(0))
    cmc.cmc_step(a, p(1))
    cmc.cmc_step(b, p(0))
    cmc.cmc_potential(b, precision)
    cmc.cmc_energy_correction(b)
    moved = b.host()
    assert b.scalars()["corr_n"] == 0
    skipped_b = b.scalars()["corr_skipped"]
    cmc.cmc_step(b, p(1))
    ha, hb = a.host(), b.host()
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(ha[key], hb[key]), key
    sa, sb = a.scalars(), b.scalars()
    for key in ("n", "dt", "trials", "corr_n"):
        assert sa[key] == sb[key], key
    assert sa["corr_n"] > 0
    # each correction call reports its own skips: a's in-step correction
    # skipped what b's standalone call did, and b's step found none pending
    assert sa["corr_skipped"] == skipped_b
    assert sb["corr_skipped"] == 0
    # and the correction did change the velocities it was given
    c = cmc.Cluster(n, m_f32=True)
    cmc.cmc_init_model(c, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)
    cmc.cmc_step(c, p(0))
    raw = c.host()
    assert np.array_equal(raw["r"], moved["r"])
    assert np.mean(raw["vr"] != moved["vr"]) > 0.9


def test_flag_leaves_the_step_itself_alone(cmc):
    """energy_corr only records and later applies the correction: the state
    a corrected step leaves equals the uncorrected step's, and a following
    step without the flag drops the pending correction unapplied."""
    n = 25_000
    a = cmc.Cluster(n)
    b = cmc.Cluster(n)
    for cl in (a, b):
        cmc.cmc_init_model(cl, n, 4, cmc.CMC_MODEL_PLUMMER, 0, 0.0)
    cmc.cmc_step(a, cmc.Params(seed=4, step=0, energy_corr=1))
    cmc.cmc_step(b, cmc.Params(seed=4, step=0))
    ha, hb = a.host(), b.host()
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(ha[key], hb[key]), key
    assert a.scalars()["corr_n"] == n and b.scalars()["corr_n"] == 0
    cmc.cmc_step(a, cmc.Params(seed=4, step=1))
    cmc.cmc_step(b, cmc.Params(seed=4, step=1))
    ha, hb = a.host(), b.host()
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(ha[key], hb[key]), key
    assert a.scalars()["corr_n"] == 0
    # a sort or a new model drops a pending correction as well
    cmc.cmc_step(a, cmc.Params(seed=4, step=2, energy_corr=1))
    assert a.scalars()["corr_n"] > 0
    nn = a.n
    a.r_new[:nn].copy_(a.r[:nn])  # the sort orders by r_new: keep the order
    cmc.cmc_sort(a)
    assert a.scalars()["corr_n"] == 0 and a.n == nn
    cmc.cmc_step(a, cmc.Params(seed=4, step=3, energy_corr=1))
    cmc.cmc_init_plummer(a, n, 4, 0)
    assert a.scalars()["corr_n"] == 0 and a.scalars()["corr_skipped"] == 0


def test_all_escape_with_correction(cmc, ora):
    """Every star leaves: the pending correction meets an empty cluster and
    does nothing; the next corrected step is a no-op too."""
    st = ora.plummer(5000, 8)
    st.vr[:] = 5.0
    cl = cmc.Cluster(st.n)
    cl.load(st.r, st.vr, st.vt, st.m, st.id)
    cmc.cmc_step(cl, cmc.Params(seed=4, step=0, energy_corr=1))
    s = cl.scalars()
    assert s["n"] == 0 and s["corr_n"] == 5000
    cmc.cmc_potential(cl)
    cmc.cmc_energy_correction(cl)
    s = cl.scalars()
    assert s["n"] == 0 and s["corr_n"] == 0 and s["corr_skipped"] == 0
    cmc.cmc_step(cl, cmc.Params(seed=4, step=1, energy_corr=1))
    s = cl.scalars()
    assert s["n"] == 0 and s["corr_n"] == 0 and s["status"] & cmc.ST_ESCAPER


SPECS = [dict(n=3000, seed=11, gamma=0.11, model=0),
         dict(n=10_007, seed=12, gamma=0.11, model=1, w0=6.0),
         dict(n=2049, seed=13, gamma=0.01, model=0, mass_spectrum=1),
         dict(n=5000, seed=14, gamma=0.11, model=1, w0=3.0, cap=6000),
         dict(n=1, seed=15, gamma=0.11, model=0)]


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_correction_equals_single_calls(cmc, precision):
    """Ensemble steps with the correction, then cmc_batch_potential and
    cmc_batch_energy_correction: bit for bit each cluster's own calls."""
    ens = cmc.Ensemble(SPECS)
    ens.init()
    singles = []
    for s in SPECS:
        cl = cmc.Cluster(int(s.get("cap", s["n"])))
        cmc.cmc_init_model(cl, s["n"], s["seed"], s["model"], s.get("mass_spectrum", 0),
                           s.get("w0", 0.0))
        singles.append(cl)
    for k in range(3):
        ens.step(cmc.Params(step=k, precision=precision, energy_corr=1))
        for cl, s in zip(singles, SPECS):
            cmc.cmc_step(cl, cmc.Params(seed=s["seed"], gamma=s["gamma"], step=k,
                                        precision=precision, energy_corr=1))
    ens.potential(precision)
    ens.energy_correction()
    for cl in singles:
        cmc.cmc_potential(cl, precision)
        cmc.cmc_energy_correction(cl)
    for a, b in zip(ens.clusters, singles):
        ha, hb = a.host(), b.host()
        for key in ("r", "vr", "vt", "m", "id"):
            assert np.array_equal(ha[key], hb[key]), key
        sa, sb = a.scalars(), b.scalars()
        for key in ("n", "dt", "corr_n", "corr_skipped"):
            assert sa[key] == sb[key], key


def test_graph_replay_with_correction(cmc):
    """A captured corrected step replayed three times, with eager work in
    between, equals three eager corrected steps bit for bit."""
    import torch
    n = 30_000
    eager = cmc.Cluster(n, m_f32=True)
    cmc.cmc_init_model(eager, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)
    for k in range(3):
        cmc.cmc_step(eager, cmc.Params(seed=9, step=k, gamma=0.01, precision=1, energy_corr=1))
    graphed = cmc.Cluster(n, m_f32=True)
    cmc.cmc_init_model(graphed, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)
    torch.cuda.synchronize()
    g = graphed.capture(cmc.Params(seed=9, gamma=0.01, precision=1, energy_corr=1))
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = cmc.cmc_diagnostics(graphed)  # eager work between replays
    ha, hb = eager.host(), graphed.host()
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(ha[key], hb[key]), key
    sa, sb = eager.scalars(), graphed.scalars()
    for key in ("n", "dt", "corr_n", "corr_skipped"):
        assert sa[key] == sb[key], key


def _energy(cmc, cl, precision):
    cmc.cmc_potential(cl, precision)
    cmc.cmc_energy_correction(cl)
    return float(cmc.cmc_diagnostics(cl)["E"])


@pytest.mark.parametrize("n,precision", [(1_000_000, 0), (1_000_000, 1)])
def test_energy_budget_at_scale(cmc, n, precision):
    """A property that holds at any size.  With the correction, T + W
    changes only by what escapers carry away and by what the few skipped
    stars could not take: over 6 steps at N = 1e6 the rest is 3.6e-7 of |E|
    in both precisions.  The same steps uncorrected drift by about 1e-5."""
    def run(corr):
        cl = cmc.Cluster(n)
        cmc.cmc_init_plummer(cl, n, 3, 0)
        E0 = _energy(cmc, cl, precision)
        E, esc, skipped = E0, 0.0, 0
        for k in range(6):
            cmc.cmc_step(cl, cmc.Params(seed=3, step=k, precision=precision, energy_corr=corr))
            esc += float(cl.scalars()["e_esc"])
            E = _energy(cmc, cl, precision)
            skipped += int(cl.scalars()["corr_skipped"])
        return E0, E, esc, skipped
    E0, E1, esc, skipped = run(1)
    _, E1u, escu, _ = run(0)
    err = abs(E1 - E0 + esc) / abs(E0)
    raw = abs(E1u - E0 + escu) / abs(E0)
    assert skipped < 1e-3 * n
    assert err < 1e-6
    assert raw > 10 * err


def test_corrected_energy_per_step_mixed_vs_oracle(cmc, ora):
    """Precision's share of the corrected step's energy: from the same sorted
    state, one mixed corrected step on the GPU and one oracle corrected step
    end at total energies within 1e-6 of |E|.  The oracle's own change is the
    escapers' and skipped stars' share only."""
    n = 20_000
    st = ora.plummer(n, 5)
    cl = cmc.Cluster(n)
    for k in range(3):
        cl.load(st.r, st.vr, st.vt, st.m, st.id)
        cl.set_scalar("dt", 0.0)
        cmc.cmc_step(cl, cmc.Params(seed=5, step=k, precision=cmc.CMC_MIXED, energy_corr=1))
        cmc.cmc_potential(cl)
        cmc.cmc_energy_correction(cl)
        eg = float(cmc.cmc_diagnostics(cl)["E"])
        cor, skipped, info = oracle_corrected_step(ora, st, 5, k, 0.11)
        eo = ora.diagnostics(cor)["E"]
        assert cl.n == cor.n
        assert abs(eg - eo) / abs(eo) < 1e-6, (k, eg, eo)
        st = cor
