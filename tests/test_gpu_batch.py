"""Ensembles (cmc_batch_*) and the King initial model on the GPU.

An ensemble runs every cluster through the same launches; each cluster must
come out exactly as the oracle's single-cluster step would leave it, and
bit for bit as the library's own single-cluster calls leave it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def same_state(h, st, tol=TOL):
    assert np.array_equal(h["id"], st.id)
    assert rel(h["r"], st.r) < tol
    vs = np.hypot(st.vr, st.vt).max() if st.n else 1.0
    assert rel(h["vt"], st.vt, vs * 1e-6) < tol
    assert np.max(np.abs(h["vr"] ** 2 - st.vr ** 2), initial=0.0) < tol * 4 * vs ** 2
    assert rel(h["m"], st.m) < tol


@pytest.mark.parametrize("n,seed,w0", [(20_000, 3, 6.0), (4_097, 4, 3.0), (1, 2, 6.0)])
def test_init_king(cmc, ora, n, seed, w0):
    cl = cmc.Cluster(n)
    cmc.cmc_init_model(cl, n, seed, cmc.CMC_MODEL_KING, 0, w0)
    st = ora.king(n, seed, w0)
    assert cl.n == n
    same_state(cl.host(), st)


def test_init_king_mass_spectrum(cmc, ora):
    n = 10_000
    cl = cmc.Cluster(n)
    cmc.cmc_init_model(cl, n, 7, cmc.CMC_MODEL_KING, 1, 6.0)
    same_state(cl.host(), ora.king(n, 7, 6.0, 1))


SPECS = [dict(n=3000, seed=11, gamma=0.11, model=0),
         dict(n=10_007, seed=12, gamma=0.11, model=1, w0=6.0),
         dict(n=2049, seed=13, gamma=0.01, model=0, mass_spectrum=1),
         dict(n=5000, seed=14, gamma=0.11, model=1, w0=3.0, cap=6000),
         dict(n=1, seed=15, gamma=0.11, model=0)]


def oracle_init(ora, s):
    if s["model"] == 1:
        return ora.king(s["n"], s["seed"], s["w0"], s.get("mass_spectrum", 0))
    return ora.plummer(s["n"], s["seed"], s.get("mass_spectrum", 0))


def test_batch_init(cmc, ora):
    ens = cmc.Ensemble(SPECS)
    ens.init()
    for cl, s in zip(ens.clusters, SPECS):
        assert cl.n == s["n"]
        same_state(cl.host(), oracle_init(ora, s))


def test_batch_step_lockstep(cmc, ora):
    """Each step starts every cluster from the oracle's state; the ensemble
    step must reproduce the oracle's step of each cluster."""
    ens = cmc.Ensemble(SPECS)
    states = [oracle_init(ora, s) for s in SPECS]
    for k in range(3):
        for cl, st in zip(ens.clusters, states):
            cl.load(st.r, st.vr, st.vt, st.m, st.id)
            cl.set_scalar("dt", 0.0)
        ens.step(cmc.Params(step=k))
        new_states = []
        for cl, st, s in zip(ens.clusters, states, SPECS):
            new, info = ora.step(st, s["seed"], k, s["gamma"])
            sc = cl.scalars()
            assert sc["n"] == new.n
            if st.n > 1:
                assert rel(sc["dt"], info["dt"]) < TOL
            same_state(cl.host(), new)
            new_states.append(new)
        states = new_states


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_calls(cmc, precision):
    """Bit for bit: the ensemble step is the single-cluster step of each
    cluster (the same kernels under a different launch map)."""
    ens = cmc.Ensemble(SPECS)
    ens.init()
    singles = []
    for s in SPECS:
        cl = cmc.Cluster(int(s.get("cap", s["n"])))
        cmc.cmc_init_model(cl, s["n"], s["seed"], s["model"], s.get("mass_spectrum", 0),
                           s.get("w0", 0.0))
        singles.append(cl)
    for k in range(3):
        ens.step(cmc.Params(step=k, precision=precision))
        for cl, s in zip(singles, SPECS):
            cmc.cmc_step(cl, cmc.Params(seed=s["seed"], gamma=s["gamma"], step=k,
                                        precision=precision))
    for a, b in zip(ens.clusters, singles):
        ha, hb = a.host(), b.host()
        for key in ("r", "vr", "vt", "m", "id"):
            assert np.array_equal(ha[key], hb[key]), key
        sa, sb = a.scalars(), b.scalars()
        for key in ("n", "dt", "status", "n_esc", "trials", "violations"):
            assert sa[key] == sb[key], key


def test_batch_radix_sort_for_large_capacity(cmc):
    """One cluster above CMC_BUCKET_CAP_MAX sends the whole ensemble's step to
    the radix sort; every cluster must still come out bit for bit as its own
    single-cluster calls (which use the bucket sort where they can)."""
    specs = SPECS[:2] + [dict(n=3000, seed=16, gamma=0.11, model=0,
                              cap=cmc.CMC_BUCKET_CAP_MAX + 1)]
    ens = cmc.Ensemble(specs)
    assert ens.handle.bucket_sort == 0
    assert cmc.Ensemble(SPECS).handle.bucket_sort == 1
    ens.init()
    singles = []
    for s in specs:
        cl = cmc.Cluster(int(s.get("cap", s["n"])))
        cmc.cmc_init_model(cl, s["n"], s["seed"], s["model"], s.get("mass_spectrum", 0),
                           s.get("w0", 0.0))
        singles.append(cl)
    for k in range(2):
        ens.step(cmc.Params(step=k))
        for cl, s in zip(singles, specs):
            cmc.cmc_step(cl, cmc.Params(seed=s["seed"], gamma=s["gamma"], step=k))
    for a, b in zip(ens.clusters, singles):
        ha, hb = a.host(), b.host()
        for key in ("r", "vr", "vt", "m", "id"):
            assert np.array_equal(ha[key], hb[key]), key
        assert a.scalars()["n"] == b.scalars()["n"]


def test_batch_graph_replay(cmc):
    """One captured ensemble step replayed three times, with eager work in
    between, equals three eager steps with explicit indices 0, 1, 2."""
    import torch
    eager = cmc.Ensemble(SPECS)
    eager.init()
    for k in range(3):
        eager.step(cmc.Params(step=k))
    graphed = cmc.Ensemble(SPECS)
    graphed.init()
    torch.cuda.synchronize()
    g = graphed.capture(cmc.Params())
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = graphed.diagnostics()  # eager work between replays
    for a, b in zip(eager.clusters, graphed.clusters):
        ha, hb = a.host(), b.host()
        for key in ("r", "vr", "vt", "id"):
            assert np.array_equal(ha[key], hb[key]), key
        assert b.scalars()["step"] == 3


@pytest.mark.parametrize("precision", [0, 1])
def test_single_graph_replay(cmc, precision):
    """One captured single-cluster step replayed three times, with eager work
    in between, equals three eager steps with indices 0, 1, 2 bit for bit."""
    import torch
    n = 30_000
    eager = cmc.Cluster(n, m_f32=True)
    cmc.cmc_init_model(eager, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)
    for k in range(3):
        cmc.cmc_step(eager, cmc.Params(seed=9, step=k, gamma=0.01, precision=precision))
    graphed = cmc.Cluster(n, m_f32=True)
    cmc.cmc_init_model(graphed, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)
    torch.cuda.synchronize()
    g = graphed.capture(cmc.Params(seed=9, gamma=0.01, precision=precision))
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = cmc.cmc_diagnostics(graphed)  # eager work between replays
    ha, hb = eager.host(), graphed.host()
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(ha[key], hb[key]), key
    sa, sb = eager.scalars(), graphed.scalars()
    for key in ("n", "dt", "trials", "violations"):
        assert sa[key] == sb[key], key
    assert sb["step"] == 3


def test_batch_diagnostics(cmc, ora):
    ens = cmc.Ensemble(SPECS[:4])
    ens.init()
    ens.potential()
    got = ens.diagnostics()
    for d, s in zip(got, SPECS[:4]):
        ref = ora.diagnostics(oracle_init(ora, s))
        for key in ("T", "W", "E", "virial", "M", "rc", "rho_c"):
            assert rel(d[key], ref[key]) < 1e-11, key


def test_batch_full_workload(cmc):
    """The benchmark's ensemble at its real size: 64 clusters, N log-uniform in
    [1e4, 1e6] (about 1.4e7 stars), half Plummer and half King W0 = 6, one
    captured mixed step.  The largest, the smallest and two more clusters come
    out bit for bit as their own single-cluster calls."""
    import os
    import sys
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    wl = bench.WORKLOADS["ensemble_64_plummer_king_w6"]
    specs = bench.ensemble_specs(cmc, wl)
    ns = [s["n"] for s in specs]
    assert len(specs) == 64 and 1.0e7 < sum(ns) < 2.0e7
    ens = cmc.Ensemble(specs)
    ens.init()
    p = cmc.Params(precision=cmc.CMC_MIXED)
    for k in range(2):
        p.step = k
        ens.step(p)
    g = ens.capture(cmc.Params(precision=cmc.CMC_MIXED))
    for cl in ens.clusters:
        cl.set_scalar("step", 2)
    g.replay()
    torch.cuda.synchronize()
    pick = sorted({int(np.argmax(ns)), int(np.argmin(ns)), 1, 62})
    for c in pick:
        s = specs[c]
        one = cmc.Cluster(s["n"])
        cmc.cmc_init_model(one, s["n"], s["seed"], s["model"], 0, s["w0"])
        for k in range(3):
            cmc.cmc_step(one, cmc.Params(seed=s["seed"], gamma=s["gamma"], step=k,
                                         precision=cmc.CMC_MIXED))
        ha, hb = ens.clusters[c].host(), one.host()
        for key in ("r", "vr", "vt", "m", "id"):
            assert np.array_equal(ha[key], hb[key]), (c, key)
        assert ens.clusters[c].scalars()["step"] == 3
        del one
