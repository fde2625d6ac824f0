"""The ensemble's per-phase calls (cmc_batch_sort, _potential, _timestep,
_relax, _orbit): each against the oracle's single-cluster phase of every
cluster, bit for bit against the library's single-cluster call, and, called
in the step's order, bit for bit against cmc_batch_step."""
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


SPECS = [dict(n=3000, seed=11, gamma=0.11, model=0),
         dict(n=10_007, seed=12, gamma=0.11, model=1, w0=6.0),
         dict(n=2049, seed=13, gamma=0.01, model=0, mass_spectrum=1),
         dict(n=5000, seed=14, gamma=0.11, model=1, w0=3.0, cap=6000),
         dict(n=1, seed=15, gamma=0.11, model=0)]


def oracle_init(ora, s):
    if s["model"] == 1:
        return ora.king(s["n"], s["seed"], s["w0"], s.get("mass_spectrum", 0))
    return ora.plummer(s["n"], s["seed"], s.get("mass_spectrum", 0))


def single(cmc, s):
    cl = cmc.Cluster(int(s.get("cap", s["n"])))
    cmc.cmc_init_model(cl, s["n"], s["seed"], s["model"], s.get("mass_spectrum", 0),
                       s.get("w0", 0.0))
    return cl


def test_batch_phases_against_oracle(cmc, ora):
    """Sec. 2.1 steps 1, 2, 3(i), 5 and 6 one call at a time, every cluster
    from the oracle's state of it, against the oracle's phase."""
    ens = cmc.Ensemble(SPECS)
    states = [oracle_init(ora, s) for s in SPECS]
    for k in range(2):
        for cl, st in zip(ens.clusters, states):
            cl.load(st.r, st.vr, st.vt, st.m, st.id)
            cl.set_scalar("dt", 0.0)
        ens.potential(cmc.CMC_FP64)
        tabs = [ora.potential(st.r, st.m) for st in states]
        for cl, tab in zip(ens.clusters, tabs):
            h = cl.host()
            assert rel(h["phi"], tab[0]) < TOL
            assert rel(h["mcum"], tab[1], 1e-300) < TOL
            assert rel(h["ssuf"], tab[2], np.abs(tab[0]).max() * 1e-3) < TOL
        p = cmc.Params(step=k)
        ens.timestep(p)
        dts = []
        for cl, st, s in zip(ens.clusters, states, SPECS):
            dt, status = ora.timestep(st, s["seed"], k, s["gamma"], 0.03)
            sc = cl.scalars()
            if st.n > 1:
                assert rel(sc["dt"], dt) < TOL
            dts.append(dt)
            cl.set_scalar("dt", dt)  # the relaxation below starts from the oracle's dt
        ens.relax(p)
        relaxed = []
        for cl, st, s, dt in zip(ens.clusters, states, SPECS, dts):
            rl = ora.relax(st, s["seed"], k, s["gamma"], dt)
            h = cl.host()
            sp = np.hypot(st.vr, st.vt).max() if st.n else 1.0
            assert rel(h["vr"], rl.vr, sp * 1e-3) < TOL
            assert rel(h["vt"], rl.vt, sp * 1e-3) < TOL
            relaxed.append(rl)
        ens.orbit(p)
        moved = []
        for cl, rl, tab, s in zip(ens.clusters, relaxed, tabs, SPECS):
            rn, vr, vt, stats = ora.orbit(rl, tab, s["seed"], k)
            h = cl.host()
            fin = np.isfinite(rn)
            assert np.array_equal(np.isfinite(h["r_new"]), fin)
            assert rel(h["r_new"][fin], rn[fin]) < TOL
            sp = np.hypot(rl.vr, rl.vt).max() if rl.n else 1.0
            assert rel(h["vt"][fin], vt[fin], sp * 1e-6) < TOL
            assert np.max(np.abs(h["vr"][fin] ** 2 - vr[fin] ** 2), initial=0.0) < TOL * 4 * sp ** 2
            sc = cl.scalars()
            assert sc["n_esc"] == stats["n_esc"] and sc["trials"] == stats["trials"]
            moved.append((rn, vr, vt))
        ens.sort()
        new_states = []
        for cl, rl, (rn, vr, vt), s in zip(ens.clusters, relaxed, moved, SPECS):
            perm = ora.sort_perm(rn)
            keep = perm[np.isfinite(rn[perm])]
            h = cl.host()
            assert cl.n == keep.size
            assert np.array_equal(h["id"], rl.id[keep])
            assert rel(h["r"], rn[keep]) < TOL
            new, _ = ora.step(states[len(new_states)], s["seed"], k, s["gamma"])
            assert np.array_equal(new.id, rl.id[keep])  # the oracle's own step agrees
            new_states.append(new)
        states = new_states


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_phases_equal_single_calls(cmc, precision):
    """Bit for bit: each ensemble phase is the single-cluster call of each
    cluster (the same kernels under the ensemble's launch map)."""
    ens = cmc.Ensemble(SPECS)
    ens.init()
    singles = [single(cmc, s) for s in SPECS]
    for k in range(2):
        p = cmc.Params(step=k, precision=precision)
        ens.potential(precision)
        ens.timestep(p)
        ens.relax(p)
        ens.orbit(p)
        mid = [cl.host() for cl in ens.clusters]
        ens.sort()
        for cl, s, hm in zip(singles, SPECS, mid):
            q = cmc.Params(seed=s["seed"], gamma=s["gamma"], step=k, precision=precision)
            cmc.cmc_potential(cl, precision)
            cmc.cmc_timestep(cl, q)
            cmc.cmc_relax(cl, q)
            cmc.cmc_orbit(cl, q)
            h = cl.host()
            for key in ("phi", "mcum", "ssuf", "r_new", "vr", "vt"):
                assert np.array_equal(h[key], hm[key]), (k, key)
            cmc.cmc_sort(cl)
        for a, b in zip(ens.clusters, singles):
            ha, hb = a.host(), b.host()
            for key in ("r", "vr", "vt", "m", "id"):
                assert np.array_equal(ha[key], hb[key]), (k, key)
            sa, sb = a.scalars(), b.scalars()
            for key in ("n", "dt", "n_esc", "trials", "violations", "status"):
                assert sa[key] == sb[key], (k, key)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_phases_sequence_equals_step(cmc, precision):
    """potential -> timestep -> relax -> orbit -> sort, one ensemble call
    each, is cmc_batch_step bit for bit (3 steps)."""
    a = cmc.Ensemble(SPECS)
    b = cmc.Ensemble(SPECS)
    a.init()
    b.init()
    for k in range(3):
        p = cmc.Params(step=k, precision=precision)
        a.potential(precision)
        a.timestep(p)
        a.relax(p)
        a.orbit(p)
        a.sort()
        b.step(p)
        for ca, cb in zip(a.clusters, b.clusters):
            ha, hb = ca.host(), cb.host()
            for key in ("r", "vr", "vt", "m", "id"):
                assert np.array_equal(ha[key], hb[key]), (k, key)
            sa, sb = ca.scalars(), cb.scalars()
            for key in ("n", "dt", "n_esc", "trials", "violations", "capped", "status"):
                assert sa[key] == sb[key], (k, key)


def test_batch_phase_argument_checks(cmc):
    import ctypes as C
    from paper_1206_5878_amd import _capi as A
    L = cmc.lib()
    ens = cmc.Ensemble(SPECS[:2])
    bad = cmc.Params(precision=7).c()
    for f in ("cmc_batch_timestep", "cmc_batch_relax", "cmc_batch_orbit"):
        assert getattr(L, f)(C.byref(ens.handle), C.byref(bad), None) == A.CMC_EINVAL
        assert getattr(L, f)(None, C.byref(cmc.Params().c()), None) == A.CMC_EINVAL
    lf = cmc.Params(rng=cmc.CMC_RNG_LFSR113).c()  # no rng arrays in this ensemble
    assert L.cmc_batch_relax(C.byref(ens.handle), C.byref(lf), None) == A.CMC_EINVAL
    assert L.cmc_batch_sort(None, None) == A.CMC_EINVAL
