"""Parity at the benchmark's full size: N = 1e7 Plummer stars with the broken
power-law masses stored as f32, ln(0.01 N), as bench.py times it.

The initial model and the potential are compared for every star.  For the
step, the oracle does the O(N) phases (potential, Delta t, relaxation) for all
stars, then the new orbit of a sample of 50000 stars only.  A star's orbit
depends on the table and its own state alone; the whole oracle pass at this N
takes minutes on one core.  The GPU's sorted output is found by star id.  The
escapers are the stars with E >= 0 after the relaxation.  The output must be
sorted with every id once.  This is done for one eager step, then for one
replay of a captured step with the graph's 5 Newton iterations, each from the
GPU's state.  FP64 is compared at 1e-12; the mixed form uses the bounds of the
mixed tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 10_000_000
SEED, GAMMA = 1, 0.01
TOL = 1e-12
MTOL = 1e-5


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


SAMPLE = 50_000


def state_of(ora, h):
    return ora.State(h["r"], h["vr"], h["vt"], h["m"], h["id"])


def oracle_sampled_step(ora, st, k, idx):
    """dt, the escaper count, and (r_new, vr, vt) of the stars at idx."""
    tab = ora.potential(st.r, st.m)
    dt, status = ora.timestep(st, SEED, k, GAMMA, 0.03)
    rl = ora.relax(st, SEED, k, GAMMA, dt)
    E = tab[0] + 0.5 * (rl.vr ** 2 + rl.vt ** 2)
    n_esc = int(np.count_nonzero(~(E < 0.0)))
    rn, vr, vt = ora.orbit_subset(rl, tab, SEED, k, idx)
    return dt, n_esc, rn, vr, vt


def check_step(h, s, before, k, idx, ora, tol, mixed):
    dt, n_esc, rn, vr, vt = oracle_sampled_step(ora, before, k, idx)
    assert rel(s["dt"], dt) < tol
    # escape is E >= 0 after the kicks; FP32 kicks may move a star across E = 0
    assert abs(s["n"] - (before.n - n_esc)) <= (3 if mixed else 0)
    # the output: sorted, every kept id once
    assert np.all(np.diff(h["r"]) >= 0)
    order = np.argsort(h["id"])
    ids = h["id"][order]
    assert np.all(np.diff(ids.astype(np.int64)) > 0)
    want_ids = before.id[idx]
    at = np.searchsorted(ids, want_ids)
    at = np.minimum(at, ids.size - 1)
    found = ids[at] == want_ids
    kept = np.isfinite(rn)
    assert np.sum(found != kept) <= (3 if mixed else 0)  # the escapers are gone
    found &= kept
    pos = order[at[found]]
    rg, vrg, vtg = h["r"][pos], h["vr"][pos], h["vt"][pos]
    ro, vro, vto = rn[found], vr[found], vt[found]
    if not mixed:
        assert rel(rg, ro) < tol
        vs = np.hypot(vro, vto).max()
        assert rel(vtg, vto, vs * 1e-6) < tol
        assert np.max(np.abs(vrg ** 2 - vro ** 2)) < tol * 4 * vs ** 2
        return
    e = np.abs(rg - ro) / np.maximum(ro, before.r[idx][found])
    flips = int(np.sum(e > tol))
    assert flips <= max(3, 2e-5 * idx.size), flips
    ok = e <= tol
    sp = np.hypot(vro, vto)[ok]
    vrms = np.sqrt(np.mean(vro ** 2 + vto ** 2))
    dj = np.abs(rg[ok] * vtg[ok] - ro[ok] * vto[ok]) / (ro[ok] * np.maximum(sp, vrms))
    assert dj.max() < tol


def sample(n):
    rng = np.random.default_rng(7)
    idx = np.unique(rng.integers(0, n, SAMPLE))
    return np.unique(np.concatenate([idx, [0, 1, n - 2, n - 1]]))  # both ends too


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size(cmc, ora, precision):
    mixed = precision == cmc.CMC_MIXED
    tol = MTOL if mixed else TOL
    cl = cmc.Cluster(N, m_f32=True)
    cmc.cmc_init_plummer(cl, N, SEED, 1)
    h = cl.host()
    if not mixed:
        # the initial model: every star by id against the oracle's generator
        r, vr, vt, m, id_ = ora.plummer_unsorted(N, SEED, 1)
        assert np.array_equal(np.sort(h["id"]), id_)
        assert rel(h["r"], r[h["id"]]) < TOL
        assert rel(h["vr"], vr[h["id"]], 1e-300) < TOL
        assert rel(h["vt"], vt[h["id"]], 1e-300) < TOL
        assert rel(h["m"], m[h["id"]].astype(np.float32)) < 1e-7
        assert np.all(np.diff(h["r"]) >= 0)
        del r, vr, vt, m, id_
        # the potential of the sorted state, every star
        cmc.cmc_potential(cl)
        hp = cl.host()
        phi, mcum, _ = ora.potential(hp["r"], hp["m"])
        assert rel(hp["phi"], phi) < TOL
        assert rel(hp["mcum"], mcum, 1e-300) < TOL
    # an eager step
    before = state_of(ora, h)
    idx = sample(before.n)
    cmc.cmc_step(cl, cmc.Params(seed=SEED, step=0, gamma=GAMMA, precision=precision))
    h1 = cl.host()
    check_step(h1, cl.scalars(), before, 0, idx, ora, tol, mixed)
    # one replay of the captured step, as the benchmark times it
    cl.set_scalar("step", 1)
    g = cl.capture(cmc.Params(seed=SEED, gamma=GAMMA, precision=precision, dt_iters=5))
    g.replay()
    s = cl.scalars()
    assert not (s["status"] & cmc.ST_DT_NOCONV)
    before = state_of(ora, h1)
    check_step(cl.host(), s, before, 1, sample(before.n), ora, tol, mixed)
    del g, cl
