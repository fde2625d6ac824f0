"""GPU parity of the LFSR113 generator variant (arXiv:1206.5878, Sec. 3.6)
against the oracle.  The raw words, the per-star stream seeding (jumps of
(base + id) * 2^80) and every state after a step are bit-exact.  Whole
steps drawing from the stars' streams match the oracle at the step's
tolerances."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12
Z0 = np.array([0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321], np.uint32)


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


def test_lfsr113_words_bitexact(cmc, ora):
    rng = np.random.default_rng(1)
    z = rng.integers(0, 2 ** 32, size=(1000, 4), dtype=np.uint64).astype(np.uint32)
    z[:, 0] |= 2
    z[:, 1] |= 8
    z[:, 2] |= 16
    z[:, 3] |= 128
    got = cmc.cmc_lfsr113(z, 7)
    for i in range(0, 1000, 37):
        _, want = ora.lfsr113_blocks(z[i], 7)
        assert np.array_equal(got[i], want), i
    assert cmc.cmc_lfsr113(z[:0], 3).shape == (0, 3, 4)


@pytest.mark.parametrize("base", [0, 123_456_789, 2 ** 33 - 1])
def test_seed_streams_bitexact(cmc, ora, base):
    n = 3000
    cl = cmc.Cluster(n, rng=True)
    cmc.cmc_init_plummer(cl, n, 3, 0)
    ids = np.arange(n, dtype=np.uint32)
    ids[-3:] = [2 ** 32 - 1, 2 ** 31, 77]  # ids far apart: high stream bits
    h = cl.host()
    cl.load(h["r"], h["vr"], h["vt"], h["m"], ids)
    cmc.cmc_rng_seed_lfsr113(cl, Z0, base)
    got = cl.host()["rng"]
    for j in list(range(0, n, 97)) + [n - 3, n - 2, n - 1]:
        want = ora.lfsr113_stream(Z0, base + int(ids[j]))
        assert np.array_equal(got[j], want), j


def test_seed_rejects_bad_input(cmc):
    cl = cmc.Cluster(100, rng=True)
    cmc.cmc_init_plummer(cl, 100, 3, 0)
    for bad in ([1, 8, 16, 128], [2, 7, 16, 128], [2, 8, 15, 128], [2, 8, 16, 127]):
        with pytest.raises(cmc.CmcError):
            cmc.cmc_rng_seed_lfsr113(cl, bad, 0)
    with pytest.raises(cmc.CmcError):
        cmc.cmc_rng_seed_lfsr113(cl, Z0, 2 ** 33)
    plain = cmc.Cluster(100)
    cmc.cmc_init_plummer(plain, 100, 3, 0)
    with pytest.raises(cmc.CmcError):
        cmc.cmc_rng_seed_lfsr113(plain, Z0, 0)
    with pytest.raises(cmc.CmcError):
        cmc.cmc_step(plain, cmc.Params(rng=cmc.CMC_RNG_LFSR113))


def _same_step(cl, new, info):
    s = cl.scalars()
    h = cl.host()
    assert rel(s["dt"], info["dt"]) < TOL
    assert s["n"] == new.n
    assert np.array_equal(h["id"], new.id)
    assert rel(h["r"], new.r) < TOL
    vs = np.hypot(new.vr, new.vt).max()
    assert rel(h["vt"], new.vt, vs * 1e-6) < TOL
    assert np.max(np.abs(h["vr"] ** 2 - new.vr ** 2)) < TOL * 4 * vs ** 2
    assert rel(h["m"], new.m) < TOL
    assert np.array_equal(h["rng"], new.rng)


@pytest.mark.parametrize("n,gamma,ms,steps", [(10_000, 0.11, 0, 3), (4_001, 0.01, 1, 2)])
def test_lfsr_step_lockstep(cmc, ora, n, gamma, ms, steps):
    """Each step starts both sides from the same (oracle) state, streams
    included; every draw comes from the drawing star's stream."""
    st = ora.plummer(n, 1, ms)
    st.rng = ora.lfsr113_seed_states(Z0, st.id)
    cl = cmc.Cluster(n, rng=True)
    for k in range(steps):
        cl.load(st.r, st.vr, st.vt, st.m, st.id, st.rng)
        cl.set_scalar("dt", 0.0)
        cmc.cmc_step(cl, cmc.Params(seed=1, step=k, gamma=gamma, rng=cmc.CMC_RNG_LFSR113))
        new, info = ora.step(st, 1, k, gamma, lfsr=True)
        _same_step(cl, new, info)
        st = new


def test_lfsr_step_large_capacity(cmc, ora):
    """Above CMC_BUCKET_CAP_MAX the step's radix sort carries the streams."""
    st = ora.plummer(3000, 5)
    st.rng = ora.lfsr113_seed_states(Z0, st.id)
    cl = cmc.Cluster(cmc.CMC_BUCKET_CAP_MAX + 1, rng=True)
    cl.load(st.r, st.vr, st.vt, st.m, st.id, st.rng)
    cmc.cmc_step(cl, cmc.Params(seed=5, step=0, gamma=0.11, rng=cmc.CMC_RNG_LFSR113))
    new, info = ora.step(st, 5, 0, 0.11, lfsr=True)
    _same_step(cl, new, info)
    del cl


def test_philox_step_carries_streams(cmc, ora):
    """A Philox step leaves every stream untouched but moves it with its
    star, and so does cmc_sort."""
    n = 20_000
    cl = cmc.Cluster(n, rng=True)
    cmc.cmc_init_plummer(cl, n, 2, 0)
    cmc.cmc_rng_seed_lfsr113(cl, Z0, 0)
    seeded = {int(i): z for i, z in zip(cl.host()["id"], cl.host()["rng"])}
    cmc.cmc_step(cl, cmc.Params(seed=2, step=0))
    h = cl.host()
    assert all(np.array_equal(z, seeded[int(i)]) for i, z in zip(h["id"], h["rng"]))
    k = cl.n
    cl.r_new[:k].copy_(cl.r[:k].flip(0))  # cmc_sort orders by r_new: reverse the order
    cmc.cmc_sort(cl)
    h2 = cl.host()
    assert np.array_equal(h2["id"], h["id"][::-1])
    assert np.array_equal(h2["rng"], h["rng"][::-1])


def test_lfsr_relax_and_timestep_streams(cmc, ora):
    """cmc_timestep only reads the streams; cmc_relax advances each pair's
    first star by one block and leaves the second alone."""
    n = 5001
    cl = cmc.Cluster(n, rng=True)
    cmc.cmc_init_plummer(cl, n, 6, 0)
    cmc.cmc_rng_seed_lfsr113(cl, Z0, 0)
    before = cl.host()["rng"]
    p = cmc.Params(seed=6, step=0, rng=cmc.CMC_RNG_LFSR113)
    cmc.cmc_potential(cl)
    cmc.cmc_timestep(cl, p)
    assert np.array_equal(cl.host()["rng"], before)
    cmc.cmc_relax(cl, p)
    after = cl.host()["rng"]
    for j in range(0, n, 53):
        want = ora.lfsr113_blocks(before[j], 1)[0] if (j % 2 == 0 and j < n - 1) else before[j]
        assert np.array_equal(after[j], want), j


SPECS = [dict(n=3000, seed=11, gamma=0.11, model=0),
         dict(n=10_007, seed=12, gamma=0.11, model=1, w0=6.0),
         dict(n=2049, seed=13, gamma=0.01, model=0, mass_spectrum=1),
         dict(n=1, seed=15, gamma=0.11, model=0)]


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_lfsr_equals_single_calls(cmc, precision):
    ens = cmc.Ensemble(SPECS, rng=True)
    assert ens.handle.lfsr_ready == 1
    assert cmc.Ensemble(SPECS).handle.lfsr_ready == 0
    ens.init()
    ens.seed_lfsr113(Z0)
    singles, base = [], 0
    for s in SPECS:
        cl = cmc.Cluster(int(s.get("cap", s["n"])), rng=True)
        cmc.cmc_init_model(cl, s["n"], s["seed"], s["model"], s.get("mass_spectrum", 0),
                           s.get("w0", 0.0))
        cmc.cmc_rng_seed_lfsr113(cl, Z0, base)
        base += cl.cap
        singles.append(cl)
    for k in range(2):
        ens.step(cmc.Params(step=k, precision=precision, rng=cmc.CMC_RNG_LFSR113))
        for cl, s in zip(singles, SPECS):
            cmc.cmc_step(cl, cmc.Params(seed=s["seed"], gamma=s["gamma"], step=k,
                                        precision=precision, rng=cmc.CMC_RNG_LFSR113))
    for a, b in zip(ens.clusters, singles):
        ha, hb = a.host(), b.host()
        for key in ("r", "vr", "vt", "m", "id", "rng"):
            assert np.array_equal(ha[key], hb[key]), key


def test_lfsr_graph_replay(cmc):
    """A captured LFSR113 step replayed three times equals three eager steps."""
    import torch
    n = 30_000

    def make():
        cl = cmc.Cluster(n, m_f32=True, rng=True)
        cmc.cmc_init_model(cl, n, 9, cmc.CMC_MODEL_PLUMMER, 1, 0.0)
        cmc.cmc_rng_seed_lfsr113(cl, Z0, 0)
        return cl

    p = cmc.Params(seed=9, gamma=0.01, precision=1, rng=cmc.CMC_RNG_LFSR113)
    eager = make()
    for k in range(3):
        p.step = k
        cmc.cmc_step(eager, p)
    graphed = make()
    torch.cuda.synchronize()
    g = graphed.capture(cmc.Params(seed=9, gamma=0.01, precision=1, rng=cmc.CMC_RNG_LFSR113))
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = cmc.cmc_diagnostics(graphed)
    ha, hb = eager.host(), graphed.host()
    for key in ("r", "vr", "vt", "m", "id", "rng"):
        assert np.array_equal(ha[key], hb[key]), key


def test_lfsr_step_full_size_sampled(cmc, ora):
    """At the benchmark's size (N = 1e7, f32 masses from the mass spectrum,
    mixed precision), sampled stars' streams after a step are their seeded
    streams advanced by the blocks they drew: one per relaxation as a pair's
    first star, one per trial, one for the sign."""
    n = 10_000_000
    cl = cmc.Cluster(n, m_f32=True, rng=True)
    cmc.cmc_init_plummer(cl, n, 1, 1)
    cmc.cmc_rng_seed_lfsr113(cl, Z0, 0)
    ids0 = cl.id[:n].cpu().numpy().view(np.uint32)
    first = np.zeros(n, bool)
    first[0:n - n % 2:2] = True
    was_first = dict(zip(ids0[::9973].tolist(), first[::9973].tolist()))
    cmc.cmc_step(cl, cmc.Params(seed=1, step=0, gamma=0.01, precision=1,
                                rng=cmc.CMC_RNG_LFSR113))
    s = cl.scalars()
    k = s["n"]
    ids = cl.id[:k].cpu().numpy().view(np.uint32)
    rng = cl.rng[:4 * k].cpu().numpy().view(np.uint32).reshape(k, 4)
    pos = {int(i): j for j, i in enumerate(ids)}
    drawn = []
    for i, f in list(was_first.items())[:600]:
        if i not in pos:
            continue  # escaped
        z = ora.lfsr113_stream(Z0, i)
        got = rng[pos[i]]
        for nb in range(0, 200):
            if np.array_equal(z, got):
                break
            z, _ = ora.lfsr113_blocks(z, 1)
        else:
            raise AssertionError(f"star {i}: state not on its stream")
        drawn.append(nb - (1 if f else 0))
    drawn = np.array(drawn)
    assert len(drawn) > 500 and drawn.min() >= 1
    # trials per star: about 1.75, as the step reports
    assert abs((drawn - 1).mean() - s["trials"] / n) < 0.15
    del cl


def test_lfsr_with_energy_correction_lockstep(cmc, ora):
    """Both options in one step: the sort carries the permutation and the
    streams together; the corrected state and every stream match the oracle."""
    n = 8_000
    st = ora.plummer(n, 4)
    st.rng = ora.lfsr113_seed_states(Z0, st.id)
    cl = cmc.Cluster(n, rng=True)
    for k in range(2):
        cl.load(st.r, st.vr, st.vt, st.m, st.id, st.rng)
        cl.set_scalar("dt", 0.0)
        cmc.cmc_step(cl, cmc.Params(seed=4, step=k, gamma=0.11, rng=cmc.CMC_RNG_LFSR113,
                                    energy_corr=1))
        cmc.cmc_potential(cl)
        cmc.cmc_energy_correction(cl)
        new, info = ora.step(st, 4, k, 0.11, moves=True, lfsr=True)
        phi, _, _ = ora.potential(new.r, new.m)
        cor, skipped = ora.energy_correction(new, phi, info["moves"])
        s = cl.scalars()
        h = cl.host()
        assert rel(s["dt"], info["dt"]) < TOL
        assert s["n"] == cor.n and s["corr_skipped"] == skipped
        assert np.array_equal(h["id"], cor.id)
        assert np.array_equal(h["rng"], cor.rng)
        assert rel(h["r"], cor.r) < TOL
        vs = np.hypot(cor.vr, cor.vt).max()
        for key in ("vr", "vt"):
            assert np.max(np.abs(h[key] ** 2 - getattr(cor, key) ** 2)) < TOL * 4 * vs ** 2
        st = cor
