"""A long run: an equal-mass Plummer sphere evolved to core collapse, the
validation run of arXiv:1206.5878 Sec. 4.  The collapse time, in initial
half-mass relaxation times, must land in the 15-18 t_rh range of the
published results the paper compares against (it reports 17.4 at N = 1e5)."""
import numpy as np
import pytest

@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1206_5878_amd as P
    P.lib()
    return P


def test_half_mass_relaxation_time():
    from paper_1206_5878_amd.evolve import half_mass_relaxation_time
    # 0.138 N / ln(0.1 N) (r_h^3 / G M)^(1/2)
    assert half_mass_relaxation_time(10**5, 1.0) == pytest.approx(0.138e5 / np.log(1e4))
    assert half_mass_relaxation_time(10**6, 4.0) == pytest.approx(8 * 0.138e6 / np.log(1e5))


def test_collapse_fits():
    """The two fits of the collapse runs recover known power laws: a sample
    with rho ~ r^-2 (mass uniform in r), and a core track rho_c ~ r_c^-2.23."""
    from paper_1206_5878_amd.evolve import core_density_slope, density_slope
    rng = np.random.default_rng(3)
    r = rng.uniform(0.0, 10.0, 400_000)            # dM/dr constant: rho ~ r^-2
    beta = density_slope(r, np.full(r.size, 1.0 / r.size), 0.5, 5.0)
    assert beta == pytest.approx(2.0, abs=0.03)
    rows = [(0.0, 0.0, 10.0 ** (0.1 * k), 0.0, 0, 0, 0.0, 10.0 ** (-0.1 * k / 2.23))
            for k in range(70)]
    assert core_density_slope(rows, 1.0) == pytest.approx(-2.23, abs=1e-9)
    assert np.isnan(core_density_slope(rows[:3], 1.0))   # too few samples in range


@pytest.mark.gpu
def test_core_collapse_n1e5(P):
    from paper_1206_5878_amd.evolve import core_collapse_run
    res = core_collapse_run(100_000, 1, precision=P.CMC_MIXED)
    cc = res["collapse"]
    assert cc is not None
    assert 15.0 <= cc["t_over_t_rh"] <= 18.0
    # the core shrinks by two orders of magnitude on the way
    rows = np.array([r[:4] for r in res["series"]])
    assert rows[0, 1] > 0.4 and cc["rc_over_rh"] < 0.02
    # rho_c rises monotonically in trend: each quarter of the run before the
    # collapse ends denser than the one before
    pre = rows[rows[:, 0] < cc["t_over_t_rh"]]
    q = np.array_split(pre[:, 2], 4)
    assert all(np.median(q[i + 1]) > np.median(q[i]) for i in range(3))
    # the self-similar profile outside the core: rho ~ r^-beta with beta about
    # 2.3 in the paper (2.23 in the literature it cites)
    assert 2.1 <= cc["density_slope"] <= 2.5
    # and the core's own track, rho_c ~ r_c^-2.3 from 1e2 to 1e5 rho_c(0) (the
    # paper fits -2.24 deeper in its N = 1e7 collapse; self-similar theory -2.23)
    assert -2.6 <= res["core_slope"] <= -2.0
    # with the potential-change energy correction, E + the energy escapers
    # took stays within 0.27 % at this N (0.03 % at 1e6); without it the same
    # run loses 6 % by the collapse
    assert abs(cc["energy_budget"]) < 0.006
    assert abs(cc["energy_drift"]) < 0.01
    raw = core_collapse_run(100_000, 1, precision=P.CMC_MIXED, energy_corr=False)
    assert abs(raw["collapse"]["energy_budget"]) > 5 * abs(cc["energy_budget"])


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["calls", "graph_lfsr", "corrected"])
def test_checkpoint_resume_bit_identical(P, tmp_path, case):
    """A run stopped after 3 steps, saved to disk, restored into a new
    cluster and continued for 3 more equals the uninterrupted 6-step run bit
    for bit (plain calls; graph replays with LFSR113 streams; steps with the
    energy correction, applied before the checkpoint)."""
    import torch
    n = 20_000
    lf = case == "graph_lfsr"
    corr = 1 if case == "corrected" else 0
    z0 = [0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321]
    p = P.Params(seed=5, gamma=0.01, precision=P.CMC_MIXED, energy_corr=corr,
                 rng=P.CMC_RNG_LFSR113 if lf else P.CMC_RNG_PHILOX)

    def fresh():
        cl = P.Cluster(n, m_f32=True, rng=lf)
        P.cmc_init_plummer(cl, n, 5, 1)
        if lf:
            P.cmc_rng_seed_lfsr113(cl, z0)
        return cl

    def advance(cl, k0, k1):
        if lf:
            g = cl.capture(p)
            for _ in range(k0, k1):
                g.replay()
            torch.cuda.synchronize()
        else:
            for k in range(k0, k1):
                p.step = k
                P.cmc_step(cl, p)

    def settle(cl):
        if corr:
            P.cmc_potential(cl, P.CMC_MIXED)
            P.cmc_energy_correction(cl)

    a = fresh()
    advance(a, 0, 3)
    settle(a)
    advance(a, 3, 6)
    b = fresh()
    advance(b, 0, 3)
    if corr:
        with pytest.raises(P.CmcError):
            b.checkpoint()
    settle(b)
    path = str(tmp_path / "ck.npz")
    b.save(path)
    c = P.Cluster(n, m_f32=True, rng=lf)
    c.restore(path)
    advance(c, 3, 6)
    ha, hc = a.host(), c.host()
    for key in ("r", "vr", "vt", "m", "id") + (("rng",) if lf else ()):
        assert np.array_equal(ha[key], hc[key]), key
    sa, sc = a.scalars(), c.scalars()
    for key in ("n", "dt", "step", "trials", "corr_n"):
        assert sa[key] == sc[key], key
