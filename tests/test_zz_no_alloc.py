"""cmc_step_noalloc (the library's static per-GPU scratch in place of the
caller's workspace) against cmc_step, through the C ABI: two calls in a row,
the second on a smaller cluster, each bit for bit equal to cmc_step on an
identical copy with its own workspace; then a capacity beyond the scratch is
refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cmc():
    import torch
    assert torch.cuda.is_available()
    import paper_1206_5878_amd as P
    P.lib()
    return P


def pair(cmc, n, seed, mass_spectrum, m_f32):
    a = cmc.Cluster(n, m_f32=m_f32)
    b = cmc.Cluster(n, m_f32=m_f32)
    for cl in (a, b):
        cmc.cmc_init_plummer(cl, n, seed, mass_spectrum)
    return a, b


def same(a, b):
    ha, hb = a.host(), b.host()
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(ha[key], hb[key]), key
    sa, sb = a.scalars(), b.scalars()
    for key in ("n", "dt", "status", "dt_iters", "n_esc", "trials", "violations", "capped",
                "e_esc", "corr_n"):
        assert sa[key] == sb[key], key


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_step_equals_cmc_step(cmc, precision):
    from paper_1206_5878_amd import _capi as A
    import torch
    # the largest capacity the scratch serves, then a smaller one
    big = 1
    while A.lib().cmc_workspace_bytes(2 * big) <= A.CMC_SCRATCH_BYTES:
        big *= 2
    sizes = [(big + big // 3 if A.lib().cmc_workspace_bytes(big + big // 3) <=
              A.CMC_SCRATCH_BYTES else big), 40_000 + 17]
    assert sizes[0] > sizes[1]
    for call, n in enumerate(sizes):
        print(f"noalloc call {call}: n={n} precision={precision}", flush=True)
        a, b = pair(cmc, n, 5 + call, call % 2, call % 2 == 1)
        for k in range(2):
            p = cmc.Params(seed=5 + call, step=k, gamma=0.11, precision=precision)
            cmc.cmc_step(a, p)
            cmc.cmc_step_noalloc(b, p)
            torch.cuda.synchronize()
            same(a, b)
        assert a.scalars()["n"] > 0.99 * n
        del a, b


def test_noalloc_refuses_capacity_beyond_scratch(cmc):
    from paper_1206_5878_amd import _capi as A
    big = 1
    while A.lib().cmc_workspace_bytes(big) <= A.CMC_SCRATCH_BYTES:
        big *= 2
    cl = cmc.Cluster(big)
    cmc.cmc_init_plummer(cl, 1000, 1, 0)
    before = cl.host()
    with pytest.raises(cmc.CmcError, match="scratch"):
        cmc.cmc_step_noalloc(cl, cmc.Params(seed=1, step=0))
    after = cl.host()
    for key in ("r", "vr", "vt", "id"):
        assert np.array_equal(before[key], after[key]), key
    with pytest.raises(cmc.CmcError):
        cmc.cmc_step_noalloc(cl, cmc.Params(seed=1, step=0, energy_corr=1))
