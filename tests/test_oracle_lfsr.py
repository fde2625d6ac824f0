"""Pins of the oracle's LFSR113 generator (arXiv:1206.5878, Sec. 3.6: L'Ecuyer's
combined Tausworthe generator, streams 2^80 steps apart).

A component LFSR of degree k has the full period 2^k - 1 only if its
recurrence is the primitive one, so the four periods pin every shift and
mask.  Jumps are checked against single steps and against their own
composition law; the streams against the jump of 2^80."""
import numpy as np
import pytest

import oracle as O

Z = np.array([0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321], np.uint32)


@pytest.mark.parametrize("c,k", [(0, 31), (1, 29), (2, 28), (3, 25)])
def test_component_full_period(c, k):
    assert O.lfsr113_component_period(c, int(Z[c]), 2 ** k) == 2 ** k - 1


def test_combined_output_is_xor_of_components():
    # single steps of the combined generator advance every component once
    z1, words = O.lfsr113_blocks(Z, 1)
    z2 = O.lfsr113_jump_pow2(Z, 2)  # 4 outputs = 4 steps
    assert np.array_equal(z1, z2)
    assert words.dtype == np.uint32 and words.shape == (1, 4)
    # the last output of the block is the XOR of the component words now
    assert words[0, 3] == z1[0] ^ z1[1] ^ z1[2] ^ z1[3]


@pytest.mark.parametrize("e", [0, 1, 2, 5, 9, 12])
def test_jump_equals_single_steps(e):
    steps = 2 ** e
    z = Z.copy()
    if steps >= 4:
        z, _ = O.lfsr113_blocks(z, steps // 4)
    else:
        for _ in range(steps):
            zz = z.copy()
            O.lib().ora_lfsr113_next(zz)
            z = zz
    assert np.array_equal(z, O.lfsr113_jump_pow2(Z, e))


def test_jump_composition_and_streams():
    for e in (40, 79):
        once = O.lfsr113_jump_pow2(Z, e + 1)
        twice = O.lfsr113_jump_pow2(O.lfsr113_jump_pow2(Z, e), e)
        assert np.array_equal(once, twice)
    assert np.array_equal(O.lfsr113_stream(Z, 0), Z)
    assert np.array_equal(O.lfsr113_stream(Z, 1), O.lfsr113_jump_pow2(Z, 80))
    for a, b in [(5, 7), (2 ** 20 + 3, 2 ** 31 - 1), (1, 2 ** 32 - 2)]:
        assert np.array_equal(O.lfsr113_stream(O.lfsr113_stream(Z, a), b),
                              O.lfsr113_stream(Z, a + b))
    # distinct streams start from distinct states
    ids = [0, 1, 2, 3, 1000, 2 ** 31]
    st = O.lfsr113_seed_states(Z, ids)
    assert len({tuple(x) for x in st}) == len(ids)


def test_output_uniform():
    _, w = O.lfsr113_blocks(O.lfsr113_stream(Z, 3), 1 << 16)
    x = w.reshape(-1)
    counts = np.bincount(x >> 24, minlength=256)
    exp = x.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert 180 < chi2 < 340  # 255 degrees of freedom, about +-4.5 sigma
    bits = np.unpackbits(x.view(np.uint8)).reshape(-1, 32).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.01)


def _blocks_between(a, b, limit=64):
    """Blocks that take state a to state b (None if more than limit)."""
    z = a.copy()
    for k in range(limit + 1):
        if np.array_equal(z, b):
            return k
        z, _ = O.lfsr113_blocks(z, 1)
    return None


def test_step_draws_from_the_stars_streams():
    """In LFSR mode each kept star's state moved on by the blocks it drew:
    one per relaxation as the pair's first star, one per rejection trial,
    one for the sign.  Other stars' streams are untouched by it."""
    st = O.plummer(2000, 4)
    st.rng = O.lfsr113_seed_states(Z, st.id)
    first = {int(i) for i in st.id[0:st.n - st.n % 2:2]}
    new, info = O.step(st, 4, 0, 0.11, lfsr=True)
    old = {int(i): st.rng[k] for k, i in enumerate(st.id)}
    used = []
    for k, i in enumerate(new.id):
        nb = _blocks_between(old[int(i)], new.rng[k])
        assert nb is not None
        used.append(nb - (1 if int(i) in first else 0))
    used = np.array(used)
    assert used.min() >= 2  # at least one trial and the sign
    # trials per star as in the Philox step: mean about 1.75
    assert 1.5 < (used - 1).mean() < 2.1
    ph, _ = O.step(st, 4, 0, 0.11)
    assert not np.array_equal(ph.r, new.r)  # another generator, another draw
    assert abs(new.n - ph.n) <= 3
