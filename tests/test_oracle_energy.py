"""Pins of the oracle's energy correction (arXiv:1206.5878, Sec. 2.1 item 6).

The correction's reading: each star's kinetic energy changes by
dT = (dPhi(r_old) - dPhi(r_new)) / 2, dPhi = Phi_new - Phi_old.  The pin
comes from the mathematics, not from the formula.  The potential of the
shells is Phi(x) = -sum_j m_j / max(x, r_j).  So sum_i m_i Phi_new(r_old_i)
and sum_i m_i Phi_old(r_new_i) are the same double sum with i and j swapped.
With that symmetry, the corrected step conserves T + W exactly when no star
escapes and none is skipped.  An escaper e takes m_e (E_e + dPhi(r_e) / 2)
with it.  A dropped half, a swapped sign, or a star paired with another star's
move breaks these identities.
"""
import numpy as np
import pytest

import oracle as O


def _energy(st):
    phi, mcum, _ = O.potential(st.r, st.m)
    return O.diagnostics(st, phi, mcum)["E"], phi


def _corrected_step(st, seed, k, gamma=0.11):
    new, info = O.step(st, seed, k, gamma, moves=True)
    phi, _, _ = O.potential(new.r, new.m)
    cor, skipped = O.energy_correction(new, phi, info["moves"])
    return new, cor, info, skipped


def test_corrected_steps_conserve_energy():
    """Steps with no escaper and no skipped star keep T + W to rounding; the
    same steps uncorrected drift by orders of magnitude more."""
    st = O.plummer(2000, 7)
    E_prev, _ = _energy(st)
    checked = 0
    for k in range(6):
        new, cor, info, skipped = _corrected_step(st, 7, k)
        E_cor, _ = _energy(cor)
        E_raw, _ = _energy(new)
        if skipped == 0 and info["orbit"]["n_esc"] == 0:
            assert abs(E_cor - E_prev) < 1e-13 * abs(E_prev)
            assert abs(E_raw - E_prev) > 1e-6 * abs(E_prev)
            checked += 1
        st, E_prev = cor, E_cor
    assert checked >= 3


def test_escaper_budget():
    """An escaper e takes m_e (E_e + dPhi(r_e) / 2) with it.  Phi_new(r_e) is
    the direct sum over the kept stars, Phi_old(r_e) the table at e."""
    st = O.plummer(1500, 12)
    fast = [200, 900]                       # pushed onto unbound orbits
    for q in fast:
        st.vr[q] = 4.0
    E0, phi_old = _energy(st)
    new, cor, info, skipped = _corrected_step(st, 12, 0)
    assert skipped == 0
    assert info["orbit"]["n_esc"] >= len(fast)
    gone = np.setdiff1d(st.id, new.id)
    pos = np.array([np.where(st.id == g)[0][0] for g in gone])
    r_e = st.r[pos]
    phi_new_e = np.array([-(new.m / np.maximum(x, new.r)).sum() for x in r_e])
    dphi_e = phi_new_e - phi_old[pos]
    E1, _ = _energy(cor)
    budget = -info["orbit"]["e_esc"] - 0.5 * float((st.m[pos] * dphi_e).sum())
    assert abs((E1 - E0) - budget) < 1e-13 * abs(E0)
    # without the escapers' half of dPhi the books do not balance
    assert abs((E1 - E0) + info["orbit"]["e_esc"]) > 1e3 * abs((E1 - E0) - budget)


def test_ratio_kept_and_skip_rule():
    """vr/vt is unchanged; a star asked for more kinetic energy than it has
    keeps its velocities and is counted, and no other star notices."""
    st = O.plummer(1200, 5)
    new, info = O.step(st, 5, 0, 0.11, moves=True)
    phi, _, _ = O.potential(new.r, new.m)
    mv = info["moves"].copy()
    base, sk0 = O.energy_correction(new, phi, mv)
    moved = (base.vr != new.vr) | (base.vt != new.vt)
    assert moved.sum() > 0.9 * new.n
    both = moved & (new.vt != 0) & (new.vr != 0)
    np.testing.assert_allclose(base.vr[both] / base.vt[both], new.vr[both] / new.vt[both],
                               rtol=1e-14)
    q = int(np.argmin(np.where(moved, new.vr ** 2 + new.vt ** 2, np.inf)))
    mv[q, 1] += 10.0                         # Phi_old(r_old) far above: dT = -5
    cor, sk1 = O.energy_correction(new, phi, mv)
    assert sk1 == sk0 + 1
    assert cor.vr[q] == new.vr[q] and cor.vt[q] == new.vt[q]
    others = np.arange(new.n) != q
    assert np.array_equal(cor.vr[others], base.vr[others])
    assert np.array_equal(cor.vt[others], base.vt[others])


def test_static_potential_changes_nothing():
    """No star moved and the potential did not change: dT = 0 for every star."""
    st = O.plummer(800, 3)
    phi, mcum, ssuf = O.potential(st.r, st.m)
    mv = np.stack([st.r, phi, phi], axis=1)
    cor, skipped = O.energy_correction(st, phi, mv)
    assert skipped == 0
    np.testing.assert_allclose(cor.vr, st.vr, rtol=1e-13, atol=0)
    np.testing.assert_allclose(cor.vt, st.vt, rtol=1e-13, atol=0)


def test_moves_are_the_old_table():
    """moves: r_old is the star's radius before the step, Phi_old(r_old) the
    old table there, Phi_old(r_new) the old potential's defining sum at r_new."""
    st = O.plummer(600, 9)
    phi, _, _ = O.potential(st.r, st.m)
    new, info = O.step(st, 9, 0, 0.11, moves=True)
    mv = info["moves"]
    assert mv.shape == (new.n, 3)
    for q in range(0, new.n, 37):
        i = int(np.where(st.id == new.id[q])[0][0])
        assert mv[q, 0] == st.r[i]
        assert mv[q, 1] == phi[i]
        direct = -(st.m / np.maximum(new.r[q], st.r)).sum()
        assert mv[q, 2] == pytest.approx(direct, rel=1e-13)


def test_empty_state():
    st = O.State(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.uint32))
    cor, skipped = O.energy_correction(st, np.zeros(0), np.zeros((0, 3)))
    assert cor.n == 0 and skipped == 0
