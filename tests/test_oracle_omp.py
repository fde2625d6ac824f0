"""The oracle's OpenMP build (the CPU baseline's all-core leg) gives the
serial build's results bit for bit: its parallel loops are the per-star and
per-pair ones, and every sum runs serially in index order."""
import numpy as np

import oracle


def test_openmp_build_equals_serial_build():
    n, seed = 60_001, 4
    st = oracle.plummer(n, seed, 1)
    st.vr[::5003] = 2.5  # escapers
    ser, info_s = oracle.step(st, seed, 3, 0.01, moves=True)
    with oracle.threads() as L:
        assert L.ora_threads() >= 1
        par, info_p = oracle.step(st, seed, 3, 0.01, moves=True)
    for key in ("r", "vr", "vt", "m", "id"):
        assert np.array_equal(getattr(ser, key), getattr(par, key)), key
    assert info_s["dt"] == info_p["dt"] and info_s["n_after"] == info_p["n_after"]
    assert info_s["orbit"] == info_p["orbit"]
    assert np.array_equal(info_s["moves"], info_p["moves"])
    assert info_s["orbit"]["n_esc"] > 5


def test_openmp_build_equals_serial_build_lfsr():
    n, seed = 20_000, 6
    st = oracle.plummer(n, seed)
    st.rng = oracle.lfsr113_seed_states([0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321],
                                        st.id)
    ser, _ = oracle.step(st, seed, 1, 0.11, lfsr=True)
    with oracle.threads():
        par, _ = oracle.step(st, seed, 1, 0.11, lfsr=True)
    for key in ("r", "vr", "vt", "id", "rng"):
        assert np.array_equal(getattr(ser, key), getattr(par, key)), key


def test_threads_context_restores_the_serial_build():
    with oracle.threads():
        assert oracle.lib() is oracle.omp_lib()
    assert oracle.lib() is not oracle.omp_lib()
    assert oracle.lib().ora_threads() == 1
