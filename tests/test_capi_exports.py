"""The C-ABI library loads on the CPU and exports every call include/cmc.h
declares; the host-side argument checks reject bad input without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "cmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_call():
    from paper_1206_5878_amd import _capi as A
    L = A.lib()
    names = declared()
    assert "cmc_step" in names and len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(A.EXPORTS) == set(names)
    assert L.cmc_abi_version() == 7


def test_host_side_checks_without_gpu():
    from paper_1206_5878_amd import _capi as A
    L = A.lib()
    assert L.cmc_workspace_bytes(0) == 0
    assert L.cmc_workspace_bytes(1000) > 1000 * 64
    assert L.cmc_workspace_bytes(2**31) == 0
    s = A.cmc_state()  # all null pointers
    s.cap = 100
    p = A.cmc_params(1, 0, A.CMC_FP64, 0.11, 0.03, 1.2, 10000, 0)
    assert L.cmc_step(C.byref(s), C.byref(p), None) == A.CMC_EINVAL
    assert L.cmc_sort(C.byref(s), None) == A.CMC_EINVAL
    assert L.cmc_potential(C.byref(s), 0, None) == A.CMC_EINVAL
    assert L.cmc_energy_correction(C.byref(s), None) == A.CMC_EINVAL
    z = (C.c_uint32 * 4)(12345, 12345, 12345, 12345)
    assert L.cmc_rng_seed_lfsr113(C.byref(s), z, 0, None) == A.CMC_EINVAL
    assert L.cmc_lfsr113(None, None, -1, 1, None) == A.CMC_EINVAL
    assert L.cmc_lfsr113(None, None, 0, 4, None) == A.CMC_OK  # nothing to do
    assert L.cmc_init_plummer(None, 10, 1, 0, None) == A.CMC_EINVAL
    assert L.cmc_philox(1, None, None, 5, None) == A.CMC_EINVAL
    assert L.cmc_philox(1, None, None, 0, None) == A.CMC_OK
    # a fake, aligned, too-small workspace is caught before anything runs
    fake = 1 << 20
    s = A.cmc_state(100, fake, fake, fake, fake, 0, 0, fake, fake, fake, fake, fake, fake,
                    fake, 10)
    assert L.cmc_sort(C.byref(s), None) == A.CMC_EWORKSPACE
    s.work_bytes = L.cmc_workspace_bytes(100)
    s.work = fake + 8  # misaligned
    assert L.cmc_sort(C.byref(s), None) == A.CMC_EINVAL
    s.work = fake
    bad = A.cmc_params(1, 0, 7, 0.11, 0.03, 1.2, 10000, 0)
    assert L.cmc_step(C.byref(s), C.byref(bad), None) == A.CMC_EINVAL
    bad = A.cmc_params(1, 0, 0, 0.11, 1.5, 1.2, 10000, 0)
    assert L.cmc_timestep(C.byref(s), C.byref(bad), None) == A.CMC_EINVAL
    assert L.cmc_init_plummer(C.byref(s), 101, 1, 0, None) == A.CMC_ERANGE
    assert L.cmc_init_plummer(C.byref(s), 10, 1, 3, None) == A.CMC_EINVAL
    assert b"workspace" in L.cmc_strerror(A.CMC_EWORKSPACE)
    # the static-scratch step: a capacity beyond the scratch, and a pending
    # correction it could not keep, are refused before anything runs
    big = 1
    while L.cmc_workspace_bytes(big) <= A.CMC_SCRATCH_BYTES:
        big *= 2
    assert big > 200_000
    s.cap = big
    good = A.cmc_params(1, 0, 0, 0.11, 0.03, 1.2, 10000, 0)
    assert L.cmc_step_noalloc(C.byref(s), C.byref(good), None) == A.CMC_ESCRATCH
    assert b"scratch" in L.cmc_strerror(A.CMC_ESCRATCH)
    s.cap = 100
    corr = A.cmc_params(1, 0, 0, 0.11, 0.03, 1.2, 10000, 0, 1)
    assert L.cmc_step_noalloc(C.byref(s), C.byref(corr), None) == A.CMC_EINVAL
    assert L.cmc_step_noalloc(None, C.byref(good), None) == A.CMC_EINVAL


def test_launch_table_host_side():
    """The launch table: bad tables are refused and leave the one in use;
    lookups pick the band of a capacity; n = 0 restores the built-in table."""
    from paper_1206_5878_amd import _capi as A
    from paper_1206_5878_amd import tune
    L = A.lib()
    before = [tune.get(c) for c in (1, 1 << 17, 1 << 24)]
    good = [dict(min_cap=0, sorted=0, bracket_blocks=512, trial_chunk=64),
            dict(min_cap=1000, sorted=1, bracket_blocks=1024, trial_chunk=256)]
    bad = [
        [dict(good[0], min_cap=5)],                               # first band not at 0
        [good[1], good[0]],                                       # not increasing
        [dict(good[0], trial_chunk=100)],                         # not a multiple of 64
        [dict(good[0], trial_chunk=2048)],
        [dict(good[0], bracket_blocks=4)],
        [dict(good[0], sorted=2)],
    ]
    try:
        for t in bad:
            arr = tune.to_c(t)
            assert L.cmc_set_tuning(arr, len(t)) == A.CMC_EINVAL
        assert [tune.get(c) for c in (1, 1 << 17, 1 << 24)] == before
        assert L.cmc_set_tuning(None, A.CMC_TUNING_MAX + 1) == A.CMC_EINVAL
        tune.set_table(good)
        assert tune.get(999) == good[0]
        assert tune.get(1000) == good[1] and tune.get(10**9) == good[1]
        assert L.cmc_get_tuning(5, None) == A.CMC_EINVAL
    finally:
        tune.set_table([])
        A._install_tuning(L)
    assert [tune.get(c) for c in (1, 1 << 17, 1 << 24)] == before


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1206_5878_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("the oracle", ""), f
