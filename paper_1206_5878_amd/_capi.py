"""ctypes declarations of libcmc.so (include/cmc.h), argument marshalling only.

Every computation runs in the HIP library; this module only mirrors the C
structs and loads the shared object.  It raises when the library is missing:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcmc.so")

CMC_OK, CMC_EINVAL, CMC_EWORKSPACE, CMC_EHIP, CMC_ERANGE, CMC_ESCRATCH = 0, -1, -2, -3, -4, -5
CMC_SCRATCH_BYTES = 64 << 20
CMC_FP64, CMC_MIXED = 0, 1
CMC_MODEL_PLUMMER, CMC_MODEL_KING = 0, 1
CMC_RNG_PHILOX, CMC_RNG_LFSR113 = 0, 1
CMC_STEP_DEVICE = 0xFFFFFFFF
CMC_BUCKET_CAP_MAX = 16383 * 2048 - 1
CMC_DIAG_N = 11
ST_NONFINITE, ST_TRIAL_CAP, ST_BOUND, ST_ESCAPER = 0x01, 0x02, 0x04, 0x08
ST_DT_DEGEN, ST_NUMERIC, ST_DT_NOCONV = 0x10, 0x20, 0x40

EXPORTS = ("cmc_workspace_bytes", "cmc_init_plummer", "cmc_init_model", "cmc_sort", "cmc_potential",
           "cmc_timestep", "cmc_relax", "cmc_orbit", "cmc_step", "cmc_step_timed", "cmc_step_noalloc",
           "cmc_energy_correction", "cmc_diagnostics", "cmc_philox", "cmc_rng_seed_lfsr113",
           "cmc_lfsr113", "cmc_strerror",
           "cmc_abi_version", "cmc_batch_device_bytes", "cmc_batch_prepare", "cmc_batch_init",
           "cmc_batch_step", "cmc_batch_sort", "cmc_batch_potential", "cmc_batch_timestep",
           "cmc_batch_relax", "cmc_batch_orbit", "cmc_batch_energy_correction",
           "cmc_batch_diagnostics", "cmc_set_tuning", "cmc_get_tuning")
CMC_TUNING_MAX = 32
CMC_SHAPES = 24


class cmc_scalars(C.Structure):
    _fields_ = [("n", C.c_int64), ("dt", C.c_double), ("status", C.c_uint32),
                ("dt_iters", C.c_uint32), ("n_esc", C.c_int64), ("trials", C.c_int64),
                ("violations", C.c_int64), ("capped", C.c_int64), ("e_esc", C.c_double),
                ("mass_norm", C.c_double), ("step", C.c_int64), ("corr_n", C.c_int64),
                ("corr_skipped", C.c_int64), ("reserved", C.c_int64 * 4)]


class cmc_state(C.Structure):
    _fields_ = [("cap", C.c_int64), ("r", C.c_void_p), ("vr", C.c_void_p),
                ("vt", C.c_void_p), ("m", C.c_void_p), ("m_f32", C.c_int32),
                ("reserved0", C.c_int32), ("id", C.c_void_p), ("phi", C.c_void_p),
                ("mcum", C.c_void_p), ("ssuf", C.c_void_p), ("r_new", C.c_void_p),
                ("sc", C.c_void_p), ("work", C.c_void_p), ("work_bytes", C.c_size_t),
                ("rng", C.c_void_p)]


class cmc_params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint32), ("precision", C.c_int32),
                ("gamma", C.c_double), ("target", C.c_double), ("bound_factor", C.c_double),
                ("trial_cap", C.c_int32), ("dt_iters", C.c_int32),
                ("energy_corr", C.c_int32), ("rng", C.c_int32)]


class cmc_cluster_spec(C.Structure):
    _fields_ = [("n", C.c_int64), ("seed", C.c_uint64), ("gamma", C.c_double),
                ("model", C.c_int32), ("mass_spectrum", C.c_int32), ("w0", C.c_double)]


class cmc_batch(C.Structure):
    _fields_ = [("clusters", C.c_int32), ("m_f32", C.c_int32), ("dev", C.c_void_p),
                ("dev_bytes", C.c_size_t), ("total", C.c_int64 * CMC_SHAPES),
                ("top_entries", C.c_int32), ("bucket_sort", C.c_int32),
                ("lfsr_ready", C.c_int32), ("sorted_searches", C.c_int32)]


class cmc_tuning(C.Structure):
    _fields_ = [("min_cap", C.c_int64), ("sorted", C.c_int32), ("bracket_blocks", C.c_int32),
                ("trial_chunk", C.c_int32), ("reserved", C.c_int32 * 3)]


assert C.sizeof(cmc_scalars) == 128
assert C.sizeof(cmc_params) == 56

_lib = None


class CmcError(RuntimeError):
    pass


def lib() -> C.CDLL:
    """The loaded libcmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CmcError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        sp, vp = C.POINTER(cmc_state), C.c_void_p
        pp = C.POINTER(cmc_params)
        L.cmc_workspace_bytes.argtypes = [C.c_int64]
        L.cmc_workspace_bytes.restype = C.c_size_t
        L.cmc_init_plummer.argtypes = [sp, C.c_int64, C.c_uint64, C.c_int32, vp]
        L.cmc_init_model.argtypes = [sp, C.c_int64, C.c_uint64, C.c_int32, C.c_int32,
                                     C.c_double, vp]
        L.cmc_sort.argtypes = [sp, vp]
        L.cmc_potential.argtypes = [sp, C.c_int32, vp]
        for f in ("cmc_timestep", "cmc_relax", "cmc_orbit", "cmc_step", "cmc_step_noalloc"):
            getattr(L, f).argtypes = [sp, pp, vp]
        L.cmc_step_timed.argtypes = [sp, pp, C.POINTER(C.c_void_p), vp]
        bp = C.POINTER(cmc_batch)
        L.cmc_batch_device_bytes.argtypes = [sp, C.c_int32]
        L.cmc_batch_device_bytes.restype = C.c_size_t
        L.cmc_batch_prepare.argtypes = [bp, sp, C.POINTER(cmc_cluster_spec), C.c_int32, vp,
                                        C.c_size_t]
        L.cmc_batch_init.argtypes = [bp, vp]
        L.cmc_batch_step.argtypes = [bp, pp, vp]
        L.cmc_batch_sort.argtypes = [bp, vp]
        for f in ("cmc_batch_timestep", "cmc_batch_relax", "cmc_batch_orbit"):
            getattr(L, f).argtypes = [bp, pp, vp]
        L.cmc_batch_potential.argtypes = [bp, C.c_int32, vp]
        L.cmc_batch_diagnostics.argtypes = [bp, vp, vp]
        L.cmc_energy_correction.argtypes = [sp, vp]
        L.cmc_batch_energy_correction.argtypes = [bp, vp]
        L.cmc_diagnostics.argtypes = [sp, vp, vp]
        L.cmc_philox.argtypes = [C.c_uint64, vp, vp, C.c_int64, vp]
        L.cmc_rng_seed_lfsr113.argtypes = [sp, C.POINTER(C.c_uint32), C.c_uint64, vp]
        L.cmc_lfsr113.argtypes = [vp, vp, C.c_int64, C.c_int32, vp]
        L.cmc_set_tuning.argtypes = [C.POINTER(cmc_tuning), C.c_int32]
        L.cmc_get_tuning.argtypes = [C.c_int64, C.POINTER(cmc_tuning)]
        L.cmc_strerror.argtypes = [C.c_int]
        L.cmc_strerror.restype = C.c_char_p
        L.cmc_abi_version.restype = C.c_int  # every other call returns int too
        _lib = L
        _install_tuning(L)
    return _lib


TUNING_PATH = os.path.join(HERE, "tuning.json")


def _install_tuning(L) -> None:
    """Install the autotuner's launch table (tune.py) when the package holds
    one; the library's built-in table serves otherwise."""
    if not os.path.exists(TUNING_PATH):
        return
    import json
    with open(TUNING_PATH) as f:
        table = json.load(f)["table"]
    arr = (cmc_tuning * len(table))()
    for k, e in enumerate(table):
        arr[k].min_cap = int(e["min_cap"])
        arr[k].sorted = int(e["sorted"])
        arr[k].bracket_blocks = int(e["bracket_blocks"])
        arr[k].trial_chunk = int(e["trial_chunk"])
    rc = L.cmc_set_tuning(arr, len(table))
    if rc != CMC_OK:
        raise CmcError(f"{TUNING_PATH}: the library refused the launch table (code {rc})")


def check(rc: int, what: str) -> None:
    if rc != CMC_OK:
        raise CmcError(f"{what}: {lib().cmc_strerror(rc).decode()} (code {rc})")
