"""Plain FP64 CPU oracle of one Henon Monte Carlo step (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``liboracle.so`` (plain C, built from
``cmc_oracle.c`` by ``oracle/build.py``) and shares no code with the HIP
library.  Method: arXiv:1206.5878, Sec. 2.1 (serial step) and Sec. 3.2 (bins).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

P_INIT_POS, P_INIT_SPEED, P_INIT_MASS = 0x10, 0x11, 0x12
P_RELAX, P_ORBIT, P_SIGN, P_ENSEMBLE = 0x20, 0x30, 0x31, 0x40

ST_NONFINITE, ST_TRIAL_CAP, ST_BOUND = 1, 2, 4
ST_ESCAPER, ST_DT_DEGEN, ST_NUMERIC = 8, 16, 32

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_vp = C.c_void_p


class OrbitStats(C.Structure):
    _fields_ = [("n_esc", C.c_int64), ("trials", C.c_int64), ("violations", C.c_int64),
                ("capped", C.c_int64), ("e_esc", C.c_double), ("status", C.c_uint32)]


class Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint32), ("gamma", C.c_double),
                ("target", C.c_double), ("dt_fixed", C.c_double), ("trial_cap", C.c_int32),
                ("bound_factor", C.c_double)]


class StepOut(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_after", C.c_int64), ("orbit", OrbitStats),
                ("status", C.c_uint32)]


_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_omp = None
_active = None  # the library the wrappers below call


def lib():
    """The library the wrappers call: the serial build, unless inside
    ``threads()``."""
    global _lib
    if _active is not None:
        return _active
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = load(_LIB_PATH)
    return _lib


def omp_lib():
    """The OpenMP build of the same source (same results bit for bit)."""
    global _omp
    if _omp is None:
        if not os.path.exists(_OMP_PATH):
            from . import build as _b
            _b.build()
        _omp = load(_OMP_PATH)
    return _omp


class threads:
    """``with oracle.threads():`` makes the wrappers call the OpenMP build
    (its team size: ``oracle.omp_lib().ora_threads()``)."""

    def __enter__(self):
        global _active
        self._prev = _active
        _active = omp_lib()
        return _active

    def __exit__(self, *exc):
        global _active
        _active = self._prev
        return False


def load(path: str):
    """A build of the oracle's C source at ``path`` with every entry point's
    argument types declared (the tests also load deliberately broken builds
    to show that the pins catch them)."""
    L = C.CDLL(path)
    L.ora_threads.restype = C.c_int
    L.ora_philox_many.argtypes = [C.c_int64, C.c_uint64, _up, _up]
    L.ora_u01.argtypes = [C.c_uint32, C.c_uint32]
    L.ora_u01.restype = C.c_double
    L.ora_u01f.argtypes = [C.c_uint32]
    L.ora_u01f.restype = C.c_float
    L.ora_plummer.argtypes = [C.c_int64, C.c_uint64, C.c_int, _dp, _dp, _dp, _dp, _up]
    L.ora_king.argtypes = [C.c_int64, C.c_uint64, C.c_double, C.c_int, _dp, _dp, _dp, _dp,
                           _up]
    L.ora_king_profile.argtypes = [C.c_double, _dp, _dp, _dp, C.c_int, _dp]
    L.ora_king_profile.restype = C.c_int
    L.ora_king_density.argtypes = [C.c_double]
    L.ora_king_density.restype = C.c_double
    L.ora_sort_perm.argtypes = [C.c_int64, _dp, _ip]
    L.ora_potential.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp]
    L.ora_phi_at.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double]
    L.ora_phi_at.restype = C.c_double
    L.ora_pair_terms.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _up, C.c_uint64,
                                 C.c_uint32, C.c_double, _dp, _dp, _dp]
    L.ora_pair_terms.restype = C.c_int64
    L.ora_mean_sin2.argtypes = [C.c_int64, _dp, _dp, C.c_double]
    L.ora_mean_sin2.restype = C.c_double
    L.ora_solve_dt.argtypes = [C.c_int64, _dp, _dp, C.c_double, C.POINTER(C.c_uint32)]
    L.ora_solve_dt.restype = C.c_double
    L.ora_relax.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _up, C.c_uint64, C.c_uint32,
                            C.c_double, C.c_double]
    L.ora_orbit.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _up, C.c_uint64,
                            C.c_uint32, C.c_int32, C.c_double, _dp,
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                            C.POINTER(OrbitStats)]
    L.ora_step.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _up, _dp, _dp,
                           C.POINTER(Params), C.POINTER(StepOut)]
    L.ora_step_ex.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _up, _dp, _dp,
                              C.POINTER(Params), C.POINTER(StepOut), _vp, _vp]
    L.ora_lfsr113_next.argtypes = [_up]
    L.ora_lfsr113_next.restype = C.c_uint32
    L.ora_lfsr113_block.argtypes = [_up, _up]
    L.ora_lfsr113_jump_pow2.argtypes = [_up, C.c_int]
    L.ora_lfsr113_stream.argtypes = [_up, C.c_uint64, _up]
    L.ora_lfsr113_component_period.argtypes = [C.c_int, C.c_uint32, C.c_int64]
    L.ora_lfsr113_component_period.restype = C.c_int64
    L.ora_energy_correction.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_energy_correction.restype = C.c_int64
    L.ora_orbit_subset.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _up,
                                   C.c_uint64, C.c_uint32, C.c_int32, C.c_double, C.c_int64,
                                   _ip, _dp]
    L.ora_diagnostics.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    return L


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _u32(x):
    return np.ascontiguousarray(x, dtype=np.uint32)


# ---------------------------------------------------------------- random numbers
def philox(key: int, ctr: np.ndarray) -> np.ndarray:
    """Philox4x32-10 blocks for counters ``ctr`` (shape (n, 4), uint32)."""
    ctr = _u32(ctr).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().ora_philox_many(ctr.shape[0], key, ctr.reshape(-1), out.reshape(-1))
    return out


def u01(hi, lo) -> float:
    return lib().ora_u01(int(hi), int(lo))


def u01f(hi) -> float:
    return lib().ora_u01f(int(hi))


def lfsr113_blocks(z, nblocks: int):
    """(state after, words (nblocks, 4)) of the LFSR113 generator from state z."""
    z = _u32(z).copy()
    out = np.empty((nblocks, 4), np.uint32)
    w = np.empty(4, np.uint32)
    for b in range(nblocks):
        lib().ora_lfsr113_block(z, w)
        out[b] = w
    return z, out


def lfsr113_jump_pow2(z, e: int):
    z = _u32(z).copy()
    lib().ora_lfsr113_jump_pow2(z, int(e))
    return z


def lfsr113_stream(z0, sid: int):
    """State of stream ``sid``: z0 advanced by sid * 2^80 steps."""
    out = np.empty(4, np.uint32)
    lib().ora_lfsr113_stream(_u32(z0).copy(), int(sid), out)
    return out


def lfsr113_component_period(c: int, z: int, limit: int) -> int:
    return lib().ora_lfsr113_component_period(int(c), int(z), int(limit))


def lfsr113_seed_states(z0, ids):
    """Every star's stream state (one stream per star id)."""
    return np.stack([lfsr113_stream(z0, int(i)) for i in ids]) if len(ids) else \
        np.zeros((0, 4), np.uint32)


# ---------------------------------------------------------------- state helpers
class State:
    """Sorted SoA star state (host, FP64); rng: optional LFSR113 states,
    shape (n, 4) uint32, that move with the stars."""

    def __init__(self, r, vr, vt, m, id_, rng=None):
        self.r = _f64(r).copy()
        self.vr = _f64(vr).copy()
        self.vt = _f64(vt).copy()
        self.m = _f64(m).copy()
        self.id = _u32(id_).copy()
        self.rng = None if rng is None else _u32(rng).reshape(-1, 4).copy()

    @property
    def n(self) -> int:
        return self.r.shape[0]

    def copy(self) -> "State":
        return State(self.r, self.vr, self.vt, self.m, self.id, self.rng)


def plummer_unsorted(n: int, seed: int, mass_spectrum: int = 0):
    r = np.empty(n); vr = np.empty(n); vt = np.empty(n); m = np.empty(n)
    id_ = np.empty(n, dtype=np.uint32)
    lib().ora_plummer(n, seed, mass_spectrum, r, vr, vt, m, id_)
    return r, vr, vt, m, id_


def sort_perm(key: np.ndarray) -> np.ndarray:
    key = _f64(key)
    perm = np.empty(key.shape[0], dtype=np.int64)
    lib().ora_sort_perm(key.shape[0], key, perm)
    return perm


def king_profile(w0: float, cap: int = 4096):
    """King (1966) profile: node arrays r, W, M and (r_t, M_t, W_pot)."""
    r = np.empty(cap); W = np.empty(cap); M = np.empty(cap); tail = np.empty(3)
    k = lib().ora_king_profile(float(w0), r, W, M, cap, tail)
    return r[:k], W[:k], M[:k], tuple(tail)


def king_density(W: float) -> float:
    return lib().ora_king_density(float(W))


def king_unsorted(n: int, seed: int, w0: float, mass_spectrum: int = 0):
    r = np.empty(max(n, 1)); vr = np.empty_like(r); vt = np.empty_like(r); m = np.empty_like(r)
    id_ = np.empty(max(n, 1), np.uint32)
    lib().ora_king(n, seed, float(w0), mass_spectrum, r, vr, vt, m, id_)
    return r[:n], vr[:n], vt[:n], m[:n], id_[:n]


def king(n: int, seed: int, w0: float, mass_spectrum: int = 0) -> State:
    """A King model, sorted by radius (as the device init leaves it)."""
    r, vr, vt, m, id_ = king_unsorted(n, seed, w0, mass_spectrum)
    p = sort_perm(r)
    return State(r[p], vr[p], vt[p], m[p], id_[p])


def plummer(n: int, seed: int, mass_spectrum: int = 0) -> State:
    """Initial Plummer model sorted by radius (ties by id)."""
    r, vr, vt, m, id_ = plummer_unsorted(n, seed, mass_spectrum)
    p = sort_perm(r)
    return State(r[p], vr[p], vt[p], m[p], id_[p])


def potential(r, m):
    """(phi, mcum, ssuf): Phi_k, inclusive mass prefix M_k, exclusive suffix
    S_k of m/r, with Phi_k = -(M_k / r_k + S_k)."""
    r = _f64(r); m = _f64(m)
    phi = np.empty_like(r); mcum = np.empty_like(r); ssuf = np.empty_like(r)
    lib().ora_potential(r.shape[0], r, m, phi, mcum, ssuf)
    return phi, mcum, ssuf


def phi_at(r, table, x: float) -> float:
    phi, mcum, ssuf = table
    return lib().ora_phi_at(r.shape[0], _f64(r), _f64(phi), _f64(mcum), _f64(ssuf),
                            float(x))


def pair_terms(st: State, seed: int, step: int, gamma: float):
    np_ = st.n // 2
    w = np.empty(max(np_, 1)); tp = np.empty(max(np_, 1)); nb = np.empty(max(np_, 1))
    lib().ora_pair_terms(st.n, st.r, st.m, st.vr, st.vt, st.id, seed, step, gamma, w, tp, nb)
    return w[:np_], tp[:np_], nb[:np_]


def mean_sin2(w, tp, dt: float) -> float:
    return lib().ora_mean_sin2(len(w), _f64(w), _f64(tp), float(dt))


def solve_dt(w, tp, target: float):
    """(dt, status) with mean sin^2(beta/2) = target."""
    if len(w) == 0:
        return 0.0, ST_DT_DEGEN
    status = C.c_uint32(0)
    dt = lib().ora_solve_dt(len(w), _f64(w), _f64(tp), target, C.byref(status))
    return dt, status.value


def timestep(st: State, seed: int, step: int, gamma: float, target: float):
    w, tp, _ = pair_terms(st, seed, step, gamma)
    return solve_dt(w, tp, target)


def relax(st: State, seed: int, step: int, gamma: float, dt: float) -> State:
    out = st.copy()
    lib().ora_relax(out.n, out.r, out.m, out.vr, out.vt, out.id, seed, step, gamma, dt)
    return out


def orbit(st: State, table, seed: int, step: int, trial_cap: int = 10000,
          bound_factor: float = 1.2, details: bool = False):
    """New orbits for a sorted state with table (phi, mcum, ssuf) from
    ``potential``.  Returns (r_new, vr_new, vt_new, stats[, details dict])."""
    phi, mcum, ssuf = table
    n = st.n
    vr = st.vr.copy(); vt = st.vt.copy()
    r_new = np.empty(max(n, 1))
    st_ = OrbitStats()
    d = {}
    keys = ("E", "J", "kmin", "kmax", "rmin", "rmax", "trials", "flags")
    ptrs = [None] * len(keys)
    if details:
        d = dict(E=np.empty(n), J=np.empty(n), kmin=np.empty(n, np.int64),
                 kmax=np.empty(n, np.int64), rmin=np.empty(n), rmax=np.empty(n),
                 trials=np.empty(n, np.int32), flags=np.empty(n, np.uint32))
        ptrs = [d[k].ctypes.data for k in keys]
    lib().ora_orbit(n, st.r, _f64(phi), _f64(mcum), _f64(ssuf), st.m, vr, vt, st.id, seed, step,
                    trial_cap, bound_factor, r_new, *ptrs, C.byref(st_))
    stats = {k: getattr(st_, k) for k, _ in OrbitStats._fields_}
    if details:
        return r_new[:n], vr, vt, stats, d
    return r_new[:n], vr, vt, stats


def orbit_subset(st: State, table, seed: int, step: int, idx, trial_cap: int = 10000,
                 bound_factor: float = 1.2):
    """``orbit`` for the stars at positions idx only: (r_new, vr, vt) of those
    stars (r_new = inf for an escaper)."""
    phi, mcum, ssuf = table
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    vr = st.vr.copy(); vt = st.vt.copy()
    r_new = np.full(max(st.n, 1), np.nan)
    lib().ora_orbit_subset(st.n, st.r, _f64(phi), _f64(mcum), _f64(ssuf), st.m, vr, vt, st.id,
                           seed, step, trial_cap, bound_factor, idx.shape[0], idx, r_new)
    return r_new[idx], vr[idx], vt[idx]


def step(st: State, seed: int, step_idx: int, gamma: float, target: float = 0.03,
         dt_fixed: float = 0.0, trial_cap: int = 10000, bound_factor: float = 1.2,
         moves: bool = False, lfsr: bool = False):
    """One whole step on a copy of ``st``.  Returns (new_state, info dict).
    moves: also info["moves"], shape (n_after, 3): each new star's
    (r_old, Phi_old(r_old), Phi_old(r_new)) for ``energy_correction``.
    lfsr: draw from the stars' LFSR113 streams (st.rng) instead of Philox."""
    s = st.copy()
    if lfsr and (s.rng is None or s.rng.shape[0] != s.n):
        raise ValueError("lfsr needs st.rng with one state per star")
    rng = s.rng.reshape(-1) if lfsr and s.n else None
    phi = np.empty(max(s.n, 1)); mcum = np.empty(max(s.n, 1))
    mv = np.empty(3 * max(s.n, 1)) if moves else None
    p = Params(seed, step_idx, gamma, target, dt_fixed, trial_cap, bound_factor)
    o = StepOut()
    lib().ora_step_ex(s.n, s.r, s.vr, s.vt, s.m, s.id, phi, mcum, C.byref(p), C.byref(o),
                      mv.ctypes.data if moves else None,
                      rng.ctypes.data if rng is not None else None)
    k = o.n_after
    new = State(s.r[:k], s.vr[:k], s.vt[:k], s.m[:k], s.id[:k],
                s.rng[:k] if lfsr else None)
    info = dict(dt=o.dt, n_after=k, status=o.status,
                orbit={f: getattr(o.orbit, f) for f, _ in OrbitStats._fields_},
                phi=phi[:st.n], mcum=mcum[:st.n])
    if moves:
        info["moves"] = mv[:3 * k].reshape(k, 3).copy()
    return new, info


def energy_correction(st: State, phi, moves) -> tuple:
    """Sec. 2.1 item 6 on a copy of ``st`` (the state a step left, ``phi`` its
    potential, ``moves`` that step's info["moves"]).  Returns (state, skipped)."""
    out = st.copy()
    mv = _f64(moves).reshape(-1)
    if mv.shape[0] != 3 * out.n:
        raise ValueError("moves must hold 3 values per star of the state")
    k = lib().ora_energy_correction(out.n, out.r, out.m, out.vr, out.vt, _f64(phi),
                                    mv if out.n else np.zeros(1))
    return out, int(k)


def diagnostics(st: State, phi=None, mcum=None) -> dict:
    if phi is None:
        phi, mcum, _ = potential(st.r, st.m)
    out = np.empty(11)
    lib().ora_diagnostics(st.n, st.r, st.vr, st.vt, st.m, _f64(phi), _f64(mcum), out)
    return dict(T=out[0], W=out[1], E=out[2], virial=out[3], M=out[4],
                r01=out[5], r10=out[6], r50=out[7], r90=out[8], rc=out[9], rho_c=out[10])
