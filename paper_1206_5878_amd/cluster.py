"""Torch-backed cluster state and thin wrappers named after the C ABI calls.

PyTorch supplies device memory (one tensor per SoA array, a zero-filled
workspace) and the current HIP stream; every step of the method runs in
libcmc.so.  Method: arXiv:1206.5878, Sec. 2.1.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi as A


@dataclass
class Params:
    """Mirror of cmc_params with the workload defaults."""
    seed: int = 1
    step: int = 0
    precision: int = A.CMC_FP64
    gamma: float = 0.11
    target: float = 0.03
    bound_factor: float = 1.2
    trial_cap: int = 10000
    dt_iters: int = 0
    energy_corr: int = 0
    rng: int = A.CMC_RNG_PHILOX

    def c(self) -> A.cmc_params:
        return A.cmc_params(self.seed, self.step, self.precision, self.gamma, self.target,
                            self.bound_factor, self.trial_cap, self.dt_iters,
                            self.energy_corr, self.rng)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Cluster:
    """Device arrays of one cluster of capacity ``cap`` (see cmc_state).
    rng: also allocate the per-star LFSR113 stream states."""

    def __init__(self, cap: int, m_f32: bool = False, device: str = "cuda", rng: bool = False):
        if cap <= 0:
            raise ValueError("cap must be positive")
        L = A.lib()
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.cap = int(cap)
        self.m_f32 = bool(m_f32)
        self.r = torch.zeros(cap, **f64)
        self.vr = torch.zeros(cap, **f64)
        self.vt = torch.zeros(cap, **f64)
        self.m = torch.zeros(cap, dtype=torch.float32 if m_f32 else torch.float64, device=dev)
        self.id = torch.zeros(cap, dtype=torch.int32, device=dev)  # uint32 bits
        self.phi = torch.zeros(cap, **f64)
        self.mcum = torch.zeros(cap, **f64)
        self.ssuf = torch.zeros(cap, **f64)
        self.r_new = torch.zeros(cap, **f64)
        self.sc = torch.zeros(16, dtype=torch.int64, device=dev)
        self.rng = torch.zeros(4 * cap, dtype=torch.int32, device=dev) if rng else None
        nbytes = int(L.cmc_workspace_bytes(cap))
        if nbytes == 0:
            raise A.CmcError("capacity out of range")
        self.work = torch.zeros(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.work.data_ptr()
        off = (-base) % 256
        self._c = A.cmc_state(cap, self.r.data_ptr(), self.vr.data_ptr(), self.vt.data_ptr(),
                              self.m.data_ptr(), 1 if m_f32 else 0, 0, self.id.data_ptr(),
                              self.phi.data_ptr(), self.mcum.data_ptr(), self.ssuf.data_ptr(),
                              self.r_new.data_ptr(), self.sc.data_ptr(), base + off, nbytes,
                              self.rng.data_ptr() if rng else None)

    # ------------------------------------------------------------ host views
    def scalars(self) -> dict:
        raw = self.sc.cpu().numpy().tobytes()
        s = A.cmc_scalars.from_buffer_copy(raw)
        return {f: getattr(s, f) for f, _ in A.cmc_scalars._fields_ if f != "reserved"}

    @property
    def n(self) -> int:
        return int(self.sc[0].item())

    def set_scalar(self, name: str, value) -> None:
        s = A.cmc_scalars.from_buffer_copy(self.sc.cpu().numpy().tobytes())
        setattr(s, name, value)
        buf = np.frombuffer(bytes(s), dtype=np.int64).copy()
        self.sc.copy_(torch.from_numpy(buf))

    def load(self, r, vr, vt, m, id_, rng=None) -> None:
        """Upload a host state (first len(r) entries; rng: (n, 4) LFSR113
        states), set n and drop any pending energy correction (it belonged to
        the stars this replaces)."""
        n = len(r)
        if n > self.cap:
            raise A.CmcError("n > cap")
        dev = self.r.device
        self.r[:n] = torch.as_tensor(np.asarray(r, np.float64), device=dev)
        self.vr[:n] = torch.as_tensor(np.asarray(vr, np.float64), device=dev)
        self.vt[:n] = torch.as_tensor(np.asarray(vt, np.float64), device=dev)
        mt = np.float32 if self.m_f32 else np.float64
        self.m[:n] = torch.as_tensor(np.asarray(m, mt), device=dev)
        self.id[:n] = torch.as_tensor(np.asarray(id_, np.uint32).view(np.int32), device=dev)
        if rng is not None:
            z = np.ascontiguousarray(rng, np.uint32).reshape(-1)
            self.rng[:4 * n] = torch.as_tensor(z.view(np.int32), device=dev)
        sc = A.cmc_scalars.from_buffer_copy(self.sc.cpu().numpy().tobytes())
        sc.n = n
        sc.corr_n = 0
        self.sc.copy_(torch.from_numpy(np.frombuffer(bytes(sc), dtype=np.int64).copy()))

    def checkpoint(self) -> dict:
        """Host copy of everything a later step reads: the active stars'
        arrays (and LFSR113 states), and the scalars block with n, the dt
        the next solve starts from and the device step counter.  Random
        draws are keyed by (id, step), so a run resumed from it repeats the
        uninterrupted run bit for bit.  A pending energy correction lives in
        the workspace: apply it first (cmc_potential, cmc_energy_correction)."""
        sc = self.scalars()
        if sc["corr_n"]:
            raise A.CmcError("a correction is pending: call cmc_potential and "
                             "cmc_energy_correction before the checkpoint")
        h = self.host()
        ck = {k: h[k] for k in ("r", "vr", "vt", "id")}
        ck["m"] = self.m[:self.n].cpu().numpy()
        if self.rng is not None:
            ck["rng"] = h["rng"]
        ck["scalars"] = self.sc.cpu().numpy().copy()
        return ck

    def save(self, path: str) -> None:
        """checkpoint() as a numpy .npz file (plain arrays, no pickles)."""
        np.savez(path, **self.checkpoint())

    def restore(self, ck) -> None:
        """Load a checkpoint (the dict, or a path to a saved one) into this
        cluster: same mass storage, capacity at least its n."""
        if isinstance(ck, str):
            with np.load(ck, allow_pickle=False) as f:
                ck = {k: f[k] for k in f.files}
        n = int(ck["r"].shape[0])
        if n > self.cap:
            raise A.CmcError("checkpoint larger than the capacity")
        if (ck["m"].dtype == np.float32) != self.m_f32:
            raise A.CmcError("checkpoint mass storage differs from the cluster's")
        if ("rng" in ck) and self.rng is None:
            raise A.CmcError("checkpoint has LFSR113 states: make the cluster with rng=True")
        dev = self.r.device
        for k in ("r", "vr", "vt"):
            getattr(self, k)[:n] = torch.as_tensor(ck[k], device=dev)
        self.m[:n] = torch.as_tensor(ck["m"], device=dev)
        self.id[:n] = torch.as_tensor(np.asarray(ck["id"], np.uint32).view(np.int32), device=dev)
        if "rng" in ck:
            z = np.ascontiguousarray(ck["rng"], np.uint32).reshape(-1)
            self.rng[:4 * n] = torch.as_tensor(z.view(np.int32), device=dev)
        self.sc.copy_(torch.as_tensor(np.asarray(ck["scalars"], np.int64), device=dev))

    def capture(self, p: Params) -> torch.cuda.CUDAGraph:
        """A graph of one cmc_step that takes its step index from the device
        counter and advances it (CMC_STEP_DEVICE): replay it once per step."""
        q = Params(**{**p.__dict__, "step": A.CMC_STEP_DEVICE})
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                cmc_step(self, q, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        return g

    def host(self, n: int | None = None) -> dict:
        """Copy the first n (default: active) entries of every array to numpy."""
        n = self.n if n is None else n
        out = {k: getattr(self, k)[:n].cpu().numpy() for k in
               ("r", "vr", "vt", "phi", "mcum", "ssuf", "r_new")}
        out["m"] = self.m[:n].cpu().numpy().astype(np.float64)
        out["id"] = self.id[:n].cpu().numpy().view(np.uint32)
        if self.rng is not None:
            out["rng"] = self.rng[:4 * n].cpu().numpy().view(np.uint32).reshape(n, 4)
        return out

    @property
    def c(self):
        return C.byref(self._c)


# ---------------------------------------------------------------- ABI calls
def cmc_init_model(cl: Cluster, n: int, seed: int, model: int, mass_spectrum: int = 0,
                   w0: float = 0.0, stream=None):
    A.check(A.lib().cmc_init_model(cl.c, n, seed, model, mass_spectrum, w0, _stream(stream)),
            "cmc_init_model")


def cmc_init_plummer(cl: Cluster, n: int, seed: int, mass_spectrum: int = 0, stream=None):
    A.check(A.lib().cmc_init_plummer(cl.c, n, seed, mass_spectrum, _stream(stream)),
            "cmc_init_plummer")


def cmc_sort(cl: Cluster, stream=None):
    A.check(A.lib().cmc_sort(cl.c, _stream(stream)), "cmc_sort")


def cmc_potential(cl: Cluster, precision: int = A.CMC_FP64, stream=None):
    A.check(A.lib().cmc_potential(cl.c, precision, _stream(stream)), "cmc_potential")


def cmc_timestep(cl: Cluster, p: Params, stream=None):
    pc = p.c()
    A.check(A.lib().cmc_timestep(cl.c, C.byref(pc), _stream(stream)), "cmc_timestep")


def cmc_relax(cl: Cluster, p: Params, stream=None):
    pc = p.c()
    A.check(A.lib().cmc_relax(cl.c, C.byref(pc), _stream(stream)), "cmc_relax")


def cmc_orbit(cl: Cluster, p: Params, stream=None):
    pc = p.c()
    A.check(A.lib().cmc_orbit(cl.c, C.byref(pc), _stream(stream)), "cmc_orbit")


def cmc_step(cl: Cluster, p: Params, stream=None):
    pc = p.c()
    A.check(A.lib().cmc_step(cl.c, C.byref(pc), _stream(stream)), "cmc_step")


def cmc_step_noalloc(cl: Cluster, p: Params, stream=None):
    """cmc_step on the library's static per-GPU scratch instead of the
    cluster's workspace (for callers that cannot allocate); caps up to
    cmc_workspace_bytes(cap) <= CMC_SCRATCH_BYTES, energy_corr = 0."""
    pc = p.c()
    A.check(A.lib().cmc_step_noalloc(cl.c, C.byref(pc), _stream(stream)), "cmc_step_noalloc")


def cmc_energy_correction(cl: Cluster, stream=None):
    A.check(A.lib().cmc_energy_correction(cl.c, _stream(stream)), "cmc_energy_correction")


def cmc_diagnostics(cl: Cluster, stream=None) -> dict:
    out = torch.zeros(A.CMC_DIAG_N, dtype=torch.float64, device=cl.r.device)
    A.check(A.lib().cmc_diagnostics(cl.c, C.c_void_p(out.data_ptr()), _stream(stream)),
            "cmc_diagnostics")
    return dict(zip(_DIAG_KEYS, out.cpu().numpy()))


def cmc_philox(key: int, ctr: np.ndarray, device: str = "cuda", stream=None) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    n = c.shape[0]
    dc = torch.as_tensor(c.view(np.int32), device=device)
    do = torch.zeros_like(dc)
    A.check(A.lib().cmc_philox(key, C.c_void_p(dc.data_ptr()), C.c_void_p(do.data_ptr()), n,
                               _stream(stream)), "cmc_philox")
    return do.cpu().numpy().view(np.uint32)


def cmc_rng_seed_lfsr113(cl: Cluster, z0, stream_base: int = 0, stream=None):
    """Every star's LFSR113 state: z0 advanced by (stream_base + id) * 2^80."""
    z = (C.c_uint32 * 4)(*[int(x) for x in z0])
    A.check(A.lib().cmc_rng_seed_lfsr113(cl.c, z, int(stream_base), _stream(stream)),
            "cmc_rng_seed_lfsr113")


def cmc_lfsr113(states: np.ndarray, blocks: int, device: str = "cuda",
                stream=None) -> np.ndarray:
    """Raw LFSR113 words: (n, blocks, 4) from n states (n, 4)."""
    z = np.ascontiguousarray(states, dtype=np.uint32).reshape(-1, 4)
    n = z.shape[0]
    dz = torch.as_tensor(z.view(np.int32), device=device)
    do = torch.zeros(n * blocks * 4, dtype=torch.int32, device=device)
    A.check(A.lib().cmc_lfsr113(C.c_void_p(dz.data_ptr()), C.c_void_p(do.data_ptr()), n,
                                blocks, _stream(stream)), "cmc_lfsr113")
    return do.cpu().numpy().view(np.uint32).reshape(n, blocks, 4)


def cmc_step_timed(cl: Cluster, p: Params, events, stream=None):
    """cmc_step recording the six HIP events ``events`` (raw hipEvent_t
    handles, see hipevents.EventSet) around its five phases."""
    pc = p.c()
    arr = (C.c_void_p * 6)(*events)
    A.check(A.lib().cmc_step_timed(cl.c, C.byref(pc), arr, _stream(stream)), "cmc_step_timed")


# ---------------------------------------------------------------- ensembles
_DIAG_KEYS = ("T", "W", "E", "virial", "M", "r01", "r10", "r50", "r90", "rc", "rho_c")


class Ensemble:
    """Independent clusters advanced by the same launches (cmc_batch_*).

    specs: one dict per cluster with keys n, seed, gamma, model, and
    optionally mass_spectrum, w0, cap (default n)."""

    def __init__(self, specs, m_f32: bool = False, device: str = "cuda", rng: bool = False):
        L = A.lib()
        self.specs = [dict(s) for s in specs]
        self.clusters = [Cluster(int(s.get("cap", s["n"])), m_f32=m_f32, device=device, rng=rng)
                         for s in self.specs]
        k = len(self.clusters)
        self._states = (A.cmc_state * k)(*[cl._c for cl in self.clusters])
        self._specs = (A.cmc_cluster_spec * k)(*[
            A.cmc_cluster_spec(int(s["n"]), int(s["seed"]), float(s["gamma"]), int(s["model"]),
                               int(s.get("mass_spectrum", 0)), float(s.get("w0", 0.0)))
            for s in self.specs])
        nbytes = int(L.cmc_batch_device_bytes(self._states, k))
        if nbytes == 0:
            raise A.CmcError("invalid ensemble states")
        self.dev = torch.zeros(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
        base = self.dev.data_ptr()
        self.handle = A.cmc_batch()
        A.check(L.cmc_batch_prepare(C.byref(self.handle), self._states, self._specs, k,
                                    C.c_void_p(base + (-base) % 256), nbytes),
                "cmc_batch_prepare")

    def __len__(self):
        return len(self.clusters)

    def init(self, stream=None):
        A.check(A.lib().cmc_batch_init(C.byref(self.handle), _stream(stream)), "cmc_batch_init")

    def seed_lfsr113(self, z0, stream=None):
        """Each cluster's stars get LFSR113 streams; cluster c's stream indices
        start after the capacities of the clusters before it."""
        base = 0
        for cl in self.clusters:
            cmc_rng_seed_lfsr113(cl, z0, base, stream)
            base += cl.cap

    def step(self, p: Params, stream=None):
        pc = p.c()
        A.check(A.lib().cmc_batch_step(C.byref(self.handle), C.byref(pc), _stream(stream)),
                "cmc_batch_step")

    def potential(self, precision: int = A.CMC_FP64, stream=None):
        A.check(A.lib().cmc_batch_potential(C.byref(self.handle), precision, _stream(stream)),
                "cmc_batch_potential")

    def sort(self, stream=None):
        A.check(A.lib().cmc_batch_sort(C.byref(self.handle), _stream(stream)), "cmc_batch_sort")

    def timestep(self, p: Params, stream=None):
        pc = p.c()
        A.check(A.lib().cmc_batch_timestep(C.byref(self.handle), C.byref(pc), _stream(stream)),
                "cmc_batch_timestep")

    def relax(self, p: Params, stream=None):
        pc = p.c()
        A.check(A.lib().cmc_batch_relax(C.byref(self.handle), C.byref(pc), _stream(stream)),
                "cmc_batch_relax")

    def orbit(self, p: Params, stream=None):
        pc = p.c()
        A.check(A.lib().cmc_batch_orbit(C.byref(self.handle), C.byref(pc), _stream(stream)),
                "cmc_batch_orbit")

    def energy_correction(self, stream=None):
        A.check(A.lib().cmc_batch_energy_correction(C.byref(self.handle), _stream(stream)),
                "cmc_batch_energy_correction")

    def diagnostics(self, stream=None) -> list:
        out = torch.zeros(A.CMC_DIAG_N * len(self), dtype=torch.float64,
                          device=self.dev.device)
        A.check(A.lib().cmc_batch_diagnostics(C.byref(self.handle), C.c_void_p(out.data_ptr()),
                                              _stream(stream)), "cmc_batch_diagnostics")
        v = out.cpu().numpy().reshape(-1, A.CMC_DIAG_N)
        return [dict(zip(_DIAG_KEYS, row)) for row in v]

    def capture(self, p: Params) -> torch.cuda.CUDAGraph:
        """A graph of one ensemble step that advances the step index on the
        device (CMC_STEP_DEVICE): replay it once per step."""
        q = Params(**{**p.__dict__, "step": A.CMC_STEP_DEVICE})
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.step(q, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        return g
