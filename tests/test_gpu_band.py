"""Free-running FP64 GPU trajectories against the oracle's, as ensembles.

N = 1e5 equal-mass Plummer, ln(0.11 N), 100 steps.  The oracle runs 8
independent trajectories (initial model and step draws from seeds 2..9) and
the GPU 8 more (seeds 10..17).  Every step redraws every orbit, so
trajectories decorrelate within a few steps and only their statistics can
be compared: after steps 10, 20, ..., 100, the relative energy change
(E - E0)/|E0|, virial ratio 2T/|W| and 10/50/90 % Lagrange radii of the two
ensembles must have the same mean, within 5 standard errors of the
difference (Welch's t; |t| > 5 at about 14 degrees of freedom has
probability 2e-4).  The paper compares runs the same way, by their
statistics (Sec. 4.1).  The ensembles take their own initial models: one
model's sampling offset persists through the 100 steps (seed 1's half-mass
radius stays about 1.6 standard deviations above the mean), so a single
trajectory against a band would test that draw rather than the step."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 100_000
GAMMA = 0.11
STEPS = 100
KEYS = ("drift", "virial", "r10", "r50", "r90")


@pytest.fixture(scope="module")
def cmc():
    import torch
    assert torch.cuda.is_available()
    import paper_1206_5878_amd as P
    P.lib()
    return P


def sample(d, e0):
    return [(d["E"] - e0) / abs(e0), d["virial"], d["r10"], d["r50"], d["r90"]]


def oracle_track(ora, seed, out):
    st = ora.plummer(N, seed)
    e0 = ora.diagnostics(st)["E"]
    rows = []
    for k in range(STEPS):
        st, _ = ora.step(st, seed, k, GAMMA)
        if k % 10 == 9:
            rows.append(sample(ora.diagnostics(st), e0))
    out[seed] = np.array(rows)


def gpu_track(cmc, seed):
    cl = cmc.Cluster(N)
    cmc.cmc_init_plummer(cl, N, seed, 0)
    cmc.cmc_potential(cl)
    e0 = float(cmc.cmc_diagnostics(cl)["E"])
    rows = []
    for k in range(STEPS):
        cmc.cmc_step(cl, cmc.Params(seed=seed, step=k, gamma=GAMMA))
        if k % 10 == 9:
            cmc.cmc_potential(cl)
            rows.append(sample(cmc.cmc_diagnostics(cl), e0))
    return np.array(rows)


def test_gpu_ensemble_matches_oracle_ensemble(cmc, ora):
    seeds = list(range(2, 10))
    out = {}
    # the oracle is plain C behind ctypes, which releases the GIL: the 8
    # trajectories run on 8 host cores at once
    th = [threading.Thread(target=oracle_track, args=(ora, s, out)) for s in seeds]
    for t in th:
        t.start()
    gpu = np.stack([gpu_track(cmc, s) for s in range(10, 18)])   # (runs, samples, keys)
    for t in th:
        t.join()
    band = np.stack([out[s] for s in seeds])
    mg, mo = gpu.mean(axis=0), band.mean(axis=0)
    vg, vo = gpu.var(axis=0, ddof=1), band.var(axis=0, ddof=1)
    tw = (mg - mo) / np.sqrt(vg / len(gpu) + vo / len(band))
    for j, key in enumerate(KEYS):
        print(f"{key} (step 100): gpu {mg[-1, j]:.5g} +- {np.sqrt(vg[-1, j]):.2g}, "
              f"oracle {mo[-1, j]:.5g} +- {np.sqrt(vo[-1, j]):.2g}; |t| max "
              f"{np.abs(tw[:, j]).max():.2f}")
    assert np.all(vg > 0) and np.all(vo > 0)
    assert np.abs(tw).max() < 5.0, tw
