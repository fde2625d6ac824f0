"""A free-running FP64 GPU trajectory inside the oracle's seed ensemble.

N = 1e5 equal-mass Plummer, ln(0.11 N), 100 steps.  The oracle runs 8
independent trajectories (initial model and step draws from seeds 2..9)
and the GPU one more (seed 1).  Every step redraws every orbit, so
trajectories decorrelate within a few steps and only their statistics can
be compared: after steps 10, 20, ..., 100 the GPU's relative energy change
(E - E0)/|E0|, virial ratio 2T/|W| and 10/50/90 % Lagrange radii must lie
within the band of the 8 oracle runs, mean +- 5 sample standard deviations
(times sqrt(1 + 1/8) for a new draw against an estimated mean; |t| > 5 at
7 degrees of freedom has probability 0.0016).  The paper compares runs the
same way, by their statistics (Sec. 4.1)."""
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


def test_gpu_trajectory_inside_oracle_seed_band(cmc, ora):
    seeds = list(range(2, 10))
    out = {}
    # the oracle is plain C behind ctypes, which releases the GIL: the 8
    # trajectories run on 8 host cores at once
    th = [threading.Thread(target=oracle_track, args=(ora, s, out)) for s in seeds]
    for t in th:
        t.start()
    cl = cmc.Cluster(N)
    cmc.cmc_init_plummer(cl, N, 1, 0)
    cmc.cmc_potential(cl)
    e0 = float(cmc.cmc_diagnostics(cl)["E"])
    gpu = []
    for k in range(STEPS):
        cmc.cmc_step(cl, cmc.Params(seed=1, step=k, gamma=GAMMA))
        if k % 10 == 9:
            cmc.cmc_potential(cl)
            gpu.append(sample(cmc.cmc_diagnostics(cl), e0))
    gpu = np.array(gpu)
    for t in th:
        t.join()
    band = np.stack([out[s] for s in seeds])          # (seeds, samples, keys)
    mean, sd = band.mean(axis=0), band.std(axis=0, ddof=1)
    z = (gpu - mean) / (sd * np.sqrt(1.0 + 1.0 / len(seeds)))
    for j, key in enumerate(KEYS):
        print(f"{key}: gpu {gpu[-1, j]:.5g}, oracle band {mean[-1, j]:.5g} +- "
              f"{sd[-1, j]:.2g} (step 100); |z| max {np.abs(z[:, j]).max():.2f}")
    assert np.all(sd > 0)
    assert np.abs(z).max() < 5.0, z
