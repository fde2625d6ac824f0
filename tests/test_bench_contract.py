"""The measurement script's contract, checked on the CPU: one GPU only, the
algorithmic bytes each phase is priced at, and the workload it reports."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


@pytest.mark.parametrize("m_bytes,expect", [
    (8, {"potential": 24, "relax": 42.8, "orbit": 60, "sort": 72}),
    (4, {"potential": 20, "relax": 38.8, "orbit": 60, "sort": 64}),
])
def test_algorithmic_bytes(m_bytes, expect):
    """Read r, m and write phi; read m, vr, vt, half an id and two bin edges
    per 20 stars, write vr, vt; read r, phi, vr, vt, id and write r_new, vr,
    vt; read and write the record r, vr, vt, m, id."""
    got = bench.alg_bytes(m_bytes)
    assert set(got) == set(expect)
    for k, v in expect.items():
        assert got[k] == pytest.approx(v), k
    assert sum(got.values()) == pytest.approx(198.8 if m_bytes == 8 else 182.8)


def test_default_workload():
    wl = bench.WORKLOADS[bench.DEFAULT_WORKLOAD]
    assert wl["n"] == 10_000_000 and wl["precision"] == "mixed" and wl["m_f32"]
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.PHASES == ("potential", "timestep", "relax", "orbit", "sort")


def test_sources_hash_is_stable():
    assert bench.sources_sha256() == bench.sources_sha256()
    assert len(bench.sources_sha256()) == 64
