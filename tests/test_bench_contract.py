"""The benchmark's accounting, checked on the CPU.

* The algorithmic bytes per solve count 3(n-1)/n interior inflow faces per
  (cell, octant) on an n^3 grid; the oracle's own per-octant designation on an
  unjittered grid gives that average exactly.
* The committed counter summaries belong to the committed sweep kernel: their
  recorded source hash is the current one, and the benchmark reads their HBM
  traffic back (a stale summary would make it report null).
* More than one GPU is refused with a message, before any GPU work.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2510_11513_amd import profiling  # noqa: E402


@pytest.mark.parametrize("n", [3, 5])
def test_inflow_faces_per_cell_and_octant(n):
    mesh = inputs.make_mesh(n, 0.0, seed=1)
    rng = np.random.default_rng(1)
    mat = inputs.materials_loguniform_blocks(mesh, 2, rng, 1, 0.0, 0.5)
    o = oracle.Oracle.from_problem(inputs.Problem("grid", mesh, mat, 1, 1, 1e-6))
    inflow = o.dag()["inflow"]                          # [8][C] face bit masks
    interior = ((o.geometry()["nbr"] >= 0) * (1 << np.arange(6))).sum(axis=1)
    count = np.array([[bin(int(m) & int(i)).count("1") for m, i in zip(inflow[q], interior)] for q in range(8)])
    assert count.mean() == pytest.approx(3.0 * (n - 1) / n, abs=1e-12)
    A, A_o, G = 32, 4, 8
    faces = (bench.bytes_per_task(n, A, A_o, G) - 32.0 - 140.0 / A - 120.0 / (A_o * G)) / 16.0
    assert faces == pytest.approx(count.mean(), abs=1e-12)


@pytest.mark.parametrize("workload", ["cfg2", "cfg3"])
def test_counter_summaries_belong_to_the_committed_kernel(workload):
    path = os.path.join(ROOT, "profiles", f"k_sweep_{workload}_pmc.md")
    text = open(path).read()
    assert f"kernel_source_sha256_16: {profiling.kernel_hash()}" in text, \
        "the sweep kernel changed after its counters were taken"
    traffic = bench.measured_traffic(workload)
    assert traffic is not None and traffic > 0
    solves = {"cfg2": 32 ** 3 * 96 * 16, "cfg3": 64 ** 3 * 256 * 64}[workload]
    algorithmic = {"cfg2": bench.bytes_per_task(32, 96, 12, 16), "cfg3": bench.bytes_per_task(64, 256, 32, 64)}
    ratio = traffic / (algorithmic[workload] * solves)
    assert 0.9 < ratio < 1.3, ratio                      # HBM bytes near the algorithmic ones


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
