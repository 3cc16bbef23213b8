"""The sweep watchdog's abort path, forced from the host (GPU).

A tiny wall-clock limit (snx_set_watchdog) makes the first workgroup that
finds no ready task set the abort flag; every other one leaves at its next
check, so the kernel ends normally with the sweep unfinished.  sweep_stats
reports the abort once and re-arms the counters and queues, a solve under the
tiny limit raises SNX_E_DEVICE, and with the default limit restored the next
sweeps give the level-synchronous comparator's bits again.  Covered for the
octant task sweep and for the per-direction unit sweep (on an unjittered mesh,
which lags no face, so no sweep reads the aborted sweep's angular flux).
"""
import numpy as np
import pytest

from paper_2510_11513_amd import inputs

pytestmark = pytest.mark.gpu


def _problem(designation):
    if designation == 0:
        return inputs.config_problem(1)
    rng = np.random.default_rng(3)
    mesh = inputs.make_mesh(6, 0.0, rng=rng)
    mat = inputs.materials_loguniform_blocks(mesh, 5, rng, 2, 0.2, 0.9)
    return inputs.Problem("flat6", mesh, mat, 2, 3, 1e-6)


@pytest.mark.parametrize("designation", [0, 2])
def test_watchdog_abort_is_reported_rearmed_and_recovered(designation):
    import torch
    from paper_2510_11513_amd import snx
    prob = _problem(designation)
    print(f"[case] watchdog abort designation={designation} C={prob.mesh.ncell} nang={prob.nang} "
          f"G={prob.mat.ngroup}", flush=True)
    p = snx.Problem.from_problem(prob, designation=designation)
    p.set_sweep_mode(snx.SWEEP_AMT)
    ref = snx.Problem.from_problem(prob, designation=designation)
    ref.set_sweep_mode(snx.SWEEP_BSP)
    if designation == 2:
        assert p.designation_stats()["lagged"] == 0
    rng = np.random.default_rng(11)
    phi = torch.from_numpy(rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, 8)).astype(np.float32)).cuda()
    want = ref.sweep(phi)

    p.set_watchdog(1e-9)                          # any wait for a ready task aborts
    p.sweep(phi)
    torch.cuda.synchronize()
    assert p.sweep_stats()["abort"] == 1
    assert p.sweep_stats()["abort"] == 0          # reported once; the schedule is re-armed
    with pytest.raises(snx.SnxError) as e:
        p.solve(1e-6, 40)
    assert e.value.code == -5, e.value

    p.set_watchdog(0.0)                           # the default limit again
    for _ in range(3):
        got = p.sweep(phi)
        torch.cuda.synchronize()
        assert p.sweep_stats()["abort"] == 0
        assert torch.equal(got, want)
    phi_a, ia = p.solve(1e-6, 400)
    phi_b, ib = ref.solve(1e-6, 400)
    assert ia["iterations"] == ib["iterations"] and torch.equal(phi_a, phi_b)
    with pytest.raises(snx.SnxError):
        p.set_watchdog(float("nan"))
    print(f"[case] watchdog designation={designation}: abort reported, re-armed, bits recovered", flush=True)
    p.close()
    ref.close()
