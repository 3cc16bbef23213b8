"""Batched problems in one persistent launch, and the schedule autotuner (GPU)."""
import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _uneven(count=5, seed=0):
    """Small uneven instances of the batch recipe: mesh edge, groups and quadrature all differ."""
    rng = np.random.default_rng(seed)
    shapes = [(3, 4, 1, 1), (4, 13, 2, 2), (5, 5, 2, 4), (2, 32, 3, 4), (6, 16, 4, 4), (4, 1, 1, 2), (3, 64, 1, 1)]
    out = []
    for i in range(count):
        n, G, npol, naz = shapes[i % len(shapes)]
        mesh = inputs.make_mesh(n, 0.2, rng=rng)
        mat = inputs.materials_two_block(mesh, G, rng, 2, scaled=True)
        out.append(inputs.Problem(f"b{i}", mesh, mat, npol, naz, 1e-6))
    return out


def _setup(probs):
    from paper_2510_11513_amd import snx
    return [snx.Problem.from_problem(pr) for pr in probs]


def test_batch_sweep_matches_single_sweeps_and_oracle():
    import torch
    from paper_2510_11513_amd import snx
    probs = _uneven(7, seed=1)
    gp = _setup(probs)
    batch = snx.Batch(gp)
    rng = np.random.default_rng(2)
    phis = [rng.uniform(0, 2, (pr.mesh.ncell, pr.mat.ngroup, 8)).astype(np.float32) for pr in probs]
    pin = [torch.from_numpy(x).cuda() for x in phis]
    out_b = [o.cpu().numpy() for o in batch.sweep(pin)]
    st = batch.stats()
    assert st["abort"] == 0 and st["tasks"] == sum(8 * pr.mesh.ncell for pr in probs), st
    for i, (pr, p) in enumerate(zip(probs, gp)):
        single = p.sweep(pin[i]).cpu().numpy()
        assert np.array_equal(single, out_b[i]), f"problem {i}: batch and single sweeps differ"
        ref = oracle.Oracle.from_problem(pr).sweep(phis[i].astype(np.float64))["phi"]
        assert H.rel_err_per_group(out_b[i].astype(np.float64), ref).max() <= TOL, i


def test_batch_solve_retires_converged_problems():
    from paper_2510_11513_amd import snx
    probs = _uneven(5, seed=3)
    gp = _setup(probs)
    batch = snx.Batch(gp)
    batch.set_schedule(chunk=4)
    phi, infos, rc = batch.solve(1e-6, 400)
    assert rc == 0
    iters = [inf["iterations"] for inf in infos]
    for i, (pr, p) in enumerate(zip(probs, gp)):
        solo, info = p.solve(1e-6, 400)
        assert info["iterations"] == iters[i], (i, info["iterations"], iters[i])
        assert np.array_equal(solo.cpu().numpy(), phi[i].cpu().numpy()), i
        ref = oracle.Oracle.from_problem(pr).solve(1e-12, 2000)
        assert H.rel_err_per_group(phi[i].cpu().numpy().astype(np.float64), ref["phi"]).max() <= TOL, i
    assert len(set(iters)) > 1        # the instances converge at different iterations


def test_batch_of_one_equals_problem_and_single_path_still_consistent():
    import torch
    from paper_2510_11513_amd import snx
    pr = inputs.config_problem(2, n=5)
    p = _setup([pr])[0]
    b = snx.Batch([p])
    x = torch.rand((pr.mesh.ncell, pr.mat.ngroup, 8), device="cuda")
    ob = b.sweep([x])[0].cpu().numpy()
    os_ = p.sweep(x).cpu().numpy()        # counters stay consistent across both schedules
    assert np.array_equal(ob, os_)
    ob2 = b.sweep([x])[0].cpu().numpy()
    assert np.array_equal(ob, ob2)


def test_tuner_picks_a_valid_schedule_and_caches(tmp_path):
    import torch
    from paper_2510_11513_amd import snx
    probs = _uneven(3, seed=5)
    gp = _setup(probs)
    batch = snx.Batch(gp)
    cache = tmp_path / "tune.jsonl"
    t, w = batch.tune(cache)
    assert t in (64, 128, 192, 256, 512) and t >= max(pr.mat.ngroup for pr in probs)
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and '"threads": %d' % t in lines[0]
    assert batch.tune(cache) == (t, w)                   # cache hit: same choice, no new line
    assert len(cache.read_text().strip().splitlines()) == 1
    x = [torch.rand((pr.mesh.ncell, pr.mat.ngroup, 8), device="cuda") for pr in probs]
    out = batch.sweep(x)
    for i, pr in enumerate(probs):
        ref = oracle.Oracle.from_problem(pr).sweep(x[i].cpu().numpy().astype(np.float64))["phi"]
        assert H.rel_err_per_group(out[i].cpu().numpy().astype(np.float64), ref).max() <= TOL
    t1, w1 = gp[0].tune(tmp_path / "single.jsonl")
    assert t1 >= probs[0].mat.ngroup
    sch = gp[0].schedule()        # the tuner also picks the sweep mode
    assert sch["threads"] == t1 and sch["mode"] in (snx.SWEEP_AMT, snx.SWEEP_BSP)


def test_batch_rejects_unready_problem():
    from paper_2510_11513_amd import snx
    pr = inputs.config_problem(1, n=3)
    p = snx.Problem.from_problem(pr, setup=False)
    with pytest.raises(snx.SnxError) as e:
        snx.Batch([p])
    assert e.value.code == -2


def test_batch_bulk_synchronous_solve_equals_dependency_driven():
    from paper_2510_11513_amd import snx
    probs = _uneven(4, seed=11)
    gp = _setup(probs)
    batch = snx.Batch(gp)
    batch.set_schedule(chunk=3)
    phi_a, inf_a, _ = batch.solve(1e-6, 300)
    batch.set_sweep_mode(snx.SWEEP_BSP)
    phi_b, inf_b, _ = batch.solve(1e-6, 300)
    for i in range(len(probs)):
        assert inf_a[i]["iterations"] == inf_b[i]["iterations"], i
        assert np.array_equal(phi_a[i].cpu().numpy(), phi_b[i].cpu().numpy()), i
