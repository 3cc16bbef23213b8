"""The LDS staging depth of the first-order sweep (GPU).

Depth 1 requests a continuation task's upwind traces together with its cell
data and a multi-round task's next-round inputs during the current round;
depth 0 requests each at its start.  Only the order of loads changes, so the
bits must not: one-round and multi-round tasks, dependency-driven and
level-synchronous, chained sweeps and a solve.  The tuner searches the depth
and records it in its cache.
"""
import json

import numpy as np
import pytest

from paper_2510_11513_amd import inputs

pytestmark = pytest.mark.gpu


def _problem(n, G, npol, naz, seed):
    rng = np.random.default_rng(seed)
    mesh = inputs.make_mesh(n, 0.2, rng=rng)
    mat = inputs.materials_loguniform_blocks(mesh, G, rng, 2, 0.2, 0.9)
    return inputs.Problem(f"stage_n{n}G{G}", mesh, mat, npol, naz, 1e-6)


@pytest.mark.parametrize("threads,mode", [(192, 0), (64, 0), (64, 1), (128, 0)])
def test_staging_depth_gives_the_same_bits(threads, mode):
    import torch
    from paper_2510_11513_amd import snx
    prob = _problem(8, 12, 2, 3, seed=threads + mode)        # A*G = 72: one round at 192 threads, two at 64
    print(f"[case] staging depth threads={threads} mode={mode} A*G={prob.nang // 8 * prob.mat.ngroup}", flush=True)
    ps = []
    for depth in (1, 0):
        p = snx.Problem.from_problem(prob, setup=False)
        p.set_schedule(threads=threads)
        p.set_staging_depth(depth)
        p.setup()
        p.set_sweep_mode(mode)
        assert p.staging_depth() == depth
        ps.append(p)
    rng = np.random.default_rng(5)
    phi = torch.from_numpy(rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, 8)).astype(np.float32)).cuda()
    for _ in range(3):
        outs = [p.sweep(phi) for p in ps]
        torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1])
        phi = outs[0]
    sols = [p.solve(1e-6, 500)[0] for p in ps]
    assert torch.equal(sols[0], sols[1])
    with pytest.raises(snx.SnxError):
        ps[0].set_staging_depth(2)
    for p in ps:
        p.close()


def test_tuner_searches_and_caches_the_staging_depth(tmp_path):
    from paper_2510_11513_amd import snx
    prob = _problem(6, 16, 2, 2, seed=9)
    p = snx.Problem.from_problem(prob)
    cache = tmp_path / "tune.jsonl"
    p.tune(cache)
    d = p.staging_depth()
    assert d in (0, 1)
    rec = json.loads(cache.read_text().strip().splitlines()[-1])
    assert rec["depth"] == d and rec["threads"] == p.schedule()["threads"]
    q = snx.Problem.from_problem(prob)                       # a cache hit restores the depth
    q.set_staging_depth(1 - d)
    q.tune(cache)
    assert q.staging_depth() == d
    p.close()
    q.close()


def test_batch_staging_depth_gives_the_same_bits():
    import torch
    from paper_2510_11513_amd import snx
    probs = [_problem(5, 24, 2, 2, seed=21), _problem(6, 8, 2, 3, seed=22)]   # A*G 96 and 48: multi-round at 64
    outs = []
    for depth in (1, 0):
        ps = [snx.Problem.from_problem(pr) for pr in probs]
        b = snx.Batch(ps)
        b.set_schedule(threads=64)
        b.set_staging_depth(depth)
        rng = np.random.default_rng(3)
        pin = [torch.from_numpy(rng.uniform(0, 2, (pr.mesh.ncell, pr.mat.ngroup, 8)).astype(np.float32)).cuda()
               for pr in probs]
        outs.append([o.clone() for o in b.sweep(pin)])
        torch.cuda.synchronize()
        assert b.stats()["abort"] == 0
        with pytest.raises(snx.SnxError):
            b.set_staging_depth(-1)
    for a, c in zip(*outs):
        assert torch.equal(a, c)
