"""Reflective boundary planes on the GPU vs the FP64 oracle (through the C ABI).

A reflective face's inflow is the mirror image's outflow at the same nodes,
from the previous sweep: the GPU keeps it as problem state (zero after setup),
the oracle reads it from the previous sweep's angular flux.  Chained sweeps
are compared sweep by sweep, then converged solves, the balance and the
combination with per-angle designation and group coupling.

Tolerance: 1e-5 relative per group on the scalar flux.
"""
import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _problem(n, G, npol, naz, seed, kind=0, c=(0.2, 0.8), jitter=0.2):
    rng = np.random.default_rng(seed)
    mesh = inputs.make_mesh(n, jitter, rng=rng)
    mat = inputs.materials_loguniform_blocks(mesh, G, rng, 2, c[0], c[1])
    prob = inputs.Problem(f"refl_n{n}G{G}", mesh, mat, npol, naz, 1e-6)
    if kind == 1:
        prob.boundary_kind = 1
        prob.psi_b = rng.uniform(0.1, 1.0, G)
    return prob


def _pair(prob, planes, designation=0, threads=None, mode=None, groups=False):
    from paper_2510_11513_amd import snx
    p = snx.Problem.from_problem(prob, setup=False, designation=designation)
    p.set_reflective(planes)
    o = oracle.Oracle.from_problem(prob, setup=False, designation=designation)
    o.set_reflective(planes)
    if groups:
        cm, sgg = inputs.split_scattering(prob.mat)
        p.set_group_scattering(cm, sgg)
        o.set_group_scattering(cm, sgg)
    if threads:
        p.set_schedule(threads=threads)
    p.setup()
    o.setup()
    if mode is not None:
        p.set_sweep_mode(mode)
    return p, o


def _phi_in(prob, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, 8)).astype(np.float32)


CASES = {
    "x0_plane": (lambda: _problem(4, 3, 2, 2, seed=1), 0b000001, None),
    "all_six_planes": (lambda: _problem(4, 4, 1, 3, seed=2), 0b111111, None),
    "three_planes_with_inflow": (lambda: _problem(5, 5, 2, 3, seed=3, kind=1), 0b101010, None),
    "multi_round_threads64": (lambda: _problem(4, 16, 3, 4, seed=4), 0b010101, 64),
}


def _chain(p, phi32, k):
    torch = _torch()
    pin = torch.from_numpy(phi32).cuda()
    outs = []
    for _ in range(k):
        out = p.sweep(pin)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy().astype(np.float64))
    return outs


@pytest.mark.parametrize("name", list(CASES))
def test_chained_sweeps_match_the_oracle(name):
    make, planes, threads = CASES[name]
    prob = make()
    print(f"[case] reflective {name}: C={prob.mesh.ncell} G={prob.mat.ngroup} nang={prob.nang} "
          f"planes={planes:06b} threads={threads}", flush=True)
    p, o = _pair(prob, planes, threads=threads)
    phi32 = _phi_in(prob, 7)
    outs = _chain(p, phi32, 3)
    st = p.sweep_stats()
    assert st["abort"] == 0 and st["tasks"] == 8 * prob.mesh.ncell, st
    prev = None
    for k in range(3):
        r = o.sweep(phi32.astype(np.float64), want_psi=True, psi_prev=prev)
        err = H.rel_err_per_group(outs[k], r["phi"])
        print(f"[case] sweep {k}: phi max rel err {err.max():.2e}", flush=True)
        assert err.max() <= TOL, (k, err)
        prev = r["psi"]
    assert np.abs(outs[1] - outs[0]).max() > 1e-4 * np.abs(outs[0]).max()   # the reflected inflow enters
    p.close()


def test_bulk_synchronous_mode_gives_the_same_bits():
    from paper_2510_11513_amd import snx
    prob = _problem(4, 3, 2, 2, seed=5)
    phi32 = _phi_in(prob, 8)
    pa, _ = _pair(prob, 0b110011)
    pb, _ = _pair(prob, 0b110011, mode=snx.SWEEP_BSP)
    for x, y in zip(_chain(pa, phi32, 3), _chain(pb, phi32, 3)):
        assert np.array_equal(x, y)


def test_converged_solution_and_balance():
    torch = _torch()
    prob = _problem(4, 3, 2, 2, seed=6, c=(0.2, 0.6))
    p, o = _pair(prob, 0b000111)
    phi, info = p.solve(1e-6, 3000)
    assert info["status"] == 0, info
    ref = o.solve(1e-12, 5000)
    err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
    print(f"[case] reflective solve: iterations gpu {info['iterations']} oracle {ref['iters']}, "
          f"rel err {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    # balance of one more sweep: the reflected inflow it used is counted
    phi32 = phi.clone()
    out = p.sweep(phi32)
    b = p.balance(phi32, out)
    assert b[:, 3].max() < 1e-4, b
    assert np.abs(b[:, 0] - b[:, 1] - b[:, 2]).max() <= 1e-5 * np.abs(b[:, 0]).max()
    p.close()


@pytest.mark.parametrize("planes", [0b101010, 0b000111])
def test_converged_solution_matches_the_oracle_with_octants_in_sequence(planes):
    """The paper's order: octants in sequence, reflected inflow from the current
    sweep where the mirrored octant came earlier (Section 2.1 and its footnote).
    The GPU runs the octants concurrently with every reflected inflow lagged a
    sweep; both iterations have the same fixed point."""
    prob = _problem(4, 3, 2, 2, seed=16, c=(0.2, 0.6))
    p, _ = _pair(prob, planes)
    phi, info = p.solve(1e-6, 3000)
    assert info["status"] == 0, info
    o = oracle.Oracle.from_problem(prob, setup=False)
    o.set_reflective(planes)
    o.set_octant_order(True)
    o.setup()
    ref = o.solve(1e-12, 5000)
    err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
    print(f"[case] reflective planes {planes:06b}, oracle octants in sequence: iterations gpu "
          f"{info['iterations']} oracle {ref['iters']}, rel err {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    p.close()


def test_per_angle_designation_with_group_coupling_and_reflection():
    prob = _problem(4, 5, 2, 3, seed=9, kind=1, jitter=0.3)
    p, o = _pair(prob, 0b001001, designation=1, groups=True)
    phi, info = p.solve_outer(5, 5, 0.0)
    ref = o.solve_outer(5, 5, 0.0)
    err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
    print(f"[case] per-angle + groups + reflective 5x5: rel err {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    p.close()


def test_batch_with_a_reflective_problem():
    torch = _torch()
    from paper_2510_11513_amd import snx
    probs = [_problem(4, 3, 2, 2, seed=10), _problem(3, 4, 1, 2, seed=11)]
    planes = [0b000011, 0]
    gp = []
    for pr, pl in zip(probs, planes):
        q = snx.Problem.from_problem(pr, setup=False)
        q.set_reflective(pl)
        q.setup()
        gp.append(q)
    batch = snx.Batch(gp)
    phis = [_phi_in(pr, 30 + i) for i, pr in enumerate(probs)]
    prev = [None, None]
    for k in range(3):
        outs = batch.sweep([torch.from_numpy(x).cuda() for x in phis])
        torch.cuda.synchronize()
        for i, pr in enumerate(probs):
            o = oracle.Oracle.from_problem(pr, setup=False)
            o.set_reflective(planes[i])
            o.setup()
            r = o.sweep(phis[i].astype(np.float64), want_psi=True, psi_prev=prev[i])
            prev[i] = r["psi"]
            err = H.rel_err_per_group(outs[i].cpu().numpy().astype(np.float64), r["phi"])
            assert err.max() <= TOL, (k, i, err)
    batch.close()
    for q in gp:
        q.close()


def test_asymmetric_quadrature_is_refused():
    from paper_2510_11513_amd import snx
    prob = _problem(2, 1, 1, 2, seed=12)
    om, w = snx.quadrature_product(1, 2)
    om = om.copy()
    t = 0.05
    x, y = om[0, 0], om[0, 1]
    om[0, 0], om[0, 1] = np.cos(t) * x - np.sin(t) * y, np.sin(t) * x + np.cos(t) * y
    p = snx.Problem.from_problem(prob, setup=False, quadrature=(om, w))
    p.set_reflective(1)
    with pytest.raises(snx.SnxError):
        p.setup()
    p.close()
