"""Group-to-group scattering and inner/outer iterations on the GPU vs the FP64
oracle (through the C ABI).

With a group-to-group matrix, a sweep takes its whole scattering source from
phi_in, one Jacobi step over groups.  snx_solve_outer runs the paper's
benchmark structure (five inner and five outer iterations, Section 3.6): each
outer iteration fixes the cross-group source from its starting flux.

Tolerance: 1e-5 relative per group on the scalar flux (the cross-group sums
run in FP32 on the GPU and in FP64 in the oracle).
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


def _problem(n, G, npol, naz, seed, kind=0, block=2, c=(0.3, 0.95)):
    rng = np.random.default_rng(seed)
    mesh = inputs.make_mesh(n, 0.2, rng=rng)
    mat = inputs.materials_loguniform_blocks(mesh, G, rng, block, c[0], c[1])
    prob = inputs.Problem(f"gs_n{n}G{G}", mesh, mat, npol, naz, 1e-6)
    if kind == 1:
        prob.boundary_kind = 1
        prob.psi_b = rng.uniform(0.1, 1.0, G)
    return prob


def _pair(prob, designation=0, within=0.6, threads=None):
    from paper_2510_11513_amd import snx
    cm, sgg = inputs.split_scattering(prob.mat, within)
    p = snx.Problem.from_problem(prob, setup=False, designation=designation)
    p.set_group_scattering(cm, sgg)
    if threads:
        p.set_schedule(threads=threads)
    p.setup()
    o = oracle.Oracle.from_problem(prob, setup=False, designation=designation)
    o.set_group_scattering(cm, sgg)
    o.setup()
    return p, o, sgg.shape[0]


def _phi_in(prob, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, 8)).astype(np.float32)


CASES = {
    "n4_G5_multi_material": (lambda: _problem(4, 5, 2, 2, seed=1), None),
    "n5_G16_inflow": (lambda: _problem(5, 16, 1, 3, seed=2, kind=1), None),
    "n4_G16_multi_round": (lambda: _problem(4, 16, 3, 4, seed=3), 64),
}


@pytest.mark.parametrize("name", list(CASES))
def test_one_sweep_with_the_coupled_source(name):
    torch = _torch()
    make, threads = CASES[name]
    prob = make()
    p, o, nmat = _pair(prob, threads=threads)
    print(f"[case] group scattering {name}: C={prob.mesh.ncell} G={prob.mat.ngroup} nang={prob.nang} "
          f"materials={nmat}", flush=True)
    phi32 = _phi_in(prob, 5)
    out = p.sweep(torch.from_numpy(phi32).cuda())
    torch.cuda.synchronize()
    ref = o.sweep(phi32.astype(np.float64), want_leak=True)
    err = H.rel_err_per_group(out.cpu().numpy().astype(np.float64), ref["phi"])
    print(f"[case] sweep phi max rel err {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    # balance counts the cross-group source
    b = p.balance(torch.from_numpy(phi32).cuda(), out)
    bo = o.balance(phi32.astype(np.float64), ref["phi"], ref["leak"])
    assert np.abs(b[:, 0] - bo[:, 0]).max() <= 1e-5 * np.abs(bo[:, 0]).max()
    p.close()


@pytest.mark.parametrize("designation", [0, 1])
def test_five_outer_five_inner_iterations(designation):
    prob = _problem(4, 6, 2, 3, seed=4, kind=1)
    p, o, _ = _pair(prob, designation=designation)
    phi, info = p.solve_outer(5, 5, 0.0)
    assert info["iterations"] == 25 and info["status"] == 0, info
    ref = o.solve_outer(5, 5, 0.0)
    assert ref["inners"] == 25
    err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
    print(f"[case] 5x5 designation {designation}: rel err {err.max():.2e}, outer change gpu "
          f"{info['residual']:.3e} oracle {ref['eps']:.3e}", flush=True)
    assert err.max() <= TOL, err
    assert abs(info["residual"] - ref["eps"]) <= 1e-3 * ref["eps"] + 1e-6
    p.close()


def test_converged_outer_iteration_and_plain_solve():
    # scattering ratios <= 0.7: a change of 1e-6 (the workloads' tolerance; FP32
    # iterates stop changing near 1e-7) leaves an error of a few 1e-6
    prob = _problem(4, 4, 2, 2, seed=6, c=(0.2, 0.7))
    p, o, _ = _pair(prob, within=0.3)
    phi_o, info_o = p.solve_outer(200, 3, 1e-6)
    phi_j, info_j = p.solve(1e-6, 600)
    ref = o.solve_outer(400, 3, 1e-12)
    assert info_o["status"] == 0 and info_j["status"] == 0 and ref["status"] == 0
    for name, phi in (("outer", phi_o), ("jacobi", phi_j)):
        err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
        print(f"[case] converged {name}: rel err {err.max():.2e}", flush=True)
        assert err.max() <= TOL, (name, err)
    p.close()


def test_batch_with_group_matrices():
    """Two coupled problems and a plain one in one batch: a sweep with the
    coupled sources, five outer x five inner iterations, and a converged outer
    solve in which each problem retires on its own tolerance."""
    torch = _torch()
    from paper_2510_11513_amd import snx
    c = (0.2, 0.7)      # a change of 1e-6 then bounds the error by a few 1e-6 (FP32 iterates)
    probs = [_problem(4, 5, 2, 2, seed=70, c=c), _problem(3, 3, 1, 2, seed=71, kind=1, c=c),
             _problem(4, 4, 2, 2, seed=72, c=c)]
    coupled = [True, True, False]
    gp, ors = [], []
    for pr, cpl in zip(probs, coupled):
        q = snx.Problem.from_problem(pr, setup=False)
        o = oracle.Oracle.from_problem(pr, setup=False)
        if cpl:
            cm, sgg = inputs.split_scattering(pr.mat, 0.4)
            q.set_group_scattering(cm, sgg)
            o.set_group_scattering(cm, sgg)
        q.setup()
        o.setup()
        gp.append(q)
        ors.append(o)
    batch = snx.Batch(gp)
    phis = [_phi_in(pr, 80 + i) for i, pr in enumerate(probs)]
    outs = batch.sweep([torch.from_numpy(x).cuda() for x in phis])
    torch.cuda.synchronize()
    for i, o in enumerate(ors):
        err = H.rel_err_per_group(outs[i].cpu().numpy().astype(np.float64), o.sweep(phis[i].astype(np.float64))["phi"])
        assert err.max() <= TOL, ("sweep", i, err)
    res, infos, _ = batch.solve_outer(5, 5, 0.0)
    for i, o in enumerate(ors):
        ref = o.solve_outer(5, 5, 0.0)
        err = H.rel_err_per_group(res[i].cpu().numpy().astype(np.float64), ref["phi"])
        print(f"[case] batch 5x5 problem {i}: rel err {err.max():.2e}", flush=True)
        assert infos[i]["iterations"] == 25 and err.max() <= TOL, (i, err)
    res, infos, rc = batch.solve_outer(300, 3, 1e-6)
    assert rc == 0, infos
    for i, o in enumerate(ors):
        ref = o.solve_outer(600, 3, 1e-12)
        err = H.rel_err_per_group(res[i].cpu().numpy().astype(np.float64), ref["phi"])
        print(f"[case] batch converged problem {i}: {infos[i]['iterations']} inner iterations, rel err {err.max():.2e}",
              flush=True)
        assert infos[i]["status"] == 0 and err.max() <= TOL, (i, err)
    batch.close()
    for q in gp:
        q.close()


def test_plain_solve_iterates_across_graph_replays():
    """snx_solve renews the cross-group source after every sweep inside its
    graph replays: a fixed number of iterations that crosses replay boundaries
    equals the oracle's source iteration iterate for iterate, before and after
    an outer solve (which keeps the source fixed within its inner iterations),
    for one problem and for a batch with a plain problem beside the coupled
    one."""
    torch = _torch()
    from paper_2510_11513_amd import snx
    prob = _problem(4, 5, 2, 2, seed=90, kind=1)
    p, o, _ = _pair(prob, within=0.4)
    phi0 = _phi_in(prob, 91)
    for k in (1, 11):
        for when in ("before", "after"):
            if when == "after":
                p.solve_outer(2, 3, 0.0)
            phi, info = p.solve(0.0, k, phi0=torch.from_numpy(phi0).cuda(), allow_noconv=True)
            assert info["iterations"] == k, info
            ref = o.solve(0.0, k, phi0=phi0.astype(np.float64), allow_noconv=True)
            err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
            print(f"[case] plain coupled solve, {k} iterations, {when} an outer solve: rel err {err.max():.2e}",
                  flush=True)
            assert err.max() <= TOL, (k, when, err)
    # the oracle's plain source iteration is one inner iteration per outer
    a = o.solve(0.0, 11, phi0=phi0.astype(np.float64), allow_noconv=True)["phi"]
    b = o.solve_outer(11, 1, 0.0, phi0=phi0.astype(np.float64), allow_noconv=True)["phi"]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    p.close()

    probs = [_problem(4, 5, 2, 2, seed=92), _problem(3, 4, 1, 2, seed=93)]
    gp, ors = [], []
    for i, pr in enumerate(probs):
        q = snx.Problem.from_problem(pr, setup=False)
        r = oracle.Oracle.from_problem(pr, setup=False)
        if i == 0:
            cm, sgg = inputs.split_scattering(pr.mat, 0.4)
            q.set_group_scattering(cm, sgg)
            r.set_group_scattering(cm, sgg)
        q.setup()
        r.setup()
        gp.append(q)
        ors.append(r)
    batch = snx.Batch(gp)
    phis = [_phi_in(pr, 94 + i) for i, pr in enumerate(probs)]
    res, infos, _ = batch.solve(0.0, 11, phi0=[torch.from_numpy(x).cuda() for x in phis], allow_noconv=True)
    for i, r in enumerate(ors):
        ref = r.solve(0.0, 11, phi0=phis[i].astype(np.float64), allow_noconv=True)
        err = H.rel_err_per_group(res[i].cpu().numpy().astype(np.float64), ref["phi"])
        print(f"[case] batch plain solve problem {i}: rel err {err.max():.2e}", flush=True)
        assert infos[i]["iterations"] == 11 and err.max() <= TOL, (i, err)
    batch.close()
    for q in gp:
        q.close()
