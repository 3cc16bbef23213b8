"""GPU sweep vs the FP64 oracle, element by element, through the C ABI.

Tolerance: the FP32 sweep must match the FP64 oracle to 1e-5 relative on the
scalar flux, per group: max_K,d |phi_gpu - phi_oracle| / max_K,d |phi_oracle|.
Integer outputs (t-levels) must match exactly.
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


def _gpu(prob, threads=None):
    from paper_2510_11513_amd import snx
    p = snx.Problem.from_problem(prob, setup=False)
    if threads:
        p.set_schedule(threads=threads)
    p.setup()
    return p


def _phi_in(prob, seed=0):
    """Same FP32 input flux for both sides."""
    rng = np.random.default_rng(seed)
    C, G = prob.mesh.ncell, prob.mat.ngroup
    phi = rng.uniform(0.0, 2.0, (C, G, 8)).astype(np.float32)
    return phi


def _sweep_pair(prob, phi32, threads=None):
    torch = _torch()
    p = _gpu(prob, threads)
    pin = torch.from_numpy(phi32).cuda()
    out = p.sweep(pin)
    torch.cuda.synchronize()
    st = p.sweep_stats()
    assert st["abort"] == 0, st
    assert st["tasks"] == 8 * prob.mesh.ncell, st
    o = oracle.Oracle.from_problem(prob)
    ref = o.sweep(phi32.astype(np.float64))["phi"]
    return out.cpu().numpy().astype(np.float64), ref, p, o


CASES = {
    "cfg1": lambda: inputs.config_problem(1),
    "cfg1_ragged5": lambda: inputs.config_problem(1, n=5),
    "cfg2_recipe_n6": lambda: inputs.config_problem(2, n=6),
    "cfg3_recipe_n5": lambda: inputs.config_problem(3, n=5),
    "cfg5_recipe_n4": lambda: inputs.config_problem(5, n=4),
    "paper16_recipe_n4": lambda: inputs.config_problem(0, n=4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_single_sweep_parity(name):
    prob = CASES[name]()
    print(f"[case] {name}: C={prob.mesh.ncell} G={prob.mat.ngroup} nang={prob.nang}", flush=True)
    got, ref, _, _ = _sweep_pair(prob, _phi_in(prob))
    err = H.rel_err_per_group(got, ref)
    assert err.max() <= TOL, err


def _custom(n, G, npol, naz, seed, jitter=0.2, kind=0):
    rng = np.random.default_rng(seed)
    mesh = inputs.make_mesh(n, jitter, rng=rng)
    mat = inputs.materials_loguniform_blocks(mesh, G, rng, 2, 0.0, 0.95)
    prob = inputs.Problem(f"n{n}G{G}", mesh, mat, npol, naz, 1e-6)
    if kind == 1:
        prob.boundary_kind = 1
        prob.psi_b = rng.uniform(0.1, 1.0, G)
    return prob


@pytest.mark.parametrize("n,G,npol,naz,kind", [
    (1, 1, 1, 1, 0),      # single cell, one group, one angle per octant
    (1, 3, 2, 2, 1),      # single cell with inflow
    (2, 13, 1, 3, 0),     # odd group count
    (3, 64, 1, 1, 1),     # G = 64 with one angle per octant
    (4, 5, 3, 3, 1),      # ragged lane rounds
    (3, 100, 2, 2, 0),    # G > 64
])
def test_edge_shapes(n, G, npol, naz, kind):
    prob = _custom(n, G, npol, naz, seed=100 + n * G, kind=kind)
    print(f"[case] edge n={n} G={G} quad={npol}x{naz} kind={kind}", flush=True)
    got, ref, _, _ = _sweep_pair(prob, _phi_in(prob, 3))
    assert H.rel_err_per_group(got, ref).max() <= TOL


@pytest.mark.parametrize("threads", [64, 128, 192, 256, 512])
def test_schedule_does_not_change_bits(threads):
    prob = inputs.config_problem(2, n=5)
    phi32 = _phi_in(prob, 7)
    got, ref, _, _ = _sweep_pair(prob, phi32, threads=threads)
    base, _, _, _ = _sweep_pair(prob, phi32, threads=64)
    assert np.array_equal(got, base)
    assert H.rel_err_per_group(got, ref).max() <= TOL


def test_run_to_run_bitwise_determinism():
    torch = _torch()
    prob = inputs.config_problem(2, n=8)
    p = _gpu(prob)
    pin = torch.from_numpy(_phi_in(prob, 1)).cuda()
    outs = [p.sweep(pin).cpu().numpy() for _ in range(4)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_levels_match_oracle_exactly():
    prob = inputs.config_problem(2, n=9)
    p = _gpu(prob)
    lev, nl = p.levels()
    d = oracle.Oracle.from_problem(prob).dag()
    assert np.array_equal(lev, d["level"])
    assert nl.tolist() == [3 * 9 - 2] * 8


def test_constant_solution_absorber():
    torch = _torch()
    rng = np.random.default_rng(4)
    mesh = inputs.make_mesh(6, 0.2, rng=rng)
    G = 4
    st = np.array([0.3, 1.0, 3.0, 9.0])
    mat = inputs.Materials(np.tile(st, (mesh.ncell, 1)), np.zeros((mesh.ncell, G)), np.ones((mesh.ncell, G)))
    prob = inputs.Problem("const", mesh, mat, 2, 3, 1e-6, 1, 1.0 / (4 * np.pi * st))
    p = _gpu(prob)
    out = p.sweep(None).cpu().numpy()
    want = (1.0 / st)[None, :, None]
    assert np.abs(out / want - 1).max() < 2e-6


def test_solve_converges_to_oracle():
    torch = _torch()
    prob = inputs.config_problem(1)          # 8^3, 32 angles, 4 groups, c = 0.5
    p = _gpu(prob)
    phi, info = p.solve(1e-6, 200)
    assert info["status"] == 0 and info["residual"] <= 1e-6
    ref = oracle.Oracle.from_problem(prob).solve(1e-12, 500)
    err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
    assert err.max() <= TOL, err
    assert abs(info["iterations"] - np.argmax(ref["hist"] <= 1e-6) - 1) <= 1


def test_solve_from_given_start_and_noconv():
    torch = _torch()
    prob = inputs.config_problem(2, n=6)
    p = _gpu(prob)
    phi, info = p.solve(1e-30, 3, allow_noconv=True)
    assert info["rc"] == -7 and info["iterations"] == 3
    o = oracle.Oracle.from_problem(prob)
    ref = o.solve(0.0, 3, allow_noconv=True)
    assert H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"]).max() <= TOL
    # resume: two more sweeps from the returned iterate equal five from zero
    phi2, info2 = p.solve(1e-30, 2, phi0=phi, allow_noconv=True)
    ref5 = o.solve(0.0, 5, allow_noconv=True)
    assert H.rel_err_per_group(phi2.cpu().numpy().astype(np.float64), ref5["phi"]).max() <= TOL


def test_balance_and_integrated_flux_match_oracle():
    torch = _torch()
    prob = inputs.config_problem(2, n=6)
    phi32 = _phi_in(prob, 5)
    got, ref, p, o = _sweep_pair(prob, phi32)
    pin = torch.from_numpy(phi32).cuda()
    out = p.sweep(pin)
    b = p.balance(pin, out)
    r = o.sweep(phi32.astype(np.float64), want_leak=True)
    bref = o.balance(phi32.astype(np.float64), r["phi"], r["leak"])
    assert np.abs(b[:, :3] - bref[:, :3]).max() <= 1e-5 * np.abs(bref[:, :3]).max()
    assert b[:, 3].max() < 1e-4          # per-cell balance of the FP32 solve
    fl = p.integrated_flux(out)
    flr = o.integrated_flux(ref)
    assert np.abs(fl - flr).max() <= 1e-5 * np.abs(flr).max()


def test_sweep_before_setup_is_a_state_error():
    from paper_2510_11513_amd import snx
    torch = _torch()
    p = snx.Problem(0)
    with pytest.raises(snx.SnxError) as e:
        p.sweep(None, torch.zeros(8, device="cuda"))
    assert e.value.code == -2


def test_mesh_with_inverted_cell_is_rejected():
    from paper_2510_11513_amd import snx
    prob = inputs.config_problem(1, n=3)
    cv = prob.mesh.cell_vert.copy()
    cv[0] = cv[0][[1, 0, 3, 2, 5, 4, 7, 6]]      # mirror one cell: detJ < 0
    p = snx.Problem(0)
    p.set_mesh(prob.mesh.xyz, cv)
    om, w = snx.quadrature_product(1, 1)
    p.set_quadrature(om, w)
    p.set_materials(prob.mat.sigma_t, prob.mat.sigma_s, prob.mat.q)
    with pytest.raises(snx.SnxError) as e:
        p.setup()
    assert e.value.code == -3


def skewed_stack(G=3, npol=1, naz=2, seed=0):
    """Two cells stacked in z with the convex cross-section (0,0), (1,0), (4,1), (0,1):
    the +x face leans so far that, for octant 0, four faces are inflow (-x, +x, -y, -z);
    in the upper cell the fourth inflow slot is the interior face to the lower cell."""
    xy = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (4.0, 1.0)]
    xyz = np.array([(x, y, 0.5 * k) for k in range(3) for (x, y) in xy])
    cv = np.array([[4 * c + (j & 3) + 4 * (j >> 2) for j in range(8)] for c in range(2)], np.int32)
    mesh = inputs.Mesh(n=1, xyz=xyz, cell_vert=cv, ijk=np.zeros((2, 3), np.int32),
                       vert_ijk=np.zeros((12, 3), np.int32))
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.5, 2.0, (2, G))
    mat = inputs.Materials(st, st * rng.uniform(0.2, 0.8, (2, G)), rng.uniform(0.5, 1.5, (2, G)))
    prob = inputs.Problem("skewed", mesh, mat, npol, naz, 1e-6, boundary_kind=1,
                          psi_b=rng.uniform(0.1, 1.0, G))
    return prob


@pytest.mark.parametrize("threads,G", [(None, 3), (64, 24)])
def test_cells_with_four_inflow_faces(threads, G):
    prob = skewed_stack(G=G, npol=1, naz=2 if G == 3 else 4)
    mask = oracle.Oracle.from_problem(prob).dag()["inflow"]          # [8][C] inflow-face bit masks
    nin = np.vectorize(lambda m: bin(int(m)).count("1"))(mask)
    assert nin.max() == 4                          # the case this test exists for
    print(f"[case] skewed stack threads={threads} G={G} inflow faces={nin.tolist()}", flush=True)
    got, ref, _, _ = _sweep_pair(prob, _phi_in(prob, 4), threads=threads)
    assert H.rel_err_per_group(got, ref).max() <= TOL


@pytest.mark.parametrize("case,threads", [("cfg2_n6", None), ("cfg2_n6", 64), ("edge", None), ("skewed", None)])
def test_bulk_synchronous_comparator_gives_the_same_bits(case, threads):
    """The level-by-level sweep (the paper's BSP scheme) runs the same task code as the
    dependency-driven one: identical results, bit for bit, and both match the oracle."""
    torch = _torch()
    from paper_2510_11513_amd import snx
    prob = {"cfg2_n6": lambda: inputs.config_problem(2, n=6), "edge": lambda: _custom(4, 5, 3, 3, seed=9, kind=1),
            "skewed": lambda: skewed_stack(G=3)}[case]()
    print(f"[case] bsp {case} threads={threads}", flush=True)
    p = _gpu(prob, threads)
    pin = torch.from_numpy(_phi_in(prob, 5)).cuda()
    amt = p.sweep(pin).cpu().numpy()
    p.set_sweep_mode(snx.SWEEP_BSP)
    bsp = p.sweep(pin).cpu().numpy()
    assert np.array_equal(amt, bsp)
    ref = oracle.Oracle.from_problem(prob).sweep(_phi_in(prob, 5).astype(np.float64))["phi"]
    assert H.rel_err_per_group(bsp.astype(np.float64), ref).max() <= TOL
    # a solve in BSP mode takes the same iterations to the same bits
    phi_b, ib = p.solve(1e-6, 500)
    p.set_sweep_mode(snx.SWEEP_AMT)
    phi_a, ia = p.solve(1e-6, 500)
    assert ib["iterations"] == ia["iterations"]
    assert np.array_equal(phi_a.cpu().numpy(), phi_b.cpu().numpy())
