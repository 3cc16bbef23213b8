"""Higher-order elements (orders 2 and 3) on the GPU vs the FP64 oracle
(oracle/ho.py), through the C ABI.

One sweep from a random flux on jittered meshes with randomly turned cells
(shared faces in every relative orientation), vacuum and isotropic inflow,
group counts that leave a ragged last round of systems; a converged source
iteration; the refused options.

Tolerance: 1e-5 relative per group on the scalar flux, as at order 1 (the
systems here have 27 and 64 unknowns, solved by unpivoted LU in FP32; the
measured errors stay below 1e-6).
"""
import numpy as np
import pytest

import oracle
from oracle import ho
from paper_2510_11513_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _problem(n, G, npol, naz, seed, kind=0, rotate=True, c=(0.2, 0.8)):
    rng = np.random.default_rng(seed)
    mesh = inputs.make_mesh(n, 0.25, rng=rng)
    if rotate:
        mesh = inputs.rotate_cells(mesh, rng)
    mat = inputs.materials_loguniform_blocks(mesh, G, rng, 2, c[0], c[1])
    prob = inputs.Problem(f"ho_n{n}G{G}", mesh, mat, npol, naz, 1e-6)
    if kind == 1:
        prob.boundary_kind = 1
        prob.psi_b = rng.uniform(0.1, 1.0, G)
    return prob


def _pair(prob, order):
    from paper_2510_11513_amd import snx
    p = snx.Problem.from_problem(prob, order=order)
    om, w = oracle.quadrature(prob.npolar, prob.nazim)
    o = ho.HOOracle(prob.mesh.xyz, prob.mesh.cell_vert, order, om, w, prob.mat.sigma_t, prob.mat.sigma_s,
                    prob.mat.q, psi_b=prob.psi_b if prob.boundary_kind == 1 else None)
    return p, o


CASES = {
    "p2_n3_G5_inflow": (2, lambda: _problem(3, 5, 1, 2, seed=1, kind=1)),
    "p2_n4_G11_ragged": (2, lambda: _problem(4, 11, 2, 2, seed=2)),
    "p2_n1_single_cell": (2, lambda: _problem(1, 3, 1, 1, seed=3, kind=1)),
    "p3_n3_G5_inflow": (3, lambda: _problem(3, 5, 1, 2, seed=4, kind=1)),
    "p3_n2_G2_unrotated": (3, lambda: _problem(2, 2, 2, 1, seed=5, rotate=False)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_one_sweep_matches_the_oracle(name):
    torch = _torch()
    order, make = CASES[name]
    prob = make()
    print(f"[case] order {order} {name}: C={prob.mesh.ncell} G={prob.mat.ngroup} nang={prob.nang}", flush=True)
    p, o = _pair(prob, order)
    rng = np.random.default_rng(7)
    phi_in = rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, o.N)).astype(np.float32)
    out = p.sweep(torch.from_numpy(phi_in).cuda())
    torch.cuda.synchronize()
    ref = o.sweep(phi_in.astype(np.float64))["phi"]
    err = H.rel_err_per_group(out.cpu().numpy().astype(np.float64), ref)
    print(f"[case] max rel err per group {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    # a sweep from zero flux (phi_in NULL) too
    out0 = p.sweep(None)
    torch.cuda.synchronize()
    err0 = H.rel_err_per_group(out0.cpu().numpy().astype(np.float64), o.sweep(None)["phi"])
    assert err0.max() <= TOL, err0
    p.close()


@pytest.mark.parametrize("order", [2, 3])
def test_converged_source_iteration(order):
    prob = _problem(3, 3, 1, 2, seed=10 + order, kind=1, c=(0.2, 0.6))
    p, o = _pair(prob, order)
    phi, info = p.solve(1e-6, 300)
    assert info["status"] == 0, info
    ref = o.solve(1e-12, 500)
    err = H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"])
    print(f"[case] order {order} solve: iterations gpu {info['iterations']} oracle {ref['iters']}, "
          f"rel err {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    p.close()


def test_profile_and_fixed_iteration_count():
    torch = _torch()
    prob = _problem(3, 4, 1, 2, seed=20)
    p, o = _pair(prob, 2)
    phi, info = p.solve(0.0, 4, allow_noconv=True)
    assert info["iterations"] == 4
    ref = o.solve(0.0, 4)
    assert H.rel_err_per_group(phi.cpu().numpy().astype(np.float64), ref["phi"]).max() <= TOL
    ms = p.profile_sweep(3, phi_in=phi)
    assert ms > 0.0
    torch.cuda.synchronize()
    p.close()


def test_refused_options_and_sizes():
    torch = _torch()
    from paper_2510_11513_amd import snx
    prob = _problem(2, 2, 1, 1, seed=30)
    p = snx.Problem.from_problem(prob, setup=False, order=2)
    p.set_reflective(1)
    with pytest.raises(snx.SnxError):
        p.setup()
    p.set_reflective(0)
    p.setup()
    with pytest.raises(snx.SnxError):
        p.solve_outer(2, 2)
    with pytest.raises(snx.SnxError):
        snx.Batch([p])
    wrong = torch.zeros((prob.mesh.ncell, prob.mat.ngroup, 8), device="cuda")
    with pytest.raises(ValueError):
        p.sweep(wrong)
    p.close()


@pytest.mark.parametrize("order", [2, 3])
def test_full_size_mirror_symmetry(order):
    """At the benchmark's size (16^3 cells, 128 angles, 16 groups) and launch
    configuration: on an unjittered mesh with uniform materials and inflow, one
    sweep's flux is symmetric under x -> 1 - x (cell (i, j, k) node (a, b, c)
    against cell (15 - i, j, k) node (p - a, b, c)); the product quadrature
    holds every direction's mirror image.  The octants run in different
    orders, so any error of the face maps, the octant designation or the
    level lists shows as an asymmetry."""
    torch = _torch()
    from paper_2510_11513_amd import snx
    n, G = 16, 16
    mesh = inputs.make_mesh(n, 0.0, seed=7)
    mat = inputs.materials_uniform(mesh, G, 1.0, 0.5, 1.0, scaled=True)
    prob = inputs.Problem("ho_mirror", mesh, mat, 4, 4, 1e-6)
    prob.boundary_kind = 1
    prob.psi_b = np.linspace(0.1, 0.5, G)
    p = snx.Problem.from_problem(prob, order=order)
    m = order + 1
    rng = np.random.default_rng(5)
    # a flux that is itself mirror-symmetric (a function of |x - 1/2|, y, z per node)
    ijk = mesh.ijk
    N = m ** 3
    base = rng.uniform(0.5, 1.5, (n, n, n, G, m, m, m))
    base = 0.5 * (base + base[::-1, :, :, :, ::-1, :, :])
    phi_in = np.empty((mesh.ncell, G, N), np.float32)
    for K in range(mesh.ncell):
        i, j, k = ijk[K]
        # node j = a + m b + m^2 c: axis order (c, b, a) in a C-ordered [m][m][m] block
        phi_in[K] = base[i, j, k].transpose(0, 3, 2, 1).reshape(G, N)
    out = p.sweep(torch.from_numpy(phi_in).cuda())
    torch.cuda.synchronize()
    phi = out.cpu().numpy().astype(np.float64).reshape(mesh.ncell, G, m, m, m)   # [K][g][c][b][a]
    where = {tuple(v): K for K, v in enumerate(ijk)}
    mirror = np.array([where[(n - 1 - i, j, k)] for i, j, k in ijk])
    asym = np.abs(phi - phi[mirror][:, :, :, :, ::-1]).max(axis=(0, 2, 3, 4)) / np.abs(phi).max(axis=(0, 2, 3, 4))
    print(f"[case] order {order} full size: max relative asymmetry per group {asym.max():.2e}", flush=True)
    assert np.all(np.isfinite(phi)) and phi.min() > 0
    assert asym.max() <= 1e-5, asym
    p.close()


@pytest.mark.parametrize("order", [2, 3])
def test_jittered_rotated_8cubed_every_node(order):
    """8^3 jittered cells, each turned at random, 16 directions, 3 groups with
    sigma_t from 0.1 to 10 (small pivots in the thin cells): one sweep from a
    random flux, every node value of every group against the oracle."""
    torch = _torch()
    prob = _problem(8, 3, 1, 2, seed=40 + order, kind=1)
    assert prob.mat.sigma_t.min() < 0.2 and prob.mat.sigma_t.max() > 5.0
    p, o = _pair(prob, order)
    N = (order + 1) ** 3
    rng = np.random.default_rng(41)
    phi32 = rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, N)).astype(np.float32)
    print(f"[case] order {order} 8^3 rotated: C={prob.mesh.ncell} nang={prob.nang} G={prob.mat.ngroup}", flush=True)
    out = p.sweep(torch.from_numpy(phi32).cuda())
    torch.cuda.synchronize()
    ref = o.sweep(phi32.astype(np.float64))["phi"]
    err = H.rel_err_per_group(out.cpu().numpy().astype(np.float64), ref)
    print(f"[case] order {order} 8^3 rotated: phi max rel err {err.max():.2e}", flush=True)
    assert err.max() <= TOL, err
    p.close()


@pytest.mark.parametrize("order", [2, 3])
def test_full_size_sampled_directions(order):
    """The benchmark's size and launch configuration (16^3 jittered cells, 128
    directions, 16 groups): the angular flux of four sampled directions, one per
    octant of a random choice, every group and node, against the oracle's sweep
    of those directions alone (the directions of one source iteration are
    independent for a given input flux)."""
    torch = _torch()
    from paper_2510_11513_amd import snx
    prob = inputs.config_problem(0)
    p = snx.Problem.from_problem(prob, order=order)
    om, w = oracle.quadrature(prob.npolar, prob.nazim)
    N = (order + 1) ** 3
    rng = np.random.default_rng(50 + order)
    phi32 = rng.uniform(0.0, 2.0, (prob.mesh.ncell, prob.mat.ngroup, N)).astype(np.float32)
    print(f"[case] order {order} full size: C={prob.mesh.ncell} nang={prob.nang} G={prob.mat.ngroup}", flush=True)
    p.sweep(torch.from_numpy(phi32).cuda())
    torch.cuda.synchronize()
    o = ho.HOOracle(prob.mesh.xyz, prob.mesh.cell_vert, order, om, w, prob.mat.sigma_t, prob.mat.sigma_s,
                    prob.mat.q)
    per = prob.nang // 8
    for oc in rng.permutation(8)[:4]:
        n = int(oc * per + rng.integers(per))
        ref = o.sweep_angle(phi32.astype(np.float64), n)              # [C][G][N]
        errs = []
        for g in range(prob.mat.ngroup):
            got = p.psi(n, g).cpu().numpy().astype(np.float64)
            errs.append(np.abs(got - ref[:, g]).max() / np.abs(ref[:, g]).max())
        print(f"[case] order {order} full size direction {n}: max rel err over groups {max(errs):.2e}", flush=True)
        assert max(errs) <= TOL, (order, n, errs)
    p.close()
