"""Pins of the oracle's reflective boundary planes (CPU, FP64).

On a reflective plane the inflow of direction n is the outflow of its mirror
image at the same nodes, taken from the previous sweep.  The checks:

* mirror symmetry: a problem with the plane x = 0 reflective has the same
  solution as the doubled problem (the mesh and its mirror image, vacuum
  everywhere) on the original half;
* infinite medium: with all six planes reflective a homogeneous medium has
  phi = Q / sigma_a, a fixed point of one sweep and the limit of the iteration;
* the balance holds with the reflected inflow;
* quadratures without the mirrored directions are refused.

With the octants in sequence (UnSNAP's order, kept so that reflective faces
can use the newest values; Section 2.1 and its footnote), a direction that
enters through a plane x = 1, y = 1 or z = 1 has its mirror image in an
earlier octant, so every reflected inflow of one sweep is current.  One such
sweep is then exactly one vacuum sweep of the mesh mirrored across those
planes, restricted to the original cells: a single-sweep pin that does not
depend on how the GPU schedules the octants.
"""
import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs

FOUR_PI = 4 * np.pi


def _mirror_x(m):
    """The mesh and its image under x -> -x, sharing the vertices on x = 0.  A
    mirrored cell lists its vertices with local bit 0 flipped, so it keeps a
    positive Jacobian."""
    xyz, cv = m.xyz, m.cell_vert
    on_plane = xyz[:, 0] == 0.0
    new_id = np.where(on_plane, np.arange(len(xyz)), len(xyz) + np.cumsum(~on_plane) - 1)
    mx = xyz[~on_plane].copy()
    mx[:, 0] = -mx[:, 0]
    xyz2 = np.concatenate([xyz, mx])
    flip = np.array([j ^ 1 for j in range(8)])
    cv2 = np.concatenate([cv, new_id[cv[:, flip]]]).astype(np.int32)
    return xyz2, cv2


@pytest.mark.parametrize("designation,L", [(0, 0), (1, 0), (0, 2)])
def test_mirror_symmetry_of_a_reflective_plane(designation, L):
    """Also under per-angle designation and anisotropic scattering: both are
    invariant under the mirror map (Omega . A_f and Omega . Omega' keep their
    values for mirrored pairs)."""
    m = inputs.make_mesh(3, 0.3 if designation else 0.2, seed=5)
    C, G = m.ncell, 2
    rng = np.random.default_rng(3)
    st = rng.uniform(0.5, 2.0, (C, G))
    ss = st * rng.uniform(0.2, 0.6, (C, G))
    q = rng.uniform(0.0, 1.0, (C, G))
    sigl = ss[:, :, None] * 0.5 ** np.arange(1, L + 1)[None, None, :]
    om, w = oracle.quadrature(2, 2)
    half = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, setup=False, designation=designation)
    half.set_reflective(1 << 0)                # plane x = 0 (outward area vector along -x)
    if L:
        half.set_anisotropy(sigl)
    half.setup()
    xyz2, cv2 = _mirror_x(m)
    full = oracle.Oracle(xyz2, cv2, om, w, np.tile(st, (2, 1)), np.tile(ss, (2, 1)), np.tile(q, (2, 1)),
                         setup=False, designation=designation)
    if L:
        full.set_anisotropy(np.tile(sigl, (2, 1, 1)))
    full.setup()
    a = half.solve(1e-14, 3000)
    b = full.solve(1e-14, 3000)
    assert a["status"] == 0 and b["status"] == 0
    if not designation and not L:
        assert a["iters"] > b["iters"]           # the reflected inflow lags one sweep
    ref = b["phi"][:C]
    assert np.abs(a["phi"] - ref).max() < 1e-10 * np.abs(ref).max()
    # the doubled solution is itself mirror-symmetric
    assert np.abs(b["phi"][C:].sum(axis=2) - ref.sum(axis=2)).max() < 1e-10 * np.abs(ref).max()


def test_infinite_medium_with_six_reflective_planes():
    m = inputs.make_mesh(3, 0.2, seed=9)
    C, G = m.ncell, 2
    st, c, Q = np.array([1.0, 3.0]), np.array([0.5, 0.8]), np.array([1.0, 2.0])
    om, w = oracle.quadrature(2, 3)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, np.tile(st, (C, 1)), np.tile(c * st, (C, 1)), np.tile(Q, (C, 1)),
                      setup=False)
    o.set_reflective(63)
    o.setup()
    phi_inf = Q / (st * (1 - c))
    phi0 = np.broadcast_to(phi_inf[None, :, None], (C, G, 8)).copy()
    psi0 = np.broadcast_to((phi_inf / FOUR_PI)[None, None, :, None], (om.shape[0], C, G, 8)).copy()
    r = o.sweep(phi0, psi_prev=psi0)
    assert np.abs(r["phi"] / phi0 - 1).max() < 1e-12
    s = o.solve(1e-13, 5000)
    assert s["status"] == 0
    assert np.abs(s["phi"] / phi0 - 1).max() < 1e-10


def test_balance_with_reflected_inflow():
    m = inputs.make_mesh(3, 0.2, seed=4)
    C, G = m.ncell, 2
    rng = np.random.default_rng(8)
    st = rng.uniform(0.5, 2.0, (C, G))
    ss = st * rng.uniform(0.2, 0.6, (C, G))
    q = rng.uniform(0.0, 1.0, (C, G))
    om, w = oracle.quadrature(1, 2)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, setup=False)
    o.set_reflective(0b100110)
    o.setup()
    phi_in = rng.uniform(0, 1, (C, G, 8))
    psi_prev = rng.uniform(0, 1, (om.shape[0], C, G, 8))
    r = o.sweep(phi_in, want_leak=True, psi_prev=psi_prev)
    b = o.balance(phi_in, r["phi"], r["leak"])
    assert b[:, 3].max() < 1e-12
    # the reflected inflow enters: without it the sweep differs
    r0 = o.sweep(phi_in)
    assert np.abs(r0["phi"] - r["phi"]).max() > 1e-3 * np.abs(r["phi"]).max()


def test_quadrature_without_mirror_images_is_refused():
    m = inputs.make_mesh(2, 0.1, seed=1)
    om, w = oracle.quadrature(1, 2)
    om = om.copy()
    # turn the first direction of octant 0 a little about z: its x-mirror is gone
    t = 0.05
    x, y = om[0, 0], om[0, 1]
    om[0, 0], om[0, 1] = np.cos(t) * x - np.sin(t) * y, np.sin(t) * x + np.cos(t) * y
    C = m.ncell
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, np.ones((C, 1)), np.zeros((C, 1)), np.ones((C, 1)), setup=False)
    o.set_reflective(1)
    with pytest.raises(oracle.OracleError):
        o.setup()


def _mirror(xyz, cv, axis):
    """The mesh and its image across the plane x_axis = max x_axis (vertices on the
    plane shared; local bit `axis` flipped so the image keeps a positive
    Jacobian).  Returns the new arrays and the local-node permutation of an
    image cell."""
    top = xyz[:, axis].max()
    on_plane = xyz[:, axis] == top
    new_id = np.where(on_plane, np.arange(len(xyz)), len(xyz) + np.cumsum(~on_plane) - 1)
    mx = xyz[~on_plane].copy()
    mx[:, axis] = 2.0 * top - mx[:, axis]
    flip = np.array([j ^ (1 << axis) for j in range(8)])
    return np.concatenate([xyz, mx]), np.concatenate([cv, new_id[cv[:, flip]]]).astype(np.int32), flip


def _mirrored_case(axes, seed=3, n=3):
    m = inputs.make_mesh(n, 0.25, seed=seed)
    assert np.all(m.xyz.max(axis=0) == 1.0)
    C, G = m.ncell, 2
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.5, 2.0, (C, G))
    ss = st * rng.uniform(0.2, 0.6, (C, G))
    q = rng.uniform(0.0, 1.0, (C, G))
    phi_in = rng.uniform(0.0, 1.0, (C, G, 8))
    xyz, cv = m.xyz, m.cell_vert
    big = [st, ss, q, phi_in]
    for a in axes:
        xyz, cv, flip = _mirror(xyz, cv, a)
        big = [np.concatenate([x, x]) for x in big[:3]] + [np.concatenate([big[3], big[3][:, :, flip]])]
    return m, (st, ss, q, phi_in), (xyz, cv, *big)


@pytest.mark.parametrize("axes", [(0,), (1,), (0, 1), (0, 1, 2)])
def test_sequential_octants_one_sweep_equals_the_mirrored_mesh(axes):
    m, (st, ss, q, phi_in), (xyz, cv, st2, ss2, q2, phi2) = _mirrored_case(axes)
    C = m.ncell
    om, w = oracle.quadrature(2, 2)
    planes = sum(1 << (2 * a + 1) for a in axes)
    half = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, setup=False)
    half.set_reflective(planes)
    half.set_octant_order(True)
    half.setup()
    full = oracle.Oracle(xyz, cv, om, w, st2, ss2, q2)
    ref = full.sweep(phi2)["phi"][:C]
    got = half.sweep(phi_in)["phi"]
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    # the concurrent reading takes last sweep's (here zero) reflected inflow instead
    half.set_octant_order(False)
    assert np.abs(half.sweep(phi_in)["phi"] - ref).max() > 1e-3 * np.abs(ref).max()


def test_sequential_and_concurrent_octants_share_the_fixed_point():
    """Both orders converge to the solution of the mirrored problem; the sequence
    needs fewer iterations on +side planes, where it has no lag at all."""
    axes = (0, 2)
    m, (st, ss, q, _), (xyz, cv, st2, ss2, q2, _) = _mirrored_case(axes, seed=7)
    C = m.ncell
    om, w = oracle.quadrature(2, 2)
    planes = sum(1 << (2 * a + 1) for a in axes)
    res = {}
    for seq in (True, False):
        o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, setup=False)
        o.set_reflective(planes)
        o.set_octant_order(seq)
        o.setup()
        res[seq] = o.solve(1e-14, 3000)
        assert res[seq]["status"] == 0
    ref = oracle.Oracle(xyz, cv, om, w, st2, ss2, q2).solve(1e-14, 3000)["phi"][:C]
    for seq in (True, False):
        assert np.abs(res[seq]["phi"] - ref).max() < 1e-10 * np.abs(ref).max()
    assert res[True]["iters"] < res[False]["iters"]


def test_sequential_octants_on_every_plane():
    """Planes of both sides: the -side planes still take last sweep's values in
    the sequence.  The infinite medium stays a fixed point, the balance holds,
    and the iteration reaches the doubled-mesh solution for x = 0 and x = 1."""
    m = inputs.make_mesh(3, 0.2, seed=9)
    C, G = m.ncell, 2
    st, c, Q = np.array([1.0, 3.0]), np.array([0.5, 0.8]), np.array([1.0, 2.0])
    om, w = oracle.quadrature(2, 3)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, np.tile(st, (C, 1)), np.tile(c * st, (C, 1)), np.tile(Q, (C, 1)),
                      setup=False)
    o.set_reflective(63)
    o.set_octant_order(True)
    o.setup()
    phi_inf = Q / (st * (1 - c))
    phi0 = np.broadcast_to(phi_inf[None, :, None], (C, G, 8)).copy()
    psi0 = np.broadcast_to((phi_inf / FOUR_PI)[None, None, :, None], (om.shape[0], C, G, 8)).copy()
    r = o.sweep(phi0, psi_prev=psi0, want_leak=True)
    assert np.abs(r["phi"] / phi0 - 1).max() < 1e-12
    rng = np.random.default_rng(4)
    phi_in = rng.uniform(0, 1, (C, G, 8))
    psi_prev = rng.uniform(0, 1, (om.shape[0], C, G, 8))
    r = o.sweep(phi_in, psi_prev=psi_prev, want_leak=True)
    assert o.balance(phi_in, r["phi"], r["leak"])[:, 3].max() < 1e-12
    # x = 0 and x = 1 together: the solution on [0,1] of the problem on [-1, 2]
    # with vacuum ends is not a finite mirror; instead check both orders agree
    m2 = inputs.make_mesh(3, 0.2, seed=10)
    rng = np.random.default_rng(5)
    st2 = rng.uniform(0.5, 2.0, (C, G))
    ss2 = st2 * rng.uniform(0.2, 0.6, (C, G))
    q2 = rng.uniform(0, 1, (C, G))
    out = []
    for seq in (True, False):
        oo = oracle.Oracle(m2.xyz, m2.cell_vert, om, w, st2, ss2, q2, setup=False)
        oo.set_reflective(0b11)
        oo.set_octant_order(seq)
        oo.setup()
        out.append(oo.solve(1e-14, 5000))
    assert out[0]["status"] == 0 and out[1]["status"] == 0
    assert np.abs(out[0]["phi"] - out[1]["phi"]).max() < 1e-10 * np.abs(out[1]["phi"]).max()
