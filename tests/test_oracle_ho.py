"""Pins of the higher-order oracle (CPU, FP64; oracle/ho.py).

* order 1 equals the first-order oracle (an independent implementation in C:
  its own neighbour search, node matching and sweep order);
* polynomial exactness: with the exact inflow and the matching source, the
  order-p sweep reproduces every polynomial of total degree <= p in x, y, z at
  the nodes (the solution lies in the element space and the equations hold
  pointwise), on jittered meshes whose cells are turned at random, so shared
  faces meet in every relative orientation; degree p + 1 is not reproduced;
* the discrete divergence theorem: each cell's source equals its absorption
  plus its net outflow;
* the mass matrix integrates 1 to the same cell volume at every order;
* a converged source iteration is a fixed point of the sweep.
"""
import numpy as np
import pytest

import oracle
from oracle import ho
from paper_2510_11513_amd import inputs


def _material(C, G, rng, c=(0.2, 0.8)):
    st = rng.uniform(0.5, 2.0, (C, G))
    ss = st * rng.uniform(c[0], c[1], (C, G))
    q = rng.uniform(0.0, 1.0, (C, G))
    return st, ss, q


def test_order_one_equals_the_first_order_oracle():
    rng = np.random.default_rng(3)
    m = inputs.rotate_cells(inputs.make_mesh(3, 0.25, seed=4), rng)
    C, G = m.ncell, 3
    st, ss, q = _material(C, G, rng)
    psi_b = rng.uniform(0.1, 1.0, G)
    om, w = oracle.quadrature(2, 2)
    a = ho.HOOracle(m.xyz, m.cell_vert, 1, om, w, st, ss, q, psi_b=psi_b)
    b = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, boundary_kind=1, psi_b=psi_b)
    phi_in = rng.uniform(0.0, 2.0, (C, G, 8))
    ra = a.sweep(phi_in, want_leak=True)
    rb = b.sweep(phi_in, want_leak=True)
    scale = np.abs(rb["phi"]).max()
    assert np.abs(ra["phi"] - rb["phi"]).max() <= 1e-12 * scale
    assert np.abs(ra["leak"] - rb["leak"]).max() <= 1e-11 * np.abs(rb["leak"]).max()


def _poly(deg, rng):
    """A random polynomial of total degree `deg` in (x, y, z): its value and gradient."""
    terms = [(i, j, k) for i in range(deg + 1) for j in range(deg + 1) for k in range(deg + 1) if i + j + k <= deg]
    coef = rng.uniform(-1.0, 1.0, len(terms))
    coef[[t for t, e in enumerate(terms) if sum(e) == deg]] += 2.0    # the top degree is really there

    def val(x):
        return sum(c * x[..., 0] ** i * x[..., 1] ** j * x[..., 2] ** k for c, (i, j, k) in zip(coef, terms))

    def grad(x):
        def pw(v, e):
            return v ** e if e >= 0 else 0.0 * v
        gx = sum(c * i * pw(x[..., 0], i - 1) * x[..., 1] ** j * x[..., 2] ** k for c, (i, j, k) in zip(coef, terms))
        gy = sum(c * j * x[..., 0] ** i * pw(x[..., 1], j - 1) * x[..., 2] ** k for c, (i, j, k) in zip(coef, terms))
        gz = sum(c * k * x[..., 0] ** i * x[..., 1] ** j * pw(x[..., 2], k - 1) for c, (i, j, k) in zip(coef, terms))
        return np.stack([gx, gy, gz], axis=-1)
    return val, grad


def _manufactured(o, val, grad):
    """Angular source and boundary inflow of the exact solution psi = val(x),
    the same in every direction and group, for a pure absorber."""
    x = o.node_xyz                                                    # [C, N, 3]
    P, dP = val(x), grad(x)
    stream = np.einsum("na,Kja->nKj", o.omega, dP)                    # Omega . grad P at the nodes
    ang = stream[:, :, None, :] + o.st[None, :, :, None] * P[None, :, None, :]
    bnd = np.zeros((o.C, 6, o.nang, o.G, o.nf))
    for f in range(6):
        bnd[:, f] = P[:, o.face_nodes[f]][:, None, None, :]
    return ang, bnd, P


@pytest.mark.parametrize("p,n", [(1, 3), (2, 3), (3, 2)])
def test_polynomials_of_degree_p_are_reproduced(p, n):
    rng = np.random.default_rng(10 + p)
    m = inputs.rotate_cells(inputs.make_mesh(n, 0.25, seed=20 + p), rng)
    C, G = m.ncell, 2
    st = rng.uniform(0.5, 3.0, (C, G))
    om, w = oracle.quadrature(1, 2)
    o = ho.HOOracle(m.xyz, m.cell_vert, p, om, w, st, np.zeros((C, G)), np.zeros((C, G)))
    for deg, exact in ((p, True), (p + 1, False)):
        val, grad = _poly(deg, rng)
        ang, bnd, P = _manufactured(o, val, grad)
        psi = o.sweep(None, want_psi=True, ang_src=ang, bnd=bnd)["psi"]
        err = np.abs(psi - P[None, :, None, :]).max() / np.abs(P).max()
        if exact:
            assert err < 1e-11, (p, deg, err)
        else:
            assert err > 1e-6, (p, deg, err)


@pytest.mark.parametrize("p", [2, 3])
def test_cell_balance(p):
    rng = np.random.default_rng(30 + p)
    m = inputs.rotate_cells(inputs.make_mesh(3 if p == 2 else 2, 0.25, seed=31), rng)
    C, G = m.ncell, 2
    st, ss, q = _material(C, G, rng)
    om, w = oracle.quadrature(1, 2)
    o = ho.HOOracle(m.xyz, m.cell_vert, p, om, w, st, ss, q, psi_b=rng.uniform(0.1, 1.0, G))
    phi_in = rng.uniform(0.0, 2.0, (C, G, o.N))
    r = o.sweep(phi_in, want_leak=True)
    b = o.balance(phi_in, r["phi"], r["leak"])
    assert b[:, 3].max() < 1e-12, b
    assert np.all(b[:, 0] > 0) and np.all(b[:, 1] > 0)


def test_volumes_agree_across_orders():
    rng = np.random.default_rng(40)
    m = inputs.rotate_cells(inputs.make_mesh(2, 0.3, seed=41), rng)
    C = m.ncell
    om, w = oracle.quadrature(1, 1)
    one = np.ones((C, 1))
    vols = [ho.HOOracle(m.xyz, m.cell_vert, p, om, w, one, 0 * one, one).volumes() for p in (1, 2, 3)]
    assert np.abs(vols[1] - vols[0]).max() < 1e-14 and np.abs(vols[2] - vols[0]).max() < 1e-14
    assert abs(vols[0].sum() - 1.0) < 1e-13     # the meshes tile the unit cube


def test_converged_solution_is_a_fixed_point():
    rng = np.random.default_rng(50)
    m = inputs.make_mesh(2, 0.2, seed=51)
    C, G = m.ncell, 2
    st, ss, q = _material(C, G, rng, c=(0.2, 0.5))
    om, w = oracle.quadrature(1, 2)
    o = ho.HOOracle(m.xyz, m.cell_vert, 2, om, w, st, ss, q)
    s = o.solve(1e-13, 200)
    assert s["status"] == 0
    again = o.sweep(s["phi"])["phi"]
    assert np.abs(again - s["phi"]).max() <= 1e-12 * np.abs(s["phi"]).max()
