"""Pins of the oracle's group-to-group scattering and inner/outer iterations (CPU).

The benchmark runs of the paper (Section 3.6) use five inner and five outer
iterations.  Here an outer iteration fixes the cross-group scattering source
from its starting flux, and the inner iterations are source iterations with
the within-group scattering.  The checks:

* a diagonal matrix equals the within-group path bit for bit;
* the infinite-medium closed form (diag(sigma_t) - S^T) phi = Q is a fixed
  point of one sweep, and outer iterations reach it from zero;
* the converged iteration equals a dense solve of the coupled
  (direction, group, cell) system on a tiny mesh;
* the per-cell balance holds with the coupled source;
* one inner iteration per outer reproduces plain source iteration with the
  full coupled source.
"""
import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs
from tests import helpers as H

FOUR_PI = 4 * np.pi


def _matrix(G, rng, up=True):
    """[G][G] scattering matrix, row g' = from, column g = to: within-group,
    downscatter falling off with the group distance, and a little upscatter."""
    S = np.zeros((G, G))
    for g in range(G):
        S[g, g] = rng.uniform(0.2, 0.5)
        for h in range(g + 1, G):
            S[g, h] = rng.uniform(0.0, 0.3) / (h - g)
        if up:
            for h in range(g):
                S[g, h] = rng.uniform(0.0, 0.05)
    return S


def _homogeneous(m, om, w, st, S, Q, boundary=0, psib=None):
    C, G = m.ncell, st.shape[0]
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, np.tile(st, (C, 1)), np.zeros((C, G)), np.tile(Q, (C, 1)),
                      boundary, psib, setup=False)
    o.set_group_scattering(np.zeros(C, np.int32), S[None])
    o.setup()
    return o


def test_diagonal_matrix_equals_within_group_scattering():
    m = inputs.make_mesh(3, 0.2, seed=3)
    G = 3
    rng = np.random.default_rng(1)
    st = rng.uniform(0.5, 3.0, (m.ncell, G))
    ss = st * rng.uniform(0.0, 0.9, (m.ncell, G))
    q = rng.uniform(0.0, 1.0, (m.ncell, G))
    om, w = oracle.quadrature(1, 2)
    a = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q)
    b = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, np.zeros_like(ss), q, setup=False)
    sgg = np.zeros((m.ncell, G, G))
    for g in range(G):
        sgg[:, g, g] = ss[:, g]
    b.set_group_scattering(np.arange(m.ncell, dtype=np.int32), sgg)
    b.setup()
    phi_in = rng.uniform(0, 2, (m.ncell, G, 8))
    assert np.array_equal(a.sweep(phi_in)["phi"], b.sweep(phi_in)["phi"])


def test_infinite_medium_closed_form():
    m = inputs.make_mesh(4, 0.2, seed=13)
    G = 3
    rng = np.random.default_rng(2)
    st = np.array([1.0, 2.0, 4.0])
    S = _matrix(G, rng)
    Q = np.array([1.0, 0.5, 0.2])
    phi_inf = np.linalg.solve(np.diag(st) - S.T, Q)      # sigma_t,g phi_g = Q_g + sum_g' S[g', g] phi_g'
    assert (phi_inf > 0).all()
    om, w = oracle.quadrature(2, 3)
    o = _homogeneous(m, om, w, st, S, Q, 1, phi_inf / FOUR_PI)
    phi0 = np.broadcast_to(phi_inf[None, :, None], (m.ncell, G, 8)).copy()
    r = o.sweep(phi0)
    assert np.abs(r["phi"] / phi0 - 1).max() < 1e-12
    s = o.solve_outer(200, 3, tol=1e-13)
    assert s["status"] == 0 and s["outers"] > 5
    assert np.abs(s["phi"] / phi0 - 1).max() < 1e-10


def test_dense_coupled_system_equals_converged_outer_iteration():
    m = inputs.make_mesh(2, 0.2, seed=31)
    om, w = oracle.quadrature(1, 1)
    nang, C, G = om.shape[0], m.ncell, 2
    st = np.array([1.3, 2.1])
    S = np.array([[0.5, 0.4], [0.1, 0.9]])
    Q = np.array([1.0, 0.3])
    o = _homogeneous(m, om, w, st, S, Q)
    g_, d_ = o.geometry(), o.dag()
    nu = 8 * C
    Mblk = np.zeros((nu, nu))
    for K in range(C):
        Mblk[8 * K:8 * K + 8, 8 * K:8 * K + 8] = g_["M"][K]
    big = np.zeros((nang * G * nu, nang * G * nu))
    rhs = np.zeros(nang * G * nu)
    blk = lambda n, g: slice((n * G + g) * nu, (n * G + g + 1) * nu)
    for n in range(nang):
        for g in range(G):
            big[blk(n, g), blk(n, g)] += H.dense_angle_matrix(g_, d_, om, n, nang, np.full(C, st[g]))
            for mm in range(nang):
                for h in range(G):       # scattering from group h into g couples every direction pair
                    big[blk(n, g), blk(mm, h)] -= S[h, g] / FOUR_PI * w[mm] * Mblk
            rhs[blk(n, g)] = Mblk @ np.full(nu, Q[g] / FOUR_PI)
    psi = np.linalg.solve(big, rhs).reshape(nang, G, C, 8)
    phi_dense = np.einsum("n,ngkj->kgj", w, psi)
    s = o.solve_outer(500, 4, tol=1e-14)
    assert s["status"] == 0
    assert np.abs(s["phi"] - phi_dense).max() < 1e-11 * np.abs(phi_dense).max()
    # plain source iteration with the full coupled source reaches the same point
    j = o.solve(1e-14, 5000)
    assert np.abs(j["phi"] - phi_dense).max() < 1e-11 * np.abs(phi_dense).max()


def test_balance_with_coupled_source():
    m = inputs.make_mesh(3, 0.2, seed=8)
    G = 3
    rng = np.random.default_rng(5)
    om, w = oracle.quadrature(1, 3)
    C = m.ncell
    st = rng.uniform(0.5, 3.0, (C, G))
    q = rng.uniform(0.0, 1.0, (C, G))
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, np.zeros((C, G)), q, setup=False)
    mats = np.stack([_matrix(G, rng) for _ in range(3)])
    o.set_group_scattering(rng.integers(0, 3, C).astype(np.int32), mats)
    o.setup()
    phi_in = rng.uniform(0, 1, (C, G, 8))
    r = o.sweep(phi_in, want_leak=True)
    b = o.balance(phi_in, r["phi"], r["leak"])
    assert b[:, 3].max() < 1e-12
    assert np.abs(b[:, 0] - b[:, 1] - b[:, 2]).max() < 1e-12 * np.abs(b[:, 0]).max()


@pytest.mark.parametrize("designation", [0, 1])
def test_one_inner_per_outer_is_plain_source_iteration(designation):
    m = inputs.make_mesh(3, 0.3, seed=0)
    G = 3
    rng = np.random.default_rng(6)
    om, w = oracle.quadrature(2, 2)
    C = m.ncell
    st = rng.uniform(0.5, 3.0, (C, G))
    q = rng.uniform(0.0, 1.0, (C, G))
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, np.zeros((C, G)), q, setup=False, designation=designation)
    o.set_group_scattering(np.zeros(C, np.int32), _matrix(G, rng)[None])
    o.setup()
    a = o.solve_outer(7, 1, tol=0.0)
    b = o.solve(0.0, 7, allow_noconv=True)
    assert a["inners"] == 7 and b["iters"] == 7
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-13 * np.abs(b["phi"]).max()
