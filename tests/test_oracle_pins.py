"""Pins of the FP64 oracle against what mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: a library
routine, a closed form, an invariant, an exact discrete solution or a dense
solve of the same discrete system assembled independently of the sweep.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs
from tests import helpers as H

FOUR_PI = 4 * np.pi


# ----------------------------------------------------------------- quadrature

@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 16])
def test_gauss_legendre_matches_numpy(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.abs(x - xr).max() < 1e-14
    assert np.abs(w - wr).max() < 1e-14


@pytest.mark.parametrize("npol,naz", [(1, 1), (2, 2), (3, 4), (4, 8), (2, 4)])
def test_product_quadrature_moments(npol, naz):
    om, w = oracle.quadrature(npol, naz)
    assert om.shape == (8 * npol * naz, 3)
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - FOUR_PI) < 1e-13                      # sum w = 4 pi
    assert np.abs((w[:, None] * om).sum(0)).max() < 1e-14       # first moment 0
    second = np.einsum("n,na,nb->ab", w, om, om)
    assert np.abs(second - FOUR_PI / 3 * np.eye(3)).max() < 1e-13
    per = npol * naz
    for n in range(om.shape[0]):                                # octant grouping
        o = (om[n, 0] < 0) + 2 * (om[n, 1] < 0) + 4 * (om[n, 2] < 0)
        assert o == n // per


def test_quadrature_polar_major_and_equal_azimuth_weights():
    om, w = oracle.quadrature(3, 4)
    mu, wmu = np.polynomial.legendre.leggauss(6)
    for k in range(3):
        for j in range(4):
            n = k * 4 + j
            assert abs(om[n, 2] - mu[3 + k]) < 1e-14
            assert abs(w[n] - wmu[3 + k] * np.pi / 8) < 1e-15
            assert abs(np.arctan2(om[n, 1], om[n, 0]) - (j + 0.5) * np.pi / 8) < 1e-14


# ------------------------------------------------------------------- geometry

def _oracle_for(mesh, G=1, st=1.0, c=0.0, q=1.0, npol=1, naz=1, **kw):
    mat = inputs.materials_uniform(mesh, G, st, c, q)
    om, w = oracle.quadrature(npol, naz)
    return oracle.Oracle(mesh.xyz, mesh.cell_vert, om, w, mat.sigma_t, mat.sigma_s, mat.q, **kw)


def test_box_cell_closed_forms():
    hx, hy, hz = 0.5, 0.25, 2.0
    m = H.affine_mesh(1, np.diag([hx, hy, hz]), t=(0.3, -1.0, 2.0), permute=False)
    g = _oracle_for(m).geometry()
    m1, d1 = H.ref_1d()
    mx, my, mz = m1 * hx / 2, m1 * hy / 2, m1 * hz / 2     # physical 1D mass on [0, h]
    kx, ky, kz = d1, d1, d1                                 # int f_a f_b' is scale free
    assert np.abs(g["M"][0] - H.kron3(mx, my, mz)).max() < 1e-15
    assert np.abs(g["S"][0, 0] - H.kron3(kx, my, mz)).max() < 1e-15
    assert np.abs(g["S"][0, 1] - H.kron3(mx, ky, mz)).max() < 1e-15
    assert np.abs(g["S"][0, 2] - H.kron3(mx, my, kz)).max() < 1e-15
    # faces: F^a on face 2*axis+side is +-(face mass) in component `axis` only
    face_mass = {0: np.kron(mz, my), 1: np.kron(mz, mx), 2: np.kron(my, mx)}
    area = {0: hy * hz, 1: hx * hz, 2: hx * hy}
    for f in range(6):
        axis, side = divmod(f, 2)
        sgn = 1.0 if side else -1.0
        for a in range(3):
            want = sgn * face_mass[axis] if a == axis else np.zeros((4, 4))
            assert np.abs(g["F"][0, f, a] - want).max() < 1e-15
        assert np.abs(g["area"][0, f] - sgn * area[axis] * np.eye(3)[axis]).max() < 1e-15


def test_affine_cell_closed_forms():
    L = np.array([[1.0, 0.3, -0.2], [0.1, 0.8, 0.25], [-0.15, 0.2, 1.2]]) * 0.5
    m = H.affine_mesh(3, L, t=(0.1, 0.2, 0.3), seed=5)
    g = _oracle_for(m).geometry()
    J = L / 3 / 2                       # d x / d xi for a cell of the 3^3 grid on [-1,1]^3
    detJ = np.linalg.det(J)
    m1, d1 = H.ref_1d()
    Mref = H.kron3(m1, m1, m1)
    Dref = [H.kron3(d1, m1, m1), H.kron3(m1, d1, m1), H.kron3(m1, m1, d1)]
    Jinv = np.linalg.inv(J)
    for K in range(m.ncell):
        assert np.abs(g["M"][K] - detJ * Mref).max() < 1e-15
        for a in range(3):
            want = detJ * sum(Jinv[b, a] * Dref[b] for b in range(3))
            assert np.abs(g["S"][K, a] - want).max() < 1e-14
    assert abs(g["M"].sum() - np.linalg.det(L)) < 1e-13


@pytest.fixture(scope="module")
def jittered():
    m = inputs.make_mesh(5, 0.2, seed=11)
    o = _oracle_for(m, G=2, st=1.0, c=0.5, npol=2, naz=2)
    return m, o, o.geometry()


def test_jittered_volume_and_closed_cells(jittered):
    m, o, g = jittered
    assert abs(g["M"].sum() - 1.0) < 1e-13                      # unit cube
    assert np.abs(g["area"].sum(axis=1)).max() < 1e-15          # closed surface
    # boundary faces tile the cube surface: total |A| = 6
    bnd = g["nbr"] < 0
    assert bnd.sum() == 6 * m.n ** 2
    assert abs(np.linalg.norm(g["area"][bnd], axis=1).sum() - 6.0) < 1e-13


def test_divergence_identity_and_linear_exactness(jittered):
    m, o, g = jittered
    for K in range(m.ncell):
        X = m.xyz[m.cell_vert[K]]                                # nodal coordinates
        rowsumM = g["M"][K].sum(axis=1)
        for a in range(3):
            # sum_i S^a_ij = boundary integral of f_j n_a
            lhs = g["S"][K, a].sum(axis=0)
            rhs = np.zeros(8)
            for f in range(6):
                fn = H.face_nodes(f)
                rhs[fn] += g["F"][K, f, a].sum(axis=0)
            assert np.abs(lhs - rhs).max() < 1e-15
            # S^a applied to the coordinate x_b gives delta_ab int f_i
            for b in range(3):
                want = rowsumM if a == b else 0.0
                assert np.abs(g["S"][K, a] @ X[:, b] - want).max() < 1e-15
        # constants are in the kernel of every S^a
        assert np.abs(g["S"][K].sum(axis=2)).max() < 1e-15


def test_face_matching_and_antisymmetry(jittered):
    m, o, g = jittered
    for K in range(m.ncell):
        for f in range(6):
            N = g["nbr"][K, f]
            if N < 0:
                continue
            fg = g["nbr_face"][K, f]
            assert g["nbr"][N, fg] == K
            fnK, fnN = H.face_nodes(f), H.face_nodes(fg)
            pos = [fnN.index(p) for p in g["perm"][K, f]]
            for k in range(4):
                assert m.cell_vert[K, fnK[k]] == m.cell_vert[N, g["perm"][K, f, k]]
            assert np.array_equal(g["area"][N, fg], -g["area"][K, f])
            for a in range(3):
                FN = g["F"][N, fg, a][np.ix_(pos, pos)]
                assert np.array_equal(FN, -g["F"][K, f, a])


# ------------------------------------------------------------------------ DAG

def _structured_levels(ijk, n, o):
    r = ijk.copy()
    for d in range(3):
        if (o >> d) & 1:
            r[:, d] = n - 1 - r[:, d]
    return r.sum(axis=1)


@pytest.mark.parametrize("n,seed", [(4, 1), (7, 2), (16, 3)])
def test_levels_match_structured_wavefronts(n, seed):
    m = inputs.make_mesh(n, 0.2, seed=seed)
    d = _oracle_for(m).dag()
    for o in range(8):
        assert np.array_equal(d["level"][o], _structured_levels(m.ijk, n, o))
        hist = np.bincount(d["level"][o])
        want = [sum(1 for i, j, k in itertools.product(range(n), repeat=3) if i + j + k == l)
                for l in range(3 * n - 2)]
        assert hist.tolist() == want


def test_topological_order_respects_inflow():
    m = inputs.make_mesh(6, 0.2, seed=4)
    o = _oracle_for(m)
    d, g = o.dag(), o.geometry()
    for oc in range(8):
        pos = np.empty(m.ncell, int)
        pos[d["order"][oc]] = np.arange(m.ncell)
        for K in range(m.ncell):
            for f in range(6):
                N = g["nbr"][K, f]
                if N >= 0 and (d["inflow"][oc, K] >> f) & 1:
                    assert pos[N] < pos[K]
                    assert not (d["inflow"][oc, N] >> g["nbr_face"][K, f]) & 1


def test_paper_grid_level_histogram_golden():
    """16^3 grid: elements per t-level (the shape compared against core counts in Fig. 4)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "levels_16cubed.txt")
    want = [int(x) for x in open(path).read().split("#")[0].split()]
    m = inputs.make_mesh(16, 0.2, seed=7)
    d = _oracle_for(m).dag()
    for o in range(8):
        assert np.bincount(d["level"][o]).tolist() == want


# ---------------------------------------------------------------------- sweep

@pytest.mark.parametrize("n,npol,naz", [(3, 1, 1), (4, 2, 2), (5, 3, 4)])
def test_constant_solution_pure_absorber(n, npol, naz):
    m = inputs.make_mesh(n, 0.2, seed=n)
    G = 3
    st = np.array([0.5, 1.0, 7.0])
    mat = inputs.Materials(np.tile(st, (m.ncell, 1)), np.zeros((m.ncell, G)), np.ones((m.ncell, G)))
    om, w = oracle.quadrature(npol, naz)
    psib = 1.0 / (FOUR_PI * st)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, mat.sigma_t, mat.sigma_s, mat.q, 1, psib)
    r = o.sweep(None, want_psi=True)
    assert np.abs(r["psi"] / psib[None, None, :, None] - 1).max() < 1e-13
    assert np.abs(r["phi"] / (1.0 / st)[None, :, None] - 1).max() < 1e-13


def test_linear_solution_is_exact():
    m = inputs.make_mesh(4, 0.2, seed=9)
    G, npol, naz = 2, 2, 2
    om, w = oracle.quadrature(npol, naz)
    nang = om.shape[0]
    st = np.array([0.7, 3.0])
    a0 = np.array([2.0, 1.0])
    bvec = np.array([[0.3, -0.5, 0.8], [-1.0, 0.2, 0.4]])
    X = m.xyz[m.cell_vert]                                   # [C][8][3]
    exact = a0[None, :, None] + np.einsum("gd,kjd->kgj", bvec, X)   # [C][G][8]
    src = np.zeros((m.ncell, nang, G, 8))
    for n in range(nang):
        src[:, n] = st[None, :, None] * exact + (bvec @ om[n])[None, :, None]
    bnd = np.zeros((m.ncell, 6, nang, G, 4))
    for f in range(6):
        fn = H.face_nodes(f)
        bnd[:, f] = exact[:, None, :, :][..., fn]
    mat = inputs.Materials(np.tile(st, (m.ncell, 1)), np.zeros((m.ncell, G)), np.zeros((m.ncell, G)))
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, mat.sigma_t, mat.sigma_s, mat.q, ang_src=src, bnd_in=bnd)
    r = o.sweep(None, want_psi=True)
    assert np.abs(r["psi"] - exact[None]).max() < 1e-12


@pytest.mark.parametrize("n", [2, 3])
def test_sweep_equals_dense_solve_per_angle(n):
    m = inputs.make_mesh(n, 0.2, seed=20 + n)
    G = 2
    rng = np.random.default_rng(5)
    st = rng.uniform(0.2, 5.0, (m.ncell, G))
    ss = st * rng.uniform(0, 0.9, (m.ncell, G))
    q = rng.uniform(0, 1, (m.ncell, G))
    om, w = oracle.quadrature(2, 2)
    psib = np.array([0.3, 0.05])
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, 1, psib)
    g, d = o.geometry(), o.dag()
    phi_in = rng.uniform(0, 2, (m.ncell, G, 8))
    r = o.sweep(phi_in, want_psi=True)
    for n_ang in range(om.shape[0]):
        for gg in range(G):
            A = H.dense_angle_matrix(g, d, om, n_ang, om.shape[0], st[:, gg])
            qn = (q[:, gg, None] + ss[:, gg, None] * phi_in[:, gg, :]) / FOUR_PI
            rhs = np.einsum("kij,kj->ki", g["M"], qn).ravel()
            rhs += H.boundary_rhs(g, d, om, n_ang, om.shape[0], psib[gg])
            x = np.linalg.solve(A, rhs).reshape(m.ncell, 8)
            assert np.abs(x - r["psi"][n_ang, :, gg]).max() < 1e-12 * max(1, np.abs(x).max())
            # the single-(angle, group) sweep used to check large problems on samples
            xa = o.sweep_angle(phi_in, n_ang, gg)
            assert np.abs(x - xa).max() < 1e-12 * max(1, np.abs(x).max())


def test_full_system_with_scattering_equals_converged_iteration():
    m = inputs.make_mesh(2, 0.2, seed=31)
    om, w = oracle.quadrature(2, 2)
    nang = om.shape[0]
    C = m.ncell
    st = np.full((C, 1), 1.3)
    ss = np.full((C, 1), 0.9)
    q = np.full((C, 1), 1.0)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q)
    g, d = o.geometry(), o.dag()
    nu = 8 * C
    big = np.zeros((nang * nu, nang * nu))
    rhs = np.zeros(nang * nu)
    Mblk = np.zeros((nu, nu))
    for K in range(C):
        Mblk[8 * K:8 * K + 8, 8 * K:8 * K + 8] = g["M"][K]
    for n in range(nang):
        big[n * nu:(n + 1) * nu, n * nu:(n + 1) * nu] = H.dense_angle_matrix(g, d, om, n, nang, st[:, 0])
        for mm in range(nang):   # scattering couples every pair of angles
            big[n * nu:(n + 1) * nu, mm * nu:(mm + 1) * nu] -= 0.9 / FOUR_PI * w[mm] * Mblk
        rhs[n * nu:(n + 1) * nu] = Mblk @ np.full(nu, 1.0 / FOUR_PI)
    psi = np.linalg.solve(big, rhs).reshape(nang, C, 8)
    phi_dense = np.einsum("n,nkj->kj", w, psi)
    s = o.solve(1e-14, 2000)
    assert np.abs(s["phi"][:, 0, :] - phi_dense).max() < 1e-11 * np.abs(phi_dense).max()


def test_infinite_medium_fixed_point():
    m = inputs.make_mesh(4, 0.2, seed=13)
    G = 2
    st, c, Q = np.array([1.0, 4.0]), np.array([0.5, 0.95]), np.array([1.0, 2.0])
    mat = inputs.Materials(np.tile(st, (m.ncell, 1)), np.tile(c * st, (m.ncell, 1)), np.tile(Q, (m.ncell, 1)))
    sa = st * (1 - c)
    psib = Q / (FOUR_PI * sa)
    om, w = oracle.quadrature(2, 4)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, mat.sigma_t, mat.sigma_s, mat.q, 1, psib)
    phi0 = np.broadcast_to((Q / sa)[None, :, None], (m.ncell, G, 8)).copy()
    r = o.sweep(phi0)
    assert np.abs(r["phi"] / phi0 - 1).max() < 1e-13


def test_balance_per_angle_per_cell_and_global():
    m = inputs.make_mesh(4, 0.2, seed=17)
    G = 2
    rng = np.random.default_rng(3)
    st = rng.uniform(0.1, 10, (m.ncell, G))
    ss = st * rng.uniform(0, 0.95, (m.ncell, G))
    q = rng.uniform(0, 1, (m.ncell, G))
    om, w = oracle.quadrature(2, 2)
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q)
    g = o.geometry()
    phi_in = rng.uniform(0, 1, (m.ncell, G, 8))
    r = o.sweep(phi_in, want_psi=True, want_leak=True, want_leak_ang=True)
    ones = np.ones(8)
    for n in range(om.shape[0]):
        for gg in range(G):
            qn = (q[:, gg, None] + ss[:, gg, None] * phi_in[:, gg]) / FOUR_PI
            rhs = np.einsum("kij,kj->k", g["M"], qn)
            absn = st[:, gg] * np.einsum("i,kij,kj->k", ones, g["M"], r["psi"][n, :, gg])
            lhs = r["leak_ang"][n, :, gg] + absn
            assert np.abs(lhs - rhs).max() < 1e-14 * max(1, np.abs(rhs).max())
    b = o.balance(phi_in, r["phi"], r["leak"])
    assert b[:, 3].max() < 1e-13
    assert np.abs(b[:, 0] - b[:, 1] - b[:, 2]).max() < 1e-13 * np.abs(b[:, 0]).max()
    # interior faces cancel: global leakage = outflow through boundary faces only
    bl = np.zeros(G)
    dag = o.dag()
    for n in range(om.shape[0]):
        oc = n // (om.shape[0] // 8)
        for K in range(m.ncell):
            for f in range(6):
                if g["nbr"][K, f] >= 0 or (dag["inflow"][oc, K] >> f) & 1:
                    continue
                OF = np.einsum("a,akl->kl", om[n], g["F"][K, f])
                fn = H.face_nodes(f)
                for gg in range(G):
                    bl[gg] += w[n] * (OF @ r["psi"][n, K, gg][fn]).sum()
    assert np.abs(bl - b[:, 2]).max() < 1e-13 * np.abs(bl).max()


def test_cell_renumbering_invariance():
    base = inputs.make_mesh(4, 0.2, seed=41, permute=False)
    rng = np.random.default_rng(2)
    perm = rng.permutation(base.ncell)
    G = 2
    st = rng.uniform(0.5, 2, (base.ncell, G))
    ss = st * 0.5
    q = rng.uniform(0, 1, (base.ncell, G))
    om, w = oracle.quadrature(2, 2)
    o1 = oracle.Oracle(base.xyz, base.cell_vert, om, w, st, ss, q)
    o2 = oracle.Oracle(base.xyz, base.cell_vert[perm], om, w, st[perm], ss[perm], q[perm])
    p1 = o1.sweep(None)["phi"]
    p2 = o2.sweep(None)["phi"]
    assert np.abs(p2 - p1[perm]).max() < 1e-14 * np.abs(p1).max()


def test_reflection_and_swap_symmetry():
    n = 4
    m = inputs.make_mesh(n, 0.0, seed=0, permute=False)
    o = _oracle_for(m, G=1, st=1.0, c=0.5, q=1.0, npol=2, naz=4)
    phi = o.solve(1e-13, 500)["phi"][:, 0, :]
    idx = {tuple(ijk): K for K, ijk in enumerate(m.ijk)}
    for K, (i, j, k) in enumerate(m.ijk):
        for axis in range(3):                       # mirror in one axis
            r = [i, j, k]
            r[axis] = n - 1 - r[axis]
            K2 = idx[tuple(r)]
            for jj in range(8):
                assert abs(phi[K, jj] - phi[K2, jj ^ (1 << axis)]) < 1e-12
        K3 = idx[(j, i, k)]                         # swap x and y
        for jj in range(8):
            a, b, c = jj & 1, (jj >> 1) & 1, jj >> 2
            assert abs(phi[K, jj] - phi[K3, b + 2 * a + 4 * c]) < 1e-12


def test_contraction_ratio_bounded_by_scattering_ratio():
    m = inputs.make_mesh(4, 0.2, seed=8)
    o = _oracle_for(m, G=1, st=2.0, c=0.8, npol=2, naz=2)
    s = o.solve(1e-12, 300)
    h = s["hist"]
    ratios = h[2:] / h[1:-1]
    assert ratios.max() <= 0.8 + 1e-9


def test_integrated_flux_identical_groups():
    m = inputs.make_mesh(3, 0.2, seed=6)
    o = _oracle_for(m, G=3, st=1.0, c=0.5, npol=1, naz=2)
    phi = o.solve(1e-12, 300)["phi"]
    fl = o.integrated_flux(phi)
    assert np.abs(fl[:, 0] - phi.sum(axis=(0, 2))).max() < 1e-12
    assert np.allclose(fl[0], fl[1], rtol=0, atol=0) and np.allclose(fl[1], fl[2], rtol=0, atol=0)
    # infinite-medium bound: volume integral of phi below Q / sigma_a over the unit cube
    assert 0 < fl[0, 1] < 1.0 / (1.0 * 0.5)


@pytest.mark.parametrize("jittered", [False, True])
def test_integrated_flux_volume_integral_closed_forms(jittered):
    """The volume column of Eq. 3's integrated flux, 1^T M phi per group, is the
    integral of the trilinear field phi over the mesh.  It holds exactly under
    the 2x2x2 rule: 1^T M phi = sum_q detJ phi_h (the basis sums to one), and
    phi_h detJ has degree at most 3 in each reference coordinate.  A linear
    function a + b.x is reproduced by its nodal values on any trilinear cell,
    so the unit cube gives a + b.(1/2, 1/2, 1/2); a constant gives itself.  The
    plain column is the sum of the nodal values."""
    m = inputs.make_mesh(4, 0.3 if jittered else 0.0, seed=13)
    C = m.ncell
    coefs = np.array([[2.5, 0.0, 0.0, 0.0],       # constant
                      [0.3, 1.0, -2.0, 0.5],      # linear
                      [-1.0, 0.25, 3.0, -4.0]])
    G = len(coefs)
    o = _oracle_for(m, G=G)
    X = m.xyz[m.cell_vert]                         # [C][8][3]: node j of cell K is its vertex j
    phi = coefs[None, :, None, 0] + np.einsum("gd,kjd->kgj", coefs[:, 1:], X)
    fl = o.integrated_flux(phi)
    want = coefs[:, 0] + coefs[:, 1:].sum(axis=1) * 0.5
    assert np.abs(fl[:, 1] - want).max() < 1e-13
    assert np.abs(fl[:, 0] - phi.sum(axis=(0, 2))).max() < 1e-12 * np.abs(phi).sum()
    # per cell the column is the cell's volume for phi = 1 (the volumes tile the cube)
    vol = o.integrated_flux(np.ones((C, G, 8)))[:, 1]
    assert np.abs(vol - 1.0).max() < 1e-14
    # a wrong weighting fails: dropping the Jacobian's variation or using a diagonal of M
    g = o.geometry()
    lumped = np.einsum("kii,kgi->g", g["M"], phi)
    if jittered:
        assert np.abs(lumped - want).max() > 1e-4


def test_regression_golden_solution():
    """A tiny converged solve pinned in tests/golden (written by make_golden.py from the oracle)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "tiny_solve.txt")
    vals = np.loadtxt(path)
    from tests.golden.make_golden import tiny_problem
    o, tol = tiny_problem()
    phi = o.solve(tol, 500)["phi"]
    fl = o.integrated_flux(phi)
    assert np.abs(fl.ravel() - vals).max() < 1e-12 * np.abs(vals).max()
