"""Pins of the oracle's per-angle upwind designation (CPU, FP64).

Designation 1 makes face f of cell K inflow for angle n when Omega_n . A_f < 0
(each direction's own mesh traversal, Section 2.1).  On jittered meshes these
per-angle graphs can contain cycles.  The sweep keeps the octant's topological
order, and an inflow face whose neighbour comes later in that order uses the
neighbour's angular flux of the previous sweep.

Each check uses an algorithm other than the oracle's sweep:

* the masks against numpy signs of the area vectors;
* one lagged sweep against a block Gauss-Seidel step of the dense global
  system, split by the octant order;
* the converged iteration against the dense global solve, where cycles need
  no special treatment;
* constant preservation and the per-cell balance.

Designation 2 sweeps each direction in its own topological order and lags
only faces inside the strongly connected components of its graph.  Its checks:

* the components against scipy's strong components;
* the lagged faces lie inside components and go down in upwind rank, and the
  order is a topological order of the remaining graph;
* one sweep against (A - U)^-1 (b - U x_prev), U holding only the lagged
  couplings of the dense global system;
* convergence to the same dense solution as designation 1, with as many
  iterations as per-octant designation needs;
* bitwise equality with per-octant designation on an orthogonal mesh, and
  invariance under cell renumbering.
"""
import numpy as np
import pytest

import oracle
from paper_2510_11513_amd import inputs
from tests import helpers as H

FOUR_PI = 4 * np.pi


def _cycle_mesh():
    """4^3 cells, jitter 0.3, seed 0, 48 directions: two directions have
    dependency cycles of their own."""
    return inputs.make_mesh(4, 0.3, seed=0), oracle.quadrature(2, 3)


def _problem(m, om, w, G=2, seed=1, boundary=0, psib=None, designation=1, c_max=0.9):
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.2, 5.0, (m.ncell, G))
    ss = st * rng.uniform(0, c_max, (m.ncell, G))
    q = rng.uniform(0, 1, (m.ncell, G))
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, ss, q, boundary, psib, designation=designation)
    return o, st, ss, q


def _numpy_masks(geo, om):
    """[nang][C] bit masks of the faces with Omega_n . A_f < 0."""
    dots = np.einsum("kfa,na->nkf", geo["area"], om)
    assert np.abs(dots).min() > 0
    return ((dots < 0) * (1 << np.arange(6))).sum(axis=2)


def _has_cycle(mask_n, nbr):
    """Kahn's algorithm on one direction's graph: True if it cannot order every cell."""
    C = len(mask_n)
    indeg = np.zeros(C, int)
    down = [[] for _ in range(C)]
    for K in range(C):
        for f in range(6):
            N = nbr[K, f]
            if N >= 0 and (mask_n[K] >> f) & 1:
                indeg[K] += 1
                down[N].append(K)
    stack = [K for K in range(C) if indeg[K] == 0]
    seen = 0
    while stack:
        K = stack.pop()
        seen += 1
        for D in down[K]:
            indeg[D] -= 1
            if indeg[D] == 0:
                stack.append(D)
    return seen < C


def test_angle_masks_are_the_signs_of_omega_dot_area():
    m, (om, w) = _cycle_mesh()
    o, *_ = _problem(m, om, w)
    geo = o.geometry()
    assert np.array_equal(o.angle_inflow(), _numpy_masks(geo, om))


def test_orthogonal_mesh_per_angle_equals_per_octant():
    """Axis-aligned faces: every direction of an octant has the octant's signs, so
    no face is lagged and the previous sweep's flux has no effect."""
    m = inputs.make_mesh(3, 0.0, seed=4)
    om, w = oracle.quadrature(2, 2)
    o1, st, ss, q = _problem(m, om, w, seed=2)
    o0, *_ = _problem(m, om, w, seed=2, designation=0)
    per = om.shape[0] // 8
    ain, inflow = o1.angle_inflow(), o0.dag()["inflow"]
    for n in range(om.shape[0]):
        assert np.array_equal(ain[n], inflow[n // per])
    rng = np.random.default_rng(9)
    phi_in = rng.uniform(0, 2, (m.ncell, 2, 8))
    psi_prev = rng.uniform(-5, 5, (om.shape[0], m.ncell, 2, 8))
    r1 = o1.sweep(phi_in, want_psi=True, psi_prev=psi_prev)
    r0 = o0.sweep(phi_in, want_psi=True)
    assert np.array_equal(r1["psi"], r0["psi"])


def test_test_mesh_has_per_angle_cycles_and_lagged_faces():
    m, (om, w) = _cycle_mesh()
    o, *_ = _problem(m, om, w)
    geo, dag = o.geometry(), o.dag()
    ain = o.angle_inflow()
    per = om.shape[0] // 8
    interior = ((geo["nbr"] >= 0) * (1 << np.arange(6))).sum(axis=1)
    lagged = sum(int(((ain[n] & ~dag["inflow"][n // per] & interior) != 0).sum()) for n in range(om.shape[0]))
    cycles = sum(_has_cycle(ain[n], geo["nbr"]) for n in range(om.shape[0]))
    assert lagged > 100 and cycles >= 1, (lagged, cycles)


@pytest.mark.parametrize("boundary", [0, 1])
def test_lagged_sweep_is_a_block_gauss_seidel_step(boundary):
    """x = (D + L)^-1 (b - U x_prev), with L the couplings to cells earlier in the
    octant's order and U those to later cells."""
    m, (om, w) = _cycle_mesh()
    G = 2
    psib = np.array([0.4, 0.1])
    o, st, ss, q = _problem(m, om, w, G=G, seed=3, boundary=boundary, psib=psib if boundary else None)
    geo, dag = o.geometry(), o.dag()
    masks = _numpy_masks(geo, om)
    rng = np.random.default_rng(12)
    phi_in = rng.uniform(0, 2, (m.ncell, G, 8))
    psi_prev = rng.uniform(0, 1, (om.shape[0], m.ncell, G, 8))
    r = o.sweep(phi_in, want_psi=True, psi_prev=psi_prev)
    nang, per, C = om.shape[0], om.shape[0] // 8, m.ncell
    for n in range(nang):
        pos = np.empty(C, int)
        pos[dag["order"][n // per]] = np.arange(C)
        later = np.repeat(pos[:, None] < pos[None, :], 8, axis=0).repeat(8, axis=1)   # block (K, N): N after K
        for g in range(G):
            A = H.dense_angle_matrix(geo, dag, om, n, nang, st[:, g], masks=masks[n])
            qn = (q[:, g, None] + ss[:, g, None] * phi_in[:, g, :]) / FOUR_PI
            rhs = np.einsum("kij,kj->ki", geo["M"], qn).ravel()
            if boundary:
                rhs += H.boundary_rhs(geo, dag, om, n, nang, psib[g], masks=masks[n])
            U = np.where(later, A, 0.0)
            x = np.linalg.solve(A - U, rhs - U @ psi_prev[n, :, g].ravel()).reshape(C, 8)
            assert np.abs(x - r["psi"][n, :, g]).max() < 1e-12 * max(1, np.abs(x).max()), (n, g)
            xa = o.sweep_angle(phi_in, n, g, psi_prev=psi_prev[n, :, g])
            assert np.abs(x - xa).max() < 1e-12 * max(1, np.abs(x).max()), (n, g)
    # the previous sweep's flux does enter: a lagged face exists
    r0 = o.sweep(phi_in, want_psi=True)
    assert np.abs(r0["psi"] - r["psi"]).max() > 1e-3


def test_lagged_iteration_converges_to_the_dense_solution():
    """Source iteration with lagged faces reaches the per-angle upwind DG solution
    (one dense solve per direction and group, cycles included)."""
    m, (om, w) = _cycle_mesh()
    G = 2
    o, st, ss, q = _problem(m, om, w, G=G, seed=5, c_max=0.0)   # no scattering: phi_in plays no part
    geo, dag = o.geometry(), o.dag()
    masks = _numpy_masks(geo, om)
    nang = om.shape[0]
    phi_dense = np.zeros((m.ncell, G, 8))
    for n in range(nang):
        for g in range(G):
            A = H.dense_angle_matrix(geo, dag, om, n, nang, st[:, g], masks=masks[n])
            rhs = np.einsum("kij,kj->ki", geo["M"], np.repeat(q[:, g, None] / FOUR_PI, 8, axis=1)).ravel()
            phi_dense[:, g] += w[n] * np.linalg.solve(A, rhs).reshape(m.ncell, 8)
    s = o.solve(1e-14, 500)
    assert s["status"] == 0 and s["iters"] > 2, s["iters"]   # the lag needs iterations even without scattering
    assert np.abs(s["phi"] - phi_dense).max() < 1e-11 * np.abs(phi_dense).max()
    # per-octant designation converges to a different discrete solution on this mesh
    o0, *_ = _problem(m, om, w, G=G, seed=5, c_max=0.0, designation=0)
    assert np.abs(o0.solve(1e-14, 500)["phi"] - phi_dense).max() > 1e-6 * np.abs(phi_dense).max()


def test_constant_flux_is_a_fixed_point_of_the_lagged_sweep():
    """psi = psi_b everywhere solves Omega.grad psi + sigma_t psi = sigma_t psi_b with
    inflow psi_b; the lagged sweep reproduces it when the previous sweep held it."""
    m, (om, w) = _cycle_mesh()
    G = 2
    psib = np.array([0.7, 1.3])
    rng = np.random.default_rng(6)
    st = rng.uniform(0.2, 5.0, (m.ncell, G))
    o = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, np.zeros((m.ncell, G)), FOUR_PI * st * psib, 1, psib,
                      designation=1)
    const = np.broadcast_to(psib[None, None, :, None], (om.shape[0], m.ncell, G, 8)).copy()
    r = o.sweep(None, want_psi=True, psi_prev=const)
    assert np.abs(r["psi"] - const).max() < 1e-12
    r0 = o.sweep(None, want_psi=True)
    assert np.abs(r0["psi"] - const).max() > 1e-3


def test_balance_of_a_lagged_sweep():
    """Per (angle, cell, group): source = absorption + net outflow, with the traces
    the sweep used (previous-sweep values on lagged faces)."""
    m, (om, w) = _cycle_mesh()
    G = 2
    o, st, ss, q = _problem(m, om, w, G=G, seed=8)
    geo = o.geometry()
    rng = np.random.default_rng(10)
    phi_in = rng.uniform(0, 1, (m.ncell, G, 8))
    psi_prev = rng.uniform(0, 1, (om.shape[0], m.ncell, G, 8))
    r = o.sweep(phi_in, want_psi=True, want_leak=True, want_leak_ang=True, psi_prev=psi_prev)
    ones = np.ones(8)
    for n in range(om.shape[0]):
        for g in range(G):
            qn = (q[:, g, None] + ss[:, g, None] * phi_in[:, g]) / FOUR_PI
            src = np.einsum("kij,kj->k", geo["M"], qn)
            absn = st[:, g] * np.einsum("i,kij,kj->k", ones, geo["M"], r["psi"][n, :, g])
            assert np.abs(r["leak_ang"][n, :, g] + absn - src).max() < 1e-13 * max(1, np.abs(src).max())
    b = o.balance(phi_in, r["phi"], r["leak"])
    assert b[:, 3].max() < 1e-12


# ------------------------------------------------ designation 2: own order

def _graph(ain_n, nbr):
    """Edges (N, K) of one direction: K depends on its neighbour N."""
    C = len(ain_n)
    return [(nbr[K, f], K, f) for K in range(C) for f in range(6) if nbr[K, f] >= 0 and (ain_n[K] >> f) & 1]


def _centroid_key(m, om_n):
    return m.xyz[m.cell_vert].mean(axis=1) @ om_n


def test_direction_order_lags_only_inside_strong_components():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    m, (om, w) = _cycle_mesh()
    o2, *_ = _problem(m, om, w, designation=2)
    o1, *_ = _problem(m, om, w, designation=1)
    geo = o2.geometry()
    ain = o2.angle_inflow()
    order, lag = o2.angle_order()
    C = m.ncell
    cyclic = 0
    for n in range(om.shape[0]):
        edges = _graph(ain[n], geo["nbr"])
        A = csr_matrix((np.ones(len(edges)), ([e[0] for e in edges], [e[1] for e in edges])), shape=(C, C))
        _, comp = connected_components(A, directed=True, connection="strong")
        key = _centroid_key(m, om[n])
        pos = np.empty(C, int)
        pos[order[n]] = np.arange(C)
        assert sorted(order[n]) == list(range(C))
        nlag = 0
        for N, K, f in edges:
            if (lag[n, K] >> f) & 1:
                nlag += 1
                assert comp[N] == comp[K] and key[N] > key[K], (n, N, K)
            else:
                assert pos[N] < pos[K], (n, N, K)         # kept edges respect the order
                assert not (comp[N] == comp[K] and key[N] > key[K])
        # lag bits only on interior inflow faces
        inflow_interior = sum(1 << f for f in range(6))
        assert all((lag[n, K] & ~ain[n, K]) == 0 for K in range(C)) and inflow_interior
        has_cycle = _has_cycle(ain[n], geo["nbr"])
        assert (nlag > 0) == has_cycle, n
        cyclic += has_cycle
    assert cyclic >= 1
    # far fewer lagged faces than the octant-order reading
    dag = o1.dag()
    per = om.shape[0] // 8
    interior = ((geo["nbr"] >= 0) * (1 << np.arange(6))).sum(axis=1)
    lag1 = sum(int(bin(int(x)).count("1")) for n in range(om.shape[0])
               for x in (ain[n] & ~dag["inflow"][n // per] & interior))
    lag2 = sum(int(bin(int(x)).count("1")) for x in lag.ravel())
    assert 0 < lag2 and 10 * lag2 < lag1, (lag2, lag1)


@pytest.mark.parametrize("boundary", [0, 1])
def test_direction_order_sweep_lags_only_the_chosen_faces(boundary):
    """x = (A - U)^-1 (b - U x_prev): U holds the couplings across lagged faces
    only; every other coupling is taken from the current sweep."""
    m, (om, w) = _cycle_mesh()
    G = 2
    psib = np.array([0.4, 0.1])
    o, st, ss, q = _problem(m, om, w, G=G, seed=3, boundary=boundary, psib=psib if boundary else None,
                            designation=2)
    geo, dag = o.geometry(), o.dag()
    masks = _numpy_masks(geo, om)
    _, lag = o.angle_order()
    rng = np.random.default_rng(12)
    phi_in = rng.uniform(0, 2, (m.ncell, G, 8))
    psi_prev = rng.uniform(0, 1, (om.shape[0], m.ncell, G, 8))
    r = o.sweep(phi_in, want_psi=True, psi_prev=psi_prev)
    nang, C = om.shape[0], m.ncell
    lagged_dirs = 0
    for n in range(nang):
        blk = np.zeros((C, C), bool)
        for K in range(C):
            for f in range(6):
                if (lag[n, K] >> f) & 1:
                    blk[K, geo["nbr"][K, f]] = True
        lagged_dirs += blk.any()
        U_mask = np.repeat(np.repeat(blk, 8, axis=0), 8, axis=1)
        for g in range(G):
            A = H.dense_angle_matrix(geo, dag, om, n, nang, st[:, g], masks=masks[n])
            qn = (q[:, g, None] + ss[:, g, None] * phi_in[:, g, :]) / FOUR_PI
            rhs = np.einsum("kij,kj->ki", geo["M"], qn).ravel()
            if boundary:
                rhs += H.boundary_rhs(geo, dag, om, n, nang, psib[g], masks=masks[n])
            U = np.where(U_mask, A, 0.0)
            x = np.linalg.solve(A - U, rhs - U @ psi_prev[n, :, g].ravel()).reshape(C, 8)
            assert np.abs(x - r["psi"][n, :, g]).max() < 1e-12 * max(1, np.abs(x).max()), (n, g)
            xa = o.sweep_angle(phi_in, n, g, psi_prev=psi_prev[n, :, g])
            assert np.abs(x - xa).max() < 1e-12 * max(1, np.abs(x).max()), (n, g)
    assert lagged_dirs >= 1


def test_direction_order_converges_to_the_dense_solution_in_per_octant_iterations():
    m, (om, w) = _cycle_mesh()
    G = 2
    o2, st, ss, q = _problem(m, om, w, G=G, seed=5, c_max=0.0, designation=2)
    geo, dag = o2.geometry(), o2.dag()
    masks = _numpy_masks(geo, om)
    nang = om.shape[0]
    phi_dense = np.zeros((m.ncell, G, 8))
    for n in range(nang):
        for g in range(G):
            A = H.dense_angle_matrix(geo, dag, om, n, nang, st[:, g], masks=masks[n])
            rhs = np.einsum("kij,kj->ki", geo["M"], np.repeat(q[:, g, None] / FOUR_PI, 8, axis=1)).ravel()
            phi_dense[:, g] += w[n] * np.linalg.solve(A, rhs).reshape(m.ncell, 8)
    s2 = o2.solve(1e-14, 500)
    assert s2["status"] == 0
    assert np.abs(s2["phi"] - phi_dense).max() < 1e-11 * np.abs(phi_dense).max()
    # with scattering: the same fixed point as the octant-order reading, and fewer
    # iterations (its many lagged faces slow the iteration)
    o2s, *_ = _problem(m, om, w, G=G, seed=6, designation=2)
    o1s, *_ = _problem(m, om, w, G=G, seed=6, designation=1)
    o0s, *_ = _problem(m, om, w, G=G, seed=6, designation=0)
    a, b, c = o2s.solve(1e-12, 2000), o1s.solve(1e-12, 2000), o0s.solve(1e-12, 2000)
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-10 * np.abs(b["phi"]).max()
    assert a["iters"] <= b["iters"] and a["iters"] <= c["iters"] + 1, (a["iters"], b["iters"], c["iters"])


def test_direction_order_equals_per_octant_on_an_orthogonal_mesh():
    m = inputs.make_mesh(3, 0.0, seed=4)
    om, w = oracle.quadrature(2, 2)
    o2, *_ = _problem(m, om, w, seed=2, designation=2)
    o0, *_ = _problem(m, om, w, seed=2, designation=0)
    assert not o2.angle_order()[1].any()
    rng = np.random.default_rng(9)
    phi_in = rng.uniform(0, 2, (m.ncell, 2, 8))
    psi_prev = rng.uniform(-5, 5, (om.shape[0], m.ncell, 2, 8))
    assert np.array_equal(o2.sweep(phi_in, want_psi=True, psi_prev=psi_prev)["psi"],
                          o0.sweep(phi_in, want_psi=True)["psi"])


def test_direction_order_is_invariant_under_cell_renumbering():
    """The lagged faces are chosen by geometry, so renumbering the cells gives the
    same lagged faces and the same flux (up to the rounding of face matrices,
    which are integrated on the side with the smaller index)."""
    base = inputs.make_mesh(4, 0.3, seed=0, permute=False)
    om, w = oracle.quadrature(2, 3)
    rng = np.random.default_rng(2)
    perm = rng.permutation(base.ncell)
    G = 2
    st = rng.uniform(0.5, 2, (base.ncell, G))
    ss = st * 0.5
    q = rng.uniform(0, 1, (base.ncell, G))
    o1 = oracle.Oracle(base.xyz, base.cell_vert, om, w, st, ss, q, designation=2)
    o2 = oracle.Oracle(base.xyz, base.cell_vert[perm], om, w, st[perm], ss[perm], q[perm], designation=2)
    l1, l2 = o1.angle_order()[1], o2.angle_order()[1]
    assert l1.any() and np.array_equal(l2, l1[:, perm])
    psi_prev = rng.uniform(0, 1, (om.shape[0], base.ncell, G, 8))
    p1 = o1.sweep(None, psi_prev=psi_prev)["phi"]
    p2 = o2.sweep(None, psi_prev=psi_prev[:, perm])["phi"]
    assert np.abs(p2 - p1[perm]).max() < 1e-13 * np.abs(p1).max()


def test_balance_and_constant_flux_under_direction_order():
    m, (om, w) = _cycle_mesh()
    G = 2
    o, st, ss, q = _problem(m, om, w, G=G, seed=8, designation=2)
    rng = np.random.default_rng(10)
    phi_in = rng.uniform(0, 1, (m.ncell, G, 8))
    psi_prev = rng.uniform(0, 1, (om.shape[0], m.ncell, G, 8))
    r = o.sweep(phi_in, want_leak=True, psi_prev=psi_prev)
    assert o.balance(phi_in, r["phi"], r["leak"])[:, 3].max() < 1e-12
    psib = np.array([0.7, 1.3])
    st = rng.uniform(0.2, 5.0, (m.ncell, G))
    oc = oracle.Oracle(m.xyz, m.cell_vert, om, w, st, np.zeros((m.ncell, G)), FOUR_PI * st * psib, 1, psib,
                       designation=2)
    const = np.broadcast_to(psib[None, None, :, None], (om.shape[0], m.ncell, G, 8)).copy()
    assert np.abs(oc.sweep(None, want_psi=True, psi_prev=const)["psi"] - const).max() < 1e-12
