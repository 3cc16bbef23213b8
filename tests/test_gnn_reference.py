"""Pins of the FP64 reference of the message-passing network (CPU only)."""
import numpy as np

import oracle
from oracle import gnn
from paper_2510_11513_amd import inputs


def _tiny_graph(n=3, G=2, seed=0):
    m = inputs.make_mesh(n, 0.2, seed=seed)
    o = oracle.Oracle(m.xyz, m.cell_vert, *oracle.quadrature(1, 1), np.ones((m.ncell, G)),
                      np.full((m.ncell, G), 0.5), np.ones((m.ncell, G)))
    g = o.geometry()
    return m, g["nbr"], g["M"].sum(axis=(1, 2)), (g["nbr"] < 0).sum(axis=1)


def _position(m):
    """Cell centroids and the mesh's bounding box."""
    return m.xyz[m.cell_vert].mean(axis=1), m.xyz.min(axis=0), m.xyz.max(axis=0)


def test_backward_matches_central_finite_differences():
    m, nbr, vol, nb = _tiny_graph()
    rng = np.random.default_rng(1)
    hidden, layers = 8, 3
    G = 2
    st = rng.uniform(0.1, 10, (m.ncell, G))
    ss = st * rng.uniform(0.9, 0.99, (m.ncell, G))
    q = rng.uniform(0, 1, (m.ncell, G))
    x = gnn.features(st, ss, q, vol, nb, *_position(m))
    y = rng.normal(0, 1, (m.ncell, G))
    theta = gnn.init_params(3, hidden, layers) + rng.normal(0, 0.05, gnn.pack(
        {k: np.zeros(s) for k, s in gnn.param_shapes(hidden, layers)}, hidden, layers).shape)
    loss, g = gnn.loss_and_grad(theta, x, nbr, y, hidden, layers)
    eps = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (gnn.loss_and_grad(tp, x, nbr, y, hidden, layers)[0] - gnn.loss_and_grad(tm, x, nbr, y, hidden, layers)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_neighbour_mean_and_isolated_cell():
    _, nbr, _, _ = _tiny_graph(1, 1)          # one cell: no neighbours, the mean is zero
    h = np.ones((1, 1, 4))
    mm, deg = gnn._neighbour_mean(h, nbr)
    assert deg[0] == 0 and np.all(mm == 0)
    m, nbr, _, _ = _tiny_graph(3, 1)
    h = np.arange(m.ncell, dtype=float)[:, None, None] * np.ones((1, 1, 2))
    mm, deg = gnn._neighbour_mean(h, nbr)
    for K in range(m.ncell):
        ns = [N for N in nbr[K] if N >= 0]
        assert abs(mm[K, 0, 0] - np.mean(ns)) < 1e-12 and deg[K] == len(ns)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -2.5, 1e-3])
    r = gnn.round_bf16(vals)
    # bfloat16 keeps 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 and goes to
    # the even mantissa (1); 1 + 2^-9 rounds down; 1 + 3*2^-9 rounds up to 1 + 2^-7
    assert r[0] == 1.0 and r[1] == 1.0
    assert r[2] == 1.0
    assert r[3] == 1.0 + 2 ** -7
    assert r[4] == -2.5
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8


def test_position_features_on_a_regular_grid():
    # unjittered n^3 grid of the unit cube: centroids (i + 1/2)/n, box [0, 1]^3
    n = 4
    m = inputs.make_mesh(n, 0.0, seed=0)
    G = 1
    one = np.ones((m.ncell, G))
    x = gnn.features(one, 0.5 * one, one, np.full(m.ncell, 1.0 / n ** 3), np.zeros(m.ncell), *_position(m))
    cen = m.xyz[m.cell_vert].mean(axis=1)
    idx = np.rint(cen * n - 0.5)
    assert np.abs(x[:, 0, 8:11] - (idx + 0.5) / n).max() < 1e-12
    assert np.abs(x[:, 0, 7] - np.minimum(idx + 0.5, n - idx - 0.5).min(axis=1) / n).max() < 1e-12
    # sigma_t = 1, c = 1/2, h = 1/n: log(sigma_t h) and log(sigma_a h)
    assert np.abs(x[:, 0, 5] - np.log(1.0 / n)).max() < 1e-12
    assert np.abs(x[:, 0, 11] - np.log(0.5 / n)).max() < 1e-12
