"""FP64 reference of the face-adjacency message-passing network (test infrastructure).

The network predicts, for every (cell, group) node of a mesh, the log of the
converged cell-average scalar flux; the prediction seeds source iteration.
Nodes of one group are joined across shared faces (the mesh's face adjacency;
groups are independent, so the graph is one copy per group).

    h0   = relu(x W_in + b_in)                     x: 12 node features
    m_l  = mean of h_{l-1} over face neighbours    (0 for a cell with none)
    h_l  = relu([h_{l-1}, m_l] W_l + b_l)          W_l: (2H) x H, l = 1..L
    z    = h_L w_out + b_out                       predicted log(phi_avg + delta)
    loss = mean over nodes of (z - y)^2

Parameters are one flat vector in the order W_in, b_in, (W_l, b_l) for l=1..L,
w_out, b_out (row-major matrices).  The backward pass is written by hand and
pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

DELTA = 1e-4
NFEAT = 12


def param_shapes(hidden: int = 64, layers: int = 4):
    shapes = [("W_in", (NFEAT, hidden)), ("b_in", (hidden,))]
    for l in range(1, layers + 1):
        shapes += [(f"W{l}", (2 * hidden, hidden)), (f"b{l}", (hidden,))]
    shapes += [("w_out", (hidden,)), ("b_out", (1,))]
    return shapes


def unpack(theta, hidden=64, layers=4):
    out, i = {}, 0
    for name, shp in param_shapes(hidden, layers):
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[i:i + n], np.float64).reshape(shp)
        i += n
    assert i == len(theta)
    return out


def pack(params, hidden=64, layers=4):
    return np.concatenate([params[name].ravel() for name, _ in param_shapes(hidden, layers)])


def features(sigma_t, sigma_s, q, volume, n_boundary_faces, centroid, lo, hi):
    """Node features [C, G, 12] of a problem: per-cell volume, boundary-face count,
    centroid [C, 3] and the mesh's bounding box lo, hi [3]."""
    st = np.asarray(sigma_t, np.float64)
    ss = np.asarray(sigma_s, np.float64)
    qq = np.asarray(q, np.float64)
    c = ss / st
    sa = st - ss
    one = np.ones_like(st)
    vol = np.asarray(volume, np.float64)[:, None] * one
    nb = np.asarray(n_boundary_faces, np.float64)[:, None] * one
    u = (np.asarray(centroid, np.float64) - np.asarray(lo, np.float64)) / (np.asarray(hi, np.float64)
                                                                          - np.asarray(lo, np.float64))
    db = np.minimum(u, 1.0 - u).min(axis=1)
    h = np.cbrt(vol)
    x = np.stack([np.log(st), c, qq, np.log(qq / sa + 1e-2), nb / 3.0, np.log(st * h),
                  np.log(np.maximum(1.0 - c, 1e-6)), db[:, None] * one,
                  u[:, 0, None] * one, u[:, 1, None] * one, u[:, 2, None] * one,
                  np.log(np.maximum(sa * h, 1e-12))], axis=-1)
    return x


def targets(phi):
    """y = log(mean over the 8 dofs of phi + delta), [C, G]."""
    return np.log(np.asarray(phi, np.float64).mean(axis=-1) + DELTA)


def _neighbour_mean(h, nbr):
    """h: [C, G, H]; mean over interior neighbours of each cell, per group."""
    C = h.shape[0]
    acc = np.zeros_like(h)
    deg = np.zeros(C)
    for f in range(6):
        N = nbr[:, f]
        ok = N >= 0
        acc[ok] += h[N[ok]]
        deg[ok] += 1
    return acc / np.maximum(deg, 1)[:, None, None], deg


def forward(theta, x, nbr, hidden=64, layers=4):
    P = unpack(theta, hidden, layers)
    hs = [np.maximum(x @ P["W_in"] + P["b_in"], 0.0)]
    ms = []
    for l in range(1, layers + 1):
        m, _ = _neighbour_mean(hs[-1], nbr)
        ms.append(m)
        a = np.concatenate([hs[-1], m], axis=-1)
        hs.append(np.maximum(a @ P[f"W{l}"] + P[f"b{l}"], 0.0))
    z = hs[-1] @ P["w_out"] + P["b_out"][0]
    return z, {"h": hs, "m": ms, "P": P}


def loss_and_grad(theta, x, nbr, y, hidden=64, layers=4):
    z, cache = forward(theta, x, nbr, hidden, layers)
    hs, ms, P = cache["h"], cache["m"], cache["P"]
    n = z.size
    r = z - y
    loss = float((r ** 2).mean())
    G = {}
    dz = 2.0 * r / n
    G["w_out"] = np.einsum("cg,cgh->h", dz, hs[-1])
    G["b_out"] = np.array([dz.sum()])
    dh = dz[..., None] * P["w_out"]
    _, deg = _neighbour_mean(hs[0], nbr)
    for l in range(layers, 0, -1):
        dpre = dh * (hs[l] > 0)
        a = np.concatenate([hs[l - 1], ms[l - 1]], axis=-1)
        G[f"W{l}"] = np.einsum("cgi,cgj->ij", a, dpre)
        G[f"b{l}"] = dpre.sum(axis=(0, 1))
        da = dpre @ P[f"W{l}"].T
        dh = da[..., :hidden].copy()
        dm = da[..., hidden:] / np.maximum(deg, 1)[:, None, None]
        for f in range(6):                  # the mean's adjoint: scatter back to the neighbours
            N = nbr[:, f]
            ok = N >= 0
            np.add.at(dh, N[ok], dm[ok])
    dpre = dh * (hs[0] > 0)
    G["W_in"] = np.einsum("cgi,cgj->ij", x, dpre)
    G["b_in"] = dpre.sum(axis=(0, 1))
    return loss, pack(G, hidden, layers)


def init_params(seed=0, hidden=64, layers=4):
    """He-style initialisation (a reference helper; the GPU library draws its own)."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in param_shapes(hidden, layers):
        if name.startswith("b"):
            P[name] = np.zeros(shp)
        else:
            fan_in = shp[0]
            P[name] = rng.normal(0.0, np.sqrt(2.0 / fan_in), shp)
    return pack(P, hidden, layers)


def round_bf16(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    rounded = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)
