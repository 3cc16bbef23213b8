"""Seeded synthetic inputs for the unstructured S_N sweep.

This module produces plain data only: hexahedral meshes of the unit cube
(vertex coordinates and 8-vertex connectivity), per-cell per-group material
arrays and problem-size recipes.  It holds none of the transport method's
arithmetic (no quadrature, no geometry integrals, no sweep), so that the CPU
checker and the GPU library can both be fed from it without sharing any code
of the method.

Mesh convention.  A cell's local vertex ``j = a + 2 b + 4 c`` (a, b, c in
{0, 1}) sits at the reference corner ``(2a-1, 2b-1, 2c-1)`` of [-1, 1]^3.  The
paper's synthetic mesh is an orthogonal hex grid made unstructured at run
time (Section 2, the UnSNAP description); here the grid is made irregular by
moving every interior vertex by an independent uniform amount in
[-j h, +j h] per coordinate, boundary vertices stay put, and cell and vertex
ids are randomly permuted so no structured ordering survives.

Seeds: instance seed = 1000 * config + index; ``numpy.random.default_rng``
draws in this order: vertex jitter, cell permutation, vertex permutation,
block materials, sources.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Mesh", "Materials", "Problem", "make_mesh", "block_index",
    "materials_uniform", "materials_two_block", "materials_loguniform_blocks",
    "group_scale", "config_problem", "batch_problems", "instance_seed", "split_scattering",
]


@dataclasses.dataclass
class Mesh:
    n: int                    # cells per edge (n^3 cells)
    xyz: np.ndarray           # [nvert, 3] float64
    cell_vert: np.ndarray     # [ncell, 8] int32, local vertex j = a + 2b + 4c
    ijk: np.ndarray           # [ncell, 3] int32 structured index of each cell (test use only)
    vert_ijk: np.ndarray      # [nvert, 3] int32 structured index of each vertex

    @property
    def ncell(self) -> int:
        return int(self.cell_vert.shape[0])

    @property
    def nvert(self) -> int:
        return int(self.xyz.shape[0])


@dataclasses.dataclass
class Materials:
    sigma_t: np.ndarray   # [ncell, G] float64
    sigma_s: np.ndarray   # [ncell, G] float64
    q: np.ndarray         # [ncell, G] float64, isotropic source density

    @property
    def ngroup(self) -> int:
        return int(self.sigma_t.shape[1])


@dataclasses.dataclass
class Problem:
    name: str
    mesh: Mesh
    mat: Materials
    npolar: int
    nazim: int
    tol: float
    boundary_kind: int = 0            # 0 vacuum, 1 isotropic inflow
    psi_b: np.ndarray | None = None   # [G] inflow value when boundary_kind == 1

    @property
    def nang(self) -> int:
        return 8 * self.npolar * self.nazim


def instance_seed(config: int, index: int = 0) -> int:
    return 1000 * config + index


def make_mesh(n: int, jitter: float = 0.2, seed: int = 0, permute: bool = True,
              rng: np.random.Generator | None = None) -> Mesh:
    """n^3 hex grid of the unit cube, interior vertices jittered by U(-jitter*h, jitter*h)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    if rng is None:
        rng = np.random.default_rng(seed)
    h = 1.0 / n
    nv1 = n + 1
    vi, vj, vk = np.meshgrid(np.arange(nv1), np.arange(nv1), np.arange(nv1), indexing="ij")
    vert_ijk = np.stack([vi.ravel(), vj.ravel(), vk.ravel()], axis=1).astype(np.int32)
    # structured vertex id = i + nv1*(j + nv1*k)
    order = np.lexsort((vert_ijk[:, 0], vert_ijk[:, 1], vert_ijk[:, 2]))
    vert_ijk = vert_ijk[order]
    xyz = vert_ijk.astype(np.float64) * h
    # 1) vertex jitter (drawn for every vertex so the stream does not depend on n's boundary share)
    shift = rng.uniform(-jitter * h, jitter * h, size=xyz.shape) if jitter > 0 else np.zeros_like(xyz)
    interior = np.all((vert_ijk > 0) & (vert_ijk < n), axis=1)
    xyz[interior] += shift[interior]

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cijk = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1).astype(np.int32)
    corder = np.lexsort((cijk[:, 0], cijk[:, 1], cijk[:, 2]))
    cijk = cijk[corder]
    cv = np.empty((n ** 3, 8), dtype=np.int64)
    for j in range(8):
        a, b, c = j & 1, (j >> 1) & 1, (j >> 2) & 1
        cv[:, j] = (cijk[:, 0] + a) + nv1 * ((cijk[:, 1] + b) + nv1 * (cijk[:, 2] + c))

    # 2) cell permutation, 3) vertex permutation
    if permute:
        cperm = rng.permutation(n ** 3)          # new cell id -> structured cell id
        vperm = rng.permutation(nv1 ** 3)        # new vertex id -> structured vertex id
    else:
        cperm = np.arange(n ** 3)
        vperm = np.arange(nv1 ** 3)
    vinv = np.empty_like(vperm)
    vinv[vperm] = np.arange(vperm.size)
    cell_vert = vinv[cv[cperm]].astype(np.int32)
    return Mesh(n=n, xyz=np.ascontiguousarray(xyz[vperm]), cell_vert=np.ascontiguousarray(cell_vert),
                ijk=np.ascontiguousarray(cijk[cperm]), vert_ijk=np.ascontiguousarray(vert_ijk[vperm]))


def rotate_cells(mesh: Mesh, rng: np.random.Generator) -> Mesh:
    """The same mesh with each cell's local vertex order turned by a random
    rotation of the reference cube (one of the 24 with determinant +1), so
    that neighbouring cells see a shared face in every relative orientation.
    Local vertex v' of the new order is the old vertex at R applied to v''s
    reference corner; the Jacobian keeps its sign."""
    rots = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        for signs in range(8):
            R = np.zeros((3, 3))
            for d in range(3):
                R[d, perm[d]] = -1.0 if (signs >> d) & 1 else 1.0
            if np.linalg.det(R) > 0:
                rots.append(R)
    corner = np.array([[2 * ((v >> d) & 1) - 1 for d in range(3)] for v in range(8)], np.float64)
    of_corner = {tuple(c): v for v, c in enumerate(corner.astype(int))}
    cv = mesh.cell_vert.copy()
    for K in range(mesh.ncell):
        R = rots[rng.integers(len(rots))]
        old = mesh.cell_vert[K]
        cv[K] = [old[of_corner[tuple((R @ corner[v]).astype(int))]] for v in range(8)]
    return Mesh(n=mesh.n, xyz=mesh.xyz, cell_vert=np.ascontiguousarray(cv), ijk=mesh.ijk, vert_ijk=mesh.vert_ijk)


def block_index(mesh: Mesh, block: int) -> np.ndarray:
    """Index of the block^3 block each cell lies in (ragged blocks at the far edges)."""
    nb = (mesh.n + block - 1) // block
    b = mesh.ijk // block
    return (b[:, 0] + nb * (b[:, 1] + nb * b[:, 2])).astype(np.int64), nb ** 3


def group_scale(G: int) -> np.ndarray:
    """Per-group multiplier 0.8 + 0.4 g/(G-1) that makes the groups differ."""
    g = np.arange(G, dtype=np.float64)
    return 0.8 + 0.4 * g / max(G - 1, 1)


def _expand(sig_t_cell, c_cell, q_cell, G, scaled):
    s = group_scale(G) if scaled else np.ones(G)
    st = np.asarray(sig_t_cell, np.float64)[:, None] * s[None, :]
    ss = np.asarray(c_cell, np.float64)[:, None] * st
    q = np.repeat(np.asarray(q_cell, np.float64)[:, None], G, axis=1)
    return Materials(np.ascontiguousarray(st), np.ascontiguousarray(ss), np.ascontiguousarray(q))


def materials_uniform(mesh: Mesh, G: int, sigma_t: float, c: float, q: float,
                      scaled: bool = False) -> Materials:
    C = mesh.ncell
    return _expand(np.full(C, sigma_t), np.full(C, c), np.full(C, q), G, scaled)


def materials_two_block(mesh: Mesh, G: int, rng: np.random.Generator, block: int = 4,
                        scaled: bool = True) -> Materials:
    """Seeded block checkerboard of two materials: (sigma_t 0.5, c 0.3, Q 1) and (5.0, 0.9, 0)."""
    bidx, nblk = block_index(mesh, block)
    pick = rng.integers(0, 2, size=nblk)[bidx]
    st = np.where(pick == 0, 0.5, 5.0)
    c = np.where(pick == 0, 0.3, 0.9)
    q = np.where(pick == 0, 1.0, 0.0)
    return _expand(st, c, q, G, scaled)


def materials_loguniform_blocks(mesh: Mesh, G: int, rng: np.random.Generator, block: int,
                                c_lo: float, c_hi: float, scaled: bool = True) -> Materials:
    """Per block: sigma_t = 10^U(-1,1), c ~ U(c_lo, c_hi), source ~ U(0, 1)."""
    bidx, nblk = block_index(mesh, block)
    st = 10.0 ** rng.uniform(-1.0, 1.0, size=nblk)
    c = rng.uniform(c_lo, c_hi, size=nblk)
    q = rng.uniform(0.0, 1.0, size=nblk)   # sources are drawn last
    return _expand(st[bidx], c[bidx], q[bidx], G, scaled)


def split_scattering(mat: Materials, within: float = 0.6):
    """Group-to-group scattering matrices with the same total scattering per
    group as mat.sigma_s: group g keeps the fraction `within` and passes the
    rest down to the higher-index groups with weights 1/2, 1/4, ... (normalised),
    and the last group keeps all of it.  Returns (cell_mat [ncell] int32,
    sigma_gg [nmat][G][G] with [m][g'][g] the cross section from g' into g), one
    material per distinct sigma_s row."""
    rows, cell_mat = np.unique(mat.sigma_s, axis=0, return_inverse=True)
    G = rows.shape[1]
    frac = np.zeros((G, G))
    for g in range(G):
        if g == G - 1:
            frac[g, g] = 1.0
            continue
        down = 0.5 ** np.arange(1, G - g)
        frac[g, g] = within
        frac[g, g + 1:] = (1.0 - within) * down / down.sum()
    sgg = rows[:, :, None] * frac[None, :, :]
    return np.ascontiguousarray(cell_mat.reshape(-1), np.int32), np.ascontiguousarray(sgg)


def config_problem(config: int, index: int = 0, scaled: bool = True, n: int | None = None) -> Problem:
    """The five workload recipes (1..5) plus 0 = the paper's 16^3 timing shape.

    1: 8^3, 2x2 product quadrature (32 angles), 4 groups, sigma_t 1, c 0.5, Q 1 (identical groups).
    2: 32^3, 3x4 (96 angles), 16 groups, two-material 4^3-block checkerboard.
    3: 64^3, 4x8 (256 angles), 64 groups, 8^3 blocks, log-uniform sigma_t, c in [0, 0.95].
    5: 32^3, 3x4, 16 groups, 4^3 blocks, log-uniform sigma_t, c in [0.9, 0.99].
    0: 16^3, 4x4 (128 angles), 16 groups, sigma_t 1, c 0.5, Q 1.
    ``n`` overrides the mesh edge (smaller parity cases of the same recipe).
    """
    rng = np.random.default_rng(instance_seed(config, index))
    if config == 1:
        mesh = make_mesh(n or 8, 0.2, rng=rng)
        mat = materials_uniform(mesh, 4, 1.0, 0.5, 1.0, scaled=False)
        return Problem("cfg1", mesh, mat, 2, 2, 1e-8)
    if config == 2:
        mesh = make_mesh(n or 32, 0.2, rng=rng)
        mat = materials_two_block(mesh, 16, rng, 4, scaled=scaled)
        return Problem("cfg2", mesh, mat, 3, 4, 1e-6)
    if config == 3:
        mesh = make_mesh(n or 64, 0.2, rng=rng)
        mat = materials_loguniform_blocks(mesh, 64, rng, 8, 0.0, 0.95, scaled=scaled)
        return Problem("cfg3", mesh, mat, 4, 8, 1e-6)
    if config == 5:
        mesh = make_mesh(n or 32, 0.2, rng=rng)
        mat = materials_loguniform_blocks(mesh, 16, rng, 4, 0.9, 0.99, scaled=scaled)
        return Problem("cfg5", mesh, mat, 3, 4, 1e-6)
    if config == 0:
        mesh = make_mesh(n or 16, 0.2, rng=rng)
        mat = materials_uniform(mesh, 16, 1.0, 0.5, 1.0, scaled=scaled)
        return Problem("paper16", mesh, mat, 4, 4, 0.0)
    raise ValueError(f"unknown config {config}")


BATCH_QUADS = ((2, 2), (2, 4), (3, 4), (4, 4))


def batch_problems(count: int = 64, config: int = 4, n_lo: int = 16, n_hi: int = 40,
                   g_lo: int = 8, g_hi: int = 32, scaled: bool = True) -> list[Problem]:
    """Uneven independent instances: n ~ U{n_lo..n_hi}, G ~ U{g_lo..g_hi}, random quadrature size."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(instance_seed(config, i))
        n = int(rng.integers(n_lo, n_hi + 1))
        G = int(rng.integers(g_lo, g_hi + 1))
        npol, naz = BATCH_QUADS[int(rng.integers(0, len(BATCH_QUADS)))]
        mesh = make_mesh(n, 0.2, rng=rng)
        mat = materials_two_block(mesh, G, rng, 4, scaled=scaled)
        out.append(Problem(f"batch{i}", mesh, mat, npol, naz, 1e-6))
    return out
