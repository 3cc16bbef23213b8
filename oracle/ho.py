"""Higher-order discontinuous Galerkin sweeps on hexahedra (FP64, numpy).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use it to check and time the GPU library.  The product library never
imports it, and it imports nothing from the product library.

The paper runs its benchmarks with first-, second- and third-order finite
elements (Section 3.6 and its table of run times) without spelling out the
element.  This module is the plain definition of the order-p sweep used here:

* basis: tensor products of the degree-p Lagrange polynomials in each
  reference coordinate, with nodes at the Gauss-Lobatto-Legendre points
  (p = 1: the cube's corners, the first-order element).  Local node
  j = a + (p+1) b + (p+1)^2 c sits at (x_a, x_b, x_c);
* geometry: the trilinear map of the cell's 8 vertices (vertex
  v = a + 2b + 4c at reference corner (2a-1, 2b-1, 2c-1));
* integrals: the (p+1)-point Gauss rule per reference direction, for cells
  and faces (p = 1: the 2-point rule of the first-order element);
* the upwind equations of one (cell K, direction n, group g), the same as
  first order with N = (p+1)^3 nodes and (p+1)^2 nodes per face:
      (sum_a Om_a S^a + sigma_t M - sum_{f in} Om . F_f) psi
          = M q - sum_{f in} (Om . F_f) psi_up,f
  with M_ij = int phi_i phi_j, S^a_ij = int phi_i d phi_j / d x_a,
  F^a_f,kl = int_f n_a phi_k phi_l dA over face f's nodes, and "in" the
  faces with s_o . A_f < 0 for the octant's sign vector s_o (one designation
  per octant; A_f = int_f n dA);
* an interior face is integrated once, on the side with the smaller
  (cell, face) index; the other side takes the negated values at the
  matching nodes, so the two sides cancel exactly.  Matching nodes are found
  by their physical coordinates;
* the scalar flux phi = sum_n w_n psi_n at every node; the isotropic source
  (Q + sigma_s phi) / (4 pi) at the nodes.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre

FOUR_PI = 4.0 * np.pi


class HOError(RuntimeError):
    pass


def gll_points(p: int) -> np.ndarray:
    """The p + 1 Gauss-Lobatto-Legendre points on [-1, 1]: the end points and
    the roots of P_p'."""
    if p < 1:
        raise HOError("order must be >= 1")
    inner = legendre.legroots(legendre.legder(np.eye(p + 1)[p])) if p > 1 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def lagrange_1d(nodes: np.ndarray, x: np.ndarray):
    """Values and derivatives of the Lagrange polynomials of `nodes` at the
    points x: arrays [len(x), len(nodes)]."""
    m = len(nodes)
    x = np.asarray(x, np.float64)
    val = np.ones((x.size, m))
    der = np.zeros((x.size, m))
    for a in range(m):
        others = [b for b in range(m) if b != a]
        den = np.prod([nodes[a] - nodes[b] for b in others])
        for b in others:
            val[:, a] *= (x - nodes[b])
        for c in others:   # product rule: drop one factor at a time
            t = np.ones(x.size)
            for b in others:
                if b != c:
                    t *= (x - nodes[b])
            der[:, a] += t
        val[:, a] /= den
        der[:, a] /= den
    return val, der


def _corner(v, d):
    return 1.0 if (v >> d) & 1 else -1.0


def _trilinear(xi):
    """Trilinear vertex functions and their reference gradients at points xi [Q, 3]."""
    Q = xi.shape[0]
    f = np.ones((Q, 8))
    df = np.ones((Q, 8, 3))
    for v in range(8):
        h = [0.5 * (1.0 + _corner(v, d) * xi[:, d]) for d in range(3)]
        dh = [0.5 * _corner(v, d) for d in range(3)]
        f[:, v] = h[0] * h[1] * h[2]
        df[:, v, 0] = dh[0] * h[1] * h[2]
        df[:, v, 1] = h[0] * dh[1] * h[2]
        df[:, v, 2] = h[0] * h[1] * dh[2]
    return f, df


class HOOracle:
    """Order-p sweeps of one problem (vacuum or isotropic psi_b inflow,
    within-group isotropic scattering, octant designation)."""

    def __init__(self, xyz, cell_vert, order, omega, w, sigma_t, sigma_s, q, psi_b=None):
        self.xyz = np.ascontiguousarray(xyz, np.float64)
        self.cv = np.ascontiguousarray(cell_vert, np.int64)
        self.p = int(order)
        self.omega = np.ascontiguousarray(omega, np.float64)
        self.w = np.ascontiguousarray(w, np.float64)
        self.st = np.ascontiguousarray(sigma_t, np.float64)
        self.ss = np.ascontiguousarray(sigma_s, np.float64)
        self.q = np.ascontiguousarray(q, np.float64)
        self.psi_b = None if psi_b is None else np.ascontiguousarray(psi_b, np.float64)
        if self.p < 1 or self.p > 3:
            raise HOError("order must be 1, 2 or 3")
        if self.omega.shape[0] % 8 or self.omega.shape[0] == 0:
            raise HOError("the quadrature must hold the same number of directions in every octant")
        self.C, self.G = self.cv.shape[0], self.st.shape[1]
        self.nang = self.omega.shape[0]
        self._setup()

    # ------------------------------------------------------------ set-up
    def _setup(self):
        p, C = self.p, self.C
        m = p + 1
        self.N, self.nf = m ** 3, m ** 2
        nodes = gll_points(p)
        self.nodes1 = nodes
        idx = np.array([(a, b, c) for c in range(m) for b in range(m) for a in range(m)])   # j = a + m b + m^2 c
        self.node_ref = nodes[idx]                                                          # [N, 3]
        # face f = 2 axis + side: nodes whose index along `axis` is side * p, increasing j
        self.face_nodes = [np.array([j for j in range(self.N) if idx[j, f // 2] == (f % 2) * p]) for f in range(6)]
        gx, gw = legendre.leggauss(m)
        # -------- cells
        qi = np.array([(a, b, c) for c in range(m) for b in range(m) for a in range(m)])
        xi = gx[qi]
        wq = gw[qi[:, 0]] * gw[qi[:, 1]] * gw[qi[:, 2]]
        phi_q, dphi_q = self._basis(xi)
        _, dtri = _trilinear(xi)
        self.M = np.zeros((C, self.N, self.N))
        self.S = np.zeros((C, 3, self.N, self.N))
        for K in range(C):
            X = self.xyz[self.cv[K]]                          # [8, 3]
            J = np.einsum("va,qvb->qab", X, dtri)             # J[q][a][b] = d x_a / d xi_b
            det = np.linalg.det(J)
            if not np.all(det > 0):
                raise HOError("non-positive Jacobian at a Gauss point")
            Jinv = np.linalg.inv(J)                           # [q][b][a] = d xi_b / d x_a
            grad = np.einsum("qba,qjb->qja", Jinv, dphi_q)    # physical gradients [q][j][a]
            wd = wq * det
            self.M[K] = np.einsum("q,qi,qj->ij", wd, phi_q, phi_q)
            self.S[K] = np.einsum("q,qi,qja->aij", wd, phi_q, grad)
        # -------- neighbours: faces matched by their vertex sets
        key = {}
        self.nbr = -np.ones((C, 6), np.int64)
        self.nbrf = -np.ones((C, 6), np.int64)
        for K in range(C):
            for f in range(6):
                verts = frozenset(int(self.cv[K, v]) for v in range(8) if ((v >> (f // 2)) & 1) == f % 2)
                if verts in key:
                    N, g = key.pop(verts)
                    self.nbr[K, f], self.nbrf[K, f] = N, g
                    self.nbr[N, g], self.nbrf[N, g] = K, f
                else:
                    key[verts] = (K, f)
        # physical node coordinates, for matching face nodes across a face
        ftri, _ = _trilinear(self.node_ref)
        self.node_xyz = np.einsum("jv,Kva->Kja", ftri, self.xyz[self.cv])       # [C, N, 3]
        h = np.max(np.ptp(self.xyz, axis=0)) / max(1.0, round(C ** (1 / 3)))
        self.perm = -np.ones((C, 6, self.nf), np.int64)    # neighbour's local node at my face node k
        for K in range(C):
            for f in range(6):
                N, g = self.nbr[K, f], self.nbrf[K, f]
                if N < 0:
                    continue
                mine = self.node_xyz[K, self.face_nodes[f]]
                theirs = self.node_xyz[N, self.face_nodes[g]]
                d = np.linalg.norm(mine[:, None, :] - theirs[None, :, :], axis=2)
                k_best = np.argmin(d, axis=1)
                if d[np.arange(self.nf), k_best].max() > 1e-9 * h or len(set(k_best)) != self.nf:
                    raise HOError("face nodes do not match across a face")
                self.perm[K, f] = self.face_nodes[g][k_best]
        # -------- faces
        self.F = np.zeros((C, 6, 3, self.nf, self.nf))
        self.area = np.zeros((C, 6, 3))
        for K in range(C):
            for f in range(6):
                N, g = self.nbr[K, f], self.nbrf[K, f]
                if N >= 0 and 6 * N + g < 6 * K + f:
                    continue
                F, A = self._face(K, f, gx, gw)
                self.F[K, f], self.area[K, f] = F, A
                if N < 0:
                    continue
                # the neighbour's face-node position of each of my face nodes
                pos = np.array([int(np.where(self.face_nodes[g] == self.perm[K, f, k])[0][0])
                                for k in range(self.nf)])
                self.area[N, g] = -A
                FN = np.zeros((3, self.nf, self.nf))
                FN[:, pos[:, None], pos[None, :]] = -F
                self.F[N, g] = FN
        # -------- designation and sweep order
        self.inflow = np.zeros((8, C), np.int64)
        self.order = []
        for o in range(8):
            s = np.array([-1.0 if (o >> d) & 1 else 1.0 for d in range(3)])
            sa = np.einsum("a,Kfa->Kf", s, self.area)
            mask = sa < 0
            self.inflow[o] = (mask * (1 << np.arange(6))).sum(axis=1)
            deps = [[int(self.nbr[K, f]) for f in range(6) if mask[K, f] and self.nbr[K, f] >= 0] for K in range(C)]
            down = [[] for _ in range(C)]
            indeg = np.zeros(C, np.int64)
            for K in range(C):
                indeg[K] = len(deps[K])
                for U in deps[K]:
                    down[U].append(K)
            ready = [K for K in range(C) if indeg[K] == 0]
            seq = []
            while ready:
                K = ready.pop()
                seq.append(K)
                for D in down[K]:
                    indeg[D] -= 1
                    if indeg[D] == 0:
                        ready.append(D)
            if len(seq) != C:
                raise HOError(f"the octant {o} designation has a cycle")
            self.order.append(seq)

    def _basis(self, xi):
        """Values [Q, N] and reference gradients [Q, N, 3] of the nodal basis."""
        v, d = zip(*(lagrange_1d(self.nodes1, xi[:, k]) for k in range(3)))
        m = self.p + 1
        idx = np.array([(a, b, c) for c in range(m) for b in range(m) for a in range(m)])
        val = v[0][:, idx[:, 0]] * v[1][:, idx[:, 1]] * v[2][:, idx[:, 2]]
        grad = np.stack([d[0][:, idx[:, 0]] * v[1][:, idx[:, 1]] * v[2][:, idx[:, 2]],
                         v[0][:, idx[:, 0]] * d[1][:, idx[:, 1]] * v[2][:, idx[:, 2]],
                         v[0][:, idx[:, 0]] * v[1][:, idx[:, 1]] * d[2][:, idx[:, 2]]], axis=2)
        return val, grad

    def _face(self, K, f, gx, gw):
        """F^a_kl = int_f n_a phi_k phi_l dA and A = int_f n dA, face f of cell K,
        by the (p+1)^2-point Gauss rule on the face's two free reference
        coordinates (increasing axis order); n dA = +-(dx/du x dx/dv) oriented
        outward."""
        axis, side = f // 2, f % 2
        u, v = [d for d in range(3) if d != axis]
        sgn = (-1.0 if axis == 1 else 1.0) * (1.0 if side else -1.0)
        m = self.p + 1
        pts = np.array([(i, k) for k in range(m) for i in range(m)])
        xi = np.zeros((m * m, 3))
        xi[:, axis] = 1.0 if side else -1.0
        xi[:, u] = gx[pts[:, 0]]
        xi[:, v] = gx[pts[:, 1]]
        wq = gw[pts[:, 0]] * gw[pts[:, 1]]
        phi_q, _ = self._basis(xi)
        _, dtri = _trilinear(xi)
        X = self.xyz[self.cv[K]]
        J = np.einsum("va,qvb->qab", X, dtri)
        Nq = sgn * np.cross(J[:, :, u], J[:, :, v]) * wq[:, None]      # [q, 3]
        fn = self.face_nodes[f]
        F = np.einsum("qa,qk,ql->akl", Nq, phi_q[:, fn], phi_q[:, fn])
        return F, Nq.sum(axis=0)

    # ------------------------------------------------------------- sweeps
    def source_nodal(self, phi_in):
        """(Q + sigma_s phi) / (4 pi) at every node: [C, G, N]."""
        ph = np.zeros((self.C, self.G, self.N)) if phi_in is None else np.asarray(phi_in, np.float64)
        return (self.q[:, :, None] + self.ss[:, :, None] * ph) / FOUR_PI

    def sweep(self, phi_in=None, want_psi=False, want_leak=False, ang_src=None, bnd=None):
        """One transport sweep of every direction and group.

        ang_src: optional [nang, C, G, N] extra source per direction at the
        nodes; bnd: optional [C, 6, nang, G, nf] inflow values at the face
        nodes of boundary faces (instead of psi_b).  Returns a dict with phi
        [C, G, N], and psi [nang, C, G, N] and leak [C, G] on request."""
        C, G, N = self.C, self.G, self.N
        qn = self.source_nodal(phi_in)
        psi = np.zeros((self.nang, C, G, N))
        phi = np.zeros((C, G, N))
        leak = np.zeros((C, G)) if want_leak else None
        for n in range(self.nang):
            lk = self._sweep_direction(n, qn, psi[n], None if ang_src is None else ang_src[n], bnd, want_leak)
            if want_leak:
                leak += self.w[n] * lk
            phi += self.w[n] * psi[n]
        out = {"phi": phi}
        if want_psi:
            out["psi"] = psi
        if want_leak:
            out["leak"] = leak
        return out

    def sweep_angle(self, phi_in, n):
        """psi [C, G, N] of direction n alone: for a given phi_in the directions
        of one source iteration are independent, so this is the direction-n
        pass of sweep()."""
        psi_n = np.zeros((self.C, self.G, self.N))
        self._sweep_direction(int(n), self.source_nodal(phi_in), psi_n, None, None, False)
        return psi_n

    def _sweep_direction(self, n, qn, psi_n, src_n, bnd, want_leak):
        """Cells of direction n in its octant's topological order: the local
        system of every group, psi_n [C, G, N] filled in place.  Returns the
        per-(cell, group) net outflow when want_leak."""
        C, G, nf = self.C, self.G, self.nf
        per = self.nang // 8
        o = n // per
        om = self.omega[n]
        leak = np.zeros((C, G)) if want_leak else None
        for K in self.order[o]:
            mask = self.inflow[o, K]
            A0 = np.einsum("a,aij->ij", om, self.S[K])
            A = A0[None, :, :] + self.st[K][:, None, None] * self.M[K][None, :, :]
            src = qn[K] if src_n is None else qn[K] + src_n[K]
            b = src @ self.M[K].T                                  # [G, N]: M q
            ups = {}
            for f in range(6):
                if not (mask >> f) & 1:
                    continue
                fn = self.face_nodes[f]
                of = np.einsum("a,akl->kl", om, self.F[K, f])
                Nb = self.nbr[K, f]
                if Nb >= 0:
                    up = psi_n[Nb][:, self.perm[K, f]]              # [G, nf]
                elif bnd is not None:
                    up = bnd[K, f, n]
                elif self.psi_b is not None:
                    up = np.repeat(self.psi_b[:, None], nf, axis=1)
                else:
                    up = np.zeros((G, nf))
                ups[f] = (of, up)
                A[:, fn[:, None], fn[None, :]] -= of[None, :, :]
                b[:, fn] -= up @ of.T
            x = np.linalg.solve(A, b[:, :, None])[:, :, 0]
            psi_n[K] = x
            if want_leak:
                lk = np.zeros(G)
                for f in range(6):
                    fn = self.face_nodes[f]
                    if f in ups:
                        of, up = ups[f]
                        lk += (up @ of.T).sum(axis=1)
                    else:
                        of = np.einsum("a,akl->kl", om, self.F[K, f])
                        lk += (x[:, fn] @ of.T).sum(axis=1)
                leak[K] = lk
        return leak

    def solve(self, tol, max_it, phi0=None):
        """Source iteration until the relative max-norm change of phi is
        <= tol or max_it sweeps (the first-order oracle's rule)."""
        cur = np.zeros((self.C, self.G, self.N)) if phi0 is None else np.array(phi0, np.float64)
        eps, it = np.inf, 0
        while it < max_it:
            new = self.sweep(cur)["phi"]
            den = np.abs(new).max()
            num = np.abs(new - cur).max()
            eps = num / den if den > 0 else (np.inf if num > 0 else 0.0)
            it += 1
            cur = new
            if eps <= tol:
                break
        return {"phi": cur, "iters": it, "eps": eps, "status": 0 if eps <= tol else -7}

    def balance(self, phi_in, phi_out, leak):
        """Per group: source 1^T M 4 pi q, absorption sigma_t 1^T M phi_out, net
        outflow, and the worst relative cell imbalance: [G, 4]."""
        qn = self.source_nodal(phi_in)
        src = FOUR_PI * np.einsum("Kij,Kgj->Kg", self.M, qn)
        ab = self.st * np.einsum("Kij,Kgj->Kg", self.M, phi_out)
        scale = np.maximum(np.abs(src), np.maximum(np.abs(ab), np.abs(leak)))
        rel = np.where(scale > 0, np.abs(src - ab - leak) / np.where(scale > 0, scale, 1.0), 0.0)
        return np.stack([src.sum(0), ab.sum(0), leak.sum(0), rel.max(0)], axis=1)

    def volumes(self):
        return self.M.sum(axis=(1, 2))
