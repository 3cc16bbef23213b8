"""FP64 CPU oracle of the unstructured S_N sweep (ctypes wrapper of snx_oracle.c).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use it to check and time the GPU library.  The product library never
imports it, and it imports nothing from the product library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsnx_oracle.so")
_SRC = os.path.join(_HERE, "snx_oracle.c")

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")

ERRORS = {0: "OK", -1: "E_ARG", -2: "E_STATE", -3: "E_MESH", -4: "E_CYCLE", -6: "E_OOM", -7: "E_NOCONV"}


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle {ERRORS.get(code, code)}: {msg}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile snx_oracle.c into libsnx_oracle.so with gcc (OpenMP over groups)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ct.CDLL(_LIB_PATH)
        vp = ct.c_void_p
        nullable_d = ct.c_void_p
        L.snxo_gauss_legendre.argtypes = [ct.c_int, _dp, _dp]
        L.snxo_quadrature.argtypes = [ct.c_int, ct.c_int, _dp, _dp]
        L.snxo_create.argtypes = [ct.POINTER(vp)]
        L.snxo_destroy.argtypes = [vp]
        L.snxo_destroy.restype = None
        L.snxo_set_mesh.argtypes = [vp, ct.c_int, ct.c_int, _dp, _ip]
        L.snxo_set_quadrature.argtypes = [vp, ct.c_int, _dp, _dp]
        L.snxo_set_materials.argtypes = [vp, ct.c_int, _dp, _dp, _dp]
        L.snxo_set_boundary.argtypes = [vp, ct.c_int, nullable_d]
        L.snxo_set_hooks.argtypes = [vp, nullable_d, nullable_d]
        L.snxo_setup.argtypes = [vp]
        L.snxo_set_designation.argtypes = [vp, ct.c_int]
        L.snxo_set_reflective.argtypes = [vp, ct.c_int]
        L.snxo_set_anisotropy.argtypes = [vp, ct.c_int, nullable_d]
        L.snxo_get_harmonics.argtypes = [vp, _dp]
        L.snxo_set_group_scattering.argtypes = [vp, ct.c_int, nullable_d, nullable_d]
        L.snxo_solve_outer.argtypes = [vp, ct.c_int, ct.c_int, ct.c_double, nullable_d, _dp,
                                       ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_double)]
        L.snxo_sweep.argtypes = [vp, nullable_d, nullable_d, _dp, nullable_d, nullable_d, nullable_d]
        L.snxo_sweep_angle.argtypes = [vp, nullable_d, ct.c_int, ct.c_int, nullable_d, _dp]
        L.snxo_solve.argtypes = [vp, ct.c_double, ct.c_int, nullable_d, _dp,
                                 ct.POINTER(ct.c_int), ct.POINTER(ct.c_double), nullable_d]
        L.snxo_balance.argtypes = [vp, nullable_d, _dp, _dp, _dp]
        L.snxo_integrated_flux.argtypes = [vp, _dp, _dp]
        L.snxo_get_geometry.argtypes = [vp] + [nullable_d] * 7
        L.snxo_get_dag.argtypes = [vp, nullable_d, nullable_d, nullable_d]
        L.snxo_get_angle_inflow.argtypes = [vp, _ip]
        L.snxo_get_angle_order.argtypes = [vp, nullable_d, nullable_d]
        L.snxo_set_octant_order.argtypes = [vp, ct.c_int]
        L.snxo_last_error.argtypes = [vp]
        L.snxo_last_error.restype = ct.c_char_p
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    rc = lib().snxo_gauss_legendre(n, x, w)
    if rc:
        raise OracleError(rc, "gauss_legendre")
    return x, w


def quadrature(npolar: int, nazim: int):
    nang = 8 * npolar * nazim
    om = np.zeros((nang, 3))
    w = np.zeros(nang)
    rc = lib().snxo_quadrature(npolar, nazim, om, w)
    if rc:
        raise OracleError(rc, "quadrature")
    return om, w


class Oracle:
    """One transport problem on the CPU in FP64.

    Arrays use the same exchange layouts as the GPU library: phi[ncell][G][8].
    """

    def __init__(self, xyz, cell_vert, omega, w, sigma_t, sigma_s, q,
                 boundary_kind: int = 0, psi_b=None, ang_src=None, bnd_in=None, setup: bool = True,
                 designation: int = 0):
        L = lib()
        h = ct.c_void_p()
        self._check(L.snxo_create(ct.byref(h)), "create")
        self.h = h
        self.xyz = np.ascontiguousarray(xyz, np.float64)
        self.cell_vert = np.ascontiguousarray(cell_vert, np.int32)
        self.omega = np.ascontiguousarray(omega, np.float64)
        self.w = np.ascontiguousarray(w, np.float64)
        self.sigma_t = np.ascontiguousarray(sigma_t, np.float64)
        self.sigma_s = np.ascontiguousarray(sigma_s, np.float64)
        self.q = np.ascontiguousarray(q, np.float64)
        self.ncell = self.cell_vert.shape[0]
        self.nang = self.omega.shape[0]
        self.G = self.sigma_t.shape[1]
        self._check(L.snxo_set_mesh(h, self.ncell, self.xyz.shape[0], self.xyz, self.cell_vert), "set_mesh")
        self._check(L.snxo_set_quadrature(h, self.nang, self.omega, self.w), "set_quadrature")
        self._check(L.snxo_set_materials(h, self.G, self.sigma_t, self.sigma_s, self.q), "set_materials")
        self.psi_b = None if psi_b is None else np.ascontiguousarray(psi_b, np.float64)
        self._check(L.snxo_set_boundary(h, boundary_kind, _ptr(self.psi_b)), "set_boundary")
        self.set_hooks(ang_src, bnd_in)
        self.designation = int(designation)
        self._check(L.snxo_set_designation(h, self.designation), "set_designation")
        if setup:
            self.setup()

    @classmethod
    def from_problem(cls, prob, **kw):
        om, w = quadrature(prob.npolar, prob.nazim)
        return cls(prob.mesh.xyz, prob.mesh.cell_vert, om, w, prob.mat.sigma_t, prob.mat.sigma_s,
                   prob.mat.q, prob.boundary_kind, prob.psi_b, **kw)

    def _check(self, rc, what):
        if rc:
            msg = lib().snxo_last_error(self.h).decode() if getattr(self, "h", None) else what
            raise OracleError(rc, f"{what}: {msg}")

    def set_hooks(self, ang_src=None, bnd_in=None):
        self._ang_src = None if ang_src is None else np.ascontiguousarray(ang_src, np.float64)
        self._bnd_in = None if bnd_in is None else np.ascontiguousarray(bnd_in, np.float64)
        self._check(lib().snxo_set_hooks(self.h, _ptr(self._ang_src), _ptr(self._bnd_in)), "set_hooks")

    def setup(self):
        self._check(lib().snxo_setup(self.h), "setup")

    def set_anisotropy(self, sigma_l):
        """sigma_l[ncell][G][L]: Legendre moments 1..L of the within-group scattering
        law (None or L = 0: isotropic).  Before setup."""
        if sigma_l is None or np.asarray(sigma_l).shape[-1] == 0:
            self._sigl = None
            self._check(lib().snxo_set_anisotropy(self.h, 0, None), "set_anisotropy")
            return
        self._sigl = np.ascontiguousarray(sigma_l, np.float64)
        if self._sigl.shape[:2] != (self.ncell, self.G):
            raise ValueError("sigma_l must be [ncell][G][L]")
        self._check(lib().snxo_set_anisotropy(self.h, self._sigl.shape[2], _ptr(self._sigl)), "set_anisotropy")

    def harmonics(self, L):
        y = np.zeros((self.nang, (L + 1) ** 2))
        self._check(lib().snxo_get_harmonics(self.h, y), "get_harmonics")
        return y

    def set_reflective(self, planes: int):
        """Reflective boundary planes, bit 2*axis + side (before setup)."""
        self._check(lib().snxo_set_reflective(self.h, int(planes)), "set_reflective")

    def set_octant_order(self, sequential: bool):
        """True: octants in sequence, reflected inflow from the current sweep where the
        mirrored octant came earlier; False (default): from the previous sweep."""
        self._check(lib().snxo_set_octant_order(self.h, int(bool(sequential))), "set_octant_order")

    def set_group_scattering(self, cell_mat, sigma_gg):
        """cell_mat[ncell] int, sigma_gg[nmat][G][G] from group g' (axis 1) into g (axis 2);
        None clears it."""
        if sigma_gg is None:
            self._cmat = self._sgg = None
            self._check(lib().snxo_set_group_scattering(self.h, 0, None, None), "set_group_scattering")
            return
        self._cmat = np.ascontiguousarray(cell_mat, np.int32)
        self._sgg = np.ascontiguousarray(sigma_gg, np.float64)
        if self._sgg.ndim != 3 or self._sgg.shape[1:] != (self.G, self.G) or self._cmat.shape != (self.ncell,):
            raise ValueError("cell_mat must be [ncell] and sigma_gg [nmat][G][G]")
        self._check(lib().snxo_set_group_scattering(self.h, self._sgg.shape[0], _ptr(self._cmat), _ptr(self._sgg)),
                    "set_group_scattering")

    def solve_outer(self, outer, inner, tol=0.0, phi0=None, allow_noconv=False):
        """Inner/outer iterations (see snxo_solve_outer)."""
        phi = self.zeros_phi()
        ko, ki, eps = ct.c_int(0), ct.c_int(0), ct.c_double(0.0)
        p0 = None if phi0 is None else np.ascontiguousarray(phi0, np.float64)
        rc = lib().snxo_solve_outer(self.h, int(outer), int(inner), float(tol), _ptr(p0), phi, ct.byref(ko),
                                    ct.byref(ki), ct.byref(eps))
        if rc and not (allow_noconv and rc == -7):
            self._check(rc, "solve_outer")
        return {"phi": phi, "outers": ko.value, "inners": ki.value, "eps": eps.value, "status": rc}

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().snxo_destroy(h)
            self.h = None

    def zeros_phi(self):
        return np.zeros((self.ncell, self.G, 8))

    def sweep(self, phi_in=None, want_psi=False, want_leak=False, want_leak_ang=False, psi_prev=None):
        """One source iteration.  psi_prev[nang][ncell][G][8] (None = zero) is the
        previous sweep's angular flux, read on lagged faces (designation 1)."""
        phi_out = self.zeros_phi()
        pin = None if phi_in is None else np.ascontiguousarray(phi_in, np.float64)
        pprev = None if psi_prev is None else np.ascontiguousarray(psi_prev, np.float64)
        if pprev is not None and pprev.shape != (self.nang, self.ncell, self.G, 8):
            raise ValueError("psi_prev must be [nang][ncell][G][8]")
        psi = np.zeros((self.nang, self.ncell, self.G, 8)) if want_psi else None
        leak = np.zeros((self.ncell, self.G)) if want_leak else None
        leak_ang = np.zeros((self.nang, self.ncell, self.G)) if want_leak_ang else None
        self._check(lib().snxo_sweep(self.h, _ptr(pin), _ptr(pprev), phi_out, _ptr(psi), _ptr(leak),
                                     _ptr(leak_ang)), "sweep")
        out = {"phi": phi_out}
        if want_psi:
            out["psi"] = psi
        if want_leak:
            out["leak"] = leak
        if want_leak_ang:
            out["leak_ang"] = leak_ang
        return out

    def sweep_angle(self, phi_in, n, g, psi_prev=None):
        """psi[ncell][8] of angle n and group g alone, for the same phi_in (and
        psi_prev[ncell][8] of this (n, g), None = zero) as sweep()."""
        psi = np.zeros((self.ncell, 8))
        pin = None if phi_in is None else np.ascontiguousarray(phi_in, np.float64)
        pprev = None if psi_prev is None else np.ascontiguousarray(psi_prev, np.float64)
        if pprev is not None and pprev.shape != (self.ncell, 8):
            raise ValueError("psi_prev must be [ncell][8]")
        self._check(lib().snxo_sweep_angle(self.h, _ptr(pin), int(n), int(g), _ptr(pprev), psi), "sweep_angle")
        return psi

    def solve(self, tol, max_it, phi0=None, allow_noconv=False):
        phi = self.zeros_phi()
        it = ct.c_int(0)
        eps = ct.c_double(0.0)
        hist = np.zeros(max_it)
        p0 = None if phi0 is None else np.ascontiguousarray(phi0, np.float64)
        rc = lib().snxo_solve(self.h, tol, max_it, _ptr(p0), phi, ct.byref(it), ct.byref(eps), _ptr(hist))
        if rc and not (allow_noconv and rc == -7):
            self._check(rc, "solve")
        return {"phi": phi, "iters": it.value, "eps": eps.value, "hist": hist[: it.value], "status": rc}

    def balance(self, phi_in, phi_out, leak):
        out = np.zeros((self.G, 4))
        pin = None if phi_in is None else np.ascontiguousarray(phi_in, np.float64)
        self._check(lib().snxo_balance(self.h, _ptr(pin), np.ascontiguousarray(phi_out), np.ascontiguousarray(leak), out), "balance")
        return out

    def integrated_flux(self, phi):
        out = np.zeros((self.G, 2))
        self._check(lib().snxo_integrated_flux(self.h, np.ascontiguousarray(phi, np.float64), out), "integrated_flux")
        return out

    def geometry(self):
        C = self.ncell
        g = {"M": np.zeros((C, 8, 8)), "S": np.zeros((C, 3, 8, 8)), "F": np.zeros((C, 6, 3, 4, 4)),
             "area": np.zeros((C, 6, 3)), "nbr": np.zeros((C, 6), np.int32),
             "nbr_face": np.zeros((C, 6), np.int32), "perm": np.zeros((C, 6, 4), np.int32)}
        self._check(lib().snxo_get_geometry(self.h, *[_ptr(g[k]) for k in
                    ("M", "S", "F", "area", "nbr", "nbr_face", "perm")]), "get_geometry")
        return g

    def angle_order(self):
        """Designation 2: ([nang][ncell] sweep order of each direction, [nang][ncell] lagged-face masks)."""
        order = np.zeros((self.nang, self.ncell), np.int32)
        lag = np.zeros((self.nang, self.ncell), np.int32)
        self._check(lib().snxo_get_angle_order(self.h, _ptr(order), _ptr(lag)), "get_angle_order")
        return order, lag

    def angle_inflow(self):
        """Designations 1 and 2: [nang][ncell] inflow-face bit masks of each angle."""
        ain = np.zeros((self.nang, self.ncell), np.int32)
        self._check(lib().snxo_get_angle_inflow(self.h, ain), "get_angle_inflow")
        return ain

    def dag(self):
        C = self.ncell
        d = {"inflow": np.zeros((8, C), np.int32), "level": np.zeros((8, C), np.int32),
             "order": np.zeros((8, C), np.int32)}
        self._check(lib().snxo_get_dag(self.h, _ptr(d["inflow"]), _ptr(d["level"]), _ptr(d["order"])), "get_dag")
        return d


def face_nodes(f: int):
    """Local vertices of face f = 2*axis + side (bit `axis` of the index equals side)."""
    axis, side = divmod(f, 2)
    return [j for j in range(8) if ((j >> axis) & 1) == side]
