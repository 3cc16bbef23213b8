"""Python binding of libsnx.so (the gfx950 S_N sweep library).

Argument marshalling only: every step of the transport path runs in the HIP
kernels behind the C ABI declared in include/snx.h.  PyTorch supplies device
memory (tensors' data pointers) and streams.  There is no fallback: if the
library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnx.so")

STATUS = {0: "SNX_OK", -1: "SNX_E_ARG", -2: "SNX_E_STATE", -3: "SNX_E_MESH", -4: "SNX_E_CYCLE",
          -5: "SNX_E_DEVICE", -6: "SNX_E_OOM", -7: "SNX_E_NOCONV"}
SNX_E_NOCONV = -7
SWEEP_AMT, SWEEP_BSP = 0, 1
DESIGNATION_OCTANT, DESIGNATION_ANGLE, DESIGNATION_DIRECTION = 0, 1, 2
NFEAT = 12          # node features of the learned initial guess (snx_gnn_features)

EXPORTS = ["snx_create", "snx_destroy", "snx_last_error", "snx_set_mesh", "snx_set_quadrature",
           "snx_quadrature_product", "snx_set_materials", "snx_set_boundary", "snx_setup", "snx_sweep",
           "snx_solve", "snx_balance", "snx_integrated_flux", "snx_get_levels", "snx_set_schedule",
           "snx_sweep_stats", "snx_profile_sweep", "snx_tune", "snx_batch_create", "snx_batch_destroy",
           "snx_batch_last_error", "snx_batch_set_schedule", "snx_batch_tune", "snx_batch_sweep",
           "snx_batch_solve", "snx_batch_profile_sweep", "snx_batch_stats", "snx_gnn_create", "snx_gnn_destroy",
           "snx_gnn_last_error", "snx_gnn_num_params", "snx_gnn_get_params", "snx_gnn_set_params", "snx_gnn_save",
           "snx_gnn_load", "snx_gnn_features", "snx_gnn_targets", "snx_gnn_forward", "snx_gnn_grad",
           "snx_gnn_train_step", "snx_gnn_train_step_graph", "snx_gnn_create_on",
           "snx_gnn_set_weight_decay", "snx_gnn_predict", "snx_set_sweep_mode", "snx_batch_set_sweep_mode",
           "snx_get_psi", "snx_set_sweep_stats", "snx_batch_set_sweep_stats", "snx_set_designation",
           "snx_designation_stats", "snx_set_group_scattering", "snx_solve_outer", "snx_set_reflective",
           "snx_set_anisotropy", "snx_get_schedule", "snx_batch_solve_outer", "snx_set_order", "snx_get_order",
           "snx_integrated_flux_noalloc", "snx_set_watchdog", "snx_set_staging_depth", "snx_get_staging_depth",
           "snx_batch_set_staging_depth"]
_NO_STATUS = ("snx_destroy", "snx_last_error", "snx_batch_destroy", "snx_batch_last_error", "snx_gnn_destroy",
              "snx_gnn_last_error")


class SnxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class SolveInfo(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("status", ct.c_int32), ("residual", ct.c_double),
                ("wall_ms", ct.c_double), ("solves_per_s", ct.c_double)]


_lib = None
_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_vp = ct.c_void_p


def load(path: str = LIB_PATH):
    """Loads libsnx.so and declares the C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_2510_11513_amd.build`")
    # torch first: its HIP runtime (soname libamdhip64.so.7) then satisfies the
    # library's dependency, so the process holds one runtime, not two.
    import torch  # noqa: F401
    L = ct.CDLL(path)
    L.snx_create.argtypes = [ct.POINTER(_vp), ct.c_int32]
    L.snx_destroy.argtypes = [_vp]
    L.snx_destroy.restype = None
    L.snx_last_error.argtypes = [_vp]
    L.snx_last_error.restype = ct.c_char_p
    L.snx_set_mesh.argtypes = [_vp, ct.c_int64, ct.c_int64, _dp, _ip]
    L.snx_set_quadrature.argtypes = [_vp, ct.c_int32, _dp, _dp]
    L.snx_quadrature_product.argtypes = [ct.c_int32, ct.c_int32, _dp, _dp]
    L.snx_set_materials.argtypes = [_vp, ct.c_int32, _dp, _dp, _dp]
    L.snx_set_boundary.argtypes = [_vp, ct.c_int32, _vp]
    L.snx_setup.argtypes = [_vp, _vp]
    L.snx_sweep.argtypes = [_vp, _vp, _vp, _vp]
    L.snx_solve.argtypes = [_vp, ct.c_double, ct.c_int32, _vp, _vp, ct.POINTER(SolveInfo), _vp]
    L.snx_balance.argtypes = [_vp, _vp, _vp, _dp, _vp]
    L.snx_integrated_flux.argtypes = [_vp, _vp, _dp, _vp]
    L.snx_integrated_flux_noalloc.argtypes = [_vp, _vp, _dp, _vp]
    L.snx_get_levels.argtypes = [_vp, _vp, _vp]
    L.snx_get_psi.argtypes = [_vp, ct.c_int32, ct.c_int32, _vp, _vp]
    L.snx_set_designation.argtypes = [_vp, ct.c_int32]
    L.snx_set_order.argtypes = [_vp, ct.c_int32]
    L.snx_get_order.argtypes = [_vp, _vp, _vp]
    L.snx_set_reflective.argtypes = [_vp, ct.c_int32]
    L.snx_get_schedule.argtypes = [_vp, _vp]
    L.snx_batch_solve_outer.argtypes = [_vp, ct.c_int32, ct.c_int32, ct.c_double, _vp, _vp, _vp, _vp]
    L.snx_set_anisotropy.argtypes = [_vp, ct.c_int32, _vp]
    L.snx_set_group_scattering.argtypes = [_vp, ct.c_int32, _vp, _vp]
    L.snx_solve_outer.argtypes = [_vp, ct.c_int32, ct.c_int32, ct.c_double, _vp, _vp, ct.POINTER(SolveInfo), _vp]
    L.snx_designation_stats.argtypes = [_vp, _vp]
    L.snx_set_sweep_stats.argtypes = [_vp, ct.c_int32]
    L.snx_batch_set_sweep_stats.argtypes = [_vp, ct.c_int32]
    L.snx_set_schedule.argtypes = [_vp, ct.c_int32, ct.c_int32, ct.c_int32]
    L.snx_set_sweep_mode.argtypes = [_vp, ct.c_int32]
    L.snx_batch_set_sweep_mode.argtypes = [_vp, ct.c_int32]
    L.snx_sweep_stats.argtypes = [_vp, _vp]
    L.snx_set_watchdog.argtypes = [_vp, ct.c_double]
    L.snx_set_staging_depth.argtypes = [_vp, ct.c_int32]
    L.snx_get_staging_depth.argtypes = [_vp, ct.POINTER(ct.c_int32)]
    L.snx_batch_set_staging_depth.argtypes = [_vp, ct.c_int32]
    L.snx_profile_sweep.argtypes = [_vp, ct.c_int32, _vp, _vp, ct.POINTER(ct.c_double), _vp]
    L.snx_tune.argtypes = [_vp, ct.c_char_p, _vp, _vp]
    L.snx_batch_create.argtypes = [ct.POINTER(_vp), ct.c_int32, _vp]
    L.snx_batch_destroy.argtypes = [_vp]
    L.snx_batch_destroy.restype = None
    L.snx_batch_last_error.argtypes = [_vp]
    L.snx_batch_last_error.restype = ct.c_char_p
    L.snx_batch_set_schedule.argtypes = [_vp, ct.c_int32, ct.c_int32, ct.c_int32]
    L.snx_batch_tune.argtypes = [_vp, ct.c_char_p, _vp, _vp]
    L.snx_batch_sweep.argtypes = [_vp, _vp, _vp, _vp]
    L.snx_batch_solve.argtypes = [_vp, ct.c_double, ct.c_int32, _vp, _vp, _vp, _vp]
    L.snx_batch_profile_sweep.argtypes = [_vp, ct.c_int32, ct.POINTER(ct.c_double), _vp]
    L.snx_batch_stats.argtypes = [_vp, _vp]
    _fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    L.snx_gnn_create.argtypes = [ct.POINTER(_vp), ct.c_int32, ct.c_int32, ct.c_uint64]
    L.snx_gnn_create_on.argtypes = [ct.POINTER(_vp), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_uint64]
    L.snx_gnn_set_weight_decay.argtypes = [_vp, ct.c_float]
    L.snx_gnn_destroy.argtypes = [_vp]
    L.snx_gnn_destroy.restype = None
    L.snx_gnn_last_error.argtypes = [_vp]
    L.snx_gnn_last_error.restype = ct.c_char_p
    L.snx_gnn_num_params.argtypes = [_vp, ct.POINTER(ct.c_int64)]
    L.snx_gnn_get_params.argtypes = [_vp, _fp]
    L.snx_gnn_set_params.argtypes = [_vp, _fp]
    L.snx_gnn_save.argtypes = [_vp, ct.c_char_p]
    L.snx_gnn_load.argtypes = [_vp, ct.c_char_p]
    L.snx_gnn_features.argtypes = [_vp, _vp, _vp, _vp]
    L.snx_gnn_targets.argtypes = [_vp, ct.c_int64, ct.c_int32, _vp, _vp]
    L.snx_gnn_forward.argtypes = [_vp, _vp, _vp, ct.c_int64, ct.c_int32, _vp, _vp]
    L.snx_gnn_grad.argtypes = [_vp, _vp, _vp, ct.c_int64, ct.c_int32, _vp, ct.POINTER(ct.c_float), _vp, _vp]
    L.snx_gnn_train_step.argtypes = [_vp, _vp, _vp, ct.c_float, ct.POINTER(ct.c_float), _vp]
    L.snx_gnn_train_step_graph.argtypes = [_vp, _vp, _vp, ct.c_int64, ct.c_int32, _vp, ct.c_float, ct.c_float,
                                           ct.POINTER(ct.c_float), _vp]
    L.snx_gnn_predict.argtypes = [_vp, _vp, _vp, _vp]
    for name in EXPORTS:
        if name not in _NO_STATUS:
            getattr(L, name).restype = ct.c_int32
    _lib = L
    return L


def quadrature_product(npolar: int, nazim: int):
    """Product quadrature from the library: (omega[8*npolar*nazim][3], w[...])."""
    nang = 8 * npolar * nazim
    om = np.zeros((nang, 3))
    w = np.zeros(nang)
    rc = load().snx_quadrature_product(npolar, nazim, om, w)
    if rc:
        raise SnxError(rc, "quadrature_product")
    return om, w


def _ptr(t):
    if t is None:
        return None
    return ct.c_void_p(t.data_ptr())


def _init_torch():
    """Initialise torch's HIP context before the library's first device call."""
    import torch
    torch.cuda.init()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


class Problem:
    """One transport problem resident on a GPU.

    Flux tensors are torch.float32 of shape [ncell, G, 8] on the problem's
    device (the exchange layout of the C ABI).
    """

    def __init__(self, device: int = 0):
        L = load()
        _init_torch()
        h = ct.c_void_p()
        rc = L.snx_create(ct.byref(h), device)
        if rc:
            raise SnxError(rc, L.snx_last_error(None).decode())
        self.h = h
        self.device = device
        self.ncell = self.G = self.nang = 0
        self.nodes = 8          # nodes per cell: (order + 1)^3

    def _check(self, rc, what, allow=()):
        if rc and rc not in allow:
            raise SnxError(rc, f"{what}: {load().snx_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().snx_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- inputs
    def set_mesh(self, xyz, cell_vert):
        xyz = np.ascontiguousarray(xyz, np.float64)
        cv = np.ascontiguousarray(cell_vert, np.int32)
        self._check(load().snx_set_mesh(self.h, cv.shape[0], xyz.shape[0], xyz, cv), "set_mesh")
        self.ncell = cv.shape[0]

    def set_quadrature(self, omega, w):
        om = np.ascontiguousarray(omega, np.float64)
        w = np.ascontiguousarray(w, np.float64)
        self._check(load().snx_set_quadrature(self.h, om.shape[0], om, w), "set_quadrature")
        self.nang = om.shape[0]

    def set_materials(self, sigma_t, sigma_s, q):
        st = np.ascontiguousarray(sigma_t, np.float64)
        ss = np.ascontiguousarray(sigma_s, np.float64)
        qq = np.ascontiguousarray(q, np.float64)
        self._check(load().snx_set_materials(self.h, st.shape[1], st, ss, qq), "set_materials")
        self.G = st.shape[1]

    def set_boundary(self, kind: int, psi_in=None):
        arr = None if psi_in is None else np.ascontiguousarray(psi_in, np.float64)
        ptr = None if arr is None else arr.ctypes.data_as(ct.c_void_p)
        self._check(load().snx_set_boundary(self.h, kind, ptr), "set_boundary")

    def set_anisotropy(self, sigma_l):
        """sigma_l[ncell][G][L] (L <= 3): Legendre moments 1..L of the within-group
        scattering law; None restores isotropic scattering.  Takes effect at setup."""
        if sigma_l is None:
            self._check(load().snx_set_anisotropy(self.h, 0, None), "set_anisotropy")
            return
        sl = np.ascontiguousarray(sigma_l, np.float64)
        if sl.ndim != 3:
            raise ValueError("sigma_l must be [ncell][G][L]")
        self._check(load().snx_set_anisotropy(self.h, sl.shape[2], sl.ctypes.data_as(ct.c_void_p)),
                    "set_anisotropy")

    def set_reflective(self, planes: int):
        """Reflective boundary planes, bit 2*axis + side; takes effect at setup."""
        self._check(load().snx_set_reflective(self.h, int(planes)), "set_reflective")

    def set_group_scattering(self, cell_mat, sigma_gg):
        """Group-to-group scattering: cell_mat[ncell] material ids, sigma_gg[nmat][G][G]
        from group g' (axis 1) into g (axis 2); None removes it.  Takes effect at setup."""
        if sigma_gg is None:
            self._check(load().snx_set_group_scattering(self.h, 0, None, None), "set_group_scattering")
            return
        cm = np.ascontiguousarray(cell_mat, np.int32)
        sg = np.ascontiguousarray(sigma_gg, np.float64)
        if sg.ndim != 3 or sg.shape[1] != sg.shape[2] or cm.ndim != 1:
            raise ValueError("cell_mat must be [ncell] and sigma_gg [nmat][G][G]")
        self._check(load().snx_set_group_scattering(self.h, sg.shape[0], cm.ctypes.data_as(ct.c_void_p),
                                                    sg.ctypes.data_as(ct.c_void_p)), "set_group_scattering")

    def set_order(self, order: int):
        """Element order 1, 2 or 3 (nodes per cell (order + 1)^3); takes effect at setup."""
        self._check(load().snx_set_order(self.h, int(order)), "set_order")
        self.nodes = (int(order) + 1) ** 3

    def set_designation(self, kind: int):
        """DESIGNATION_OCTANT (default) or DESIGNATION_ANGLE (per direction, lagged
        faces where a direction goes against its octant's order); takes effect at setup."""
        self._check(load().snx_set_designation(self.h, int(kind)), "set_designation")

    def designation_stats(self):
        out = np.zeros(4, np.int64)
        self._check(load().snx_designation_stats(self.h, out.ctypes.data_as(ct.c_void_p)), "designation_stats")
        return {"designation": int(out[0]), "differing": int(out[1]), "lagged": int(out[2]), "tasks": int(out[3])}

    def setup(self, stream=None):
        self._check(load().snx_setup(self.h, _stream(stream)), "setup")

    @classmethod
    def from_problem(cls, prob, device: int = 0, setup: bool = True, quadrature=None, designation: int = 0,
                     order: int = 1):
        """Loads a generated problem (paper_2510_11513_amd.inputs.Problem) into the library."""
        p = cls(device)
        if designation:
            p.set_designation(designation)
        if order != 1:
            p.set_order(order)
        p.set_mesh(prob.mesh.xyz, prob.mesh.cell_vert)
        om, w = quadrature if quadrature is not None else quadrature_product(prob.npolar, prob.nazim)
        p.set_quadrature(om, w)
        p.set_materials(prob.mat.sigma_t, prob.mat.sigma_s, prob.mat.q)
        if prob.boundary_kind:
            p.set_boundary(prob.boundary_kind, prob.psi_b)
        if setup:
            p.setup()
        return p

    # ------------------------------------------------------------- compute
    def empty_phi(self):
        import torch
        return torch.empty((self.ncell, self.G, self.nodes), dtype=torch.float32, device=f"cuda:{self.device}")

    def _flux(self, *ts):
        """Refuses flux tensors of the wrong size before the library reads them."""
        want = self.ncell * self.G * self.nodes
        if want == 0:       # no mesh or materials yet: the library reports the state error
            return
        for t in ts:
            if t is not None and (t.numel() != want or not t.is_contiguous()):
                raise ValueError(f"flux arrays hold [ncell][G][{self.nodes}] contiguous floats")

    def sweep(self, phi_in=None, phi_out=None, stream=None):
        if phi_out is None:
            phi_out = self.empty_phi()
        self._flux(phi_in, phi_out)
        self._check(load().snx_sweep(self.h, _ptr(phi_in), _ptr(phi_out), _stream(stream)), "sweep")
        return phi_out

    def solve(self, tol: float, max_it: int, phi0=None, phi=None, stream=None, allow_noconv=False):
        if phi is None:
            phi = self.empty_phi()
        self._flux(phi0, phi)
        info = SolveInfo()
        rc = load().snx_solve(self.h, tol, max_it, _ptr(phi0), _ptr(phi), ct.byref(info), _stream(stream))
        self._check(rc, "solve", allow=(SNX_E_NOCONV,) if allow_noconv else ())
        return phi, {"iterations": info.iterations, "status": info.status, "residual": info.residual,
                     "wall_ms": info.wall_ms, "solves_per_s": info.solves_per_s, "rc": rc}

    def solve_outer(self, outer: int, inner: int, tol: float = 0.0, phi0=None, phi=None, stream=None,
                    allow_noconv=False):
        """Inner/outer iterations (snx_solve_outer); returns (phi, info)."""
        if phi is None:
            phi = self.empty_phi()
        info = SolveInfo()
        rc = load().snx_solve_outer(self.h, int(outer), int(inner), float(tol), _ptr(phi0), _ptr(phi),
                                    ct.byref(info), _stream(stream))
        self._check(rc, "solve_outer", allow=(SNX_E_NOCONV,) if allow_noconv else ())
        return phi, {"iterations": info.iterations, "status": info.status, "residual": info.residual,
                     "wall_ms": info.wall_ms, "solves_per_s": info.solves_per_s, "rc": rc}

    def balance(self, phi_in, phi_out, stream=None):
        out = np.zeros((self.G, 4))
        self._check(load().snx_balance(self.h, _ptr(phi_in), _ptr(phi_out), out, _stream(stream)), "balance")
        return out

    def integrated_flux(self, phi, stream=None):
        out = np.zeros((self.G, 2))
        self._check(load().snx_integrated_flux(self.h, _ptr(phi), out, _stream(stream)), "integrated_flux")
        return out

    def integrated_flux_noalloc(self, phi, stream=None):
        """As integrated_flux, through the library's fixed device scratch (allocates nothing)."""
        out = np.zeros((self.G, 2))
        self._check(load().snx_integrated_flux_noalloc(self.h, _ptr(phi), out, _stream(stream)),
                    "integrated_flux_noalloc")
        return out

    def levels(self):
        lev = np.zeros((8, self.ncell), np.int32)
        nl = np.zeros(8, np.int32)
        self._check(load().snx_get_levels(self.h, lev.ctypes.data_as(ct.c_void_p), nl.ctypes.data_as(ct.c_void_p)),
                    "get_levels")
        return lev, nl

    def psi(self, angle: int, group: int, stream=None):
        """psi[ncell][nodes] (device, FP32) of one direction and group from the last sweep."""
        import torch
        out = torch.empty((self.ncell, self.nodes), dtype=torch.float32, device=f"cuda:{self.device}")
        self._check(load().snx_get_psi(self.h, int(angle), int(group), _ptr(out), _stream(stream)), "get_psi")
        return out

    def set_schedule(self, threads: int = 0, wg_per_cu: int = 0, chunk: int = 0):
        self._check(load().snx_set_schedule(self.h, threads, wg_per_cu, chunk), "set_schedule")

    def schedule(self):
        """The sweep schedule: threads, workgroups per CU (0: occupancy), chunk, mode."""
        out = np.zeros(4, np.int32)
        self._check(load().snx_get_schedule(self.h, out.ctypes.data_as(ct.c_void_p)), "get_schedule")
        return {"threads": int(out[0]), "wg_per_cu": int(out[1]), "chunk": int(out[2]), "mode": int(out[3])}

    def set_sweep_mode(self, mode: int):
        """SWEEP_AMT (dependency-driven, default) or SWEEP_BSP (level by level, the comparator)."""
        self._check(load().snx_set_sweep_mode(self.h, mode), "set_sweep_mode")

    def profile_sweep(self, nsweeps: int, phi_in=None, phi_out=None, stream=None) -> float:
        """Mean duration (ms) of the sweep kernel alone, from HIP events on its stream."""
        if phi_out is None:
            phi_out = self.empty_phi()
        self._flux(phi_in, phi_out)
        ms = ct.c_double(0.0)
        self._check(load().snx_profile_sweep(self.h, nsweeps, _ptr(phi_in), _ptr(phi_out), ct.byref(ms),
                                             _stream(stream)), "profile_sweep")
        return ms.value

    def tune(self, cache_path=None, stream=None):
        """Autotunes the sweep schedule on this problem; returns (threads, workgroups per CU)."""
        chosen = np.zeros(2, np.int32)
        path = None if cache_path is None else str(cache_path).encode()
        self._check(load().snx_tune(self.h, path, chosen.ctypes.data_as(ct.c_void_p), _stream(stream)), "tune")
        return int(chosen[0]), int(chosen[1])

    def sweep_stats(self):
        out = np.zeros(11, np.int64)
        self._check(load().snx_sweep_stats(self.h, out.ctypes.data_as(ct.c_void_p)), "sweep_stats")
        return _stats(out)

    def set_staging_depth(self, depth: int):
        """1: inputs requested one task (traces) or round ahead; 0: at their start (same bits)."""
        self._check(load().snx_set_staging_depth(self.h, int(depth)), "set_staging_depth")

    def staging_depth(self) -> int:
        d = ct.c_int32()
        self._check(load().snx_get_staging_depth(self.h, ct.byref(d)), "get_staging_depth")
        return int(d.value)

    def set_watchdog(self, seconds: float):
        """Wall-clock limit on a dependency-driven sweep's wait for a ready task (<= 0: the 20 s default)."""
        self._check(load().snx_set_watchdog(self.h, float(seconds)), "set_watchdog")

    def set_sweep_stats(self, phases: bool):
        """Per-phase cycle statistics in sweep_stats() (off by default: they cost ~2 % of sweep time)."""
        self._check(load().snx_set_sweep_stats(self.h, int(bool(phases))), "set_sweep_stats")


def _stats(out):
    return {"tasks": int(out[0]), "empty_polls": int(out[1]), "abort": int(out[2]), "grid": int(out[3]),
            "continued": int(out[4]), "threads": int(out[5]),
            "cycles": dict(zip(("queue_wait", "stage", "build", "solve", "publish"), map(int, out[6:11])))}


def _ptr_array(tensors):
    arr = (ct.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


class Batch:
    """Independent set-up problems sharing every sweep launch (see snx_batch_* in snx.h)."""

    def __init__(self, problems):
        L = load()
        self.problems = list(problems)       # keeps the problems alive
        hs = (ct.c_void_p * len(self.problems))(*[p.h.value for p in self.problems])
        h = ct.c_void_p()
        rc = L.snx_batch_create(ct.byref(h), len(self.problems), hs)
        if rc:
            raise SnxError(rc, L.snx_batch_last_error(None).decode())
        self.h = h

    def _check(self, rc, what, allow=()):
        if rc and rc not in allow:
            raise SnxError(rc, f"{what}: {load().snx_batch_last_error(self.h).decode()}")
        return rc

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().snx_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, threads: int = 0, wg_per_cu: int = 0, chunk: int = 0):
        self._check(load().snx_batch_set_schedule(self.h, threads, wg_per_cu, chunk), "batch_set_schedule")

    def set_sweep_mode(self, mode: int):
        self._check(load().snx_batch_set_sweep_mode(self.h, mode), "batch_set_sweep_mode")

    def set_staging_depth(self, depth: int):
        self._check(load().snx_batch_set_staging_depth(self.h, int(depth)), "batch_set_staging_depth")

    def tune(self, cache_path=None, stream=None):
        chosen = np.zeros(2, np.int32)
        path = None if cache_path is None else str(cache_path).encode()
        self._check(load().snx_batch_tune(self.h, path, chosen.ctypes.data_as(ct.c_void_p), _stream(stream)),
                    "batch_tune")
        return int(chosen[0]), int(chosen[1])

    def sweep(self, phi_in=None, phi_out=None, stream=None):
        if phi_out is None:
            phi_out = [p.empty_phi() for p in self.problems]
        pin = None if phi_in is None else _ptr_array(phi_in)
        self._check(load().snx_batch_sweep(self.h, pin, _ptr_array(phi_out), _stream(stream)), "batch_sweep")
        return phi_out

    def solve(self, tol: float, max_it: int, phi0=None, phi=None, stream=None, allow_noconv=False):
        if phi is None:
            phi = [p.empty_phi() for p in self.problems]
        infos = (SolveInfo * len(self.problems))()
        p0 = None if phi0 is None else _ptr_array(phi0)
        rc = load().snx_batch_solve(self.h, tol, max_it, p0, _ptr_array(phi), infos, _stream(stream))
        self._check(rc, "batch_solve", allow=(SNX_E_NOCONV,) if allow_noconv else ())
        return phi, [{"iterations": i.iterations, "status": i.status, "residual": i.residual,
                      "wall_ms": i.wall_ms, "solves_per_s": i.solves_per_s} for i in infos], rc

    def solve_outer(self, outer: int, inner: int, tol: float = 0.0, phi0=None, phi=None, stream=None,
                    allow_noconv=False):
        """Inner/outer iterations of every problem (snx_batch_solve_outer)."""
        if phi is None:
            phi = [p.empty_phi() for p in self.problems]
        infos = (SolveInfo * len(self.problems))()
        p0 = None if phi0 is None else _ptr_array(phi0)
        rc = load().snx_batch_solve_outer(self.h, int(outer), int(inner), float(tol), p0, _ptr_array(phi), infos,
                                          _stream(stream))
        self._check(rc, "batch_solve_outer", allow=(SNX_E_NOCONV,) if allow_noconv else ())
        return phi, [{"iterations": i.iterations, "status": i.status, "residual": i.residual,
                      "wall_ms": i.wall_ms, "solves_per_s": i.solves_per_s} for i in infos], rc

    def profile_sweep(self, nsweeps: int, stream=None) -> float:
        ms = ct.c_double(0.0)
        self._check(load().snx_batch_profile_sweep(self.h, nsweeps, ct.byref(ms), _stream(stream)),
                    "batch_profile_sweep")
        return ms.value

    def stats(self):
        out = np.zeros(11, np.int64)
        self._check(load().snx_batch_stats(self.h, out.ctypes.data_as(ct.c_void_p)), "batch_stats")
        return _stats(out)

    def set_sweep_stats(self, phases: bool):
        self._check(load().snx_batch_set_sweep_stats(self.h, int(bool(phases))), "batch_set_sweep_stats")


class Gnn:
    """The message-passing network of the learned initial guess, on one GPU.

    Device inputs are torch tensors: features x [C*G, NFEAT] float32, adjacency
    nbr [C, 6] int32, targets y [C*G] float32.
    """

    def __init__(self, device: int = 0, layers: int = 4, seed: int = 0, hidden: int = 64):
        L = load()
        _init_torch()
        h = ct.c_void_p()
        rc = L.snx_gnn_create_on(ct.byref(h), device, hidden, layers, seed)
        if rc:
            raise SnxError(rc, L.snx_gnn_last_error(None).decode())
        self.h = h
        self.device = device
        self.layers = layers
        n = ct.c_int64()
        self._check(L.snx_gnn_num_params(h, ct.byref(n)), "num_params")
        self.nparams = n.value

    def _check(self, rc, what):
        if rc:
            raise SnxError(rc, f"{what}: {load().snx_gnn_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().snx_gnn_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(self.nparams, np.float32)
        self._check(load().snx_gnn_get_params(self.h, out), "get_params")
        return out

    def set_params(self, theta):
        arr = np.ascontiguousarray(theta, np.float32)
        if arr.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {arr.size}")
        self._check(load().snx_gnn_set_params(self.h, arr), "set_params")

    def save(self, path):
        self._check(load().snx_gnn_save(self.h, os.fsencode(str(path))), "save")

    def load_file(self, path):
        self._check(load().snx_gnn_load(self.h, os.fsencode(str(path))), "load")

    @staticmethod
    def features(problem: "Problem", stream=None):
        """(x [C*G, NFEAT], nbr [C, 6]) of a set-up problem, on its device."""
        import torch
        dev = torch.device("cuda", problem.device)
        x = torch.empty((problem.ncell * problem.G, NFEAT), dtype=torch.float32, device=dev)
        nbr = torch.empty((problem.ncell, 6), dtype=torch.int32, device=dev)
        rc = load().snx_gnn_features(problem.h, _ptr(x), _ptr(nbr), _stream(stream))
        problem._check(rc, "gnn_features")
        return x, nbr

    @staticmethod
    def targets(phi, stream=None):
        import torch
        C, G = phi.shape[0], phi.shape[1]
        y = torch.empty(C * G, dtype=torch.float32, device=phi.device)
        rc = load().snx_gnn_targets(_ptr(phi.contiguous()), C, G, _ptr(y), _stream(stream))
        if rc:
            raise SnxError(rc, "gnn_targets")
        return y

    @staticmethod
    def _shape(x, nbr):
        C = nbr.shape[0]
        if x.shape[0] % C or x.shape[1] != NFEAT or nbr.shape[1] != 6:
            raise ValueError(f"x must be [C*G, {NFEAT}] and nbr [C, 6]")
        if x.dtype.itemsize != 4 or nbr.dtype.itemsize != 4 or not x.is_contiguous() or not nbr.is_contiguous():
            raise ValueError("x float32 and nbr int32, contiguous")
        return C, x.shape[0] // C

    def forward(self, x, nbr, stream=None):
        import torch
        C, G = self._shape(x, nbr)
        z = torch.empty(C * G, dtype=torch.float32, device=x.device)
        self._check(load().snx_gnn_forward(self.h, _ptr(x), _ptr(nbr), C, G, _ptr(z), _stream(stream)), "forward")
        return z

    def grad(self, x, nbr, y, stream=None):
        C, G = self._shape(x, nbr)
        loss = ct.c_float()
        g = np.zeros(self.nparams, np.float32)
        self._check(load().snx_gnn_grad(self.h, _ptr(x), _ptr(nbr), C, G, _ptr(y), ct.byref(loss),
                                        g.ctypes.data_as(ct.c_void_p), _stream(stream)), "grad")
        return loss.value, g

    def train_step(self, x, nbr, y, lr: float, weight_decay: float = 0.0, stream=None) -> float:
        """One AdamW step on a stored graph (snx_gnn_train_step_graph); returns the loss before it."""
        C, G = self._shape(x, nbr)
        loss = ct.c_float()
        self._check(load().snx_gnn_train_step_graph(self.h, _ptr(x), _ptr(nbr), C, G, _ptr(y), lr, weight_decay,
                                                    ct.byref(loss), _stream(stream)), "train_step_graph")
        return loss.value

    def train_step_problem(self, problem: "Problem", phi_target, lr: float, stream=None) -> float:
        """One AdamW step towards a converged flux of a set-up problem (snx_gnn_train_step)."""
        if phi_target.numel() != problem.ncell * problem.G * 8 or not phi_target.is_contiguous():
            raise ValueError("phi_target holds [ncell][G][8] contiguous floats")
        loss = ct.c_float()
        self._check(load().snx_gnn_train_step(self.h, problem.h, _ptr(phi_target), lr, ct.byref(loss),
                                              _stream(stream)), "train_step")
        return loss.value

    def set_weight_decay(self, weight_decay: float):
        self._check(load().snx_gnn_set_weight_decay(self.h, weight_decay), "set_weight_decay")

    def predict(self, problem: "Problem", stream=None):
        """Starting flux [C, G, 8] of a set-up problem."""
        phi0 = problem.empty_phi()
        self._check(load().snx_gnn_predict(self.h, problem.h, _ptr(phi0), _stream(stream)), "predict")
        return phi0
