"""Python binding of the MI355X harmonic-balance GLS Navier-Stokes library.

Argument marshalling only: every step of the computation runs in the HIP
library ``libhb.so`` (see include/hb.h for the meaning, layout and
ownership of each argument).  PyTorch provides device memory and streams.
The binding raises if the library is missing; it never falls back to
another implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhb.so")

HB_OK, HB_ERR_ARG, HB_ERR_MESH, HB_ERR_DEVICE, HB_ERR_NOCONV, HB_ERR_NAN, HB_ERR_OOM = (
    0, -1, -2, -3, -4, -5, -6)
HB_JV_EXACT, HB_JV_PAPER, HB_F64, HB_F32 = 0, 1, 0, 2
HB_MIXED = 1
HB_F32_BASIS = 2
HB_PREC_JACOBI, HB_PREC_NODE_TIME, HB_PREC_MEANFLOW = 0, 1, 2


class HBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hb status {status}: {msg}")
        self.status = status


class _Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("period", C.c_double),
                ("K", C.c_int32), ("C_I", C.c_double), ("beta_bf", C.c_double)]


class _BC(C.Structure):
    _fields_ = [("dirichlet", C.c_void_p), ("outlet_h", C.c_void_p), ("outlet_R", C.c_void_p)]


class _TmStep(C.Structure):
    _fields_ = [("dt", C.c_double), ("omega_hat", C.c_double), ("y_old", C.c_void_p),
                ("a_old", C.c_void_p), ("dirichlet", C.c_void_p), ("outlet_h", C.c_void_p),
                ("outlet_R", C.c_void_p)]


class _TmOpts(C.Structure):
    _fields_ = [("t0", C.c_double), ("dt", C.c_double), ("n_steps", C.c_int32),
                ("rtol", C.c_double), ("atol", C.c_double), ("gmres_eta", C.c_double),
                ("restart", C.c_int32), ("max_newton", C.c_int32), ("max_gmres", C.c_int32),
                ("omega_hat", C.c_double), ("verbose", C.c_int32), ("precond", C.c_int32)]


class _TmReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("newton_iters", C.c_int32), ("gmres_iters", C.c_int32),
                ("status", C.c_int32), ("max_step_residual", C.c_double), ("wall_s", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("r_ref", C.c_double), ("gmres_eta", C.c_double),
                ("cfl", C.c_double), ("c1", C.c_double), ("restart", C.c_int32),
                ("max_newton", C.c_int32), ("max_gmres", C.c_int32), ("precision", C.c_int32),
                ("jv_kind", C.c_int32), ("verbose", C.c_int32), ("precond", C.c_int32),
                ("cfl_max", C.c_double), ("graphs", C.c_int32), ("amg_sweeps", C.c_int32),
                ("amg_cycles", C.c_int32), ("amg_weight", C.c_double),
                ("reject_ratio", C.c_double), ("dt_growth", C.c_double),
                ("amg_aggregation", C.c_int32), ("amg_coarse_weight", C.c_double),
                ("amg_smoother", C.c_int32), ("amg_wcycle", C.c_int32),
                ("amg_fp32", C.c_int32), ("forcing", C.c_int32)]


class _PcOpts(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("cycles", C.c_int32), ("weight", C.c_double),
                ("coarse_max", C.c_int32), ("aggregation", C.c_int32),
                ("coarse_weight", C.c_double), ("smoother", C.c_int32), ("wcycle", C.c_int32),
                ("fp32", C.c_int32)]


class _Report(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("gmres_iters", C.c_int32), ("status", C.c_int32),
                ("r0", C.c_double), ("r_final", C.c_double), ("r_ref", C.c_double),
                ("wall_s", C.c_double), ("jv_ms", C.c_double), ("n_jv", C.c_int32),
                ("rejected", C.c_int32), ("pc_ms", C.c_double), ("mass_defect", C.c_double)]


_lib = None


def load():
    """Load libhb.so (built by paper_2411_14315_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HBError(HB_ERR_DEVICE, f"{LIB_PATH} is missing: run paper_2411_14315_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.hb_mesh_create.argtypes = [i64, vp, i64, vp, i64, vp, vp, i32, vp, C.POINTER(vp)]
    lib.hb_mesh_destroy.argtypes = [vp]
    lib.hb_mesh_destroy.restype = None
    lib.hb_mesh_info.argtypes = [vp, vp]
    lib.hb_residual.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp, vp, vp]
    lib.hb_jvp.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp, vp, vp, i32, vp]
    lib.hb_jacobi.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp, dbl, vp, vp]
    lib.hb_tm_residual.argtypes = [vp, C.POINTER(_Params), C.POINTER(_TmStep), vp, vp, vp]
    lib.hb_tm_jvp.argtypes = [vp, C.POINTER(_Params), C.POINTER(_TmStep), vp, vp, vp, vp]
    lib.hb_tm_march.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp, vp, vp,
                                C.POINTER(_TmOpts), C.POINTER(_TmReport), vp]
    lib.hb_newton_solve.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp,
                                    C.POINTER(_Opts), C.POINTER(_Report), vp]
    lib.hb_set_timing.argtypes = [vp, i32]
    lib.hb_last_timings.argtypes = [vp, vp]
    lib.hb_mlp_create.argtypes = [i32, vp, vp, C.c_uint64, C.POINTER(vp)]
    lib.hb_mlp_destroy.argtypes = [vp]
    lib.hb_mlp_destroy.restype = None
    lib.hb_mlp_num_params.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.hb_mlp_get_params.argtypes = [vp, vp]
    lib.hb_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
    lib.hb_mlp_forward_noalloc.argtypes = [vp, vp, i32, vp, vp]
    lib.hb_mlp_loss_grad.argtypes = [vp, vp, vp, i32, vp, C.POINTER(C.c_double), vp]
    lib.hb_mlp_adam_step.argtypes = [vp, vp, C.c_float, vp]
    lib.hb_pod_expand.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp]
    lib.hb_pod_fit.argtypes = [vp, vp, i64, i64, i32, dbl, vp, vp, vp, vp, C.POINTER(i32), vp]
    lib.hb_sym_eig.argtypes = [i32, vp, vp, vp]
    lib.hb_precond_apply.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp, dbl,
                                     C.POINTER(_PcOpts), i32, vp, vp, vp]
    lib.hb_precond_levels.argtypes = [vp, vp, i32, C.POINTER(i32)]
    lib.hb_precond_hierarchy.argtypes = [i64, i64, vp, i32, i32, i32, vp, C.POINTER(i32), vp, vp]
    lib.hb_outlet_flow.argtypes = [vp, C.POINTER(_Params), C.POINTER(_BC), vp, vp, vp, vp]
    lib.hb_last_error.restype = C.c_char_p
    for name in ("hb_mesh_create", "hb_mesh_info", "hb_residual", "hb_jvp", "hb_jacobi",
                 "hb_newton_solve", "hb_set_timing", "hb_last_timings", "hb_mlp_create",
                 "hb_mlp_num_params", "hb_mlp_get_params", "hb_mlp_forward",
                 "hb_mlp_forward_noalloc", "hb_mlp_loss_grad",
                 "hb_mlp_adam_step", "hb_pod_expand", "hb_pod_fit", "hb_sym_eig",
                 "hb_tm_residual", "hb_tm_jvp",
                 "hb_tm_march", "hb_precond_apply", "hb_precond_levels", "hb_outlet_flow",
                 "hb_precond_hierarchy"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != HB_OK:
        raise HBError(status, load().hb_last_error().decode())


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise HBError(HB_ERR_ARG, "expected a contiguous device tensor")
    return t.data_ptr()


def _arg(t, name, shape, dtypes=("float64",), device=None):
    """Check a device tensor argument before anything is launched: contiguous,
    on the device, of one of ``dtypes`` and exactly ``shape``; same device as
    ``device`` if given.  Returns its pointer."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise HBError(HB_ERR_ARG, f"{name}: expected a device tensor")
    if str(t.dtype).replace("torch.", "") not in dtypes:
        raise HBError(HB_ERR_ARG, f"{name}: dtype {t.dtype}, expected {'/'.join(dtypes)}")
    if tuple(t.shape) != tuple(shape):
        raise HBError(HB_ERR_ARG, f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_cuda or not t.is_contiguous():
        raise HBError(HB_ERR_ARG, f"{name}: expected a contiguous device tensor")
    if device is not None and t.device != device:
        raise HBError(HB_ERR_ARG, f"{name}: on {t.device}, expected {device}")
    return t.data_ptr()


def _host(a, name, shape):
    """Check a host array argument (None allowed) and return its pointer."""
    if a is None:
        return None
    if a.dtype != np.float64 or a.shape != tuple(shape) or not a.flags.c_contiguous:
        raise HBError(HB_ERR_ARG, f"{name}: expected float64 {tuple(shape)}, got "
                                  f"{a.dtype} {a.shape}")
    return a.ctypes.data


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Mesh:
    """Owns an hb_mesh handle; built from host arrays."""

    def __init__(self, xyz, tets, faces, face_group, group_kind):
        lib = load()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        faces = np.ascontiguousarray(faces, dtype=np.int32)
        face_group = np.ascontiguousarray(face_group, dtype=np.int32)
        group_kind = np.ascontiguousarray(group_kind, dtype=np.int32)
        h = C.c_void_p()
        _check(lib.hb_mesh_create(xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data,
                                  faces.shape[0], faces.ctypes.data, face_group.ctypes.data,
                                  group_kind.shape[0], group_kind.ctypes.data, C.byref(h)))
        self._h = h
        self.n_nodes = xyz.shape[0]
        self.n_outlets = int(np.sum(group_kind == 2))

    @classmethod
    def from_mesh(cls, m):
        return cls(m.xyz, m.tets, m.faces, m.face_group, m.group_kind)

    def info(self) -> dict:
        out = np.zeros(8, np.int64)
        _check(load().hb_mesh_info(self._h, out.ctypes.data))
        keys = ("n_nodes", "n_tets", "n_dirichlet", "n_outlet_faces", "n_outlets",
                "n_reoriented", "n_inlet", "device_bytes")
        return dict(zip(keys, map(int, out)))

    def set_timing(self, enable: bool = True):
        _check(load().hb_set_timing(self._h, 1 if enable else 0))

    STAGES = ("state_to_samples", "direction_to_samples", "outlet_flux", "element",
              "outlet_faces", "samples_to_modal")

    def last_timings(self) -> dict:
        out = np.zeros(6)
        _check(load().hb_last_timings(self._h, out.ctypes.data))
        return dict(zip(self.STAGES, map(float, out)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hb_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Params:
    rho: float = 1.06
    mu: float = 0.04
    period: float = 1.0
    K: int = 2
    C_I: float = 3.0
    beta_bf: float = 0.2

    @property
    def N(self):
        return 2 * self.K + 1

    def _c(self):
        return _Params(self.rho, self.mu, self.period, self.K, self.C_I, self.beta_bf)


class BC:
    """Boundary data: ``dirichlet`` a device tensor (3, N, n); ``outlet_h``
    host (n_outlets, N) modal traction or None; ``outlet_R`` host
    (n_outlets,) or None."""

    def __init__(self, dirichlet, outlet_h=None, outlet_R=None):
        self.dirichlet = dirichlet
        self.outlet_h = None if outlet_h is None else np.ascontiguousarray(outlet_h, np.float64)
        self.outlet_R = None if outlet_R is None else np.ascontiguousarray(outlet_R, np.float64)

    def _c(self, mesh=None, N=None):
        if mesh is None:
            return _BC(_ptr(self.dirichlet),
                       None if self.outlet_h is None else self.outlet_h.ctypes.data,
                       None if self.outlet_R is None else self.outlet_R.ctypes.data)
        no = mesh.n_outlets
        hp = _host(self.outlet_h, "bc.outlet_h", (no, N))
        rp = _host(self.outlet_R, "bc.outlet_R", (no,))
        return _BC(_arg(self.dirichlet, "bc.dirichlet", (3, N, mesh.n_nodes)), hp, rp)


def _params(p):
    if isinstance(p, Params):
        return p
    return Params(p.rho, p.mu, p.period, p.K, p.C_I, p.beta_bf)


def _modal_shape(mesh, p):
    return (4, p.N, mesh.n_nodes)


def residual(mesh: Mesh, params, bc: BC, Y, R=None, stream=None):
    import torch
    p = _params(params)
    shp = _modal_shape(mesh, p)
    yp = _arg(Y, "Y", shp)
    if R is None:
        R = torch.empty_like(Y)
    rp = _arg(R, "R", shp, device=Y.device)
    pc, bcc = p._c(), bc._c(mesh, p.N)
    _check(load().hb_residual(mesh._h, C.byref(pc), C.byref(bcc), yp, rp, _stream(stream)))
    return R


def jvp(mesh: Mesh, params, bc: BC, Y, V, JV=None, kind: str = "exact", stream=None):
    import torch
    p = _params(params)
    shp = _modal_shape(mesh, p)
    yp = _arg(Y, "Y", shp)
    vp_ = _arg(V, "V", shp, ("float64", "float32"), device=Y.device)
    if JV is None:
        JV = torch.empty_like(V)
    jp = _arg(JV, "JV", shp, (str(V.dtype).replace("torch.", ""),), device=Y.device)
    if kind not in ("exact", "paper"):
        raise HBError(HB_ERR_ARG, f"unknown tangent kind {kind!r}")
    flags = HB_JV_EXACT if kind == "exact" else HB_JV_PAPER
    if V.dtype == torch.float32:
        flags |= HB_F32
    pc, bcc = p._c(), bc._c(mesh, p.N)
    _check(load().hb_jvp(mesh._h, C.byref(pc), C.byref(bcc), yp, vp_, jp, flags, _stream(stream)))
    return JV


class TmStep:
    """One time-marching step's data: ``y_old`` device (4, n) state at t_n,
    ``a_old`` device (3, n) acceleration at t_n, ``dirichlet`` device (3, n)
    Dirichlet velocity at t_{n+1}; ``outlet_h`` and ``outlet_R`` host
    (n_outlets,) or None."""

    def __init__(self, dt, omega_hat, y_old, a_old, dirichlet, outlet_h=None, outlet_R=None):
        self.dt, self.omega_hat = float(dt), float(omega_hat)
        self.y_old, self.a_old, self.dirichlet = y_old, a_old, dirichlet
        self.outlet_h = None if outlet_h is None else np.ascontiguousarray(outlet_h, np.float64)
        self.outlet_R = None if outlet_R is None else np.ascontiguousarray(outlet_R, np.float64)

    def _c(self, mesh):
        n, no = mesh.n_nodes, mesh.n_outlets
        return _TmStep(self.dt, self.omega_hat, _arg(self.y_old, "tm.y_old", (4, n)),
                       _arg(self.a_old, "tm.a_old", (3, n)),
                       _arg(self.dirichlet, "tm.dirichlet", (3, n)),
                       _host(self.outlet_h, "tm.outlet_h", (no,)),
                       _host(self.outlet_R, "tm.outlet_R", (no,)))


def tm_residual(mesh: Mesh, params, tm: TmStep, Y, R=None, stream=None):
    import torch
    n = mesh.n_nodes
    yp = _arg(Y, "Y", (4, n))
    if R is None:
        R = torch.empty_like(Y)
    rp = _arg(R, "R", (4, n), device=Y.device)
    pc, tc = _params(params)._c(), tm._c(mesh)
    _check(load().hb_tm_residual(mesh._h, C.byref(pc), C.byref(tc), yp, rp, _stream(stream)))
    return R


def tm_jvp(mesh: Mesh, params, tm: TmStep, Y, V, JV=None, stream=None):
    import torch
    n = mesh.n_nodes
    yp = _arg(Y, "Y", (4, n))
    vp_ = _arg(V, "V", (4, n), device=Y.device)
    if JV is None:
        JV = torch.empty_like(V)
    jp = _arg(JV, "JV", (4, n), device=Y.device)
    pc, tc = _params(params)._c(), tm._c(mesh)
    _check(load().hb_tm_jvp(mesh._h, C.byref(pc), C.byref(tc), yp, vp_, jp, _stream(stream)))
    return JV


@dataclass
class TmOptions:
    t0: float = 0.0
    dt: float = 0.01
    n_steps: int = 1
    rtol: float = 1e-10
    atol: float = 0.0
    gmres_eta: float = 1e-6
    restart: int = 50
    max_newton: int = 20
    max_gmres: int = 1000
    omega_hat: float = -1.0  # < 0: eq. tauhat from each step's starting state
    verbose: int = 0
    precond: int = HB_PREC_JACOBI

    def _c(self):
        return _TmOpts(self.t0, self.dt, self.n_steps, self.rtol, self.atol, self.gmres_eta,
                       self.restart, self.max_newton, self.max_gmres, self.omega_hat,
                       self.verbose, self.precond)


def tm_march(mesh: Mesh, params, bc: BC, Y, A, opts: TmOptions, traj=None, stream=None,
             raise_on_noconv: bool = True) -> dict:
    """March in place: Y (4, n) and A (3, n) hold the state and acceleration
    at opts.t0 on entry and after the last step on return; ``traj`` (a
    device tensor (n_steps, 4, n)) or None receives every step's state."""
    rep = _TmReport()
    p = _params(params)
    n = mesh.n_nodes
    yp = _arg(Y, "Y", (4, n))
    ap_ = _arg(A, "A", (3, n), device=Y.device)
    tp = None if traj is None else _arg(traj, "traj", (opts.n_steps, 4, n), device=Y.device)
    pc, bcc, oc = p._c(), bc._c(mesh, p.N), opts._c()
    st = load().hb_tm_march(mesh._h, C.byref(pc), C.byref(bcc), yp, ap_, tp, C.byref(oc),
                            C.byref(rep), _stream(stream))
    out = {k: getattr(rep, k) for k, _ in _TmReport._fields_}
    if st != HB_OK and not (st == HB_ERR_NOCONV and not raise_on_noconv):
        _check(st)
    return out


def jacobi(mesh: Mesh, params, bc: BC, Y, shift: float = 0.0, D=None, stream=None):
    import torch
    p = _params(params)
    yp = _arg(Y, "Y", _modal_shape(mesh, p))
    if D is None:
        D = torch.empty((2, p.N, mesh.n_nodes), dtype=torch.float64, device=Y.device)
    dp = _arg(D, "D", (2, p.N, mesh.n_nodes), device=Y.device)
    pc, bcc = p._c(), bc._c(mesh, p.N)
    _check(load().hb_jacobi(mesh._h, C.byref(pc), C.byref(bcc), yp, float(shift), dp,
                            _stream(stream)))
    return D


@dataclass
class SolveOptions:
    rtol: float = 1e-8
    r_ref: float = 0.0
    gmres_eta: float = 0.03
    cfl: float = 1.0
    c1: float = 1.5
    restart: int = 50
    max_newton: int = 50
    max_gmres: int = 1000
    precision: int = HB_F64
    jv_kind: int = HB_JV_EXACT
    verbose: int = 0
    precond: int = HB_PREC_NODE_TIME
    cfl_max: float = 0.0
    graphs: int = 0  # 1: replay captured Arnoldi steps (HIP graphs) at launch-bound sizes
    amg_sweeps: int = 0   # HB_PREC_MEANFLOW: Jacobi sweeps per level (0: 2)
    amg_cycles: int = 0   # HB_PREC_MEANFLOW: V-cycles per application (0: 1)
    amg_weight: float = 0.0  # HB_PREC_MEANFLOW: Jacobi damping (0: 0.7)
    reject_ratio: float = 0.0  # damp steps whose residual grows beyond this ratio (0: 100; <0: never)
    dt_growth: float = 0.0     # least pseudo-step growth after a non-increasing step (0: 1)
    amg_aggregation: int = 0   # HB_PREC_MEANFLOW: 0 pairwise matching twice, 1 node + neighbours
    amg_coarse_weight: float = 0.0  # HB_PREC_MEANFLOW: coarse-correction weight (0: 0.7)
    amg_smoother: int = 0      # HB_PREC_MEANFLOW: 0 block Jacobi, 1 block Gauss-Seidel
    amg_wcycle: int = 0        # HB_PREC_MEANFLOW: 0 V-cycles, 1 W-cycles
    amg_fp32: int = 0          # HB_PREC_MEANFLOW: 1 cycles on FP32 vectors and coefficients
    forcing: int = 0           # GMRES forcing: 0 fixed gmres_eta, 1 Eisenstat-Walker

    def _c(self):
        return _Opts(self.rtol, self.r_ref, self.gmres_eta, self.cfl, self.c1, self.restart,
                     self.max_newton, self.max_gmres, self.precision, self.jv_kind, self.verbose,
                     self.precond, self.cfl_max, self.graphs, self.amg_sweeps, self.amg_cycles,
                     self.amg_weight, self.reject_ratio, self.dt_growth, self.amg_aggregation,
                     self.amg_coarse_weight, self.amg_smoother, self.amg_wcycle, self.amg_fp32,
                     self.forcing)


def newton_solve(mesh: Mesh, params, bc: BC, Y, opts: SolveOptions | None = None,
                 stream=None, raise_on_noconv: bool = True) -> dict:
    """Solve in place (Y holds the guess on entry, the solution on return)."""
    opts = opts or SolveOptions()
    rep = _Report()
    p = _params(params)
    yp = _arg(Y, "Y", _modal_shape(mesh, p))
    pc, bcc, oc = p._c(), bc._c(mesh, p.N), opts._c()
    st = load().hb_newton_solve(mesh._h, C.byref(pc), C.byref(bcc), yp, C.byref(oc),
                                C.byref(rep), _stream(stream))
    out = {k: getattr(rep, k) for k, _ in _Report._fields_}
    if st != HB_OK and not (st == HB_ERR_NOCONV and not raise_on_noconv):
        _check(st)
    return out


def precond_apply(mesh: Mesh, params, bc: BC, Y, X, shift: float = 0.0, op: str = "inverse",
                  sweeps: int = 2, cycles: int = 1, weight: float = 0.7, coarse_max: int = 64,
                  aggregation: int = 0, coarse_weight: float = 0.7, smoother: int = 0,
                  wcycle: int = 0, fp32: int = 0, OUT=None, stream=None):
    """The mean-flow modal preconditioner at the state Y: ``op="operator"``
    applies its operator A, ``op="inverse"`` its multigrid approximation of
    A^-1 (modal (4, N, n) arrays; see hb_precond_apply)."""
    import torch
    p = _params(params)
    shp = _modal_shape(mesh, p)
    yp = _arg(Y, "Y", shp)
    xp = _arg(X, "X", shp, device=Y.device)
    if OUT is None:
        OUT = torch.empty_like(X)
    op_ = {"operator": 0, "inverse": 1}.get(op)
    if op_ is None:
        raise HBError(HB_ERR_ARG, f"unknown op {op!r}")
    outp = _arg(OUT, "OUT", shp, device=Y.device)
    o = _PcOpts(int(sweeps), int(cycles), float(weight), int(coarse_max), int(aggregation),
                float(coarse_weight), int(smoother), int(wcycle), int(fp32))
    pc, bcc = p._c(), bc._c(mesh, p.N)
    _check(load().hb_precond_apply(mesh._h, C.byref(pc), C.byref(bcc), yp, float(shift),
                                   C.byref(o), op_, xp, outp, _stream(stream)))
    return OUT


def precond_hierarchy(n_nodes: int, tets: np.ndarray, coarse_max: int = 24,
                      aggregation: int = 0):
    """The multigrid hierarchy of a mesh's node graph, built on the host
    (hb_precond_hierarchy): (level sizes, aggregate of each fine node,
    colour class of each fine node)."""
    t = np.ascontiguousarray(tets, np.int32)
    if t.ndim != 2 or t.shape[1] != 4:
        raise HBError(HB_ERR_ARG, "tets must be (n_tets, 4)")
    sizes = np.zeros(32, np.int64)
    nl = C.c_int32()
    agg = np.zeros(int(n_nodes), np.int32)
    col = np.zeros(int(n_nodes), np.int32)
    _check(load().hb_precond_hierarchy(int(n_nodes), t.shape[0], t.ctypes.data, int(coarse_max),
                                       int(aggregation), 32, sizes.ctypes.data, C.byref(nl),
                                       agg.ctypes.data, col.ctypes.data))
    return [int(x) for x in sizes[:min(nl.value, 32)]], agg, col


def precond_levels(mesh: Mesh) -> list:
    """Node counts of the preconditioner hierarchy's levels (empty before use)."""
    sizes = np.zeros(32, np.int64)
    nl = C.c_int32()
    _check(load().hb_precond_levels(mesh._h, sizes.ctypes.data, 32, C.byref(nl)))
    return [int(x) for x in sizes[:nl.value]]


def outlet_flow(mesh: Mesh, params, bc: BC, Y, stream=None):
    """Outlet flow rates Q (n_outlets, N) at the sample times and the mass
    balance defect (N,) = net boundary outflow per sample (the continuity
    rows summed over all nodes); see hb_outlet_flow."""
    p = _params(params)
    yp = _arg(Y, "Y", _modal_shape(mesh, p))
    Q = np.zeros((mesh.n_outlets, p.N))
    d = np.zeros(p.N)
    pc, bcc = p._c(), bc._c(mesh, p.N)
    _check(load().hb_outlet_flow(mesh._h, C.byref(pc), C.byref(bcc), yp, Q.ctypes.data,
                                 d.ctypes.data, _stream(stream)))
    return Q, d
