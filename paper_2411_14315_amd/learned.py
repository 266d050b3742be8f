"""Learned Newton warm start: a POD of harmonic-balance solutions that the
solver itself generates, and a small MLP (BF16 weights, FP32 accumulation;
forward, backward and Adam are the library's own HIP kernels) mapping the
problem parameters to POD coefficients.  The predicted state is used as the
initial guess only if its FP64 residual is below that of the plain steady
start; otherwise the plain start is kept, and the final FP64 residual decides
convergence either way.

Only argument marshalling and small host-side statistics (standardisation
of the parameters and coefficients) happen here: the POD (hb_pod_fit: mean,
Gram matrix and modes on the device, the small eigenproblem in the library's
host code), every network step and the expansion of the guess run in the
library.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, replace

import numpy as np

from . import (BC, HB_F64, HB_PREC_MEANFLOW, Mesh, SolveOptions, _arg, _check, _stream, load,
               newton_solve, residual)


class MLP:
    """hb_mlp handle; widths = [in, hidden..., out]."""

    def __init__(self, widths, params: np.ndarray | None = None, seed: int = 0):
        lib = load()
        self.widths = [int(w) for w in widths]
        w = np.asarray(self.widths, np.int32)
        p = None if params is None else np.ascontiguousarray(params, np.float32)
        h = C.c_void_p()
        _check(lib.hb_mlp_create(len(w) - 1, w.ctypes.data,
                                 None if p is None else p.ctypes.data, C.c_uint64(seed),
                                 C.byref(h)))
        self._h = h
        n = C.c_int64()
        _check(lib.hb_mlp_num_params(h, C.byref(n)))
        self.n_params = int(n.value)

    def params(self) -> np.ndarray:
        """The BF16 weights the kernels use, widened to FP32."""
        out = np.zeros(self.n_params, np.float32)
        _check(load().hb_mlp_get_params(self._h, out.ctypes.data))
        return out

    def forward(self, X, Y=None, stream=None):
        import torch
        B = int(X.shape[0])
        xp = _arg(X, "X", (B, self.widths[0]), ("float32",))
        if Y is None:
            Y = torch.empty((B, self.widths[-1]), dtype=torch.float32, device=X.device)
        yp = _arg(Y, "Y", (B, self.widths[-1]), ("float32",), device=X.device)
        _check(load().hb_mlp_forward(self._h, xp, B, yp, _stream(stream)))
        return Y

    def forward_noalloc(self, X, Y, stream=None):
        """The same forward pass with the hidden activations in the library's
        fixed device array (no allocation; Y must be given)."""
        B = int(X.shape[0])
        xp = _arg(X, "X", (B, self.widths[0]), ("float32",))
        yp = _arg(Y, "Y", (B, self.widths[-1]), ("float32",), device=X.device)
        _check(load().hb_mlp_forward_noalloc(self._h, xp, B, yp, _stream(stream)))
        return Y

    def loss_grad(self, X, T, grad=None, want_loss=True, stream=None):
        """Forward + backward of the mean squared error; the gradient goes to
        ``grad`` (FP32 device tensor of n_params) or the handle's own buffer."""
        loss = C.c_double()
        B = int(X.shape[0])
        xp = _arg(X, "X", (B, self.widths[0]), ("float32",))
        tp = _arg(T, "T", (B, self.widths[-1]), ("float32",), device=X.device)
        gp = None if grad is None else _arg(grad, "grad", (self.n_params,), ("float32",),
                                            device=X.device)
        _check(load().hb_mlp_loss_grad(self._h, xp, tp, B, gp,
                                       C.byref(loss) if want_loss else None, _stream(stream)))
        return float(loss.value) if want_loss else None

    def adam_step(self, lr: float, grad=None, stream=None):
        gp = None if grad is None else _arg(grad, "grad", (self.n_params,), ("float32",))
        _check(load().hb_mlp_adam_step(self._h, gp, C.c_float(lr), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hb_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pod_expand(mean, basis, coef, Y, base=None, stream=None):
    """Y = base + mean + basis^T coef on the device (basis rows are POD
    modes; base optional and may be Y itself)."""
    r = 0 if basis is None else int(basis.shape[0])
    L = int(mean.numel())
    mp = _arg(mean, "mean", tuple(mean.shape))
    yp = _arg(Y, "Y", tuple(Y.shape), device=mean.device)
    if int(Y.numel()) != L:
        raise ValueError(f"Y has {Y.numel()} values, mean {L}")
    bp = None
    if base is not None:
        bp = _arg(base, "base", tuple(base.shape), device=mean.device)
        if int(base.numel()) != L:
            raise ValueError(f"base has {base.numel()} values, mean {L}")
    Bp = cp = None
    if r:
        Bp = _arg(basis, "basis", (r, L), device=mean.device)
        cp = _arg(coef, "coef", (r,), ("float32",), device=mean.device)
    _check(load().hb_pod_expand(L, r, bp, mp, Bp, cp, yp, _stream(stream)))
    return Y


def pod_fit(S, rank: int, base=None, floor_rel: float = 1e-14, stream=None):
    """POD of the rows of S (minus the rows of base): returns (mean (L,),
    basis (r, L) orthonormal rows, coef (ns, r) host, lam (ns,) host, r)
    with r <= rank modes (see hb_pod_fit)."""
    import torch
    ns, L = int(S.shape[0]), int(S.shape[1])
    sp = _arg(S, "S", (ns, L))
    bp = None if base is None else _arg(base, "base", (ns, L), device=S.device)
    mean = torch.empty(L, dtype=torch.float64, device=S.device)
    basis = torch.empty((int(rank), L), dtype=torch.float64, device=S.device)
    coef = np.zeros((ns, int(rank)))
    lam = np.zeros(ns)
    r = C.c_int32()
    _check(load().hb_pod_fit(sp, bp, ns, L, int(rank), float(floor_rel), mean.data_ptr(),
                             basis.data_ptr(), coef.ctypes.data, lam.ctypes.data, C.byref(r),
                             _stream(stream)))
    r = int(r.value)
    return mean, basis[:r], np.ascontiguousarray(coef[:, :r]), lam, r


def sym_eig(A: np.ndarray):
    """Host symmetric eigenproblem (hb_sym_eig): w descending, V columns."""
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    w, V = np.zeros(n), np.zeros((n, n))
    _check(load().hb_sym_eig(n, A.ctypes.data, w.ctypes.data, V.ctypes.data))
    return w, V


def sample_norm(R, K: int) -> float:
    """2-norm over time samples of modal rows (Parseval for the real DFT),
    on a host copy."""
    N = 2 * K + 1
    R = R.cpu().numpy()
    R = R.reshape(-1, N, R.shape[-1]) if R.ndim == 3 else R
    return float(N * ((R[:, 0] ** 2).sum() + 0.5 * (R[:, 1:] ** 2).sum())) ** 0.5


@dataclass
class Case:
    """One problem on the device."""
    problem: object
    mesh: Mesh
    bc: BC
    bc0: BC

    @classmethod
    def build(cls, problem, device="cuda:0"):
        import torch
        d = torch.from_numpy(np.ascontiguousarray(problem.dirichlet)).to(device)
        h = problem.outlet_h
        return cls(problem, Mesh.from_mesh(problem.mesh), BC(d, h, problem.outlet_R),
                   BC(d[:, :1].contiguous(), None if h is None else h[:, :1], problem.outlet_R))

    @property
    def params(self):
        return self.problem.params

    def plain_start(self, rtol=1e-10):
        """The steady (K = 0) solution broadcast to every sample: the mean
        mode holds it and the harmonics are zero."""
        import torch
        n = self.mesh.n_nodes
        dev = self.bc.dirichlet.device
        Ys = torch.zeros((4, 1, n), dtype=torch.float64, device=dev)
        newton_solve(self.mesh, replace(self.params, K=0), self.bc0, Ys,
                     SolveOptions(rtol=rtol, max_newton=100, max_gmres=500,
                                  precond=HB_PREC_MEANFLOW, amg_cycles=2),
                     raise_on_noconv=False)
        Y = torch.zeros((4, self.params.N, n), dtype=torch.float64, device=dev)
        Y[:, 0] = Ys[:, 0]
        return Y

    def residual_norm(self, Y) -> float:
        return sample_norm(residual(self.mesh, self.params, self.bc, Y), self.params.K)

    def solve(self, Y, r_ref: float, rtol=1e-8, max_newton=300, precision=HB_F64, cfl=1.0,
              verbose=0):
        import torch
        torch.cuda.synchronize()
        t = time.perf_counter()
        rep = newton_solve(self.mesh, self.params, self.bc, Y,
                           SolveOptions(rtol=rtol, r_ref=r_ref, max_newton=max_newton,
                                        max_gmres=500, precision=precision, cfl=cfl,
                                        precond=HB_PREC_MEANFLOW, amg_cycles=2,
                                        amg_fp32=int(precision != HB_F64), verbose=verbose),
                           raise_on_noconv=False)
        torch.cuda.synchronize()
        rep["wall_s"] = time.perf_counter() - t
        return rep


def generate_snapshots(problems, batch: int = 1, rtol=1e-9, device="cuda:0", precision=HB_F64,
                       log=None, max_newton=400, verbose=0):
    """Solve every problem (same topology) with the method itself, from the
    plain start, to the FP64 residual rtol ||r(plain start)||; `batch`
    problems at a time as one disjoint-union mesh (worth it only for meshes
    too small to fill the GPU: GMRES on the union converges as on its
    hardest member, or slower).  `precision` is the Krylov precision
    (HB_MIXED: FP32 Jv, basis and multigrid cycles).  Returns the
    (n_kept, 4 N n) FP64 device matrices of the solutions and of the plain
    starts, and statistics; with batch = 1 a draw whose solve does not
    converge within max_newton steps is left out (its index is not in
    stats["kept"]).  verbose = 1 prints every Newton step (stderr)."""
    import torch
    from hbinputs.problems import stack
    sols, starts = [], []
    stats = dict(solves=0, newton=0, gmres=0, unconverged=0, kept=[])
    t0 = time.perf_counter()

    def rows(Y, g, n):
        return Y.view(4, -1, g, n).permute(2, 0, 1, 3).reshape(g, -1)

    for i in range(0, len(problems), batch):
        group = problems[i:i + batch]
        c = Case.build(group[0] if len(group) == 1 else stack(group), device)
        Y = c.plain_start()
        n = group[0].mesh.n_nodes
        Ys = rows(Y, len(group), n).clone()
        rep = c.solve(Y, r_ref=0.0, rtol=rtol, max_newton=max_newton, precision=precision,
                      verbose=verbose)
        stats["solves"] += 1
        stats["newton"] += rep["newton_iters"]
        stats["gmres"] += rep["gmres_iters"]
        stats["unconverged"] += int(rep["status"] != 0)
        if rep["status"] == 0 or len(group) > 1:
            starts.append(Ys)
            sols.append(rows(Y, len(group), n))
            stats["kept"].extend(range(i, i + len(group)))
        c.mesh.close()
        if log is not None:
            log(f"snapshots {i + len(group)}/{len(problems)}: newton {rep['newton_iters']} "
                f"gmres {rep['gmres_iters']} status {rep['status']} "
                f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    stats["wall_s"] = time.perf_counter() - t0
    return torch.cat(sols).contiguous(), torch.cat(starts).contiguous(), stats


class WarmStart:
    """POD + MLP initial-guess model.

    target "correction": the model predicts the solution minus the plain
    steady start, and the guess is that start plus the prediction (the
    steady solve is still needed; the model supplies the harmonics and the
    nonlinear correction of the mean).  target "solution": the model predicts
    the whole state, and no steady solve is needed for the guess."""

    def __init__(self, rank: int = 64, hidden=(256, 256), seed: int = 0,
                 target: str = "correction"):
        if target not in ("correction", "solution"):
            raise ValueError("target is 'correction' or 'solution'")
        self.rank = rank
        self.hidden = tuple(hidden)
        self.seed = seed
        self.target = target

    def fit(self, thetas: np.ndarray, Y, Y0=None, steps: int = 3000, lr: float = 1e-3):
        """thetas (n, p) on the host; Y (n, L) FP64 device solutions; Y0 the
        plain starts (required for the correction target)."""
        import torch
        t = time.perf_counter()
        if self.target == "correction" and Y0 is None:
            raise ValueError("the correction target needs the plain starts")
        base = Y0 if self.target == "correction" else None
        self.mean, self.basis, coef, lam, _ = pod_fit(Y, self.rank, base=base)
        self.energy = float(lam[:self.basis.shape[0]].sum() / max(lam[lam > 0].sum(), 1e-300))
        self.r = int(self.basis.shape[0])
        self.x_mu, self.x_sd = thetas.mean(0), thetas.std(0) + 1e-12
        # one scale for every coefficient, so that the loss measures the
        # error of the expanded state (the trailing modes carry little energy)
        self.c_mu = coef.mean(0)
        self.c_sd = np.full(self.r, coef.std(0).max() + 1e-300)
        Xn = torch.from_numpy(((thetas - self.x_mu) / self.x_sd).astype(np.float32)).to(Y.device)
        Cn = torch.from_numpy(((coef - self.c_mu) / self.c_sd).astype(np.float32)).to(Y.device)
        self.net = MLP([thetas.shape[1], *self.hidden, self.r], seed=self.seed)
        self.losses = []
        for it in range(steps):
            want = it % 250 == 0 or it == steps - 1
            loss = self.net.loss_grad(Xn, Cn, want_loss=want)
            if want:
                self.losses.append(loss)
            self.net.adam_step(lr * 0.5 * (1.0 + np.cos(np.pi * it / steps)))
        torch.cuda.synchronize()
        self.fit_s = time.perf_counter() - t
        return self

    def guess(self, theta: np.ndarray, shape, plain=None):
        """Modal state (4, N, n): [plain +] mean + Phi c(theta)."""
        import torch
        if self.target == "correction" and plain is None:
            raise ValueError("the correction target needs the plain start")
        x = ((np.atleast_2d(theta) - self.x_mu) / self.x_sd).astype(np.float32)
        c = self.net.forward(torch.from_numpy(x).to(self.mean.device)).cpu().numpy()[0]
        cd = torch.from_numpy((c * self.c_sd + self.c_mu).astype(np.float32)).to(self.mean.device)
        Y = torch.empty(shape, dtype=torch.float64, device=self.mean.device)
        base = plain.reshape(-1) if self.target == "correction" else None
        pod_expand(self.mean, self.basis, cd, Y.view(-1), base=base)
        return Y


def compare_starts(model: WarmStart, case: Case, theta, rtol=1e-8, learned_max_newton=60,
                   precision=HB_F64, verbose=0):
    """Plain start vs learned guess, both to the same absolute FP64 residual
    rtol * ||r(plain start)|| with the given Krylov precision.  If Newton from
    the guess does not converge within learned_max_newton steps (or breaks
    down), the plain start is solved instead and both attempts are charged
    to the learned path."""
    import torch
    from . import HBError
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Yp = case.plain_start()
    r_plain = case.residual_norm(Yp)
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    Yg = model.guess(theta, Yp.shape, plain=Yp)
    r_guess = case.residual_norm(Yg)
    t_guess = time.perf_counter() - t0
    if model.target == "correction":
        t_guess += t_plain           # the guess is built on the steady start
    Yl = Yg.clone()
    t0 = time.perf_counter()
    try:
        rep_l = case.solve(Yl, r_plain, rtol, max_newton=learned_max_newton,
                           precision=precision, verbose=verbose)
    except HBError as e:         # non-finite residual on the way
        torch.cuda.synchronize()
        rep_l = dict(status=e.status, newton_iters=learned_max_newton, gmres_iters=0,
                     wall_s=time.perf_counter() - t0)
    used = "learned"
    if rep_l["status"] != 0:
        Yl = Yp.clone()
        rep_f = case.solve(Yl, r_plain, rtol, precision=precision, verbose=verbose)
        rep_l = dict(rep_f, newton_iters=rep_l["newton_iters"] + rep_f["newton_iters"],
                     gmres_iters=rep_l["gmres_iters"] + rep_f["gmres_iters"],
                     wall_s=rep_l["wall_s"] + rep_f["wall_s"])
        used = "plain"
    Y0 = Yp.clone()
    rep_p = case.solve(Yp, r_plain, rtol, precision=precision, verbose=verbose)
    root = Yp.cpu().numpy()
    nrm = np.linalg.norm(root)

    def err(Y):
        return float(np.linalg.norm(Y.cpu().numpy() - root) / nrm)

    return {"plain": dict(rep_p, start_s=t_plain, r_start=r_plain, start_err=err(Y0)),
            "learned": dict(rep_l, start_s=t_guess, r_start=r_guess, start_err=err(Yg),
                            used=used),
            "solution_rel_diff": err(Yl)}
