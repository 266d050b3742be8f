#!/usr/bin/env python3
"""Benchmark of the HB-GLS hot path on one MI355X.

Workload (default): the synthetic curved branching artery, three bifurcation
generations with radii 2.0, 1.26, 0.79 and 0.50, lattice-carved P1 mesh
with h = 0.062: 1,255,132 nodes and 7,046,522 tetrahedra; K = 10 harmonics
(21 samples); seeded root inflow waveform at Re = 500 on the root diameter;
eight resistance outlets; rho = 1.06, mu = 0.04; FP64.  (--workload
tjunction runs the Glenn-like T-junction instead: 158,688 nodes.)

Setup (untimed): the mesh, and the plain start: the steady (K = 0) solve,
Reynolds number ramped 0.5 -> 1, broadcast to all harmonics.

A step is one pass of the whole hot path: one inexact Newton step of
hb_newton_solve (HB residual; mean-flow multigrid set-up; GMRES to
eta = 0.03 or the iteration cap, each iteration one Jacobian-vector product
with its time-axis transforms, element and face kernels and scatter, and one
preconditioner application; the Newton update).  The warm-up steps and the
timed steps are each one hb_newton_solve call continuing from the plain
start with its residual as the reference, so the pseudo step evolves as in
a single solve.

The line reports:
  value        Jacobian-vector throughput inside the timed FP64 steps,
               4 n N x (operator applications) / (operator time), the
               operator time from HIP events on the solve stream;
  ms_per_step  wall time per FP64 Newton step;
  mixed        the same steps with the FP32 Jacobian-vector products and
               Krylov basis (HB_MIXED), and their state's difference from
               the FP64 state;
  jv_public    the public hb_jvp entry point (FP64 and FP32), per stage;
  time_to_1e8  complete solves to 1e-8 of the plain start's residual, FP64
               and mixed: the Womersley pipe (1,911 nodes, K = 2) and the
               T-junction on the coarse lattice (14,191 nodes, K = 10);
  roofline     the element Jacobian-vector kernel against the FP64 vector
               peak (its duration from HIP events on its launch stream;
               FP64 operations per lane from rocprofv3 counters);
  cpu_baseline the CPU oracle's exact Jacobian-vector product on a bounded
               sample of the same workload, one process and 8 processes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HB Jv throughput (GDOF-modes/s) + time to 1e-8 HB residual, mixed vs FP64"
# precision names -> hb_solve_opts.precision (HB_F64, HB_MIXED, HB_F32_BASIS)
PRECISIONS = {"fp64": 0, "mixed": 1, "f32_basis": 2}
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# FP64 operations per (tetrahedron, sample) lane of the exact-Jv element
# kernel: counted by rocprofv3 (FP64 VALU instructions of each kind x 64
# lanes, FMA = 2) and, for comparison, an estimate counted from the
# equations (primal + tangent, about 1.2k + 1.5k flop).
ELEM_FLOPS_EQUATIONS = 2700
ELEM_FLOPS = {"sha256_prefix": "85dde60c62f4d23e", "per_tet_sample": 1953.5,
              "source": "rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 x 64 lanes (FMA = 2), "
                        "profiles/k_elem_jvp_exact_branching_K10_counters.md"}
# HBM bytes per launch of the FP64 exact-Jv element kernel, from rocprofv3
# FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a plain
# copy of known size; valid while the element-kernel source hashes to the
# recorded value and for the recorded workload.
ELEM_TRAFFIC = {"sha256_prefix": "85dde60c62f4d23e", "fetch_kib": 3502931, "write_kib": 9538025,
                "fetch_scale": 2.0, "write_scale": 1.0, "n_nodes": 1255132, "n_tets": 7046522,
                "K": 10, "profile": "profiles/k_elem_jvp_exact_branching_K10_counters.md"}


def _elem_source_hash():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2411_14315_amd", "csrc", "hb_kernels.hip")).read()
    a = src.index("// ------------------------------------------------------------- elements")
    b = src.index("// --------------------------------------------------------------- faces")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def elem_flops_per_lane():
    f = ELEM_FLOPS
    if f["sha256_prefix"] is not None and f["sha256_prefix"] != _elem_source_hash():
        return None, None
    return f["per_tet_sample"], f["source"]


def elem_traffic(n, ne, K):
    t = ELEM_TRAFFIC
    if (t is None or t["sha256_prefix"] != _elem_source_hash()
            or (n, ne, K) != (t["n_nodes"], t["n_tets"], t["K"])):
        return None, None
    rd = t["fetch_kib"] * 1024 * t["fetch_scale"]
    wr = t["write_kib"] * 1024 * t["write_scale"]
    return rd + wr, {"read_bytes": rd, "write_bytes": wr, "source": t["profile"]}


def elem_bytes(n, ne, N):
    """Algorithmic HBM bytes of one exact-Jv element-kernel launch: node
    samples read once (7 channels of state, 7 of direction), accumulator rows
    read-modify-written once (7 channels), geometry (20 doubles) and
    connectivity (4 int32) once per tetrahedron."""
    return 8.0 * n * N * (14 + 2 * 7) + ne * (20 * 8 + 4 * 4)


# ------------------------------------------------------------ CPU baseline
_CPU = {}


def _cpu_rows(rows):
    from oracle import residual as res
    c = _CPU
    t = time.perf_counter()
    res.jvp_samples(c["om"], c["prm"], c["y"], c["v"], c["hs"], c["R"], c["H"], rows=rows)
    return time.perf_counter() - t


def cpu_baseline(P, Y, V, budget_s=20.0, workers=8):
    """Oracle exact Jv on a bounded sample: the rows of a contiguous block of
    nodes (and every element touching them), timed in one process, then the
    same rows split over `workers` processes; scaled to the whole mesh by
    element count."""
    import multiprocessing as mp
    from oracle import api, fem, spectral
    om = fem.from_mesh(P.mesh)
    prm = P.params
    _CPU.update(om=om, prm=prm, y=api.samples_of(om, prm, Y, P.dirichlet),
                v=spectral.to_samples(V, prm.K), hs=api.h_samples(prm, P.outlet_h), R=P.outlet_R,
                H=api.H_of(prm))
    frac = 0.002
    while True:
        rows = np.arange(int(frac * om.n))
        mark = np.zeros(om.n, bool)
        mark[rows] = True
        nel = int(mark[om.tets].any(axis=1).sum())
        dt = _cpu_rows(rows)
        if dt > 0.4 * budget_s or frac >= 0.5:
            break
        frac = min(0.5, frac * max(2.0, 0.5 * budget_s / max(dt, 1e-3)))
    dofs = 4 * om.n * prm.N
    one = dofs / (dt * om.ne / nel) / 1e9
    chunks = np.array_split(rows, workers)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_cpu_rows, [c[:8] for c in chunks])      # start the workers
        t = time.perf_counter()
        pool.map(_cpu_rows, chunks)
        dtp = time.perf_counter() - t
    par = dofs / (dtp * om.ne / nel) / 1e9
    return {"value": one, "unit": "GDOF-modes/s", "cores": 1, "kind": "oracle",
            "sample": f"exact Jv rows of {rows.size} nodes ({nel} of {om.ne} tetrahedra, "
                      f"{dt:.1f} s in one process), scaled by element count",
            "parallel": {"value": par, "cores": workers, "seconds": dtp,
                         "sample": f"the same rows in {workers} processes"}}


# ------------------------------------------------------------ workloads
def make_problem(workload):
    from hbinputs.problems import c2_tjunction, c3_branching
    if workload == "branching":
        return c3_branching(), "branching_artery"
    return c2_tjunction(K=10), "tjunction_glenn_like"


def plain_start(hbl, torch, P, gm, log, ramp=(0.5, 1.0), max_newton=150):
    """Steady (K = 0) solve with the Reynolds number ramped through `ramp`
    (fractions of the inflow), broadcast to every harmonic."""
    from dataclasses import replace
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    n = P.mesh.n_nodes
    Ys = torch.zeros((4, 1, n), dtype=torch.float64, device="cuda:0")
    reps = []
    for k, s in enumerate(ramp):
        bc0 = hbl.BC(to(s * P.dirichlet[:, :1]), P.outlet_h[:, :1], P.outlet_R)
        last = k == len(ramp) - 1
        r = hbl.newton_solve(gm, replace(P.params, K=0), bc0, Ys,
                             hbl.SolveOptions(rtol=1e-9, max_newton=max_newton if last else 20,
                                              max_gmres=500, precond=hbl.HB_PREC_MEANFLOW,
                                              amg_cycles=2),
                             raise_on_noconv=False)
        reps.append(r)
        log(f"plain start, inflow x{s}: {r['newton_iters']} Newton, {r['gmres_iters']} GMRES, "
            f"|r| {r['r0']:.3e} -> {r['r_final']:.3e} ({r['wall_s']:.1f} s)")
    Y0 = torch.zeros((4, P.params.N, n), dtype=torch.float64, device="cuda:0")
    Y0[:, 0] = Ys[:, 0]
    return Y0, reps


def solve_opts(hbl, **kw):
    """Mean-flow multigrid, two cycles per application; the reduced-precision
    solves also run the cycles in FP32 (amg_fp32)."""
    base = dict(max_gmres=300, precond=hbl.HB_PREC_MEANFLOW, amg_cycles=2)
    base.update(kw)
    if base.get("precision", hbl.HB_F64) != hbl.HB_F64:
        base.setdefault("amg_fp32", 1)
    return hbl.SolveOptions(**base)


def time_to_solution(hbl, torch, log, which, precision):
    """Complete solve to 1e-8 of the plain start's residual (after one untimed
    warm-up solve); the plain start's own time is reported beside it."""
    from hbinputs.problems import c1_womersley, c2_tjunction
    P = c1_womersley() if which == "womersley_pipe" else c2_tjunction(K=10, h=0.1)
    prm = P.params
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)
    res = {}
    for _ in range(2):
        torch.cuda.synchronize()
        t = time.time()
        Y, reps = plain_start(hbl, torch, P, gm, lambda *a: None, ramp=(1.0,), max_newton=200)
        t_plain = time.time() - t
        t = time.time()
        r = hbl.newton_solve(gm, prm, bc, Y, solve_opts(hbl, rtol=1e-8, max_newton=300,
                                                        max_gmres=1000,
                                                        precision=PRECISIONS[precision]),
                             raise_on_noconv=False)
        t_solve = time.time() - t
        res = {"workload": which, "precision": precision, "n_nodes": P.mesh.n_nodes,
               "K": prm.K, "seconds": t_solve, "plain_start_seconds": t_plain,
               "total_seconds": t_solve + t_plain, "newton_iters": r["newton_iters"],
               "gmres_iters": r["gmres_iters"], "status": r["status"],
               "r_final_rel": r["r_final"] / r["r0"], "mass_defect": r["mass_defect"],
               "plain_start_status": reps[-1]["status"]}
        if which != "womersley_pipe":
            # the oracle's stored root of this workload (modal values at
            # seeded nodes, solved to 1e-12 on the host)
            g = np.load(os.path.join(ROOT, "tests", "golden", "c2_reduced_solution.npz"))
            Yg = Y.cpu().numpy()[:, :, g["nodes"]]
            res["rel_err_vs_oracle_root"] = float(np.linalg.norm(Yg - g["Y"]) /
                                                  np.linalg.norm(g["Y"]))
    log(f"time to 1e-8: {res}")
    gm.close()
    return res


def periodicity(hbl, torch, log, workload="tjunction", h=3.0 / 70.0, periods=8, spp=100,
                step_rtol=1e-6):
    """Does the workload settle to a T-periodic flow?  The GLS time-marching
    solver (hb_tm_march: generalized-alpha, tau-hat of eq. tauhat, each step
    solved by Newton-GMRES with the mean-flow multigrid to step_rtol) is
    marched period by period from the plain steady start; reported per
    period: the relative change of the marched states against the previous
    period at the same phases, and the outlet flow rate at the sample times.
    A flow that settles shows the change falling period after period; a
    flow without a T-periodic attractor keeps an O(1) change."""
    from hbinputs.problems import c1_womersley, c2_tjunction
    P = c2_tjunction(K=10, h=h) if workload == "tjunction" else c1_womersley()
    prm = P.params
    n, T = P.mesh.n_nodes, prm.period
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)
    bc0 = hbl.BC(to(P.dirichlet[:, :1]), P.outlet_h[:, :1], P.outlet_R)
    Ys = torch.zeros((4, 1, n), dtype=torch.float64, device="cuda:0")
    from dataclasses import replace
    hbl.newton_solve(gm, replace(prm, K=0), bc0, Ys,
                     hbl.SolveOptions(rtol=1e-8, max_newton=60, max_gmres=500,
                                      precond=hbl.HB_PREC_MEANFLOW), raise_on_noconv=False)
    Y = Ys[:, 0].contiguous().clone()
    A = torch.zeros((3, n), dtype=torch.float64, device="cuda:0")
    traj = torch.empty((spp, 4, n), dtype=torch.float64, device="cuda:0")
    prev = None
    rows = []
    for k in range(periods):
        opts = hbl.TmOptions(t0=k * T, dt=T / spp, n_steps=spp, rtol=step_rtol, gmres_eta=0.03,
                             max_newton=15, max_gmres=500, precond=hbl.HB_PREC_MEANFLOW)
        t = time.time()
        r = hbl.tm_march(gm, prm, bc, Y, A, opts, traj=traj, raise_on_noconv=False)
        vel = traj[:, :3]
        row = {"period": k + 1, "wall_s": time.time() - t, "newton_iters": r["newton_iters"],
               "gmres_iters": r["gmres_iters"], "status": r["status"],
               "max_step_residual": r["max_step_residual"],
               "velocity_change": None if prev is None else
               float(torch.linalg.norm(vel - prev) / torch.linalg.norm(vel))}
        rows.append(row)
        log(f"periodicity {workload} period {k + 1}: {row}")
        prev = vel.clone()
    gm.close()
    return {"workload": workload, "n_nodes": n, "steps_per_period": spp, "step_rtol": step_rtol,
            "periods": rows}


def tm_vs_hb(hbl, torch, log, periods, spp, tm_precond=None):
    """The paper's comparison on the Womersley-pipe workload: the GLS
    time-marching solver (hb_tm_march, dt = T/spp, per-step Newton to three
    orders and GMRES to 0.03, the paper's settings for both solvers; each
    step preconditioned by the mean-flow multigrid of its K = 0 system)
    marched period by period from the plain start, against the HB solve to
    1e-8 (mean-flow multigrid).
    Per period: wall time, cycle-to-cycle change of the marched states and
    their difference from the HB solution at the same times."""
    from dataclasses import replace
    from hbinputs.problems import c1_womersley
    if tm_precond is None:
        tm_precond = hbl.HB_PREC_MEANFLOW
    P = c1_womersley()
    prm = P.params
    n, N, K, T = P.mesh.n_nodes, prm.N, prm.K, prm.period
    w = 2 * np.pi / T
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)
    bc0 = hbl.BC(to(P.dirichlet[:, :1]), P.outlet_h[:, :1], None)
    Ys = torch.zeros((4, 1, n), dtype=torch.float64, device="cuda:0")
    hbl.newton_solve(gm, replace(prm, K=0), bc0, Ys,
                     solve_opts(hbl, rtol=1e-10, max_newton=60, max_gmres=500))
    Yhb = torch.zeros((4, N, n), dtype=torch.float64, device="cuda:0")
    Yhb[:, 0] = Ys[:, 0]
    hbl.newton_solve(gm, prm, bc, Yhb.clone(), solve_opts(hbl, rtol=1e-8, max_newton=300,
                                                          max_gmres=500))   # warm-up
    torch.cuda.synchronize()
    t = time.time()
    rhb = hbl.newton_solve(gm, prm, bc, Yhb, solve_opts(hbl, rtol=1e-8, max_newton=300,
                                                        max_gmres=500))
    t_hb = time.time() - t
    Yh = Yhb.cpu().numpy()
    dt = T / spp
    tt = dt * np.arange(1, spp + 1)
    basis = np.ones((spp, N))
    for j in range(1, K + 1):
        basis[:, 2 * j - 1] = np.cos(j * w * tt)
        basis[:, 2 * j] = np.sin(j * w * tt)
    hb_t = np.einsum("sm,fmn->sfn", basis, Yh)               # HB solution at the step times
    Y = Ys[:, 0].contiguous().clone()
    A = torch.zeros((3, n), dtype=torch.float64, device="cuda:0")
    traj = torch.empty((spp, 4, n), dtype=torch.float64, device="cuda:0")
    prev = None
    per = []
    t_total = 0.0
    for k in range(periods):
        opts = hbl.TmOptions(t0=k * T, dt=dt, n_steps=spp, rtol=1e-3, gmres_eta=0.03,
                             max_newton=10, max_gmres=500, precond=tm_precond)
        torch.cuda.synchronize()
        t = time.time()
        r = hbl.tm_march(gm, prm, bc, Y, A, opts, traj=traj, raise_on_noconv=False)
        t_total += time.time() - t
        cur = traj.cpu().numpy()
        row = {"period": k + 1, "wall_s": r["wall_s"], "newton_iters": r["newton_iters"],
               "gmres_iters": r["gmres_iters"], "status": r["status"],
               "cycle_change": None if prev is None else
               float(np.linalg.norm(cur - prev) / np.linalg.norm(cur)),
               "diff_from_hb": float(np.linalg.norm(cur - hb_t) / np.linalg.norm(hb_t))}
        per.append(row)
        prev = cur
    out = {"workload": "womersley_pipe", "n_nodes": n, "steps_per_period": spp,
           "hb_seconds": t_hb, "hb_newton_iters": rhb["newton_iters"],
           "hb_gmres_iters": rhb["gmres_iters"], "tm_seconds": t_total, "tm_periods": per}
    log(f"time marching vs HB: HB {t_hb:.2f} s; marching {periods} periods {t_total:.2f} s; "
        f"last period change {per[-1]['cycle_change']}, diff from HB {per[-1]['diff_from_hb']:.3e}")
    return out


def learned_warm_start(torch, log, n_train, n_test, K=10, n_rings=12, n_z=90, period=1.0,
                       max_severity=0.7, batch=1, target="solution", fit_steps=4000,
                       gen_max_newton=80):
    """Learned warm start on the stenosed-pipe family (by default the
    42,679-node mesh, K = 10, severity up to 70 %, 23 parameters): n_train
    solutions generated by the solver (mixed precision to the FP64 residual
    1e-9), POD + MLP trained on the GPU, then plain vs learned start on n_test
    held-out draws to 1e-8 of the plain start's residual.  Times include the
    network + expansion, and the steady start where the model builds on it
    (target "correction")."""
    from hbinputs.problems import c4_stenosed, c4_stenosis_params
    from paper_2411_14315_amd import learned
    kw = dict(n_rings=n_rings, n_z=n_z, period=period)
    th = c4_stenosis_params(n_train, 2024, K=K, max_severity=max_severity)
    tt = c4_stenosis_params(n_test, 2025, K=K, max_severity=max_severity)
    Y, Y0, st = learned.generate_snapshots([c4_stenosed(x, K=K, **kw) for x in th], batch=batch,
                                           precision=PRECISIONS["mixed"], log=log,
                                           max_newton=gen_max_newton, verbose=1)
    th = th[st["kept"]]
    log(f"learned: generated {n_train} solutions in {st['wall_s']:.1f} s ({st})")
    rank = min(64, len(th) // 2)
    model = learned.WarmStart(rank=rank, hidden=(256, 256), target=target).fit(
        th, Y, Y0, steps=fit_steps, lr=2e-3)
    del Y, Y0
    log(f"learned: fit in {model.fit_s:.1f} s, loss {model.losses[0]:.3g} -> "
        f"{model.losses[-1]:.3g}, POD energy {model.energy:.6f}")
    rows, rows_mixed = [], []
    n_nodes = 0
    for i, x in enumerate(tt):
        case = learned.Case.build(c4_stenosed(x, K=K, **kw))
        n_nodes = case.mesh.n_nodes
        if i == 0:
            case.solve(case.plain_start(), 0.0, 1e-8)       # warm caches, untimed
        rows.append(learned.compare_starts(model, case, x, verbose=1))
        rows_mixed.append(learned.compare_starts(model, case, x, precision=PRECISIONS["mixed"],
                                                 verbose=1))
        r = rows[-1]
        log(f"learned: draw {i}: newton plain {r['plain']['newton_iters']} learned "
            f"{r['learned']['newton_iters']}, total s plain "
            f"{r['plain']['start_s'] + r['plain']['wall_s']:.3f} learned "
            f"{r['learned']['start_s'] + r['learned']['wall_s']:.3f}, start error "
            f"{r['learned']['start_err']:.3g} ({r['learned']['used']})")
        case.mesh.close()

    def avg(k, f):
        return float(np.mean([f(r[k]) for r in rows]))

    womersley = float(np.sqrt(2.0 * np.pi / period * 1.06 / 0.04))
    out = {"workload": "stenosed_pipe_family", "n_nodes": n_nodes, "K": K,
           "womersley": womersley, "max_severity": max_severity, "target": target,
           "params": int(th.shape[1]), "n_train": n_train,
           "n_train_converged": int(len(th)), "n_test": n_test,
           "generation": st,
           "pod_rank": model.r, "pod_energy": model.energy,
           "mlp": [int(th.shape[1]), 256, 256, model.r], "generation_s": st["wall_s"],
           "fit_s": model.fit_s, "fallbacks": sum(r["learned"]["used"] != "learned" for r in rows),
           "max_solution_rel_diff": max(r["solution_rel_diff"] for r in rows)}
    for k in ("plain", "learned"):
        out[k] = {"newton_iters": avg(k, lambda r: r["newton_iters"]),
                  "gmres_iters": avg(k, lambda r: r["gmres_iters"]),
                  "start_s": avg(k, lambda r: r["start_s"]),
                  "solve_s": avg(k, lambda r: r["wall_s"]),
                  "total_s": avg(k, lambda r: r["start_s"] + r["wall_s"]),
                  "start_rel_error": avg(k, lambda r: r["start_err"])}
    # the same comparison with mixed-precision (HB_MIXED) solves
    for k in ("plain", "learned"):
        out[k + "_mixed"] = {
            "newton_iters": float(np.mean([r[k]["newton_iters"] for r in rows_mixed])),
            "gmres_iters": float(np.mean([r[k]["gmres_iters"] for r in rows_mixed])),
            "total_s": float(np.mean([r[k]["start_s"] + r[k]["wall_s"] for r in rows_mixed])),
            "converged": int(sum(r[k]["status"] == 0 for r in rows_mixed))}
    # residual of the start relative to the plain start's, per draw
    out["learned"]["start_residual_ratio"] = float(np.mean(
        [r["learned"]["r_start"] / r["plain"]["r_start"] for r in rows]))
    log(f"learned warm start: {out}")
    return out


def learned_scale(args):
    if args.learned_scale == "small":
        return dict(K=2, n_rings=3, n_z=24, period=10.41, max_severity=0.5, batch=128,
                    gen_max_newton=400)
    return dict(batch=args.learned_batch)


def cfl_study(hbl, torch, log, workload="tjunction", cfls=(0.25, 1.0, 4.0, 16.0), steps=40):
    """Pseudo-time step study (Section 2.3 sets dt ~ h_c / u_c): FP64 Newton
    steps (mean-flow multigrid) from the plain start with the pseudo step
    held fixed at dt = cfl h_c / u_c (no growth), recording the residual
    relative to the plain start's after every step."""
    from dataclasses import replace
    from hbinputs.problems import c1_womersley, c2_tjunction
    P = c2_tjunction(K=10) if workload == "tjunction" else c1_womersley()
    prm = P.params
    n, N = P.mesh.n_nodes, prm.N
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)
    bc0 = hbl.BC(to(P.dirichlet[:, :1]), P.outlet_h[:, :1], P.outlet_R)
    Ys = torch.zeros((4, 1, n), dtype=torch.float64, device="cuda:0")
    hbl.newton_solve(gm, replace(prm, K=0), bc0, Ys,
                     solve_opts(hbl, rtol=1e-10, max_newton=60), raise_on_noconv=False)
    Y0 = torch.zeros((4, N, n), dtype=torch.float64, device="cuda:0")
    Y0[:, 0] = Ys[:, 0]
    r0 = hbl.newton_solve(gm, prm, bc, Y0.clone(), solve_opts(hbl, max_newton=0),
                          raise_on_noconv=False)["r0"]
    out = {"workload": workload, "n_nodes": n, "K": prm.K, "steps": steps, "runs": {}}
    for cfl in cfls:
        Y = Y0.clone()
        opts = solve_opts(hbl, rtol=1e-30, r_ref=r0, max_newton=1, max_gmres=300, cfl=cfl,
                          cfl_max=cfl)
        hist, gm_its = [], 0
        torch.cuda.synchronize()
        t = time.time()
        for _ in range(steps):
            try:
                rep = hbl.newton_solve(gm, prm, bc, Y, opts, raise_on_noconv=False)
            except hbl.HBError:
                hist.append(float("nan"))
                break
            hist.append(rep["r_final"] / r0)
            gm_its += rep["gmres_iters"]
        torch.cuda.synchronize()
        out["runs"][str(cfl)] = {"rel_residual": hist, "gmres_iters": gm_its,
                                 "seconds": time.time() - t}
        log(f"cfl {cfl}: residual after {len(hist)} steps {hist[-1]:.3e}, {gm_its} GMRES")
    gm.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["branching", "tjunction"], default="branching")
    ap.add_argument("--jv-reps", type=int, default=10)
    ap.add_argument("--max-gmres", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-time-to-solution", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--jv-only", action="store_true",
                    help="setup, then only public hb_jvp calls (for kernel profiling)")
    ap.add_argument("--plain-newton", type=int, default=150,
                    help="Newton steps of the plain start's last stage (0: no plain start; a "
                         "seeded state stands in, for kernel profiling)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--learned-train", type=int, default=0,
                    help="training solutions of the learned warm-start leg (0: skip it)")
    ap.add_argument("--learned-test", type=int, default=12)
    ap.add_argument("--learned-target", choices=["solution", "correction"], default="solution")
    ap.add_argument("--learned-batch", type=int, default=1,
                    help="draws solved together as one disjoint-union mesh")
    ap.add_argument("--learned-scale", choices=["full", "small"], default="full",
                    help="full: 42,679 nodes, K = 10, severity <= 0.7; small: 925 nodes, K = 2, "
                         "Womersley number 4, severity <= 0.5, draws solved 128 at a time")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned warm-start leg")
    ap.add_argument("--cfl-study", choices=["tjunction", "womersley"], default=None,
                    help="fixed-pseudo-step CFL study on this workload (skips the main bench)")
    ap.add_argument("--periodicity", choices=["tjunction", "womersley"], default=None,
                    help="march the workload period by period with the time-marching solver "
                         "and report the cycle-to-cycle change (skips the main bench)")
    ap.add_argument("--h", type=float, default=3.0 / 70.0)
    ap.add_argument("--tm-periods", type=int, default=0,
                    help="periods of the time-marching comparison on the Womersley pipe (0: off)")
    ap.add_argument("--tm-spp", type=int, default=50, help="time-marching steps per period")
    ap.add_argument("--tm-only", action="store_true",
                    help="run only the time-marching comparison (--tm-periods, default 6)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU "
                                   "(spatial partition + halo sum) design is not built"}))
        sys.exit(2)

    import torch
    import paper_2411_14315_amd as hbl
    from hbinputs.problems import seeded_state

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.periodicity:
        print(json.dumps({"periodicity": periodicity(hbl, torch, log, args.periodicity,
                                                     h=args.h, periods=args.tm_periods or 8)}),
              flush=True)
        return
    if args.cfl_study:
        print(json.dumps({"cfl_study": cfl_study(hbl, torch, log, args.cfl_study)}), flush=True)
        return
    if args.tm_only:
        print(json.dumps({"tm_vs_hb": tm_vs_hb(hbl, torch, log, args.tm_periods or 6,
                                               args.tm_spp)}), flush=True)
        return
    if args.learned_only:
        print(json.dumps({"learned_warm_start": learned_warm_start(
            torch, log, max(args.learned_train, 2), args.learned_test, target=args.learned_target,
            **learned_scale(args))}), flush=True)
        return

    dev = torch.device("cuda:0")
    t0 = time.time()
    P, wname = make_problem(args.workload)
    prm = P.params
    n, ne, N = P.mesh.n_nodes, P.mesh.n_tets, prm.N
    log(f"workload {wname}: {n} nodes, {ne} tets, N={N} ({time.time() - t0:.1f} s to generate)")
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)

    if args.calib_copy_mib:
        x = torch.empty(args.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        x.fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + written")

    t = time.time()
    if args.plain_newton > 0:
        Y0, preps = plain_start(hbl, torch, P, gm, log, max_newton=args.plain_newton)
    else:
        Y0, preps = to(seeded_state(P, 0)), [{"newton_iters": 0, "status": -4, "r_final": None}]
    plain_s = time.time() - t
    V = to(seeded_state(P, 1))
    dofs = 4 * n * N

    # public hb_jvp with stage timing (FP64 and FP32 directions)
    gm.set_timing(True)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def public_jv(Vx):
        JVx = torch.empty_like(Vx)
        for _ in range(3):
            hbl.jvp(gm, prm, bc, Y0, Vx, JVx)
        torch.cuda.synchronize()
        stages = {k: 0.0 for k in hbl.Mesh.STAGES}
        tot = 0.0
        for _ in range(args.jv_reps):
            e0.record(st)
            hbl.jvp(gm, prm, bc, Y0, Vx, JVx)
            e1.record(st)
            tt = gm.last_timings()
            for k in stages:
                stages[k] += tt[k] / args.jv_reps
            e1.synchronize()
            tot += e0.elapsed_time(e1) / args.jv_reps
        return tot, stages

    tot, stages = public_jv(V)
    tot32, stages32 = public_jv(V.float())
    gm.set_timing(False)
    log(f"hb_jvp: {tot:.3f} ms ({dofs / tot / 1e6:.2f} GDOF-modes/s); stages {stages}")
    if args.jv_only:
        gm.close()
        return

    elem_ms = stages["element"]
    per_lane, flop_src = elem_flops_per_lane()
    flops = (per_lane or 0.0) * ne * N
    roofline = {"bound": "alu", "achieved": flops / (elem_ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / (elem_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                "traffic": None, "kernel": "k_elem_block<1,double> (exact Jv)",
                "kernel_ms": elem_ms, "flop_per_lane": per_lane, "flop_source": flop_src,
                "frac_equation_count": ELEM_FLOPS_EQUATIONS * ne * N / (elem_ms * 1e-3) / 1e12
                / FP64_PEAK_TFLOPS,
                "hbm_algorithmic_GBs": elem_bytes(n, ne, N) / (elem_ms * 1e-3) / 1e9}
    traffic, traffic_detail = elem_traffic(n, ne, prm.K)
    if traffic is not None:
        roofline["traffic"] = traffic
        roofline["traffic_detail"] = dict(traffic_detail,
                                          hbm_measured_GBs=traffic / (elem_ms * 1e-3) / 1e9)

    r_ref = hbl.newton_solve(gm, prm, bc, Y0.clone(), hbl.SolveOptions(max_newton=0),
                             raise_on_noconv=False)["r0"]

    def newton_steps(precision):
        Y = Y0.clone()
        if args.warmup:
            hbl.newton_solve(gm, prm, bc, Y, solve_opts(hbl, rtol=1e-30, r_ref=r_ref,
                                                        max_newton=args.warmup,
                                                        max_gmres=args.max_gmres,
                                                        precision=precision,
                                                        verbose=int(args.verbose)),
                             raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.time()
        rep = hbl.newton_solve(gm, prm, bc, Y, solve_opts(hbl, rtol=1e-30, r_ref=r_ref,
                                                          max_newton=args.steps,
                                                          max_gmres=args.max_gmres,
                                                          precision=precision,
                                                          verbose=int(args.verbose)),
                               raise_on_noconv=False)
        torch.cuda.synchronize()
        wall = (time.time() - t) / args.steps
        return Y, {"jv_gdofs": dofs * rep["n_jv"] / (rep["jv_ms"] * 1e-3) / 1e9,
                   "ms_per_step": wall * 1e3, "gmres_iters": rep["gmres_iters"],
                   "gmres_per_step": rep["gmres_iters"] / args.steps,
                   "jv_ms_avg": rep["jv_ms"] / max(rep["n_jv"], 1),
                   "precond_ms_avg": rep["pc_ms"] / max(rep["n_jv"], 1),
                   "residual_rel": rep["r_final"] / r_ref}

    Y64, r64 = newton_steps(PRECISIONS["fp64"])
    log(f"FP64 Newton steps: {r64}")
    out = {"metric": METRIC, "value": r64["jv_gdofs"], "unit": "GDOF-modes/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": wname, "n_nodes": n, "n_tets": ne, "K": prm.K, "samples": N,
                      "reynolds": 500, "outlets": "resistance x" + str(len(P.outlet_R)),
                      "precision": "fp64", "preconditioner": "mean-flow multigrid"},
           "step": "one inexact Newton step (residual, mean-flow multigrid set-up, GMRES "
                   "eta=0.03 with the exact Jv, update), continuing one solve",
           "fp64": r64, "plain_start_s": plain_s,
           "plain_start": {"newton_iters": sum(r["newton_iters"] for r in preps),
                           "status": preps[-1]["status"],
                           "r_final": preps[-1]["r_final"]},
           "multigrid_levels": hbl.precond_levels(gm)}
    if not args.no_mixed:
        Ym, rm = newton_steps(PRECISIONS["mixed"])
        rm["state_rel_diff_vs_fp64"] = float(torch.linalg.norm(Ym - Y64) / torch.linalg.norm(Y64))
        rm["speedup_per_step_vs_fp64"] = r64["ms_per_step"] / rm["ms_per_step"]
        out["mixed"] = rm
        log(f"mixed Newton steps: {rm}")
    out["jv_public"] = {"value": dofs / (tot * 1e-3) / 1e9, "unit": "GDOF-modes/s", "ms": tot,
                        "stages_ms": stages}
    out["jv_public_fp32"] = {"value": dofs / (tot32 * 1e-3) / 1e9, "unit": "GDOF-modes/s",
                             "ms": tot32, "stages_ms": stages32}
    out["roofline"] = roofline
    if not args.no_time_to_solution:
        out["time_to_1e8"] = {f"{w}:{p_}": time_to_solution(hbl, torch, log, w, p_)
                              for w in ("womersley_pipe", "tjunction_h0.1")
                              for p_ in ("fp64", "mixed")}
    if args.tm_periods > 0:
        out["tm_vs_hb"] = tm_vs_hb(hbl, torch, log, args.tm_periods, args.tm_spp)
    if args.learned_train > 0:
        out["learned_warm_start"] = learned_warm_start(torch, log, args.learned_train,
                                                       args.learned_test,
                                                       target=args.learned_target,
                                                       **learned_scale(args))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, Y0.cpu().numpy(), V.cpu().numpy())
    gm.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
