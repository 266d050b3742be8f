#!/usr/bin/env python3
"""Benchmark of the HB-GLS hot path on one MI355X.

Workload: synthetic Glenn-like T-junction (two inlets r = 0.5 meeting
head-on, outlet r = 0.6, lattice-carved P1 mesh with h = 3/70: 158,688
nodes, 848,252 tetrahedra), K = 10 harmonics (21 samples), seeded inflow
waveforms at Re = 500, one resistance outlet, rho = 1.06, mu = 0.04, FP64.

A step is one pass of the whole hot path: one inexact Newton step of
hb_newton_solve (HB residual; Jacobi diagonal and per-node time blocks;
GMRES to eta = 0.03 or the iteration cap, each iteration one Jacobian-vector
product with its time-axis transforms, element and face kernels and
scatter; the Newton update), continuing from the previous step's state.
The state before the first timed step is the plain start (a bounded K = 0
solve broadcast to all harmonics) advanced by the warm-up steps.

The line reports:
  value        Jacobian-vector throughput inside the timed steps,
               4 n N x (operator applications) / (operator time), with the
               operator time from HIP events on the solve stream;
  ms_per_step  wall time per Newton step;
  jv_public    throughput of the public modal hb_jvp entry point;
  tm_step_jv   one time-marching step's exact Jv (hb_tm_jvp) on the same
               mesh, and how many of them one HB Jv costs;
  tm_vs_hb     the paper's comparison on the Womersley pipe: the GLS
               time-marching solver marched period by period against the
               HB solve (wall time, cycle-to-cycle change, difference);
  time_to_1e8  a complete FP64 solve to 1e-8 of the Womersley-pipe workload
               (1,911 nodes, K = 2) from its plain start;
  roofline     the element Jacobian-vector kernel against the FP64 vector
               peak, its duration from HIP events on its launch stream;
  cpu_baseline the CPU oracle's Jacobian-vector throughput on a bounded
               sample of the same workload.
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
# FP64 operations per (tetrahedron, sample) lane of the element kernels,
# counted from their source (fused multiply-add = 2).
ELEM_FLOPS = {"exact": 1680, "paper": 970, "residual": 1040}


# HBM bytes per launch of the FP64 exact-Jv element kernel at the benchmark
# size, from rocprofv3 FETCH_SIZE (x 2.0) and WRITE_SIZE (x 1.0) counters,
# each scale read off a plain 1 GiB device copy; valid while the
# element-kernel source section hashes to the recorded value.
ELEM_TRAFFIC = {"sha256_prefix": "85dde60c62f4d23e", "fetch_kib": 394036, "write_kib": 1193487,
                "fetch_scale": 2.0, "write_scale": 1.0, "n_nodes": 158688, "n_tets": 848252,
                "K": 10, "profile": "profiles/k_elem_jvp_exact_tjunction_K10_traffic.md"}


def elem_traffic(n, ne, K):
    import hashlib
    src = open(os.path.join(ROOT, "paper_2411_14315_amd", "csrc", "hb_kernels.hip")).read()
    a = src.index("// ------------------------------------------------------------- elements")
    b = src.index("// --------------------------------------------------------------- faces")
    t = ELEM_TRAFFIC
    if (hashlib.sha256(src[a:b].encode()).hexdigest()[:16] != t["sha256_prefix"]
            or (n, ne, K) != (t["n_nodes"], t["n_tets"], t["K"])):
        return None, None
    rd = t["fetch_kib"] * 1024 * t["fetch_scale"]
    wr = t["write_kib"] * 1024 * t["write_scale"]
    return rd + wr, {"read_bytes": rd, "write_bytes": wr, "source": t["profile"]}


def elem_bytes(n, ne, N, kind):
    """Algorithmic HBM bytes of one element-kernel launch: node samples read
    once (7 channels of state, 7 of direction for Jv), accumulator rows
    read-modify-written once (7 channels), geometry (20 doubles: each lane
    of a quad reads its own node gradient) and
    connectivity (4 int32) once per tetrahedron."""
    node_ch = 14 if kind != "residual" else 7
    return 8.0 * n * N * (node_ch + 2 * 7) + ne * (20 * 8 + 4 * 4)


def cpu_baseline(P, Y, V, budget_s=30.0):
    """Oracle exact Jv on a bounded sample: the rows of a contiguous block of
    nodes (all elements touching them), timed, scaled to the full mesh."""
    from oracle import api, fem, residual as res, spectral
    om = fem.from_mesh(P.mesh)
    prm = P.params
    y = api.samples_of(om, prm, Y, P.dirichlet)
    v = spectral.to_samples(V, prm.K)
    H = api.H_of(prm)
    hs = api.h_samples(prm, P.outlet_h)
    frac = 0.02
    while True:
        rows = np.arange(int(frac * om.n))
        mark = np.zeros(om.n, bool)
        mark[rows] = True
        nel = int(mark[om.tets].any(axis=1).sum())
        t = time.perf_counter()
        res.jvp_samples(om, prm, y, v, hs, P.outlet_R, H, rows=rows)
        dt = time.perf_counter() - t
        if dt > 0.25 * budget_s or frac >= 0.5:
            break
        frac = min(0.5, frac * max(2.0, 0.5 * budget_s / max(dt, 1e-3)))
    t_full = dt * om.ne / nel
    return {"value": 4 * om.n * prm.N / t_full / 1e9, "unit": "GDOF-modes/s", "cores": 1,
            "kind": "oracle",
            "sample": f"exact Jv rows of {rows.size} nodes ({nel} of {om.ne} tetrahedra, "
                      f"{dt:.1f} s), scaled by element count"}


def tm_step_jv(hbl, torch, P, gm, Y0, V, st, reps):
    """Exact Jv of one time-marching step (hb_tm_jvp: one time level, the
    mean modes of the HB state and direction as the step's state and
    direction, dt = T/200, omega-hat = 2 pi / T) on the same mesh, timed
    with HIP events on the launch stream."""
    n = P.mesh.n_nodes
    y = Y0[:, 0].contiguous()
    v = V[:, 0].contiguous()
    a_old = torch.zeros((3, n), dtype=torch.float64, device="cuda:0")
    g = torch.from_numpy(np.ascontiguousarray(P.dirichlet[:, 0])).to("cuda:0")
    h = np.ascontiguousarray(P.outlet_h[:, 0])
    tm = hbl.TmStep(P.params.period / 200, 2 * np.pi / P.params.period, y.clone(), a_old, g, h,
                    P.outlet_R)
    jv = torch.empty_like(v)
    for _ in range(5):
        hbl.tm_jvp(gm, P.params, tm, y, v, jv)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        hbl.tm_jvp(gm, P.params, tm, y, v, jv)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms": ms, "value": 4 * n / (ms * 1e-3) / 1e9, "unit": "GDOF/s"}


def womersley_time_to_solution(hbl, torch, log, precision="fp64"):
    """Complete FP64 solve of the Womersley-pipe workload to 1e-8 from its
    plain start (K = 0 solve broadcast), after one untimed warm-up solve."""
    from dataclasses import replace
    from hbinputs.problems import c1_womersley
    P = c1_womersley()
    prm = P.params
    n, N = P.mesh.n_nodes, prm.N
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)
    bc0 = hbl.BC(to(P.dirichlet[:, :1]), P.outlet_h[:, :1], None)
    res = {}
    for rep_i in range(2):
        torch.cuda.synchronize()
        t = time.time()
        Ys = torch.zeros((4, 1, n), dtype=torch.float64, device="cuda:0")
        r0 = hbl.newton_solve(gm, replace(prm, K=0), bc0, Ys,
                              hbl.SolveOptions(rtol=1e-10, max_newton=60, max_gmres=500))
        t_plain = time.time() - t
        Y = torch.zeros((4, N, n), dtype=torch.float64, device="cuda:0")
        Y[:, 0] = Ys[:, 0]
        t = time.time()
        r = hbl.newton_solve(gm, prm, bc, Y, hbl.SolveOptions(
            rtol=1e-8, max_newton=300, max_gmres=500,
            precision=PRECISIONS[precision]),
            raise_on_noconv=False)
        t_solve = time.time() - t
        res = {"workload": "womersley_pipe", "precision": precision, "n_nodes": n, "K": prm.K,
               "seconds": t_solve, "plain_start_seconds": t_plain,
               "total_seconds": t_solve + t_plain, "newton_iters": r["newton_iters"],
               "gmres_iters": r["gmres_iters"], "status": r["status"],
               "r_final_rel": r["r_final"] / r["r0"]}
    log(f"womersley pipe time to 1e-8: {res}")
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


def tm_vs_hb(hbl, torch, log, periods, spp):
    """The paper's comparison on the Womersley-pipe workload: the GLS
    time-marching solver (hb_tm_march, dt = T/spp, per-step Newton to three
    orders and GMRES to 0.03, the paper's settings for both solvers) marched
    period by period from the plain start, against the HB solve to 1e-8.
    Per period: wall time, cycle-to-cycle change of the marched states and
    their difference from the HB solution at the same times."""
    from dataclasses import replace
    from hbinputs.problems import c1_womersley
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
                     hbl.SolveOptions(rtol=1e-10, max_newton=60, max_gmres=500))
    Yhb = torch.zeros((4, N, n), dtype=torch.float64, device="cuda:0")
    Yhb[:, 0] = Ys[:, 0]
    torch.cuda.synchronize()
    t = time.time()
    rhb = hbl.newton_solve(gm, prm, bc, Yhb, hbl.SolveOptions(rtol=1e-8, max_newton=300,
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
                             max_newton=10, max_gmres=500)
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


def learned_warm_start(torch, log, n_train, n_test, K=2):
    """Learned warm start on the stenosed-pipe family (925 nodes, Womersley
    number 4, severity up to 50 %): n_train solutions generated by the
    solver (batched as disjoint-union meshes), POD + MLP trained on the GPU,
    then plain vs learned start on n_test held-out draws to 1e-8 of the
    plain start's residual.  Times include the steady start (which the
    correction model builds on) and the network + expansion."""
    from hbinputs.problems import c4_stenosed, c4_stenosis_params
    from paper_2411_14315_amd import learned
    kw = dict(n_rings=3, n_z=24, period=10.41)
    th = c4_stenosis_params(n_train, 2024, K=K, max_severity=0.5)
    tt = c4_stenosis_params(n_test, 2025, K=K, max_severity=0.5)
    Y, Y0, st = learned.generate_snapshots([c4_stenosed(x, K=K, **kw) for x in th], batch=128)
    log(f"learned: generated {n_train} solutions in {st['wall_s']:.1f} s")
    rank = min(64, n_train // 2)
    model = learned.WarmStart(rank=rank, hidden=(256, 256)).fit(th, Y, Y0, steps=4000, lr=2e-3)
    log(f"learned: fit in {model.fit_s:.1f} s, loss {model.losses[0]:.3g} -> {model.losses[-1]:.3g}")
    rows, rows_mixed = [], []
    for x in tt:
        case = learned.Case.build(c4_stenosed(x, K=K, **kw))
        case.solve(case.plain_start(), 0.0, 1e-8)       # warm caches, untimed
        rows.append(learned.compare_starts(model, case, x))
        rows_mixed.append(learned.compare_starts(model, case, x, precision=PRECISIONS["mixed"]))
        case.mesh.close()

    def avg(k, f):
        return float(np.mean([f(r[k]) for r in rows]))

    out = {"workload": "stenosed_pipe_family", "n_nodes": 925, "K": K, "womersley": 4.0,
           "params": int(th.shape[1]), "n_train": n_train, "n_test": n_test,
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


def branching_leg(hbl, torch, log, steps=3, plain_newton=10):
    """Branching artery (1,255,132 nodes, 7,046,522 tets, K = 10, eight
    resistance outlets): public Jv in FP64 and FP32, then `steps` inexact
    Newton steps from the same plain start in FP64, HB_MIXED and
    HB_F32_BASIS, with the reduced-precision states compared to the FP64
    state after the same steps."""
    from dataclasses import replace
    from hbinputs.problems import c3_branching
    t = time.time()
    P = c3_branching()
    log(f"branching artery mesh: {P.mesh.n_nodes} nodes, {P.mesh.n_tets} tets, {time.time() - t:.1f} s")
    prm = P.params
    n, N = P.mesh.n_nodes, prm.N
    gm = hbl.Mesh.from_mesh(P.mesh)
    to = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")  # noqa: E731
    bc = hbl.BC(to(P.dirichlet), P.outlet_h, P.outlet_R)
    bc0 = hbl.BC(to(P.dirichlet[:, :1]), P.outlet_h[:, :1], P.outlet_R)
    Ys = torch.zeros((4, 1, n), dtype=torch.float64, device="cuda:0")
    hbl.newton_solve(gm, replace(prm, K=0), bc0, Ys,
                     hbl.SolveOptions(rtol=1e-10, max_newton=plain_newton, max_gmres=300),
                     raise_on_noconv=False)
    Y0 = torch.zeros((4, N, n), dtype=torch.float64, device="cuda:0")
    Y0[:, 0] = Ys[:, 0]
    dofs = 4.0 * n * N
    V = Y0.clone()
    out = {"workload": "branching_artery", "n_nodes": n, "n_tets": P.mesh.n_tets, "K": prm.K,
           "outlets": int(P.outlet_R.size)}
    for name, Vx in (("jv_fp64", V), ("jv_fp32", V.float())):
        for _ in range(3):
            hbl.jvp(gm, prm, bc, Y0, Vx)
        torch.cuda.synchronize()
        t = time.time()
        for _ in range(10):
            hbl.jvp(gm, prm, bc, Y0, Vx)
        torch.cuda.synchronize()
        ms = (time.time() - t) / 10 * 1e3
        out[name] = {"ms": ms, "gdofs": dofs / (ms * 1e-3) / 1e9}
    states = {}
    for p_ in ("fp64", "mixed", "f32_basis"):
        opts = hbl.SolveOptions(rtol=1e-30, max_newton=1, max_gmres=300, precision=PRECISIONS[p_])
        Y = Y0.clone()
        torch.cuda.synchronize()
        t = time.time()
        reps = [hbl.newton_solve(gm, prm, bc, Y, opts, raise_on_noconv=False) for _ in range(steps)]
        torch.cuda.synchronize()
        states[p_] = Y
        out[p_] = {"ms_per_step": (time.time() - t) / steps * 1e3,
                   "gmres_iters_per_step": [r["gmres_iters"] for r in reps],
                   "residual_per_step": [r["r_final"] for r in reps]}
        if p_ != "fp64":
            out[p_]["state_rel_diff_vs_fp64"] = float(
                torch.linalg.norm(Y - states["fp64"]) / torch.linalg.norm(states["fp64"]))
    log(f"branching artery: {out}")
    gm.close()
    return out


def cfl_study(hbl, torch, log, workload="tjunction", cfls=(0.25, 1.0, 4.0, 16.0), steps=40):
    """Pseudo-time step study (Section 2.3 sets dt ~ h_c / u_c): FP64 Newton
    steps from the plain start with the pseudo step held fixed at
    dt = cfl h_c / u_c (no growth), recording the residual relative to the
    plain start's after every step."""
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
                     hbl.SolveOptions(rtol=1e-10, max_newton=30, max_gmres=300),
                     raise_on_noconv=False)
    Y0 = torch.zeros((4, N, n), dtype=torch.float64, device="cuda:0")
    Y0[:, 0] = Ys[:, 0]
    r0 = hbl.newton_solve(gm, prm, bc, Y0.clone(), hbl.SolveOptions(max_newton=0),
                          raise_on_noconv=False)["r0"]
    out = {"workload": workload, "n_nodes": n, "K": prm.K, "steps": steps, "runs": {}}
    for cfl in cfls:
        Y = Y0.clone()
        opts = hbl.SolveOptions(rtol=1e-30, r_ref=r0, max_newton=1, max_gmres=300, cfl=cfl,
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
    ap.add_argument("--jv-reps", type=int, default=20)
    ap.add_argument("--mode", choices=["solve", "jv"], default="solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--h", type=float, default=3.0 / 70.0)
    ap.add_argument("--K", type=int, default=10)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--plain-newton", type=int, default=30)
    ap.add_argument("--max-gmres", type=int, default=300)
    ap.add_argument("--cfl-max", type=float, default=0.0)
    ap.add_argument("--precision", choices=["fp64", "mixed", "f32_basis", "both"], default="both",
                    help="'both': FP64 plus the two reduced-precision Krylov forms")
    ap.add_argument("--no-time-to-solution", action="store_true")
    ap.add_argument("--learned-train", type=int, default=384,
                    help="training solutions of the learned warm-start leg (0: skip it)")
    ap.add_argument("--learned-test", type=int, default=12)
    ap.add_argument("--cfl-study", choices=["tjunction", "womersley"], default=None,
                    help="fixed-pseudo-step CFL study on this workload (skips the main bench)")
    ap.add_argument("--periodicity", choices=["tjunction", "womersley"], default=None,
                    help="march the workload period by period with the time-marching solver "
                         "and report the cycle-to-cycle change (skips the main bench)")
    ap.add_argument("--tm-periods", type=int, default=6,
                    help="periods of the time-marching comparison on the Womersley pipe (0: off)")
    ap.add_argument("--tm-spp", type=int, default=50, help="time-marching steps per period")
    ap.add_argument("--branching", type=int, default=0,
                    help="Newton steps of the branching-artery leg (0: skip it; the mesh "
                         "takes about a minute to generate)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU "
                                   "(spatial partition + halo sum) design is not built"}))
        sys.exit(2)

    import torch
    import paper_2411_14315_amd as hbl
    from hbinputs.problems import c2_tjunction, seeded_state

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.periodicity:
        print(json.dumps({"periodicity": periodicity(hbl, torch, log, args.periodicity,
                                                     h=args.h, periods=args.tm_periods)}),
              flush=True)
        return
    if args.cfl_study:
        print(json.dumps({"cfl_study": cfl_study(hbl, torch, log, args.cfl_study)}), flush=True)
        return

    dev = torch.device("cuda:0")
    t0 = time.time()
    P = c2_tjunction(K=args.K, h=args.h)
    prm = P.params
    n, ne, N = P.mesh.n_nodes, P.mesh.n_tets, prm.N
    log(f"workload: {n} nodes, {ne} tets, N={N} ({time.time() - t0:.1f} s to generate)")
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

    # plain start: a bounded steady K = 0 solve broadcast to all harmonics
    from dataclasses import replace
    p0 = replace(prm, K=0)
    bc0 = hbl.BC(to(P.dirichlet[:, :1]), P.outlet_h[:, :1], P.outlet_R)
    Ys = torch.zeros((4, 1, n), dtype=torch.float64, device=dev)
    t = time.time()
    rep0 = hbl.newton_solve(gm, p0, bc0, Ys,
                            hbl.SolveOptions(rtol=1e-6, max_newton=args.plain_newton,
                                             max_gmres=300, cfl_max=args.cfl_max,
                                             verbose=int(args.verbose)),
                            raise_on_noconv=False)
    plain_s = time.time() - t
    log(f"plain start: {rep0['newton_iters']} Newton, {rep0['gmres_iters']} GMRES, "
        f"|r| {rep0['r0']:.3e} -> {rep0['r_final']:.3e}, {plain_s:.2f} s")
    Y0 = torch.zeros((4, N, n), dtype=torch.float64, device=dev)
    Y0[:, 0] = Ys[:, 0]
    V = to(seeded_state(P, 1))

    # public hb_jvp microbenchmark with stage timing
    gm.set_timing(True)
    st = torch.cuda.current_stream()
    JV = torch.empty_like(V)
    for _ in range(5):
        hbl.jvp(gm, prm, bc, Y0, V, JV)
    torch.cuda.synchronize()
    stages = {k: 0.0 for k in hbl.Mesh.STAGES}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tot = 0.0
    for _ in range(args.jv_reps):
        e0.record(st)
        hbl.jvp(gm, prm, bc, Y0, V, JV)
        e1.record(st)
        tt = gm.last_timings()
        for k in stages:
            stages[k] += tt[k] / args.jv_reps
        e1.synchronize()
        tot += e0.elapsed_time(e1) / args.jv_reps
    V32 = V.float()
    JV32 = torch.empty_like(V32)
    for _ in range(5):
        hbl.jvp(gm, prm, bc, Y0, V32, JV32)
    torch.cuda.synchronize()
    stages32 = {k: 0.0 for k in hbl.Mesh.STAGES}
    tot32 = 0.0
    for _ in range(args.jv_reps):
        e0.record(st)
        hbl.jvp(gm, prm, bc, Y0, V32, JV32)
        e1.record(st)
        tt = gm.last_timings()
        for k in stages32:
            stages32[k] += tt[k] / args.jv_reps
        e1.synchronize()
        tot32 += e0.elapsed_time(e1) / args.jv_reps
    gm.set_timing(False)
    dofs = 4 * n * N
    jv_public = dofs / (tot * 1e-3) / 1e9
    log(f"hb_jvp: {tot:.3f} ms ({jv_public:.2f} GDOF-modes/s); stages {stages}")
    tm_jv = tm_step_jv(hbl, torch, P, gm, Y0, V, st, args.jv_reps)
    log(f"hb_tm_jvp (one time-marching step's Jv): {tm_jv['ms']:.3f} ms; "
        f"HB Jv / step Jv = {tot / tm_jv['ms']:.1f}")

    elem_ms = stages["element"]
    flops = ELEM_FLOPS["exact"] * ne * N
    eb = elem_bytes(n, ne, N, "exact")
    traffic, traffic_detail = elem_traffic(n, ne, args.K)
    roofline = {"bound": "alu", "achieved": flops / (elem_ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / (elem_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                "traffic": traffic,
                "kernel": "k_elem_jvp_exact", "kernel_ms": elem_ms,
                "hbm_algorithmic_GBs": eb / (elem_ms * 1e-3) / 1e9}
    if traffic is not None:
        roofline["traffic_detail"] = dict(traffic_detail,
                                          hbm_measured_GBs=traffic / (elem_ms * 1e-3) / 1e9)

    out = {"metric": METRIC, "unit": "GDOF-modes/s", "n_gpus": 1, "higher_is_better": True,
           "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "tjunction_glenn_like", "n_nodes": n, "n_tets": ne, "K": args.K,
                      "samples": N, "reynolds": 500, "outlet": "resistance",
                      "precision": "fp64", "rtol": 1e-8}}
    if args.mode == "jv":
        out.update({"value": jv_public, "steps": args.jv_reps, "warmup": 5, "ms_per_step": tot,
                    "step": "one public hb_jvp call"})
    else:
        def newton_steps(precision):
            opts = hbl.SolveOptions(rtol=1e-30, max_newton=1, max_gmres=args.max_gmres,
                                    cfl_max=args.cfl_max, verbose=int(args.verbose),
                                    precision=precision)
            Y = Y0.clone()
            for _ in range(args.warmup):
                hbl.newton_solve(gm, prm, bc, Y, opts, raise_on_noconv=False)
            torch.cuda.synchronize()
            reps = []
            t = time.time()
            for _ in range(args.steps):
                reps.append(hbl.newton_solve(gm, prm, bc, Y, opts, raise_on_noconv=False))
            torch.cuda.synchronize()
            wall = (time.time() - t) / args.steps
            n_jv = sum(r["n_jv"] for r in reps)
            jv_ms = sum(r["jv_ms"] for r in reps)
            return {"jv_gdofs": dofs * n_jv / (jv_ms * 1e-3) / 1e9, "ms_per_step": wall * 1e3,
                    "gmres_iters_per_step": [r["gmres_iters"] for r in reps],
                    "residual_per_step": [r["r_final"] for r in reps],
                    "jv_ms_avg": jv_ms / max(n_jv, 1)}
        main_prec = "fp64" if args.precision == "both" else args.precision
        res = {p_: newton_steps(PRECISIONS[p_])
               for p_ in (["fp64", "mixed", "f32_basis"] if args.precision == "both"
                          else [main_prec])}
        r0 = res[main_prec]
        out.update({"value": r0["jv_gdofs"], "steps": args.steps, "warmup": args.warmup,
                    "ms_per_step": r0["ms_per_step"],
                    "step": f"one {main_prec.upper()} inexact Newton step (residual, "
                            "preconditioner, GMRES eta=0.03 with exact Jv, update) on the "
                            "T-junction",
                    "gmres_iters_per_step": r0["gmres_iters_per_step"],
                    "residual_per_step": r0["residual_per_step"],
                    "plain_start_s": plain_s, "jv_ms_avg": r0["jv_ms_avg"]})
        for p_ in ("mixed", "f32_basis"):
            if p_ in res and main_prec != p_:
                out[p_] = res[p_]
        if not args.no_time_to_solution:
            out["time_to_1e8"] = {p_: womersley_time_to_solution(hbl, torch, log, p_)
                                  for p_ in res}
        if args.tm_periods > 0:
            out["tm_vs_hb"] = tm_vs_hb(hbl, torch, log, args.tm_periods, args.tm_spp)
        if args.branching > 0:
            out["branching_artery"] = branching_leg(hbl, torch, log, args.branching)
        if args.learned_train > 0:
            out["learned_warm_start"] = learned_warm_start(torch, log, args.learned_train,
                                                           args.learned_test)
    out["jv_public"] = {"value": jv_public, "unit": "GDOF-modes/s", "ms": tot,
                        "stages_ms": stages}
    out["jv_public_fp32"] = {"value": dofs / (tot32 * 1e-3) / 1e9, "unit": "GDOF-modes/s",
                             "ms": tot32, "stages_ms": stages32}
    tm_jv["hb_jv_over_step_jv"] = tot / tm_jv["ms"]
    out["tm_step_jv"] = tm_jv
    out["roofline"] = roofline
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, Y0.cpu().numpy(), V.cpu().numpy())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
