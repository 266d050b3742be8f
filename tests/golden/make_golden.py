"""Write stored expected values computed by the CPU oracle only.

c1_solution.npz: the Womersley-pipe workload (cylinder R=1, L=6, 5 rings x
20 layers, K = 2, T = 1, Poiseuille inflow Q = 1 + 0.5 sin wt, zero traction)
solved by oracle.solve from the plain steady start to ||r|| <= 1e-12 ||r(y0)||.

c2_reduced_solution.npz: the T-junction workload on the coarse lattice
h = 0.1 (14,191 nodes), K = 10, Re = 500, one resistance outlet, solved the
same way (python make_golden.py c2; about two hours on one core).  Stored:
the solution's modal values at 2,048 seeded nodes (the full state is 9.5 MB),
the initial residual norm and the Newton count.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from hbinputs.problems import c1_womersley, c2_tjunction  # noqa: E402
from oracle import fem, solve  # noqa: E402


def c1_solution(path):
    P = c1_womersley()
    om = fem.from_mesh(P.mesh)
    t = time.time()
    Y0, r0 = solve.plain_start(om, P.params, P.dirichlet, P.outlet_h, P.outlet_R, rtol=1e-13)
    Y, rep = solve.newton_solve(om, P.params, Y0, P.dirichlet, P.outlet_h, P.outlet_R,
                                rtol=1e-12, verbose=True)
    assert rep.converged
    np.savez_compressed(path, Y=Y, Y0=Y0, r0=rep.r0, r_final=rep.r_final,
                        newton_iters=rep.newton_iters, seconds=time.time() - t)
    print("wrote", path, rep.newton_iters, rep.r0, rep.r_final, time.time() - t)


def c2_reduced_solution(path):
    P = c2_tjunction(K=10, h=0.1)
    om = fem.from_mesh(P.mesh)
    t = time.time()
    Y0, _ = solve.plain_start(om, P.params, P.dirichlet, P.outlet_h, P.outlet_R, rtol=1e-13,
                              max_newton=100, verbose=True)
    Y, rep = solve.newton_solve(om, P.params, Y0, P.dirichlet, P.outlet_h, P.outlet_R,
                                rtol=1e-12, max_newton=100, verbose=True)
    assert rep.converged
    np.savez_compressed(path + ".full.npz", Y=Y, Y0=Y0, r0=rep.r0, r_final=rep.r_final,
                        newton_iters=rep.newton_iters, seconds=time.time() - t)
    reduce_c2(path + ".full.npz", path)


def reduce_c2(full, path, n_sample=2048):
    """Keep the solution at a seeded sample of nodes."""
    g = np.load(full)
    n = g["Y"].shape[2]
    nodes = np.sort(np.random.default_rng(0).choice(n, n_sample, replace=False))
    np.savez_compressed(path, nodes=nodes, Y=g["Y"][:, :, nodes], r0=g["r0"],
                        r_final=g["r_final"], newton_iters=g["newton_iters"],
                        seconds=g["seconds"])
    print("wrote", path, int(g["newton_iters"]), float(g["r0"]), float(g["r_final"]))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "c2":
        c2_reduced_solution(os.path.join(HERE, "c2_reduced_solution.npz"))
    elif len(sys.argv) > 2 and sys.argv[1] == "c2-reduce":
        reduce_c2(sys.argv[2], os.path.join(HERE, "c2_reduced_solution.npz"))
    else:
        c1_solution(os.path.join(HERE, "c1_solution.npz"))
