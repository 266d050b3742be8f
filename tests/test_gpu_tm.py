"""GPU parity of one time-marching step (hb_tm_residual, hb_tm_jvp)
against the oracle's GLS time-marching solver, through the C ABI.

Bar: relative L2 error <= 1e-10 in FP64 at seeded states, on the Womersley
pipe and on the coarse T-junction (two inlets, resistance outlet), and an
HB call after time-marching calls still matches the oracle (the library's
cached time table is swapped back)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2411_14315_amd as hbl  # noqa: E402
from hbinputs.problems import c1_womersley, c2_tjunction, seeded_state  # noqa: E402
from oracle import api, fem, march  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


class TmCase:
    def __init__(self, P):
        self.P = P
        self.om = fem.from_mesh(P.mesh)
        self.gm = hbl.Mesh.from_mesh(P.mesh)

    def step(self, seed, dt=0.01, what=3.0, t1=0.37):
        """Seeded step data: y (candidate, (4, n)), y_old, a_old, Dirichlet
        values and outlet traction at t1."""
        P, om = self.P, self.om
        K, w = P.params.K, 2 * np.pi / P.params.period
        rng = np.random.default_rng(100 + seed)
        g1 = march.modal_at(P.dirichlet, K, w, t1)
        g0 = march.modal_at(P.dirichlet, K, w, t1 - dt)
        h1 = march.modal_at(P.outlet_h[:, :, None], K, w, t1)[:, 0]
        y = seeded_state(P, seed)[:, 0].copy()
        y_old = seeded_state(P, seed + 50)[:, 0].copy()
        y_old[:3][:, om.dirichlet] = g0[:, om.dirichlet]
        a_old = P.u_ref * rng.standard_normal((3, om.n))
        return y, y_old, a_old, g1, h1, dt, what


@pytest.fixture(scope="module")
def c1():
    return TmCase(c1_womersley())


@pytest.fixture(scope="module")
def tj():
    return TmCase(c2_tjunction(K=10, h=0.1))


@pytest.mark.parametrize("case", ["c1", "tj"])
@pytest.mark.parametrize("seed", [0, 1])
def test_tm_residual_and_jvp_parity(case, seed, request):
    c = request.getfixturevalue(case)
    P, om = c.P, c.om
    print(f"tm parity case={case} seed={seed} n={om.n}", flush=True)
    y, y_old, a_old, g1, h1, dt, what = c.step(seed)
    tm = hbl.TmStep(dt, what, dev(y_old), dev(a_old), dev(g1), h1, P.outlet_R)
    y_in = y.copy()
    y[:3][:, om.dirichlet] = g1[:, om.dirichlet]
    ref = march.tm_residual(om, P.params, y, y_old[:3], a_old, dt, what, h1, P.outlet_R)
    got = host(hbl.tm_residual(c.gm, P.params, tm, dev(y_in)))
    assert rel(got, ref) <= TOL, rel(got, ref)
    assert np.all(got[:3][:, om.dirichlet] == 0.0)
    v = seeded_state(P, seed + 20)[:, 0].copy()
    refj = march.tm_jvp(om, P.params, y, v, y_old[:3], a_old, dt, what, P.outlet_R)
    gotj = host(hbl.tm_jvp(c.gm, P.params, tm, dev(y_in), dev(v)))
    assert rel(gotj, refj) <= TOL, rel(gotj, refj)


def test_tm_then_hb_calls(c1):
    """A time-marching call between two HB calls leaves the HB path intact."""
    P, om = c1.P, c1.om
    bc = hbl.BC(dev(P.dirichlet), P.outlet_h, P.outlet_R)
    Y = seeded_state(P, 3)
    ref = api.residual_modal(om, P.params, Y, P.dirichlet, P.outlet_h, P.outlet_R)
    first = host(hbl.residual(c1.gm, P.params, bc, dev(Y)))
    y, y_old, a_old, g1, h1, dt, what = c1.step(4)
    tm = hbl.TmStep(dt, what, dev(y_old), dev(a_old), dev(g1), h1, P.outlet_R)
    hbl.tm_residual(c1.gm, P.params, tm, dev(y))
    second = host(hbl.residual(c1.gm, P.params, bc, dev(Y)))
    assert rel(first, ref) <= 1e-10 and rel(second, ref) <= 1e-10


def test_tm_argument_errors(c1):
    P = c1.P
    y, y_old, a_old, g1, h1, dt, what = c1.step(5)
    for bad_dt, bad_w in ((0.0, 1.0), (-1.0, 1.0), (0.01, -1.0), (0.01, float("nan"))):
        tm = hbl.TmStep(bad_dt, bad_w, dev(y_old), dev(a_old), dev(g1), h1, None)
        with pytest.raises(hbl.HBError) as e:
            hbl.tm_residual(c1.gm, P.params, tm, dev(y))
        assert e.value.status == hbl.HB_ERR_ARG


def _small_pipe():
    """259-node pipe, Q = 1 + 0.5 sin(w t), resistance outlet with a modal
    traction (exercises h(t) and R Q at every step)."""
    from hbinputs.meshes import cylinder_mesh
    from hbinputs.problems import Params, Problem, poiseuille_dirichlet, womersley_like_flow
    m = cylinder_mesh(1.0, 6.0, 3, 6)
    K = 2
    prm = Params(K=K, period=1.0)
    d = poiseuille_dirichlet(m, K, [womersley_like_flow(K)])
    oh = np.array([[0.2, 0.05, -0.1, 0.0, 0.03]])
    return Problem("pipe", m, prm, d, oh, np.array([0.5]), u_ref=2 / np.pi)


@pytest.mark.parametrize("what", [None, 2.0])
def test_tm_march_matches_oracle(what):
    """hb_tm_march against oracle.march: every step's state, the final
    acceleration.  Both sides solve each step to ||r|| <= 1e-12 ||r_0||, so
    the states agree to the step Jacobian's conditioning times that."""
    P = _small_pipe()
    om, prm = fem.from_mesh(P.mesh), P.params
    gm = hbl.Mesh.from_mesh(P.mesh)
    K, w = prm.K, 2 * np.pi / prm.period
    dt, n_steps = 0.02, 8
    print(f"tm march what={what} n={om.n} steps={n_steps}", flush=True)
    y0 = np.zeros((4, om.n))
    g0 = march.modal_at(P.dirichlet, K, w, 0.0)
    y0[:3][:, om.dirichlet] = g0[:, om.dirichlet]
    a0 = np.zeros((3, om.n))
    ys, a_ref, rep_ref = march.march(
        om, prm, y0, a0, dt, n_steps, lambda t: march.modal_at(P.dirichlet, K, w, t),
        lambda t: march.modal_at(P.outlet_h[:, :, None], K, w, t)[:, 0], P.outlet_R,
        what=what, rtol=1e-12, atol=0.0, eta=1e-8)
    assert rep_ref.max_step_residual < 1e-9
    Y, A = dev(y0), dev(a0)
    traj = torch.empty((n_steps, 4, om.n), dtype=torch.float64, device="cuda")
    bc = hbl.BC(dev(P.dirichlet), P.outlet_h, P.outlet_R)
    opts = hbl.TmOptions(dt=dt, n_steps=n_steps, rtol=1e-12, atol=0.0, gmres_eta=1e-8,
                         max_newton=30, max_gmres=2000, omega_hat=-1.0 if what is None else what)
    rep = hbl.tm_march(gm, prm, bc, Y, A, opts, traj=traj)
    assert rep["steps"] == n_steps and rep["status"] == hbl.HB_OK
    got = host(traj)
    for k in range(n_steps):
        e = rel(got[k], ys[k + 1])
        assert e <= 1e-9, (k, e)
    assert rel(host(Y), ys[-1]) <= 1e-9
    assert rel(host(A), a_ref) <= 1e-7


def test_tm_march_zero_steps_and_errors(c1):
    P = c1.P
    n = c1.om.n
    y0 = np.random.default_rng(9).standard_normal((4, n))
    Y, A = dev(y0), dev(np.zeros((3, n)))
    bc = hbl.BC(dev(P.dirichlet), P.outlet_h, P.outlet_R)
    rep = hbl.tm_march(c1.gm, P.params, bc, Y, A, hbl.TmOptions(n_steps=0))
    assert rep["steps"] == 0 and np.array_equal(host(Y), y0)
    for bad in (dict(dt=0.0), dict(n_steps=-1), dict(rtol=0.0), dict(restart=0),
                dict(omega_hat=float("nan"))):
        with pytest.raises(hbl.HBError) as e:
            hbl.tm_march(c1.gm, P.params, bc, Y, A, hbl.TmOptions(**bad))
        assert e.value.status == hbl.HB_ERR_ARG
