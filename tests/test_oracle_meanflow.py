"""Pins of the oracle's mean-flow operator (oracle/tangent.py), the operator
that the solver's HB_PREC_MEANFLOW preconditioner approximates.

* At the zero state there is no advection, tau does not depend on the
  state and the strong residual vanishes, so the frozen-coefficient tangent
  equals the exact derivative of the residual (itself pinned by complex
  step), shift term included.
* The cyclic-shift average commutes with time shifts, and therefore maps a
  single harmonic to itself (the operator is block-diagonal in the Fourier
  modes, with H acting as i m w).
* For a time-independent state the average changes nothing.
"""
import numpy as np
import pytest

from hbinputs.problems import c1_womersley, seeded_state
from oracle import api, fem, residual as res, spectral, tangent


@pytest.fixture(scope="module")
def small():
    P = c1_womersley(n_rings=2, n_z=4)
    om = fem.from_mesh(P.mesh)
    return P, om


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_frozen_tangent_is_exact_tangent_at_rest(small):
    P, om = small
    prm = P.params
    y = np.zeros((4, prm.N, om.n))
    v = spectral.to_samples(seeded_state(P, 1), prm.K)
    H = api.H_of(prm)
    hs = np.zeros((om.n_outlets, prm.N))
    for shift in (0.0, 7.5):
        ex = res.jvp_samples(om, prm, y, v, hs, None, H, res.Options(backflow=False), shift=shift)
        fr = tangent.frozen_tangent_apply(om, prm, y, v, shift)
        assert _rel(fr, ex) <= 1e-13


def test_meanflow_commutes_with_time_shift(small):
    P, om = small
    prm = P.params
    y = api.samples_of(om, prm, seeded_state(P, 2), P.dirichlet)
    v = spectral.to_samples(seeded_state(P, 3), prm.K)
    a = tangent.meanflow_apply(om, prm, y, v, 2.0)
    for k in (1, 2):
        b = tangent.meanflow_apply(om, prm, y, np.roll(v, -k, axis=1), 2.0)
        assert _rel(np.roll(a, -k, axis=1), b) <= 1e-14
    # the frozen tangent itself does not commute at an unsteady state
    f0 = tangent.frozen_tangent_apply(om, prm, y, v, 2.0)
    f1 = tangent.frozen_tangent_apply(om, prm, y, np.roll(v, -1, axis=1), 2.0)
    assert _rel(np.roll(f0, -1, axis=1), f1) > 1e-3


def test_meanflow_keeps_each_harmonic(small):
    P, om = small
    prm = P.params
    y = api.samples_of(om, prm, seeded_state(P, 4), P.dirichlet)
    V = seeded_state(P, 5)
    for m in range(prm.K + 1):
        Vm = np.zeros_like(V)
        cols = [0] if m == 0 else [2 * m - 1, 2 * m]
        Vm[:, cols] = V[:, cols]
        out = spectral.to_modal(tangent.meanflow_apply(om, prm, y, spectral.to_samples(Vm, prm.K)),
                                prm.K)
        other = np.delete(out, cols, axis=1)
        assert np.linalg.norm(other) <= 1e-13 * np.linalg.norm(out)
    # the frozen tangent at the same unsteady state mixes harmonics
    V1 = np.zeros_like(V)
    V1[:, 1:3] = V[:, 1:3]
    fo = spectral.to_modal(tangent.frozen_tangent_apply(om, prm, y, spectral.to_samples(V1, prm.K)),
                           prm.K)
    assert np.linalg.norm(fo[:, 0]) > 1e-4 * np.linalg.norm(fo)


def test_meanflow_of_steady_state_is_frozen_tangent(small):
    P, om = small
    prm = P.params
    y = api.samples_of(om, prm, seeded_state(P, 6), P.dirichlet)
    ys = np.repeat(y[:, :1], prm.N, axis=1)
    v = spectral.to_samples(seeded_state(P, 7), prm.K)
    assert _rel(tangent.meanflow_apply(om, prm, ys, v, 1.0),
                tangent.frozen_tangent_apply(om, prm, ys, v, 1.0)) <= 1e-13
