"""Modal-interface wrappers: the same calls as the C library, computed by
the oracle.

Y, R, V, JV are (4, N, n) real modal arrays [a_0, a_1, b_1, ..., a_K, b_K]
per field (u1, u2, u3, p) and node.  Dirichlet velocity entries of Y are
replaced by the given boundary coefficients (Section 2.3: the Dirichlet
condition is built into the unknowns); those of V are treated as zero.
Residual and Jv rows are returned as modal coefficients of the time-sample
rows, R = F r (F the real DFT).
"""
from __future__ import annotations

import numpy as np

from . import residual as res
from . import spectral, tangent
from .fem import OMesh


def omega(prm) -> float:
    return 2.0 * np.pi / prm.period


def H_of(prm) -> np.ndarray:
    return spectral.hb_matrix(prm.K, omega(prm))


def apply_dirichlet_modal(om: OMesh, Y: np.ndarray, dirichlet: np.ndarray) -> np.ndarray:
    Y = np.array(Y, copy=True)
    Y[:3][:, :, om.dirichlet] = dirichlet[:, :, om.dirichlet]
    return Y


def samples_of(om: OMesh, prm, Y, dirichlet):
    return spectral.to_samples(apply_dirichlet_modal(om, Y, dirichlet), prm.K)


def h_samples(prm, outlet_h):
    oh = np.asarray(outlet_h, dtype=float).reshape(-1, prm.N)
    return spectral.to_samples(oh.T[:, :], prm.K).T if oh.size else np.zeros((0, prm.N))


def residual_modal(om: OMesh, prm, Y, dirichlet, outlet_h, outlet_R=None,
                   opt: res.Options | None = None, rows=None) -> np.ndarray:
    y = samples_of(om, prm, Y, dirichlet)
    r = res.residual_samples(om, prm, y, h_samples(prm, outlet_h), outlet_R, H_of(prm), opt, rows)
    return spectral.to_modal(r, prm.K)


def jvp_modal(om: OMesh, prm, Y, V, dirichlet, outlet_h, outlet_R=None, kind: str = "exact",
              opt: res.Options | None = None, rows=None) -> np.ndarray:
    y = samples_of(om, prm, Y, dirichlet)
    v = spectral.to_samples(V, prm.K)
    if kind == "exact":
        jv = res.jvp_samples(om, prm, y, v, h_samples(prm, outlet_h), outlet_R, H_of(prm), opt,
                             rows=rows)
    elif kind == "paper":
        jv = paper_jvp_samples(om, prm, y, v)
    else:
        raise ValueError(kind)
    return spectral.to_modal(jv, prm.K)


def paper_jvp_samples(om: OMesh, prm, y, v, shift: float = 0.0) -> np.ndarray:
    """(C + P) v with Dirichlet velocity columns dropped and rows zeroed."""
    N = y.shape[1]
    A = tangent.assemble_paper_tangent(om, prm, y, H_of(prm), shift)
    mk = tangent.dirichlet_masks(om, N).ravel()
    vv = np.array(v, dtype=float).ravel()
    vv[mk] = 0.0
    out = A @ vv
    out[mk] = 0.0
    return out.reshape(y.shape)


def jacobi_samples(om: OMesh, prm, Y, dirichlet, shift: float = 0.0) -> np.ndarray:
    y = samples_of(om, prm, Y, dirichlet)
    return tangent.jacobi_diagonal(om, prm, y, shift)


def sample_norm(R_modal: np.ndarray, K: int) -> float:
    """2-norm of the time-sample residual recovered from modal rows."""
    return float(np.linalg.norm(spectral.to_samples(R_modal, K)))
