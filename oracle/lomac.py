"""Adaptive-weight LoMaC projection, reconstruction and correction (oracle).

Supplement B:
  * discrete weight: omega^(mu) = max(|u_1^(mu)|, delta), u_1^(mu) the first
    left singular vector of the mode-v_mu matricisation of F* (equal to
    column 0 of the v_mu leaf after the truncation), Omega* = (x)_mu omega^(mu)
    (eq. (omega_star_tensor));
  * 1D weighted inner product <p,q>_mu = sum_k p_k q_k w_k / omega_k with
    w_k = Delta v_mu; Gram--Schmidt quantities gamma_mu, q1, eta_mu, beta_mu,
    q2 (section "Weighted Gram--Schmidt construction");
  * Q_0 = Omega*, Q_{1,mu} = ... (x) q1^(mu) (x) ..., Q_2 = sum_mu ... (x)
    q2^(mu) (x) ...; squared norms as products of 1D norms;
  * coefficients eqs. (C0_def)-(C2_def) from the raw moments;
  * reconstruction eq. (reconstruction_supp) from conserved variables via
    eq. (raw_from_conserved_supp);
  * correction eq. (LoMaC_update_discrete):
      F^{n+1} = F* - R(U(F*)) + R(U^{n+1}) = F* + sum_k dC_k (x) Q_k.

The floor parameter delta is not given a value in the paper; 1e-12 is used
(absolute, on the unit-norm u_1).  Moment preservation holds for any
delta > 0.
"""
from __future__ import annotations

import numpy as np

from . import spectral as SP

DELTA = 1e-12


def weight_1d(u1: np.ndarray, delta: float = DELTA) -> np.ndarray:
    return np.maximum(np.abs(u1), delta)


def gram_schmidt_1d(omega: np.ndarray, v: np.ndarray, h: float) -> dict:
    w = np.full_like(omega, h)

    def ip(p, q):
        return float(np.sum(p * q * w / omega))

    vo = v * omega
    v2o = v * v * omega
    n0 = ip(omega, omega)
    gamma = ip(vo, omega) / n0
    q1 = vo - gamma * omega
    eta = ip(v2o, omega) / n0
    n1 = ip(q1, q1)
    beta = ip(v2o, q1) / n1
    q2 = v2o - eta * omega - beta * q1
    n2 = ip(q2, q2)
    return {"omega": omega, "q1": q1, "q2": q2, "gamma": gamma, "eta": eta,
            "beta": beta, "n0": n0, "n1": n1, "n2": n2}


def _outer(vecs):
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out


def basis(u1_list, vgrids, hs, delta: float = DELTA) -> dict:
    """All 1D quantities, dense Q_k (K = dv+2) and their squared norms."""
    dv = len(u1_list)
    gs = [gram_schmidt_1d(weight_1d(u1_list[m], delta), vgrids[m], hs[m]) for m in range(dv)]
    om = [g["omega"] for g in gs]
    Q = [_outer(om)]
    NQ = [float(np.prod([g["n0"] for g in gs]))]
    for m in range(dv):
        vecs = list(om)
        vecs[m] = gs[m]["q1"]
        Q.append(_outer(vecs))
        NQ.append(gs[m]["n1"] * float(np.prod([gs[n]["n0"] for n in range(dv) if n != m])))
    Q2 = 0.0
    n2 = 0.0
    for m in range(dv):
        vecs = list(om)
        vecs[m] = gs[m]["q2"]
        Q2 = Q2 + _outer(vecs)
        n2 += gs[m]["n2"] * float(np.prod([gs[n]["n0"] for n in range(dv) if n != m]))
    Q.append(Q2)
    NQ.append(n2)
    return {"g": gs, "Q": np.stack(Q), "NQ": np.array(NQ), "dv": dv}


def coefficients(Mraw: np.ndarray, B: dict) -> np.ndarray:
    """Eqs. (C0_def)-(C2_def).  Mraw = (M0, M1_1..M1_dv, M2) on the x-grid."""
    dv = B["dv"]
    g = B["g"]
    M0 = Mraw[0]
    M2 = Mraw[dv + 1]
    C = [M0 / B["NQ"][0]]
    for m in range(dv):
        C.append((Mraw[1 + m] - g[m]["gamma"] * M0) / B["NQ"][1 + m])
    num = M2 - sum(g[m]["eta"] for m in range(dv)) * M0
    for m in range(dv):
        num = num - g[m]["beta"] * (Mraw[1 + m] - g[m]["gamma"] * M0)
    C.append(num / B["NQ"][dv + 1])
    return np.stack(C)


def e_p_of(U0: np.ndarray, n_i: float, lengths) -> np.ndarray:
    _, E = SP.poisson(U0, n_i, lengths)
    return SP.field_energy_density(E)


def raw_from_conserved(U: np.ndarray, n_i: float, lengths) -> np.ndarray:
    """Eq. (M from U) with m_e = 1: M0 = U0, M1 = U1, M2 = 2 (U2 - e_p(U0))."""
    dv = U.shape[0] - 2
    M = U.copy()
    M[dv + 1] = 2.0 * (U[dv + 1] - e_p_of(U[0], n_i, lengths))
    return M


def conserved_from_raw(Mraw: np.ndarray, n_i: float, lengths) -> np.ndarray:
    """U = (n, m n u, e_k + e_p) with e_k = M2/2 (eq. (physical_moments))."""
    dv = Mraw.shape[0] - 2
    U = Mraw[: dv + 2].copy()
    U[dv + 1] = 0.5 * Mraw[dv + 1] + e_p_of(Mraw[0], n_i, lengths)
    return U


def expand(C: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """sum_k C_k (x) Q_k as a dense phase-space tensor."""
    return np.tensordot(C, Q, axes=([0], [0]))


def project_dense(Ffull: np.ndarray, dx: int, B: dict, vgrids, dvol: float) -> np.ndarray:
    """P* F via eq. (phase_proj_closed), for a dense F (pins)."""
    dv = B["dv"]
    Vs = np.meshgrid(*vgrids, indexing="ij")
    ax = tuple(range(dx, Ffull.ndim))
    M = [np.sum(Ffull, axis=ax) * dvol]
    M += [np.sum(Ffull * Vs[m], axis=ax) * dvol for m in range(dv)]
    M.append(np.sum(Ffull * sum(V * V for V in Vs), axis=ax) * dvol)
    return expand(coefficients(np.stack(M), B), B["Q"])


def mode_filter(n: int) -> np.ndarray:
    """sigma(m) = exp(-36 kappa^8), kappa = |m| / (n / 2), for the FFT mode
    indices 0..n-1 of an axis of n cells (|m| the distance to mode 0)."""
    i = np.arange(n)
    kap = np.minimum(i, n - i) / (0.5 * n)
    return np.exp(-36.0 * kap ** 8)


def filter_correction(U: np.ndarray, U0: np.ndarray) -> np.ndarray:
    """Band-limited correction (a stabilisation of this implementation, not
    in the paper): U0 + sigma (U - U0) per component, sigma the tensor
    product of ``mode_filter`` over the x axes.  Mode 0 has sigma = 1, so
    the totals of U are kept."""
    d = U - U0
    axes = tuple(range(1, U.ndim))
    sig = 1.0
    for a in axes:
        shape = [1] * U.ndim
        shape[a] = U.shape[a]
        sig = sig * mode_filter(U.shape[a]).reshape(shape)
    return U0 + np.real(np.fft.ifftn(sig * np.fft.fftn(d, axes=axes), axes=axes))


def velocity_integrals(B: dict, psis, dvol: float) -> np.ndarray:
    """<psi, Q_k> = sum_v psi Q_k w^v for each psi: shape (npsi, K)."""
    Q = B["Q"]
    ax = list(range(1, Q.ndim))
    return np.stack([np.tensordot(Q, p, axes=(ax, list(range(p.ndim)))) * dvol for p in psis])
