"""Spectral Poisson solve and derivatives on the periodic x-grid (oracle).

Eqs. (Poisson), (Efromphi): -Laplace(phi) = rho (eps_0 = 1), E = -grad phi.
Section 3.2.3: E, the field-energy flux and the auxiliary Poisson problem
for d_t phi are all evaluated with FFT-based spectral differentiation so the
discrete gradient, divergence and Laplacian are algebraically compatible.

Reading of that compatibility: the first-derivative symbol is i k with the
Nyquist wavenumber set to 0 (so it is a real, skew operator), the Laplacian
is the composition D.D, and the Poisson solve applies its pseudo-inverse
(zero on the modes where the symbol vanishes).  This gives
sum_x rho E = 0 and sum_x D.F = 0 exactly in exact arithmetic.
The conservative flux difference of the macroscopic update (deferred by the
paper to earlier work) is the same spectral divergence.
"""
from __future__ import annotations

import math

import numpy as np


def wavenumbers(n: int, L: float) -> np.ndarray:
    k = np.fft.fftfreq(n, d=1.0 / n) * (2.0 * math.pi / L)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def _kgrid(shape, lengths):
    ks = [wavenumbers(n, L) for n, L in zip(shape, lengths)]
    return np.meshgrid(*ks, indexing="ij")


def deriv(f: np.ndarray, axis: int, lengths) -> np.ndarray:
    K = _kgrid(f.shape, lengths)
    return np.real(np.fft.ifftn(1j * K[axis] * np.fft.fftn(f)))


def div(F: np.ndarray, lengths) -> np.ndarray:
    """F has shape (dx, N...)."""
    return sum(deriv(F[m], m, lengths) for m in range(F.shape[0]))


def grad(f: np.ndarray, lengths) -> np.ndarray:
    return np.stack([deriv(f, m, lengths) for m in range(f.ndim)])


def inv_neg_laplace(rho: np.ndarray, lengths) -> np.ndarray:
    """phi with -D.D phi = rho on the non-null modes, 0 on the null ones."""
    K = _kgrid(rho.shape, lengths)
    k2 = sum(k * k for k in K)
    rh = np.fft.fftn(rho)
    ph = np.zeros_like(rh)
    nz = k2 > 0
    ph[nz] = rh[nz] / k2[nz]
    return np.real(np.fft.ifftn(ph))


def poisson(n_e: np.ndarray, n_i: float, lengths):
    """rho = q_i n_i + q_e n_e = n_i - n_e  ->  (phi, E)  (eq. (charge_density))."""
    rho = n_i - n_e
    phi = inv_neg_laplace(rho, lengths)
    E = -grad(phi, lengths)
    return phi, E


def field_energy_density(E: np.ndarray) -> np.ndarray:
    """e_p = (eps_0/2)|E|^2 (section 2.2)."""
    return 0.5 * np.sum(E * E, axis=0)
