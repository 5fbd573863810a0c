"""Optical properties from real-time dipole trajectories (host-side post-processing).

The propagation itself runs in the library; this module turns the dipole time
series it returns into the paper's observables (Sec. 2.2):

* absorption spectra: alpha_bb(w) = mu~_b(w) / E~_b(w) with the Fourier
  transform f~(w) = (1/2 pi) int f(t) exp(i w t) dt, and the dipole strength
  I(w) ~ Im sum_b alpha_bb(w) (Sec. 2.2.1); the transforms either as sums over
  the samples or through Pade approximants of the sampled series (Sec. 3);
* four-point central finite differences over field amplitudes A, -A, 2A, -2A
  for the first- and second-order dipoles mu^(1)(t), mu^(2)(t) (Sec. 2.2.2);
* alpha(w) as the amplitude of mu^(1)(t) = alpha cos(w t) (eq. cc3-polar-alpha)
  and beta(-2w; w, w), beta(0; w, -w) from mu^(2)(t) = 1/4 [beta_SHG cos(2 w t)
  + beta_OR] (eq. cc3-polar-beta), each by least squares over the part of the
  trajectory after the ramp, with the coefficient of determination R^2.

Plain numpy; nothing here is on the propagation's path.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "finite_field_mu1",
    "finite_field_mu2",
    "fit_alpha",
    "fit_beta",
    "fourier",
    "pade_fourier",
    "absorption_spectrum",
]


def finite_field_mu1(mu_p1, mu_m1, mu_p2, mu_m2, A):
    """mu^(1)(t) = {8 [mu(A) - mu(-A)] - [mu(2A) - mu(-2A)]} / (12 A) (Sec. 2.2.2).
    Exact for a dipole polynomial in A up to fourth order."""
    mu_p1, mu_m1, mu_p2, mu_m2 = (np.asarray(x) for x in (mu_p1, mu_m1, mu_p2, mu_m2))
    return (8.0 * (mu_p1 - mu_m1) - (mu_p2 - mu_m2)) / (12.0 * A)


def finite_field_mu2(mu_p1, mu_m1, mu_p2, mu_m2, mu0, A):
    """mu^(2)(t) = {16 [mu(A) + mu(-A)] - [mu(2A) + mu(-2A)] - 30 mu^(0)} / (24 A^2)
    (Sec. 2.2.2).  Exact for a dipole polynomial in A up to fifth order."""
    mu_p1, mu_m1, mu_p2, mu_m2, mu0 = (np.asarray(x) for x in (mu_p1, mu_m1, mu_p2, mu_m2, mu0))
    return (16.0 * (mu_p1 + mu_m1) - (mu_p2 + mu_m2) - 30.0 * mu0) / (24.0 * A * A)


def _lstsq_fit(t, y, columns):
    X = np.stack(columns, axis=1)
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    res = y - X @ coef
    ss_tot = np.sum((y - y.mean()) ** 2)
    r2 = 1.0 - np.sum(res ** 2) / ss_tot if ss_tot > 0 else (1.0 if np.allclose(res, 0) else 0.0)
    return coef, float(r2)


def _window(t, y, t_start, t_end):
    t = np.asarray(t, dtype=np.float64)
    y = np.real(np.asarray(y))
    m = (t >= t_start) & (t <= (np.inf if t_end is None else t_end))
    if m.sum() < 3:
        raise ValueError("fewer than three samples in the fitting window")
    return t[m], y[m]


def fit_alpha(t, mu1, omega, t_start=0.0, t_end=None):
    """alpha(w): least-squares amplitude of mu^(1)(t) = alpha cos(w t) over
    t_start <= t <= t_end (eq. cc3-polar-alpha).  Returns (alpha, R^2)."""
    tt, y = _window(t, mu1, t_start, t_end)
    (a,), r2 = _lstsq_fit(tt, y, [np.cos(omega * tt)])
    return float(a), r2


def fit_beta(t, mu2, omega, t_start=0.0, t_end=None):
    """beta(-2w; w, w) and beta(0; w, -w): least squares of mu^(2)(t) =
    1/4 [beta_SHG cos(2 w t) + beta_OR] (eq. cc3-polar-beta).  Returns
    (beta_SHG, beta_OR, R^2)."""
    tt, y = _window(t, mu2, t_start, t_end)
    (a, b), r2 = _lstsq_fit(tt, y, [0.25 * np.cos(2.0 * omega * tt), 0.25 * np.ones_like(tt)])
    return float(a), float(b), r2


def fourier(f, dt, omegas, damping=0.0):
    """f~(w) = (1/2 pi) int f(t) exp(i w t) dt for samples f[n] = f(n dt), n = 0..N-1,
    by the trapezoidal rule, optionally with an exp(-damping t) window."""
    f = np.asarray(f, dtype=np.complex128)
    t = dt * np.arange(len(f))
    w = np.full(len(f), dt)
    w[0] = w[-1] = 0.5 * dt
    g = f * w * np.exp(-damping * t)
    return np.exp(1j * np.outer(np.asarray(omegas, dtype=np.float64), t)) @ g / (2.0 * np.pi)


def pade_fourier(f, dt, omegas, damping=0.0):
    """Fourier transform of the sampled series through a diagonal Pade
    approximant of its z-transform (Bruner, LaMaster and Lopata, J. Chem. Theory
    Comput. 2016).  With z = exp(i w dt), X(z) = sum_n f[n] z^n is replaced by
    P(z) / Q(z) of degrees M, M (N = 2M + 1 samples used), whose coefficients
    match the series through order 2M:
      sum_{k=0..M} b_k f[m - k] = 0 for m = M+1..2M  (b_0 = 1),
      a_m = sum_{k=0..m} b_k f[m - k] for m = 0..M.
    Returns dt / (2 pi) * P/Q at each w (the rectangle-rule transform that the
    series stands for, extrapolated beyond the sampled time)."""
    f = np.asarray(f, dtype=np.complex128) * np.exp(-damping * dt * np.arange(len(f)))
    M = (len(f) - 1) // 2
    if M < 1:
        raise ValueError("need at least three samples")
    f = f[: 2 * M + 1]
    # Toeplitz system for b_1..b_M: sum_k b_k f[M + m - k] = -f[M + m], m = 1..M
    G = np.array([[f[M + m - k] for k in range(1, M + 1)] for m in range(1, M + 1)])
    b = np.concatenate([[1.0], np.linalg.solve(G, -f[M + 1: 2 * M + 1])])
    a = np.array([np.dot(b[: m + 1], f[m::-1][: m + 1]) for m in range(M + 1)])
    z = np.exp(1j * np.asarray(omegas, dtype=np.float64) * dt)
    P = np.polyval(a[::-1], z)
    Q = np.polyval(b[::-1], z)
    return dt / (2.0 * np.pi) * P / Q


def absorption_spectrum(mu, field, dt, omegas, damping=0.0, method="fourier"):
    """alpha_bb(w) = mu~_b(w) / E~_b(w) for the axes b whose field is non-zero, and
    the dipole strength S(w) = Im sum_b alpha_bb(w) (Sec. 2.2.1).

    mu[n, b], field[n, b]: dipole (induced part taken against mu[0]) and field on
    a uniform grid of spacing dt.  Returns (S, alpha[b]) with alpha a dict."""
    mu = np.asarray(mu)
    field = np.asarray(field, dtype=np.float64)
    tf = {"fourier": fourier, "pade": pade_fourier}[method]
    alpha = {}
    for b in range(field.shape[1]):
        if not np.any(field[:, b]):
            continue
        num = tf(mu[:, b] - mu[0, b], dt, omegas, damping)
        den = fourier(field[:, b], dt, omegas, 0.0)
        alpha[b] = num / den
    S = np.imag(sum(alpha.values())) if alpha else np.zeros(len(omegas))
    return S, alpha
