"""Pins of the property post-processing (paper_2407_18947_amd/properties.py) and
of the ramped-wave fields, against exact algebra and exact quantum dynamics:

* the four-point finite-field formulas are exact for dipoles polynomial in the
  amplitude (to fourth order for mu^(1), fifth for mu^(2));
* the cosine fits recover alpha and beta_SHG / beta_OR of synthetic
  trajectories exactly (R^2 = 1);
* the QRCW envelope and its slope are continuous (Sec. 2.2.4);
* the Pade transform is exact for a sum of damped exponentials whose number
  does not exceed its degree; the sample-sum transform of a Gaussian matches the
  analytic transform;
* the dipole strength of a damped two-level response peaks at its frequency;
* end to end: alpha(w) from exact time propagation (determinant space, two
  electrons) under QRCW fields of +-A, +-2A agrees with the sum-over-states
  polarisability of the same Hamiltonian.
"""
import numpy as np
import pytest

from fci_harness import FockSpace
from oracle import rtcc3 as orc
from paper_2407_18947_amd import properties as P
from paper_2407_18947_amd.inputs import field_ramped_cw, make_system, ramp_lrcw, ramp_qrcw


def test_finite_field_formulas_exact_on_polynomials():
    rng = np.random.default_rng(0)
    t = np.linspace(0, 10, 50)
    c = [rng.normal(size=t.size) for _ in range(6)]  # mu(t, A) = sum_k c_k(t) A^k

    def mu(A, kmax):
        return sum(c[k] * A ** k for k in range(kmax + 1))

    A = 0.003
    m1 = P.finite_field_mu1(mu(A, 4), mu(-A, 4), mu(2 * A, 4), mu(-2 * A, 4), A)
    assert np.abs(m1 - c[1]).max() < 1e-10
    m2 = P.finite_field_mu2(mu(A, 5), mu(-A, 5), mu(2 * A, 5), mu(-2 * A, 5), mu(0, 5), A)
    assert np.abs(m2 - c[2]).max() < 1e-6
    # a fifth-order term leaves mu^(1) an error of order A^4
    m1b = P.finite_field_mu1(mu(A, 5), mu(-A, 5), mu(2 * A, 5), mu(-2 * A, 5), A)
    assert np.abs(m1b - c[1]).max() > 0


def test_cosine_fits_recover_alpha_and_beta():
    w = 0.0656
    t = np.linspace(0, 2 * 2 * np.pi / w, 4001)
    t_r = 2 * np.pi / w
    alpha, b_shg, b_or = 7.31, -19.5, 4.25
    mu1 = alpha * np.cos(w * t)
    mu1[t < t_r] += 3.0 * np.exp(-t[t < t_r])  # transient inside the ramp, outside the window
    a, r2 = P.fit_alpha(t, mu1, w, t_start=t_r)
    assert abs(a - alpha) < 1e-12 and abs(r2 - 1) < 1e-14
    mu2 = 0.25 * (b_shg * np.cos(2 * w * t) + b_or)
    s, o, r2 = P.fit_beta(t, mu2, w, t_start=t_r)
    assert abs(s - b_shg) < 1e-11 and abs(o - b_or) < 1e-11 and abs(r2 - 1) < 1e-14
    # noise lowers R^2 below one
    a, r2 = P.fit_alpha(t, mu1 + 0.5 * np.sin(3.3 * t), w, t_start=t_r)
    assert r2 < 0.999


def test_ramped_wave_envelopes():
    t_r = 10.0
    t = np.linspace(0, 20, 20001)
    q = ramp_qrcw(t, t_r)
    assert q[0] == 0 and np.all(q[t >= t_r] == 1)
    assert abs(ramp_qrcw(0.5 * t_r, t_r) - 0.5) < 1e-15
    # value and slope continuous (the QRCW is smooth, Sec. 2.2.4)
    eps = 1e-7
    for tc in (0.5 * t_r, t_r):
        assert abs(ramp_qrcw(tc - eps, t_r) - ramp_qrcw(tc + eps, t_r)) < 1e-6
        dl = (ramp_qrcw(tc - eps, t_r) - ramp_qrcw(tc - 2 * eps, t_r)) / eps
        dr = (ramp_qrcw(tc + 2 * eps, t_r) - ramp_qrcw(tc + eps, t_r)) / eps
        assert abs(dl - dr) < 1e-5
    lr = ramp_lrcw(t, t_r)
    assert abs(ramp_lrcw(2.5, t_r) - 0.25) < 1e-15 and np.all(lr[t >= t_r] == 1)
    w, A, dt = 0.5, 0.002, 0.05
    f = field_ramped_cw(400, dt, A, w, kind="qrcw", n_r=1, direction="y")
    tt = 0.5 * dt * np.arange(801)
    full = tt >= 2 * np.pi / w
    assert np.abs(f[full, 1] - A * np.cos(w * tt[full])).max() < 1e-15
    assert np.all(f[:, 0] == 0) and np.all(f[:, 2] == 0)


def test_pade_exact_for_damped_exponentials():
    dt = 0.1
    n = np.arange(61)
    r = [0.97 * np.exp(0.31j), 0.9 * np.exp(-0.74j), 0.99 * np.exp(1.4j)]
    c = [1.0, 0.5j, -0.3]
    x = sum(ci * ri ** n for ci, ri in zip(c, r))
    w = np.linspace(-20, 20, 41)
    exact = dt / (2 * np.pi) * sum(ci / (1 - ri * np.exp(1j * w * dt)) for ci, ri in zip(c, r))
    assert np.abs(P.pade_fourier(x[:7], dt, w) - exact).max() < 1e-13
    assert np.abs(P.pade_fourier(x, dt, w) - exact).max() < 1e-9


def test_fourier_of_gaussian():
    dt, s, t0 = 0.01, 0.7, 5.0
    t = dt * np.arange(1001)
    f = np.exp(-((t - t0) ** 2) / (2 * s * s))
    w = np.linspace(-4, 4, 17)
    exact = s / np.sqrt(2 * np.pi) * np.exp(1j * w * t0 - 0.5 * (w * s) ** 2)
    assert np.abs(P.fourier(f, dt, w) - exact).max() < 1e-12


@pytest.mark.parametrize("method", ["fourier", "pade"])
def test_absorption_spectrum_peaks_at_transition(method):
    """Kicked damped two-level response mu(t) = d^2 E0 dt sin(w0 t) exp(-g t): the
    dipole strength peaks at w0."""
    w0, g, dt, steps = 0.8, 0.02, 0.05, 4000
    t = dt * np.arange(steps)
    field = np.zeros((steps, 3))
    field[0, 2] = 1.0 / dt * 2  # a kick of area 1 under the trapezoidal rule
    mu = np.zeros((steps, 3), complex)
    mu[:, 2] = 0.1 + np.sin(w0 * t) * np.exp(-g * t)
    w = np.linspace(0.3, 1.3, 1001)
    S, alpha = P.absorption_spectrum(mu, field, dt, w, damping=0.0, method=method)
    assert list(alpha) == [2]
    assert abs(w[np.argmax(S)] - w0) < 2e-3


def _tdse_dipoles(H0, M, psi0, dt, fields):
    """Exact propagation with the field at each step's midpoint; mu(t_n) = <psi|M|psi>."""
    out = []
    for f in fields:
        psi = psi0.copy()
        mus = [np.real(psi.conj() @ (M @ psi))]
        for n in range((len(f) - 1) // 2):
            w, V = np.linalg.eigh(H0 - f[2 * n + 1] * M)  # exp(-i dt H) through the eigenbasis
            psi = V @ (np.exp(-1j * dt * w) * (V.conj().T @ psi))
            mus.append(np.real(psi.conj() @ (M @ psi)))
        out.append(np.array(mus))
    return out


def test_dynamic_polarisability_from_ramped_waves_matches_sum_over_states():
    """alpha_zz(w) of a two-electron system (o = 1, v = 3) from exact time
    propagation under QRCW fields of +-A, +-2A (one ramped and one fitted cycle,
    the paper's default), against sum_n 2 w_n |<0|mu_z|n>|^2 / (w_n^2 - w^2)."""
    o, v = 1, 3
    s = make_system(o, v, seed=46)
    m = orc.Model.from_system(s)
    fs = FockSpace(o, v)
    g = np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)
    H0 = fs.hamiltonian(m.h0.numpy().astype(complex), g).toarray()
    M = fs.one_body(s.mu[2].astype(complex)).toarray()
    E, U = np.linalg.eigh(H0)
    k0 = int(np.argmax(np.abs(U.T.conj() @ fs.ref)))
    psi0 = U[:, k0]
    wn = E - E[k0]
    dn = U.T.conj() @ (M @ psi0)
    w = 0.3
    exc = np.arange(len(E)) != k0
    alpha_sos = np.sum(2 * wn[exc] * np.abs(dn[exc]) ** 2 / (wn[exc] ** 2 - w * w))
    dt, A = 0.02, 0.001
    t_c = 2 * np.pi / w
    steps = int(round(2 * t_c / dt))
    fields = [field_ramped_cw(steps, dt, k * A, w, kind="qrcw", n_r=1)[:, 2] for k in (1, -1, 2, -2)]
    mu_p1, mu_m1, mu_p2, mu_m2 = _tdse_dipoles(H0, M, psi0, dt, fields)
    mu1 = P.finite_field_mu1(mu_p1, mu_m1, mu_p2, mu_m2, A)
    t = dt * np.arange(steps + 1)
    alpha, r2 = P.fit_alpha(t, mu1, w, t_start=t_c)
    assert r2 > 0.999
    assert abs(alpha - alpha_sos) < 1e-3 * abs(alpha_sos), (alpha, alpha_sos)
