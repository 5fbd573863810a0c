"""Pins of the oracle's derivatives along a direction (rhs_tangent,
propagate_tangent), on the CPU:

* fourth-order central differences of the right-hand side and the dipole
  along a general direction (state, field and dipole-integral scale);
* the discrete Cauchy formula's result does not depend on its number of points
  once that exceeds the polynomial degree, and is linear in the direction;
* exact dynamics: for two electrons (o = 1, where CC is exact) the derivative of
  the Lagrangian dipole series with respect to a static field's amplitude
  equals that of the exact time-dependent Schroedinger equation in determinant
  space (central differences of exact exponential propagation);
* the derivative with respect to the dipole-integral scale equals central
  differences over models with scaled dipole matrices.
"""
import dataclasses
import itertools

import numpy as np
import scipy.linalg as sla
import torch

from fci_harness import FockSpace
from oracle import rtcc3 as orc
from paper_2407_18947_amd.inputs import field_delta_kick, initial_state, make_system, random_state

E0 = np.array([0.01, -0.02, 0.015])
EDOT = np.array([0.3, 0.1, -0.2])


def _setup(o, v, seed):
    s = make_system(o, v, seed=seed)
    return s, orc.Model.from_system(s)


def test_rhs_tangent_equals_fourth_order_differences():
    o, v = 2, 3
    s, m = _setup(o, v, 5)
    y = torch.tensor(random_state(o, v, 3, 0.1))
    yd = torch.tensor(random_state(o, v, 4, 0.1))
    kd = 0.7
    _, _, fd, md = orc.rhs_tangent(m, y, E0, yd, EDOT, kd)

    def g(h):
        f, mu = orc.rhs(m, y + h * yd, (1 + h * kd) * (E0 + h * EDOT), triples="explicit", with_dipole=True)
        return f, (1 + h * kd) * mu

    h = 1e-4
    (fp, mp), (fm, mm), (fp2, mp2), (fm2, mm2) = g(h), g(-h), g(2 * h), g(-2 * h)
    f4 = (8 * (fp - fm) - (fp2 - fm2)) / (12 * h)
    m4 = (8 * (mp - mm) - (mp2 - mm2)) / (12 * h)
    assert (fd - f4).abs().max() < 1e-10 * fd.abs().max()
    assert (md - m4).abs().max() < 1e-10 * md.abs().max()


def test_rhs_tangent_exact_in_the_number_of_points_and_linear():
    o, v = 2, 3
    s, m = _setup(o, v, 6)
    y = torch.tensor(random_state(o, v, 7, 0.1))
    d1 = torch.tensor(random_state(o, v, 8, 0.1))
    d2 = torch.tensor(random_state(o, v, 9, 0.1))
    _, _, a16, m16 = orc.rhs_tangent(m, y, E0, d1, EDOT, 0.0, npts=16)
    _, _, a20, m20 = orc.rhs_tangent(m, y, E0, d1, EDOT, 0.0, npts=20)
    assert (a16 - a20).abs().max() < 1e-13 * a16.abs().max()
    assert (m16 - m20).abs().max() < 1e-13 * m16.abs().max()
    _, _, b, mb = orc.rhs_tangent(m, y, E0, d2, 0 * EDOT, 0.0)
    _, _, c, mc = orc.rhs_tangent(m, y, E0, 2.0 * d1 - 3.0 * d2, 2.0 * EDOT, 0.0)
    assert (c - (2.0 * a16 - 3.0 * b)).abs().max() < 1e-12 * c.abs().max()
    assert (mc - (2.0 * m16 - 3.0 * mb)).abs().max() < 1e-12 * mc.abs().max()


def test_two_electron_amplitude_derivative_equals_exact_dynamics():
    """o = 1, v = 3, static field A e with A = 0.02 along e = (0.3, -0.5, 1): the
    derivative of the dipole series with respect to A (40 RK4 steps of 0.005)
    equals the derivative of the exact TDSE expectation value."""
    o, v = 1, 3
    s, m = _setup(o, v, 31)
    fs = FockSpace(o, v)
    rng = np.random.default_rng(12)
    t1 = 0.2 * (rng.normal(size=(o, v)) + 1j * rng.normal(size=(o, v)))
    t2 = 0.2 * (rng.normal(size=(o, o, v, v)) + 1j * rng.normal(size=(o, o, v, v)))
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    T0 = (fs.T1(t1) + fs.T2(t2)).toarray()
    psi0 = sla.expm(T0) @ fs.ref
    r = (psi0.conj() / (psi0.conj() @ psi0)) @ sla.expm(T0)  # <0|(1 + Lambda) from the exact bra
    l1 = np.array([[r @ (fs.E(o + a, i) @ fs.ref) for a in range(v)] for i in range(o)])
    l2 = np.zeros((o, o, v, v), complex)
    for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
        l2[i, j, a, b] = r @ (fs.E(o + a, i) @ (fs.E(o + b, j) @ fs.ref))
    y0 = orc.pack(*[torch.tensor(x) for x in (t1, t2, l1, l2)])
    e = np.array([0.3, -0.5, 1.0])
    A, dt, steps = 0.02, 0.005, 40
    f = np.tile(A * e, (2 * steps + 1, 1))
    fdot = np.tile(e, (2 * steps + 1, 1))
    _, _, mu, mud = orc.propagate_tangent(m, y0, dt, f, fdot)
    g = np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)
    M = [fs.one_body(s.mu[x].astype(complex)).toarray() for x in range(3)]

    def exact(Aval, n):
        H = fs.hamiltonian(m.h(Aval * e).numpy().astype(complex), g).toarray()
        psi = sla.expm(-1j * H * dt * n) @ psi0
        return np.array([(psi.conj() @ (Mx @ psi)) / (psi.conj() @ psi) for Mx in M])

    h = 1e-5
    for n in (10, 40):
        want = (exact(A + h, n) - exact(A - h, n)) / (2 * h)
        assert np.abs(mud[n].numpy() - want).max() < 1e-7 * np.abs(want).max(), n
        assert np.abs(mu[n].numpy() - exact(A, n)).max() < 1e-9


def test_dipole_scale_derivative_equals_scaled_models():
    o, v, steps, dt = 2, 3, 3, 0.05
    s, m = _setup(o, v, 14)
    y0 = initial_state(s)
    f = field_delta_kick(steps, dt, 0.002, "z")
    _, _, _, mud = orc.propagate_tangent(m, y0, dt, f, None, 1.0)
    h = 1e-5

    def run(scale):
        ms = orc.Model.from_system(dataclasses.replace(s, mu=s.mu * scale))
        return orc.propagate(ms, y0, dt, f, triples="explicit")[1]

    want = (run(1 + h) - run(1 - h)) / (2 * h)
    assert (mud - want).abs().max() < 1e-8 * want.abs().max()
