"""Pins of the oracle's one-electron operator, field coupling, dipole and
stationary states against determinant-space quantum mechanics
(tests/fci_harness.py), which shares no code with the oracle.

* h0: the closed-shell reference of H built from Model.h0 is canonical with
  orbital energies eps, checked through determinant-space matrix elements
  (Brillouin condition, reference energy, singles-singles block);
* V = -mu.E (Sec. 2.2.1): the Hamiltonian the oracle builds at field E is
  H0 - sum_x E_x mu_x with mu_x the one-body dipole operator;
* dipole (Sec. 2.2.3): Hellmann-Feynman, mu_x = -dL/dE_x at fixed amplitudes,
  for the CCSD Lagrangian and for the triples terms of the density; the
  reference determinant's dipole is 2 sum_i mu_ii;
* stationary amplitudes: for two electrons CC3 reduces to CCSD, which is
  exact, so the ground-state energy at every static field equals the
  full-CI one and the Lagrangian dipole equals the full-CI expectation value;
  with triples (o = 2), the stationary amplitudes stay put under RK4 at zero
  field and the dipole stays constant.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

from fci_harness import FockSpace
from oracle import rtcc3 as orc
from paper_2407_18947_amd.inputs import make_system


def _setup(o, v, seed):
    s = make_system(o, v, seed=seed)
    return s, orc.Model.from_system(s)


def _bare_g(s):
    return np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)


def _random_state(o, v, seed, scale=0.1):
    rng = np.random.default_rng(seed)

    def rc(*sh):
        return scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))

    t1, l1 = rc(o, v), rc(o, v)
    t2, l2 = rc(o, o, v, v), rc(o, o, v, v)
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    l2 = 0.5 * (l2 + l2.transpose(1, 0, 3, 2))
    return t1, t2, l1, l2


def _h0_hamiltonian(fs, s, m):
    return fs.hamiltonian(m.h0.numpy().astype(complex), _bare_g(s))


@pytest.mark.parametrize("o,v", [(1, 3), (2, 3)])
def test_reference_is_canonical_with_orbital_energies(o, v):
    """With H = sum h0 E + 1/2 sum (pq|rs)(EE - dE) the reference determinant has
    Fock matrix diag(eps): <0|H E_ai|0> = 2 f_ia = 0 (Brillouin), <0|H|0> =
    sum_i (h0_ii + eps_i), and the singles block <0|E_ia H E_bj|0> - 2 E0 d_ij d_ab
    = 2 [d_ij eps_a d_ab - d_ab eps_i d_ij + 2 (ai|jb) - (ab|ji)]."""
    s, m = _setup(o, v, seed=41)
    fs = FockSpace(o, v)
    H = _h0_hamiltonian(fs, s, m)
    ref = fs.ref
    E0 = (ref.conj() @ (H @ ref)).real
    h0 = m.h0.numpy()
    assert abs(E0 - sum(h0[i, i] + s.eps[i] for i in range(o))) < 1e-12
    g = _bare_g(s).real
    kets = {(j, b): fs.E(o + b, j) @ ref for j in range(o) for b in range(v)}
    Href = H @ ref
    for (i, a), k in kets.items():
        assert abs(k.conj() @ Href) < 1e-13, "Brillouin condition"
    for (i, a), ki in kets.items():
        Hk = None
        for (j, b), kj in kets.items():
            Hk = H @ kj
            got = ki.conj() @ Hk - 2.0 * E0 * (i == j) * (a == b)
            want = 2.0 * ((i == j) * (a == b) * (s.eps[o + a] - s.eps[i])
                          + 2.0 * g[o + a, i, j, o + b] - g[o + a, o + b, j, i])
            assert abs(got - want) < 1e-12, (i, a, j, b, got, want)


def test_field_coupling_is_minus_mu_dot_E():
    """The Hamiltonian at field E is H0 - sum_x E_x mu_x (V = -mu.E, Sec. 2.2.1),
    with mu_x = sum_pq mu^x_pq E_pq built in determinant space."""
    o, v = 2, 2
    s, m = _setup(o, v, seed=42)
    fs = FockSpace(o, v)
    E = np.array([0.013, -0.021, 0.034])
    H0 = _h0_hamiltonian(fs, s, m)
    want = H0 - sum(E[x] * fs.one_body(s.mu[x].astype(complex)) for x in range(3))
    got = fs.hamiltonian(m.h(E).numpy().astype(complex), _bare_g(s))
    assert abs(got - want).max() < 1e-13


def test_reference_determinant_dipole():
    """t = lambda = 0: the Lagrangian dipole is the reference's 2 sum_i mu^x_ii,
    with and without the triples terms (which vanish there)."""
    o, v = 3, 4
    s, m = _setup(o, v, seed=43)
    y = np.zeros(2 * (o * v + o * o * v * v), complex)
    want = 2.0 * np.array([np.trace(s.mu[x][:o, :o]) for x in range(3)])
    for tri in (False, True):
        mu = orc.dipole(m, y, [0.01, 0.0, -0.02], triples="explicit", with_triples=tri).numpy()
        assert np.abs(mu - want).max() < 1e-14


def _left_right(fs, t1, t2, l1, l2):
    T = fs.T1(t1) + fs.T2(t2)
    psi = fs.expm_apply(T, fs.ref)
    left = fs.expm_apply(T.T.tocsr(), fs.ref + fs.bra_from_lambda(l1, l2, orc.C2), sign=-1.0)
    return left, psi


def test_hellmann_feynman_ccsd():
    """At fixed (non-stationary) amplitudes, mu_x = -dL/dE_x for the CCSD Lagrangian
    <0|(1+Lambda) exp(-T) H(E) exp(T)|0> with H(E) = H0 - E.mu built in determinant
    space: central differences in a static E_x, and the oracle's own Lagrangian."""
    o, v = 2, 3
    s, m = _setup(o, v, seed=44)
    t1, t2, l1, l2 = _random_state(o, v, 6)
    y = orc.pack(*[torch.tensor(x) for x in (t1, t2, l1, l2)])
    fs = FockSpace(o, v)
    left, psi = _left_right(fs, t1, t2, l1, l2)
    H0 = _h0_hamiltonian(fs, s, m)
    M = [fs.one_body(s.mu[x].astype(complex)) for x in range(3)]
    E0 = np.array([0.004, -0.003, 0.002])
    mu = orc.dipole(m, y, E0, triples="explicit", with_triples=False).numpy()
    h = 1e-3
    for x in range(3):
        e = np.zeros(3)
        e[x] = h

        def lag_fci(E):
            return left @ ((H0 - sum(E[k] * M[k] for k in range(3))) @ psi)

        fd = (lag_fci(E0 + e) - lag_fci(E0 - e)) / (2 * h)
        assert abs(-fd - mu[x]) < 1e-9, (x, -fd, mu[x])
        fo = (orc.lagrangian(m, y, E0 + e, with_triples=False)
              - orc.lagrangian(m, y, E0 - e, with_triples=False)).item() / (2 * h)
        assert abs(-fo - mu[x]) < 1e-9, (x, -fo, mu[x])


def test_hellmann_feynman_triples_density():
    """The triples part of the dipole is -d/dE_x of the field terms of the CC3
    Lagrangian's triples block, <Lambda2|[V~,T3]|0> + <Lambda3|[V~,T3] +
    1/2 [[V~,T2],T2]|0> with V~ = exp(-T1) (-E.mu) exp(T1), T3|0> from the
    stationarity of the Lagrangian in Lambda3, <Lambda3| from its stationarity in
    T3 (both at V = 0), all in determinant space."""
    o, v = 2, 3
    s, m = _setup(o, v, seed=45)
    t1, t2, l1, l2 = _random_state(o, v, 7)
    y = orc.pack(*[torch.tensor(x) for x in (t1, t2, l1, l2)])
    E0 = np.array([0.0, 0.0, 0.0])
    fs = FockSpace(o, v)
    g = _bare_g(s)
    H0 = fs.hamiltonian(m.h0.numpy().astype(complex), g).toarray()
    T1m = fs.T1(t1).toarray()
    Hd = sla.expm(-T1m) @ H0 @ sla.expm(T1m)
    T2 = fs.T2(t2).toarray()
    ref = fs.ref
    den = fs.energy_denominators(s.eps)
    mask = fs.rank == 3
    comm = Hd @ (T2 @ ref) - T2 @ (Hd @ ref)
    t3s = np.zeros(fs.dim, complex)
    t3s[mask] = -comm[mask] / den[mask]
    bH = fs.bra_from_lambda(l1, l2, orc.C2) @ Hd
    l3b = np.zeros(fs.dim, complex)
    l3b[mask] = -bH[mask] / den[mask]
    b2 = fs.bra_from_lambda(0 * l1, l2, orc.C2)
    mu_tri = (orc.dipole(m, y, E0, triples="explicit", with_triples=True)
              - orc.dipole(m, y, E0, triples="explicit", with_triples=False)).numpy()
    for x in range(3):
        Mt = sla.expm(-T1m) @ fs.one_body(s.mu[x].astype(complex)).toarray() @ sla.expm(T1m)

        def lag_tri(e):
            V = -e * Mt
            v0 = ref.conj() @ (V @ ref)
            val = b2 @ (V @ t3s) + l3b @ (V @ t3s) - v0 * (l3b @ t3s)
            dd = V @ (T2 @ (T2 @ ref)) - 2 * (T2 @ (V @ (T2 @ ref))) + T2 @ (T2 @ (V @ ref))
            return val + 0.5 * (l3b @ dd)

        h = 1e-3
        fd = (lag_tri(h) - lag_tri(-h)) / (2 * h)
        assert abs(-fd - mu_tri[x]) < 1e-12, (x, -fd, mu_tri[x])
    assert np.abs(mu_tri).max() > 1e-6  # the test compares a non-trivial quantity


def _fci_ground(fs, H):
    w, U = np.linalg.eigh(H)
    k = int(np.argmax(np.abs(U.T.conj() @ fs.ref)))
    return w[k], U[:, k]


def test_two_electron_ground_state_is_full_ci():
    """o = 1: the triples vanish and CCSD is exact, so the oracle's stationary
    amplitudes give the full-CI ground-state energy at every static field, the
    Lagrangian dipole is the full-CI expectation value, and the four-point
    finite-field polarisability (Sec. 2.2.2) agrees."""
    o, v = 1, 3
    s, m = _setup(o, v, seed=46)
    fs = FockSpace(o, v)
    H0 = _h0_hamiltonian(fs, s, m).toarray()
    Mz = fs.one_body(s.mu[2].astype(complex)).toarray()
    A = 0.002
    e_cc, e_fci = {}, {}
    for k in (-2, -1, 0, 1, 2):
        F = np.array([0.0, 0.0, k * A])
        y, e = orc.ground_state(m, F, lam=(k == 0))
        w, psi = _fci_ground(fs, H0 - F[2] * Mz)
        e_cc[k], e_fci[k] = e.real, w
        assert abs(e.real - w) < 1e-10 and abs(e.imag) < 1e-12, (k, e, w)
        if k == 0:
            mu = orc.dipole(m, y, F, triples="explicit").numpy()
            want = (psi.conj() @ (Mz @ psi)).real
            assert abs(mu[2] - want) < 1e-9, (mu[2], want)

    def alpha(e):
        return -(-e[2] + 16 * e[1] - 30 * e[0] + 16 * e[-1] - e[-2]) / (12 * A * A)

    assert abs(alpha(e_cc) - alpha(e_fci)) < 1e-4 * abs(alpha(e_fci))
    assert alpha(e_fci) > 0
    # Hellmann-Feynman on the exact energies: <mu_z> = -dE/dF_z
    mu_fd = -(e_fci[-2] - 8 * e_fci[-1] + 8 * e_fci[1] - e_fci[2]) / (12 * A)
    y0, _ = orc.ground_state(m, [0, 0, 0])
    assert abs(orc.dipole(m, y0, [0, 0, 0], triples="explicit").numpy()[2].real - mu_fd) < 1e-8


def test_ground_state_is_stationary_with_triples():
    """o = 2, v = 3, CC3 with triples: the stationary amplitudes at zero field do
    not move under 20 RK4 steps (dt = 0.05), and the dipole and the Lagrangian
    stay constant."""
    o, v = 2, 3
    s, m = _setup(o, v, seed=47)
    y0, e0 = orc.ground_state(m)
    dy = orc.rhs(m, y0, [0, 0, 0], triples="explicit")
    assert dy.abs().max() < 1e-11
    steps = 20
    yf, mu = orc.propagate(m, y0, 0.05, np.zeros((2 * steps + 1, 3)), triples="explicit")
    assert (yf - y0).abs().max() < 1e-10
    assert (mu - mu[0]).abs().max() < 1e-10
    assert abs(orc.lagrangian(m, yf, [0, 0, 0]) - orc.lagrangian(m, y0, [0, 0, 0])) < 1e-10
    # the stationary T amplitudes have non-trivial triples
    t1, t2, l1, l2 = orc.unpack(m, y0)
    ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h([0, 0, 0])))
    assert orc.t3_full(m, ti, t2).abs().max() > 1e-5
