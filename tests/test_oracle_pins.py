"""Pins of the CPU oracle against things other than itself.

* a determinant-space (second-quantized) construction of exp(-T) H exp(T),
  of the triples state and of bra-ket densities (tests/fci_harness.py);
* Lagrangian derivatives by automatic differentiation, checked themselves by
  finite differences;
* exact results: the triples vanish for two electrons, the P(ijk/abc)
  symmetry of t3, conservation of the Lagrangian at zero field, RK4
  time-reversal, and exact two-electron dynamics against the TDSE.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from fci_harness import FockSpace, dress_integrals
from oracle import rtcc3 as orc
from paper_2407_18947_amd.inputs import initial_state, make_system

FIELD = np.array([0.01, -0.02, 0.03])


def _random_state(o, v, seed, scale=0.1):
    rng = np.random.default_rng(seed)

    def rc(*sh):
        return scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))

    t1, l1 = rc(o, v), rc(o, v)
    t2, l2 = rc(o, o, v, v), rc(o, o, v, v)
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    l2 = 0.5 * (l2 + l2.transpose(1, 0, 3, 2))
    return t1, t2, l1, l2


def _setup(o, v, seed=11):
    s = make_system(o, v, seed=seed)
    return s, orc.Model.from_system(s)


def _bare_g(s):
    return np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)


@pytest.mark.parametrize("o,v", [(2, 2), (2, 3)])
def test_dressing_is_similarity_transform(o, v):
    s, m = _setup(o, v)
    t1, *_ = _random_state(o, v, 3)
    fs = FockSpace(o, v)
    h = m.h(FIELD).numpy().astype(complex)
    H = fs.hamiltonian(h, _bare_g(s)).toarray()
    T1 = fs.T1(t1).toarray()
    ref = sla.expm(-T1) @ H @ sla.expm(T1)
    d = orc.Dressed(m, torch.tensor(t1), m.h(FIELD))
    gt = torch.einsum("Ppq,Prs->pqrs", d.B, d.B).numpy()
    Hd = fs.hamiltonian(d.h.numpy(), gt).toarray()
    assert np.abs(Hd - ref).max() < 1e-13


@pytest.mark.parametrize("o,v", [(1, 3), (2, 3), (3, 3)])
def test_ccsd_residual_is_projection(o, v):
    s, m = _setup(o, v)
    t1, t2, _, _ = _random_state(o, v, 3)
    fs = FockSpace(o, v)
    H = fs.hamiltonian(m.h(FIELD).numpy().astype(complex), _bare_g(s))
    T = fs.T1(t1) + fs.T2(t2)
    hbar = fs.expm_apply(T, H @ fs.expm_apply(T, fs.ref), sign=-1.0)
    w1, w2 = fs.coefficients(hbar)
    d = orc.Dressed(m, torch.tensor(t1), m.h(FIELD))
    r1, r2 = orc.ccsd_omega(d, torch.tensor(t2))
    assert np.abs(r1.numpy() - w1).max() < 1e-12
    assert np.abs(r2.numpy() - w2).max() < 1e-12
    e = orc.ccsd_energy(d, torch.tensor(t2)).item()
    assert abs(e - hbar @ fs.ref) < 1e-12


def _harness_triples(fs, s, m, t1, t2):
    o, v = fs.o, fs.v
    h = m.h(FIELD).numpy().astype(complex)
    ht, gt = dress_integrals(o, v, t1, h, s.B)
    Hd = fs.hamiltonian(ht, gt)
    T2 = fs.T2(t2)
    comm = Hd @ (T2 @ fs.ref) - T2 @ (Hd @ fs.ref)
    den = fs.energy_denominators(s.eps)
    mask = fs.rank == 3
    t3s = np.zeros(fs.dim, complex)
    t3s[mask] = -comm[mask] / den[mask]
    return Hd, T2, t3s, den, mask


@pytest.mark.parametrize("o,v", [(2, 3), (3, 3)])
def test_t3_state_and_x(o, v):
    """T3|0> = -P3 [U,T2]|0> / eps and X = <mu|[H,T3]|0> (eq. cc3-t3-no-pert, cc3-x1-exp, cc3-x2-exp)."""
    s, m = _setup(o, v)
    t1, t2, _, _ = _random_state(o, v, 5)
    fs = FockSpace(o, v)
    Hd, _, t3s, _, _ = _harness_triples(fs, s, m, t1, t2)
    ti = orc.TriplesIntegrals(orc.Dressed(m, torch.tensor(t1), m.h(FIELD)))
    t3 = orc.t3_full(m, ti, torch.tensor(t2)).numpy()
    st = fs.triples_basis() @ t3.ravel() / 6.0
    assert np.abs(st - t3s).max() < 1e-15 * max(1, 1e3 * np.abs(t3s).max()) + 1e-16
    w1, w2 = fs.coefficients(Hd @ t3s)
    X1, X2 = orc.x_full(ti, torch.tensor(t3))
    assert np.abs(X1.numpy() - w1).max() < 1e-16 + 1e-12 * np.abs(w1).max()
    assert np.abs(X2.numpy() - w2).max() < 1e-16 + 1e-12 * np.abs(w2).max()


def test_loop_equals_explicit():
    o, v = 3, 4
    s, m = _setup(o, v)
    t1, t2, l1, l2 = (torch.tensor(x) for x in _random_state(o, v, 7))
    ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(FIELD)))
    ex = orc.triples_explicit(m, ti, t2, l1, l2, True)
    lp = orc.triples_loop(m, ti, t2, l1, l2, True)
    for k in ["X1", "X2", "Y1", "Y2", "Dij", "Dab", "Dia"]:
        assert (ex[k] - lp[k]).abs().max() < 1e-14 * max(1.0, ex[k].abs().max().item()), k


def test_t3_permutational_symmetry():
    """t_ijk^abc = t_jik^bac = t_ikj^acb = t_kji^cba = t_kij^cab = t_jki^bca."""
    o, v = 3, 4
    s, m = _setup(o, v)
    t1, t2, l1, l2 = (torch.tensor(x) for x in _random_state(o, v, 9))
    ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(FIELD)))
    for fn in (lambda i, j, k: orc.t3_block(m, ti, t2, i, j, k),
               lambda i, j, k: orc.l3_block(m, ti, l1, l2, i, j, k)):
        ref = fn(0, 1, 2)
        assert (fn(1, 0, 2).permute(1, 0, 2) - ref).abs().max() == 0 or \
            (fn(1, 0, 2).permute(1, 0, 2) - ref).abs().max() < 1e-16
        assert (fn(0, 2, 1).permute(0, 2, 1) - ref).abs().max() < 1e-16
        assert (fn(2, 1, 0).permute(2, 1, 0) - ref).abs().max() < 1e-16
        assert (fn(2, 0, 1).permute(1, 2, 0) - ref).abs().max() < 1e-16
        assert (fn(1, 2, 0).permute(2, 0, 1) - ref).abs().max() < 1e-16


def test_two_electron_triples_vanish():
    """o = 1: t_111^abc is symmetric in abc, so X1, X2, Y1, Y2 and the triples density vanish."""
    o, v = 1, 6
    s, m = _setup(o, v)
    t1, t2, l1, l2 = (torch.tensor(x) for x in _random_state(o, v, 2))
    ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(FIELD)))
    out = orc.triples_loop(m, ti, t2, l1, l2, True)
    for k in ["X1", "X2", "Y1", "Y2", "Dia"]:
        assert out[k].abs().max() < 1e-17, k
    ex = orc.triples_explicit(m, ti, t2, l1, l2, True)
    assert ex["l3"].abs().max() < 1e-16


def _holo_grad(f, x):
    xv = x.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(f(xv), [xv], grad_outputs=torch.ones((), dtype=torch.complex128))
    return g.conj()


def test_autograd_matches_finite_difference():
    o, v = 2, 3
    s, m = _setup(o, v)
    t1, t2, l1, l2 = (torch.tensor(x) for x in _random_state(o, v, 4))
    L1, L2 = l1, l2

    def lag(t1x, t2x):
        d = orc.Dressed(m, t1x, m.h(FIELD))
        r1, r2 = orc.ccsd_omega(d, t2x)
        return orc.ccsd_energy(d, t2x) + (L1 * r1).sum() + orc.C2 * (L2 * r2).sum()

    g1 = _holo_grad(lambda x: lag(x, t2), t1)
    g2 = _holo_grad(lambda x: lag(t1, x), t2)
    rng = np.random.default_rng(0)
    d1 = torch.tensor(rng.normal(size=t1.shape) + 1j * rng.normal(size=t1.shape))
    d2 = torch.tensor(rng.normal(size=t2.shape) + 1j * rng.normal(size=t2.shape))
    h = 1e-5
    fd1 = (lag(t1 + h * d1, t2) - lag(t1 - h * d1, t2)) / (2 * h)
    fd2 = (lag(t1, t2 + h * d2) - lag(t1, t2 - h * d2)) / (2 * h)
    assert abs(fd1 - (g1 * d1).sum()) < 1e-8
    assert abs(fd2 - (g2 * d2).sum()) < 1e-8


def test_printed_triples_lambda_terms_are_lagrangian_derivatives():
    """Y1 (eq. cc3-y1-exp) = dL/dt1 and Y2 (eq. cc3-y2-exp) = sym(dL/dt2)/C2 of
    the triples part l1.X1 + C2 l2.X2 with t3 at its closed form."""
    o, v = 3, 4
    s, m = _setup(o, v)
    t1, t2, l1, l2 = (torch.tensor(x) for x in _random_state(o, v, 5))

    def lt(t1x, t2x):
        d = orc.Dressed(m, t1x, m.h(FIELD))
        ti = orc.TriplesIntegrals(d)
        X1, X2 = orc.x_full(ti, orc.t3_full(m, ti, t2x))
        return (l1 * X1).sum() + orc.C2 * (l2 * X2).sum()

    g1 = _holo_grad(lambda x: lt(x, t2), t1)
    g2 = _holo_grad(lambda x: lt(t1, x), t2)
    g2 = 0.5 * (g2 + g2.permute(1, 0, 3, 2)) / orc.C2
    ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(FIELD)))
    ex = orc.triples_explicit(m, ti, t2, l1, l2)
    assert (ex["Y1"] - g1).abs().max() < 1e-15
    assert (ex["Y2"] - g2).abs().max() < 1e-15


def test_braket_lagrangian_density_and_lambda3():
    """Against <0|(1+Lambda) e^{-T} ... e^{T}|0> built in determinant space:
    the CCSD Lagrangian, the CCSD density, lambda3 (eq. cc3-l3) and the triples
    density terms (eq. cc3-dij and the following two)."""
    o, v = 2, 3
    s, m = _setup(o, v)
    t1, t2, l1, l2 = _random_state(o, v, 5)
    y = orc.pack(*[torch.tensor(x) for x in (t1, t2, l1, l2)])
    fs = FockSpace(o, v)
    n = o + v
    H = fs.hamiltonian(m.h(FIELD).numpy().astype(complex), _bare_g(s))
    T = fs.T1(t1) + fs.T2(t2)
    psi = fs.expm_apply(T, fs.ref)
    left = fs.expm_apply(T.T.tocsr(), fs.ref + fs.bra_from_lambda(l1, l2, orc.C2), sign=-1.0)
    assert abs(left @ (H @ psi) - orc.lagrangian(m, y, FIELD, with_triples=False).item()) < 1e-12
    Db = np.array([[left @ (fs.E(p, q) @ psi) for q in range(n)] for p in range(n)])
    Dt, d0 = orc.density_dressed(m, y, FIELD, with_triples=False)
    assert np.abs(Db - (d0.X.T @ Dt @ d0.Y.T).detach().numpy()).max() < 1e-12
    # triples: Lambda3 bra from stationarity, <Lambda3| = -P3 <(Lambda1+Lambda2) H| / eps
    Hd, T2, t3s, den, mask = _harness_triples(fs, s, m, t1, t2)
    bH = Hd.T @ fs.bra_from_lambda(l1, l2, orc.C2)
    l3b = np.zeros(fs.dim, complex)
    l3b[mask] = -bH[mask] / den[mask]
    ti = orc.TriplesIntegrals(orc.Dressed(m, torch.tensor(t1), m.h(FIELD)))
    ex = orc.triples_explicit(m, ti, torch.tensor(t2), torch.tensor(l1), torch.tensor(l2), True)
    lam_h = (l3b @ fs.triples_basis()).reshape(o, o, o, v, v, v)
    assert np.abs(lam_h - ex["l3"].numpy()).max() < 1e-15
    b2 = fs.bra_from_lambda(0 * l1, l2, orc.C2)
    c3 = l3b @ t3s
    DT = np.zeros((n, n), complex)
    for p in range(n):
        for q in range(n):
            Ep = fs.E(p, q)
            val = b2 @ (Ep @ t3s) + l3b @ (Ep @ t3s)
            if p == q and p < o:
                val -= 2.0 * c3
            x = T2 @ (T2 @ (Ep @ fs.ref)) - 2 * (T2 @ (Ep @ (T2 @ fs.ref))) + Ep @ (T2 @ (T2 @ fs.ref))
            DT[p, q] = val + 0.5 * (l3b @ x)
    assert np.abs(DT[:o, :o] - ex["Dij"].numpy()).max() < 1e-16
    assert np.abs(DT[o:, o:] - ex["Dab"].numpy()).max() < 1e-16
    assert np.abs(DT[:o, o:] - ex["Dia"].numpy()).max() < 1e-16
    assert np.abs(DT[o:, :o]).max() < 1e-18


def test_zero_field_conserves_lagrangian():
    """With a time-independent H, dL/dt = 0 along the EOMs; the RK4 drift falls at least like dt^4."""
    o, v = 2, 4
    s, m = _setup(o, v, seed=21)
    y0 = orc.pack(*[torch.tensor(x) for x in _random_state(o, v, 8, scale=0.05)])
    L0 = orc.lagrangian(m, y0, [0, 0, 0])
    drifts = []
    for dt, steps in [(0.02, 10), (0.01, 20)]:
        y, _ = orc.propagate(m, y0, dt, np.zeros((2 * steps + 1, 3)), triples="explicit")
        drifts.append(abs(orc.lagrangian(m, y, [0, 0, 0]) - L0).item())
    assert drifts[1] < 1e-8
    # global RK4 error over a fixed time falls at least like dt^4
    assert drifts[0] / drifts[1] > 14.0


def test_rk4_time_reversal():
    """Real amplitudes and a real Hamiltonian: y(-tau) = conj(y(tau)) for RK4 as well."""
    s, m = _setup(2, 4, seed=22)
    y0 = initial_state(s)
    f = np.zeros((7, 3))
    f[:, 2] = 0.003
    yf, muf = orc.propagate(m, y0, 0.05, f, triples="explicit")
    yb, mub = orc.propagate(m, y0, -0.05, f, triples="explicit")
    assert (yb - yf.conj()).abs().max() < 1e-14
    assert (mub - muf.conj()).abs().max() < 1e-13


def test_two_electron_dynamics_are_exact():
    """o = 1: CCSD is exact (CC3 triples vanish), so with the bra set to the normalised
    conjugate ket the Lagrangian dipole follows the exact TDSE in determinant space."""
    o, v = 1, 3
    s, m = _setup(o, v, seed=31)
    fs = FockSpace(o, v)
    t1, t2, _, _ = _random_state(o, v, 12, scale=0.2)
    T0 = (fs.T1(t1) + fs.T2(t2)).toarray()
    psi0 = sla.expm(T0) @ fs.ref
    bra = psi0.conj() / (psi0.conj() @ psi0)
    r = bra @ sla.expm(T0)  # <0|(1 + Lambda) = <Psi~| e^{T}
    assert abs(r @ fs.ref - 1) < 1e-13
    l1 = np.array([[r @ (fs.E(o + a, i) @ fs.ref) for a in range(v)] for i in range(o)])
    l2 = np.zeros((o, o, v, v), complex)
    for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
        l2[i, j, a, b] = r @ (fs.E(o + a, i) @ (fs.E(o + b, j) @ fs.ref))
    y0 = orc.pack(*[torch.tensor(x) for x in (t1, t2, l1, l2)])
    E = np.array([0.02, -0.01, 0.05])
    H = fs.hamiltonian(m.h(E).numpy().astype(complex), _bare_g(s)).toarray()
    dt, steps = 0.005, 40
    f = np.tile(E, (2 * steps + 1, 1))
    _, mu = orc.propagate(m, y0, dt, f)
    for n in (0, 10, 40):
        psi = sla.expm(-1j * H * dt * n) @ psi0
        for x in range(3):
            M = fs.one_body(s.mu[x].astype(complex))
            ex = (psi.conj() @ (M @ psi)) / (psi.conj() @ psi)
            assert abs(mu[n, x].item() - ex) < 1e-9
