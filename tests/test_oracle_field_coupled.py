"""Pins of the oracle's field-coupled triples (the CC3 Lagrangian with the field
terms of its triples block, App. A) against determinant space, and the size of
the approximation the GPU path integrates (the same Lagrangian without those
terms, exact at zero field).

* <mu3|[V,T3]|0> and 1/2 <mu3|[[V,T2],T2]|0> in amplitude form equal the
  determinant-space commutators for a general (non-symmetric, T1-transformed)
  one-electron operator;
* at a static field, t3 and lambda3 iterated by the oracle equal the
  determinant-space solutions of the triples equations of App. A
  (0 = <mu3|[H,T2] + [F+V,T3] + 1/2[[V,T2],T2]|0> and
  0 = <Lambda1+Lambda2|[H,tau3]|0> + <Lambda3|[F+V,tau3]|0>);
* at zero field the field-coupled right-hand side and dipole equal the closed-form
  ones; at any field the dipole (-dL/dE) equals the CC3 density expectation
  (CCSD part plus eq. cc3-dij and the two after it) with the field-coupled t3, lambda3;
* a short delta-kick propagation quantifies the difference of the two models.
"""
import numpy as np
import scipy.linalg as sla
import torch

from fci_harness import FockSpace
from oracle import rtcc3 as orc
from paper_2407_18947_amd.inputs import field_delta_kick, initial_state, make_system, random_state


def _setup(o, v, seed=5):
    s = make_system(o, v, seed=seed)
    return s, orc.Model.from_system(s)


def _bare_g(s):
    return np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)


def test_field_terms_equal_determinant_space_commutators():
    o, v = 2, 3
    s, m = _setup(o, v)
    t1, t2, l1, l2 = orc.unpack(m, random_state(o, v, 3, 0.1))
    fs = FockSpace(o, v)
    n = o + v
    Vb = np.random.default_rng(1).normal(size=(n, n))  # a general one-electron operator
    T1m = fs.T1(t1.numpy()).toarray()
    Vt = sla.expm(-T1m) @ fs.one_body(Vb.astype(complex)).toarray() @ sla.expm(T1m)
    d = orc.Dressed(m, t1, m.h([0, 0, 0]))
    vt = d.transform(torch.tensor(Vb))
    ti = orc.TriplesIntegrals(d)
    t3 = orc.t3_full(m, ti, t2)
    Tb = fs.triples_basis()
    ref, mask = fs.ref, fs.rank == 3
    T3s = Tb @ t3.numpy().ravel() / 6
    want = Vt @ T3s - (ref.conj() @ (Vt @ ref)) * T3s
    want[~mask] = 0
    got = Tb @ orc.vt3_full(vt, t3, o).numpy().ravel() / 6
    assert np.abs(got - want).max() < 1e-15 * max(1, 1e3 * np.abs(want).max())
    T2 = fs.T2(t2.numpy()).toarray()
    want = 0.5 * (Vt @ (T2 @ (T2 @ ref)) - 2 * (T2 @ (Vt @ (T2 @ ref))) + T2 @ (T2 @ (Vt @ ref)))
    want[~mask] = 0
    got = Tb @ orc.vtt_full(vt, t2, o).numpy().ravel() / 6
    assert np.abs(got - want).max() < 1e-15 * max(1, 1e3 * np.abs(want).max())
    assert np.abs(want).max() > 1e-3


def test_field_coupled_triples_equal_determinant_space_solutions():
    o, v = 2, 3
    s, m = _setup(o, v, seed=6)
    E = np.array([0.05, -0.04, 0.06])  # strong enough that the field terms matter
    t1, t2, l1, l2 = orc.unpack(m, random_state(o, v, 4, 0.1))
    t3, l3 = orc.field_coupled_triples(m, t1, t2, l1, l2, E)
    fs = FockSpace(o, v)
    H = fs.hamiltonian(m.h(E).numpy().astype(complex), _bare_g(s)).toarray()
    T1m = fs.T1(t1.numpy()).toarray()
    Hd = sla.expm(-T1m) @ H @ sla.expm(T1m)
    Vt = sla.expm(-T1m) @ fs.one_body((-np.einsum("x,xpq->pq", E, s.mu)).astype(complex)).toarray() @ sla.expm(T1m)
    ref, mask = fs.ref, fs.rank == 3
    den = fs.energy_denominators(s.eps)
    T2 = fs.T2(t2.numpy()).toarray()
    v0 = ref.conj() @ (Vt @ ref)
    comm = Hd @ (T2 @ ref) - T2 @ (Hd @ ref)
    dd = 0.5 * (Vt @ (T2 @ (T2 @ ref)) - 2 * (T2 @ (Vt @ (T2 @ ref))) + T2 @ (T2 @ (Vt @ ref)))
    s3 = np.zeros(fs.dim, complex)
    for _ in range(100):
        x = comm + (Vt @ s3 - v0 * s3) + dd
        new = np.zeros(fs.dim, complex)
        new[mask] = -x[mask] / den[mask]
        s3 = new
    Tb = fs.triples_basis()
    assert np.abs(Tb @ t3.numpy().ravel() / 6 - s3).max() < 1e-14
    bH = fs.bra_from_lambda(l1.numpy(), l2.numpy(), orc.C2) @ Hd
    l3b = np.zeros(fs.dim, complex)
    for _ in range(100):
        x = bH + (l3b @ Vt - v0 * l3b)
        new = np.zeros(fs.dim, complex)
        new[mask] = -x[mask] / den[mask]
        l3b = new
    lam = (l3b @ Tb).reshape(o, o, o, v, v, v)
    assert np.abs(lam - l3.numpy()).max() < 1e-13 * max(1, np.abs(lam).max())
    # and they differ from the closed forms the GPU path uses
    ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(E)))
    assert (orc.t3_full(m, ti, t2) - t3).abs().max() > 1e-6


def test_field_coupled_model_at_zero_field_and_its_density():
    o, v = 2, 3
    s, m = _setup(o, v, seed=7)
    y = torch.tensor(random_state(o, v, 5, 0.1))
    dy, mu = orc.rhs_field_coupled(m, y, [0, 0, 0], with_dipole=True)
    dy0, mu0 = orc.rhs(m, y, [0, 0, 0], triples="explicit", with_dipole=True)
    assert (dy - dy0).abs().max() < 1e-14 and (mu - mu0).abs().max() < 1e-14
    # at a field: -dL/dE is the density expectation with the field-coupled amplitudes
    E = np.array([0.02, 0.0, -0.03])
    _, mu = orc.rhs_field_coupled(m, y, E, with_dipole=True)
    t1, t2, l1, l2 = orc.unpack(m, y)
    t3, l3 = orc.field_coupled_triples(m, t1, t2, l1, l2, E)
    D, d0 = orc.density_dressed(m, y, E, with_triples=False)
    Dij, Dab, Dia = orc.density_triples_full(t2, l2, t3, l3)
    D = D.detach().clone()
    D[:o, :o] += Dij
    D[o:, o:] += Dab
    D[:o, o:] += Dia
    want = torch.stack([(D * d0.transform(m.mu[x])).sum() for x in range(3)])
    assert (mu - want).abs().max() < 1e-13


def test_closed_form_triples_approximation_over_a_kick():
    """Delta kick 0.002 a.u. (o = 2, v = 4, dt = 0.05, 10 steps): the dipole of the
    closed-form model the GPU path integrates stays within 1e-8 a.u. of the
    field-coupled model, which differs only while the field is on."""
    o, v = 2, 4
    s, m = _setup(o, v, seed=8)
    y0 = initial_state(s)
    steps, dt = 10, 0.05
    f = field_delta_kick(steps, dt, 0.002, "z")
    _, mu_fc = orc.propagate_field_coupled(m, y0, dt, f)
    _, mu_cf = orc.propagate(m, y0, dt, f, triples="explicit")
    diff = (mu_fc - mu_cf).abs().max().item()
    print(f"closed-form vs field-coupled triples: max dipole difference {diff:.3e} a.u.")
    assert 1e-13 < diff < 1e-8
