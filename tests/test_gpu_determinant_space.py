"""The HIP path against the determinant-space construction directly.

The GPU's CCSD part follows the same sequence of intermediates as the oracle,
so parity with the oracle alone would not catch a mistake the two share.  Here
the GPU's residuals and triples terms are compared, through the C ABI, with the
second-quantized construction of tests/fci_harness.py, which shares no code with
either:

* Omega_mu = <mu| exp(-T) H(E) exp(T) |0> for singles and doubles
  (the CCSD residual with the field coupling, Sec. 2.1 and 2.2.1);
* T3|0> = -P3 [H~, T2]|0> / eps (the closed-form t3 of eq. cc3-t3-no-pert with
  the T1-dressed, field-included Hamiltonian) and
  X_mu = <mu| [H~, T3] |0> (eq. cc3-x1-exp and cc3-x2-exp);
* the Lambda residuals as derivatives of the CCSD Lagrangian
  L = <0|(1 + Lambda) exp(-T) H exp(T)|0> with respect to the amplitudes,
  dL/dt_mu = <0|(1 + Lambda) exp(-T) [H, tau_mu] exp(T)|0> (the doubles divided
  by the weight 1/2 of l2 in the Lagrangian);
* the dipole from the densities (Sec. 2.2.3): the CCSD part as the bra-ket
  density <0|(1 + Lambda) exp(-T) E_pq exp(T)|0> with the bare dipole
  integrals, the triples part (eq. cc3-dij and the two after it, with lambda3
  from stationarity, eq. cc3-l3) with the T1-transformed ones;
* Y1 and Y2 (eq. cc3-y1-exp and cc3-y2-exp) as the amplitude derivatives of the
  triples part of the Lagrangian, <0|(Lambda1 + Lambda2) H~ T3|0> with T3 at its
  closed form, by four-point differences of the determinant-space construction.
"""
import itertools

import numpy as np
import pytest
import torch

from fci_harness import FockSpace, dress_integrals
from oracle import rtcc3 as orc
from paper_2407_18947_amd import _lib
from paper_2407_18947_amd.inputs import make_system

pytestmark = pytest.mark.gpu
FIELD = np.array([0.01, -0.02, 0.03])
C2 = 0.5  # weight of l2 in the Lagrangian and in the bra <0|(1 + Lambda)


def _state(o, v, seed, scale=0.1):
    rng = np.random.default_rng(seed)

    def rc(*sh):
        return scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))

    t1, l1 = rc(o, v), rc(o, v)
    t2, l2 = rc(o, o, v, v), rc(o, o, v, v)
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    l2 = 0.5 * (l2 + l2.transpose(1, 0, 3, 2))
    return t1, t2, l1, l2


def _gpu_terms(s, y):
    ctx = _lib.Context(s, _lib.RTCC3_FP64)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    td = torch.zeros(ctx.terms_size(), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    _lib.rtcc3_rhs_terms(ctx.ctx, FIELD, yd, td, 1)
    out = ctx.split_terms(td.cpu().numpy())
    ctx.close()
    return out


def _close(name, a, b, tol=1e-11):
    err = np.abs(np.asarray(a) - np.asarray(b)).max()
    scale = np.abs(b).max()
    assert err <= tol * scale + 1e-15, f"{name}: max|diff| = {err:.3e} (largest element {scale:.3e})"


@pytest.mark.parametrize("o,v", [(2, 3), (3, 3)])
def test_gpu_residual_and_triples_equal_determinant_space(o, v):
    print(f"determinant space o={o} v={v}", flush=True)
    s = make_system(o, v, seed=11)
    m = orc.Model.from_system(s)
    t1, t2, l1, l2 = _state(o, v, 3)
    y = np.concatenate([x.ravel() for x in (t1, t2, l1, l2)])  # the state layout of the C ABI
    g = _gpu_terms(s, y)

    fs = FockSpace(o, v)
    h = m.h(FIELD).numpy().astype(complex)  # h0 - mu.E (its sign and h0 are pinned on the CPU)
    gbare = np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)
    H = fs.hamiltonian(h, gbare)
    T = fs.T1(t1) + fs.T2(t2)
    hbar = fs.expm_apply(T, H @ fs.expm_apply(T, fs.ref), sign=-1.0)
    w1, w2 = fs.coefficients(hbar)
    _close("R1", g["R1"], w1)
    _close("R2", g["R2"], w2)

    ht, gt = dress_integrals(o, v, t1, h, s.B)
    Hd = fs.hamiltonian(ht, gt)
    T2 = fs.T2(t2)
    comm = Hd @ (T2 @ fs.ref) - T2 @ (Hd @ fs.ref)
    den = fs.energy_denominators(s.eps)
    mask = fs.rank == 3
    t3s = np.zeros(fs.dim, complex)
    t3s[mask] = -comm[mask] / den[mask]
    x1, x2 = fs.coefficients(Hd @ t3s)
    _close("X1", g["X1"], x1)
    _close("X2", g["X2"], x2)

    # Lambda residuals: derivatives of the CCSD Lagrangian
    psi = fs.expm_apply(T, fs.ref)
    left = fs.expm_apply(T.T.tocsr(), fs.ref + fs.bra_from_lambda(l1, l2, C2), sign=-1.0)
    hpsi = H @ psi

    def dl(tau):
        return left @ (H @ (tau @ psi)) - left @ (tau @ hpsi)

    G1 = np.zeros((o, v), complex)
    for i, a in itertools.product(range(o), range(v)):
        e = np.zeros((o, v), complex)
        e[i, a] = 1.0
        G1[i, a] = dl(fs.T1(e))
    G2 = np.zeros((o, o, v, v), complex)
    for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
        e = np.zeros((o, o, v, v), complex)
        e[i, j, a, b] = 1.0
        G2[i, j, a, b] = dl(fs.T2(e)) / C2
    _close("G1", g["G1"], G1)
    _close("G2", g["G2"], G2)

    # dipole: CCSD bra-ket density (bare integrals) + triples density (T1-transformed integrals)
    nn = o + v
    Db = np.array([[left @ (fs.E(p, q) @ psi) for q in range(nn)] for p in range(nn)])
    bH = Hd.T @ fs.bra_from_lambda(l1, l2, C2)
    l3b = np.zeros(fs.dim, complex)
    l3b[mask] = -bH[mask] / den[mask]
    b2 = fs.bra_from_lambda(0 * l1, l2, C2)
    c3 = l3b @ t3s
    DT = np.zeros((nn, nn), complex)
    for p in range(nn):
        for q in range(nn):
            Ep = fs.E(p, q)
            val = b2 @ (Ep @ t3s) + l3b @ (Ep @ t3s)
            if p == q and p < o:
                val -= 2.0 * c3
            x = T2 @ (T2 @ (Ep @ fs.ref)) - 2 * (T2 @ (Ep @ (T2 @ fs.ref))) + Ep @ (T2 @ (T2 @ fs.ref))
            DT[p, q] = val + 0.5 * (l3b @ x)
    tm = np.zeros((nn, nn), complex)
    tm[o:, :o] = t1.T
    Xf, Yf = np.eye(nn) - tm, np.eye(nn) + tm  # h~ = X h Y
    mus = s.mu.astype(complex)
    mu = np.array([np.sum(Db * mus[x]) + np.sum(DT * (Xf @ mus[x] @ Yf)) for x in range(3)])
    _close("mu", g["mu"], mu)


def test_gpu_triples_lambda_terms_equal_determinant_space_derivatives():
    o, v = 2, 3
    print(f"determinant space Y1, Y2 o={o} v={v}", flush=True)
    s = make_system(o, v, seed=11)
    m = orc.Model.from_system(s)
    t1, t2, l1, l2 = _state(o, v, 3)
    y = np.concatenate([x.ravel() for x in (t1, t2, l1, l2)])
    g = _gpu_terms(s, y)

    fs = FockSpace(o, v)
    h = m.h(FIELD).numpy().astype(complex)
    den = fs.energy_denominators(s.eps)
    mask = fs.rank == 3
    bra = fs.bra_from_lambda(l1, l2, C2)

    def l3(t1x, t2x):  # <0|(Lambda1 + Lambda2) H~ T3|0>, T3|0> = -P3 [H~, T2]|0> / eps
        ht, gt = dress_integrals(o, v, t1x, h, s.B)
        Hd = fs.hamiltonian(ht, gt)
        T2 = fs.T2(t2x)
        comm = Hd @ (T2 @ fs.ref) - T2 @ (Hd @ fs.ref)
        t3s = np.zeros(fs.dim, complex)
        t3s[mask] = -comm[mask] / den[mask]
        return bra @ (Hd @ t3s)

    hh = 1e-3  # four-point differences: error O(hh^4) of the smooth, holomorphic l3

    def d4(f, x, e):
        return (8 * (f(x + hh * e) - f(x - hh * e)) - (f(x + 2 * hh * e) - f(x - 2 * hh * e))) / (12 * hh)

    Y1 = np.zeros((o, v), complex)
    for i, a in itertools.product(range(o), range(v)):
        e = np.zeros((o, v))
        e[i, a] = 1.0
        Y1[i, a] = d4(lambda x: l3(x, t2), t1, e)
    Y2 = np.zeros((o, o, v, v), complex)
    for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
        e = np.zeros((o, o, v, v))
        e[i, j, a, b] = 1.0
        Y2[i, j, a, b] = d4(lambda x: l3(t1, x), t2, e)
    Y2 = 0.5 * (Y2 + Y2.transpose(1, 0, 3, 2)) / C2
    _close("Y1", g["Y1"], Y1, 1e-9)
    _close("Y2", g["Y2"], Y2, 1e-9)
