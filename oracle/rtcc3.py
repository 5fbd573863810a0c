"""Oracle: a plain, slow, complex128 CPU implementation of real-time CC3.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the HIP implementation.

What it computes (arXiv 2407.18947, Sec. 2.1 and Appendix A):

* the perturbed Hamiltonian H(t) = F + U - mu.E(t) (Sec. 2.1, eq. cc3-h-pert;
  dipole coupling of Sec. 2.2.1), in the canonical orbital basis with
  (pq|rs) = sum_P B[P,p,q] B[P,r,s];
* the T1 transformation O = exp(-T1) O exp(T1) (Sec. 2.1, Appendix A);
* the right-hand sides of the amplitude equations, i dt/dt = <mu|Hbar|0>
  (eq. cc3-rt-t) and -i dlambda/dt = dL/dt (eq. cc3-rt-l, obtained from the
  Euler-Lagrange equations of the CC3 Lagrangian in Appendix A):
    - singles/doubles CCSD parts: closed-shell T1-transformed CCSD (the
      paper uses the existing CCSD equations and does not print them);
      the Lambda side is the derivative of the Lagrangian, taken by
      automatic differentiation, which is the Euler-Lagrange equation itself;
    - triples: t3 from the closed form of eq. cc3-t3-no-pert, lambda3 from
      eq. cc3-l3 in its spin-adapted form (eq. cc3-l3-exp), and their
      contributions X1 (eq. cc3-x1-exp), X2 (eq. cc3-x2-exp), Y1
      (eq. cc3-y1-exp) and Y2 (eq. cc3-y2-exp), evaluated for one occupied
      triple (i,j,k) at a time (Sec. 2.1) or, for tiny systems, with the full
      six-index tensors;
* the one-electron density (CCSD part plus the triples terms of eq. cc3-dij
  and the following two equations) and the dipole Tr(D mu) (Sec. 2.2.3);
* classic RK4 propagation (Sec. 3).

Readings of places where the paper is silent or garbled are listed with the
code that takes them (search for "Reading").

Layouts: t1[i,a], t2[i,j,a,b] = t_ij^ab, l1[i,a] = lambda_a^i,
l2[i,j,a,b] = lambda_ab^ij, t3[i,j,k,a,b,c] = t_ijk^abc.  Integrals are
Mulliken (pq|rs); the paper's physicist <pq|rs> equals (pr|qs).
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

R64 = torch.float64
C128 = torch.complex128

# Reading: pairing of the Lagrangian.  The Lagrangian used is
#   L = E + sum_ia l1_ia Omega_ia + C2 * sum_ijab l2_ijab Omega_ijab
# over all tensor elements.  Its value is fixed by requiring the paper's
# printed triples equations (lambda3, Y1, Y2, density) to be its derivatives;
# the tests pin it (tests/test_oracle_pins.py: the printed Y1, Y2 are the
# Lagrangian's derivatives, and lambda3 and the densities equal their
# determinant-space bra-ket expressions).
C2 = 0.5


def _t(x, dtype=C128):
    return torch.as_tensor(np.asarray(x), dtype=dtype)


class Model:
    """Bare (field-free) integrals and dipole matrices of one system."""

    def __init__(self, o, v, eps, B, mu):
        self.o, self.v = int(o), int(v)
        self.n = self.o + self.v
        self.eps = _t(eps, R64)
        self.B = _t(B, R64)
        self.mu = _t(mu, R64)
        o = self.o
        # Bare one-electron operator h0 such that the Fock matrix built from it
        # with the closed-shell reference is diag(eps):
        #   f_pq = h_pq + sum_i [2 (pq|ii) - (pi|iq)]   (normal-ordered H, App. A)
        Bd = torch.einsum("Pii->P", self.B[:, :o, :o])
        J = torch.einsum("Ppq,P->pq", self.B, Bd)
        K = torch.einsum("Ppi,Piq->pq", self.B[:, :, :o], self.B[:, :o, :])
        self.h0 = torch.diag(self.eps) - (2.0 * J - K)
        self._d3 = None

    @property
    def d3(self):
        """D_ijk^abc for all six indices (explicit mode; built on first use)."""
        if self._d3 is None:
            eo, ev = self.eps[:self.o], self.eps[self.o:]
            self._d3 = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None]
                        + eo[None, None, :, None, None, None] - ev[None, None, None, :, None, None]
                        - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
        return self._d3

    @classmethod
    def from_system(cls, s):
        return cls(s.o, s.v, s.eps, s.B, s.mu)

    def h(self, E):
        """One-electron operator with the dipole coupling V = -mu.E (Sec. 2.2.1).

        E may be complex (the derivatives below evaluate the equations, which are
        polynomials in E, at complex fields)."""
        E = np.asarray(E)
        if np.iscomplexobj(E):
            Ec = torch.as_tensor(E.astype(np.complex128))
            return self.h0.to(C128) - torch.einsum("x,xpq->pq", Ec, self.mu.to(C128))
        E = torch.as_tensor(E.astype(np.float64))
        return self.h0 - torch.einsum("x,xpq->pq", E, self.mu)

    def denom3(self, i, j, k):
        """D_ijk^abc = e_i + e_j + e_k - e_a - e_b - e_c = -epsilon_mu3 (App. A)."""
        o = self.o
        eo, ev = self.eps[:o], self.eps[o:]
        return (eo[i] + eo[j] + eo[k]) - ev[:, None, None] - ev[None, :, None] - ev[None, None, :]


# -----------------------------------------------------------------------------
# T1 transformation (Sec. 2.1; Appendix A)
# -----------------------------------------------------------------------------

class Dressed:
    """T1-transformed one-electron operator, DF factors and Fock matrix.

    exp(-T1) a+_i exp(T1) = a+_i - sum_a t_i^a a+_a and
    exp(-T1) a_a exp(T1) = a_a + sum_i t_i^a a_i, so every one-index object
    x_pq transforms as (1 - T) x (1 + T), where T[a,i] = t_i^a is the only
    non-zero block of the n x n matrix T.
    """

    def __init__(self, m: Model, t1, h):
        o, n = m.o, m.n
        Tm = torch.zeros((n, n), dtype=C128)
        Tm = Tm.index_put((torch.arange(o, n)[:, None], torch.arange(o)[None, :]), t1.transpose(0, 1))
        eye = torch.eye(n, dtype=C128)
        self.X = eye - Tm
        self.Y = eye + Tm
        self.o = o
        self.h = self.X @ h.to(C128) @ self.Y
        self.B = torch.einsum("pr,Prs,sq->Ppq", self.X, m.B.to(C128), self.Y)
        Bd = torch.einsum("Pkk->P", self.B[:, :o, :o])
        J = torch.einsum("Ppq,P->pq", self.B, Bd)
        K = torch.einsum("Ppk,Pkq->pq", self.B[:, :, :o], self.B[:, :o, :])
        self.F = self.h + 2.0 * J - K

    def g(self, s: str):
        """Dressed Mulliken block (pq|rs)~ for an index-space string like 'ovov'."""
        o = self.o
        sl = {"o": slice(0, o), "v": slice(o, None)}
        p, q, r, t = (sl[c] for c in s)
        return torch.einsum("Ppq,Prs->pqrs", self.B[:, p, q], self.B[:, r, t])

    def transform(self, x):
        return self.X @ x.to(C128) @ self.Y


# -----------------------------------------------------------------------------
# CCSD parts: closed-shell T1-transformed CCSD (standard theory; the paper's
# "existing CCSD equations", Sec. 2.1).  Omega = expansion coefficients of
# exp(-T2) H exp(T2)|0> in {E_ai|0>, 1/2 E_ai E_bj|0>} (pinned in the tests
# against a determinant-space construction).
# -----------------------------------------------------------------------------

def _perm_ijab(x):
    """P_ij^ab x = x_ij^ab + x_ji^ba (eq. cc3-pijab)."""
    return x + x.permute(1, 0, 3, 2)


def ccsd_energy(d: Dressed, t2):
    o = d.o
    gov = d.g("ovov")
    L = 2.0 * gov - gov.permute(0, 3, 2, 1)
    e_ref = torch.einsum("ii->", d.h[:o, :o]) + torch.einsum("ii->", d.F[:o, :o])
    return e_ref + torch.einsum("ijab,iajb->", t2, L)


def ccsd_omega(d: Dressed, t2):
    o = d.o
    F = d.F
    Foo, Fov, Fvo, Fvv = F[:o, :o], F[:o, o:], F[o:, :o], F[o:, o:]
    u = 2.0 * t2 - t2.permute(0, 1, 3, 2)
    g_ovov = d.g("ovov")
    L_ovov = 2.0 * g_ovov - g_ovov.permute(0, 3, 2, 1)
    # singles
    r1 = (torch.einsum("kicd,adkc->ia", u, d.g("vvov"))
          - torch.einsum("klac,kilc->ia", u, d.g("ooov"))
          + torch.einsum("ikac,kc->ia", u, Fov)
          + Fvo.transpose(0, 1))
    # doubles
    A2 = d.g("vovo").permute(1, 3, 0, 2) + torch.einsum("ijcd,acbd->ijab", t2, d.g("vvvv"))
    Xkl = d.g("oooo").permute(0, 2, 1, 3) + torch.einsum("ijcd,kcld->klij", t2, g_ovov)
    B2 = torch.einsum("klab,klij->ijab", t2, Xkl)
    Y = d.g("oovv") - 0.5 * torch.einsum("liad,kdlc->kiac", t2, g_ovov)
    Cx = -0.5 * torch.einsum("kjbc,kiac->ijab", t2, Y) - torch.einsum("kibc,kjac->ijab", t2, Y)
    Lt_voov = 2.0 * d.g("voov") - d.g("vvoo").permute(0, 3, 2, 1)
    Z = Lt_voov + 0.5 * torch.einsum("ilad,ldkc->aikc", u, L_ovov)
    D2 = 0.5 * torch.einsum("jkbc,aikc->ijab", u, Z)
    E2 = (torch.einsum("ijac,bc->ijab", t2, Fvv - torch.einsum("klbd,ldkc->bc", u, g_ovov))
          - torch.einsum("ikab,kj->ijab", t2, Foo + torch.einsum("ljcd,kdlc->kj", u, g_ovov)))
    r2 = A2 + B2 + _perm_ijab(Cx + D2 + E2)
    return r1, r2


# -----------------------------------------------------------------------------
# Triples (eq. cc3-t3-no-pert, eq. cc3-x1-exp, eq. cc3-x2-exp, eq. cc3-l3-exp,
# eq. cc3-y1-exp, eq. cc3-y2-exp, eq. cc3-dij and the following two)
# -----------------------------------------------------------------------------

# P_ijk^abc (eq. cc3-pijkabc) as permutations of (i,j,k) applied to both the
# occupied and virtual slots: f_ijk^abc, f_jik^bac, f_ikj^acb, f_kji^cba,
# f_kij^cab, f_jki^bca.
_P3 = [(0, 1, 2), (1, 0, 2), (0, 2, 1), (2, 1, 0), (2, 0, 1), (1, 2, 0)]


def p3_full(x):
    """P_ijk^abc on a full [o,o,o,v,v,v] tensor."""
    out = torch.zeros_like(x)
    for s in _P3:
        # term[i,j,k,a,b,c] = x[s-permuted (i,j,k)], same for (a,b,c)
        inv = [s.index(q) for q in range(3)]
        out = out + x.permute(*inv, *[3 + q for q in inv])
    return out


class TriplesIntegrals:
    """Integral blocks the triples equations use (dressed where the paper puts a tilde)."""

    def __init__(self, d: Dressed):
        self.g_vovv = d.g("vovv")  # (ck|be)~  = <cb|ke>~
        self.g_oovo = d.g("oovo")  # (mj|ck)~  = <mc|jk>~
        self.g_vvov = d.g("vvov")  # (ac|ke)~  = <ak|ce>~
        self.g_ooov = d.g("ooov")  # (ki|mc)~  = <km|ic>~
        self.g_ovoo = d.g("ovoo")  # (ka|jl)~  = <kj|al>~
        self.g_ovvv = d.g("ovvv")  # (ka|db)~  = <kd|ab>~
        self.g_vvvo = d.g("vvvo")  # (da|el)~  = <de|al>~
        self.g_oovv = d.g("oovv")  # (jl|da)~  = <jd|la>~
        self.g_voov = d.g("voov")  # (dl|ja)~  = <dj|la>~
        self.g_vvvv = d.g("vvvv")  # (da|eb)~  = <de|ab>~
        self.g_oooo = d.g("oooo")  # (il|jm)~  = <ij|lm>~
        gov = d.g("ovov")           # (ia|jb), dressing-invariant
        self.g_ovov = gov
        self.L_ovov = 2.0 * gov - gov.permute(0, 3, 2, 1)  # L_iajb = 2(ia|jb) - (ib|ja)
        o = d.o
        self.Fov = d.F[:o, o:]
        # Lt_ijal = 2<ij|al>~ - <ij|la>~ = 2(ia|jl)~ - (il|ja)~
        self.Lt_ovoo = 2.0 * self.g_ovoo - self.g_ooov.permute(0, 3, 2, 1)
        # Lt_djab = 2<dj|ab>~ - <dj|ba>~ = 2(da|jb)~ - (db|ja)~
        self.Lt_vvov = 2.0 * self.g_vvov - self.g_vvov.permute(0, 3, 2, 1)


def w_prime_block(ti: TriplesIntegrals, t2, i, j, k):
    """W'_ijk^abc = sum_e t_ij^ae <cb|ke>~ - sum_m t_im^ab <mc|jk>~ (eq. cc3-t3-no-pert, spin-adapted)."""
    return (torch.einsum("ae,cbe->abc", t2[i, j], ti.g_vovv[:, k, :, :])
            - torch.einsum("mab,mc->abc", t2[i], ti.g_oovo[:, j, :, k]))


def m_prime_block(ti: TriplesIntegrals, l1, l2, i, j, k):
    """The bracket of eq. cc3-l3-exp for one ordered (i,j,k), before P_ijk^abc."""
    L = ti.L_ovov
    Fov = ti.Fov
    x = (torch.einsum("ab,c->abc", L[i, :, j, :], l1[k])
         - torch.einsum("ac,b->abc", L[i, :, j, :], l1[k])
         + torch.einsum("a,bc->abc", Fov[i], l2[j, k])
         + torch.einsum("al,lbc->abc", ti.g_ovoo[k, :, j, :], l2[:, i])
         - torch.einsum("adb,cd->abc", ti.g_ovvv[k], l2[i, j]))

    def half(i, j, ab):
        y = (-torch.einsum("a,bc->abc", Fov[j], l2[i, k])
             - torch.einsum("al,lbc->abc", ti.Lt_ovoo[i, :, j, :], l2[:, k])
             + torch.einsum("dab,cd->abc", ti.Lt_vvov[:, :, j, :], l2[k, i]))
        return y if not ab else y.permute(1, 0, 2)

    # 1/2 P_ij^ab (...): the term plus its (i<->j, a<->b) image
    x = x + 0.5 * (half(i, j, False) + half(j, i, True))
    return x


_PERM_BLOCK = {
    # block of the permuted occupied triple, rearranged into [a,b,c] order
    (0, 1, 2): (0, 1, 2),
    (1, 0, 2): (1, 0, 2),
    (0, 2, 1): (0, 2, 1),
    (2, 1, 0): (2, 1, 0),
    (2, 0, 1): (1, 2, 0),
    (1, 2, 0): (2, 0, 1),
}


def sym_block(fn, i, j, k):
    """P_ijk^abc applied blockwise: sum over the six (i,j,k)/(a,b,c) permutations."""
    occ = (i, j, k)
    out = None
    for s in _P3:
        blk = fn(occ[s[0]], occ[s[1]], occ[s[2]])
        term = blk.permute(*_PERM_BLOCK[s])
        out = term if out is None else out + term
    return out


def t3_block(m: Model, ti, t2, i, j, k):
    """t_ijk^abc = P_ijk^abc W'_ijk^abc / D_ijk^abc for one ordered triple."""
    w = sym_block(lambda a, b, c: w_prime_block(ti, t2, a, b, c), i, j, k)
    return w / m.denom3(i, j, k)


def l3_block(m: Model, ti, l1, l2, i, j, k):
    """lambda_abc^ijk = P_ijk^abc {...} / D_ijk^abc (eq. cc3-l3-exp with eq. cc3-l3's denominator)."""
    w = sym_block(lambda a, b, c: m_prime_block(ti, l1, l2, a, b, c), i, j, k)
    return w / m.denom3(i, j, k)


def t3_full(m: Model, ti, t2):
    wp = (torch.einsum("ijae,ckbe->ijkabc", t2, ti.g_vovv)
          - torch.einsum("imab,mjck->ijkabc", t2, ti.g_oovo))
    return p3_full(wp) / m.d3


def l3_full(m: Model, ti, l1, l2):
    L, Fov = ti.L_ovov, ti.Fov
    x = (torch.einsum("iajb,kc->ijkabc", L, l1)
         - torch.einsum("iajc,kb->ijkabc", L, l1)
         + torch.einsum("ia,jkbc->ijkabc", Fov, l2)
         + torch.einsum("kajl,libc->ijkabc", ti.g_ovoo, l2)
         - torch.einsum("kadb,ijcd->ijkabc", ti.g_ovvv, l2))
    y = (-torch.einsum("ja,ikbc->ijkabc", Fov, l2)
         - torch.einsum("iajl,lkbc->ijkabc", ti.Lt_ovoo, l2)
         + torch.einsum("dajb,kicd->ijkabc", ti.Lt_vvov, l2))
    x = x + 0.5 * (y + y.permute(1, 0, 2, 4, 3, 5))
    return p3_full(x) / m.d3


def x_full(ti: TriplesIntegrals, t3):
    """X1 (eq. cc3-x1-exp) and X2 (eq. cc3-x2-exp) from a full t3."""
    tz = t3 - t3.permute(0, 1, 2, 5, 4, 3)  # t_ijk^abc - t_ijk^cba
    X1 = torch.einsum("ijkabc,jbkc->ia", tz, ti.L_ovov)
    x2 = torch.einsum("ijkabc,kc->ijab", tz, ti.Fov)
    z = 2.0 * t3 - t3.permute(0, 1, 2, 3, 5, 4) - t3.permute(0, 1, 2, 5, 4, 3)  # [ijk, c b e]
    x2 = x2 + torch.einsum("ijkcbe,acke->ijab", z, ti.g_vvov)
    zh = 2.0 * t3.permute(0, 1, 2, 5, 4, 3) - t3.permute(0, 1, 2, 5, 3, 4) - t3  # [mjk, a b c]
    x2 = x2 - torch.einsum("mjkabc,kimc->ijab", zh, ti.g_ooov)
    return X1, _perm_ijab(x2)


def y_full(ti: TriplesIntegrals, t2, l2, t3, l3):
    """Y1 (eq. cc3-y1-exp) and Y2 (eq. cc3-y2-exp) from full t3 and lambda3."""
    gov, L = ti.g_ovov, ti.L_ovov
    Y1 = (torch.einsum("jklbcd,icjd,klab->ia", t3, gov, l2)
          + torch.einsum("jklbcd,kalb,ijcd->ia", t3, gov, l2)
          + torch.einsum("jklbcd,iajb,klcd->ia", t3, L, l2)
          - torch.einsum("jklbcd,iajc,klbd->ia", t3, L, l2)
          - torch.einsum("jklbcd,jbic,klad->ia", t3, L, l2)
          # Reading: the printed L_ijab of this term carries the wrong occupied
          # index; the derivative of the lambda2.X2 pairing with respect to t1
          # gives L_kjab = 2(ka|jb) - (kb|ja).
          - torch.einsum("jklbcd,kajb,ilcd->ia", t3, L, l2)
          - torch.einsum("jkbc,jlda,lkibcd->ia", t2, ti.g_oovv, l3)
          - torch.einsum("jkbc,dlja,iklbcd->ia", t2, ti.g_voov, l3)
          - torch.einsum("jkbc,ildb,lkjacd->ia", t2, ti.g_oovv, l3)
          # Reading: the printed <di|la> repeats 'a' and leaves 'b' free; the
          # term is read as <di|lb>~ = (dl|ib)~, the exchange partner of the
          # preceding <id|lb>~ term.
          - torch.einsum("jkbc,dlib,jklacd->ia", t2, ti.g_voov, l3)
          + torch.einsum("jkbc,daeb,kijcde->ia", t2, ti.g_vvvv, l3)
          + torch.einsum("jkbc,iljm,lmkabc->ia", t2, ti.g_oooo, l3))
    y2 = torch.einsum("dael,ijldbe->ijab", ti.g_vvvo, l3)
    y2 = y2 - torch.einsum("imdl,mjlabd->ijab", ti.g_oovo, l3)
    return Y1, _perm_ijab(y2)


def density_triples_full(t2, l2, t3, l3):
    """D_ij, D_ab, D_ia of eq. cc3-dij and the two equations after it."""
    Dij = -0.5 * torch.einsum("ilkabc,jlkabc->ij", t3, l3)
    Dab = 0.5 * torch.einsum("ijkbdc,ijkadc->ab", t3, l3)
    Dia = (torch.einsum("ijkabc,jkbc->ia", t3 - t3.permute(0, 1, 2, 4, 3, 5), l2)
           - torch.einsum("jklbcd,ilcd,kjab->ia", l3, t2, t2))
    return Dij, Dab, Dia


def triples_loop(m: Model, ti: TriplesIntegrals, t2, l1, l2, want_density=False, max_blocks=None, only=None):
    """Triples contributions evaluated one occupied triple at a time (Sec. 2.1).

    The loop runs over (l,k) and, inside, over i, building the [v,v,v] blocks
    t3_{ilk} and lambda3_{ilk}; the o blocks sharing (l,k) serve D_ij.
    Every other contraction takes the block of one ordered triple at a time.
    max_blocks stops after that many blocks; only(I, J, K) -> bool skips the
    blocks it rejects.  Either gives partial sums, exact for the elements that
    depend only on the blocks visited.
    """
    o, v = m.o, m.v
    X1 = torch.zeros((o, v), dtype=C128)
    x2 = torch.zeros((o, o, v, v), dtype=C128)
    Y1 = torch.zeros((o, v), dtype=C128)
    y2 = torch.zeros((o, o, v, v), dtype=C128)
    Dij = torch.zeros((o, o), dtype=C128)
    Dab = torch.zeros((v, v), dtype=C128)
    Dia = torch.zeros((o, v), dtype=C128)
    gov, L = ti.g_ovov, ti.L_ovov
    done = 0
    for J in range(o):
        for K in range(o):
            if max_blocks is not None and done >= max_blocks:
                break
            tstack, lstack = [], []
            for I in range(o):
                done += 1
                if only is not None and not only(I, J, K):
                    continue
                t = t3_block(m, ti, t2, I, J, K)
                lam = l3_block(m, ti, l1, l2, I, J, K)
                tstack.append(t)
                lstack.append(lam)
                # --- X1, X2 (block (I,J,K) as (i,j,k), and as (m,j,k))
                tz = t - t.permute(2, 1, 0)
                X1[I] += torch.einsum("abc,bc->a", tz, L[J, :, K, :])
                x2[I, J] += torch.einsum("abc,c->ab", tz, ti.Fov[K])
                z = 2.0 * t - t.permute(0, 2, 1) - t.permute(2, 1, 0)
                x2[I, J] += torch.einsum("cbe,ace->ab", z, ti.g_vvov[:, :, K, :])
                zh = 2.0 * t.permute(2, 1, 0) - t.permute(2, 0, 1) - t
                x2[:, J] -= torch.einsum("abc,xc->xab", zh, ti.g_ooov[K, :, I, :])
                # --- Y2 (block as (i,j,l) and as (m,j,l))
                y2[I, J] += torch.einsum("dbe,dae->ab", lam, ti.g_vvvo[:, :, :, K])
                y2[:, J] -= torch.einsum("abd,xd->xab", lam, ti.g_oovo[:, I, :, K])
                # --- Y1: t3 lambda2 terms, block t3 as (j,k,l) = (I,J,K)
                Y1 += torch.einsum("bcd,xcd,ab->xa", t, gov[:, :, I, :], l2[J, K])
                Y1 += torch.einsum("bcd,ab,xcd->xa", t, gov[J, :, K, :], l2[:, I])
                Y1 += torch.einsum("bcd,cd,xab->xa", t, l2[J, K], L[:, :, I, :])
                Y1 -= torch.einsum("bcd,bd,xac->xa", t, l2[J, K], L[:, :, I, :])
                Y1 -= torch.einsum("bcd,ad,bxc->xa", t, l2[J, K], L[I])
                Y1 -= torch.einsum("bcd,ab,xcd->xa", t, L[J, :, I, :], l2[:, K])
                # --- Y1: t2 lambda3 terms
                # lambda_bcd^{lki}: block (I,J,K) = (l,k,i) -> output i = K
                Y1[K] -= torch.einsum("jbc,jda,bcd->a", t2[:, J], ti.g_oovv[:, I], lam)
                # lambda_bcd^{ikl}: block = (i,k,l) -> output i = I
                Y1[I] -= torch.einsum("jbc,dja,bcd->a", t2[:, J], ti.g_voov[:, K], lam)
                # lambda_acd^{lkj}: block = (l,k,j)
                Y1 -= torch.einsum("bc,xdb,acd->xa", t2[K, J], ti.g_oovv[:, I], lam)
                # lambda_acd^{jkl}: block = (j,k,l)
                Y1 -= torch.einsum("bc,dxb,acd->xa", t2[I, J], ti.g_voov[:, K], lam)
                # lambda_cde^{kij}: block = (k,i,j) -> output i = J
                zb = torch.einsum("bc,cde->bde", t2[K, I], lam)
                Y1[J] += torch.einsum("bde,daeb->a", zb, ti.g_vvvv)
                # lambda_abc^{lmk}: block = (l,m,k)
                Y1 += torch.einsum("jbc,xj,abc->xa", t2[:, K], ti.g_oooo[:, I, :, J], lam)
                if want_density:
                    Dab += 0.5 * torch.einsum("bdc,adc->ab", t, lam)
                    Dia[I] += torch.einsum("abc,bc->a", t - t.permute(1, 0, 2), l2[J, K])
                    # - sum lambda_bcd^{jkl} t_il^cd t_kj^ab, block = (j,k,l)
                    zz = torch.einsum("bcd,xcd->bx", lam, t2[:, K])
                    Dia -= torch.einsum("bx,ab->xa", zz, t2[J, I])
            if want_density and tstack:
                # D_ij = -1/2 sum t_{ilk} lambda_{jlk}, here (l,k) = (J,K)
                ts = torch.stack(tstack)
                ls = torch.stack(lstack)
                Dij -= 0.5 * torch.einsum("iabc,jabc->ij", ts, ls)
    out = dict(X1=X1, X2=_perm_ijab(x2), Y1=Y1, Y2=_perm_ijab(y2))
    if want_density:
        out.update(Dij=Dij, Dab=Dab, Dia=Dia)
    return out


def triples_explicit(m: Model, ti: TriplesIntegrals, t2, l1, l2, want_density=False):
    t3 = t3_full(m, ti, t2)
    l3 = l3_full(m, ti, l1, l2)
    X1, X2 = x_full(ti, t3)
    Y1, Y2 = y_full(ti, t2, l2, t3, l3)
    out = dict(X1=X1, X2=X2, Y1=Y1, Y2=Y2, t3=t3, l3=l3)
    if want_density:
        Dij, Dab, Dia = density_triples_full(t2, l2, t3, l3)
        out.update(Dij=Dij, Dab=Dab, Dia=Dia)
    return out


# -----------------------------------------------------------------------------
# Right-hand side, density, dipole, RK4
# -----------------------------------------------------------------------------

_ONE = torch.ones((), dtype=C128)


def _holo_grad(L, inputs):
    """Holomorphic derivative dL/dz (torch returns its conjugate for grad_outputs = 1)."""
    gs = torch.autograd.grad(L, inputs, grad_outputs=_ONE)
    return [g.conj().resolve_conj() for g in gs]


def unpack(m: Model, y):
    o, v = m.o, m.v
    y = torch.as_tensor(np.asarray(y), dtype=C128)
    ov, oovv = o * v, o * o * v * v
    return (y[:ov].reshape(o, v), y[ov:ov + oovv].reshape(o, o, v, v),
            y[ov + oovv:2 * ov + oovv].reshape(o, v), y[2 * ov + oovv:].reshape(o, o, v, v))


def pack(t1, t2, l1, l2):
    return torch.cat([x.reshape(-1) for x in (t1, t2, l1, l2)])


def rhs_terms(m: Model, y, E, triples="loop", with_triples=True, with_density=True):
    """The separate pieces of the right-hand side at state y and field E.

    R1, R2: CCSD part of <mu|Hbar|0>; G1 = dL/dt1 and G2 = sym(dL/dt2)/C2 of
    the CCSD Lagrangian; X1, X2, Y1, Y2: triples contributions; D: the
    T1-frame one-electron density; mu: the dipole.
    """
    t1, t2, l1, l2 = unpack(m, y)
    t1v = t1.clone().requires_grad_(True)
    t2v = t2.clone().requires_grad_(True)
    d = Dressed(m, t1v, m.h(E))
    r1, r2 = ccsd_omega(d, t2v)
    L = ccsd_energy(d, t2v) + (l1 * r1).sum() + C2 * (l2 * r2).sum()
    g1, g2, gh = _holo_grad(L, [t1v, t2v, d.h])
    o, v = m.o, m.v
    out = dict(R1=r1.detach(), R2=r2.detach(), G1=g1, G2=0.5 * (g2 + g2.permute(1, 0, 3, 2)) / C2)
    with torch.no_grad():
        dd = Dressed(m, t1, m.h(E))
        if with_triples:
            ti = TriplesIntegrals(dd)
            fn = triples_loop if triples == "loop" else triples_explicit
            tri = fn(m, ti, t2, l1, l2, want_density=with_density)
            for k in ("X1", "X2", "Y1", "Y2"):
                out[k] = tri[k]
        else:
            tri = None
            out.update(X1=torch.zeros((o, v), dtype=C128), X2=torch.zeros((o, o, v, v), dtype=C128),
                       Y1=torch.zeros((o, v), dtype=C128), Y2=torch.zeros((o, o, v, v), dtype=C128))
        if with_density:
            D = gh.detach().clone()
            if tri is not None:
                D[:o, :o] += tri["Dij"]
                D[o:, o:] += tri["Dab"]
                D[:o, o:] += tri["Dia"]
            out["D"] = D
            out["mu"] = torch.stack([(D * dd.transform(m.mu[x])).sum() for x in range(3)])
    return out


def rhs(m: Model, y, E, triples="loop", with_dipole=False, with_triples=True):
    """dy/dt for y = (t1, t2, l1, l2) at field E (three Cartesian components).

    i dt/dt = Omega(t) + X(t3)                      (eq. cc3-rt-t)
    -i dl/dt = dL/dt, with the CCSD part of L differentiated automatically
               and the triples part from Y1, Y2     (eq. cc3-rt-l)
    The doubles pairing carries C2, so -i dl2/dt = sym(dL/dt2) / C2.
    """
    tm = rhs_terms(m, y, E, triples, with_triples, with_density=with_dipole)
    dy = pack(-1j * (tm["R1"] + tm["X1"]), -1j * (tm["R2"] + tm["X2"]),
              1j * (tm["G1"] + tm["Y1"]), 1j * (tm["G2"] + tm["Y2"]))
    if with_dipole:
        return dy, tm["mu"]
    return dy


def density_dressed(m: Model, y, E, triples="loop", with_triples=True):
    """One-electron density in the T1-transformed frame (coefficients of h~_pq)."""
    t1, t2, l1, l2 = unpack(m, y)
    t1v = t1.clone()
    d0 = Dressed(m, t1v, m.h(E))
    hl = d0.h.detach().clone().requires_grad_(True)
    # rebuild the Lagrangian with h~ as a leaf
    d0.h = hl
    Bd = torch.einsum("Pkk->P", d0.B[:, :m.o, :m.o])
    J = torch.einsum("Ppq,P->pq", d0.B, Bd)
    K = torch.einsum("Ppk,Pkq->pq", d0.B[:, :, :m.o], d0.B[:, :m.o, :])
    d0.F = hl + 2.0 * J - K
    r1, r2 = ccsd_omega(d0, t2)
    L = ccsd_energy(d0, t2) + (l1 * r1).sum() + C2 * (l2 * r2).sum()
    (D,) = _holo_grad(L, [hl])
    if with_triples:
        with torch.no_grad():
            ti = TriplesIntegrals(d0)
            fn = triples_loop if triples == "loop" else triples_explicit
            tri = fn(m, ti, t2, l1, l2, want_density=True)
        o = m.o
        D = D.clone()
        D[:o, :o] += tri["Dij"]
        D[o:, o:] += tri["Dab"]
        D[:o, o:] += tri["Dia"]
    return D, d0


def dipole(m: Model, y, E, triples="loop", with_triples=True):
    """mu_x = sum_pq D~_pq mu~^x_pq (Sec. 2.2.3), complex; D~, mu~ T1-transformed."""
    D, d0 = density_dressed(m, y, E, triples, with_triples)
    with torch.no_grad():
        return torch.stack([(D * d0.transform(m.mu[x])).sum() for x in range(3)])


def propagate(m: Model, y0, dt, field, steps=None, triples="loop", with_triples=True, callback=None):
    """Classic RK4 (Sec. 3) with the field sampled at t, t+dt/2, t+dt/2, t+dt.

    field: [(2*steps+1), 3] samples E(k dt / 2).  Returns (y_final, mu[steps+1, 3]).
    The dipole at t_n comes from the first stage of step n (same amplitudes and field).
    """
    field = np.asarray(field, dtype=np.float64)
    if steps is None:
        steps = (field.shape[0] - 1) // 2
    y = torch.as_tensor(np.asarray(y0), dtype=C128).clone()
    mus = []
    kw = dict(triples=triples, with_triples=with_triples)
    for n in range(steps):
        k1, mu = rhs(m, y, field[2 * n], with_dipole=True, **kw)
        mus.append(mu)
        k2 = rhs(m, y + 0.5 * dt * k1, field[2 * n + 1], **kw)
        k3 = rhs(m, y + 0.5 * dt * k2, field[2 * n + 1], **kw)
        k4 = rhs(m, y + dt * k3, field[2 * n + 2], **kw)
        y = y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if callback is not None:
            callback(n, y)
    mus.append(dipole(m, y, field[2 * steps], **kw))
    return y, torch.stack(mus)


def lagrangian(m: Model, y, E, triples="explicit", with_triples=True):
    """L = E + l1.(Omega1 + X1) + C2 l2.(Omega2 + X2) with t3 at its closed form."""
    t1, t2, l1, l2 = unpack(m, y)
    d = Dressed(m, t1, m.h(E))
    r1, r2 = ccsd_omega(d, t2)
    val = ccsd_energy(d, t2) + (l1 * r1).sum() + C2 * (l2 * r2).sum()
    if with_triples:
        ti = TriplesIntegrals(d)
        t3 = t3_full(m, ti, t2)
        X1, X2 = x_full(ti, t3)
        val = val + (l1 * X1).sum() + C2 * (l2 * X2).sum()
    return val


# -----------------------------------------------------------------------------
# Stationary (ground-state) amplitudes at a static field
# -----------------------------------------------------------------------------

def _diis(x0, step, tol, maxiter, nvec=8):
    """Fixed-point iteration x <- x + dx(x) with Pulay (DIIS) extrapolation over
    the last nvec iterates; stops when the residual norm reported by step is
    below tol.  step(x) returns (dx, residual max-norm)."""
    xs, es = [], []
    x = x0
    for it in range(maxiter):
        dx, res = step(x)
        if res < tol:
            return x, it
        xs.append(x + dx)
        es.append(dx)
        if len(xs) > nvec:
            xs.pop(0)
            es.pop(0)
        k = len(xs)
        if k < 2:
            x = xs[-1]
            continue
        Bm = np.zeros((k + 1, k + 1), dtype=np.complex128)
        for a in range(k):
            for b in range(k):
                Bm[a, b] = np.vdot(es[a], es[b])
        Bm[k, :k] = Bm[:k, k] = -1.0
        rhs_ = np.zeros(k + 1, dtype=np.complex128)
        rhs_[k] = -1.0
        try:
            c = np.linalg.solve(Bm, rhs_)[:k]
        except np.linalg.LinAlgError:
            c = np.zeros(k, dtype=np.complex128)
            c[-1] = 1.0
        x = sum(ci * xi for ci, xi in zip(c, xs))
    raise RuntimeError(f"ground state: no convergence in {maxiter} iterations (residual {res:.3e})")


def _denominators(m: Model):
    o = m.o
    eo, ev = m.eps[:o].numpy(), m.eps[o:].numpy()
    d1 = ev[None, :] - eo[:, None]
    d2 = (ev[None, None, :, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, :, None, None])
    return d1, d2


def ground_state(m: Model, E=(0.0, 0.0, 0.0), triples="explicit", with_triples=True, tol=1e-12, maxiter=300,
                 lam=True):
    """Stationary amplitudes of the field-free (or static-field) equations.

    The time derivatives of eq. cc3-rt-t and eq. cc3-rt-l vanish when
    Omega + X = 0 (the T equations) and dL/dt = G + Y = 0 (the Lambda
    equations).  Both are solved by Jacobi steps with the orbital-energy
    denominators (e_a - e_i, e_a + e_b - e_i - e_j) and DIIS, T first (it does
    not involve Lambda), then Lambda at the converged T.  The starting point is
    t = 0, lambda = 0.  Returns (y, energy) with the CC energy
    E = <0|H~|0> + sum t2 L of the T1-transformed Hamiltonian.
    """
    o, v = m.o, m.v
    ov, oovv = o * v, o * o * v * v
    d1, d2 = _denominators(m)
    dvec = np.concatenate([d1.ravel(), d2.ravel()])
    Eh = m.h(E)

    def t_step(x):
        t1 = torch.as_tensor(x[:ov].reshape(o, v))
        t2 = torch.as_tensor(x[ov:].reshape(o, o, v, v))
        with torch.no_grad():
            d = Dressed(m, t1, Eh)
            r1, r2 = ccsd_omega(d, t2)
            if with_triples:
                ti = TriplesIntegrals(d)
                if triples == "explicit":
                    X1, X2 = x_full(ti, t3_full(m, ti, t2))
                else:
                    z1 = torch.zeros_like(t1)
                    tri = triples_loop(m, ti, t2, z1, torch.zeros_like(t2))
                    X1, X2 = tri["X1"], tri["X2"]
                r1, r2 = r1 + X1, r2 + X2
        r = torch.cat([r1.reshape(-1), r2.reshape(-1)]).numpy()
        return -r / dvec, np.abs(r).max()

    xt, _ = _diis(np.zeros(ov + oovv, dtype=np.complex128), t_step, tol, maxiter)
    t1 = torch.as_tensor(xt[:ov].reshape(o, v))
    t2 = torch.as_tensor(xt[ov:].reshape(o, o, v, v))
    with torch.no_grad():
        energy = ccsd_energy(Dressed(m, t1, Eh), t2).item()
    if not lam:
        return pack(t1, t2, torch.zeros_like(t1), torch.zeros_like(t2)), energy

    def l_step(x):
        y = pack(t1, t2, torch.as_tensor(x[:ov].reshape(o, v)), torch.as_tensor(x[ov:].reshape(o, o, v, v)))
        tm = rhs_terms(m, y, E, triples=triples, with_triples=with_triples, with_density=False)
        r = torch.cat([(tm["G1"] + tm["Y1"]).reshape(-1), (tm["G2"] + tm["Y2"]).reshape(-1)]).numpy()
        return -r / dvec, np.abs(r).max()

    xl, _ = _diis(np.zeros(ov + oovv, dtype=np.complex128), l_step, tol, maxiter)
    y = pack(t1, t2, torch.as_tensor(xl[:ov].reshape(o, v)), torch.as_tensor(xl[ov:].reshape(o, o, v, v)))
    return y, energy


# -----------------------------------------------------------------------------
# Field-coupled triples: the CC3 Lagrangian with its field terms (App. A)
# -----------------------------------------------------------------------------
#
# With the field on, the triples block of L_CC3 is
#   <Lambda3| [H,T2] + [F + beta V, T3] + 1/2 [[beta V, T2], T2] |0>
# (V T1-transformed), so t3 and lambda3 have no closed form and are iterated
# (App. A, Sec. 2.1).  Reading: the field terms are taken from the commutators
# of the Euler-Lagrange equations; in amplitude form (pinned against the
# determinant-space commutators)
#   <mu3|[V,T3]|0>          = sum_d v_ad t_ijk^dbc + (b, c slots) - sum_l v_li t_ljk^abc - (j, k slots),
#   1/2 <mu3|[[V,T2],T2]|0> = -P_ijk^abc sum_ld v_ld t_ij^ad t_kl^cb,
# the second as printed in the spin-adapted t3, the first with the sign of
# every slot and the order of v's indices fixed by the commutator (the printed
# spin-adapted t3 and lambda3 disagree in these signs).
# lambda3 pairs with the triples residual as C3 sum lambda3 x3, C3 = 1/6
# (lambda_ijk^abc = <Lambda3|E_ai E_bj E_ck|0>).

C3 = 1.0 / 6.0


def vt3_full(v, t3, o):
    """<mu3|[V,T3]|0> for a one-electron operator v [n,n] (amplitude form)."""
    vv, oo = v[o:, o:], v[:o, :o]
    return (torch.einsum("ad,ijkdbc->ijkabc", vv, t3) + torch.einsum("bd,ijkadc->ijkabc", vv, t3)
            + torch.einsum("cd,ijkabd->ijkabc", vv, t3) - torch.einsum("li,ljkabc->ijkabc", oo, t3)
            - torch.einsum("lj,ilkabc->ijkabc", oo, t3) - torch.einsum("lk,ijlabc->ijkabc", oo, t3))


def vtt_full(v, t2, o):
    """1/2 <mu3|[[V,T2],T2]|0> (amplitude form)."""
    return -p3_full(torch.einsum("ld,ijad,klcb->ijkabc", v[:o, o:], t2, t2))


def _field_operator(m: Model, d: Dressed, E):
    """The T1-transformed dipole coupling V~ = (1 - T)(-E.mu)(1 + T)."""
    E = torch.as_tensor(np.asarray(E, dtype=np.float64)) if not torch.is_tensor(E) else E
    return d.transform(-torch.einsum("x,xpq->pq", E.to(C128), m.mu.to(C128)))


def _lagrangian_cc3(m: Model, t1, t2, l1, l2, t3, l3, E):
    """L_CC3 with the field terms of its triples block, at independent t3 and lambda3."""
    d = Dressed(m, t1, m.h(E) if not torch.is_tensor(E) else m.h0 - torch.einsum("x,xpq->pq", E, m.mu))
    r1, r2 = ccsd_omega(d, t2)
    ti = TriplesIntegrals(d)
    X1, X2 = x_full(ti, t3)
    v = _field_operator(m, d, E)
    o = m.o
    wp = (torch.einsum("ijae,ckbe->ijkabc", t2, ti.g_vovv) - torch.einsum("imab,mjck->ijkabc", t2, ti.g_oovo))
    x3 = p3_full(wp) - m.d3 * t3 + vt3_full(v, t3, o) + vtt_full(v, t2, o)
    return (ccsd_energy(d, t2) + (l1 * r1).sum() + C2 * (l2 * r2).sum() + (l1 * X1).sum() + C2 * (l2 * X2).sum()
            + C3 * (l3 * x3).sum())


def field_coupled_triples(m: Model, t1, t2, l1, l2, E, tol=1e-14, maxiter=200):
    """t3 and lambda3 of L_CC3 at field E by Jacobi iteration (App. A):
    t3 from dL/dlambda3 = 0, i.e. P W' - eps t3 + <mu3|[V,T3] + 1/2 [[V,T2],T2]|0> = 0
    (eps = -D), and lambda3 from the stationarity of L in t3 within the
    P(ijk/abc)-symmetric amplitudes, P(dL/dt3) = 0, linear in lambda3."""
    o = m.o
    with torch.no_grad():
        d = Dressed(m, t1, m.h(E))
        ti = TriplesIntegrals(d)
        v = _field_operator(m, d, E)
        src = p3_full(torch.einsum("ijae,ckbe->ijkabc", t2, ti.g_vovv)
                      - torch.einsum("imab,mjck->ijkabc", t2, ti.g_oovo)) + vtt_full(v, t2, o)
        t3 = src / m.d3
        for _ in range(maxiter):
            new = (src + vt3_full(v, t3, o)) / m.d3
            done = (new - t3).abs().max().item() <= tol * max(1.0, new.abs().max().item())
            t3 = new
            if done:
                break
        else:
            raise RuntimeError("field-coupled t3: no convergence")
    l3 = l3_full(m, TriplesIntegrals(Dressed(m, t1, m.h(E))), l1, l2).detach()
    for _ in range(maxiter):
        t3v = t3.clone().requires_grad_(True)
        (g,) = _holo_grad(_lagrangian_cc3(m, t1, t2, l1, l2, t3v, l3, E), [t3v])
        g = p3_full(g) / 6.0
        new = l3 - g / (C3 * (-m.d3))
        done = (new - l3).abs().max().item() <= tol * max(1.0, new.abs().max().item())
        l3 = new.detach()
        if done:
            break
    else:
        raise RuntimeError("field-coupled lambda3: no convergence")
    return t3, l3


def rhs_field_coupled(m: Model, y, E, with_dipole=False):
    """dy/dt from the Euler-Lagrange equations of L_CC3 with the field terms of
    its triples block (explicit six-index mode, tiny systems):
      i dt/dt   = Omega + X(t3),                t3 from field_coupled_triples,
      -i dl1/dt = dL/dt1,  -i dl2/dt = sym(dL/dt2)/C2   at fixed t3, lambda3,
    and optionally the dipole mu_x = -dL/dE_x at fixed amplitudes (Sec. 2.2.3)."""
    t1, t2, l1, l2 = unpack(m, y)
    t3, l3 = field_coupled_triples(m, t1, t2, l1, l2, E)
    t1v = t1.clone().requires_grad_(True)
    t2v = t2.clone().requires_grad_(True)
    Ev = torch.as_tensor(np.asarray(E, dtype=np.float64)).clone().requires_grad_(True)
    L = _lagrangian_cc3(m, t1v, t2v, l1, l2, t3, l3, Ev)
    g1, g2 = _holo_grad(L, [t1v, t2v])
    with torch.no_grad():
        d = Dressed(m, t1, m.h(E))
        r1, r2 = ccsd_omega(d, t2)
        X1, X2 = x_full(TriplesIntegrals(d), t3)
    G2 = 0.5 * (g2 + g2.permute(1, 0, 3, 2)) / C2
    dy = pack(-1j * (r1 + X1), -1j * (r2 + X2), 1j * g1, 1j * G2)
    if not with_dipole:
        return dy
    L = _lagrangian_cc3(m, t1, t2, l1, l2, t3, l3, Ev)
    gr = torch.autograd.grad(L.real, [Ev], retain_graph=True)[0]
    gi = torch.autograd.grad(L.imag, [Ev])[0]
    return dy, -(gr + 1j * gi)


def propagate_field_coupled(m: Model, y0, dt, field, steps=None):
    """Classic RK4 (Sec. 3) of rhs_field_coupled; returns (y_final, mu[steps+1, 3])."""
    field = np.asarray(field, dtype=np.float64)
    if steps is None:
        steps = (field.shape[0] - 1) // 2
    y = torch.as_tensor(np.asarray(y0), dtype=C128).clone()
    mus = []
    for n in range(steps):
        k1, mu = rhs_field_coupled(m, y, field[2 * n], with_dipole=True)
        mus.append(mu)
        k2 = rhs_field_coupled(m, y + 0.5 * dt * k1, field[2 * n + 1])
        k3 = rhs_field_coupled(m, y + 0.5 * dt * k2, field[2 * n + 1])
        k4 = rhs_field_coupled(m, y + dt * k3, field[2 * n + 2])
        y = (y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)).detach()
    mus.append(rhs_field_coupled(m, y, field[2 * steps], with_dipole=True)[1])
    return y, torch.stack(mus).detach()


# -----------------------------------------------------------------------------
# Derivatives along a direction (forward mode)
# -----------------------------------------------------------------------------

def rhs_tangent(m: Model, y, E, ydot, Edot, kdot=0.0, triples="explicit", with_triples=True, npts=16):
    """The right-hand side and the dipole at (y, E) and their derivatives along
    the direction (ydot, Edot, kdot), kdot being that of a scale of the dipole
    integrals, mu -> (1 + kappa) mu in the coupling -mu.E and in the dipole,
    taken at kappa = 0.

    Along s the right-hand side and the dipole,
        g(s) = (f, mu)(y + s ydot, (1 + s kdot)(E + s Edot)) * (1, 1 + s kdot),
    are polynomials (the amplitude equations and the density are polynomial in
    the amplitudes, and h is linear in the field), so the first Taylor
    coefficient g'(0) is the discrete Cauchy integral over the npts-th roots of
    unity, g'(0) = (1/npts) sum_k g(r w^k) / (r w^k), exact (up to rounding) when
    the degree is below npts + 1.  The radius r scales the direction to a
    perturbation of 0.1 in its largest component.

    Returns (dy, mu, dy_dot, mu_dot)."""
    y = torch.as_tensor(np.asarray(y), dtype=C128)
    ydot = torch.as_tensor(np.asarray(ydot), dtype=C128)
    E = np.asarray(E, dtype=np.float64)
    Edot = np.asarray(Edot, dtype=np.float64)
    size = max(float(ydot.abs().max()) if ydot.numel() else 0.0, float(np.abs(Edot).max()), abs(float(kdot)))
    if size == 0.0:
        dy, mu = rhs(m, y, E, triples=triples, with_dipole=True, with_triples=with_triples)
        return dy, mu, torch.zeros_like(dy), torch.zeros_like(mu)
    r = 0.1 / size
    acc_f, acc_mu = 0.0, 0.0
    for k in range(npts):
        z = r * np.exp(2j * np.pi * k / npts)
        Ez = (1.0 + z * kdot) * (E + z * Edot)
        f, mu = rhs(m, y + z * ydot, Ez, triples=triples, with_dipole=True, with_triples=with_triples)
        acc_f = acc_f + f / z
        acc_mu = acc_mu + (1.0 + z * kdot) * mu / z
    dy, mu = rhs(m, y, E, triples=triples, with_dipole=True, with_triples=with_triples)
    return dy, mu, acc_f / npts, acc_mu / npts


def propagate_tangent(m: Model, y0, dt, field, field_dot=None, kdot=0.0, ydot0=None, steps=None,
                      triples="explicit", with_triples=True, npts=16):
    """RK4 of propagate() together with its derivative along a direction of the
    inputs (field samples field_dot, dipole scale kdot, initial state ydot0):
    every stage's derivative is that of the right-hand side at the stage, so
    this is the exact derivative of the discrete propagation.

    Returns (y, ydot, mu[steps+1, 3], mu_dot[steps+1, 3])."""
    field = np.asarray(field, dtype=np.float64)
    if steps is None:
        steps = (field.shape[0] - 1) // 2
    fdot = np.zeros_like(field) if field_dot is None else np.asarray(field_dot, dtype=np.float64)
    y = torch.as_tensor(np.asarray(y0), dtype=C128).clone()
    yd = torch.zeros_like(y) if ydot0 is None else torch.as_tensor(np.asarray(ydot0), dtype=C128).clone()
    kw = dict(triples=triples, with_triples=with_triples, npts=npts)
    mus, mds = [], []
    for n in range(steps):
        k1, mu, k1d, mud = rhs_tangent(m, y, field[2 * n], yd, fdot[2 * n], kdot, **kw)
        mus.append(mu)
        mds.append(mud)
        k2, _, k2d, _ = rhs_tangent(m, y + 0.5 * dt * k1, field[2 * n + 1], yd + 0.5 * dt * k1d,
                                    fdot[2 * n + 1], kdot, **kw)
        k3, _, k3d, _ = rhs_tangent(m, y + 0.5 * dt * k2, field[2 * n + 1], yd + 0.5 * dt * k2d,
                                    fdot[2 * n + 1], kdot, **kw)
        k4, _, k4d, _ = rhs_tangent(m, y + dt * k3, field[2 * n + 2], yd + dt * k3d, fdot[2 * n + 2], kdot, **kw)
        y = y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        yd = yd + (dt / 6.0) * (k1d + 2.0 * k2d + 2.0 * k3d + k4d)
    _, mu, _, mud = rhs_tangent(m, y, field[2 * steps], yd, fdot[2 * steps], kdot, **kw)
    mus.append(mu)
    mds.append(mud)
    return y, yd, torch.stack(mus), torch.stack(mds)
