"""Determinant-space (second-quantized) reference for tiny closed-shell systems.

Independent of the oracle: it builds creation/annihilation operators as sparse
matrices over all N-electron determinants of 2n spin orbitals, the
unitary-group generators E_pq = a+_{p alpha} a_{q alpha} + a+_{p beta} a_{q beta}
(App. A), the spin-free Hamiltonian

    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps)

and cluster operators T1 = sum t_i^a E_ai, T2 = 1/2 sum t_ij^ab E_ai E_bj,
T3 = 1/6 sum t_ijk^abc E_ai E_bj E_ck (eq. cc3-T1 .. cc3-T3).  Everything else
(similarity transforms, projections, expectation values) is plain linear
algebra on these matrices.  Intended for n <= 7 orbitals.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np
import scipy.sparse as sp


class FockSpace:
    def __init__(self, o: int, v: int):
        self.o, self.v = o, v
        self.n = n = o + v
        self.nso = 2 * n  # spin orbital p_alpha = p, p_beta = n + p
        nel = 2 * o
        dets = []
        for occ in itertools.combinations(range(self.nso), nel):
            m = 0
            for q in occ:
                m |= 1 << q
            dets.append(m)
        self.dets = np.array(dets, dtype=np.int64)
        self.index = {int(d): k for k, d in enumerate(self.dets)}
        self.dim = len(dets)
        ref = 0
        for i in range(o):
            ref |= (1 << i) | (1 << (n + i))
        self.ref = np.zeros(self.dim, dtype=np.complex128)
        self.ref[self.index[ref]] = 1.0
        # excitation rank = number of electrons in virtual spin orbitals
        vmask = 0
        for a in range(o, n):
            vmask |= (1 << a) | (1 << (n + a))
        self.rank = np.array([bin(int(d) & vmask).count("1") for d in self.dets])
        self._E = {}

    def _cre_ann(self, p: int, q: int):
        """a+_p a_q on spin orbitals."""
        rows, cols, vals = [], [], []
        for k, d in enumerate(self.dets):
            d = int(d)
            if not (d >> q) & 1:
                continue
            s = bin(d & ((1 << q) - 1)).count("1")
            d1 = d & ~(1 << q)
            if (d1 >> p) & 1:
                continue
            s += bin(d1 & ((1 << p) - 1)).count("1")
            d2 = d1 | (1 << p)
            rows.append(self.index[d2])
            cols.append(k)
            vals.append(-1.0 if s % 2 else 1.0)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim), dtype=np.complex128)

    def E(self, p: int, q: int):
        key = (p, q)
        if key not in self._E:
            n = self.n
            self._E[key] = (self._cre_ann(p, q) + self._cre_ann(n + p, n + q)).tocsr()
        return self._E[key]

    # ------------------------------------------------------------------ operators
    def hamiltonian(self, h, g):
        """Spin-free H for arbitrary (possibly non-symmetric, complex) h, g."""
        n = self.n
        H = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
        for p in range(n):
            for q in range(n):
                if h[p, q] != 0:
                    H = H + h[p, q] * self.E(p, q)
        for p in range(n):
            for q in range(n):
                G = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
                for r in range(n):
                    for s in range(n):
                        if g[p, q, r, s] != 0:
                            G = G + g[p, q, r, s] * self.E(r, s)
                H = H + 0.5 * (self.E(p, q) @ G)
        for p in range(n):
            for s in range(n):
                c = sum(g[p, q, q, s] for q in range(n))
                if c != 0:
                    H = H - 0.5 * c * self.E(p, s)
        return H.tocsr()

    def one_body(self, x):
        n = self.n
        M = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
        for p in range(n):
            for q in range(n):
                if x[p, q] != 0:
                    M = M + x[p, q] * self.E(p, q)
        return M.tocsr()

    def T1(self, t1):
        o, v = self.o, self.v
        M = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
        for i in range(o):
            for a in range(v):
                M = M + t1[i, a] * self.E(o + a, i)
        return M.tocsr()

    def T2(self, t2):
        o, v = self.o, self.v
        M = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
        for i, j in itertools.product(range(o), repeat=2):
            for a, b in itertools.product(range(v), repeat=2):
                c = t2[i, j, a, b]
                if c != 0:
                    M = M + 0.5 * c * (self.E(o + a, i) @ self.E(o + b, j))
        return M.tocsr()

    # ---------------------------------------------------------------- vectors
    def expm_apply(self, T, x, sign=1.0):
        """exp(sign T) x for a nilpotent excitation operator T (series terminates)."""
        out = x.copy()
        term = x.copy()
        for k in range(1, 4 * self.o + 3):
            term = sign * (T @ term) / k
            if not np.any(term):
                break
            out = out + term
        return out

    @lru_cache(maxsize=None)
    def singles_basis(self):
        o, v = self.o, self.v
        cols = [self.E(o + a, i) @ self.ref for i in range(o) for a in range(v)]
        return np.stack(cols, axis=1)

    @lru_cache(maxsize=None)
    def doubles_basis(self):
        """Columns 1/2 E_ai E_bj |0> in the order (i,j,a,b)."""
        o, v = self.o, self.v
        cols = []
        for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
            cols.append(0.5 * (self.E(o + a, i) @ (self.E(o + b, j) @ self.ref)))
        return np.stack(cols, axis=1)

    @lru_cache(maxsize=None)
    def triples_basis(self):
        """Columns E_ai E_bj E_ck |0> in the order (i,j,k,a,b,c)."""
        o, v = self.o, self.v
        cols = []
        for i, j, k, a, b, c in itertools.product(range(o), range(o), range(o), range(v), range(v), range(v)):
            cols.append(self.E(o + a, i) @ (self.E(o + b, j) @ (self.E(o + c, k) @ self.ref)))
        return np.stack(cols, axis=1)

    def project_rank(self, x, r):
        y = x.copy()
        y[self.rank != r] = 0.0
        return y

    def coefficients(self, x):
        """Expansion coefficients (omega1[i,a], omega2[i,j,a,b]) of the rank-1/2 parts of x
        in {E_ai|0>, 1/2 E_ai E_bj|0>}, with omega2 symmetric under (ia)<->(jb)."""
        o, v = self.o, self.v
        x1 = self.project_rank(x, 1)
        x2 = self.project_rank(x, 2)
        w1, *_ = np.linalg.lstsq(self.singles_basis(), x1, rcond=None)
        w2, *_ = np.linalg.lstsq(self.doubles_basis(), x2, rcond=None)
        r1 = np.linalg.norm(self.singles_basis() @ w1 - x1)
        r2 = np.linalg.norm(self.doubles_basis() @ w2 - x2)
        assert r1 < 1e-10 * max(1.0, np.linalg.norm(x1)) and r2 < 1e-10 * max(1.0, np.linalg.norm(x2))
        return w1.reshape(o, v), w2.reshape(o, o, v, v)

    def bra_from_lambda(self, l1, l2, c2):
        """The functional <Lambda| on rank 1 and 2 with <Lambda|X> = sum l1 x1 + c2 sum l2 x2,
        where |X> = sum x1 E_ai|0> + 1/2 sum x2 E_ai E_bj|0> (x2 symmetric)."""
        S = self.singles_basis()
        D = self.doubles_basis()
        b1 = np.linalg.pinv(S).T @ l1.ravel()
        b2 = np.linalg.pinv(D).T @ (c2 * l2.ravel())
        # bras as row vectors: <Lambda|y> = b . y  (no conjugation)
        return b1 + b2

    def energy_denominators(self, eps):
        """Orbital-energy excitation energy of each determinant relative to |0>."""
        n = self.n
        e = np.zeros(self.dim)
        e0 = 2.0 * np.sum(eps[: self.o])
        for k, d in enumerate(self.dets):
            d = int(d)
            s = 0.0
            for p in range(n):
                s += eps[p] * (((d >> p) & 1) + ((d >> (n + p)) & 1))
            e[k] = s - e0
        return e


def mulliken_from_B(B):
    return np.einsum("Ppq,Prs->pqrs", B, B)


def dress_integrals(o, v, t1, h, B):
    """h~ = (1 - T) h (1 + T), B~ = (1 - T) B (1 + T), T[a,i] = t_i^a (stand-alone copy)."""
    n = o + v
    T = np.zeros((n, n), dtype=np.complex128)
    T[o:, :o] = t1.T
    X = np.eye(n) - T
    Y = np.eye(n) + T
    ht = X @ h @ Y
    Bt = np.einsum("pr,Prs,sq->Ppq", X, B, Y)
    return ht, np.einsum("Ppq,Prs->pqrs", Bt, Bt)
