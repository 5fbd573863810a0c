"""Seeded synthetic inputs for real-time CC3 runs.

This module holds no part of the RT-CC3 method: it draws orbital energies,
density-fitting factors and dipole matrices from a seed, builds the initial
amplitude state, and samples electric-field shapes on the RK4 half-step grid.
Both the CPU oracle and the GPU path take their inputs from here.

The integrals stand in for water-cluster double-zeta workloads (the paper's
timing study, Sec. 4.1, Table 1: monomer o=5, v=19; dimer and trimer scale by
2 and 3).  Real molecular integrals are not available, so a seeded generator
supplies the shapes and magnitudes:

* occupied orbital energies uniform in [-1.4, -0.4] Eh (sorted), virtual
  uniform in [0.15, 3.0] Eh (sorted);
* density-fitting factors B[P, p, q] (naux = 3 n), symmetric in (p, q),
  entries N(0, 0.05) scaled by exp(-0.3 |p - q|), giving
  (pq|rs) = sum_P B[P,p,q] B[P,r,s];
* dipole matrices mu[x, p, q] symmetric, entries N(0, 0.3).

Initial state: t1 = lambda1 = 0, t2 = MP2-like (ia|jb)/(e_i + e_j - e_a - e_b),
lambda2 = t2.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "System",
    "make_system",
    "initial_state",
    "state_size",
    "pack_state",
    "unpack_state",
    "random_state",
    "field_delta_kick",
    "field_gaussian_sine",
    "field_sine",
    "field_ramped_cw",
    "ramp_lrcw",
    "ramp_qrcw",
    "CONFIGS",
]


@dataclasses.dataclass
class System:
    """A closed-shell system: o occupied, v virtual orbitals, naux DF vectors."""

    o: int
    v: int
    naux: int
    eps: np.ndarray  # [n] orbital energies (canonical Fock diagonal)
    B: np.ndarray  # [naux, n, n] real, symmetric in the last two indices
    mu: np.ndarray  # [3, n, n] real symmetric dipole matrices
    seed: int

    @property
    def n(self) -> int:
        return self.o + self.v

    @property
    def fock(self) -> np.ndarray:
        return np.diag(self.eps)


def _sym_upper(z: np.ndarray) -> np.ndarray:
    """Keep the upper triangle (with diagonal) of the last two axes and mirror it."""
    up = np.triu(z)
    return up + np.swapaxes(np.triu(z, 1), -1, -2)


def make_system(o: int, v: int, seed: int, naux: int | None = None) -> System:
    if o < 1 or v < 1:
        raise ValueError("need o >= 1 and v >= 1")
    n = o + v
    if naux is None:
        naux = 3 * n
    rng = np.random.default_rng(seed)
    e_occ = np.sort(rng.uniform(-1.4, -0.4, size=o))
    e_vir = np.sort(rng.uniform(0.15, 3.0, size=v))
    eps = np.concatenate([e_occ, e_vir])
    p = np.arange(n)
    decay = np.exp(-0.3 * np.abs(p[:, None] - p[None, :]))
    z = rng.normal(0.0, 0.05, size=(naux, n, n)) * decay[None]
    B = _sym_upper(z)
    m = rng.normal(0.0, 0.3, size=(3, n, n))
    mu = _sym_upper(m)
    return System(o=o, v=v, naux=naux, eps=eps, B=np.ascontiguousarray(B),
                  mu=np.ascontiguousarray(mu), seed=seed)


def state_size(o: int, v: int) -> int:
    return 2 * (o * v + o * o * v * v)


def pack_state(t1, t2, l1, l2) -> np.ndarray:
    """Pack [t1 | t2 | l1 | l2] (row-major t1[i,a], t2[i,j,a,b]) into one c128 vector."""
    return np.concatenate([np.asarray(x, dtype=np.complex128).ravel() for x in (t1, t2, l1, l2)])


def unpack_state(y: np.ndarray, o: int, v: int):
    y = np.asarray(y)
    ov, oovv = o * v, o * o * v * v
    t1 = y[:ov].reshape(o, v)
    t2 = y[ov:ov + oovv].reshape(o, o, v, v)
    l1 = y[ov + oovv:2 * ov + oovv].reshape(o, v)
    l2 = y[2 * ov + oovv:].reshape(o, o, v, v)
    return t1, t2, l1, l2


def random_state(o: int, v: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """A seeded complex state (t1, t2, l1, l2) with entries scale * (N(0,1) + i N(0,1)),
    t2 and l2 symmetrised under (i,a) <-> (j,b); a generic point for comparing
    right-hand sides (not a physical state)."""
    rng = np.random.default_rng(seed)

    def rc(*sh):
        return scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))

    t1, l1 = rc(o, v), rc(o, v)
    t2, l2 = rc(o, o, v, v), rc(o, o, v, v)
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    l2 = 0.5 * (l2 + l2.transpose(1, 0, 3, 2))
    return pack_state(t1, t2, l1, l2)


def initial_state(sys: System) -> np.ndarray:
    """t1 = l1 = 0, t2 = (ia|jb)/(e_i+e_j-e_a-e_b), l2 = t2."""
    o, v = sys.o, sys.v
    Bov = sys.B[:, :o, o:]
    g_iajb = np.einsum("Pia,Pjb->iajb", Bov, Bov)
    eo, ev = sys.eps[:o], sys.eps[o:]
    d = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    t2 = np.transpose(g_iajb, (0, 2, 1, 3)) / d
    z1 = np.zeros((o, v))
    return pack_state(z1, t2, z1, t2)


# ----------------------------------------------------------------------------
# Field shapes sampled on the RK4 half-step grid: E[k] = E(k dt / 2), k = 0..2*steps
# ----------------------------------------------------------------------------

def _grid(steps: int, dt: float) -> np.ndarray:
    return 0.5 * dt * np.arange(2 * steps + 1)


def _axis(direction) -> np.ndarray:
    if isinstance(direction, str):
        d = np.zeros(3)
        d["xyz".index(direction)] = 1.0
        return d
    return np.asarray(direction, dtype=np.float64)


def field_delta_kick(steps: int, dt: float, amplitude: float = 0.002, direction="z") -> np.ndarray:
    """Constant field of the given amplitude for 0 <= t <= dt, zero afterwards.

    This stands in for the narrow Gaussian 'delta' pulse of the paper's
    computational details, whose width is below the RK4 sampling step.
    """
    t = _grid(steps, dt)
    e = np.where(t <= dt * (1 + 1e-12), amplitude, 0.0)
    return np.ascontiguousarray(e[:, None] * _axis(direction)[None, :])


def field_gaussian_sine(steps: int, dt: float, amplitude: float = 0.002, omega: float = 0.0656,
                        width: float = 5.0, center: float = 5.0, direction="z") -> np.ndarray:
    """A sin(omega t) exp(-(t - center)^2 / (2 width^2)) along one axis."""
    t = _grid(steps, dt)
    e = amplitude * np.sin(omega * t) * np.exp(-((t - center) ** 2) / (2 * width ** 2))
    return np.ascontiguousarray(e[:, None] * _axis(direction)[None, :])


def field_sine(steps: int, dt: float, amplitude: float = 0.001, omega: float = 0.0773, direction="x") -> np.ndarray:
    t = _grid(steps, dt)
    e = amplitude * np.sin(omega * t)
    return np.ascontiguousarray(e[:, None] * _axis(direction)[None, :])


def ramp_lrcw(t, t_r):
    """Linear ramp of the LRCW (Sec. 2.2.4): t / t_r for t < t_r, then 1."""
    t = np.asarray(t, dtype=np.float64)
    return np.where(t < t_r, t / t_r, 1.0)


def ramp_qrcw(t, t_r):
    """Quadratic ramp of the QRCW (Sec. 2.2.4): 2 t^2 / t_r^2 for t < t_r / 2,
    1 - 2 (t - t_r)^2 / t_r^2 for t_r / 2 <= t < t_r, then 1."""
    t = np.asarray(t, dtype=np.float64)
    up = 2.0 * t * t / (t_r * t_r)
    down = 1.0 - 2.0 * (t - t_r) ** 2 / (t_r * t_r)
    return np.where(t < 0.5 * t_r, up, np.where(t < t_r, down, 1.0))


def field_ramped_cw(steps: int, dt: float, amplitude: float, omega: float, kind: str = "qrcw", n_r: int = 1,
                    direction="z") -> np.ndarray:
    """A ramped continuous wave A F(t) cos(omega t) along one axis (Sec. 2.2.4), with
    the ramp over n_r optical cycles t_c = 2 pi / omega; kind 'lrcw' or 'qrcw'."""
    t = _grid(steps, dt)
    t_r = n_r * 2.0 * np.pi / omega
    ramp = {"lrcw": ramp_lrcw, "qrcw": ramp_qrcw}[kind](t, t_r)
    e = amplitude * ramp * np.cos(omega * t)
    return np.ascontiguousarray(e[:, None] * _axis(direction)[None, :])


# Workloads (sizes, seeds and fields).  Seeds follow the config index.
CONFIGS = {
    "monomer": dict(o=5, v=19, seed=1, field="delta", amplitude=0.002, direction="z", dt=0.05, steps=20),
    "dimer": dict(o=10, v=38, seed=2, field="gauss_sine", amplitude=0.002, direction="z", dt=0.05, steps=200),
    "trimer": dict(o=15, v=57, seed=3, field="delta", amplitude=0.002, direction="z", dt=0.05, steps=100),
    "pentamer": dict(o=25, v=95, seed=5, field="sine", amplitude=0.001, direction="x", dt=0.05, steps=50),
}


def config_field(name: str, steps: int | None = None) -> np.ndarray:
    c = CONFIGS[name]
    k = c["steps"] if steps is None else steps
    if c["field"] == "delta":
        return field_delta_kick(k, c["dt"], c["amplitude"], c["direction"])
    if c["field"] == "gauss_sine":
        return field_gaussian_sine(k, c["dt"], c["amplitude"], direction=c["direction"])
    if c["field"] == "sine":
        return field_sine(k, c["dt"], c["amplitude"], direction=c["direction"])
    raise KeyError(c["field"])
