"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Element by element on seeded inputs, FP64 tolerance 1e-11 relative to the
largest element of each term (plus 1e-15 absolute, for terms that vanish
exactly in the oracle and leave rounding residue on the GPU): the oracle and
the GPU sum in different orders, and FP64 rounding of up to ~1e5 terms per
element stays near 1e-13 relative.  Full workload sizes are compared with
stored oracle values (tests/golden/make_golden.py, oracle only).  Every case
prints its name before it touches the GPU.
"""
import os
import re

import numpy as np
import pytest
import torch

from oracle import rtcc3 as orc
from paper_2407_18947_amd import _lib
from paper_2407_18947_amd.inputs import initial_state, make_system, random_state

pytestmark = pytest.mark.gpu
FIELD = np.array([0.01, -0.02, 0.03])
TOL = 1e-11
ATOL = 1e-15
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(msg, flush=True)


def _random_state(o, v, seed, scale=0.1):
    return random_state(o, v, seed, scale)


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_golden.py"
    return np.load(path)


def _gpu_terms(s, y, E, with_triples, precision=0, window_blocks=0):
    ctx = _lib.Context(s, precision)
    if window_blocks:
        ctx.set_option(_lib.RTCC3_OPT_WINDOW_BLOCKS, window_blocks)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    td = torch.zeros(ctx.terms_size(), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    _lib.rtcc3_rhs_terms(ctx.ctx, E, yd, td, with_triples)
    out = ctx.split_terms(td.cpu().numpy())
    ctx.close()
    return out


def _close(name, a, b, tol=TOL, atol=ATOL):
    """max|a - b| <= tol * max|b| + atol: relative to the term's largest element."""
    a, b = np.asarray(a), np.asarray(b)
    scale = np.abs(b).max() if b.size else 0.0
    err = np.abs(a - b).max() if a.size else 0.0
    assert err <= tol * scale + atol, f"{name}: max|diff| = {err:.3e} (largest element {scale:.3e})"


@pytest.mark.parametrize(
    "M,N,K",
    [(1, 1, 1), (17, 33, 5), (64, 64, 16), (100, 70, 129), (3, 200, 40),
     # narrow N (64x16 tiles), narrow M (transposed onto N), long K (split K)
     (70, 15, 300), (15, 70, 300), (16, 17, 64), (130, 3, 1000)],
)
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_zgemm_selftest(M, N, K, prec):
    _say(f"zgemm {M}x{N}x{K} prec={prec}")
    rng = np.random.default_rng(M * 1000 + N + K)
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(K, N)) + 1j * rng.normal(size=(K, N))
    C = _lib.rtcc3_zgemm_selftest(A, B, prec)
    ref = A @ B
    # unit roundoff of the operands times a small factor: FP64, FP32, three and
    # two bf16 slices (24 and 16 significand bits)
    tol = {0: 1e-13, 1: 2e-6, 2: 4e-6, 3: 2e-4}[prec]
    err = np.abs(C - ref)
    bad = np.nonzero(err.max(axis=1) > tol * np.sqrt(K) * max(1, np.abs(ref).max()))[0]
    assert bad.size == 0, f"rows with errors: {bad[:20].tolist()} max err {err.max():.3e}"


@pytest.mark.parametrize("M,N,K", [(64, 64, 16), (100, 70, 129), (70, 15, 300), (15, 70, 300), (130, 3, 1000)])
def test_zgemm_fp64_real_operands_stay_real(M, N, K):
    """FP64 forms a complex product from three real products, (Ar+Ai)Br,
    Ar(Bi-Br) and Ai(Br+Bi).  Real operands must still give an exactly real
    product, and an imaginary A times a real B an exactly imaginary one (the
    two products that cancel are the same numbers with opposite signs)."""
    _say(f"zgemm real/imaginary {M}x{N}x{K}")
    rng = np.random.default_rng(7 * M + N + K)
    Ar, Br = rng.normal(size=(M, K)), rng.normal(size=(K, N))
    C = _lib.rtcc3_zgemm_selftest(Ar.astype(complex), Br.astype(complex), 0)
    assert np.all(C.imag == 0.0), f"imaginary part {np.abs(C.imag).max():.3e}"
    _close("real x real", C.real, Ar @ Br, 1e-13 * np.sqrt(K))
    C = _lib.rtcc3_zgemm_selftest(1j * Ar, Br.astype(complex), 0)
    assert np.all(C.real == 0.0), f"real part {np.abs(C.real).max():.3e}"
    _close("imaginary x real", C.imag, Ar @ Br, 1e-13 * np.sqrt(K))


@pytest.mark.parametrize("o,v", [(2, 3), (3, 4), (5, 19)])
def test_ccsd_terms(o, v):
    _say(f"ccsd terms o={o} v={v}")
    s = make_system(o, v, seed=11)
    m = orc.Model.from_system(s)
    y = _random_state(o, v, 3)
    g = _gpu_terms(s, y, FIELD, 0)
    r = orc.rhs_terms(m, y, FIELD, with_triples=False)
    for k in ["R1", "R2", "G1", "G2", "D", "mu"]:
        _close(k, g[k], r[k].numpy())


@pytest.mark.parametrize("o,v", [(1, 4), (2, 3), (3, 4), (4, 7), (5, 19), (15, 10),
                                 # o = 16: X1 and Z by the separate sweep, D_ij on 16 rows;
                                 # o = 17: D_ij by the general product as well
                                 (16, 3), (17, 2),
                                 # v = 57 (rows padded to 64), v > 64 (two row tiles, padded
                                 # rows of 72 and 96 elements)
                                 (4, 57), (3, 70), (2, 96)])
def test_triples_terms(o, v):
    _say(f"triples terms o={o} v={v}")
    s = make_system(o, v, seed=12)
    m = orc.Model.from_system(s)
    y = _random_state(o, v, 4)
    g = _gpu_terms(s, y, FIELD, 1)
    r = orc.rhs_terms(m, y, FIELD, triples="explicit" if o * v < 40 else "loop")
    for k in ["X1", "X2", "Y1", "Y2", "D", "mu", "R1", "G2"]:
        _close(k, g[k], r[k].numpy())


@pytest.mark.parametrize("o,v,wb", [(3, 4, 6), (5, 19, 30), (15, 10, 400)])
def test_triples_terms_small_windows(o, v, wb):
    """A window cap below o^3 splits the density pass into pair windows (each
    holding the slabs of a few occupied pairs and owning part of their blocks)."""
    _say(f"triples terms o={o} v={v} window_blocks={wb}")
    s = make_system(o, v, seed=15)
    m = orc.Model.from_system(s)
    y = _random_state(o, v, 7)
    g = _gpu_terms(s, y, FIELD, 1, window_blocks=wb)
    r = orc.rhs_terms(m, y, FIELD, triples="explicit" if o * v < 40 else "loop")
    for k in ["X1", "X2", "Y1", "Y2", "D", "mu"]:
        _close(k, g[k], r[k].numpy())


@pytest.mark.parametrize("wb", [0, 6, 20])
def test_rhs_matches_oracle_windows(wb):
    """The right-hand side alone runs over windows of whole canonical triples;
    caps of 6 and 20 blocks give one or a few triples per window."""
    o, v = 4, 6
    _say(f"rhs o={o} v={v} window_blocks={wb}")
    s = make_system(o, v, seed=16)
    m = orc.Model.from_system(s)
    y = _random_state(o, v, 8)
    ctx = _lib.Context(s)
    if wb:
        ctx.set_option(_lib.RTCC3_OPT_WINDOW_BLOCKS, wb)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    dy = torch.zeros_like(yd)
    torch.cuda.synchronize()
    _lib.rtcc3_rhs(ctx.ctx, FIELD, yd, dy)
    ref = orc.rhs(m, y, FIELD, triples="explicit").numpy()
    _close("dy", dy.cpu().numpy(), ref)
    ctx.close()


def test_single_stream_matches_default():
    """With every kernel on one stream the terms are those of the default
    three-stream run (up to the order of atomic additions)."""
    o, v = 5, 9
    _say(f"single stream o={o} v={v}")
    s = make_system(o, v, seed=21)
    y = _random_state(o, v, 10)
    ref = _gpu_terms(s, y, FIELD, 1)
    ctx = _lib.Context(s)
    ctx.set_option(_lib.RTCC3_OPT_SINGLE_STREAM, 1)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    td = torch.zeros(ctx.terms_size(), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    _lib.rtcc3_rhs_terms(ctx.ctx, FIELD, yd, td, 1)
    got = ctx.split_terms(td.cpu().numpy())
    ctx.close()
    for name in ref:
        _close(name, got[name], ref[name], 1e-12)


def test_rhs_matches_oracle():
    o, v = 3, 5
    _say(f"rhs o={o} v={v}")
    s = make_system(o, v, seed=13)
    m = orc.Model.from_system(s)
    y = _random_state(o, v, 6)
    ctx = _lib.Context(s)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    dy = torch.zeros_like(yd)
    torch.cuda.synchronize()
    _lib.rtcc3_rhs(ctx.ctx, FIELD, yd, dy)
    ref = orc.rhs(m, y, FIELD, triples="explicit").numpy()
    _close("dy", dy.cpu().numpy(), ref)
    ctx.close()


def test_propagate_short_matches_oracle():
    o, v = 2, 5
    _say(f"propagate o={o} v={v}")
    s = make_system(o, v, seed=14)
    m = orc.Model.from_system(s)
    y0 = initial_state(s)
    f = np.zeros((7, 3))
    f[:3, 2] = 0.002
    ctx = _lib.Context(s)
    ctx.set_state(y0)
    mu = ctx.propagate(3, 0.05, f)
    yg = ctx.get_state()
    yr, mur = orc.propagate(m, y0, 0.05, f, triples="explicit")
    _close("mu", mu, mur.numpy(), 1e-12)
    _close("y", yg, yr.numpy(), 1e-12)
    ctx.close()


def test_monomer_dipole_series_matches_stored_oracle():
    """Monomer-sized workload (o=5, v=19, seed 1), delta kick 0.002 a.u. along z,
    dt = 0.05, 20 RK4 steps: the dipole series agrees with the stored oracle
    series (tests/golden/make_golden.py) to 1e-10 a.u."""
    import os

    from paper_2407_18947_amd.inputs import CONFIGS, config_field

    _say("monomer 20 steps")
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "monomer_20steps.npz"))
    c = CONFIGS["monomer"]
    s = make_system(c["o"], c["v"], seed=c["seed"])
    ctx = _lib.Context(s)
    ctx.set_state(initial_state(s))
    mu = ctx.propagate(c["steps"], c["dt"], config_field("monomer"))
    y = ctx.get_state()
    ctx.close()
    assert np.abs(mu - g["mu"]).max() < 1e-10, np.abs(mu - g["mu"]).max()
    assert np.abs(y - g["y"]).max() < 1e-9 * max(1, np.abs(g["y"]).max())


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_reduced_precision_dipole_within_target(prec):
    """The reduced-precision triples paths (FP32; bf16 split with three or two
    slices) on the monomer workload, 20 steps: the dipole series stays within
    1e-7 a.u. of the stored FP64 oracle series (the target for reduced
    precision), and within the error each form is expected to have."""
    import os

    from paper_2407_18947_amd.inputs import CONFIGS, config_field

    _say(f"monomer 20 steps precision {prec}")
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "monomer_20steps.npz"))
    c = CONFIGS["monomer"]
    s = make_system(c["o"], c["v"], seed=c["seed"])
    ctx = _lib.Context(s, prec)
    ctx.set_state(initial_state(s))
    mu = ctx.propagate(c["steps"], c["dt"], config_field("monomer"))
    ctx.close()
    err = np.abs(mu - g["mu"]).max()
    _say(f"  max dipole error {err:.3e}")
    assert err < {1: 1e-9, 2: 1e-9, 3: 1e-8}[prec], err
    assert err < 1e-7


def _rhs_dy(s, y, E):
    ctx = _lib.Context(s)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    dy = torch.zeros_like(yd)
    torch.cuda.synchronize()
    _lib.rtcc3_rhs(ctx.ctx, E, yd, dy)
    out = dy.cpu().numpy()
    ctx.close()
    return out


def _compare_terms_golden(name, o, v, seed, state_seed, scale):
    """Every term at a full workload size against the stored oracle values: X1, Y1,
    D, mu, R1, G1 in full and doubles rows of X2, Y2, R2, G2, through the density
    pass (rtcc3_rhs_terms); the same rows of dy through the plain right-hand side
    (rtcc3_rhs, which runs over windows of whole canonical triples)."""
    g = _golden(name)
    s = make_system(o, v, seed=seed)
    y = random_state(o, v, state_seed, scale)
    E = g["field"]
    t = _gpu_terms(s, y, E, 1)
    for k in ("X1", "Y1", "D", "mu", "R1", "G1"):
        _close(k, t[k], g[k])
    rows = [tuple(r) for r in g["rows"]]
    for k in ("X2", "Y2", "R2", "G2"):
        _close(k + " rows", np.stack([t[k][i, j] for i, j in rows]), g[k + "_rows"])
    dy = _rhs_dy(s, y, E)
    ov, oovv = o * v, o * o * v * v
    dt2 = dy[ov:ov + oovv].reshape(o, o, v, v)
    dl2 = dy[2 * ov + oovv:].reshape(o, o, v, v)
    _close("dt1", dy[:ov].reshape(o, v), -1j * (g["R1"] + g["X1"]))
    _close("dl1", dy[ov + oovv:2 * ov + oovv].reshape(o, v), 1j * (g["G1"] + g["Y1"]))
    _close("dt2 rows", np.stack([dt2[i, j] for i, j in rows]), -1j * (g["R2_rows"] + g["X2_rows"]))
    _close("dl2 rows", np.stack([dl2[i, j] for i, j in rows]), 1j * (g["G2_rows"] + g["Y2_rows"]))


def test_trimer_size_all_terms():
    """Full workload size (o=15, v=57, the benchmark's single window of all 3375
    blocks, both streams): every term against the oracle's loop over all blocks."""
    _say("trimer-size terms o=15 v=57")
    _compare_terms_golden("trimer_terms", 15, 57, 3, 8, 0.02)


def test_o17_v24_all_terms():
    """o = 17 > 16 at a realistic v: X1 and Z34 by the separate sweep, D_ij by the
    general product, column segments of more than 16 columns."""
    _say("terms o=17 v=24")
    _compare_terms_golden("o17v24_terms", 17, 24, 12, 4, 0.1)


def test_o16_v66_all_terms():
    """o = 16 > 15 with v = 66 > 64: the separate sweep for X1, the f~ term of X2 and
    Z34 over blocks wider than one wave (two 64-wide chunks of the unit-stride
    index), two row tiles in the products, padded rows of 72."""
    _say("terms o=16 v=66")
    _compare_terms_golden("o16v66_terms", 16, 66, 13, 5, 0.05)


def test_pentamer_size_sampled_elements():
    """o=25, v=95 (naux 360; v > 64 and o > 16: two row tiles, padded rows of 96,
    the separate X1 sweep with more than 64 virtuals, windows of whole canonical
    triples and pair windows for the density pass): X1[0], X2[0,0], Y2[0,0] and the
    CCSD parts against the stored oracle values (X1[0] depends only on the blocks
    with first occupied index 0, X2[0,0] and Y2[0,0] on those with second index 0)."""
    o, v = 25, 95
    _say(f"pentamer-size sampled elements o={o} v={v}")
    g = _golden("pentamer_sampled")
    s = make_system(o, v, seed=5)
    y = random_state(o, v, 9, 0.02)
    E = g["field"]
    dy = _rhs_dy(s, y, E)
    ov, oovv = o * v, o * o * v * v
    dt1 = dy[:ov].reshape(o, v)
    dt2 = dy[ov:ov + oovv].reshape(o, o, v, v)
    dl2 = dy[2 * ov + oovv:].reshape(o, o, v, v)
    # dt1[0] = -i (R1[0] + X1[0]); the Y1 of dl1 needs every block (not stored)
    _close("dt1[0]", dt1[0], -1j * (g["R1"][0] + g["X1_0"]))
    _close("dt2[0,0]", dt2[0, 0], -1j * (g["R2_00"] + g["X2_00"]))
    _close("dl2[0,0]", dl2[0, 0], 1j * (g["G2_00"] + g["Y2_00"]))
    # and the separate terms through the density pass
    t = _gpu_terms(s, y, E, 1)
    _close("X1[0]", t["X1"][0], g["X1_0"])
    _close("X2[0,0]", t["X2"][0, 0], g["X2_00"])
    _close("Y2[0,0]", t["Y2"][0, 0], g["Y2_00"])
    _close("R1", t["R1"], g["R1"])
    _close("G1", t["G1"], g["G1"])


def test_dimer_dipole_series_matches_stored_oracle():
    """Dimer workload (o=10, v=38, seed 2, sine field with a Gaussian envelope along
    z, dt = 0.05): the first 30 RK4 steps' dipole series agrees with the stored
    oracle series to 1e-10 a.u., and the final amplitudes agree."""
    from paper_2407_18947_amd.inputs import CONFIGS, config_field

    _say("dimer 30 steps")
    g = _golden("dimer_30steps")
    c = CONFIGS["dimer"]
    steps = int(g["steps"])
    s = make_system(c["o"], c["v"], seed=c["seed"])
    ctx = _lib.Context(s)
    ctx.set_state(initial_state(s))
    mu = ctx.propagate(steps, c["dt"], config_field("dimer", steps))
    y = ctx.get_state()
    ctx.close()
    err = np.abs(mu - g["mu"]).max()
    _say(f"  max dipole difference {err:.3e}")
    assert err < 1e-10, err
    assert np.abs(y - g["y"]).max() < 1e-9 * max(1, np.abs(g["y"]).max())


@pytest.mark.parametrize("prec", [1, 2])
def test_dimer_reduced_precision_dipole_within_target(prec):
    """The FP32 and bf16x3 triples paths on the dimer workload (30 steps): dipole
    series within 1e-7 a.u. of the stored FP64 oracle series."""
    from paper_2407_18947_amd.inputs import CONFIGS, config_field

    _say(f"dimer 30 steps precision {prec}")
    g = _golden("dimer_30steps")
    c = CONFIGS["dimer"]
    steps = int(g["steps"])
    s = make_system(c["o"], c["v"], seed=c["seed"])
    ctx = _lib.Context(s, prec)
    ctx.set_state(initial_state(s))
    mu = ctx.propagate(steps, c["dt"], config_field("dimer", steps))
    ctx.close()
    err = np.abs(mu - g["mu"]).max()
    _say(f"  max dipole error {err:.3e}")
    assert err < 1e-7, err


def test_divergence_keeps_last_finite_state():
    """An absurd step makes the amplitudes overflow (non-finite numbers, not a
    fault): rtcc3_propagate returns EDIVERGED, the dipoles up to the last finite
    state are finite and the later ones NaN, and the state is the last finite one,
    equal to a propagation stopped right there."""
    o, v = 2, 3
    _say(f"divergence o={o} v={v}")
    s = make_system(o, v, seed=17)
    y0 = initial_state(s)
    # the oracle overflows to NaN in the second step of this propagation
    steps, dt = 6, 40.0
    f = np.zeros((2 * steps + 1, 3))
    f[:3, 2] = 0.5
    ctx = _lib.Context(s)
    ctx.set_state(y0)
    with pytest.raises(_lib.RTCC3Error) as e:
        ctx.propagate(steps, dt, f)
    assert e.value.code == _lib.RTCC3_EDIVERGED
    kept = int(re.search(r"left after (\d+) steps", str(e.value)).group(1))
    assert 0 <= kept < steps
    mu = ctx.last_dipoles
    assert np.isnan(mu[kept + 1:]).all()
    y_div = ctx.get_state()
    assert np.isfinite(y_div).all()
    ctx.close()
    ref = _lib.Context(s)
    ref.set_state(y0)
    mu_ref = ref.propagate(kept, dt, f[: 2 * kept + 1]) if kept > 0 else None
    y_ref = ref.get_state()
    ref.close()
    _close("state", y_div, y_ref, 1e-12)
    if kept > 0:
        _close("dipoles", mu[:kept], mu_ref[:kept], 1e-12)


def test_no_device_allocation_after_create():
    """Everything a context needs is allocated in rtcc3_create: propagation,
    right-hand sides, terms and dipoles leave the device's free memory unchanged."""
    o, v = 5, 19
    _say(f"allocation o={o} v={v}")
    s = make_system(o, v, seed=18)
    ctx = _lib.Context(s)
    ctx.set_state(initial_state(s))
    yd = torch.tensor(_random_state(o, v, 3), dtype=torch.complex128, device="cuda")
    dy = torch.zeros_like(yd)
    td = torch.zeros(ctx.terms_size(), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    f = np.zeros((2 * 3 + 1, 3))
    f[:3, 2] = 0.002
    ctx.propagate(3, 0.05, f)
    _lib.rtcc3_rhs(ctx.ctx, FIELD, yd, dy)
    _lib.rtcc3_rhs_terms(ctx.ctx, FIELD, yd, td, 1)
    ctx.dipole(FIELD)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    ctx.close()
    assert free1 == free0, (free0, free1)


def test_two_electron_dynamic_polarisability_matches_sum_over_states():
    """End to end on the GPU: two electrons (o = 1, v = 3, where RT-CC3 is exact),
    QRCW fields of +-A, +-2A at w = 0.3 (one ramped, one fitted cycle), alpha_zz(w)
    from the four-point formula and the cosine fit (Sec. 2.2.2) against the
    sum-over-states polarisability of the same Hamiltonian in determinant space."""
    from fci_harness import FockSpace
    from paper_2407_18947_amd import properties as P
    from paper_2407_18947_amd.inputs import field_ramped_cw

    o, v = 1, 3
    _say(f"dynamic polarisability o={o} v={v}")
    s = make_system(o, v, seed=46)
    m = orc.Model.from_system(s)
    fs = FockSpace(o, v)
    g = np.einsum("Ppq,Prs->pqrs", s.B, s.B).astype(complex)
    H0 = fs.hamiltonian(m.h0.numpy().astype(complex), g).toarray()
    M = fs.one_body(s.mu[2].astype(complex)).toarray()
    E, U = np.linalg.eigh(H0)
    k0 = int(np.argmax(np.abs(U.T.conj() @ fs.ref)))
    wn = E - E[k0]
    dn = U.T.conj() @ (M @ U[:, k0])
    w = 0.3
    exc = np.arange(len(E)) != k0
    alpha_sos = np.sum(2 * wn[exc] * np.abs(dn[exc]) ** 2 / (wn[exc] ** 2 - w * w))
    y0, _ = orc.ground_state(m)
    dt, A = 0.05, 0.001
    t_c = 2 * np.pi / w
    steps = int(round(2 * t_c / dt))
    ctx = _lib.Context(s)
    mus = []
    for k in (1, -1, 2, -2):
        ctx.set_state(y0.numpy())
        mus.append(ctx.propagate(steps, dt, field_ramped_cw(steps, dt, k * A, w, kind="qrcw", n_r=1))[:, 2].real)
    ctx.close()
    mu1 = P.finite_field_mu1(*mus, A)
    alpha, r2 = P.fit_alpha(dt * np.arange(steps + 1), mu1, w, t_start=t_c)
    _say(f"  alpha {alpha:.8f}  sum over states {alpha_sos:.8f}  R^2 {r2:.6f}")
    assert r2 > 0.999
    assert abs(alpha - alpha_sos) < 1e-3 * abs(alpha_sos)
