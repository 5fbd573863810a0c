"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Element by element on seeded inputs, FP64 tolerance 1e-11 relative to the
largest element of each term (the oracle and the GPU sum in different orders;
FP64 rounding of o(1e3) terms per element stays near 1e-14).  Every case prints
its name before it touches the GPU.
"""
import numpy as np
import pytest
import torch

from oracle import rtcc3 as orc
from paper_2407_18947_amd import _lib
from paper_2407_18947_amd.inputs import initial_state, make_system

pytestmark = pytest.mark.gpu
FIELD = np.array([0.01, -0.02, 0.03])
TOL = 1e-11


def _say(msg):
    print(msg, flush=True)


def _random_state(o, v, seed, scale=0.1):
    rng = np.random.default_rng(seed)

    def rc(*sh):
        return scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))

    t1, l1 = rc(o, v), rc(o, v)
    t2, l2 = rc(o, o, v, v), rc(o, o, v, v)
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    l2 = 0.5 * (l2 + l2.transpose(1, 0, 3, 2))
    return np.concatenate([x.ravel() for x in (t1, t2, l1, l2)])


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


def _close(name, a, b, tol=TOL):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(1.0, np.abs(b).max())
    err = np.abs(a - b).max() if a.size else 0.0
    assert err <= tol * scale, f"{name}: max|diff| = {err:.3e} (scale {scale:.3e})"


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
                                 (16, 3), (17, 2)])
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


def test_trimer_size_sampled_elements():
    """Full workload size (o=15, v=57, the benchmark's windows and streams):
    the (i,j) = (0,0) blocks of X2 and Y2 against the oracle's triples loop over
    the blocks with second index 0, which are all that those elements depend on
    (after the P_ij^ab symmetrisation, X2_00^ab = x2_00^ab + x2_00^ba, where x2_{.0}
    collects blocks (.,0,.), and likewise Y2); both through the density pass
    (rtcc3_rhs_terms) and the plain right-hand side (rtcc3_rhs, dy = -i(Omega2 +
    X2), +i(G2 + Y2) for those elements)."""
    o, v = 15, 57
    _say(f"trimer-size sampled elements o={o} v={v}")
    s = make_system(o, v, seed=3)
    m = orc.Model.from_system(s)
    y = _random_state(o, v, 8, scale=0.02)
    E = np.array([0.001, -0.002, 0.002])
    g = _gpu_terms(s, y, E, 1)
    ctx = _lib.Context(s)
    yd = torch.tensor(y, dtype=torch.complex128, device="cuda")
    dy = torch.zeros_like(yd)
    torch.cuda.synchronize()
    _lib.rtcc3_rhs(ctx.ctx, E, yd, dy)
    dy = dy.cpu().numpy()
    ctx.close()
    with torch.no_grad():
        t1, t2, l1, l2 = orc.unpack(m, y)
        ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(E)))
        part = orc.triples_loop(m, ti, t2, l1, l2, want_density=False, max_blocks=o * o)
    ccsd = orc.rhs_terms(m, y, E, with_triples=False, with_density=False)
    X2, Y2 = part["X2"][0, 0].numpy(), part["Y2"][0, 0].numpy()
    _close("X2[0,0]", g["X2"][0, 0], X2)
    _close("Y2[0,0]", g["Y2"][0, 0], Y2)
    ov, oovv = o * v, o * o * v * v
    dt2 = dy[ov:ov + oovv].reshape(o, o, v, v)[0, 0]
    dl2 = dy[2 * ov + oovv:].reshape(o, o, v, v)[0, 0]
    _close("dt2[0,0]", dt2, -1j * (ccsd["R2"][0, 0].numpy() + X2))
    _close("dl2[0,0]", dl2, 1j * (ccsd["G2"][0, 0].numpy() + Y2))
