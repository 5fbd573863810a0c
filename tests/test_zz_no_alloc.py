"""The allocation-free GEMM self-test (rtcc3_zgemm_selftest_noalloc) against the
allocating one, through the C ABI: the same arithmetic on the same operands, on
two calls in a row (the second smaller, so stale contents of the shared staging
area would show), and a size beyond the staging area rejected on the host."""
import numpy as np
import pytest

from paper_2407_18947_amd import _lib

pytestmark = pytest.mark.gpu


def _ops(M, N, K, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(K, N)) + 1j * rng.normal(size=(K, N))
    return A, B


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_matches_selftest_twice(prec):
    tol = {0: 1e-13, 1: 2e-6, 2: 4e-6}[prec]
    for M, N, K, seed in [(150, 90, 700, 1), (37, 20, 65, 2)]:
        print(f"noalloc zgemm {M}x{N}x{K} prec={prec}", flush=True)
        A, B = _ops(M, N, K, seed)
        ref = _lib.rtcc3_zgemm_selftest(A, B, prec)
        got = _lib.rtcc3_zgemm_selftest_noalloc(A, B, prec)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= tol * np.sqrt(K) * scale
        # and against the exact product at the precision's own bar
        assert np.abs(got - A @ B).max() <= tol * np.sqrt(K) * np.abs(A @ B).max()


def test_noalloc_rejects_oversize():
    A = np.zeros((2048, 1024), complex)
    B = np.zeros((1024, 2048), complex)
    with pytest.raises(_lib.RTCC3Error) as e:
        _lib.rtcc3_zgemm_selftest_noalloc(A, B, 0)
    assert e.value.code == _lib.RTCC3_EINVAL and "staging area" in str(e.value)
