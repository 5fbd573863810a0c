"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and rejects bad arguments before it
touches the device."""
import os
import re

import numpy as np
import pytest

from paper_2407_18947_amd import _lib
from paper_2407_18947_amd.inputs import make_system

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rtcc3.h")).read()
    return sorted(set(re.findall(r"\b(rtcc3_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    L = _lib.load()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == names


def _sys():
    return make_system(2, 3, seed=1)


def test_create_rejects_bad_sizes():
    s = _sys()
    for o, v in [(0, 3), (2, 0)]:
        with pytest.raises(_lib.RTCC3Error) as e:
            _lib.rtcc3_create(o, v, s.fock, s.B, s.mu)
        assert e.value.code == _lib.RTCC3_EINVAL


def test_create_rejects_bad_inputs():
    s = _sys()
    f = s.fock.copy()
    f[0, 1] = 1e-3
    with pytest.raises(_lib.RTCC3Error) as e:
        _lib.rtcc3_create(2, 3, f, s.B, s.mu)
    assert e.value.code == _lib.RTCC3_EINVAL and "diagonal" in str(e.value)
    B = s.B.copy()
    B[0, 0, 1] += 1e-6
    with pytest.raises(_lib.RTCC3Error) as e:
        _lib.rtcc3_create(2, 3, s.fock, B, s.mu)
    assert "symmetric" in str(e.value)
    mu = s.mu.copy()
    mu[2, 3, 4] = np.nan
    with pytest.raises(_lib.RTCC3Error) as e:
        _lib.rtcc3_create(2, 3, s.fock, s.B, mu)
    assert "non-finite" in str(e.value)
    with pytest.raises(_lib.RTCC3Error):
        _lib.rtcc3_create(2, 3, s.fock, s.B, s.mu, precision=7)


def test_gemm_selftest_rejects_bad_sizes():
    L = _lib.load()
    assert L.rtcc3_zgemm_selftest(0, 1, 1, 0, None, None, None) == _lib.RTCC3_EINVAL
    assert L.rtcc3_zgemm_selftest(1, 1, 1, 5, None, None, None) == _lib.RTCC3_EINVAL
