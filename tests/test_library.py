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


def test_header_constants_match_binding():
    """Every enumerator the header defines has the same value in the binding."""
    txt = open(os.path.join(ROOT, "include", "rtcc3.h")).read()
    consts = {}
    for body in re.findall(r"enum\s*\{([^}]*)\}", txt):
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        for name, val in re.findall(r"\b(RTCC3_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            consts[name] = int(val)
    assert {"RTCC3_OK", "RTCC3_FP64", "RTCC3_OPT_WINDOW_BLOCKS", "RTCC3_OPT_SINGLE_STREAM"} <= set(consts)
    for name, val in consts.items():
        assert getattr(_lib, name) == val, name


def test_options_reject_null_context():
    L = _lib.load()
    for opt in (_lib.RTCC3_OPT_TRIPLES, _lib.RTCC3_OPT_PRECISION, _lib.RTCC3_OPT_WINDOW_BLOCKS,
                _lib.RTCC3_OPT_SINGLE_STREAM):
        assert L.rtcc3_set_option(None, opt, 1) == _lib.RTCC3_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stdout
