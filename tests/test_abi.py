"""The C-ABI library: it loads, exports every symbol include/rtcur.h
declares, validates arguments, and its host sampler reproduces the oracle's
index sets bit for bit (no device needed for any of this)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import paper_2108_10448_amd as rt
from oracle.sampler import draw_sample

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rt.LIB_PATH):
        from paper_2108_10448_amd.build import build
        build()
    return rt.lib()


def _declared():
    with open(os.path.join(ROOT, "include", "rtcur.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(rtcur_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "rtcur_solve" in names and len(names) >= 11
    for name in names:
        assert hasattr(L, name), name
    assert sorted(rt.SYMBOLS) == names


def test_create_without_device_reports_hip_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    out = ctypes.c_void_p(123)
    assert L.rtcur_create(ctypes.byref(out), 0, None, 0, 0) == rt.E_HIP
    assert out.value is None


def test_argument_checks_without_device(L):
    out = ctypes.c_void_p()
    assert L.rtcur_create(None, 0, None, 0, 0) == rt.E_INVAL
    assert L.rtcur_create(ctypes.byref(out), 0, None, 7, 0) == rt.E_INVAL
    assert L.rtcur_create(ctypes.byref(out), 0, None, 0, 9) == rt.E_INVAL
    assert L.rtcur_destroy(None) == rt.OK
    assert L.rtcur_solve(None, None, 0, 3, None, None, None, None, 0.0, 0.7, 1e-5,
                         10, 0, None) == rt.E_INVAL
    assert L.rtcur_reconstruct(None, None, 0) == rt.E_INVAL
    assert L.rtcur_outliers(None, None, 0, 0.0, None, None, 0) == rt.E_INVAL
    # batch: no handles, a null handle, a repeated handle
    assert L.rtcur_solve_batch(None, 1, 0, None, 0, None, None, None, None, None, None,
                               0.7, 1e-5, 10, None, None, 0, None, None) == rt.E_INVAL
    nul = (ctypes.c_void_p * 1)(None)
    assert L.rtcur_solve_batch(nul, 1, 0, None, 0, None, None, None, None, None, None,
                               0.7, 1e-5, 10, None, None, 0, None, None) == rt.E_INVAL
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: rejected as repeated
    two = (ctypes.c_void_p * 2)(fake, fake)
    assert L.rtcur_solve_batch(two, 2, 0, None, 0, None, None, None, None, None, None,
                               0.7, 1e-5, 10, None, None, 0, None, None) == rt.E_INVAL
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.rtcur_strerror(s)
    assert L.rtcur_strerror(99) == b"unknown status"


def test_sampler_bad_arguments(L):
    with pytest.raises(rt.RTCURError):
        rt.sample(0, 0, [10, 10], [11, 3], None, 0, 0)      # |I| > d
    with pytest.raises(rt.RTCURError):
        rt.sample(0, 0, [10, 10], [3, 3], [11, 3], 0, 1)    # |J| > prod
    with pytest.raises(rt.RTCURError):
        rt.sample(0, 0, [10], [3], None, 0, 0)              # n < 2


def test_library_sampler_matches_known_answers(L):
    with open(os.path.join(ROOT, "tests", "golden", "sampler_kat.json")) as f:
        cases = json.load(f)
    for c in cases:
        n = len(c["dims"])
        for i in range(n):
            got = rt.sample(c["seed"], c["t"], c["dims"], c["I_sizes"], c["J_sizes"], i, 0)
            assert got.tolist() == c["I"][i]
            if c["J_sizes"] is not None:
                got = rt.sample(c["seed"], c["t"], c["dims"], c["I_sizes"], c["J_sizes"], i, 1)
                assert got.tolist() == c["J_cols"][i]


@pytest.mark.parametrize("seed", [0, 1, 12345, 2 ** 63 + 5])
def test_library_sampler_matches_oracle(L, seed):
    for dims, I, J in [((300, 300, 300), (86, 86, 86), None),
                       ((40, 50, 60), (10, 11, 12), (30, 40, 50)),
                       ((7, 8, 9, 10), (3, 4, 5, 6), None),
                       ((7, 8, 9, 10), (3, 4, 5, 6), (20, 30, 40, 50))]:
        for t in (0, 1, 7):
            o = draw_sample(seed, t, dims, I, J)
            for i in range(len(dims)):
                assert np.array_equal(rt.sample(seed, t, dims, I, J, i, 0), o.I[i])
                assert np.array_equal(rt.sample(seed, t, dims, I, J, i, 1), o.J_cols[i])


def test_info_layout_matches_header(tmp_path):
    # the binding's rtcur_info mirror has the C header's size and offsets
    # (a C program built from include/rtcur.h prints them)
    import shutil
    import subprocess
    import paper_2108_10448_amd as rt
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = [f[0] for f in rt.RtcurInfo._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'printf("%zu ", offsetof(rtcur_info, {n}));' for n in names)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"rtcur.h\"\n"
                   "int main(void) {" + body + 'printf("%zu\\n", sizeof(rtcur_info)); return 0; }\n')
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(rt.RtcurInfo, n).offset for n in names] + [ctypes.sizeof(rt.RtcurInfo)]
    assert got == want
