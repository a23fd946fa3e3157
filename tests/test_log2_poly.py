"""The FP32 logarithm of the point-cloud near field of FMM_FP32 plans
(Sec. 5.3: a polynomial fit of log2(x)/(x - 1)), host only.

* log2_poly.h is what gen_log2_poly.py writes (the table is generated, not
  hand-edited).
* The kernel's evaluation, emulated step by step in numpy float32 (exponent
  from the bits, mantissa folded into [1/sqrt(2), sqrt(2)), Horner's rule,
  one final multiply-add), against numpy's FP64 log2 over 240 binades:
  within 2.5e-7 of max(1, |log2 x|), i.e. a few FP32 units in the last place.
"""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_3339_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_log2_poly", os.path.join(CSRC, "gen_log2_poly.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _header_coefficients():
    txt = open(os.path.join(CSRC, "log2_poly.h")).read()
    body = txt[txt.index("kLog2Poly["):]
    return np.array([float(v) for v in re.findall(r"(-?\d\.\d+e[+-]\d+)f", body)], dtype=np.float32)


def test_header_is_generated():
    g = _gen()
    assert open(os.path.join(CSRC, "log2_poly.h")).read() == g.header_text(g.coefficients())


def _log2_poly(x, c):
    """The device function, in float32 arithmetic (fma emulated in float64 and rounded)."""
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32)
    e = (b >> 23).astype(np.int64) - 127
    m = ((b & np.uint32(0x007FFFFF)) | np.uint32(0x3F800000)).view(np.float32)
    big = m > np.float32(1.41421356)
    m = np.where(big, m * np.float32(0.5), m).astype(np.float32)
    e = e + big
    u = (m - np.float32(1.0)).astype(np.float32)
    p = np.full_like(u, c[-1])
    for ci in c[-2::-1]:
        p = (p.astype(np.float64) * u + np.float64(ci)).astype(np.float32)
    return (u.astype(np.float64) * p + e.astype(np.float64)).astype(np.float32)


def test_log2_poly_accuracy():
    c = _header_coefficients()
    assert len(c) == 9
    rng = np.random.default_rng(3)
    m = rng.uniform(1.0, 2.0, 200000)
    k = rng.integers(-120, 120, 200000)
    x = (m * np.exp2(k.astype(np.float64))).astype(np.float32)
    x = np.concatenate([x, np.float32([1.0, 2.0, 0.5, 1.41421356, 1.4142137, 0.70710677])])
    ref = np.log2(x.astype(np.float64))
    got = _log2_poly(x, c).astype(np.float64)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2.5e-7, err.max()
    # exact at powers of two
    assert np.all(_log2_poly(np.float32([1.0, 2.0, 0.5, 2.0 ** -40, 2.0 ** 70]), c)
                  == np.float32([0.0, 1.0, -1.0, -40.0, 70.0]))
