"""The taper's sine and cosine polynomials used by the FP64 node arithmetic.

csrc/taper_poly.h must be what paper_1910_01235_amd/taper_poly.py writes, and
the polynomials must reproduce sin z and cos z on |z| <= pi/2 (the taper's
range) to FP64 rounding."""
import math
import re

import numpy as np
import pytest

from paper_1910_01235_amd import taper_poly as TP

mp = pytest.importorskip("mpmath")


def _header():
    text = open(TP.HEADER).read()
    out = {}
    for name in ("kTaperS", "kTaperC"):
        body = re.search(name + r"\[\d+\] = \{([^}]*)\}", text).group(1)
        out[name] = [float(v) for v in body.split(",")]
    return out["kTaperS"], out["kTaperC"]


def test_header_is_the_generator_output():
    S, C = TP.fit()
    hs, hc = _header()
    assert hs == S and hc == C


def test_polynomials_reproduce_sine_and_cosine():
    S, C = _header()
    zs = np.concatenate([np.linspace(-math.pi / 2, math.pi / 2, 2001), [0.0, 1e-9, -1e-9]])
    mp.mp.dps = 30
    worst_s = worst_c = 0.0
    for z in zs:
        w = z * z
        ps = S[0]
        for c in S[1:]:
            ps = ps * w + c
        sinz = z * (1.0 - ps * w)
        pc = C[0]
        for c in C[1:]:
            pc = pc * w + c
        cosz = 1.0 + w * (-0.5 + pc * w)
        worst_s = max(worst_s, abs(float(mp.mpf(sinz) - mp.sin(mp.mpf(z)))))
        worst_c = max(worst_c, abs(float(mp.mpf(cosz) - mp.cos(mp.mpf(z)))))
    # a few ulp of 1 (Horner without fused multiply-adds in Python)
    assert worst_s < 4e-16 and worst_c < 4e-16, (worst_s, worst_c)
