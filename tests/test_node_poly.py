"""The remainder polynomials of the FP64 node arithmetic.

csrc/node_poly.h must be what paper_1910_01235_amd/node_poly.py writes, and the
polynomials must reproduce e^r on |r| <= ln2/2 (the range left by the
reduction y = n + f, r = f ln2; also in the base-2 form the kernels evaluate)
and sin z, cos z on |z| <= pi/2 (the taper's range) to FP64 rounding."""
import math
import re

import numpy as np
import pytest

from paper_1910_01235_amd import node_poly as NP

mp = pytest.importorskip("mpmath")


def _header():
    text = open(NP.HEADER).read()
    out = {}
    for name in ("kExpE", "kTaperS", "kTaperC"):
        body = re.search(name + r"\[\d+\] = \{([^}]*)\}", text).group(1)
        out[name] = [float(v) for v in body.split(",")]
    return out["kExpE"], out["kTaperS"], out["kTaperC"]


def test_header_is_the_generator_output():
    assert _header() == NP.fit()


def test_exponential_polynomial():
    E, _, _ = _header()
    h = math.log(2.0) / 2
    mp.mp.dps = 30
    worst = 0.0
    for r in np.concatenate([np.linspace(-h, h, 4001), [0.0, 1e-12, -1e-12]]):
        p = E[0]
        for c in E[1:]:
            p = p * r + c
        v = 1.0 + r * (1.0 + r * (0.5 + r * p))
        ex = mp.exp(mp.mpf(r))
        worst = max(worst, abs(float((mp.mpf(v) - ex) / ex)))
    # a few ulp (Horner without fused multiply-adds in Python)
    assert worst < 4e-16, worst


def test_base_two_form_of_the_exponential():
    """The kernels evaluate 2^f on |f| <= 1/2 as 1 + f (ln2 + f (ln2^2/2 + f E2(f)))
    with E2(f) = ln2^3 E(f ln2), the coefficients rounded from higher precision."""
    E, _, _ = _header()
    mp.mp.dps = 40
    ln2 = mp.log(2)
    deg = len(E) - 1
    E2 = [float(mp.mpf(c) * ln2 ** (deg - k + 3)) for k, c in enumerate(E)]
    l1, l2h = float(ln2), float(ln2 * ln2 / 2)
    worst = 0.0
    for f in np.concatenate([np.linspace(-0.5, 0.5, 4001), [0.0, 1e-12, -1e-12]]):
        p = E2[0]
        for c in E2[1:]:
            p = p * f + c
        v = 1.0 + f * (l1 + f * (l2h + f * p))
        ex = mp.power(2, mp.mpf(f))
        worst = max(worst, abs(float((mp.mpf(v) - ex) / ex)))
    assert worst < 4e-16, worst


def test_polynomials_reproduce_sine_and_cosine():
    _, S, C = _header()
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
