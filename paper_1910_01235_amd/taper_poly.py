"""Writes csrc/taper_poly.h: near-minimax polynomials for the taper's sine and
cosine on |z| <= pi/2, in w = z^2,

    sin z = z (1 - w S(w)),    cos z = 1 + w (-1/2 + w C(w)),

with S of degree 7 and C of degree 6 (Chebyshev interpolation in mpmath at 40
digits). The fixed leading terms stay exact; the fitted remainders are accurate
to about 1e-18 (sine) and 6e-17 (cosine) in absolute terms.

    python -m paper_1910_01235_amd.taper_poly      # rewrites the header
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "csrc", "taper_poly.h")
DEG_SIN, DEG_COS = 7, 6


def fit():
    """(S, C) coefficient lists, highest degree first, as Python floats."""
    import mpmath as mp
    mp.mp.dps = 40
    W = (mp.pi / 2) ** 2

    def fS(w):
        if w < mp.mpf("1e-30"):
            return mp.mpf(1) / 6
        r = mp.sqrt(w)
        return (1 - mp.sin(r) / r) / w

    def fC(w):
        if w < mp.mpf("1e-30"):
            return mp.mpf(1) / 24
        return (mp.cos(mp.sqrt(w)) - 1 + w / 2) / w ** 2

    S = mp.chebyfit(fS, [0, W], DEG_SIN + 1)
    C = mp.chebyfit(fC, [0, W], DEG_COS + 1)
    return [float(c) for c in S], [float(c) for c in C]


def render(S, C) -> str:
    f = lambda v: ", ".join(repr(x) for x in v)
    return (
        "// Written by paper_1910_01235_amd/taper_poly.py; do not edit.\n"
        "// Taper sine and cosine on |z| <= pi/2 in w = z^2, highest degree first:\n"
        "//   sin z = z (1 - w S(w)),  cos z = 1 + w (-1/2 + w C(w)).\n"
        "#pragma once\n"
        f"constexpr double kTaperS[{len(S)}] = {{{f(S)}}};\n"
        f"constexpr double kTaperC[{len(C)}] = {{{f(C)}}};\n")


if __name__ == "__main__":
    S, C = fit()
    with open(HEADER, "w") as fh:
        fh.write(render(S, C))
    print(HEADER)
