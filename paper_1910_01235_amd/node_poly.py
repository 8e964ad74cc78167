"""Writes csrc/node_poly.h: near-minimax polynomials of the FP64 node arithmetic.

* Exponential on |r| <= ln2/2 (the reduction y = n + f, |f| <= 1/2, r = f ln2):
      e^r = 1 + r (1 + r (1/2 + r E(r))),   E of degree 8,
  relative error of e^r below 4e-17 (Taylor to degree 12 would leave 2.3e-16).
  The plan scales E to the base-2 form the kernels evaluate.
* Taper sine and cosine on |z| <= pi/2, in w = z^2:
      sin z = z (1 - w S(w)),   cos z = 1 + w (-1/2 + w C(w)),
  S of degree 7 and C of degree 6, absolute errors about 1e-18 and 6e-17.

The fixed leading terms stay exact; only the remainders E, S, C are fitted
(Chebyshev interpolation in mpmath at 40 digits), highest degree first.

    python -m paper_1910_01235_amd.node_poly      # rewrites the header
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "csrc", "node_poly.h")
DEG_EXP, DEG_SIN, DEG_COS = 8, 7, 6


def fit():
    """(E, S, C) coefficient lists, highest degree first, as Python floats."""
    import mpmath as mp
    mp.mp.dps = 40
    h = mp.log(2) / 2
    W = (mp.pi / 2) ** 2

    def fE(r):
        if abs(r) < mp.mpf("1e-12"):
            return mp.mpf(1) / 6 + r / 24
        return (mp.exp(r) - 1 - r - r * r / 2) / r ** 3

    def fS(w):
        if w < mp.mpf("1e-30"):
            return mp.mpf(1) / 6
        r = mp.sqrt(w)
        return (1 - mp.sin(r) / r) / w

    def fC(w):
        if w < mp.mpf("1e-30"):
            return mp.mpf(1) / 24
        return (mp.cos(mp.sqrt(w)) - 1 + w / 2) / w ** 2

    E = mp.chebyfit(fE, [-h, h], DEG_EXP + 1)
    S = mp.chebyfit(fS, [0, W], DEG_SIN + 1)
    C = mp.chebyfit(fC, [0, W], DEG_COS + 1)
    return [float(c) for c in E], [float(c) for c in S], [float(c) for c in C]


def render(E, S, C) -> str:
    f = lambda v: ", ".join(repr(x) for x in v)
    return (
        "// Written by paper_1910_01235_amd/node_poly.py; do not edit.\n"
        "// Remainder polynomials of the FP64 node arithmetic, highest degree first:\n"
        "//   e^r = 1 + r (1 + r (1/2 + r E(r))) on |r| <= ln2/2,\n"
        "//   sin z = z (1 - w S(w)),  cos z = 1 + w (-1/2 + w C(w)) on |z| <= pi/2, w = z^2.\n"
        "#pragma once\n"
        f"constexpr double kExpE[{len(E)}] = {{{f(E)}}};\n"
        f"constexpr double kTaperS[{len(S)}] = {{{f(S)}}};\n"
        f"constexpr double kTaperC[{len(C)}] = {{{f(C)}}};\n")


if __name__ == "__main__":
    E, S, C = fit()
    with open(HEADER, "w") as fh:
        fh.write(render(E, S, C))
    print(HEADER)
