"""Write tests/golden/psi_coeffs.json from the oracle's 50-digit solver only.

Usage: python tests/golden/make_psi_golden.py
The stored coefficients let the GPU library's own coefficient setup be
checked without re-running the 50-digit solve.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import psi  # noqa: E402

CASES = [("galerkin", a) for a in (0.3, 0.4, 0.45, 0.5, 0.55, 0.6, 0.7)] + \
        [("uniform", a) for a in (0.3, 0.5, 0.7, 0.9)] + \
        [("momentum", a) for a in (0.3, 0.5, 0.7)]


def main():
    out = []
    for interp, alpha in CASES:
        a, b, ident = psi.psi_coeffs(interp, alpha)
        out.append(dict(interp=interp, alpha=alpha, psi_e=[repr(v) for v in a],
                        psi_b=[repr(v) for v in b], identity=ident,
                        positive=psi.psi_positive(a, b)))
    doc = {"source": "oracle/psi.py, 50-digit rational interpolation, nodes j/8, b0 = 1",
           "cases": out}
    with open(os.path.join(HERE, "psi_coeffs.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
