"""Write the golden fixtures in this folder from the closed forms printed in the paper.

Each fixture evaluates one printed formula of Maranville, "An implementation of
an efficient direct Fourier transform of polygonal areas and volumes", at fixed
parameters. Nothing here calls the oracle or the library. Run:
    python tests/golden/make_golden.py
"""
import json
import math
import os

import numpy as np
from scipy.special import gamma, jv

HERE = os.path.dirname(os.path.abspath(__file__))


def c2l(z):
    return [[float(np.real(x)), float(np.imag(x))] for x in np.atleast_1d(z)]


def rectangle():
    """Section 'Transform of a rectangle': eq. rectangle_integral and the four edge terms of eq. rectangle_sum."""
    a, b = 1.7, 0.6
    qs = [(0.9, -1.3), (2.5, 0.4), (-3.1, -2.2), (0.05, 4.0)]
    rows = []
    for qx, qy in qs:
        Q2 = qx * qx + qy * qy
        e = lambda x: np.exp(1j * x)  # noqa: E731
        # edge terms as printed (counter-clockwise from the origin corner)
        t1 = (1 / Q2) * (qy * a) / (qx * a) * (e(qx * a) - e(0.0))
        t2 = (1 / Q2) * (-qx * b) / (qy * b) * (e(qx * a + qy * b) - e(qx * a))
        t3 = (1 / Q2) * (-qy * a) / (-qx * a) * (e(qy * b) - e(qx * a + qy * b))
        t4 = (1 / Q2) * (qx * b) / (-qy * b) * (e(0.0) - e(qy * b))
        direct = -1.0 / (qx * qy) * (e(qx * a) - 1) * (e(qy * b) - 1)
        ft_rect = (1 / Q2) * (qx * qx + qy * qy) / (qx * qy) * (e(qy * b) + e(qx * a) - e(qx * a + qy * b) - 1)
        rows.append({"q": [qx, qy], "edge_terms": c2l([t1, t2, t3, t4]), "integral": c2l(direct)[0],
                     "ft_rect": c2l(ft_rect)[0]})
    return {"citation": "paper, section 'Transform of a rectangle': eq. rectangle_integral, eq. rectangle_sum "
                        "(edge terms) and the FT_Rect expression",
            "a": a, "b": b, "rows": rows}


def prism():
    """Section 'Rectangular prism': eq. prism_direct and the top / bottom face terms I_{z=c}, I_{z=0}."""
    a, b, c = 1.1, 0.8, 1.4
    qs = [(0.7, -1.9, 1.2), (2.3, 0.6, -0.4), (-1.5, -2.5, 3.0)]
    rows = []
    for qx, qy, qz in qs:
        Q2 = qx * qx + qy * qy + qz * qz
        e = lambda x: np.exp(1j * x)  # noqa: E731
        xy = (e(qx * a) - 1) * (e(qy * b) - 1) / (qx * qy)
        top = 1j * qz * e(qz * c) / Q2 * xy
        bottom = -1j * qz / Q2 * xy
        direct = 1j * (e(qx * a) - 1) * (e(qy * b) - 1) * (e(qz * c) - 1) / (qx * qy * qz)
        rows.append({"q": [qx, qy, qz], "I_top": c2l(top)[0], "I_bottom": c2l(bottom)[0],
                     "integral": c2l(direct)[0]})
    return {"citation": "paper, section 'Rectangular prism': eq. prism_direct and the face terms I_{z=c}, I_{z=0}",
            "a": a, "b": b, "c": c, "rows": rows}


def sphere():
    """Section 'Sphere': FT_V(Q) = (4 pi / 3) Gamma(5/2) J_{3/2}(Q) / (Q/2)^{3/2} for the unit sphere."""
    qs = [0.25, 1.0, 2.5, 4.493409457909064, 7.0, 12.0, 31.4]
    vals = [(4 * math.pi / 3) * gamma(2.5) * jv(1.5, q) / (q / 2) ** 1.5 for q in qs]
    return {"citation": "paper, section 'Sphere': the unit-sphere transform in terms of Gamma(5/2) and J_{3/2}",
            "q": qs, "F": [float(v) for v in vals]}


def main():
    for name, fn in (("rectangle_2d.json", rectangle), ("prism_3d.json", prism), ("sphere_unit.json", sphere)):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
