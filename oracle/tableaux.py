"""IMEX ARK tableaux for the oracle's LHEVI stage recipe (test infrastructure).

Both methods are ESDIRK/ERK pairs with b = b~ and c = c~ (Sec. 4.1: explicit
first stage, constant diagonal a~_ii, b = b~ to conserve linear invariants).

* ARK2 = ARK(2,3,2) of Giraldo, Kelly & Constantinescu (2013), the method the
  paper calls ARK2 (Sec. 5).  gamma = 1 - 1/sqrt(2), delta = 1/(2 sqrt(2)),
  and the free explicit coefficient a_32 = 1/2 for variant "b" (the de facto
  NUMA choice) or (3 + 2 sqrt(2))/6 for variant "a" (Sec. 4.1 text).
* ARK3 = ARK3(2)4L[2]SA of Kennedy & Carpenter (2003), the paper's ARK3
  (Sec. 5).  The paper does not print these coefficients; they are transcribed
  from the cited publication and pinned only by their order conditions and by
  the observed third-order convergence on a linear column (tests).  Parity of
  the coefficient values themselves is unpinned by the paper.

Values are exact: rationals as fractions.Fraction, sqrt(2)-based entries as
mpmath numbers at 50 digits; ``as_float`` converts to float64 arrays.
"""
from __future__ import annotations

from fractions import Fraction as F

import mpmath as mp
import numpy as np

mp.mp.dps = 50


def ark2(variant: str = "b"):
    s2 = mp.sqrt(2)
    gam = 1 - 1 / s2
    dlt = 1 / (2 * s2)
    a32 = mp.mpf(1) / 2 if variant == "b" else (3 + 2 * s2) / 6
    z = mp.mpf(0)
    Aimp = [[z, z, z], [gam, gam, z], [dlt, dlt, gam]]
    Aexp = [[z, z, z], [2 * gam, z, z], [1 - a32, a32, z]]
    b = [dlt, dlt, gam]
    return {"name": f"ARK2{variant}", "Aexp": Aexp, "Aimp": Aimp, "b": b, "order": 2}


def ark3():
    g = F(1767732205903, 4055673282236)
    z = F(0)
    Aexp = [
        [z, z, z, z],
        [F(1767732205903, 2027836641118), z, z, z],
        [F(5535828885825, 10492691773637), F(788022342437, 10882634858940), z, z],
        [F(6485989280629, 16251701735622), F(-4246266847089, 9704473918619),
         F(10755448449292, 10357097424841), z],
    ]
    Aimp = [
        [z, z, z, z],
        [g, g, z, z],
        [F(2746238789719, 10658868560708), F(-640167445237, 6845629431997), g, z],
        [F(1471266399579, 7840856788654), F(-4482444167858, 7529755066697),
         F(11266239266428, 11593286722821), g],
    ]
    b = [F(1471266399579, 7840856788654), F(-4482444167858, 7529755066697),
         F(11266239266428, 11593286722821), g]
    return {"name": "ARK3", "Aexp": Aexp, "Aimp": Aimp, "b": b, "order": 3}


def as_float(tab):
    def cv(x):
        return float(x) if not isinstance(x, mp.mpf) else float(x)
    return {
        "name": tab["name"],
        "Aexp": np.array([[cv(v) for v in row] for row in tab["Aexp"]]),
        "Aimp": np.array([[cv(v) for v in row] for row in tab["Aimp"]]),
        "b": np.array([cv(v) for v in tab["b"]]),
        "order": tab["order"],
    }


def lhevi_coeffs(tab, i):
    """c_j = (a~_ij - a_ij) / a~_ii for j < i (Sec. 4.3, eq. lhevi-ark-final-3)."""
    return [(tab["Aimp"][i][j] - tab["Aexp"][i][j]) / tab["Aimp"][i][i] for j in range(i)]
