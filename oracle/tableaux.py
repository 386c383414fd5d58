"""IMEX ARK tableaux for the oracle's LHEVI stage recipe (test infrastructure).

All methods are ESDIRK/ERK pairs with b = b~ and c = c~ (Sec. 4.1: explicit
first stage, constant diagonal a~_ii, b = b~ to conserve linear invariants).

* ARK2 = ARK(2,3,2) of Giraldo, Kelly & Constantinescu (2013), the method the
  paper calls ARK2 (Sec. 6).  gamma = 1 - 1/sqrt(2), delta = 1/(2 sqrt(2)),
  and the free explicit coefficient a_32 = 1/2 for variant "b" (the de facto
  NUMA choice) or (3 + 2 sqrt(2))/6 for variant "a" (Sec. 4.1 text).
* ARK3 = ARK3(2)4L[2]SA of Kennedy & Carpenter (2003), the paper's ARK3
  (Sec. 6).  The paper does not print these coefficients; they are transcribed
  from the cited publication and pinned only by their order conditions and by
  the observed third-order convergence on a linear column (tests).  Parity of
  the coefficient values themselves is unpinned by the paper.

* ARS343 = ARS(3,4,3) of Ascher, Ruuth & Spiteri (1997), one of the further
  integrators the paper lists (Sec. 6; coefficients not printed there).  The
  implicit part is the L-stable three-stage DIRK with gamma the root in (1/3, 1/2)
  of 6 g^3 - 18 g^2 + 9 g - 1 = 0; the explicit coefficients are the published
  10-digit values, with a_31 and a_41 taken from the row sums so that c = c~
  holds exactly.  Its order conditions then hold to the published digits
  (about 1e-10); pinned by those and by observed third-order convergence.

* ARK4 = ARK4(3)6L[2]SA of Kennedy & Carpenter (2003), the paper's ARK4, the
  six-stage ARK(5,6,4) (Sec. 6; coefficients not printed there).  gamma = 1/4 and
  c = (0, 1/2, 83/250, 31/50, 17/20, 1); the implicit coefficients are exact
  rationals, the explicit ones the published rational approximations.  Pinned by
  the fourth-order conditions (exact row sums for the implicit part, about 1e-12
  for the explicit one) and by observed fourth-order convergence.

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


def ars343():
    g = mp.findroot(lambda x: 6 * x ** 3 - 18 * x ** 2 + 9 * x - 1, mp.mpf("0.4358665215"))
    b1 = -3 * g ** 2 / 2 + 4 * g - mp.mpf(1) / 4
    b2 = 3 * g ** 2 / 2 - 5 * g + mp.mpf(5) / 4
    c3 = (1 + g) / 2
    a32 = mp.mpf("0.3966543747")
    a42 = a43 = mp.mpf("0.5529291479")
    z = mp.mpf(0)
    Aexp = [[z, z, z, z], [g, z, z, z], [c3 - a32, a32, z, z], [1 - a42 - a43, a42, a43, z]]
    Aimp = [[z, z, z, z], [z, g, z, z], [z, (1 - g) / 2, g, z], [z, b1, b2, g]]
    b = [z, b1, b2, g]
    return {"name": "ARS343", "Aexp": Aexp, "Aimp": Aimp, "b": b, "order": 3}


def ark4():
    q = F(1, 4)
    z = F(0)
    Aexp = [
        [z] * 6,
        [F(1, 2), z, z, z, z, z],
        [F(13861, 62500), F(6889, 62500), z, z, z, z],
        [F(-116923316275, 2393684061468), F(-2731218467317, 15368042101831),
         F(9408046702089, 11113171139209), z, z, z],
        [F(-451086348788, 2902428689909), F(-2682348792572, 7519795681897),
         F(12662868775082, 11960479115383), F(3355817975965, 11060851509271), z, z],
        [F(647845179188, 3216320057751), F(73281519250, 8382639484533),
         F(552539513391, 3454668386233), F(3354512671639, 8306763924573), F(4040, 17871), z],
    ]
    b = [F(82889, 524892), z, F(15625, 83664), F(69875, 102672), F(-2260, 8211), q]
    Aimp = [
        [z] * 6,
        [q, q, z, z, z, z],
        [F(8611, 62500), F(-1743, 31250), q, z, z, z],
        [F(5012029, 34652500), F(-654441, 2922500), F(174375, 388108), q, z, z],
        [F(15267082809, 155376265600), F(-71443401, 120774400), F(730878875, 902184768),
         F(2285395, 8070912), q, z],
        list(b),
    ]
    return {"name": "ARK4", "Aexp": Aexp, "Aimp": Aimp, "b": b, "order": 4}


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
