"""Pins of the oracle against facts fixed by the paper and by mathematics.

Each test names the plausible mistakes it would catch.  None of these tests
uses the HIP library.
"""
from fractions import Fraction as Fr

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import tableaux
from paper_2311_11425_amd import inputs

CONSTS = inputs.CONSTS
R, CP, G, PA = CONSTS
GAM = CP / (CP - R)


def relerr_per_var(x, ref):
    """max over variables of ||x_v - ref_v|| / ||ref_v|| for an interleaved vector."""
    out = 0.0
    for v in range(5):
        d = np.linalg.norm(ref[v::5])
        if d > 0:
            out = max(out, np.linalg.norm(x[v::5] - ref[v::5]) / d)
    return out


def flat_column(N, Ne, H=30.0e3, nhat=(0.0, 0.0, 1.0), T=300.0):
    col = inputs.make_columns(N, Ne, 1, z_top=H, profile="isothermal", seed=5)
    nh = np.asarray(nhat, dtype=float)
    nh = nh / np.linalg.norm(nh)
    h = H / Ne
    for m in range(3):
        col["gz"][m, :, 0] = 2.0 / h * nh[m]
    col["nhat"][0] = nh
    return col


# ---------------------------------------------------------------------------
# GLL tables (Sec. 3)

GLL_CLOSED = {
    1: ([-1, 1], [1, 1]),
    2: ([-1, 0, 1], [Fr(1, 3), Fr(4, 3), Fr(1, 3)]),
    3: ([-1, -mp.sqrt(mp.mpf(1) / 5), mp.sqrt(mp.mpf(1) / 5), 1],
        [Fr(1, 6), Fr(5, 6), Fr(5, 6), Fr(1, 6)]),
    4: ([-1, -mp.sqrt(mp.mpf(3) / 7), 0, mp.sqrt(mp.mpf(3) / 7), 1],
        [Fr(1, 10), Fr(49, 90), Fr(32, 45), Fr(49, 90), Fr(1, 10)]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_form(N):
    """Textbook closed-form Lobatto nodes/weights (catches a wrong root or weight formula)."""
    xi, w, D = oracle.gll(N)
    xs, ws = GLL_CLOSED[N]
    assert np.allclose(xi, [float(v) for v in xs], rtol=0, atol=1e-15)
    assert np.allclose(w, [float(v) for v in ws], rtol=0, atol=2e-16)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_gll_exactness(N):
    """Quadrature exact to degree 2N-1, derivative exact to degree N, rows sum to 0
    (catches a transposed D or a wrong diagonal)."""
    xi, w, D = oracle.gll(N)
    for p in range(2 * N):
        exact = (1 - (-1) ** (p + 1)) / (p + 1)
        assert abs(np.dot(w, xi ** p) - exact) < 1e-14
    for p in range(N + 1):
        dp = p * xi ** (p - 1) if p > 0 else np.zeros_like(xi)
        assert np.abs(D @ xi ** p - dp).max() < 1e-12 * max(1, N * N)
    assert np.abs(D.sum(1)).max() < 1e-12


def test_gll_vs_mpmath_order7():
    """Nodes of order 7 against 40-digit roots of P_7' (catches Newton stopping early)."""
    mp.mp.dps = 40
    N = 7
    xi, w, D = oracle.gll(N)
    dP = lambda x: mp.diff(lambda t: mp.legendre(N, t), x)
    for j in range(1, N):
        r = mp.findroot(dP, xi[j])
        assert abs(float(r) - xi[j]) < 1e-15
        assert abs(float(2 / (N * (N + 1) * mp.legendre(N, r) ** 2)) - w[j]) < 1e-15


# ---------------------------------------------------------------------------
# equation of state (Appendix A.1)

def test_reference_eos_mpmath():
    """theta0 and c_Theta = gamma P/Theta against 40-digit evaluation of the closed form."""
    mp.mp.dps = 40
    col = inputs.config2(ncols=3)
    th, cT = oracle.reference(col["rho0"].ravel(), col["Theta0"].ravel(), CONSTS)
    gam = mp.mpf(CP) / (mp.mpf(CP) - mp.mpf(R))
    for r0, T0, t, c in zip(col["rho0"].ravel(), col["Theta0"].ravel(), th, cT):
        P = mp.mpf(PA) * (mp.mpf(R) * mp.mpf(T0) / mp.mpf(PA)) ** gam
        assert abs(float(mp.mpf(T0) / mp.mpf(r0)) - t) <= 2e-16 * t
        assert abs(float(gam * P / mp.mpf(T0)) - c) <= 1e-14 * c


def test_reference_eos_ideal_gas():
    """For a hydrostatic ideal-gas reference, c_Theta theta0 = gamma R T = c^2 (catches
    a wrong exponent in the EOS)."""
    col = inputs.config1(ncols=2)
    th, cT = oracle.reference(col["rho0"].ravel(), col["Theta0"].ravel(), CONSTS)
    c2 = GAM * R * col["T"].ravel()
    assert np.allclose(th * cT, c2, rtol=1e-13)


# ---------------------------------------------------------------------------
# P1: exact rational brute force (GE + assembly indexing)

def _rational_gll(N):
    if N == 1:
        return [Fr(1), Fr(1)], [[Fr(-1, 2), Fr(1, 2)], [Fr(-1, 2), Fr(1, 2)]]
    if N == 2:
        return ([Fr(1, 3), Fr(4, 3), Fr(1, 3)],
                [[Fr(-3, 2), Fr(2), Fr(-1, 2)], [Fr(-1, 2), Fr(0), Fr(1, 2)],
                 [Fr(1, 2), Fr(-2), Fr(3, 2)]])
    raise ValueError


def _rational_solve(N, Ne, g, z, J, gz, th0, cT, lam, b, pr=None):
    """Exact (Fraction) assembly of I - lam L and Gauss-Jordan solve (pr: the
    dP/drho column of set 3C, None for set 2C)."""
    w, D = _rational_gll(N)
    nz = Ne * N + 1
    n = 5 * nz
    B = [[Fr(0)] * n for _ in range(n)]
    M = [Fr(0)] * nz
    for e in range(Ne):
        for i in range(N + 1):
            ki = e * N + i
            dphi = g * sum(D[i][j] * z[e * N + j] for j in range(N + 1))
            M[ki] += w[i] * J[ki]
            for m in range(3):
                B[5 * ki + 1 + m][5 * ki] += w[i] * J[ki] * dphi * gz[ki][m]
            for j in range(N + 1):
                kj = e * N + j
                for m in range(3):
                    B[5 * ki][5 * kj + 1 + m] += -w[j] * D[j][i] * J[kj] * gz[kj][m]
                    B[5 * ki + 1 + m][5 * kj + 4] += w[i] * D[i][j] * J[kj] * gz[kj][m] * cT[kj]
                    if pr is not None:
                        B[5 * ki + 1 + m][5 * kj] += w[i] * D[i][j] * J[kj] * gz[kj][m] * pr[kj]
                    B[5 * ki + 4][5 * kj + 1 + m] += w[i] * D[i][j] * J[kj] * gz[kj][m] * th0[kj]
    A = [[(Fr(1) if r == c else Fr(0)) + lam * B[r][c] / M[r // 5] for c in range(n)]
         for r in range(n)]
    for k in (0, nz - 1):
        for m in range(3):
            A[5 * k + 1 + m] = [Fr(1) if c == 5 * k + 1 + m else Fr(0) for c in range(n)]
    # Gauss-Jordan with exact arithmetic
    Ab = [row[:] + [b[r]] for r, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if Ab[r][c] != 0)
        Ab[c], Ab[p] = Ab[p], Ab[c]
        piv = Ab[c][c]
        Ab[c] = [v / piv for v in Ab[c]]
        for r in range(n):
            if r != c and Ab[r][c] != 0:
                f = Ab[r][c]
                Ab[r] = [a - f * bb for a, bb in zip(Ab[r], Ab[c])]
    return [Ab[r][n] for r in range(n)]


@pytest.mark.parametrize("N,Ne,with_pr", [(1, 2, False), (2, 2, False), (2, 1, False),
                                          (2, 2, True), (1, 3, True)])
def test_p1_rational_brute_force(N, Ne, with_pr):
    """Oracle solve vs exact rational arithmetic; n = (3/5, 0, 4/5) so the boundary
    projection is exact (catches index, sign and pivoting bugs in assembly and GE).
    with_pr adds the set-3C dP/drho column of the momentum rows."""
    nz = Ne * N + 1
    h = Fr(3000)
    nh = (Fr(3, 5), Fr(0), Fr(4, 5))
    if N == 1:
        pos = [Fr(k) for k in range(nz)]
    else:
        pos = [Fr(k, 2) for k in range(nz)]
    z = [Fr(100) + h * p for p in pos]
    J = [h / 2 * (1 + Fr(k, 7)) for k in range(nz)]
    gz = [[Fr(2) / h * c * (1 + Fr(k, 11)) for c in nh] for k in range(nz)]
    th0 = [Fr(300) + 7 * k for k in range(nz)]
    cT = [Fr(1, 3) + Fr(k, 13) for k in range(nz)]
    g = Fr(49, 5)
    lam = Fr(17, 2)
    rng = np.random.default_rng(9)
    b = [Fr(int(v), 64) for v in rng.integers(-256, 256, 5 * nz)]
    for k in (0, nz - 1):  # make the boundary momentum tangential (projection then exact)
        bu = b[5 * k + 1:5 * k + 4]
        d = sum(a * c for a, c in zip(bu, nh))
        for m in range(3):
            b[5 * k + 1 + m] = bu[m] - nh[m] * d
    pr = [-Fr(2, 5) * g * zz for zz in z] if with_pr else None
    x_exact = np.array([float(v) for v in _rational_solve(N, Ne, g, z, J, gz, th0, cT, lam, b,
                                                          pr)])
    f = lambda a: np.array([float(v) for v in a])
    L = oracle.assemble_L(N, Ne, float(g), f(z), f(J), np.array([[float(v) for v in r] for r in gz]),
                          f(th0), f(cT), f(pr) if with_pr else None)
    A = oracle.form_A(L, float(lam))
    x = oracle.lu_solve_dense(A, f(b), refine=0)
    assert np.linalg.norm(x - x_exact) / np.linalg.norm(x_exact) < 1e-14


# ---------------------------------------------------------------------------
# P2: identity at Lambda = 0

def test_p2_identity_at_zero_lambda():
    col = inputs.config1(heterogeneous=True, ncols=4)
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    b[1:4] += 0.3  # boundary normal momentum present: the projection must remove it
    x = oracle.solve_batch(col, 0.0, b, refine=0)
    for c in range(4):
        z, J, gz, r0, T0 = oracle.column_of(col, c)
        bp = oracle.bc_project(col["nz"], gz, oracle.vec_of(b, c))
        assert np.array_equal(oracle.vec_of(x, c), bp)
    # projected boundary momentum is tangential
    for k in (0, col["nz"] - 1):
        n = col["gz"][:, k, :] / np.linalg.norm(col["gz"][:, k, :], axis=0)
        assert np.abs((n * x[1:4, k, :]).sum(0)).max() < 1e-15


# ---------------------------------------------------------------------------
# P3: closed-form isothermal acoustic-gravity eigenvalues

def _omega(m, H, T=300.0):
    c = np.sqrt(GAM * R * T)
    Hs = R * T / G
    return c * np.sqrt((m * np.pi / H) ** 2 + 1.0 / (4 * Hs ** 2))


@pytest.mark.parametrize("Ne,tols", [(8, (1e-10, 1e-8, 1e-6)), (16, (1e-12, 1e-10, 1e-8))])
def test_p3_acoustic_eigenvalues(Ne, tols):
    """Eigenvalues +-i omega_m of the rigid-lid isothermal column (omega^2 =
    c^2((m pi/H)^2 + 1/(4 H_s^2))): catches a dropped gravity term, a wrong sign of the
    pressure gradient, a wrong theta0/c_Theta product, a transposed D or a wrong BC."""
    H = 30.0e3
    col = flat_column(4, Ne, H=H, nhat=(0.36, 0.48, 0.8))
    L = oracle.column_L(4, Ne, CONSTS, *oracle.column_of(col, 0))
    ev = np.linalg.eigvals(L)
    for m, tol in zip((1, 2, 3), tols):
        w = _omega(m, H)
        best = ev[np.argmin(np.abs(ev - 1j * w))]
        assert abs(best - 1j * w) / w < tol, (m, best, w)
        assert abs(best.real) < tol * w
    # first mode value computed by hand (T=300 K, H=30 km): 0.04138558 s^-1
    assert abs(_omega(1, H) - 0.04138558) < 1e-8
    # the mixed weak/strong discretisation is not skew: complex quartets with a small
    # real part exist (about 1.5% of the spectral radius here), so only bound them
    assert np.abs(ev.real).max() < 0.03 * np.abs(ev).max()


# ---------------------------------------------------------------------------
# P4 / P5: conservation of column mass and rho-theta

@pytest.mark.parametrize("hetero", [False, True])
def test_p4_p5_conservation(hetero):
    """sum_k M_k x_k = sum_k M_k b_k for rho and Theta (M from closed-form weights):
    catches a transposed weak-form D, a wrong mass or a wrong DSS."""
    col = inputs.config1(heterogeneous=hetero, ncols=6)
    if hetero:
        col = inputs.make_columns(4, 8, 6, profile="isothermal", seed=4, surface_max=2e3,
                                  deep=True)
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    lam = (1 - 1 / np.sqrt(2)) * 30.0
    x = oracle.solve_batch(col, lam, b, refine=1)
    w = np.array([float(v) for v in GLL_CLOSED[4][1]])
    for c in range(6):
        M = np.zeros(col["nz"])
        for e in range(col["Ne"]):
            for i in range(5):
                M[4 * e + i] += w[i] * col["J"][4 * e + i, c]
        for v, tol in ((0, 1e-13), (4, 1e-13)):
            lhs = np.dot(M, x[v, :, c])
            rhs = np.dot(M, b[v, :, c])
            scale = np.dot(M, np.abs(b[v, :, c]))
            assert abs(lhs - rhs) <= tol * scale


# ---------------------------------------------------------------------------
# P6: weak and strong continuity rows agree under the rigid lid

@pytest.mark.parametrize("cfg", [1, 2])
def test_p6_weak_equals_strong(cfg):
    col = inputs.config1(ncols=3) if cfg == 1 else inputs.config2(ncols=3)
    lam = (1 - 1 / np.sqrt(2)) * 30.0 if cfg == 1 else 0.4358665215 * 300
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    xw = oracle.solve_batch(col, lam, b, refine=1, rho_weak=True)
    xs = oracle.solve_batch(col, lam, b, refine=1, rho_weak=False)
    for c in range(3):
        assert relerr_per_var(oracle.vec_of(xs, c), oracle.vec_of(xw, c)) < 1e-12


# ---------------------------------------------------------------------------
# P7: tangential momentum untouched

def test_p7_tangential_momentum():
    col = inputs.config1(heterogeneous=True, ncols=5)
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    lam = 40.0
    x = oracle.solve_batch(col, lam, b, refine=1)
    for c in range(5):
        n = col["nhat"][c]
        P = np.eye(3) - np.outer(n, n)
        xt = P @ x[1:4, :, c]
        bt = P @ b[1:4, :, c]
        assert np.abs(xt - bt).max() <= 1e-13 * np.abs(bt).max()


# ---------------------------------------------------------------------------
# P8: hydrostatic null vectors

def test_p8_hydrostatic_null_vector():
    """rho' balancing the pressure gradient of any Theta' (gravity coefficient g n) is
    a null vector of L_z, so x = b for every Lambda: catches a wrong gravity column,
    a wrong Phi derivative or a gravity term not divided by the mass."""
    col = inputs.config1(heterogeneous=True, ncols=2)
    rng = np.random.default_rng(4)
    for c in range(2):
        z, J, gz, r0, T0 = oracle.column_of(col, c)
        nz = col["nz"]
        L = oracle.column_L(4, 8, CONSTS, z, J, gz, r0, T0)
        v = np.zeros(5 * nz)
        v[4::5] = 1e-2 * T0 * rng.uniform(-1, 1, nz)
        p = L @ v
        n = col["nhat"][c]
        for k in range(1, nz - 1):
            pk = p[5 * k + 1:5 * k + 4]
            assert np.linalg.norm(pk - n * (n @ pk)) <= 1e-12 * np.linalg.norm(pk)
            v[5 * k] = (n @ pk) / G
        Lv = L @ v
        assert np.linalg.norm(Lv) <= 1e-13 * np.linalg.norm(L, 2) * np.linalg.norm(v)
        for lam in (10.0, 1000.0):
            x = oracle.lu_solve_dense(oracle.form_A(L, lam), v, refine=1)
            assert relerr_per_var(x, v) < 1e-12


# ---------------------------------------------------------------------------
# P9: rotation equivariance

def test_p9_rotation_equivariance():
    col = inputs.config1(heterogeneous=True, ncols=3)
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    lam = 25.0
    x = oracle.solve_batch(col, lam, b, refine=1)
    Q = sla.expm(np.array([[0, -0.3, 0.5], [0.3, 0, -0.7], [-0.5, 0.7, 0]]))
    col2 = dict(col)
    col2["gz"] = np.einsum("ij,jkc->ikc", Q, col["gz"])
    b2 = b.copy()
    b2[1:4] = np.einsum("ij,jkc->ikc", Q, b[1:4])
    x2 = oracle.solve_batch(col2, lam, b2, refine=1)
    xr = x.copy()
    xr[1:4] = np.einsum("ij,jkc->ikc", Q, x[1:4])
    for c in range(3):
        assert relerr_per_var(oracle.vec_of(x2, c), oracle.vec_of(xr, c)) < 1e-13


# ---------------------------------------------------------------------------
# P10: LAPACK band solve (the paper's own solver) on the assembled band

@pytest.mark.parametrize("cfg", [1, 2])
def test_p10_lapack_band(cfg):
    col = inputs.config1(ncols=2) if cfg == 1 else inputs.config2(ncols=2)
    N, Ne = col["N"], col["Ne"]
    lam = (1 - 1 / np.sqrt(2)) * 30.0 if cfg == 1 else 0.4358665215 * 300
    qn, qref = inputs.perturbed_state(col)
    kl = ku = 5 * (N + 1) - 1
    for c in range(2):
        z, J, gz, r0, T0 = oracle.column_of(col, c)
        L = oracle.column_L(N, Ne, CONSTS, z, J, gz, r0, T0)
        A = oracle.form_A(L, lam)
        n = A.shape[0]
        ii, jj = np.nonzero(A)
        assert np.abs(ii - jj).max() <= kl
        ab = np.zeros((kl + ku + 1, n))
        for j in range(n):
            for i in range(max(0, j - ku), min(n, j + kl + 1)):
                ab[ku + i - j, j] = A[i, j]
        b = oracle.bc_project(col["nz"], gz, oracle.vec_of(qn - qref, c))
        xl = sla.solve_banded((kl, ku), ab, b)
        x0 = oracle.lu_solve_dense(A, b, refine=0)
        x1 = oracle.lu_solve_dense(A, b, refine=1)
        assert relerr_per_var(x0, xl) < 5e-12
        assert relerr_per_var(x1, xl) < 5e-12


# ---------------------------------------------------------------------------
# P11: certification of the oracle+ mode with 30-digit arithmetic

@pytest.mark.parametrize("cfg", [1, 2])
def test_p11_mpmath_certification(cfg):
    mp.mp.dps = 30
    col = inputs.config1(ncols=1) if cfg == 1 else inputs.config2(ncols=1)
    N, Ne = col["N"], col["Ne"]
    lam = (1 - 1 / np.sqrt(2)) * 30.0 if cfg == 1 else 0.4358665215 * 300
    qn, qref = inputs.perturbed_state(col)
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    L = oracle.column_L(N, Ne, CONSTS, z, J, gz, r0, T0)
    A = oracle.form_A(L, lam)
    b = oracle.bc_project(col["nz"], gz, oracle.vec_of(qn - qref, 0))
    xm = mp.lu_solve(mp.matrix(A.tolist()), mp.matrix(b.tolist()))
    xm = np.array([float(v) for v in xm])
    x1 = oracle.lu_solve_dense(A, b, refine=1)
    assert relerr_per_var(x1, xm) < 1e-15
    x0 = oracle.lu_solve_dense(A, b, refine=0)
    assert relerr_per_var(x0, xm) < 2e-12


# ---------------------------------------------------------------------------
# P13: tableau order conditions

def _conds(tab):
    cv = lambda v: mp.mpf(v.numerator) / v.denominator if isinstance(v, Fr) else mp.mpf(v)
    A = [[cv(v) for v in row] for row in tab["Aexp"]]
    At = [[cv(v) for v in row] for row in tab["Aimp"]]
    b = [cv(v) for v in tab["b"]]
    s = len(b)
    c = [sum(A[i][j] for j in range(s)) for i in range(s)]
    ct = [sum(At[i][j] for j in range(s)) for i in range(s)]
    out = {
        "sum_b": sum(b) - 1,
        "b_c": sum(b[i] * c[i] for i in range(s)) - mp.mpf(1) / 2,
        "c_eq_ct": max(abs(c[i] - ct[i]) for i in range(s)),
    }
    if tab["order"] >= 3:
        third = mp.mpf(1) / 3
        sixth = mp.mpf(1) / 6
        out["b_c2"] = sum(b[i] * c[i] ** 2 for i in range(s)) - third
        out["bAc"] = sum(b[i] * A[i][j] * c[j] for i in range(s) for j in range(s)) - sixth
        out["bAtc"] = sum(b[i] * At[i][j] * c[j] for i in range(s) for j in range(s)) - sixth
        out["bAct"] = sum(b[i] * A[i][j] * ct[j] for i in range(s) for j in range(s)) - sixth
        out["bAtct"] = sum(b[i] * At[i][j] * ct[j] for i in range(s) for j in range(s)) - sixth
    if tab["order"] >= 4:
        # with b = b~ and c = c~ the additive fourth-order conditions are those of
        # the four order-4 trees with every inner vertex taking A or A~ (1 + 2 + 2 + 4)
        Ms = {"E": A, "I": At}
        out["b_c3"] = sum(b[i] * c[i] ** 3 for i in range(s)) - mp.mpf(1) / 4
        for xn, X in Ms.items():
            out[f"bc{xn}c"] = sum(b[i] * c[i] * X[i][j] * c[j]
                                  for i in range(s) for j in range(s)) - mp.mpf(1) / 8
            out[f"b{xn}c2"] = sum(b[i] * X[i][j] * c[j] ** 2
                                  for i in range(s) for j in range(s)) - mp.mpf(1) / 12
            for yn, Y in Ms.items():
                out[f"b{xn}{yn}c"] = sum(b[i] * X[i][j] * Y[j][k] * c[k] for i in range(s)
                                         for j in range(s) for k in range(s)) - mp.mpf(1) / 24
    return out


@pytest.mark.parametrize("tab", [tableaux.ark2("b"), tableaux.ark2("a"), tableaux.ark3(),
                                 tableaux.ars343(), tableaux.ark4()])
def test_p13_order_conditions(tab):
    mp.mp.dps = 50
    # ARS(3,4,3)'s explicit coefficients are published to 10 digits; ARK4's
    # published rationals meet every condition to about 1e-26, so a slip in the
    # last digit of one of its 13-digit numerators (about 1e-13) must fail
    tol = {"ARS343": 1e-9, "ARK4": 1e-20}.get(tab["name"], 1e-11)
    for k, v in _conds(tab).items():
        assert abs(float(v)) < tol, (tab["name"], k, float(v))
    s = len(tab["b"])
    # ESDIRK structure: explicit first stage, constant diagonal, b = last implicit row
    assert all(tab["Aimp"][0][j] == 0 for j in range(s))
    d = tab["Aimp"][1][1]
    assert all(abs(float(tab["Aimp"][i][i] - d)) < 1e-30 for i in range(1, s))
    # LHEVI coefficients sum to -1 (R14): the stage recipe is offset-free
    for i in range(1, s):
        assert abs(float(1 + sum(tableaux.lhevi_coeffs(tab, i)))) < 1e-11


def test_ark2_lhevi_coefficients_and_paper_a32():
    """ARK(2,3,2)b has a_32 = 1/2 and ARK(2,3,2)a has a_32 = (3+2 sqrt 2)/6 (Sec. 4.1);
    the LHEVI coefficients of ARK2b are -1 and (-1/2, -1/2)."""
    tb = tableaux.ark2("b")
    ta = tableaux.ark2("a")
    assert tb["Aexp"][2][1] == mp.mpf(1) / 2
    assert abs(ta["Aexp"][2][1] - (3 + 2 * mp.sqrt(2)) / 6) < 1e-40
    assert abs(float(tableaux.lhevi_coeffs(tb, 1)[0]) + 1) < 1e-15
    c3 = tableaux.lhevi_coeffs(tb, 2)
    assert abs(float(c3[0]) + 0.5) < 1e-15 and abs(float(c3[1]) + 0.5) < 1e-15


# ---------------------------------------------------------------------------
# P12: ARK order on a linear column against the matrix exponential

@pytest.mark.parametrize("tabname,order", [("ARK2b", 2), ("ARK2a", 2), ("ARK3", 3),
                                            ("ARS343", 3), ("ARK4", 4)])
def test_p12_ark_order(tabname, order):
    """Observed order of the oracle's LHEVI ARK recipe with an explicit Coriolis term
    (catches a wrong c_j, a wrong q^E or a wrong final update)."""
    tab = tableaux.as_float({"ARK2b": lambda: tableaux.ark2("b"),
                             "ARK2a": lambda: tableaux.ark2("a"), "ARK3": tableaux.ark3,
                             "ARS343": tableaux.ars343, "ARK4": tableaux.ark4}[tabname]())
    col = inputs.make_columns(4, 8, 1, z_top=30e3, profile="isothermal", seed=21)
    qn, qref = inputs.smooth_state(col, modes=(1, 2))
    omega = 2e-3
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    L = oracle.column_L(4, 8, CONSTS, z, J, gz, r0, T0)
    nz = col["nz"]
    C = np.zeros_like(L)
    n = col["nhat"][0]
    X = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    for k in range(nz):
        C[5 * k + 1:5 * k + 4, 5 * k + 1:5 * k + 4] = -2 * omega * X
    T = 600.0
    # keep the slow modes only (|lambda| < 0.06 s^-1): the fast acoustic modes are damped
    # by the implicit part at these step sizes and hide the asymptotic order (stability regions, Sec. 6)
    lam_, V = np.linalg.eig(L + C)
    a = np.linalg.solve(V, oracle.vec_of(qn - qref, 0).astype(complex))
    slow = np.abs(lam_) < 0.06
    q0 = (V[:, slow] @ a[slow]).real
    qstart = qref.copy()
    for v in range(5):
        qstart[v, :, 0] += q0[v::5]
    exact = sla.expm((L + C) * T) @ q0
    errs = []
    dts = [30.0, 15.0, 7.5, 3.75]
    for dt in dts:
        q = qstart.copy()
        for _ in range(int(round(T / dt))):
            q = oracle.ark_step_batch(col, tab, dt, q, qref, refine=1, omega=omega)
        errs.append(np.linalg.norm(oracle.vec_of(q - qref, 0) - exact) / np.linalg.norm(exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > order - 0.25, (errs, rates)
    assert rates[-1] < order + 0.6, (errs, rates)


def _explicit_linear_order(tab):
    """Largest p with b A^(k-1) 1 = 1/k! for k = 1..p over the explicit tableau:
    the order of its stability polynomial (to 1e-9: ARS(3,4,3) is published to
    10 digits)."""
    cv = lambda v: mp.mpf(v.numerator) / v.denominator if isinstance(v, Fr) else mp.mpf(v)
    A = mp.matrix([[cv(v) for v in row] for row in tab["Aexp"]])
    b = mp.matrix([cv(v) for v in tab["b"]])
    v = mp.matrix([1] * len(tab["b"]))
    p = 0
    while abs((b.T * v)[0] - 1 / mp.factorial(p + 1)) < 1e-9:
        p += 1
        v = A * v
    return p


@pytest.mark.parametrize("tabname", ["ARK2b", "ARK2a", "ARK3", "ARS343", "ARK4"])
def test_p12b_explicit_part_order(tabname):
    """Observed order of the explicit part alone.  An inertial oscillation
    (horizontal momentum perpendicular to n^, which L_z leaves untouched) is
    turned only by the Coriolis term, explicit in the stage recipe, so the
    implicit part plays no role and the rate must be the linear order of the
    explicit tableau: 2, 3 for ARK2a (its a_32 gives b A c = 1/6), 3, 4
    (ARS(3,4,3)'s explicit part also meets b A^3 1 = 1/24) and 4.  Catches a wrong explicit coefficient or a wrong q^E
    that the implicit-dominated test above cannot see: ARK3 and ARS(3,4,3) share
    their implicit stability function and agree there to ten digits."""
    mp.mp.dps = 50
    t = {"ARK2b": lambda: tableaux.ark2("b"), "ARK2a": lambda: tableaux.ark2("a"),
         "ARK3": tableaux.ark3,
         "ARS343": tableaux.ars343, "ARK4": tableaux.ark4}[tabname]()
    p = _explicit_linear_order(t)
    assert p == {"ARK2b": 2, "ARK2a": 3, "ARK3": 3, "ARS343": 4, "ARK4": 4}[tabname]
    tab = tableaux.as_float(t)
    col = inputs.make_columns(4, 8, 1, z_top=30e3, profile="isothermal", seed=21)
    _, qref = inputs.smooth_state(col, modes=(1,))
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    L = oracle.column_L(4, 8, CONSTS, z, J, gz, r0, T0)
    nz = col["nz"]
    n = col["nhat"][0]
    e1 = np.cross(n, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    prof = np.sin(np.pi * (z - z[0]) / (z[-1] - z[0]))
    q0 = np.zeros(5 * nz)
    for k in range(nz):
        q0[5 * k + 1:5 * k + 4] = 0.1 * prof[k] * r0[k] * e1
    assert np.linalg.norm(L @ q0) < 1e-14 * np.linalg.norm(q0)
    omega = 5e-3
    X = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    C = np.zeros_like(L)
    for k in range(nz):
        C[5 * k + 1:5 * k + 4, 5 * k + 1:5 * k + 4] = -2 * omega * X
    T = 600.0
    exact = sla.expm((L + C) * T) @ q0
    qstart = qref.copy()
    for v in range(5):
        qstart[v, :, 0] += q0[v::5]
    errs = []
    for dt in (60.0, 30.0, 15.0, 7.5):
        q = qstart.copy()
        for _ in range(int(round(T / dt))):
            q = oracle.ark_step_batch(col, tab, dt, q, qref, refine=1, omega=omega)
        errs.append(np.linalg.norm(oracle.vec_of(q - qref, 0) - exact) / np.linalg.norm(exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(rates[-1] - p) < 0.15, (errs, rates)


# ---------------------------------------------------------------------------
# Set 3C (total energy; Appendix A.1 eq. set3c, Appendix A.3 eq. set3c_jacobian)

def _to_3c(col, c, v2):
    """The set-2C perturbation v2 = (rho', U', Theta') of column c as set-3C
    variables (rho', U', E'): linearising E = P/(gamma-1) + U.U/(2 rho) + rho Phi
    (eq. set3c_pressure) at rest with P' = c_Theta Theta' (eq. set2c_pressure) gives
    E' = c_Theta Theta'/(gamma - 1) + Phi rho', Phi = g z."""
    z, J, gz, r0, T0 = oracle.column_of(col, c)
    _, cT = oracle.reference(r0, T0, CONSTS)
    v = v2.copy()
    v[4::5] = cT * v2[4::5] / (GAM - 1) + G * z * v2[0::5]
    return v


def _L_both(col, c):
    z, J, gz, r0, T0 = oracle.column_of(col, c)
    N, Ne = col["N"], col["Ne"]
    L2 = oracle.column_L(N, Ne, CONSTS, z, J, gz, r0, T0)
    L3 = oracle.column_L(N, Ne, CONSTS, z, J, gz, r0, col["E0"][:, c], eqset="3C")
    return L2, L3


def test_3c_reference_ideal_gas():
    """For the ideal-gas reference E0 = rho0 c_v T + rho0 g z: P0 = rho0 R T, so
    dP/dE (h - Phi) = (gamma-1) c_p T = gamma R T = c^2, and dP/drho = -(gamma-1) g z
    (catches E0/rho0 in place of (E0+P0)/rho0, a dropped Phi or a wrong gamma)."""
    col = inputs.config2(ncols=3)
    z = col["z"].ravel()
    hE, dPdE, dPdr = oracle.reference_3c(col["rho0"].ravel(), col["E0"].ravel(), z, CONSTS)
    T = col["T"].ravel()
    assert np.allclose(dPdE * (hE - G * z), GAM * R * T, rtol=1e-12)
    assert np.allclose(dPdr, -(GAM - 1) * G * z, rtol=1e-15, atol=0)
    assert np.all(dPdE == GAM - 1)


@pytest.mark.parametrize("profile", ["isothermal", "lapse"])
def test_3c_momentum_rows_equal_2c(profile):
    """Under E' = c_Theta Theta'/(gamma-1) + Phi rho' the linearised pressure of set
    3C, (gamma-1)(E' - Phi rho'), is set 2C's c_Theta Theta' node by node, and the
    continuity rows are the same: so the rho and momentum rows of L_3C T v and
    T L_2C v agree to rounding at any resolution.  Catches a wrong sign or a
    missing dP/drho entry, a dP/dE other than gamma-1 or the pressure column put in
    the wrong place."""
    col = inputs.make_columns(4, 6, 2, profile=profile, seed=3, surface_max=1e3, tilt=0.05)
    qn, qref = inputs.perturbed_state(col)
    for c in range(2):
        L2, L3 = _L_both(col, c)
        v2 = oracle.vec_of(qn - qref, c)
        a = L3 @ _to_3c(col, c, v2)
        b = _to_3c(col, c, L2 @ v2)
        assert np.array_equal(a[0::5], b[0::5])
        for v in (1, 2, 3):
            assert np.linalg.norm(a[v::5] - b[v::5]) <= 1e-13 * np.linalg.norm(b[v::5])


@pytest.mark.parametrize("profile", ["isothermal", "lapse"])
def test_3c_energy_row_converges_to_2c(profile):
    """The energy rows of L_3C T v and T L_2C v differ only by the discrete product
    rule (h = (gamma-1)^-1 c_Theta theta0 + Phi up to the hydrostatic balance of the
    reference), so their difference falls at the spectral rate, by about 2^(N) per
    halving of the element size for N = 4, for a smooth perturbation.  Catches a
    wrong energy flux coefficient (an O(1) difference that does not converge) or a
    transposed derivative in the energy row."""
    errs = []
    for Ne in (4, 8, 16):
        col = inputs.make_columns(4, Ne, 1, profile=profile, seed=3, surface_max=1e3)
        qn, qref = inputs.smooth_state(col)
        L2, L3 = _L_both(col, 0)
        v2 = oracle.vec_of(qn - qref, 0)
        a = L3 @ _to_3c(col, 0, v2)
        b = _to_3c(col, 0, L2 @ v2)
        errs.append(np.linalg.norm(a[4::5] - b[4::5]) / np.linalg.norm(a[4::5]))
    assert errs[-1] < 2e-6, errs
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs


@pytest.mark.parametrize("Ne,tols", [(8, (1e-10, 1e-8, 1e-6)), (16, (1e-12, 1e-10, 1e-8))])
def test_3c_acoustic_eigenvalues(Ne, tols):
    """The isothermal rigid-lid column in set 3C has the same acoustic-gravity
    frequencies as in set 2C (the linear dynamics do not depend on the choice of
    thermodynamic variable): catches a wrong energy flux, a wrong dP/dE or dP/drho."""
    H = 30.0e3
    col = inputs.as_set(flat_column(4, Ne, H=H, nhat=(0.36, 0.48, 0.8)), "3C")
    L = oracle.column_L(4, Ne, CONSTS, *oracle.column_of(col, 0), eqset="3C")
    ev = np.linalg.eigvals(L)
    for m, tol in zip((1, 2, 3), tols):
        w = _omega(m, H)
        best = ev[np.argmin(np.abs(ev - 1j * w))]
        assert abs(best - 1j * w) / w < tol, (m, best, w)
        assert abs(best.real) < tol * w
    assert np.abs(ev.real).max() < 0.03 * np.abs(ev).max()


@pytest.mark.parametrize("hetero", [False, True])
def test_3c_mass_and_total_energy_conservation(hetero):
    """Set 3C conserves mass and total energy (Sec. 3 and the Appendix A.1
    remarks): sum_k M_k x_k = sum_k M_k b_k for rho and E under the rigid lid
    (catches a transposed derivative or a wrong DSS in the energy row)."""
    col = inputs.make_columns(4, 8, 4, profile="lapse", seed=4,
                              surface_max=2e3 if hetero else 0.0, deep=hetero)
    col = inputs.as_set(col, "3C")
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    lam = 0.4358665215 * 300
    x = oracle.solve_batch(col, lam, b, refine=1)
    w = np.array([float(v) for v in GLL_CLOSED[4][1]])
    for c in range(4):
        M = np.zeros(col["nz"])
        for e in range(col["Ne"]):
            for i in range(5):
                M[4 * e + i] += w[i] * col["J"][4 * e + i, c]
        for v in (0, 4):
            lhs = np.dot(M, x[v, :, c])
            rhs = np.dot(M, b[v, :, c])
            assert abs(lhs - rhs) <= 1e-13 * np.dot(M, np.abs(b[v, :, c]))


def test_3c_hydrostatic_null_vector():
    """The set-2C hydrostatic null vector (rho' balancing the pressure gradient of
    Theta') mapped to (rho', 0, E') is a null vector of L_3C, so x = b for every
    Lambda (catches a gravity or dP/drho term that does not cancel)."""
    col = inputs.config1(heterogeneous=True, ncols=1)
    rng = np.random.default_rng(4)
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    nz = col["nz"]
    L2, L3 = _L_both(col, 0)
    v = np.zeros(5 * nz)
    v[4::5] = 1e-2 * T0 * rng.uniform(-1, 1, nz)
    p = L2 @ v
    n = col["nhat"][0]
    for k in range(1, nz - 1):
        v[5 * k] = (n @ p[5 * k + 1:5 * k + 4]) / G
    v3 = _to_3c(col, 0, v)
    assert np.linalg.norm(L3 @ v3) <= 1e-13 * np.linalg.norm(L3, 2) * np.linalg.norm(v3)
    for lam in (10.0, 1000.0):
        x = oracle.lu_solve_dense(oracle.form_A(L3, lam), v3, refine=1)
        assert relerr_per_var(x, v3) < 1e-12


def test_3c_lapack_band_and_mpmath():
    """Set-3C solve at the ne=30 shape against the LAPACK band solver (the paper's
    solver, Sec. 4.2.2) and 30-digit elimination (the oracle+ mode)."""
    mp.mp.dps = 30
    col = inputs.as_set(inputs.config2(ncols=1), "3C")
    N, Ne = col["N"], col["Ne"]
    lam = 0.4358665215 * 300
    qn, qref = inputs.perturbed_state(col)
    z, J, gz, r0, E0 = oracle.column_of(col, 0)
    L = oracle.column_L(N, Ne, CONSTS, z, J, gz, r0, E0, eqset="3C")
    A = oracle.form_A(L, lam)
    n = A.shape[0]
    kl = ku = 5 * (N + 1) - 1
    ii, jj = np.nonzero(A)
    assert np.abs(ii - jj).max() <= kl
    ab = np.zeros((kl + ku + 1, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[ku + i - j, j] = A[i, j]
    b = oracle.bc_project(col["nz"], gz, oracle.vec_of(qn - qref, 0))
    xl = sla.solve_banded((kl, ku), ab, b)
    xm = np.array([float(v) for v in mp.lu_solve(mp.matrix(A.tolist()), mp.matrix(b.tolist()))])
    x1 = oracle.lu_solve_dense(A, b, refine=1)
    assert relerr_per_var(x1, xm) < 1e-15
    assert relerr_per_var(x1, xl) < 5e-12
    # the batched driver runs the same definition
    xb = oracle.solve_batch(col, lam, qn - qref, refine=1)
    assert relerr_per_var(oracle.vec_of(xb, 0), x1) < 1e-15


@pytest.mark.parametrize("eqset", ["2C", "3C"])
def test_3c_rotation_and_tangential(eqset):
    """Rotation equivariance and untouched tangential momentum hold for both sets."""
    col = inputs.as_set(inputs.config1(heterogeneous=True, ncols=3), eqset)
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    lam = 25.0
    x = oracle.solve_batch(col, lam, b, refine=1)
    Q = sla.expm(np.array([[0, -0.3, 0.5], [0.3, 0, -0.7], [-0.5, 0.7, 0]]))
    col2 = dict(col)
    col2["gz"] = np.einsum("ij,jkc->ikc", Q, col["gz"])
    b2 = b.copy()
    b2[1:4] = np.einsum("ij,jkc->ikc", Q, b[1:4])
    x2 = oracle.solve_batch(col2, lam, b2, refine=1)
    xr = x.copy()
    xr[1:4] = np.einsum("ij,jkc->ikc", Q, x[1:4])
    for c in range(3):
        assert relerr_per_var(oracle.vec_of(x2, c), oracle.vec_of(xr, c)) < 1e-13
        n = col["nhat"][c]
        P = np.eye(3) - np.outer(n, n)
        assert np.abs(P @ x[1:4, :, c] - P @ b[1:4, :, c]).max() <= 1e-13 * np.abs(b[1:4]).max()


# ---------------------------------------------------------------------------
# LHEVI-PS (Sec. 4.3.1): the Jacobian of the vertical operator at a moving state

def _nonlinear_V(col, c, q):
    """The set-2C discrete vertical operator V(q) of column c (Appendix A.2), written
    from its nonlinear fluxes F_rho = J U^z, F_U = J (U U^z/rho + P(Theta) grad zeta),
    F_Theta = J Theta U^z/rho (U^z = grad(zeta).U) with the same element derivatives,
    gravity, DSS, mass and rigid lid as the oracle's operator; q interleaved (5k+v)."""
    N, Ne = col["N"], col["Ne"]
    nz = Ne * N + 1
    _, w, D = oracle.gll(N)
    z, J, gz, _, _ = oracle.column_of(col, c)
    rho, Th = q[0::5], q[4::5]
    U = np.stack([q[1::5], q[2::5], q[3::5]], 1)
    Uz = (gz * U).sum(1)
    P = PA * (R * Th / PA) ** GAM
    Fr = J * Uz
    FU = J[:, None] * (U * (Uz / rho)[:, None] + P[:, None] * gz)
    FT = J * Th * Uz / rho
    B = np.zeros((nz, 5))
    M = np.zeros(nz)
    for e in range(Ne):
        for i in range(N + 1):
            ki = e * N + i
            M[ki] += w[i] * J[ki]
            dphi = G * sum(D[i, j] * z[e * N + j] for j in range(N + 1))
            B[ki, 1:4] += w[i] * J[ki] * dphi * gz[ki] * rho[ki]
            for j in range(N + 1):
                kj = e * N + j
                B[ki, 0] += -w[j] * D[j, i] * Fr[kj]
                B[ki, 1:4] += w[i] * D[i, j] * FU[kj]
                B[ki, 4] += w[i] * D[i, j] * FT[kj]
    V = -B / M[:, None]
    V[0, 1:4] = 0.0
    V[-1, 1:4] = 0.0
    return V.reshape(-1)


def _ps_col():
    return inputs.with_wind(inputs.make_columns(4, 6, 2, profile="lapse", seed=3,
                                                surface_max=1e3, tilt=0.05))


def test_ps_rest_limit():
    """At U0 = 0 the LHEVI-PS operator is the reference-state operator (catches an entry
    of the general Jacobian that survives at rest, or an assembly slip of the general
    path)."""
    col = _ps_col()
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    Lrs = oracle.column_L(4, 6, CONSTS, z, J, gz, r0, T0)
    L0 = oracle.column_L(4, 6, CONSTS, z, J, gz, r0, T0, U0_k3=np.zeros((len(z), 3)))
    assert np.abs(L0 - Lrs).max() <= 1e-15 * np.abs(Lrs).max()


def test_ps_jacobian_matches_nonlinear_operator():
    """L_PS v against centred differences of the nonlinear operator V at q0 = (rho0, U0,
    Theta0): the second-order error at this step is ~1e-10, while any dropped or
    mis-signed Jacobian entry (advection of U and Theta, the u_l U^z/rho products, the
    -Theta U^z/rho^2 term) leaves 1e-4 or more; the rest-state operator misses by 1e-3."""
    col = _ps_col()
    qn, qref = inputs.perturbed_state(col)
    for c in range(2):
        z, J, gz, r0, T0 = oracle.column_of(col, c)
        L = oracle.column_L(4, 6, CONSTS, z, J, gz, r0, T0, U0_k3=oracle.u0_of(col, c))
        Lrs = oracle.column_L(4, 6, CONSTS, z, J, gz, r0, T0)
        q0 = oracle.vec_of(qref, c)
        v = oracle.vec_of(qn - qref, c)
        eps = 1e-2
        fd = (_nonlinear_V(col, c, q0 + eps * v) - _nonlinear_V(col, c, q0 - eps * v)) / (2 * eps)
        Lv, Lv_rs = L @ v, Lrs @ v
        for k in range(5):
            d = np.linalg.norm(Lv[k::5])
            assert np.linalg.norm(fd[k::5] - Lv[k::5]) < 1e-9 * d, (c, k)
        assert max(np.linalg.norm(fd[k::5] - Lv_rs[k::5]) / np.linalg.norm(Lv_rs[k::5])
                   for k in range(1, 5)) > 1e-4


def test_ps_conservation():
    """Mass and rho-theta stay conserved with the moving linearisation state (flux form;
    the vertical wind of the state vanishes at the lid)."""
    col = inputs.with_wind(inputs.make_columns(4, 8, 4, profile="lapse", seed=4,
                                               surface_max=2e3, deep=True))
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    x = oracle.solve_batch(col, 0.4358665215 * 300, b, refine=1)
    w = np.array([float(v) for v in GLL_CLOSED[4][1]])
    for c in range(4):
        M = np.zeros(col["nz"])
        for e in range(col["Ne"]):
            for i in range(5):
                M[4 * e + i] += w[i] * col["J"][4 * e + i, c]
        for v in (0, 4):
            assert abs(np.dot(M, x[v, :, c]) - np.dot(M, b[v, :, c])) <= \
                1e-13 * np.dot(M, np.abs(b[v, :, c]))


def test_ps_lapack_band_and_mpmath():
    """An LHEVI-PS column of the ne=30 shape: the paper's band structure (kl = ku =
    5(N+1) - 1) holds, the LAPACK band solver and 30-digit elimination agree with the
    oracle, and the batched driver equals the dense solve."""
    mp.mp.dps = 30
    col = inputs.with_wind(inputs.config2(ncols=1))
    N, Ne = col["N"], col["Ne"]
    lam = 0.4358665215 * 300
    qn, qref = inputs.perturbed_state(col)
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    L = oracle.column_L(N, Ne, CONSTS, z, J, gz, r0, T0, U0_k3=oracle.u0_of(col, 0))
    A = oracle.form_A(L, lam)
    n = A.shape[0]
    kl = ku = 5 * (N + 1) - 1
    ii, jj = np.nonzero(A)
    assert np.abs(ii - jj).max() <= kl
    ab = np.zeros((kl + ku + 1, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[ku + i - j, j] = A[i, j]
    b = oracle.bc_project(col["nz"], gz, oracle.vec_of(qn - qref, 0))
    xl = sla.solve_banded((kl, ku), ab, b)
    xm = np.array([float(v) for v in mp.lu_solve(mp.matrix(A.tolist()), mp.matrix(b.tolist()))])
    x1 = oracle.lu_solve_dense(A, b, refine=1)
    assert relerr_per_var(x1, xm) < 1e-15
    assert relerr_per_var(x1, xl) < 5e-12
    xb = oracle.solve_batch(col, lam, qn - qref, refine=1)
    assert relerr_per_var(oracle.vec_of(xb, 0), x1) < 1e-15


def test_ps_rotation_equivariance():
    """Rotating grad(zeta), the state's momentum and the right-hand side's momentum
    rotates the LHEVI-PS solution."""
    col = inputs.with_wind(inputs.config1(heterogeneous=True, ncols=3))
    qn, qref = inputs.perturbed_state(col)
    b = qn - qref
    lam = 25.0
    x = oracle.solve_batch(col, lam, b, refine=1)
    Q = sla.expm(np.array([[0, -0.3, 0.5], [0.3, 0, -0.7], [-0.5, 0.7, 0]]))
    col2 = dict(col)
    col2["gz"] = np.einsum("ij,jkc->ikc", Q, col["gz"])
    col2["U0"] = np.einsum("ij,jkc->ikc", Q, col["U0"])
    b2 = b.copy()
    b2[1:4] = np.einsum("ij,jkc->ikc", Q, b[1:4])
    x2 = oracle.solve_batch(col2, lam, b2, refine=1)
    xr = x.copy()
    xr[1:4] = np.einsum("ij,jkc->ikc", Q, x[1:4])
    for c in range(3):
        assert relerr_per_var(oracle.vec_of(x2, c), oracle.vec_of(xr, c)) < 1e-13


# ---------------------------------------------------------------------------
# NHEVI-LU (Sec. 4.2.2): Newton on F(q) = q - Lambda V(q) - R per implicit stage

def test_nhevi_vertical_op_derivative():
    """Centred differences of the oracle's nonlinear operator V at a moving state equal
    the LHEVI-PS Jacobian there (two independent derivations of the same operator), and
    V conserves column mass (flux form, rigid lid)."""
    col = _ps_col()
    qn, qref = inputs.perturbed_state(col)
    for c in range(2):
        z, J, gz, r0, T0 = oracle.column_of(col, c)
        L = oracle.column_L(4, 6, CONSTS, z, J, gz, r0, T0, U0_k3=oracle.u0_of(col, c))
        q0 = oracle.vec_of(qref, c)
        v = oracle.vec_of(qn - qref, c)
        eps = 1e-2
        fd = (oracle.vertical_op(4, 6, CONSTS, z, J, gz, q0 + eps * v)
              - oracle.vertical_op(4, 6, CONSTS, z, J, gz, q0 - eps * v)) / (2 * eps)
        Lv = L @ v
        for k in range(5):
            assert np.linalg.norm(fd[k::5] - Lv[k::5]) < 1e-9 * np.linalg.norm(Lv[k::5]), (c, k)
        # the numpy operator written from the fluxes in this file agrees too
        assert np.allclose(oracle.vertical_op(4, 6, CONSTS, z, J, gz, q0 + v),
                           _nonlinear_V(col, c, q0 + v), rtol=1e-12, atol=1e-14 * np.abs(q0).max())
        _, w, _ = oracle.gll(4)
        M = np.zeros(len(z))
        for e in range(6):
            for i in range(5):
                M[4 * e + i] += w[i] * J[4 * e + i]
        V = oracle.vertical_op(4, 6, CONSTS, z, J, gz, q0 + v)
        assert abs(M @ V[0::5]) <= 1e-13 * (M @ np.abs(V[0::5]))


def test_nhevi_newton_converges_quadratically():
    """Distance to the stage roots after 1, 2, 3 Newton iterations (fixed counts):
    quadratic convergence (catches a wrong Jacobian, which converges linearly at best,
    or a wrong sign of the update)."""
    col = inputs.config1(heterogeneous=True, ncols=2)
    tab = tableaux.as_float(tableaux.ark2("b"))
    qn, _ = inputs.perturbed_state(col, amp=1e-2)
    root, _ = oracle.nhevi_step_batch(col, tab, 30.0, qn, tol=0.0, maxit=10)
    d = []
    for m in (1, 2, 3):
        qm, its = oracle.nhevi_step_batch(col, tab, 30.0, qn, tol=0.0, maxit=m)
        assert np.all(its == m)
        d.append(max(np.linalg.norm((qm - root)[v]) / np.linalg.norm((root - qn)[v])
                     for v in range(5)))
    assert d[0] < 0.1 and d[1] < 10 * d[0] ** 2 and d[2] < 1e-12, d


def test_nhevi_linear_limit():
    """For a small perturbation of the reference state the NHEVI-LU step's response
    (the step of q_ref + delta minus that of q_ref) tends to the implicit Runge-Kutta
    step of the linearised operator L_z applied to delta, written here directly from the
    tableau; the relative difference falls linearly with the amplitude (the neglected
    terms are quadratic).  Catches a wrong stage right-hand side R, a wrong final
    combination or a Newton solve that does not reach the root."""
    col = inputs.config1(heterogeneous=True, ncols=1)
    tab = tableaux.as_float(tableaux.ark2("b"))
    dt = 30.0
    A, b = np.array(tab["Aimp"]), np.array(tab["b"])
    z, J, gz, r0, T0 = oracle.column_of(col, 0)
    L = oracle.column_L(4, 8, CONSTS, z, J, gz, r0, T0)
    n = L.shape[0]
    errs = []
    for amp in (1e-3, 1e-4):
        qn, qref = inputs.perturbed_state(col, amp=amp)
        q1, _ = oracle.nhevi_step_batch(col, tab, dt, qn, tol=1e-10, maxit=10)
        q0, _ = oracle.nhevi_step_batch(col, tab, dt, qref, tol=1e-10, maxit=10)
        d = oracle.vec_of(qn - qref, 0)
        Qs = [d]
        for i in range(1, len(b)):
            rhs = d + dt * sum(A[i][j] * (L @ Qs[j]) for j in range(i))
            Qs.append(np.linalg.solve(np.eye(n) - dt * A[i][i] * L, rhs))
        dl = d + dt * sum(b[i] * (L @ Qs[i]) for i in range(len(b)))
        dn = oracle.vec_of(q1 - q0, 0)
        errs.append(max(np.linalg.norm(dn[v::5] - dl[v::5]) / np.linalg.norm(dl[v::5])
                        for v in range(5)))
    assert errs[1] < 1e-3 and 5 < errs[0] / errs[1] < 20, errs


def test_nhevi_mass_conservation():
    """The NHEVI-LU step conserves column mass: sum_k M_k rho_k."""
    col = inputs.config1(heterogeneous=True, ncols=3)
    tab = tableaux.as_float(tableaux.ark3())
    qn, _ = inputs.perturbed_state(col, amp=1e-2)
    q1, _ = oracle.nhevi_step_batch(col, tab, 30.0, qn, tol=1e-10, maxit=8)
    w = np.array([float(v) for v in GLL_CLOSED[4][1]])
    for c in range(3):
        M = np.zeros(col["nz"])
        for e in range(col["Ne"]):
            for i in range(5):
                M[4 * e + i] += w[i] * col["J"][4 * e + i, c]
        assert abs(M @ q1[0, :, c] - M @ qn[0, :, c]) <= 1e-14 * (M @ qn[0, :, c])
