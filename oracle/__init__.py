"""Serial FP64 reference (oracle) for the batched LHEVI column solve.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` are the only callers.  The product path
(``paper_2311_11425_amd``) never imports this package, and this package imports
nothing from the product.

The arithmetic lives in ``hevi_oracle.c`` (plain C, built with gcc into
``libhevi_oracle.so`` next to this file); this module only marshals numpy
arrays.  Array layout matches the batched convention used throughout: a per-node
field is ``[k][c]`` (column index fastest), a state vector ``[v][k][c]`` with
``v = (rho, rho u, rho v, rho w, q_T)`` with ``q_T`` the thermodynamic variable of
the equation set (``Theta = rho theta`` for set 2C, the total energy ``E`` for
set 3C), ``grad(zeta)`` is ``[m][k][c]``.  A column batch names its set in
``col["eqset"]`` ("2C" when absent); a set-3C batch carries ``E0``.  A batch with
``col["U0"]`` (momentum [m][k][c] of a moving linearisation state, set 2C) is solved
with the LHEVI-PS operator: the Jacobian of the vertical operator at (rho0, U0, Theta0).

Parity status per function is documented in ``hevi_oracle.c``; every function
has at least one pin in ``tests/test_oracle_pins.py``.  The ARK tableaux in
``oracle/tableaux.py`` are pinned only by their order conditions and the
observed convergence order (the coefficients of the third-order method are not
printed in the paper): "parity unpinned" by the paper itself for those numbers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hevi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhevi_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no BLAS) into libhevi_oracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-shared", "-fPIC", "-pthread",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ho_gll.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        lib.ho_gll.restype = ctypes.c_int
        lib.ho_reference.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, _dp, _dp]
        lib.ho_reference.restype = None
        lib.ho_reference_3c.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        lib.ho_reference_3c.restype = None
        lib.ho_assemble_L.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp,
                                      _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        lib.ho_assemble_L.restype = ctypes.c_int
        lib.ho_jacobian_2c.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.ho_jacobian_2c.restype = None
        lib.ho_assemble_L_K.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp,
                                        _dp, ctypes.c_int, _dp]
        lib.ho_assemble_L_K.restype = ctypes.c_int
        lib.ho_bc_project.argtypes = [ctypes.c_int, _dp, _dp]
        lib.ho_bc_project.restype = None
        lib.ho_form_A.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        lib.ho_form_A.restype = None
        lib.ho_lu_factor.argtypes = [ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int)]
        lib.ho_lu_factor.restype = ctypes.c_int
        lib.ho_lu_solve.argtypes = [ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int), _dp, _dp]
        lib.ho_lu_solve.restype = None
        lib.ho_solve_refined.argtypes = [ctypes.c_int, _dp, _dp, ctypes.POINTER(ctypes.c_int),
                                         _dp, _dp, ctypes.c_int, _dp]
        lib.ho_solve_refined.restype = None
        common = [ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                  _dp]
        lib.ho_solve_batch.argtypes = common + [ctypes.c_double, _dp, _dp, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, _dp,
                                                ctypes.POINTER(ctypes.c_long)]
        lib.ho_solve_batch.restype = ctypes.c_int
        lib.ho_apply_batch.argtypes = common + [_dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp,
                                                ctypes.POINTER(ctypes.c_long)]
        lib.ho_apply_batch.restype = ctypes.c_int
        lib.ho_ark_step_batch.argtypes = common + [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                                   ctypes.c_double, _dp, _dp, _dp, _dp, _dp,
                                                   ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_long)]
        lib.ho_ark_step_batch.restype = ctypes.c_int
        lib.ho_vertical_op.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                       ctypes.c_int, _dp]
        lib.ho_vertical_op.restype = ctypes.c_int
        lib.ho_nhevi_step_batch.argtypes = common + [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp,
                                                     ctypes.c_double, ctypes.c_int, _dp, _dp, _dp,
                                                     ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                                     ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
        lib.ho_nhevi_step_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# small per-column building blocks (Sec. 3, Appendix A)

def gll(N: int):
    """GLL nodes, weights and D[i, j] = h_j'(xi_i) for order N."""
    lib = _load()
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    D = np.zeros((N + 1, N + 1))
    if lib.ho_gll(N, _p(xi), _p(w), _p(D)) != 0:
        raise ValueError("order out of range")
    return xi, w, D


def reference(rho0, Theta0, consts):
    """theta0 and c_Theta = dP/dTheta from the set-2C equation of state."""
    lib = _load()
    rho0 = _f64(rho0)
    Theta0 = _f64(Theta0)
    th = np.zeros_like(rho0)
    cT = np.zeros_like(rho0)
    R, cp, g, pA = consts
    lib.ho_reference(rho0.size, _p(rho0), _p(Theta0), R, cp, pA, _p(th), _p(cT))
    return th, cT


def reference_3c(rho0, E0, z, consts):
    """Set-3C coefficients at rest: h = (E0 + P0)/rho0, dP/dE, dP/drho."""
    lib = _load()
    rho0, E0, z = _f64(rho0), _f64(E0), _f64(z)
    hE, dPdE, dPdr = (np.zeros_like(rho0) for _ in range(3))
    R, cp, g, pA = consts
    lib.ho_reference_3c(rho0.size, _p(rho0), _p(E0), _p(z), R, cp, g, _p(hE), _p(dPdE),
                        _p(dPdr))
    return hE, dPdE, dPdr


def assemble_L(N, Ne, g, z, J, gz_k3, hq, cq, pr=None, rho_weak=True, theta_weak=False):
    """Dense L_z of ONE column.  gz_k3 is [k][3]; hq, cq, pr are the flux
    coefficient, dP/dq_T and dP/drho per node (pr None: zero, set 2C).
    Returns (5nz x 5nz)."""
    lib = _load()
    nz = Ne * N + 1
    L = np.zeros((5 * nz, 5 * nz))
    args = [_f64(a) for a in (z, J, gz_k3, hq, cq)]
    prp = _f64(pr) if pr is not None else None
    rc = lib.ho_assemble_L(N, Ne, g, *[_p(a) for a in args], _p(prp), int(rho_weak),
                           int(theta_weak), _p(L))
    if rc:
        raise ValueError("assemble failed")
    return L


def jacobian_2c(gz_k3, rho0, U0_k3, Theta0, cTheta):
    """Set-2C flux Jacobian at (rho0, U0, Theta0) per node: array [k][5][5]."""
    lib = _load()
    nz = len(rho0)
    K = np.zeros((nz, 5, 5))
    lib.ho_jacobian_2c(nz, *[_p(_f64(a)) for a in (gz_k3, rho0, U0_k3, Theta0, cTheta)], _p(K))
    return K


def assemble_L_K(N, Ne, g, z, J, gz_k3, K, rho_weak=True):
    """Dense L_z from per-node flux Jacobians K [k][5][5]."""
    lib = _load()
    nz = Ne * N + 1
    L = np.zeros((5 * nz, 5 * nz))
    rc = lib.ho_assemble_L_K(N, Ne, g, *[_p(_f64(a)) for a in (z, J, gz_k3, K)], int(rho_weak),
                             _p(L))
    if rc:
        raise ValueError("assemble failed")
    return L


def column_L(N, Ne, consts, z, J, gz_k3, rho0, thermo0, rho_weak=True, theta_weak=False,
             eqset="2C", U0_k3=None):
    """Dense L_z of one column of set ``eqset``; thermo0 is Theta0 (2C) or E0 (3C).
    U0_k3 ([k][3], set 2C): LHEVI-PS, the Jacobian at (rho0, U0, Theta0)."""
    if U0_k3 is not None:
        hq, cq = reference(rho0, thermo0, consts)
        K = jacobian_2c(gz_k3, rho0, U0_k3, thermo0, cq)
        return assemble_L_K(N, Ne, consts[2], z, J, gz_k3, K, rho_weak)
    if eqset == "3C":
        hq, cq, pr = reference_3c(rho0, thermo0, z, consts)
    else:
        hq, cq = reference(rho0, thermo0, consts)
        pr = None
    return assemble_L(N, Ne, consts[2], z, J, gz_k3, hq, cq, pr, rho_weak, theta_weak)


def bc_project(nz, gz_k3, b):
    lib = _load()
    b = _f64(b).copy()
    lib.ho_bc_project(nz, _p(_f64(gz_k3)), _p(b))
    return b


def form_A(L, lam):
    lib = _load()
    L = _f64(L)
    A = np.zeros_like(L)
    lib.ho_form_A(L.shape[0], lam, _p(L), _p(A))
    return A


def lu_solve_dense(A, b, refine=0):
    """x = A^{-1} b by the oracle's GEPP (+ long-double refinement steps)."""
    lib = _load()
    A = _f64(A)
    n = A.shape[0]
    LU = A.copy()
    piv = np.zeros(n, dtype=np.int32)
    rc = lib.ho_lu_factor(n, _p(LU), piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc:
        raise ZeroDivisionError(f"zero pivot at step {rc - 1}")
    x = np.zeros(n)
    work = np.zeros(n)
    lib.ho_solve_refined(n, _p(A), _p(LU), piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                         _p(_f64(b)), _p(x), refine, _p(work))
    return x


# --------------------------------------------------------------------------
# batched drivers (columns stored column-fastest)

def _eqset(col):
    """0 for set 2C, 1 for set 3C."""
    return 1 if col.get("eqset", "2C") == "3C" else 0


def _thermo_key(col):
    return "E0" if _eqset(col) else "Theta0"


def _geom_args(col):
    return [_f64(col[k]) for k in ("z", "J", "gz", "rho0", _thermo_key(col))]


def _u0(col):
    """LHEVI-PS linearisation momentum [m][k][c], or None (state at rest)."""
    return _f64(col["U0"]) if col.get("U0") is not None else None


def solve_batch(col, lam, b, refine=1, rho_weak=True, nthreads=None):
    """x = (I - lam L_z)^{-1} P(b) for every column of the batch ``col``."""
    lib = _load()
    N, Ne = col["N"], col["Ne"]
    ncols = col["z"].shape[1]
    g = _geom_args(col)
    b = _f64(b)
    x = np.zeros_like(b)
    bad = ctypes.c_long(-1)
    consts = _f64(col["consts"])
    rc = lib.ho_solve_batch(N, Ne, ncols, nthreads or os.cpu_count() or 1, _p(consts),
                            *[_p(a) for a in g], lam, _p(b), _p(x), refine, int(rho_weak),
                            _eqset(col), _p(_u0(col)), ctypes.byref(bad))
    if rc:
        raise RuntimeError(f"oracle solve failed ({rc}) at column {bad.value}")
    return x


def apply_batch(col, x, xref=None, rho_weak=True, nthreads=None):
    """y = L_z (x - xref) for every column."""
    lib = _load()
    N, Ne = col["N"], col["Ne"]
    ncols = col["z"].shape[1]
    g = _geom_args(col)
    x = _f64(x)
    xr = _f64(xref) if xref is not None else None
    y = np.zeros_like(x)
    bad = ctypes.c_long(-1)
    consts = _f64(col["consts"])
    rc = lib.ho_apply_batch(N, Ne, ncols, nthreads or os.cpu_count() or 1, _p(consts),
                            *[_p(a) for a in g], _p(x), _p(xr), _p(y), int(rho_weak),
                            _eqset(col), _p(_u0(col)), ctypes.byref(bad))
    if rc:
        raise RuntimeError(f"oracle apply failed ({rc}) at column {bad.value}")
    return y


def ark_step_batch(col, tab, dt, qn, qref, refine=1, rho_weak=True, nthreads=None,
                   want_stages=False, omega=0.0):
    """One LHEVI ARK step.  ``tab`` holds float arrays Aexp, Aimp (s x s), b (s).

    ``omega`` adds the explicit Coriolis term -2 omega n x U (time-convergence
    studies only).  Returns q^{n+1} and, if requested, the stage values Q and tendencies S as
    arrays [s][v][k][c]."""
    lib = _load()
    N, Ne = col["N"], col["Ne"]
    ncols = col["z"].shape[1]
    g = _geom_args(col)
    Aexp = _f64(tab["Aexp"])
    Aimp = _f64(tab["Aimp"])
    bw = _f64(tab["b"])
    s = bw.size
    qn = _f64(qn)
    qref = _f64(qref)
    qnp1 = np.zeros_like(qn)
    Q = np.zeros((s,) + qn.shape) if want_stages else None
    S = np.zeros((s,) + qn.shape) if want_stages else None
    bad = ctypes.c_long(-1)
    consts = _f64(col["consts"])
    rc = lib.ho_ark_step_batch(N, Ne, ncols, nthreads or os.cpu_count() or 1, _p(consts),
                               *[_p(a) for a in g], s, _p(Aexp), _p(Aimp), _p(bw), dt, omega,
                               _p(qn),
                               _p(qref), _p(qnp1), _p(Q), _p(S), refine, int(rho_weak),
                               _eqset(col), _p(_u0(col)), ctypes.byref(bad))
    if rc:
        raise RuntimeError(f"oracle ARK step failed ({rc}) at column {bad.value}")
    if want_stages:
        return qnp1, Q, S
    return qnp1


def u0_of(col, c):
    """The LHEVI-PS linearisation momentum of column c as [k][3] (None at rest)."""
    return None if col.get("U0") is None else np.ascontiguousarray(col["U0"][:, :, c].T)


def column_of(col, c):
    """Per-column arrays of column c: z, J, gz [k][3], rho0 and the set's
    thermodynamic reference (Theta0 for 2C, E0 for 3C)."""
    gz = np.ascontiguousarray(col["gz"][:, :, c].T)
    return (np.ascontiguousarray(col["z"][:, c]), np.ascontiguousarray(col["J"][:, c]), gz,
            np.ascontiguousarray(col["rho0"][:, c]),
            np.ascontiguousarray(col[_thermo_key(col)][:, c]))


def vec_of(v, c):
    """Column c of a batched state [v][k][c] as the interleaved vector (5k+v)."""
    return np.ascontiguousarray(v[:, :, c].T).reshape(-1)


def vertical_op(N, Ne, consts, z, J, gz_k3, q, rho_weak=True):
    """Nonlinear set-2C vertical operator V(q) of one column (q interleaved 5k+v)."""
    lib = _load()
    q = _f64(q)
    V = np.zeros_like(q)
    rc = lib.ho_vertical_op(N, Ne, _p(_f64(consts)), *[_p(_f64(a)) for a in (z, J, gz_k3)],
                            _p(q), int(rho_weak), _p(V))
    if rc:
        raise ValueError("vertical operator failed")
    return V


def nhevi_step_batch(col, tab, dt, qn, tol=1e-12, maxit=8, refine=1, rho_weak=True,
                     nthreads=None, want_stages=False):
    """One NHEVI-LU step (Newton per implicit stage with the Jacobian rebuilt at every
    iterate) of every column; ``tab`` as for ark_step_batch (only Aimp and b are used:
    there is no explicit operator).  Returns q^{n+1}, the per-column Newton iteration
    counts and, if requested, the stage values Q and V(Q) as [s][v][k][c]."""
    lib = _load()
    N, Ne = col["N"], col["Ne"]
    ncols = col["z"].shape[1]
    g = _geom_args(col)
    Aimp = _f64(tab["Aimp"])
    bw = _f64(tab["b"])
    s = bw.size
    qn = _f64(qn)
    qnp1 = np.zeros_like(qn)
    Q = np.zeros((s,) + qn.shape) if want_stages else None
    V = np.zeros((s,) + qn.shape) if want_stages else None
    its = np.zeros(ncols, dtype=np.int32)
    bad = ctypes.c_long(-1)
    consts = _f64(col["consts"])
    rc = lib.ho_nhevi_step_batch(N, Ne, ncols, nthreads or os.cpu_count() or 1, _p(consts),
                                 *[_p(a) for a in g], s, _p(Aimp), _p(bw), dt, _p(qn), tol,
                                 maxit, _p(qnp1), _p(Q), _p(V),
                                 its.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), refine,
                                 int(rho_weak), ctypes.byref(bad))
    if rc:
        raise RuntimeError(f"oracle NHEVI step failed ({rc}) at column {bad.value}")
    if want_stages:
        return qnp1, its, Q, V
    return qnp1, its
