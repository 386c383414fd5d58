"""Seeded synthetic column inputs shared by tests and the benchmark.

This module holds no arithmetic of the method: it only builds grids, reference
atmospheres and perturbations (the inputs of the column solve).  Neither the
oracle nor the HIP library import it; both receive the arrays it produces.

Recipes (the paper's baroclinic-instability and gravity-wave set-ups, Sec. 7,
are stood in for by their vertical structure: 30 km model top, order-4 GLL
elements, hydrostatic stratified reference):

* geometry: shallow, terrain-following column between the surface height z_s
  and the model top; N_e uniform elements; node heights at the GLL points of
  each element; metric Jacobian J = (h/2) * J_h (J_h a per-column horizontal
  area factor, constant along the column); grad(zeta) = (2/h) n with n the
  radial unit vector of the column, drawn uniformly on the sphere.  Optional
  per-node tilt of grad(zeta) and a deep-atmosphere factor on J exercise the
  general per-node metric inputs.
* reference state: hydrostatic p(z) for an isothermal or piecewise lapse-rate
  temperature profile (closed forms), rho0 = p/(R T),
  Theta0 = rho0 T (P_A/p)^(R/c_p), at rest; for set 3C (total energy) the same
  atmosphere as E0 = rho0 c_v T + rho0 g z (internal plus potential energy).
* perturbation: drho = 1e-3 rho0 xi, dq_T = 1e-3 q_T0 xi (q_T = Theta or E),
  dU = 1e-3 rho0 c0 xi_vec with c0 = sqrt(gamma R T) and xi ~ U(-1, 1); the
  normal momentum at the bottom and top nodes is removed.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as _leg

R_DRY = 287.0
CP_DRY = 1004.5
GRAV = 9.80616
P_A = 1.0e5
CONSTS = (R_DRY, CP_DRY, GRAV, P_A)
EARTH_R = 6.371e6


def _gll_nodes(N):
    # node positions for placing grid points (library routine, grid generation only)
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = np.sort(_leg.Legendre.basis(N).deriv().roots().real)
    return np.concatenate([[-1.0], inner, [1.0]])


def temperature_profile(kind, z):
    z = np.asarray(z, dtype=np.float64)
    if kind == "isothermal":
        return np.full_like(z, 300.0)
    if kind == "lapse":
        return 310.0 - 6.5e-3 * z
    if kind == "lapse_capped":
        return np.maximum(310.0 - 6.5e-3 * z, 200.0)
    raise ValueError(kind)


def hydrostatic_pressure(kind, z, p_s=1.0e5):
    """Closed-form hydrostatic p(z) with p(0) = p_s for the profile ``kind``."""
    z = np.asarray(z, dtype=np.float64)
    if kind == "isothermal":
        return p_s * np.exp(-GRAV * z / (R_DRY * 300.0))
    lapse = 6.5e-3
    T0 = 310.0
    expo = GRAV / (R_DRY * lapse)
    if kind == "lapse":
        return p_s * ((T0 - lapse * z) / T0) ** expo
    if kind == "lapse_capped":
        z_c = (T0 - 200.0) / lapse
        p_c = p_s * (200.0 / T0) ** expo
        below = p_s * ((T0 - lapse * np.minimum(z, z_c)) / T0) ** expo
        above = p_c * np.exp(-GRAV * (z - z_c) / (R_DRY * 200.0))
        return np.where(z <= z_c, below, above)
    raise ValueError(kind)


def random_unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def make_columns(N, Ne, ncols, *, z_top=30.0e3, z_s=None, profile="isothermal", seed=1,
                 surface_seed=None, surface_max=0.0, tilt=0.0, deep=False, J_h=None):
    """Batch of ``ncols`` columns: dict with N, Ne, consts and the per-node fields
    z, J, rho0, Theta0 ([k][c]) and gz ([m][k][c])."""
    rng = np.random.default_rng(seed)
    nz = Ne * N + 1
    nhat = random_unit_vectors(rng, ncols)                      # (c, 3)
    if z_s is None:
        if surface_max > 0.0:
            srng = np.random.default_rng(surface_seed if surface_seed is not None else seed + 1)
            z_s = srng.uniform(0.0, surface_max, ncols)
        else:
            z_s = np.zeros(ncols)
    z_s = np.broadcast_to(np.asarray(z_s, dtype=np.float64), (ncols,)).copy()
    xi = _gll_nodes(N)
    h = (z_top - z_s) / Ne                                      # (c,)
    pos = np.zeros(nz)
    for e in range(Ne):
        for i in range(N + 1):
            pos[e * N + i] = e + 0.5 * (xi[i] + 1.0)
    pos[-1] = Ne
    z = z_s[None, :] + pos[:, None] * h[None, :]                # (k, c)
    if J_h is None:
        J_h = np.ones(ncols)
    J = np.broadcast_to(0.5 * h * J_h, (nz, ncols)).copy()
    if deep:
        J = J * ((EARTH_R + z) / EARTH_R) ** 2
    gz = np.empty((3, nz, ncols))
    for m in range(3):
        gz[m] = (2.0 / h)[None, :] * nhat[:, m][None, :]
    if tilt > 0.0:
        trng = np.random.default_rng(seed + 7)
        gz = gz + tilt * (2.0 / h)[None, None, :] * trng.uniform(-1, 1, gz.shape)
    T = temperature_profile(profile, z)
    p = hydrostatic_pressure(profile, z)
    rho0 = p / (R_DRY * T)
    theta = T * (P_A / p) ** (R_DRY / CP_DRY)
    Theta0 = rho0 * theta
    E0 = rho0 * (CP_DRY - R_DRY) * T + rho0 * GRAV * z
    return {"N": N, "Ne": Ne, "nz": nz, "ncols": ncols, "consts": np.array(CONSTS),
            "z": np.ascontiguousarray(z), "J": np.ascontiguousarray(J),
            "gz": np.ascontiguousarray(gz), "rho0": np.ascontiguousarray(rho0),
            "Theta0": np.ascontiguousarray(Theta0), "E0": np.ascontiguousarray(E0), "T": T,
            "nhat": nhat, "profile": profile, "z_top": z_top, "eqset": "2C"}


def as_set(col, eqset):
    """The same batch with its equation set switched ("2C": state (rho, U, Theta);
    "3C": state (rho, U, E))."""
    if eqset not in ("2C", "3C"):
        raise ValueError(eqset)
    out = dict(col)
    out["eqset"] = eqset
    return out


def thermo0(col):
    """The reference of the set's thermodynamic variable: Theta0 (2C) or E0 (3C)."""
    return col["E0"] if col.get("eqset", "2C") == "3C" else col["Theta0"]


def with_wind(col, u_h=20.0, w0=0.5, seed=13):
    """The batch with a moving linearisation state (LHEVI-PS, a previous solution):
    momentum U0 = rho0 (u_t(z) + w(z) n) with a horizontal wind u_t tangential to the
    column, growing linearly from 0.5 u_h at the bottom to 1.5 u_h at the top in a random
    tangential direction, and a vertical wind w = w0 sin(pi s) (s the normalised
    height) that vanishes at the bottom and top nodes, as the rigid lid requires."""
    rng = np.random.default_rng(seed)
    out = dict(col)
    z = col["z"]
    s = (z - z[:1]) / (z[-1:] - z[:1])
    nh = col["nhat"]                                           # (c, 3)
    t = rng.standard_normal(nh.shape)
    t -= (t * nh).sum(1, keepdims=True) * nh
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    w = w0 * np.sin(np.pi * s)
    w[0] = 0.0
    w[-1] = 0.0
    U0 = np.empty((3,) + z.shape)
    for m in range(3):
        U0[m] = col["rho0"] * (u_h * (0.5 + s) * t[:, m][None, :] + w * nh[:, m][None, :])
    out["U0"] = np.ascontiguousarray(U0)
    return out


def reference_vector(col):
    """q_ref = (rho0, U0 or 0, Theta0 or E0) as [v][k][c] (U0: a moving linearisation
    state, see with_wind)."""
    q = np.zeros((5,) + col["rho0"].shape)
    q[0] = col["rho0"]
    if col.get("U0") is not None:
        q[1:4] = col["U0"]
    q[4] = thermo0(col)
    return q


def _remove_boundary_normal(col, q):
    gz = col["gz"]
    for k in (0, gz.shape[1] - 1):
        n = gz[:, k, :] / np.linalg.norm(gz[:, k, :], axis=0, keepdims=True)
        d = (n * q[1:4, k, :]).sum(0)
        q[1:4, k, :] -= n * d[None, :]
    return q


def perturbed_state(col, seed=3, amp=1.0e-3):
    """q^n = q_ref + perturbation (uniform noise of relative size ``amp``)."""
    rng = np.random.default_rng(seed)
    qref = reference_vector(col)
    shape = col["rho0"].shape
    gam = CP_DRY / (CP_DRY - R_DRY)
    c0 = np.sqrt(gam * R_DRY * col["T"])
    q = qref.copy()
    q[0] += amp * col["rho0"] * rng.uniform(-1, 1, shape)
    for m in range(3):
        q[1 + m] += amp * col["rho0"] * c0 * rng.uniform(-1, 1, shape)
    q[4] += amp * thermo0(col) * rng.uniform(-1, 1, shape)
    return _remove_boundary_normal(col, q), qref


def smooth_state(col, amp=1.0e-3, modes=(1, 2)):
    """Low-mode perturbation (for time-convergence studies): sin(m pi s) in the
    normalised height s, same relative amplitudes as ``perturbed_state``."""
    z = col["z"]
    s = (z - z[:1]) / (z[-1:] - z[:1])
    qref = reference_vector(col)
    gam = CP_DRY / (CP_DRY - R_DRY)
    c0 = np.sqrt(gam * R_DRY * col["T"])
    shape = sum(np.sin(m * np.pi * s) / m for m in modes)
    cshape = sum(np.cos(m * np.pi * s) / m for m in modes)
    q = qref.copy()
    q[0] += amp * col["rho0"] * cshape
    q[4] += amp * thermo0(col) * 0.5 * cshape
    nh = col["nhat"].T[:, None, :]
    q[1:4] += amp * col["rho0"] * c0 * shape * nh
    return _remove_boundary_normal(col, q), qref


# named workload recipes ----------------------------------------------------

def config1(heterogeneous=False, ncols=256):
    """256 columns, order 4, 8 elements, isothermal 300 K, 30 km top."""
    return make_columns(4, 8, ncols, z_top=30.0e3, profile="isothermal", seed=1,
                        surface_max=2.0e3 if heterogeneous else 0.0, surface_seed=2)


def config2(ncols=86402):
    """Cubed-sphere ne=30 order-4 column count (6 (30*4)^2 + 2 = 86,402), 10
    elements of order 4, lapse-rate reference (310 K surface, 6.5 K/km)."""
    return make_columns(4, 10, ncols, z_top=30.0e3, profile="lapse", seed=11)


def uneven_problems(n_problems=64, seed=40, col_range=(1000, 50000), scale=1.0):
    """Uneven batch: order N ~ U{3..7}, N_e ~ U{8..16}, columns ~ U[1k, 50k]."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n_problems):
        N = int(rng.integers(3, 8))
        Ne = int(rng.integers(8, 17))
        nc = int(rng.integers(col_range[0], col_range[1] + 1) * scale)
        out.append({"N": N, "Ne": Ne, "ncols": max(nc, 1), "seed": seed * 1000 + p})
    return out


def serving_simulations(n_sims=16, seed=50, scale=1.0):
    """Serving mix: tops {30, 60, 120} km, N_e ~ U{10..40}, order 4, columns
    ~ U[5k, 86,402]; isothermal below 60 km tops, capped lapse rate otherwise."""
    rng = np.random.default_rng(seed)
    tops = [30.0e3, 60.0e3, 120.0e3]
    out = []
    for s in range(n_sims):
        top = tops[int(rng.integers(0, 3))]
        Ne = int(rng.integers(10, 41))
        nc = int(rng.integers(5000, 86403) * scale)
        prof = "isothermal" if rng.random() < 0.5 else "lapse_capped"
        out.append({"N": 4, "Ne": Ne, "ncols": max(nc, 1), "z_top": top, "profile": prof,
                    "seed": seed * 1000 + s})
    return out


def spec_columns(spec):
    """The column batch of one problem spec from uneven_problems or
    serving_simulations (isothermal 300 K and a 30 km top unless the spec says
    otherwise)."""
    return make_columns(spec["N"], spec["Ne"], spec["ncols"], z_top=spec.get("z_top", 30.0e3),
                        profile=spec.get("profile", "isothermal"), seed=spec["seed"])
