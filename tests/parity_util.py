"""Helpers shared by the GPU parity tests (not collected by pytest)."""
from __future__ import annotations

import numpy as np


def relerr_cols(a, ref, floor=0.0):
    """Max over (variable, column) of ||a[v,:,c] - ref[v,:,c]||_2 / ||ref[v,:,c]||_2.

    Arrays are [v][k][c].  Pairs whose reference norm is <= floor are compared
    against the largest reference norm of that column instead."""
    a = np.asarray(a)
    ref = np.asarray(ref)
    num = np.sqrt(((a - ref) ** 2).sum(axis=1))          # (v, c)
    den = np.sqrt((ref ** 2).sum(axis=1))                # (v, c)
    colmax = den.max(axis=0, keepdims=True)
    den = np.where(den > floor, den, colmax)
    den = np.where(den > 0, den, 1.0)
    return float((num / den).max()) if num.size else 0.0


def sub_batch(col, idx):
    """The columns idx of a batch as a new batch (columns are independent)."""
    out = dict(col)
    for k in ("z", "J", "rho0", "Theta0", "E0", "T"):
        if k in col:
            out[k] = np.ascontiguousarray(col[k][:, idx])
    out["gz"] = np.ascontiguousarray(col["gz"][:, :, idx])
    out["nhat"] = np.ascontiguousarray(col["nhat"][idx])
    out["ncols"] = len(idx)
    return out


def sub_state(q, idx):
    return np.ascontiguousarray(q[..., idx])


def increment_floor(oracle, col, tab, dt, qn, qref, Q, trials=2, seed=0):
    """Arithmetic floor of a step-level comparison: the relative change of the
    increment q^{n+1} - q^n when every stage value Q_i is perturbed by one unit
    of FP64 rounding (relative 2^-52).  S(Q) = L_z (Q - q_ref) subtracts a
    reference state about 10^3 times larger than the perturbation and L_z
    differentiates, so two correct FP64 implementations can differ by this much.
    """
    rng = np.random.default_rng(seed)
    eps = 2.0 ** -52
    b = tab["b"]
    s = len(b)
    base = qn + dt * sum(b[i] * oracle.apply_batch(col, Q[i], qref) for i in range(s))
    worst = 0.0
    for _ in range(trials):
        Sp = [oracle.apply_batch(col, Q[i] * (1 + eps * rng.uniform(-1, 1, Q[i].shape)), qref)
              for i in range(s)]
        qp = qn + dt * sum(b[i] * Sp[i] for i in range(s))
        worst = max(worst, relerr_cols(qp - qn, base - qn))
    return worst


def increment_sensitivity(oracle, col, tab, dt, qn, qref, Q, rel, trials=2, seed=1):
    """Relative change of q^{n+1} - q^n when every stage increment Q_i - q^n is
    perturbed elementwise by a relative amount `rel` (the parity bar of a stage
    solve).  The end-of-step update evaluates S = L_z (Q - q_ref) explicitly at a
    step far beyond its explicit stability limit, so it amplifies stage errors."""
    rng = np.random.default_rng(seed)
    b = tab["b"]
    s = len(b)
    base = qn + dt * sum(b[i] * oracle.apply_batch(col, Q[i], qref) for i in range(s))
    worst = 0.0
    for _ in range(trials):
        Sp = []
        for i in range(s):
            d = Q[i] - qn
            Sp.append(oracle.apply_batch(col, Q[i] + rel * d * rng.uniform(-1, 1, d.shape), qref))
        qp = qn + dt * sum(b[i] * Sp[i] for i in range(s))
        worst = max(worst, relerr_cols(qp - qn, base - qn))
    return worst


def step_tolerance(oracle, col, tab, dt, qn, qref, Q, bar):
    """max(bar, 4 x rounding floor, 2 x sensitivity of the update to stage errors at the bar)."""
    return max(bar, 4 * increment_floor(oracle, col, tab, dt, qn, qref, Q),
               2 * increment_sensitivity(oracle, col, tab, dt, qn, qref, Q, bar))


def stage_floor(oracle, col, lam, qE, P, Qi, x, seed=2):
    """Rounding floor of a stage-solve comparison whose input q^ = q^E + P and
    output q_tt = Q_i + P are formed from reference-sized terms that cancel:
    perturb q^ by one ulp of |q^E| + |P| and q_tt by one ulp of |Q_i| + |P|."""
    rng = np.random.default_rng(seed)
    eps = 2.0 ** -52
    noise_in = eps * (np.abs(qE) + np.abs(P)) * rng.uniform(-1, 1, qE.shape)
    x_in = oracle.solve_batch(col, lam, qE + P + noise_in, refine=1)
    noise_out = eps * (np.abs(Qi) + np.abs(P)) * rng.uniform(-1, 1, Qi.shape)
    return relerr_cols(x_in, x) + relerr_cols(x + noise_out, x)
