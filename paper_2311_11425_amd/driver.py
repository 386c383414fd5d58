"""Device-resident column batches and the LHEVI ARK step as a sequence of C-ABI calls.

Orchestration only: every arithmetic step runs in libhevi.so kernels
(hevi_apply_op, hevi_factor / hevi_refactor, hevi_stage_solve, hevi_combine).
The step follows the LHEVI ARK recipe (Sec. 4.1 stage and update formulas,
Sec. 4.3 eq. lhevi-ark-final-3) with the explicit tendency
S(q) = L_z (q - q_ref):

    Q_1 = q^n;  for i >= 2:  c_j = (a~_ij - a_ij) / a~_ii,
    Q_i = stage_solve(E = {q^n, S_1..S_{i-1}}, e = {1, dt a_i1, ...},
                      Qprev = {Q_1..Q_{i-1}}, c),   S_i = L_z (Q_i - q_ref)
    q^{n+1} = q^n + dt sum_i b_i S_i.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import hevi


def to_dev(a, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


class ColumnBatch:
    """Device copies of one batch of columns and its compact operator."""

    def __init__(self, ctx: hevi.Context, col: dict, device="cuda", stream=None):
        self.ctx = ctx
        self.N, self.Ne = int(col["N"]), int(col["Ne"])
        self.nz = self.N * self.Ne + 1
        self.ncols = int(col["z"].shape[1])
        self.consts = tuple(float(v) for v in col["consts"])
        self.z = to_dev(col["z"], device)
        self.J = to_dev(col["J"], device)
        self.gz = to_dev(col["gz"], device)
        self.rho0 = to_dev(col["rho0"], device)
        # the set's thermodynamic reference: Theta0 (set 2C) or the total energy E0 (3C)
        self.eqset = col.get("eqset", "2C")
        self.Theta0 = to_dev(col["E0"] if self.eqset == "3C" else col["Theta0"], device)
        if col.get("U0") is not None:
            # LHEVI-PS: linearised at the moving state (rho0, U0, Theta0)
            self.U0 = to_dev(col["U0"], device)
            self.ops = ctx.build_column_ops_ps(self.N, self.Ne, self.ncols, self.consts, self.z,
                                               self.J, self.gz, self.rho0, self.U0, self.Theta0,
                                               stream=stream)
        else:
            self.ops = ctx.build_column_ops(self.N, self.Ne, self.ncols, self.consts, self.z,
                                            self.J, self.gz, self.rho0, self.Theta0,
                                            stream=stream, eqset=self.eqset)
        self.device = device

    def empty_state(self):
        return torch.empty((5, self.nz, self.ncols), dtype=torch.float64, device=self.device)


class ArkStepper:
    """One LHEVI ARK time step per call, factors reused across stages."""

    def __init__(self, ctx: hevi.Context, batch: ColumnBatch, tableau="ARK3", dt=300.0,
                 precision=hevi.HEVI_FP64, refine=(4, 1e-13, 0), stream=None):
        self.ctx, self.batch = ctx, batch
        tab = hevi.tableau(tableau)
        self.s = tab["s"]
        self.Aexp, self.Aimp, self.b = tab["Aexp"], tab["Aimp"], tab["b"]
        self.dt = float(dt)
        self.lam = self.Aimp[1][1] * self.dt
        self.precision = precision
        self.refine = refine
        self.Q = [batch.empty_state() for _ in range(self.s)]
        self.S = [batch.empty_state() for _ in range(self.s)]
        self.factors = ctx.factor(batch.ops, self.lam, precision, stream=stream)

    def coeffs(self, i):
        aii = self.Aimp[i][i]
        return [(self.Aimp[i][j] - self.Aexp[i][j]) / aii for j in range(i)]

    def calls(self, qn, qref, out, stream=None):
        """The C-ABI calls of one step, marshalled once: a list of (name, function,
        arguments) for fixed buffers (cached per buffer set and stream)."""
        key = (qn.data_ptr(), qref.data_ptr(), out.data_ptr(), stream)
        if getattr(self, "_calls_key", None) == key:
            return self._calls
        lib, ctx, ops, f = self.ctx.lib, self.ctx, self.batch.ops, self.factors
        st = hevi._stream(stream)
        P = hevi._ptr
        ref = hevi.Refine(*(tuple(self.refine) + (0,) * (3 - len(self.refine))))
        keep = [ref]
        self.Q[0] = qn
        seq = [("refactor", lib.hevi_refactor, (ctx.handle, f.handle, ctypes.c_double(self.lam), st)),
               ("apply_op", lib.hevi_apply_op, (ctx.handle, ops.handle, P(qn), P(qref),
                                                P(self.S[0]), st))]
        for i in range(1, self.s):
            E = [qn] + self.S[:i]
            e = [1.0] + [self.dt * self.Aexp[i][j] for j in range(i)]
            Ep, ep = hevi._ptr_array(E), hevi._dbl_array(e)
            Qp, cp = hevi._ptr_array(self.Q[:i]), hevi._dbl_array(self.coeffs(i))
            keep += [Ep, ep, Qp, cp]
            seq.append(("stage_solve", lib.hevi_stage_solve,
                        (ctx.handle, f.handle, len(E), Ep, ep, i, Qp, cp, P(self.Q[i]),
                         ctypes.byref(ref), None, st)))
            seq.append(("apply_op", lib.hevi_apply_op, (ctx.handle, ops.handle, P(self.Q[i]),
                                                        P(qref), P(self.S[i]), st)))
        V = [qn] + self.S
        Vp, vc = hevi._ptr_array(V), hevi._dbl_array([1.0] + [self.dt * bi for bi in self.b])
        keep += [Vp, vc]
        seq.append(("combine", lib.hevi_combine, (ctx.handle, ops.handle, len(V), Vp, vc, P(out),
                                                  st)))
        self._calls, self._calls_key, self._keep = seq, key, keep
        return seq

    def step(self, qn, qref, out, refactor=True, info=False, stream=None):
        """One ARK step.  info=True waits after every stage solve and returns its
        report (one dict per implicit stage)."""
        if not info:
            for name, fn, args in self.calls(qn, qref, out, stream):
                if name == "refactor" and not refactor:
                    continue
                code = fn(*args)
                if code != 0:
                    raise hevi.HeviError(code, name)
            return []
        ctx, ops = self.ctx, self.batch.ops
        if refactor:
            ctx.refactor(self.factors, self.lam, stream=stream)
        infos = []
        self.Q[0] = qn
        ctx.apply_op(ops, qn, self.S[0], xref=qref, stream=stream)
        for i in range(1, self.s):
            E = [qn] + self.S[:i]
            e = [1.0] + [self.dt * self.Aexp[i][j] for j in range(i)]
            inf = ctx.stage_solve(self.factors, E, e, self.Q[:i], self.coeffs(i), self.Q[i],
                                  refine=self.refine, info=True, stream=stream)
            infos.append(inf)
            ctx.apply_op(ops, self.Q[i], self.S[i], xref=qref, stream=stream)
        ctx.combine(ops, [qn] + self.S, [1.0] + [self.dt * bi for bi in self.b], out,
                    stream=stream)
        return infos


class NheviStepper:
    """One NHEVI-LU time step per call (Sec. 4.2.2).

    Every implicit stage i >= 2 solves F(q) = q - Lambda V(q) - R = 0, R = q^n +
    dt sum_{j<i} a~_ij V(Q_j), by Newton's method from q = Q_{i-1}: per iteration
    V(q), the Jacobian rebuilt at q (hevi_ops_relinearize of the batch's LHEVI-PS
    operator) and factored (hevi_refactor), the increment dq = J^{-1}(R - q + Lambda V(q))
    (hevi_stage_solve), q += dq (hevi_combine), until the measure of
    hevi_newton_increment is <= tol or maxit iterations.  There is no explicit operator
    here; q^{n+1} = q^n + dt sum_i b_i V(Q_i).  The batch's operator is relinearised by
    every step (it ends at the last stage's iterate)."""

    def __init__(self, ctx: hevi.Context, batch: ColumnBatch, tableau="ARK3", dt=300.0,
                 tol=1e-5, maxit=8, stream=None):
        if getattr(batch, "U0", None) is None:
            raise ValueError("NHEVI-LU needs an LHEVI-PS operator (a batch with U0)")
        self.ctx, self.batch = ctx, batch
        tab = hevi.tableau(tableau)
        self.s = tab["s"]
        self.Aimp, self.b = tab["Aimp"], tab["b"]
        self.dt = float(dt)
        self.lam = self.Aimp[1][1] * self.dt
        self.tol, self.maxit = float(tol), int(maxit)
        self.Q = [batch.empty_state() for _ in range(self.s)]
        self.V = [batch.empty_state() for _ in range(self.s)]
        self.R, self.Vq, self.dq = batch.empty_state(), batch.empty_state(), batch.empty_state()
        self.factors = ctx.factor(batch.ops, self.lam, hevi.HEVI_FP64, stream=stream)

    def step(self, qn, out, stream=None):
        """One step; returns the Newton iterations of each implicit stage and the last
        stopping measure of each."""
        ctx, ops, f = self.ctx, self.batch.ops, self.factors
        self.Q[0] = qn
        ctx.vertical_op(ops, qn, self.V[0], stream=stream)
        its, meas = [], []
        for i in range(1, self.s):
            ctx.combine(ops, [qn] + self.V[:i],
                        [1.0] + [self.dt * self.Aimp[i][j] for j in range(i)], self.R,
                        stream=stream)
            q = self.Q[i]
            ctx.combine(ops, [self.Q[i - 1]], [1.0], q, stream=stream)
            rel = float("inf")
            m = 0
            while m < self.maxit:
                m += 1
                ctx.vertical_op(ops, q, self.Vq, stream=stream)
                ctx.relinearize(ops, q[0], q[1:4], q[4], stream=stream)
                ctx.refactor(f, self.lam, stream=stream)
                ctx.stage_solve(f, [self.R, q, self.Vq], [1.0, -1.0, self.lam], [], [],
                                self.dq, stream=stream)
                ctx.combine(ops, [q, self.dq], [1.0, 1.0], q, stream=stream)
                rel = ctx.newton_increment(ops, self.dq, q, qn, stream=stream)
                if rel <= self.tol:
                    break
            its.append(m)
            meas.append(rel)
            ctx.vertical_op(ops, q, self.V[i], stream=stream)
        ctx.combine(ops, [qn] + self.V, [1.0] + [self.dt * bi for bi in self.b], out,
                    stream=stream)
        return its, meas
