"""Thin ctypes binding of the C ABI in include/hevi.h.

Argument marshalling only: every step of the solve runs in the HIP kernels of
libhevi.so.  Device buffers are torch tensors on a ROCm device (torch is used
for device memory and streams only).  If the library is missing the import of
this module fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhevi.so")

HEVI_FP64 = 0
HEVI_FP32_REFINE = 1
HEVI_SET_2C = 0
HEVI_SET_3C = 1
EQSETS = {"2C": HEVI_SET_2C, "3C": HEVI_SET_3C}

STATUS = {0: "HEVI_OK", 1: "HEVI_E_INVALID", 2: "HEVI_E_SHAPE", 3: "HEVI_E_NOMEM",
          4: "HEVI_E_DEVICE", 5: "HEVI_E_SINGULAR", 6: "HEVI_E_NOT_CONVERGED", 7: "HEVI_E_BUSY",
          8: "HEVI_E_CLOSED", 9: "HEVI_E_NONFINITE", 10: "HEVI_E_SCRATCH"}

# every symbol include/hevi.h declares
EXPORTS = ["hevi_create", "hevi_destroy", "hevi_status_str", "hevi_build_column_ops",
           "hevi_build_column_ops_set", "hevi_build_column_ops_ps", "hevi_ops_relinearize",
           "hevi_vertical_op", "hevi_newton_increment",
           "hevi_ops_check", "hevi_ops_free", "hevi_apply_op", "hevi_factor", "hevi_refactor",
           "hevi_factors_check", "hevi_factors_band_entries", "hevi_factors_free",
           "hevi_stage_solve", "hevi_solve_noalloc", "hevi_combine",
           "hevi_tableau", "hevi_sizes", "hevi_group_create", "hevi_group_set_plan",
           "hevi_group_get_plan", "hevi_group_step", "hevi_group_check", "hevi_group_autotune",
           "hevi_group_free", "hevi_serve_create", "hevi_serve_register", "hevi_serve_submit",
           "hevi_serve_poll", "hevi_serve_wait", "hevi_serve_release", "hevi_serve_destroy"]

HEVI_MAX_STAGES = 8
LAUNCH_MODES = {"one": 0, "per_order": 1, "per_member": 2}


class HeviError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [("order_N", ctypes.c_int32), ("n_elem", ctypes.c_int32), ("n_cols", ctypes.c_int64)]


class Consts(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("cp", ctypes.c_double), ("g", ctypes.c_double),
                ("p_A", ctypes.c_double)]


class Refine(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("rel_residual_target", ctypes.c_double),
                ("full_sweeps", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("max_sweeps_used", ctypes.c_int32),
                ("first_bad_col", ctypes.c_int64), ("n_bad_cols", ctypes.c_int64),
                ("max_rel_correction", ctypes.c_double)]

    def as_dict(self):
        return {"status": STATUS.get(self.status, self.status), "max_sweeps_used": self.max_sweeps_used,
                "first_bad_col": self.first_bad_col, "n_bad_cols": self.n_bad_cols,
                "max_rel_correction": self.max_rel_correction}


class GroupMember(ctypes.Structure):
    _fields_ = [("ops", ctypes.c_void_p), ("d_qn", ctypes.c_void_p), ("d_qref", ctypes.c_void_p),
                ("d_out", ctypes.c_void_p), ("d_Q", ctypes.c_void_p * HEVI_MAX_STAGES),
                ("d_S", ctypes.c_void_p * HEVI_MAX_STAGES)]


class GroupPlan(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("grid", ctypes.c_int32), ("use_graph", ctypes.c_int32)]

    def as_dict(self):
        mode = {v: k for k, v in LAUNCH_MODES.items()}.get(self.mode, self.mode)
        return {"mode": mode, "grid": self.grid, "use_graph": bool(self.use_graph)}


class TuneResult(ctypes.Structure):
    _fields_ = [("plan", GroupPlan), ("ms_per_step", ctypes.c_double)]


_vp = ctypes.c_void_p
_lib = None


def load():
    """Load libhevi.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; load it first so that libhevi.so binds to
    # the same runtime instance (one address space for device pointers)
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2311_11425_amd/build.py "
                           "(no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pp = ctypes.POINTER(_vp)
    pd = ctypes.POINTER(dbl)
    sig = {
        "hevi_create": ([ctypes.c_int, pp], ctypes.c_int),
        "hevi_destroy": ([_vp], None),
        "hevi_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "hevi_build_column_ops": ([_vp, ctypes.POINTER(Shape), ctypes.POINTER(Consts), _vp, _vp, _vp,
                                   _vp, _vp, pp, _vp], ctypes.c_int),
        "hevi_build_column_ops_set": ([_vp, ctypes.POINTER(Shape), ctypes.POINTER(Consts),
                                       ctypes.c_int, _vp, _vp, _vp, _vp, _vp, pp, _vp],
                                      ctypes.c_int),
        "hevi_build_column_ops_ps": ([_vp, ctypes.POINTER(Shape), ctypes.POINTER(Consts), _vp,
                                      _vp, _vp, _vp, _vp, _vp, pp, _vp], ctypes.c_int),
        "hevi_ops_relinearize": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "hevi_vertical_op": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "hevi_newton_increment": ([_vp, _vp, _vp, _vp, _vp, pd, _vp], ctypes.c_int),
        "hevi_ops_check": ([_vp, _vp, ctypes.POINTER(i64), _vp], ctypes.c_int),
        "hevi_ops_free": ([_vp], None),
        "hevi_apply_op": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "hevi_factor": ([_vp, _vp, dbl, ctypes.c_int, pp, _vp], ctypes.c_int),
        "hevi_refactor": ([_vp, _vp, dbl, _vp], ctypes.c_int),
        "hevi_factors_check": ([_vp, _vp, ctypes.POINTER(Info), _vp], ctypes.c_int),
        "hevi_factors_band_entries": ([_vp, _vp, ctypes.POINTER(ctypes.c_int64), _vp],
                                      ctypes.c_int),
        "hevi_factors_free": ([_vp], None),
        "hevi_stage_solve": ([_vp, _vp, i32, pp, pd, i32, pp, pd, _vp, ctypes.POINTER(Refine),
                              ctypes.POINTER(Info), _vp], ctypes.c_int),
        "hevi_solve_noalloc": ([_vp, _vp, dbl, ctypes.c_int, i32, pp, pd, i32, pp, pd, _vp,
                                ctypes.POINTER(Refine), ctypes.POINTER(Info), _vp], ctypes.c_int),
        "hevi_combine": ([_vp, _vp, i32, pp, pd, _vp, _vp], ctypes.c_int),
        "hevi_tableau": ([ctypes.c_char_p, ctypes.POINTER(i32), pd, pd, pd], ctypes.c_int),
        "hevi_sizes": ([ctypes.POINTER(Shape), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t),
                        ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                        ctypes.POINTER(ctypes.c_size_t)],
                       ctypes.c_int),
        "hevi_group_create": ([_vp, i32, ctypes.POINTER(GroupMember), ctypes.c_char_p, dbl,
                               ctypes.c_int, ctypes.POINTER(Refine), pp, _vp], ctypes.c_int),
        "hevi_group_set_plan": ([_vp, _vp, ctypes.POINTER(GroupPlan)], ctypes.c_int),
        "hevi_group_get_plan": ([_vp, ctypes.POINTER(GroupPlan)], ctypes.c_int),
        "hevi_group_step": ([_vp, _vp, i32, _vp], ctypes.c_int),
        "hevi_group_check": ([_vp, _vp, ctypes.POINTER(Info), _vp], ctypes.c_int),
        "hevi_group_autotune": ([_vp, _vp, i32, ctypes.POINTER(TuneResult), i32,
                                 ctypes.POINTER(i32), _vp], ctypes.c_int),
        "hevi_group_free": ([_vp], None),
        "hevi_serve_create": ([_vp, ctypes.c_size_t, i32, _vp, pp], ctypes.c_int),
        "hevi_serve_register": ([_vp, _vp, dbl, ctypes.c_int, ctypes.POINTER(i32)], ctypes.c_int),
        "hevi_serve_submit": ([_vp, i32, i32, pp, pd, i32, pp, pd, _vp,
                               ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "hevi_serve_poll": ([_vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(Info), pd],
                            ctypes.c_int),
        "hevi_serve_wait": ([_vp, ctypes.c_uint64, ctypes.POINTER(Info), pd], ctypes.c_int),
        "hevi_serve_release": ([_vp, i32], ctypes.c_int),
        "hevi_serve_destroy": ([_vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(code, what):
    if code != 0:
        raise HeviError(code, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr_array(ts):
    arr = (_vp * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def _dbl_array(vals):
    arr = (ctypes.c_double * max(1, len(vals)))()
    for i, v in enumerate(vals):
        arr[i] = float(v)
    return arr


def tableau(name):
    lib = load()
    s = ctypes.c_int32(0)
    a = (ctypes.c_double * 64)()
    ai = (ctypes.c_double * 64)()
    b = (ctypes.c_double * 8)()
    _check(lib.hevi_tableau(name.encode(), ctypes.byref(s), a, ai, b), f"tableau {name}")
    n = s.value
    return {"name": name, "s": n,
            "Aexp": [[a[i * n + j] for j in range(n)] for i in range(n)],
            "Aimp": [[ai[i * n + j] for j in range(n)] for i in range(n)],
            "b": [b[i] for i in range(n)]}


def sizes(N, Ne, ncols=1, precision=HEVI_FP64):
    lib = load()
    sh = Shape(N, Ne, ncols)
    o, f, p, r = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.hevi_sizes(ctypes.byref(sh), precision, ctypes.byref(o), ctypes.byref(f),
                          ctypes.byref(p), ctypes.byref(r)), "sizes")
    return {"ops": o.value, "factors": f.value, "paper_band": p.value, "resident": r.value}


class Ops:
    def __init__(self, ctx, handle, shape, keep):
        self.ctx, self.handle, self.shape, self._keep = ctx, handle, shape, keep

    def check(self, stream=None):
        bad = ctypes.c_int64(-1)
        code = load().hevi_ops_check(self.ctx.handle, self.handle, ctypes.byref(bad), _stream(stream))
        return code, bad.value

    def free(self):
        if self.handle:
            load().hevi_ops_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Factors:
    def __init__(self, ctx, handle, ops, precision, lam):
        self.ctx, self.handle, self.ops, self.precision, self.lam = ctx, handle, ops, precision, lam

    def check(self, stream=None):
        inf = Info()
        code = load().hevi_factors_check(self.ctx.handle, self.handle, ctypes.byref(inf),
                                         _stream(stream))
        return code, inf.as_dict()

    def band_entries(self, stream=None):
        """U entries the solves read (each row up to its last nonzero), summed over
        the columns (see hevi_factors_band_entries)."""
        u = ctypes.c_int64(0)
        _check(load().hevi_factors_band_entries(self.ctx.handle, self.handle, ctypes.byref(u),
                                                _stream(stream)), "hevi_factors_band_entries")
        return u.value

    def free(self):
        if self.handle:
            load().hevi_factors_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """One library context on one HIP device."""

    def __init__(self, device=0):
        self.lib = load()
        h = ctypes.c_void_p()
        _check(self.lib.hevi_create(device, ctypes.byref(h)), "hevi_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self.lib.hevi_destroy(self.handle)
            self.handle = None

    def build_column_ops(self, N, Ne, ncols, consts, z, J, gz, rho0, Theta0, stream=None,
                         eqset="2C"):
        """Column operator of set ``eqset``: "2C" (Theta0 is rho0 theta0) or "3C"
        (the argument is the reference total energy E0)."""
        sh = Shape(N, Ne, ncols)
        k = Consts(*consts)
        out = ctypes.c_void_p()
        if eqset == "2C":
            _check(self.lib.hevi_build_column_ops(self.handle, ctypes.byref(sh), ctypes.byref(k),
                                                  _ptr(z), _ptr(J), _ptr(gz), _ptr(rho0),
                                                  _ptr(Theta0), ctypes.byref(out),
                                                  _stream(stream)),
                   "hevi_build_column_ops")
        else:
            _check(self.lib.hevi_build_column_ops_set(self.handle, ctypes.byref(sh),
                                                      ctypes.byref(k), EQSETS[eqset], _ptr(z),
                                                      _ptr(J), _ptr(gz), _ptr(rho0),
                                                      _ptr(Theta0), ctypes.byref(out),
                                                      _stream(stream)),
                   "hevi_build_column_ops_set")
        return Ops(self, out, (N, Ne, ncols), None)

    def build_column_ops_ps(self, N, Ne, ncols, consts, z, J, gz, rho0, U0, Theta0,
                            stream=None):
        """LHEVI-PS operator: the Jacobian at the moving state (rho0, U0, Theta0)."""
        sh = Shape(N, Ne, ncols)
        k = Consts(*consts)
        out = ctypes.c_void_p()
        _check(self.lib.hevi_build_column_ops_ps(self.handle, ctypes.byref(sh), ctypes.byref(k),
                                                 _ptr(z), _ptr(J), _ptr(gz), _ptr(rho0),
                                                 _ptr(U0), _ptr(Theta0), ctypes.byref(out),
                                                 _stream(stream)),
               "hevi_build_column_ops_ps")
        return Ops(self, out, (N, Ne, ncols), None)

    def relinearize(self, ops, rho0, U0, Theta0, stream=None):
        _check(self.lib.hevi_ops_relinearize(self.handle, ops.handle, _ptr(rho0), _ptr(U0),
                                             _ptr(Theta0), _stream(stream)),
               "hevi_ops_relinearize")

    def vertical_op(self, ops, q, V, stream=None):
        _check(self.lib.hevi_vertical_op(self.handle, ops.handle, _ptr(q), _ptr(V),
                                         _stream(stream)), "hevi_vertical_op")

    def newton_increment(self, ops, dq, q, qn, stream=None):
        r = ctypes.c_double(0.0)
        _check(self.lib.hevi_newton_increment(self.handle, ops.handle, _ptr(dq), _ptr(q),
                                              _ptr(qn), ctypes.byref(r), _stream(stream)),
               "hevi_newton_increment")
        return r.value

    def apply_op(self, ops, x, y, xref=None, stream=None):
        _check(self.lib.hevi_apply_op(self.handle, ops.handle, _ptr(x), _ptr(xref), _ptr(y),
                                      _stream(stream)), "hevi_apply_op")

    def factor(self, ops, lam, precision=HEVI_FP64, stream=None):
        out = ctypes.c_void_p()
        _check(self.lib.hevi_factor(self.handle, ops.handle, float(lam), precision,
                                    ctypes.byref(out), _stream(stream)), "hevi_factor")
        return Factors(self, out, ops, precision, lam)

    def refactor(self, f, lam, stream=None):
        _check(self.lib.hevi_refactor(self.handle, f.handle, float(lam), _stream(stream)),
               "hevi_refactor")
        f.lam = lam

    def stage_solve(self, f, E, e, Qprev, c, Qi, refine=None, info=False, stream=None):
        """Qi <- one LHEVI stage (see include/hevi.h); returns the info dict if requested.

        refine = (max_sweeps, rel_residual_target[, full_sweeps])."""
        Ep, ep = _ptr_array(E), _dbl_array(e)
        Qp, cp = _ptr_array(Qprev), _dbl_array(c)
        ref = None
        if refine is not None:
            r = tuple(refine) + (0,) * (3 - len(refine))
            ref = Refine(int(r[0]), float(r[1]), int(r[2]))
        inf = Info() if info else None
        _check(self.lib.hevi_stage_solve(self.handle, f.handle, len(E), Ep, ep, len(Qprev), Qp, cp,
                                         _ptr(Qi), ctypes.byref(ref) if ref else None,
                                         ctypes.byref(inf) if inf else None, _stream(stream)),
               "hevi_stage_solve")
        return inf.as_dict() if inf else None

    def solve_noalloc(self, ops, lam, precision, E, e, Qprev, c, Qi, refine=None, info=False,
                      stream=None):
        """hevi_solve_noalloc: factor A = I - lam L_z and one stage solve, with the
        library's fixed per-GPU scratch (no allocation); arguments as stage_solve."""
        Ep, ep = _ptr_array(E), _dbl_array(e)
        Qp, cp = _ptr_array(Qprev), _dbl_array(c)
        ref = None
        if refine is not None:
            r = tuple(refine) + (0,) * (3 - len(refine))
            ref = Refine(int(r[0]), float(r[1]), int(r[2]))
        inf = Info() if info else None
        _check(self.lib.hevi_solve_noalloc(self.handle, ops.handle, ctypes.c_double(lam),
                                           int(precision), len(E), Ep, ep, len(Qprev), Qp, cp,
                                           _ptr(Qi), ctypes.byref(ref) if ref else None,
                                           ctypes.byref(inf) if inf else None, _stream(stream)),
               "hevi_solve_noalloc")
        return inf.as_dict() if inf else None

    def combine(self, ops, V, coef, out, stream=None):
        _check(self.lib.hevi_combine(self.handle, ops.handle, len(V), _ptr_array(V), _dbl_array(coef),
                                     _ptr(out), _stream(stream)), "hevi_combine")


class Group:
    """Members advanced together by hevi_group_step (see include/hevi.h).

    members: list of dicts with keys ops (Ops), qn, qref, out, Q (list of s
    tensors; Q[0] is ignored), S (list of s tensors)."""

    def __init__(self, ctx, members, tableau="ARK3", dt=300.0, precision=HEVI_FP64, refine=None,
                 stream=None):
        self.ctx = ctx
        self.lib = load()
        self.members = members  # keep tensors alive
        n = len(members)
        arr = (GroupMember * max(1, n))()
        for i, m in enumerate(members):
            gm = arr[i]
            gm.ops = m["ops"].handle.value if isinstance(m["ops"].handle, ctypes.c_void_p) else m["ops"].handle
            gm.d_qn = m["qn"].data_ptr()
            gm.d_qref = m["qref"].data_ptr()
            gm.d_out = m["out"].data_ptr()
            for j, t in enumerate(m["Q"]):
                if t is not None:
                    gm.d_Q[j] = t.data_ptr()
            for j, t in enumerate(m["S"]):
                gm.d_S[j] = t.data_ptr()
        ref = None
        if refine is not None:
            r = tuple(refine) + (0,) * (3 - len(refine))
            ref = Refine(int(r[0]), float(r[1]), int(r[2]))
        h = ctypes.c_void_p()
        _check(self.lib.hevi_group_create(ctx.handle, n, arr, tableau.encode(), float(dt), precision,
                                          ctypes.byref(ref) if ref else None, ctypes.byref(h),
                                          _stream(stream)), "hevi_group_create")
        self.handle = h
        self.n = n

    def set_plan(self, mode="one", grid=0, use_graph=False):
        p = GroupPlan(LAUNCH_MODES[mode] if isinstance(mode, str) else int(mode), int(grid),
                      int(bool(use_graph)))
        _check(self.lib.hevi_group_set_plan(self.ctx.handle, self.handle, ctypes.byref(p)),
               "hevi_group_set_plan")

    def plan(self):
        p = GroupPlan()
        _check(self.lib.hevi_group_get_plan(self.handle, ctypes.byref(p)), "hevi_group_get_plan")
        return p.as_dict()

    def step(self, refactor=True, stream=None):
        _check(self.lib.hevi_group_step(self.ctx.handle, self.handle, int(bool(refactor)),
                                        _stream(stream)), "hevi_group_step")

    def check(self, stream=None):
        infos = (Info * max(1, self.n))()
        code = self.lib.hevi_group_check(self.ctx.handle, self.handle, infos, _stream(stream))
        if code == 4:
            raise HeviError(code, "hevi_group_check")
        return code, [infos[i].as_dict() for i in range(self.n)]

    def autotune(self, reps=3, stream=None):
        cap = 64
        res = (TuneResult * cap)()
        nr = ctypes.c_int32(0)
        _check(self.lib.hevi_group_autotune(self.ctx.handle, self.handle, int(reps), res, cap,
                                            ctypes.byref(nr), _stream(stream)),
               "hevi_group_autotune")
        return [dict(res[i].plan.as_dict(), ms_per_step=res[i].ms_per_step)
                for i in range(min(cap, nr.value))]

    def free(self):
        if self.handle:
            self.lib.hevi_group_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching stage-solve server (hevi_serve_*, see include/hevi.h).
    Calls are thread-safe; ctypes releases the GIL while the library waits."""

    def __init__(self, ctx, hbm_budget_bytes, max_inflight=1024, refine=None):
        """refine: (max_sweeps, rel_target) of the FP32-factor simulations (None:
        the library default)."""
        self.ctx = ctx
        self.lib = load()
        h = ctypes.c_void_p()
        ref = None if refine is None else Refine(*(tuple(refine) + (0,) * (3 - len(refine))))
        _check(self.lib.hevi_serve_create(ctx.handle, int(hbm_budget_bytes), int(max_inflight),
                                          ctypes.byref(ref) if ref is not None else None,
                                          ctypes.byref(h)), "hevi_serve_create")
        self.handle = h

    def register(self, ops, lam, precision=HEVI_FP64):
        """Simulation id, or raises HeviError (code 3 = not admitted within the budget)."""
        sid = ctypes.c_int32(-1)
        _check(self.lib.hevi_serve_register(self.handle, ops.handle, float(lam), precision,
                                            ctypes.byref(sid)), "hevi_serve_register")
        return sid.value

    def submit_raw(self, sim, Ep, ep, ne, Qp, cp, nq, Qi_ptr):
        """Submit with prepared ctypes arrays (no per-call marshalling); returns
        (status, ticket)."""
        t = ctypes.c_uint64(0)
        code = self.lib.hevi_serve_submit(self.handle, sim, ne, Ep, ep, nq, Qp, cp, Qi_ptr,
                                          ctypes.byref(t))
        return code, t.value

    def submit(self, sim, E, e, Qprev, c, Qi):
        code, t = self.submit_raw(sim, _ptr_array(E), _dbl_array(e), len(E), _ptr_array(Qprev),
                                  _dbl_array(c), len(Qprev), _ptr(Qi))
        _check(code, "hevi_serve_submit")
        return t

    def poll(self, ticket):
        done = ctypes.c_int32(0)
        inf = Info()
        lat = ctypes.c_double(0.0)
        _check(self.lib.hevi_serve_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(inf),
                                        ctypes.byref(lat)), "hevi_serve_poll")
        return (inf.as_dict(), lat.value) if done.value else None

    def wait(self, ticket):
        inf = Info()
        lat = ctypes.c_double(0.0)
        _check(self.lib.hevi_serve_wait(self.handle, ticket, ctypes.byref(inf), ctypes.byref(lat)),
               "hevi_serve_wait")
        return inf.as_dict(), lat.value

    def release(self, sim):
        _check(self.lib.hevi_serve_release(self.handle, int(sim)), "hevi_serve_release")

    def close(self):
        if self.handle:
            self.lib.hevi_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
