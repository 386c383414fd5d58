"""The continuous-batching server (hevi_serve_*) through the C ABI.

* A request's result is bit-identical to hevi_stage_solve of the same operands,
  whether it runs alone or batched with requests of other simulations, and it
  matches the FP64 oracle.
* A whole six-stage ARK4 step driven request by request through the server
  gives the single-problem step's bits.
* Admission within the HBM budget, backpressure (HEVI_E_BUSY), unknown and
  retired ids (HEVI_E_CLOSED), release, and submits from several threads.
"""
import threading

import numpy as np
import pytest

import oracle
from paper_2311_11425_amd import inputs
from parity_util import relerr_cols, stage_floor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = 300.0
GAMMA = 1767732205903.0 / 4055673282236.0  # ARK3 diagonal
LAM = GAMMA * DT
A21 = 1767732205903.0 / 2027836641118.0    # ARK3 explicit a_21

SPECS = [
    {"N": 4, "Ne": 12, "ncols": 300, "seed": 501, "z_top": 60e3, "profile": "lapse_capped"},
    {"N": 4, "Ne": 20, "ncols": 65, "seed": 502},
    {"N": 3, "Ne": 9, "ncols": 130, "seed": 503},
    {"N": 4, "Ne": 10, "ncols": 1, "seed": 504, "z_top": 120e3, "profile": "lapse_capped"},
]


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_11425_amd import hevi
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = hevi.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


class SimData:
    """One simulation: columns, ops, and the operands of an ARK3 second-stage solve."""

    def __init__(self, ctx, spec):
        from paper_2311_11425_amd.driver import ColumnBatch
        self.col = inputs.spec_columns(spec)
        self.B = ColumnBatch(ctx, self.col)
        qn, qref = inputs.perturbed_state(self.col, seed=spec["seed"] + 3)
        self.qn_h, self.qref_h = qn, qref
        self.qn, self.qref = dev(qn), dev(qref)
        self.S1 = self.B.empty_state()
        ctx.apply_op(self.B.ops, self.qn, self.S1, xref=self.qref)
        self.E, self.e = [self.qn, self.S1], [1.0, DT * A21]
        self.Qp, self.c = [self.qn], [-1.0]

    def out(self):
        return torch.full_like(self.qn, float("nan"))


def reference(ctx, sd, prec):
    f = ctx.factor(sd.B.ops, LAM, prec)
    x = sd.out()
    ctx.stage_solve(f, sd.E, sd.e, sd.Qp, sd.c, x, refine=(4, 1e-13, 0))
    torch.cuda.synchronize()
    f.free()
    return x.cpu()


@pytest.mark.parametrize("prec", [0, 1])
def test_serve_alone_and_mixed_match_stage_solve(ctx, prec):
    from paper_2311_11425_amd import hevi
    sims = [SimData(ctx, sp) for sp in SPECS]
    ref = [reference(ctx, sd, prec) for sd in sims]
    srv = hevi.Server(ctx, 1 << 34, max_inflight=64)
    ids = [srv.register(sd.B.ops, LAM, prec) for sd in sims]
    # alone: one request at a time
    for sd, sid, r in zip(sims, ids, ref):
        x = sd.out()
        inf, lat = srv.wait(srv.submit(sid, sd.E, sd.e, sd.Qp, sd.c, x))
        assert inf["status"] == "HEVI_OK", inf
        assert lat > 0
        torch.cuda.synchronize()
        assert torch.equal(x.cpu(), r)
    # mixed: every simulation twice, submitted together (separate outputs)
    outs = [[sd.out(), sd.out()] for sd in sims]
    tickets = [srv.submit(sid, sd.E, sd.e, sd.Qp, sd.c, o)
               for rep in range(2) for sd, sid, o in zip(sims, ids, [oo[rep] for oo in outs])]
    for t in tickets:
        inf, _ = srv.wait(t)
        assert inf["status"] == "HEVI_OK", inf
    torch.cuda.synchronize()
    for oo, r in zip(outs, ref):
        for o in oo:
            assert torch.equal(o.cpu(), r)
    # the oracle on every simulation: q^ = q^E - Q_1 with Q_1 = q^n, q_tt = Q_2 + Q_1
    for sd, r in zip(sims, ref):
        qE = sd.qn_h + DT * A21 * sd.S1.cpu().numpy()
        P = -sd.qn_h
        x_or = oracle.solve_batch(sd.col, LAM, qE + P, refine=1)
        err = relerr_cols(r.numpy() + P, x_or)
        tol = max(1e-12 if prec == 0 else 1e-10,
                  4 * stage_floor(oracle, sd.col, LAM, qE, P, r.numpy(), x_or))
        print(f"N={sd.col['N']} Ne={sd.col['Ne']}: {err:.2e} (tol {tol:.2e})", flush=True)
        assert err < tol
    for sid in ids:
        srv.release(sid)
    srv.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_serve_ark4_step_matches_stepper(ctx, prec):
    """A whole ARK4 step (six stages, so up to five previous stages per request)
    driven through the server for two simulations whose requests share launches:
    every Q_i, S_i and q^{n+1} carries the same bits as the single-problem step."""
    from paper_2311_11425_amd import hevi
    from paper_2311_11425_amd.driver import ArkStepper
    dt = 30.0
    sims = [SimData(ctx, sp) for sp in (SPECS[0], SPECS[2])]
    steps, refs = [], []
    for sd in sims:
        st = ArkStepper(ctx, sd.B, "ARK4", dt, precision=prec, refine=(4, 1e-13, 0))
        out = sd.B.empty_state()
        for inf in st.step(sd.qn, sd.qref, out, info=True):
            assert inf["status"] == "HEVI_OK", inf
        torch.cuda.synchronize()
        steps.append(st)
        refs.append(([t.cpu() for t in st.Q[1:]], [t.cpu() for t in st.S], out.cpu()))
    srv = hevi.Server(ctx, 1 << 34, max_inflight=16)
    ids = [srv.register(sd.B.ops, st.lam, prec) for sd, st in zip(sims, steps)]
    Q = [[sd.qn] + [sd.out() for _ in range(1, st.s)] for sd, st in zip(sims, steps)]
    S = [[sd.B.empty_state() for _ in range(st.s)] for sd, st in zip(sims, steps)]
    for sd, S_ in zip(sims, S):
        ctx.apply_op(sd.B.ops, sd.qn, S_[0], xref=sd.qref)
    s = steps[0].s
    assert s == 6
    for i in range(1, s):
        tickets = []
        for k, (sd, st, sid) in enumerate(zip(sims, steps, ids)):
            e = [1.0] + [dt * st.Aexp[i][j] for j in range(i)]
            tickets.append(srv.submit(sid, [sd.qn] + S[k][:i], e, Q[k][:i], st.coeffs(i),
                                      Q[k][i]))
        for t in tickets:
            inf, _ = srv.wait(t)
            assert inf["status"] == "HEVI_OK", inf
        for k, sd in enumerate(sims):
            ctx.apply_op(sd.B.ops, Q[k][i], S[k][i], xref=sd.qref)
    for k, (sd, st) in enumerate(zip(sims, steps)):
        out = sd.out()
        ctx.combine(sd.B.ops, [sd.qn] + S[k], [1.0] + [dt * bi for bi in st.b], out)
        torch.cuda.synchronize()
        rQ, rS, rout = refs[k]
        for i in range(1, s):
            assert torch.equal(Q[k][i].cpu(), rQ[i - 1]), (k, "Q", i)
        for i in range(s):
            assert torch.equal(S[k][i].cpu(), rS[i]), (k, "S", i)
        assert torch.equal(out.cpu(), rout), (k, "out")
    for sid in ids:
        srv.release(sid)
    srv.close()


def resident_bytes(spec, prec):
    """What the server charges for a simulation: hevi_sizes' resident bytes per
    column over the 64-column tiles it allocates."""
    from paper_2311_11425_amd import hevi
    per_col = hevi.sizes(spec["N"], spec["Ne"], spec["ncols"], precision=prec)["resident"]
    return per_col * 64 * ((spec["ncols"] + 63) // 64)


def test_serve_admission_busy_closed(ctx):
    from paper_2311_11425_amd import hevi
    a, b = SimData(ctx, SPECS[0]), SimData(ctx, SPECS[1])
    for bad in ((4, 1e-13, 1), (-1, 1e-13), (65, 1e-13), (4, -1.0)):
        with pytest.raises(hevi.HeviError) as e:
            hevi.Server(ctx, 1 << 20, refine=bad)
        assert e.value.code == 1
    srv = hevi.Server(ctx, 1, max_inflight=2)  # a 1-byte budget admits nothing
    with pytest.raises(hevi.HeviError) as e:
        srv.register(a.B.ops, LAM)
    assert e.value.code == 3
    srv.close()
    # a budget one byte short of both simulations: a fits, b is refused until a is
    # released, then admitted
    ra, rb = resident_bytes(SPECS[0], 0), resident_bytes(SPECS[1], 0)
    srv = hevi.Server(ctx, ra + rb - 1, max_inflight=2)
    sa = srv.register(a.B.ops, LAM)
    with pytest.raises(hevi.HeviError) as e:
        srv.register(b.B.ops, LAM)
    assert e.value.code == 3
    # backpressure: a burst beyond max_inflight sees HEVI_E_BUSY
    outs = [a.out() for _ in range(40)]
    tickets, busy = [], 0
    for o in outs:
        try:
            tickets.append(srv.submit(sa, a.E, a.e, a.Qp, a.c, o))
        except hevi.HeviError as err:
            assert err.code == 7
            busy += 1
    for t in tickets:
        srv.wait(t)
    assert busy > 0 and len(tickets) >= 2
    # retired and unknown tickets / ids
    with pytest.raises(hevi.HeviError) as e:
        srv.wait(tickets[0])
    assert e.value.code == 8
    with pytest.raises(hevi.HeviError) as e:
        srv.submit(12345, a.E, a.e, a.Qp, a.c, outs[0])
    assert e.value.code == 8
    # a request still queued when its simulation is released completes first and
    # its ticket can be waited for afterwards
    t_last = srv.submit(sa, a.E, a.e, a.Qp, a.c, outs[0])
    srv.release(sa)
    inf, _ = srv.wait(t_last)
    assert inf["status"] == "HEVI_OK"
    with pytest.raises(hevi.HeviError) as e:
        srv.submit(sa, a.E, a.e, a.Qp, a.c, outs[0])
    assert e.value.code == 8
    sb = srv.register(b.B.ops, LAM)  # fits after the release
    srv.release(sb)
    srv.close()
    # exactly both fit
    srv = hevi.Server(ctx, ra + rb, max_inflight=2)
    ids = [srv.register(a.B.ops, LAM), srv.register(b.B.ops, LAM)]
    for sid in ids:
        srv.release(sid)
    srv.close()



def test_serve_threads(ctx):
    """Four host threads submit and wait concurrently; every result is the reference."""
    from paper_2311_11425_amd import hevi
    sims = [SimData(ctx, sp) for sp in SPECS[:3]]
    ref = [reference(ctx, sd, 0) for sd in sims]
    srv = hevi.Server(ctx, 1 << 34, max_inflight=256)
    ids = [srv.register(sd.B.ops, LAM) for sd in sims]
    errors = []

    def client(k):
        try:
            for rep in range(6):
                j = (k + rep) % len(sims)
                o = sims[j].out()
                t = srv.submit(ids[j], sims[j].E, sims[j].e, sims[j].Qp, sims[j].c, o)
                inf, _ = srv.wait(t)
                assert inf["status"] == "HEVI_OK"
                torch.cuda.synchronize()
                assert torch.equal(o.cpu(), ref[j])
        except Exception as ex:  # reported in the main thread
            errors.append(repr(ex))

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    srv.close()
