"""Groups of uneven column batches advanced by one persistent launch per phase
(hevi_group_*), through the C ABI.

* Every launch plan (one launch over all orders, one per order, one per member;
  persistent grids smaller than the item count; HIP graph replays) gives the
  same bits as the single-problem path (the same per-tile code).
* The stage solves of every member match the FP64 oracle (bars as in
  test_gpu_parity: 1e-10 for FP32 factors + refinement, the FP64 bar for FP64).
* The autotuner times every candidate and keeps the fastest.
"""
import numpy as np
import pytest

import oracle
from paper_2311_11425_amd import inputs
from parity_util import relerr_cols, stage_floor

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# small uneven batch: orders 2..7, ragged tile tails, one single-column member,
# one empty member
SPECS = [
    {"N": 7, "Ne": 9, "ncols": 70, "seed": 401},
    {"N": 3, "Ne": 16, "ncols": 257, "seed": 402},
    {"N": 5, "Ne": 8, "ncols": 130, "seed": 403},
    {"N": 4, "Ne": 12, "ncols": 64, "seed": 404},
    {"N": 3, "Ne": 11, "ncols": 1, "seed": 405},
    {"N": 6, "Ne": 10, "ncols": 100, "seed": 406},
    {"N": 4, "Ne": 9, "ncols": 0, "seed": 407},
    {"N": 2, "Ne": 14, "ncols": 129, "seed": 408},
]
TAB, DT = "ARK3", 300.0


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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make_members(ctx, specs, s):
    from paper_2311_11425_amd.driver import ColumnBatch
    members, cols = [], []
    for sp in specs:
        col = inputs.spec_columns(sp)
        if sp["ncols"] > 0:
            qn, qref = inputs.perturbed_state(col, seed=sp["seed"] + 7)
        else:
            qn = qref = np.zeros((5, col["nz"], 0))
        B = ColumnBatch(ctx, col)
        m = {"batch": B, "ops": B.ops, "qn": dev(qn), "qref": dev(qref), "out": B.empty_state(),
             "Q": [None] + [B.empty_state() for _ in range(1, s)],
             "S": [B.empty_state() for _ in range(s)], "col": col, "qn_h": qn, "qref_h": qref}
        members.append(m)
        cols.append(col)
    return members


def snapshot(members):
    torch.cuda.synchronize()
    return [[m["out"].cpu()] + [t.cpu() for t in m["Q"][1:]] + [t.cpu() for t in m["S"]]
            for m in members]


def single_path(ctx, members, prec, refine, tab=TAB, dt=DT):
    """Reference: the single-problem kernels through ArkStepper, member by member."""
    from paper_2311_11425_amd.driver import ArkStepper
    ref = []
    for m in members:
        st = ArkStepper(ctx, m["batch"], tab, dt, precision=prec, refine=refine)
        out = m["batch"].empty_state()
        st.step(m["qn"], m["qref"], out)
        torch.cuda.synchronize()
        ref.append([out.cpu()] + [t.cpu() for t in st.Q[1:]] + [t.cpu() for t in st.S])
    return ref


def assert_same(a, b, what):
    for p, (xa, xb) in enumerate(zip(a, b)):
        for k, (ta, tb) in enumerate(zip(xa, xb)):
            assert torch.equal(ta, tb), (what, p, k, float((ta - tb).abs().max()))


PLANS = [("one", 0, False), ("one", 3, False), ("per_order", 0, False), ("per_order", 2, False),
         ("per_member", 0, False), ("one", 5, True), ("per_order", 0, True),
         ("per_member", 0, True)]


@pytest.mark.parametrize("prec", [0, 1])
def test_group_plans_match_single_path(ctx, prec):
    from paper_2311_11425_amd import hevi
    refine = (4, 1e-13, 0)
    members = make_members(ctx, SPECS, 4)
    ref = single_path(ctx, members, prec, refine)
    g = hevi.Group(ctx, members, TAB, DT, precision=prec, refine=refine)
    for mode, grid, graph in PLANS:
        print(f"plan {mode} grid={grid} graph={graph} prec={prec}", flush=True)
        g.set_plan(mode, grid, graph)
        for rep in range(3 if graph else 1):  # graph replays with eager work between them
            for m in members:
                m["out"].fill_(np.nan)
                for t in m["Q"][1:] + m["S"]:
                    t.fill_(np.nan)
            g.step(refactor=True)
            assert_same(snapshot(members), ref, (mode, grid, graph, rep))
        code, infos = g.check()
        assert code == 0, infos
    g.free()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tab", ["ARS343", "ARK4"])
def test_group_other_tableaux_match_single_path(ctx, tab, prec):
    """Other tableaux through the group: ARS(3,4,3) (an explicit first stage and a
    zero first implicit column) and the six-stage ARK4 (five previous stages per
    solve).  The same bits as the single-problem path."""
    from paper_2311_11425_amd import hevi
    refine = (4, 1e-13, 0)
    members = make_members(ctx, SPECS, hevi.tableau(tab)["s"])
    ref = single_path(ctx, members, prec, refine, tab=tab, dt=30.0)
    g = hevi.Group(ctx, members, tab, 30.0, precision=prec, refine=refine)
    for mode, grid, graph in (("one", 0, False), ("per_order", 2, True)):
        g.set_plan(mode, grid, graph)
        g.step(refactor=True)
        assert_same(snapshot(members), ref, (tab, mode, grid, graph))
    code, infos = g.check()
    assert code == 0, infos
    g.free()


@pytest.mark.parametrize("prec", [0, 1])
def test_group_stagewise_oracle(ctx, prec):
    """Each member's stage solves against the oracle (q^ rebuilt from the GPU's Q_j, S_j)."""
    from paper_2311_11425_amd import hevi
    tab = hevi.tableau(TAB)
    s, Ae, Ai = tab["s"], tab["Aexp"], tab["Aimp"]
    lam = Ai[1][1] * DT
    members = make_members(ctx, SPECS, s)
    g = hevi.Group(ctx, members, TAB, DT, precision=prec, refine=(4, 1e-13, 0))
    g.set_plan("one", 0, False)
    g.step(refactor=True)
    code, infos = g.check()
    assert code == 0, infos
    bar = 1e-12 if prec == 0 else 1e-10
    for p, m in enumerate(members):
        if m["col"]["ncols"] == 0:
            continue
        col, qn, qref = m["col"], m["qn_h"], m["qref_h"]
        Q = [qn] + [host(t) for t in m["Q"][1:]]
        S = [host(t) for t in m["S"]]
        for i in range(1, s):
            c = [(Ai[i][j] - Ae[i][j]) / Ai[i][i] for j in range(i)]
            qE = qn + sum(DT * Ae[i][j] * S[j] for j in range(i))
            P = sum(c[j] * Q[j] for j in range(i))
            x_or = oracle.solve_batch(col, lam, qE + P, refine=1)
            err = relerr_cols(Q[i] + P, x_or)
            tol = max(bar, 4 * stage_floor(oracle, col, lam, qE, P, Q[i], x_or))
            print(f"member {p} N={col['N']} stage {i + 1}: {err:.2e} (tol {tol:.2e})", flush=True)
            assert err < tol, (p, i, err, tol)
            assert relerr_cols(S[i], oracle.apply_batch(col, Q[i], qref)) < 1e-12
        # end of step: a sum of s + 1 terms, so within a few ulp of the sum of magnitudes
        out = host(m["out"])
        terms = [qn] + [DT * tab["b"][i] * S[i] for i in range(s)]
        expect = sum(terms)
        bound = 8 * np.finfo(np.float64).eps * sum(np.abs(t) for t in terms)
        assert np.all(np.abs(out - expect) <= bound), float(np.max(np.abs(out - expect) / bound))
    g.free()


def test_group_autotune(ctx):
    from paper_2311_11425_amd import hevi
    members = make_members(ctx, SPECS[:4], 4)
    g = hevi.Group(ctx, members, TAB, DT, precision=1)
    res = g.autotune(reps=2)
    assert len(res) >= 10
    best = min(res, key=lambda r: r["ms_per_step"])
    plan = g.plan()
    assert (plan["mode"], plan["grid"], plan["use_graph"]) == (best["mode"], best["grid"],
                                                               best["use_graph"])
    assert all(np.isfinite(r["ms_per_step"]) and r["ms_per_step"] > 0 for r in res)
    g.free()


def test_group_rejects_bad_members(ctx):
    from paper_2311_11425_amd import hevi
    members = make_members(ctx, SPECS[:2], 4)
    bad = dict(members[0])
    bad["S"] = list(bad["S"])
    bad["S"][1] = bad["S"][0]  # two outputs alias
    with pytest.raises(hevi.HeviError):
        hevi.Group(ctx, [bad, members[1]], TAB, DT)
    with pytest.raises(hevi.HeviError):
        hevi.Group(ctx, members, TAB, DT, refine=(4, 1e-13, 1))  # full sweeps not in groups
    with pytest.raises(hevi.HeviError):
        hevi.Group(ctx, members, "ARK9", DT)
