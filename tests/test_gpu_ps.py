"""Parity of the LHEVI-PS path (Sec. 4.3.1: the operator linearised at a moving
state, the whole 5 n_z band factored with partial pivoting) with the oracle.

Bars as for the reference-state path: the FP64 solve <= 1e-12 relative L2 per column
and variable against the oracle with one long-double refinement step (or 4 x the
rounding floor of the stage recipe, stage_floor, where that is larger); the operator
apply <= 1e-12.
"""
import numpy as np
import pytest

import oracle
from oracle import tableaux
from paper_2311_11425_amd import inputs
from parity_util import relerr_cols, stage_floor, step_tolerance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


W = inputs.with_wind


def cases():
    return {
        "cfg1_hetero": lambda: W(inputs.config1(heterogeneous=True, ncols=130)),
        "cfg2_ragged150": lambda: W(inputs.config2(ncols=150)),
        "N3_tilt_deep": lambda: W(inputs.make_columns(3, 5, 70, profile="lapse", seed=31,
                                                      surface_max=1500.0, tilt=0.2, deep=True)),
        "N5": lambda: W(inputs.make_columns(5, 3, 65, profile="isothermal", seed=32)),
        "N4_Ne1": lambda: W(inputs.make_columns(4, 1, 40, profile="isothermal", seed=39)),
        "N1": lambda: W(inputs.make_columns(1, 6, 40, profile="isothermal", seed=34)),
        "N2_strong_wind": lambda: W(inputs.make_columns(2, 4, 40, profile="lapse", seed=35),
                                    u_h=60.0, w0=3.0),
    }


def lam_for(col):
    return 0.4358665215 * 300.0 if col["Ne"] == 10 else (1 - 1 / np.sqrt(2)) * 30.0


def rhs(col, seed=7):
    qn, qref = inputs.perturbed_state(col, seed=seed)
    b = qn - qref
    rng = np.random.default_rng(seed + 1)
    b[1:4, 0, :] += 0.05 * rng.uniform(-1, 1, b[1:4, 0, :].shape)
    b[1:4, -1, :] += 0.05 * rng.uniform(-1, 1, b[1:4, -1, :].shape)
    return b


@pytest.mark.parametrize("name", list(cases()))
def test_ps_apply_parity(ctx, name):
    from paper_2311_11425_amd.driver import ColumnBatch
    col = cases()[name]()
    print(f"PS apply {name} N={col['N']} Ne={col['Ne']} ncols={col['z'].shape[1]}", flush=True)
    B = ColumnBatch(ctx, col)
    code, bad = B.ops.check()
    assert code == 0 and bad == -1
    qn, qref = inputs.perturbed_state(col, seed=5)
    y = B.empty_state()
    ctx.apply_op(B.ops, dev(qn), y, xref=dev(qref))
    assert relerr_cols(host(y), oracle.apply_batch(col, qn, qref)) < 1e-12


@pytest.mark.parametrize("name", list(cases()))
def test_ps_solve_parity(ctx, name):
    from paper_2311_11425_amd.driver import ColumnBatch
    col = cases()[name]()
    print(f"PS solve {name} ncols={col['z'].shape[1]}", flush=True)
    B = ColumnBatch(ctx, col)
    lam = lam_for(col)
    b = rhs(col)
    f = ctx.factor(B.ops, lam, 0)
    code, inf = f.check()
    assert code == 0, inf
    x = B.empty_state()
    inf = ctx.stage_solve(f, [dev(b)], [1.0], [], [], x, info=True)
    assert inf["status"] == "HEVI_OK", inf
    xo = oracle.solve_batch(col, lam, b, refine=1)
    err = relerr_cols(host(x), xo)
    plain = relerr_cols(oracle.solve_batch(col, lam, b, refine=0), xo)
    print(f"rel err {err:.2e} (the oracle's plain GEPP: {plain:.2e})", flush=True)
    assert err < TOL64, err


@pytest.mark.parametrize("which", ["ARK3_cfg2_sample", "ARK2_cfg1"])
def test_ps_ark_stagewise_parity(ctx, which):
    """Each stage solve of a GPU ARK step with the LHEVI-PS operator (the explicit
    tendency S(q) = L_PS (q - q0) through the same operator), against the oracle from the
    GPU's own stage values."""
    from paper_2311_11425_amd.driver import ArkStepper, ColumnBatch
    if which == "ARK2_cfg1":
        col, tabname, dt = W(inputs.config1(heterogeneous=True, ncols=100)), "ARK2", 30.0
    else:
        col, tabname, dt = W(inputs.config2(ncols=130)), "ARK3", 300.0
    print(f"PS stagewise {which}", flush=True)
    B = ColumnBatch(ctx, col)
    st = ArkStepper(ctx, B, tabname, dt, precision=0)
    qn, qref = inputs.perturbed_state(col)
    out = B.empty_state()
    for inf in st.step(dev(qn), dev(qref), out, info=True):
        assert inf["status"] == "HEVI_OK", inf
    Q = [host(t) for t in st.Q]
    S = [host(t) for t in st.S]
    for i in range(1, st.s):
        c = st.coeffs(i)
        qE = qn + sum(dt * st.Aexp[i][j] * S[j] for j in range(i))
        P = sum(c[j] * Q[j] for j in range(i))
        x_or = oracle.solve_batch(col, st.lam, qE + P, refine=1)
        err = relerr_cols(Q[i] + P, x_or)
        tol = max(TOL64, 4 * stage_floor(oracle, col, st.lam, qE, P, Q[i], x_or))
        print(f"stage {i + 1}: solve rel err {err:.2e} (tolerance {tol:.2e})", flush=True)
        assert err < tol, (i, err, tol)
        assert relerr_cols(S[i], oracle.apply_batch(col, Q[i], qref)) < 1e-12


def test_ps_ark_step_parity(ctx):
    """Two ARK3 steps with the LHEVI-PS operator against the oracle's step."""
    from paper_2311_11425_amd.driver import ArkStepper, ColumnBatch
    col = W(inputs.config2(ncols=130))
    tab, dt = tableaux.as_float(tableaux.ark3()), 300.0
    B = ColumnBatch(ctx, col)
    st = ArkStepper(ctx, B, "ARK3", dt, precision=0)
    qn, qref = inputs.perturbed_state(col)
    q, qr, qo = dev(qn), dev(qref), qn.copy()
    for n in range(2):
        out = B.empty_state()
        for inf in st.step(q, qr, out, info=True):
            assert inf["status"] == "HEVI_OK", inf
        qo_next, Qo, _ = oracle.ark_step_batch(col, tab, dt, qo, qref, refine=1, want_stages=True)
        tol = step_tolerance(oracle, col, tab, dt, qo, qref, Qo, TOL64)
        for i in range(1, st.s):
            assert relerr_cols(host(st.Q[i]) - qo, Qo[i] - qo) < tol
        assert relerr_cols(host(out) - qo, qo_next - qo) < tol
        q, qo = out, qo_next


def test_ps_relinearize_equals_fresh_build(ctx):
    """hevi_ops_relinearize to a new state gives bitwise the operator (apply) and the
    solve of a fresh build at that state."""
    from paper_2311_11425_amd.driver import ColumnBatch
    col1 = W(inputs.config2(ncols=100), u_h=10.0, w0=0.2, seed=1)
    col2 = W(inputs.config2(ncols=100), u_h=30.0, w0=1.0, seed=2)
    B1, B2 = ColumnBatch(ctx, col1), ColumnBatch(ctx, col2)
    ctx.relinearize(B1.ops, B2.rho0, B2.U0, B2.Theta0)
    code, bad = B1.ops.check()
    assert code == 0
    lam = lam_for(col2)
    b = rhs(col2)
    qn, qref = inputs.perturbed_state(col2, seed=5)
    outs = []
    for B in (B1, B2):
        y = B.empty_state()
        ctx.apply_op(B.ops, dev(qn), y, xref=dev(qref))
        f = ctx.factor(B.ops, lam, 0)
        x = B.empty_state()
        ctx.stage_solve(f, [dev(b)], [1.0], [], [], x)
        outs.append((host(y), host(x)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_ps_limits(ctx):
    """FP32 factors, orders above 5, the allocation-free entry point, groups and the
    server are refused for LHEVI-PS operators."""
    from paper_2311_11425_amd import hevi
    from paper_2311_11425_amd.driver import ColumnBatch
    col = W(inputs.config1(ncols=70))
    B = ColumnBatch(ctx, col)
    with pytest.raises(hevi.HeviError) as ei:
        ctx.factor(B.ops, 10.0, hevi.HEVI_FP32_REFINE)
    assert ei.value.code == 1
    with pytest.raises(hevi.HeviError) as ei:
        ColumnBatch(ctx, W(inputs.make_columns(6, 2, 10, seed=3)))
    assert ei.value.code == 2
    b = rhs(col)
    x = B.empty_state()
    with pytest.raises(hevi.HeviError) as ei:
        ctx.solve_noalloc(B.ops, 10.0, 0, [dev(b)], [1.0], [], [], x)
    assert ei.value.code == 1
    srv = hevi.Server(ctx, 1 << 30)
    with pytest.raises(hevi.HeviError) as ei:
        srv.register(B.ops, 10.0)
    assert ei.value.code == 1
    srv.close()


def test_ps_rest_state_matches_reference_path(ctx):
    """With U0 = 0 the LHEVI-PS path (full band) and the reference-state path (reduced
    band) solve the same system: equal to 1e-12."""
    from paper_2311_11425_amd.driver import ColumnBatch
    col = inputs.config2(ncols=90)
    colp = dict(col)
    colp["U0"] = np.zeros((3,) + col["z"].shape)
    Bp, Br = ColumnBatch(ctx, colp), ColumnBatch(ctx, col)
    lam = lam_for(col)
    b = rhs(col)
    xs = []
    for B in (Bp, Br):
        f = ctx.factor(B.ops, lam, 0)
        x = B.empty_state()
        ctx.stage_solve(f, [dev(b)], [1.0], [], [], x)
        xs.append(host(x))
    assert relerr_cols(xs[0], xs[1]) < 1e-12


@pytest.mark.parametrize("N,Ne", [(4, 149), (5, 119)])
def test_ps_tall_columns(ctx, N, Ne):
    """Columns at the largest supported height (n_z <= 600, 2,985 unknowns, 47 blocks of 64
    substitution steps): the band solve's normwise backward error against the oracle's
    dense A is at rounding level, and one more element is refused with HEVI_E_SHAPE."""
    from paper_2311_11425_amd import hevi
    from paper_2311_11425_amd.driver import ColumnBatch
    col = W(inputs.make_columns(N, Ne, 2, profile="lapse", seed=43, surface_max=800.0))
    nz = col["z"].shape[0]
    print(f"PS tall N={N} Ne={Ne} nz={nz}", flush=True)
    B = ColumnBatch(ctx, col)
    lam = 0.4358665215 * 300.0
    b = rhs(col)
    f = ctx.factor(B.ops, lam, 0)
    code, inf = f.check()
    assert code == 0, inf
    x = B.empty_state()
    inf = ctx.stage_solve(f, [dev(b)], [1.0], [], [], x, info=True)
    assert inf["status"] == "HEVI_OK", inf
    xg = host(x)
    for c in range(2):
        z, J, gz, r0, T0 = oracle.column_of(col, c)
        A = oracle.form_A(oracle.column_L(N, Ne, inputs.CONSTS, z, J, gz, r0, T0,
                                          U0_k3=oracle.u0_of(col, c)), lam)
        bb = oracle.bc_project(nz, gz, oracle.vec_of(b, c))
        xc = oracle.vec_of(xg, c)
        res = np.abs(A @ xc - bb).max()
        berr = res / (np.abs(A).sum(1).max() * np.abs(xc).max() + np.abs(bb).max())
        print(f"column {c}: backward error {berr:.2e}", flush=True)
        assert berr < 1e-14, berr
    with pytest.raises(hevi.HeviError) as ei:
        B2 = ColumnBatch(ctx, W(inputs.make_columns(N, Ne + (5 if N == 4 else 1), 1)))
        ctx.factor(B2.ops, lam, 0)
    assert ei.value.code == 2
