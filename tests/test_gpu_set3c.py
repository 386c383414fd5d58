"""Parity of the set-3C (total energy) path of the HIP library with the oracle.

Set 3C (Appendix A.1 eq. set3c, Jacobian eq. set3c_jacobian at rest) carries the
total energy E as the fifth state variable; its operator adds a dP/drho column to
the pressure gradient of the momentum rows.  Same bars as set 2C: FP64 path
<= 1e-12, FP32 factors + reduced refinement <= 1e-10 (relative L2 per column and
variable against the oracle with one long-double refinement step), or 4 x the
rounding floor of the stage recipe (stage_floor) where that is larger.
"""
import numpy as np
import pytest

import oracle
from oracle import tableaux
from paper_2311_11425_amd import inputs
from parity_util import relerr_cols, stage_floor, step_tolerance, sub_batch, sub_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMIX = 1e-10


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


def c3(col):
    return inputs.as_set(col, "3C")


def cases():
    return {
        "cfg1_hetero": lambda: c3(inputs.config1(heterogeneous=True)),
        "cfg2_ragged300": lambda: c3(inputs.config2(ncols=300)),
        "N3_tilt_deep": lambda: c3(inputs.make_columns(3, 5, 130, profile="lapse", seed=31,
                                                       surface_max=1500.0, tilt=0.2, deep=True)),
        "N6": lambda: c3(inputs.make_columns(6, 3, 70, profile="lapse", seed=37)),
        # N > 6: assembly kernel + split-window LU
        "N7": lambda: c3(inputs.make_columns(7, 2, 70, profile="lapse_capped", z_top=60e3,
                                             seed=33)),
        "N8_tilt": lambda: c3(inputs.make_columns(8, 2, 66, profile="isothermal", seed=38,
                                                  tilt=0.05)),
        "N4_Ne1": lambda: c3(inputs.make_columns(4, 1, 65, profile="isothermal", seed=39)),
        "N1": lambda: c3(inputs.make_columns(1, 6, 40, profile="isothermal", seed=34)),
        # 161 nodes: the three-kernel stage path
        "N4_Ne40": lambda: c3(inputs.make_columns(4, 40, 70, profile="lapse_capped",
                                                  z_top=120e3, seed=36)),
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
def test_3c_apply_parity(ctx, name):
    from paper_2311_11425_amd.driver import ColumnBatch
    col = cases()[name]()
    print(f"3C apply {name} N={col['N']} Ne={col['Ne']} ncols={col['z'].shape[1]}", flush=True)
    B = ColumnBatch(ctx, col)
    code, bad = B.ops.check()
    assert code == 0 and bad == -1
    qn, qref = inputs.perturbed_state(col, seed=5)
    y = B.empty_state()
    ctx.apply_op(B.ops, dev(qn), y, xref=dev(qref))
    assert relerr_cols(host(y), oracle.apply_batch(col, qn, qref)) < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", list(cases()))
def test_3c_solve_parity(ctx, name, prec):
    from paper_2311_11425_amd.driver import ColumnBatch
    col = cases()[name]()
    print(f"3C solve {name} prec={prec} ncols={col['z'].shape[1]}", flush=True)
    B = ColumnBatch(ctx, col)
    lam = lam_for(col)
    b = rhs(col)
    f = ctx.factor(B.ops, lam, prec)
    code, inf = f.check()
    assert code == 0, inf
    x = B.empty_state()
    inf = ctx.stage_solve(f, [dev(b)], [1.0], [], [], x, refine=(4, 1e-13), info=True)
    assert inf["status"] == "HEVI_OK", inf
    xo = oracle.solve_batch(col, lam, b, refine=1)
    err = relerr_cols(host(x), xo)
    tol = TOL64 if prec == 0 else TOLMIX
    print(f"rel err {err:.2e} (tol {tol:.2e}) info {inf}", flush=True)
    assert err < tol, err
    x1 = B.empty_state()
    inf = ctx.stage_solve(f, [dev(b)], [1.0], [], [], x1, refine=(4, 1e-13, 1), info=True)
    assert inf["status"] == "HEVI_OK", inf
    assert relerr_cols(host(x1), xo) < TOL64


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("which", ["ARK3_cfg2_sample", "ARK2_cfg1"])
def test_3c_ark_stagewise_parity(ctx, which, mode):
    """Each stage solve of a GPU ARK step in set 3C, against the oracle from the GPU's
    own stage values (as the set-2C stagewise test)."""
    from paper_2311_11425_amd.driver import ArkStepper, ColumnBatch
    if which == "ARK2_cfg1":
        col, tabname, dt = c3(inputs.config1(heterogeneous=True)), "ARK2", 30.0
    else:
        col, tabname, dt = c3(inputs.config2(ncols=200)), "ARK3", 300.0
    prec, refine, bar = {"fp64": (0, (0, 1e-12, 0), TOL64),
                         "mixed": (1, (4, 1e-13, 0), TOLMIX)}[mode]
    print(f"3C stagewise {which} {mode}", flush=True)
    B = ColumnBatch(ctx, col)
    st = ArkStepper(ctx, B, tabname, dt, precision=prec, refine=refine)
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
        tol = max(bar, 4 * stage_floor(oracle, col, st.lam, qE, P, Q[i], x_or))
        print(f"stage {i + 1}: solve rel err {err:.2e} (tolerance {tol:.2e})", flush=True)
        assert err < tol, (i, err, tol)
        assert relerr_cols(S[i], oracle.apply_batch(col, Q[i], qref)) < 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_3c_ark_step_parity(ctx, prec):
    """Two ARK3 steps of a set-3C ne=30-shape sample: stage increments and updates."""
    from paper_2311_11425_amd.driver import ArkStepper, ColumnBatch
    col = c3(inputs.config2(ncols=200))
    tab, dt = tableaux.as_float(tableaux.ark3()), 300.0
    print(f"3C ark prec={prec}", flush=True)
    B = ColumnBatch(ctx, col)
    st = ArkStepper(ctx, B, "ARK3", dt, precision=prec)
    qn, qref = inputs.perturbed_state(col)
    q, qr, qo = dev(qn), dev(qref), qn.copy()
    for n in range(2):
        out = B.empty_state()
        for inf in st.step(q, qr, out, info=True):
            assert inf["status"] == "HEVI_OK", inf
        qo_next, Qo, _ = oracle.ark_step_batch(col, tab, dt, qo, qref, refine=1, want_stages=True)
        tol = step_tolerance(oracle, col, tab, dt, qo, qref, Qo, TOL64 if prec == 0 else TOLMIX)
        for i in range(1, st.s):
            assert relerr_cols(host(st.Q[i]) - qo, Qo[i] - qo) < tol
        assert relerr_cols(host(out) - qo, qo_next - qo) < tol
        q, qo = out, qo_next


def test_3c_full_size_sampled(ctx):
    """86,402 set-3C columns (the ne=30 shape, one wavefront per tile), one ARK3 step;
    96 sampled columns against the oracle."""
    from paper_2311_11425_amd.driver import ArkStepper, ColumnBatch
    col = c3(inputs.config2())
    print("3C full cfg2", flush=True)
    B = ColumnBatch(ctx, col)
    st = ArkStepper(ctx, B, "ARK3", 300.0)
    qn, qref = inputs.perturbed_state(col)
    out = B.empty_state()
    for inf in st.step(dev(qn), dev(qref), out, info=True):
        assert inf["status"] == "HEVI_OK", inf
    rng = np.random.default_rng(78)
    idx = np.sort(np.concatenate([rng.choice(col["z"].shape[1], 93, replace=False),
                                  [0, 64, col["z"].shape[1] - 1]]))
    sc = sub_batch(col, idx)
    tab = tableaux.as_float(tableaux.ark3())
    qs, qrs = sub_state(qn, idx), sub_state(qref, idx)
    qo_next, Qo, _ = oracle.ark_step_batch(sc, tab, 300.0, qs, qrs, refine=1, want_stages=True)
    tol = step_tolerance(oracle, sc, tab, 300.0, qs, qrs, Qo, TOL64)
    for i in range(1, 4):
        assert relerr_cols(host(st.Q[i])[..., idx] - qs, Qo[i] - qs) < tol
    assert relerr_cols(host(out)[..., idx] - qs, qo_next - qs) < tol


def test_3c_invalid_energy_reported(ctx):
    """A reference total energy at or below the potential energy rho0 g z leaves no
    positive pressure (P0 = (gamma-1)(E0 - rho0 Phi)): the column is reported invalid."""
    from paper_2311_11425_amd.driver import ColumnBatch
    col = c3(inputs.config1(ncols=100))
    col["E0"] = col["E0"].copy()
    col["E0"][7, 41] = col["rho0"][7, 41] * inputs.GRAV * col["z"][7, 41]
    B = ColumnBatch(ctx, col)
    code, bad = B.ops.check()
    assert code == 1 and bad == 41


@pytest.mark.parametrize("prec", [0, 1])
def test_3c_noalloc_matches(ctx, prec):
    """The allocation-free entry point runs the set-3C kernels too: bitwise equal to
    hevi_factor + hevi_stage_solve."""
    from paper_2311_11425_amd.driver import ColumnBatch
    col = c3(inputs.config2(ncols=257))
    B = ColumnBatch(ctx, col)
    lam = lam_for(col)
    b = rhs(col)
    f = ctx.factor(B.ops, lam, prec)
    x = B.empty_state()
    ctx.stage_solve(f, [dev(b)], [1.0], [], [], x, refine=(4, 1e-13))
    x2 = B.empty_state()
    ctx.solve_noalloc(B.ops, lam, prec, [dev(b)], [1.0], [], [], x2, refine=(4, 1e-13))
    assert np.array_equal(host(x), host(x2))


def test_3c_rejected_by_group_and_server(ctx):
    """Group steps and the server run the set-2C multi-problem kernels only."""
    from paper_2311_11425_amd import hevi
    from paper_2311_11425_amd.driver import ColumnBatch
    col = c3(inputs.config1(ncols=70))
    B = ColumnBatch(ctx, col)
    qn, qref = inputs.perturbed_state(col)
    member = {"ops": B.ops, "qn": dev(qn), "qref": dev(qref), "out": B.empty_state(),
              "Q": [None] + [B.empty_state() for _ in range(3)],
              "S": [B.empty_state() for _ in range(4)]}
    with pytest.raises(hevi.HeviError) as ei:
        hevi.Group(ctx, [member], "ARK3", 30.0)
    assert ei.value.code == 1
    srv = hevi.Server(ctx, 1 << 30)
    with pytest.raises(hevi.HeviError) as ei:
        srv.register(B.ops, 10.0)
    assert ei.value.code == 1
    srv.close()
