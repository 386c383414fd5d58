"""CPU-side checks of the C ABI: the library loads, exports every declared symbol,
validates arguments without a GPU, and its tableaux/sizes agree with independent
definitions.  No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import tableaux as otab
from paper_2311_11425_amd import hevi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hevi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hevi_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = hevi.load()
    decl = declared_symbols()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(hevi.EXPORTS) == decl


def test_status_strings():
    lib = hevi.load()
    for code in range(10):
        s = lib.hevi_status_str(code)
        assert s and s != b"unknown status"
    assert lib.hevi_status_str(99) == b"unknown status"


def test_create_rejects_missing_device():
    lib = hevi.load()
    h = ctypes.c_void_p()
    code = lib.hevi_create(1000, ctypes.byref(h))
    assert code == 4 and not h.value
    assert lib.hevi_create(0, None) == 1


@pytest.mark.parametrize("name,ref", [("ARK2", otab.ark2("b")), ("ARK2b", otab.ark2("b")),
                                      ("ARK2a", otab.ark2("a")), ("ARK3", otab.ark3()),
                                      ("ARS343", otab.ars343()), ("ARK4", otab.ark4())])
def test_tableau_matches_independent_transcription(name, ref):
    t = hevi.tableau(name)
    r = otab.as_float(ref)
    assert t["s"] == len(r["b"])
    assert np.allclose(t["Aexp"], r["Aexp"], rtol=0, atol=2e-16)
    assert np.allclose(t["Aimp"], r["Aimp"], rtol=0, atol=2e-16)
    assert np.allclose(t["b"], r["b"], rtol=0, atol=2e-16)


def test_tableau_unknown():
    with pytest.raises(hevi.HeviError):
        hevi.tableau("RK4")


def test_sizes():
    s = hevi.sizes(4, 10)
    nz = 41
    assert s["ops"] == nz * 8 * 8
    # U (4N+1) and L (2N) entries plus three byte planes (pivots, U extents, row scales)
    assert s["factors"] == nz * (17 + 8) * 8 + 3 * nz
    s32 = hevi.sizes(4, 10, precision=1)
    assert s32["factors"] == nz * 25 * 4 + 3 * nz
    # resident: factors + 6 FP64 scratch fields per node; FP32 factors of orders with
    # the fused factorisation hold no FP64 assembly buffer
    assert s["resident"] == s["factors"] + nz * 6 * 8
    assert s32["resident"] == s32["factors"] + nz * 6 * 8
    s7 = hevi.sizes(7, 10, precision=1)
    nz7 = 71
    assert s7["resident"] == s7["factors"] + nz7 * 6 * 8 + nz7 * 29 * 8
    # an FP32-factor simulation holds about 60% of an FP64 one (151 against 251 bytes per
    # node at order 4: FP32 U and L, the same byte planes and FP64 scratch)
    assert s32["resident"] <= 0.605 * s["resident"]
    # paper layout: LAPACK band with kl = ku = 5(N+1)-1, ldab = 2kl+ku+1 rows
    n = 5 * nz
    kl = 5 * 5 - 1
    assert s["paper_band"] == n * (2 * kl + kl + 1) * 8 + 4 * n


@pytest.mark.parametrize("N,Ne,nc", [(0, 4, 1), (9, 4, 1), (4, 0, 1), (4, 5000, 1), (4, 4, -1)])
def test_sizes_rejects_bad_shapes(N, Ne, nc):
    with pytest.raises(hevi.HeviError) as e:
        hevi.sizes(N, Ne, nc)
    assert e.value.code == 2


def test_serve_and_group_reject_null_handles():
    """Failure handling that needs no device: NULL handles and bad arguments are
    rejected synchronously (HEVI_E_INVALID), destroy/free accept NULL."""
    import ctypes
    lib = hevi.load()
    out = ctypes.c_void_p()
    assert lib.hevi_serve_create(None, 1 << 20, 4, None, ctypes.byref(out)) == 1
    sid = ctypes.c_int32(0)
    assert lib.hevi_serve_register(None, None, 1.0, 0, ctypes.byref(sid)) == 1
    t = ctypes.c_uint64(0)
    assert lib.hevi_serve_submit(None, 0, 1, None, None, 0, None, None, None, ctypes.byref(t)) == 1
    done = ctypes.c_int32(0)
    assert lib.hevi_serve_poll(None, 1, ctypes.byref(done), None, None) == 1
    assert lib.hevi_serve_wait(None, 1, None, None) == 1
    assert lib.hevi_serve_release(None, 0) == 1
    lib.hevi_serve_destroy(None)
    assert lib.hevi_group_create(None, 1, None, b"ARK3", 1.0, 0, None, ctypes.byref(out),
                                 None) == 1
    assert lib.hevi_group_step(None, None, 1, None) == 1
    assert lib.hevi_group_set_plan(None, None, None) == 1
    lib.hevi_group_free(None)


def test_kernel_gll_tables_match_oracle():
    """The kernels' compile-time GLL tables (csrc/hevi_gll.h, correctly rounded from 50-digit
    values) agree with the oracle's independent double-precision Newton tables to a few ulp,
    and every row of each differentiation matrix sums to zero to within rounding."""
    import oracle
    txt = open(os.path.join(ROOT, "paper_2311_11425_amd", "csrc", "hevi_gll.h")).read()
    for N in range(1, 9):
        blk = txt[txt.index(f"struct Gll<{N}>"):]
        blk = blk[:blk.index("};\n};")]
        nums = [float.fromhex(t) for t in re.findall(r"-?0x[0-9a-fp.+-]+", blk)]
        assert len(nums) == (N + 1) + (N + 1) ** 2
        w = np.array(nums[:N + 1])
        D = np.array(nums[N + 1:]).reshape(N + 1, N + 1)
        _, ow, oD = oracle.gll(N)
        oD = np.asarray(oD).reshape(N + 1, N + 1)
        assert np.abs(w - ow).max() <= 4e-16 * max(1.0, np.abs(ow).max())
        assert np.abs(D - oD).max() <= 2e-14 * max(1.0, np.abs(oD).max())
        assert np.abs(D.sum(axis=1)).max() <= 1e-15 * np.abs(D).max() * (N + 1)
        assert abs(w.sum() - 2.0) <= 4e-16 * (N + 1)
