"""Host-side tests of the C ABI (no GPU): the library loads and exports every
function include/rklt.h declares, and the host transform designer
(rklt_build_transform, its own Newton/bisection root finder) and zig-zag
table agree with the oracle on dense parameter grids and reject what the
paper rules out."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import rklt_oracle as o
from golden_io import integers, matrices
from paper_2111_14239_amd import rklt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "rklt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rklt_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    declared = _declared_functions()
    assert len(declared) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", rklt.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (rklt_\w+)", out))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    assert set(rklt.EXPORTED) == set(declared)


def test_struct_sizes_match_header_layout():
    # rklt_result is 32 bytes, rklt_image 64, rklt_tuning 16 (x86-64 SysV)
    import ctypes as C
    assert C.sizeof(rklt.Result) == 32
    assert C.sizeof(rklt.Image) == 64
    assert C.sizeof(rklt.Tuning) == 16


@pytest.mark.parametrize("N", [2, 3, 4, 5, 8, 16, 32])
def test_transform_matches_oracle_on_rho_grid(N):
    for rho in np.concatenate([np.linspace(0.02, 0.98, 25), [0.01, 0.3, 0.5, 0.95, 0.99]]):
        K = o.klt(N, float(rho))
        gamma = float(np.max(np.abs(K)))
        for alpha in (2.0, 3.0, 8.0 / gamma):
            T = o.rounded_klt(N, float(rho), alpha)
            try:
                d, s = o.scaling(T)
            except o.OracleError:
                with pytest.raises(rklt.RkltError) as e:
                    rklt.build_transform(N, float(rho), alpha)
                assert e.value.status == rklt.E_SINGULAR
                continue
            t = rklt.build_transform(N, float(rho), alpha)
            assert np.allclose(t.K, K, rtol=0, atol=1e-12), (N, rho)
            assert np.array_equal(t.T, T), (N, rho, alpha)
            assert np.array_equal(t.d, d)
            assert np.allclose(t.s, s, rtol=1e-15)
            That = np.diag(s) @ T
            assert np.allclose(t.G @ That, np.eye(N), atol=1e-10)
            assert t.orthogonal == o.is_orthogonal(T)
            assert t.adds_only == bool(np.all(np.abs(T) <= 1))
            assert t.max_abs == int(np.max(np.abs(T)))
            assert t.max_row_l1 == int(np.max(np.sum(np.abs(T), axis=1)))


def test_transform_reproduces_table1():
    gold = matrices("table1_rklt.txt")
    for name in ("T1", "T2", "T3", "T4"):
        for rho in gold[name]["rho"]:
            t = rklt.build_transform(8, rho, 2.0)
            assert np.array_equal(t.T, gold[name]["rows"])
            assert list(t.d) == gold[name]["d"]
    assert rklt.build_transform(8, 0.2, 2.0).orthogonal
    assert not rklt.build_transform(8, 0.5, 2.0).orthogonal
    assert not rklt.build_transform(8, 0.7, 2.0).orthogonal
    assert rklt.build_transform(8, 0.9, 2.0).orthogonal


@pytest.mark.parametrize("edge", [0.3890638, 0.3902400, 0.6022009, 0.7972576])
def test_transform_switch_points_match_oracle(edge):
    # T changes at these rho (N = 8, alpha = 2); both sides must agree there
    for rho in (edge - 2e-7, edge + 2e-7, edge - 1e-4, edge + 1e-4):
        assert np.array_equal(rklt.build_transform(8, rho, 2.0).T, o.rounded_klt(8, rho, 2.0)), rho


def test_transform_errors():
    with pytest.raises(rklt.RkltError) as e:
        rklt.build_transform(8, 0.5, 1.0)  # every |K_ij| < 1/2: T = 0
    assert e.value.status == rklt.E_SINGULAR and "zero" in str(e.value)
    for N, rho, alpha in ((8, 0.0, 2.0), (8, 1.0, 2.0), (8, -0.5, 2.0), (1, 0.5, 2.0), (33, 0.5, 2.0),
                          (8, 0.5, 0.0), (8, 0.5, -2.0), (8, 0.5, math.inf), (8, math.nan, 2.0)):
        with pytest.raises(rklt.RkltError) as e:
            rklt.build_transform(N, rho, alpha)
        assert e.value.status == rklt.E_INVAL, (N, rho, alpha)
        assert str(e.value)
    # the message is cleared by the next successful call
    rklt.build_transform(8, 0.5, 2.0)
    assert rklt.lib().rklt_last_error() == b""


def test_zigzag_matches_jpeg_and_oracle():
    assert list(rklt.zigzag(8)) == integers("jpeg_zigzag8.txt")
    for N in range(1, 33):
        assert list(rklt.zigzag(N)) == [i * N + j for i, j in o.zigzag_order(N)], N
    with pytest.raises(rklt.RkltError):
        rklt.zigzag(0)
    with pytest.raises(rklt.RkltError):
        rklt.zigzag(33)


def test_null_arguments_are_rejected_without_a_gpu():
    import ctypes as C
    L = rklt.lib()
    assert L.rklt_build_transform(8, 0.5, 2.0, None) == rklt.E_INVAL
    assert L.rklt_zigzag(8, None) == rklt.E_INVAL
    assert L.rklt_ctx_create(0, None) == rklt.E_INVAL
    assert L.rklt_ctx_destroy(None) == rklt.E_INVAL
    assert L.rklt_plan_destroy(None) == rklt.E_INVAL
    assert L.rklt_plan_run(None, None, None) == rklt.E_INVAL
    assert L.rklt_codec(None, None, None, None, None) == rklt.E_INVAL
    assert L.rklt_copy_bytes(None, None, 16, None) == rklt.E_INVAL
    h = C.c_void_p()
    assert L.rklt_plan_create(None, None, 0, None, C.byref(h)) == rklt.E_INVAL
    assert L.rklt_plan_update(None, None, 0, None) == rklt.E_INVAL
    assert L.rklt_plan_autotune(None, None, 1, None, None) == rklt.E_INVAL
    assert L.rklt_plan_mssim(None, None, None) == rklt.E_INVAL
    f = C.c_int32()
    assert L.rklt_ctx_mfma_form(None, 0, 1, C.byref(f)) == rklt.E_INVAL
    assert L.rklt_klt_matrix(8, 0.5, None) == rklt.E_INVAL
    assert L.rklt_dct_matrix(8, None) == rklt.E_INVAL
    M = (C.c_double * 64)()
    assert L.rklt_ctx_add_float_transform(None, 8, M, C.byref(f)) == rklt.E_INVAL
    assert L.rklt_ctx_add_quantizer(None, 0, M, C.byref(f)) == rklt.E_INVAL


def test_comparison_transforms_match_oracle():
    # the float arms of the experiment: exact KLT (§2.1) and the orthonormal
    # DCT-II, from the library's own host code, against the oracle's
    from oracle import metrics as m
    for N in (2, 4, 8, 16, 32):
        assert np.allclose(rklt.dct_matrix(N), m.dct_matrix(N), atol=1e-15, rtol=0)
        for rho in (0.05, 0.3, 0.4, 0.7, 0.8, 0.95):
            assert np.allclose(rklt.klt_matrix(N, rho), o.klt(N, rho), atol=1e-12, rtol=0), (N, rho)
            # the same K that rklt_build_transform reports
            assert np.array_equal(rklt.klt_matrix(N, rho), rklt.build_transform(N, rho, 4.0).K)
    for bad in ((1, 0.5), (33, 0.5), (8, 0.0), (8, 1.0), (8, math.nan)):
        with pytest.raises(rklt.RkltError) as e:
            rklt.klt_matrix(*bad)
        assert e.value.status == rklt.E_INVAL
    for N in (1, 33):
        with pytest.raises(rklt.RkltError):
            rklt.dct_matrix(N)


def test_library_uses_torchs_hip_runtime():
    # torch's device pointers and stream handles are only valid in the HIP
    # runtime torch itself loaded; the binding must make the library bind to it
    import torch
    maps = open("/proc/self/maps").read()
    hips = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(hips) == 1, hips
    assert os.path.dirname(torch.__file__) in next(iter(hips))
