"""Host-side design tools of the library (no GPU): the figures of merit of
§3.1 and Algorithm 1 (§3), in the library's own C++, against the values the
paper prints (Tables 1 and 2, tests/golden/) and against the oracle's
independent numpy versions on parameter grids."""
import math

import numpy as np
import pytest

from golden_io import matrices, table
from oracle import metrics as m
from oracle import rklt_oracle as o
from paper_2111_14239_amd import rklt


def _that(N, rho, alpha):
    T = o.rounded_klt(N, rho, alpha)
    _, s = o.scaling(T)
    return np.diag(s) @ T.astype(np.float64)


def test_algorithm1_reproduces_table1():
    gold = matrices("table1_rklt.txt")
    found = rklt.algorithm1(8, 2.0, 0.1)
    assert [round(a, 6) for a, _, _ in found] == [0.1, 0.4, 0.7, 0.8]
    # T_4 (the RDCT) holds from 0.8 to the top of the grid
    assert [round(b, 6) for _, b, _ in found] == [0.3, 0.6, 0.7, 0.9]
    for (_, _, T), name in zip(found, ("T1", "T2", "T3", "T4")):
        assert np.array_equal(T, gold[name]["rows"])


@pytest.mark.parametrize("N,alpha,step", [(8, 2.0, 0.01), (8, 3.0, 0.02), (4, 4.0, 0.05), (16, 6.0, 0.05),
                                          (8, 1.0, 0.1), (32, 8.0, 0.1)])
def test_algorithm1_matches_oracle_sweep(N, alpha, step):
    got = rklt.algorithm1(N, alpha, step)
    want = m.derive_matrices(N, alpha, step)
    assert len(got) == len(want)
    for (a, _, T), (rho, Tw) in zip(got, want):
        assert a == pytest.approx(rho, abs=1e-12) and np.array_equal(T, Tw)
    # the last rho of each entry is the grid point before the next entry's first
    for (_, b, _), (a2, _, _) in zip(got, got[1:]):
        assert a2 - b == pytest.approx(step, abs=1e-9)


def test_algorithm1_size_query_and_errors():
    L = rklt.lib()
    import ctypes as C
    n = C.c_int32()
    assert L.rklt_algorithm1(8, 2.0, 0.1, None, 0, C.byref(n)) == rklt.OK and n.value == 4
    one = (rklt.DesignEntry * 1)()
    assert L.rklt_algorithm1(8, 2.0, 0.1, one, 1, C.byref(n)) == rklt.OK and n.value == 4
    assert round(one[0].rho_first, 6) == 0.1 and round(one[0].rho_last, 6) == 0.3
    for args in ((1, 2.0, 0.1), (33, 2.0, 0.1), (8, 0.0, 0.1), (8, math.inf, 0.1), (8, 2.0, 0.0),
                 (8, 2.0, 0.6), (8, 2.0, 1e-8)):
        assert L.rklt_algorithm1(*args, None, 0, C.byref(n)) == rklt.E_INVAL, args
    assert L.rklt_algorithm1(8, 2.0, 0.1, None, 0, None) == rklt.E_INVAL
    assert L.rklt_algorithm1(8, 2.0, 0.1, None, 3, C.byref(n)) == rklt.E_INVAL


def test_measures_reproduce_table2():
    rows = {r[0]: r for r in table("table2_measures.txt")}
    for i, rho in ((1, 0.3), (2, 0.4), (3, 0.7), (4, 0.8)):
        K = rklt.klt_matrix(8, rho)
        kr = rows[f"K{rho}"]
        mk = rklt.transform_measures(K, K, rho)
        assert round(mk["coding_gain_db"], 4) == pytest.approx(float(kr[2]), abs=1e-4)
        assert mk["efficiency_pct"] == pytest.approx(100.0, abs=1e-9)
        assert mk["mse"] == 0 and mk["error_energy"] == 0
        tr = rows[f"That{i}"]
        mt = rklt.transform_measures(_that(8, rho, 2.0), K, rho)
        assert mt["error_energy"] == pytest.approx(float(tr[4]), abs=1e-4)
        assert mt["mse"] == pytest.approx(float(tr[5]), abs=1e-4)
        if i in (1, 4):  # orthogonal T: both coding-gain readings coincide
            assert mt["coding_gain_db"] == pytest.approx(float(tr[2]), abs=1e-4)
            assert mt["coding_gain_tt_db"] == pytest.approx(mt["coding_gain_db"], abs=1e-12)
            assert mt["efficiency_pct"] == pytest.approx(float(tr[3]), abs=1e-4)
        else:
            assert mt["coding_gain_tt_db"] == pytest.approx(float(tr[2]), abs=1e-4)
    ref = rows["RDCTvsDCT"]
    md = rklt.transform_measures(_that(8, 0.95, 2.0), rklt.dct_matrix(8), 0.95)
    assert md["error_energy"] == pytest.approx(float(ref[4]), abs=1e-4)
    assert md["mse"] == pytest.approx(float(ref[5]), abs=1e-4)


@pytest.mark.parametrize("N", [4, 8, 16])
def test_measures_match_oracle_on_grid(N):
    for rho in (0.05, 0.3, 0.5, 0.8, 0.95):
        for alpha in (2.0, 3.0, 5.0):
            T = o.rounded_klt(N, rho, alpha)
            try:
                Th = _that(N, rho, alpha)
            except o.OracleError:
                continue  # singular: not a transform
            K = o.klt(N, rho)
            R = o.markov_covariance(N, rho)
            got = rklt.transform_measures(Th, K, rho)
            assert got["coding_gain_db"] == pytest.approx(m.coding_gain(Th, R), abs=1e-9)
            assert got["coding_gain_tt_db"] == pytest.approx(m.coding_gain(Th, R, Th.T), abs=1e-9)
            assert got["efficiency_pct"] == pytest.approx(m.transform_efficiency(Th, R), abs=1e-9)
            assert got["mse"] == pytest.approx(m.mse_vs_klt(K, Th, R), abs=1e-12)
            assert got["error_energy"] == pytest.approx(m.total_error_energy(K, Th), abs=1e-10)


def test_measures_errors():
    C8 = rklt.dct_matrix(8)
    with pytest.raises(rklt.RkltError) as e:
        rklt.transform_measures(np.ones((8, 8)), C8, 0.5)
    assert e.value.status == rklt.E_SINGULAR
    for rho in (0.0, 1.0, math.nan):
        with pytest.raises(rklt.RkltError) as e:
            rklt.transform_measures(C8, C8, rho)
        assert e.value.status == rklt.E_INVAL
    bad = C8.copy()
    bad[0, 0] = math.inf
    with pytest.raises(rklt.RkltError):
        rklt.transform_measures(bad, C8, 0.5)
    assert rklt.lib().rklt_transform_measures(8, None, None, 0.5, None) == rklt.E_INVAL
