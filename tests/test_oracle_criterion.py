"""Pins of the criterion exponent (Sec. 3.3, Sec. 4.1): the error balance of a
k-th order scheme opens a cell when N' >= (c 2^l / L)^(2k-2); for k = 2 the
supraconvergent error bound balances with h ~ N'^(-1/4), exponent 4.

A uniform lattice of 8^6 particles fixes the answer by hand: a level-l cell holds
N' = 8^(6-l).  With c = 1 and L = 1, exponent 2 opens while 8^(6-l) >= 4^l (levels
0-3, so the leaves are the 8^4 cells of level 4), exponent 4 while 8^(6-l) >= 16^l
(levels 0-2: 8^3 leaves), exponent 1 while 8^(6-l) >= 2^l (levels 0-4: 8^5 leaves).
"""
import pytest

from workloads import uniform_lattice_points


@pytest.mark.parametrize("pw,n", [(0, 8 ** 4), (2, 8 ** 4), (4, 8 ** 3), (1, 8 ** 5)])
def test_lattice_leaves(oracle_mod, pw, n):
    O = oracle_mod.OracleCloud(uniform_lattice_points(6), order=2, c=1.0, max_depth=8,
                               criterion_pow=pw)
    assert O.n == n and O.n == 1 + 7 * O.n_opened


def test_exponent_in_thresholds(oracle_mod):
    T2 = oracle_mod.thresholds(order=2, c=0.5, max_depth=6)
    T4 = oracle_mod.thresholds(order=2, c=0.5, max_depth=6, criterion_pow=4)
    T44 = oracle_mod.thresholds(order=4, c=0.5, max_depth=6)  # 2k - 2 = 6 for k = 4
    for l in range(7):
        t = 0.5 * 2 ** l
        assert T2[l] == pytest.approx(t ** 2, rel=1e-15)
        assert T4[l] == pytest.approx(t ** 4, rel=1e-15)
        assert T44[l] == pytest.approx(t ** 6, rel=1e-15)


def test_rejects_bad_exponent(oracle_mod):
    with pytest.raises(RuntimeError):
        oracle_mod.OracleCloud(uniform_lattice_points(2), order=2, c=1.0, max_depth=4,
                               criterion_pow=-1)
