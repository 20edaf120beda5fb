"""Pins of the oracle's primitives: Philox, bounded draws, Q16 encoding."""

import math

import numpy as np
import pytest

import oracle
from conftest import golden_path


def _kat():
    rows = []
    for line in open(golden_path("philox4x32_10_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert oracle.philox4x32_10(ctr, key) == out


def test_bounded_range_one_is_zero():
    for s in range(50):
        assert oracle.bounded(123, s, 0, 0, 0, 1) == 0


@pytest.mark.parametrize("rng", [2, 3, 7, 10, 1000])
def test_bounded_uniform_small_ranges(rng):
    draws = np.array([oracle.bounded(99, s, 1, 2, 3, rng) for s in range(20000)])
    assert draws.min() >= 0 and draws.max() < rng
    counts = np.bincount(draws, minlength=rng)
    expected = draws.size / rng
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 99.9% quantile of chi-square with rng-1 dof is below dof + 5*sqrt(2 dof) + 10.
    dof = rng - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof) + 10


def test_bounded_high_rejection_range_is_uniform():
    # range = 2^63 + 1 rejects almost half of all 64-bit words; the accepted
    # outputs must still be uniform on [0, range): mean ~ 2^62, both halves hit.
    rng = (1 << 63) + 1
    draws = np.array([oracle.bounded(5, s, 0, 0, 1, rng) for s in range(4000)], dtype=np.float64)
    assert draws.max() < rng
    mean = draws.mean() / 2.0 ** 62
    assert abs(mean - 1.0) < 0.1
    assert (draws < 2.0 ** 62).mean() > 0.4


def test_bounded_streams_are_distinct():
    a = [oracle.bounded(1, s, 0, 0, 0, 1 << 40) for s in range(100)]
    b = [oracle.bounded(1, s, 0, 0, 1, 1 << 40) for s in range(100)]
    c = [oracle.bounded(2, s, 0, 0, 0, 1 << 40) for s in range(100)]
    assert len(set(a)) == 100 and a != b and a != c


def test_log2fx_exact_on_powers_of_two():
    for p in range(64):
        assert oracle.log2fx(1 << p) == p << 16


def test_log2fx_error_bound():
    # Truncating to 12 mantissa bits loses at most log2(1 + 1/4096); table
    # rounding adds at most half a Q16 unit.
    bound = math.log2(1 + 1 / 4096) + 0.5 / 65536 + 1e-12
    rng = np.random.Generator(np.random.PCG64(0))
    xs = list(range(1, 5000)) + [int(x) for x in rng.integers(1, 1 << 62, size=5000)]
    for x in xs:
        err = oracle.log2fx(x) / 65536.0 - math.log2(x)
        assert -bound <= err <= 0.5 / 65536 + 1e-12, x


def test_log2fx_monotone():
    vals = [oracle.log2fx(x) for x in range(1, 20000)]
    assert all(a <= b for a, b in zip(vals, vals[1:]))


def test_weight_from_log_values():
    assert oracle.weight_from_log(0, 0) == 1 << 31
    for s in range(31):
        assert oracle.weight_from_log(s << 16, 0) == 1 << (31 - s)
    assert oracle.weight_from_log(40 << 16, 0) == 1  # floored, never zero
    rng = np.random.Generator(np.random.PCG64(1))
    for d in rng.integers(0, 16 << 16, size=2000):
        q = oracle.weight_from_log(int(d), 0)
        exact = 2.0 ** (31 - int(d) / 65536.0)
        # the fraction of the exponent is truncated to 12 bits (so the table
        # entry is at most 2^(1/4096) above), then table rounding and the shift
        assert exact - 1.5 <= q <= exact * 2 ** (1 / 4096) + 0.5


def test_fixed_point_tables_shape():
    lt, et = oracle.fixed_point_tables()
    assert lt[0] == 0 and et[0] == 1 << 31
    assert np.all(np.diff(lt) >= 0) and np.all(np.diff(et.astype(np.int64)) <= 0)
    assert lt[-1] < 65536 and et[-1] > (1 << 30)
