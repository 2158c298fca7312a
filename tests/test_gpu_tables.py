"""Transition tables built on the device against the oracle's exact solve.

The hybrid strategy (Sec. III-C) samples stratified cubes from cached tables
of the exact discrete SGF (Eq. 8).  The library builds them on the GPU (sine
transform in the plane, tridiagonal solves along the stratification axis,
binary64) and stores an inverse CDF in 32-bit fixed point.  Here the cached
tables themselves are read back (mw_sgf_table) and compared entry by entry
with the CDF formed from the oracle's independent conjugate-gradient solve
of the same lattice: every CDF entry within one 32-bit step, first-transition
sign bits equal wherever the weight is not negligible, and the weight sum
within 1e-6 relative.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_09730_amd as lib
    lib.mw_init(0)
    return lib


def _code(eps):
    return int(np.rint(np.float64(np.float32(eps)) * 65536.0))


def _profiles(n):
    """Plane-code sequences: uniform, two layers, three layers with a high-k
    film, and random codes per plane."""
    rng = np.random.Generator(np.random.PCG64(1000 + n))
    half = n // 2
    return {
        "uniform": [_code(3.9)] * n,
        "two_layers": [_code(3.9)] * half + [_code(2.7)] * (n - half),
        "film": [_code(3.9)] * (n // 4) + [_code(25.0)] * (n // 4) + [_code(2.7)] * (n - 2 * (n // 4)),
        "random": [_code(e) for e in rng.choice([2.5, 3.9, 7.0, 25.0], size=n)],
    }


def _expected_cdf(wts):
    wts = np.abs(np.asarray(wts, dtype=np.float64))
    cum = np.cumsum(wts) / wts.sum()
    return np.minimum(np.ceil(cum * 4294967296.0), 4294967295.0)


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hop_tables_match_exact_solve(mw, oracle_lib, n, axis):
    for name, codes in _profiles(n).items():
        g = mw.mw_sgf_table(codes, axis, kind=0)
        P = oracle_lib.hop_table(codes, axis)
        want = _expected_cdf(P)
        diff = np.abs(g["cdf"].astype(np.float64) - want)
        print(n, axis, name, "max CDF step difference", diff.max())
        assert diff.max() <= 1.0, (name, int(np.argmax(diff)))
        assert g["cdf"][-1] == 0xffffffff


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("axis,normal", [(2, 2), (2, 0), (0, 1), (1, 1)])
def test_first_transition_tables_match_exact_solve(mw, oracle_lib, n, axis, normal):
    for name, codes in _profiles(n).items():
        g = mw.mw_sgf_table(codes, axis, kind=1, normal_axis=normal)
        Pc, Pp, Pm, Gp, Gm = oracle_lib.first_table(codes, axis, normal)
        w = 0.5 * (Gp * (Pc - Pp) + Gm * (Pm - Pc))
        K = np.abs(w).sum()
        want = _expected_cdf(w)
        diff = np.abs(g["cdf"].astype(np.float64) - want)
        print(n, axis, normal, name, "max CDF step difference", diff.max(), "K h", g["kh"], K)
        assert diff.max() <= 1.0, (name, int(np.argmax(diff)))
        big = np.abs(w) > 1e-9 * K
        assert np.array_equal(g["sign"][big], (w > 0)[big])
        assert abs(g["kh"] - K) <= 1e-6 * K
        # the kernel sums to zero: the flux of a potential that is zero on
        # the boundary (each exit distribution sums to one)
        assert abs(w.sum()) < 1e-9 * K


def test_table_arguments_are_checked(mw):
    with pytest.raises(mw.MWError) as e:
        mw.mw_sgf_table([_code(3.9)] * 7, 2)
    assert e.value.status == mw.MW_EINVAL
    with pytest.raises(mw.MWError) as e:
        mw.mw_sgf_table([_code(3.9)] * 8, 3)
    assert e.value.status == mw.MW_EINVAL
    with pytest.raises(mw.MWError) as e:
        mw.mw_sgf_table([1] * 8, 2)
    assert e.value.status == mw.MW_EINVAL
