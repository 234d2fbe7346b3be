"""The table-driven e^{-x} of the integration kernels (Tang's method with 64
table entries), replayed step by step in exact rational arithmetic with one
rounding per device operation, against e^{-x} to 40 digits. The reduction
constants are read from the kernel source, so this checks the constants the
device uses. The device computes its table with the library exp2; here the
table entries are the correctly rounded 2^{-j/64}."""
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
getcontext().prec = 40


def _source_constants():
    src = open(os.path.join(ROOT, "paper_2007_03143_amd", "csrc", "integrate.hip")).read()
    body = src[src.index("__device__ inline double exp_neg(double x)"):]
    body = body[:body.index("\n}\n")]
    c0 = float(re.search(r"rint\(x \* ([0-9.e+-]+)\)", body).group(1))
    c1, c2 = (float(v) for v in re.findall(r"fma\(-nd, ([0-9.e+-]+), [xr]\)", body))
    return c0, c1, c2


def _source_clamp():
    src = open(os.path.join(ROOT, "paper_2007_03143_amd", "csrc", "integrate.hip")).read()
    body = src[src.index("__device__ inline double exp_neg(double x)"):]
    body = body[:body.index("\n}\n")]
    return float(re.search(r"x = fmin\(x, ([0-9.e+-]+)\);", body).group(1))


def _rd(q):
    """Nearest double of a rational (round half to even)."""
    return float(q)


def _fma(a, b, c):
    return _rd(Fraction(a) * Fraction(b) + Fraction(c))


def _table():
    return [_rd(Fraction(Decimal(2) ** (Decimal(-j) / 64))) for j in range(64)]


def _exp_neg(x, c0, c1, c2, tab, clamp=None):
    if clamp is not None:
        x = clamp if (np.isnan(x) or x > clamp) else x     # fmin(x, clamp)
    nd = float(np.rint(_rd(Fraction(x) * Fraction(c0))))
    n = int(nd)
    r = _fma(-nd, c1, x)
    r = _fma(-nd, c2, r)
    p = _fma(r, _rd(Fraction(1, 720)), _rd(Fraction(-1, 120)))
    for c in (Fraction(1, 24), Fraction(-1, 6), Fraction(1, 2), Fraction(-1), Fraction(1)):
        p = _fma(r, p, _rd(c))
    return float(np.ldexp(_rd(Fraction(tab[n & 63]) * Fraction(p)), -(n >> 6)))


def test_reduction_constants():
    c0, c1, c2 = _source_constants()
    ln2 = Decimal(2).ln()
    ln2_d = float(ln2)
    assert c1 == ln2_d / 64                       # exact: division by a power of 2
    assert abs(Decimal(c2) - (ln2 - Decimal(ln2_d)) / 64) < Decimal(c2) * Decimal(2) ** -52
    assert abs(c0 - 64 / ln2_d) < 1e-12


def test_exp_neg_within_two_ulp():
    c0, c1, c2 = _source_constants()
    tab = _table()
    rng = np.random.default_rng(7)
    xs = list(rng.uniform(0.0, 1.0, 300)) + list(rng.uniform(0.0, 50.0, 300)) + \
        list(np.exp(rng.uniform(np.log(1e-12), np.log(700.0), 300))) + \
        [0.0, 1e-300, 1e-16, 0.5 * np.log(2) / 64, np.log(2) / 64, 1.0, 700.0, 708.0]
    worst = 0.0
    for x in xs:
        got = _exp_neg(float(x), c0, c1, c2, tab)
        ref = (-Decimal(float(x))).exp()
        ulp = np.spacing(float(ref))
        err = abs(Decimal(got) - ref) / Decimal(ulp)
        worst = max(worst, float(err))
    assert worst <= 2.0, worst


def test_exp_neg_underflows_to_zero():
    c0, c1, c2 = _source_constants()
    clamp = _source_clamp()
    tab = _table()
    # the clamp itself lies where e^{-x} rounds to zero in FP64
    assert (-Decimal(clamp)).exp() < Decimal(2) ** -1075
    assert _exp_neg(clamp, c0, c1, c2, tab) == 0.0
    assert _exp_neg(750.0, c0, c1, c2, tab, clamp) == 0.0
    assert _exp_neg(0.0, c0, c1, c2, tab, clamp) == 1.0
    # arguments whose integer conversion would overflow without the clamp
    # (a tight exponent far outside its cutoff sphere, +inf, NaN)
    for x in (3e7, 1e300, float("inf"), float("nan")):
        assert _exp_neg(x, c0, c1, c2, tab, clamp) == 0.0
    # below the clamp the clamped and plain replays agree
    for x in (1e-3, 3.0, 700.0, 745.0):
        assert _exp_neg(x, c0, c1, c2, tab, clamp) == _exp_neg(x, c0, c1, c2, tab)
