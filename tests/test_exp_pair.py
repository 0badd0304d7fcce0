"""exp_pair (the ray trace's cell transmission e = exp(-x) and absorption m = 1 - e,
rt_internal.h) on the CPU: its float64 steps simulated with correctly rounded fma,
against 40-digit exp and expm1, with the constants read from the header; and its
polynomial checked to be the Remez solution the generator prints."""
import math
import os
import re

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1001_3301_amd", "csrc", "rt_internal.h")
ULP = 2.0 ** -52


def _source():
    with open(HEADER) as f:
        s = f.read()
    i = s.index("void exp_pair(")
    return s[i:s.index("\n}\n", i)]


def _poly_lines(src):
    body = src[src.index("// BEGIN expm1 minimax"):src.index("// END expm1 minimax")]
    return [l for l in body.splitlines()[1:] if l.strip()]


def _constants(src):
    get = lambda name: float(re.search(name + r" = ([0-9.e+-]+);", src).group(1))
    coef = [float(re.search(r"([0-9.e+-]+)\)?;$", l.strip()).group(1)) for l in _poly_lines(src)]
    return get("kInvLn2"), get("kLn2Hi"), get("kLn2Lo"), get("kRound"), coef


def _fma(a, b, c):
    return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def _exp_pair(x, inv, hi, lo, rnd, coef):
    """exp_pair's steps in order, each rounded to float64 as the device rounds it."""
    x = min(x, 2000.0)
    t = _fma(x, -inv, rnd)       # rounds -x/ln2 to an integer in one step
    nk = t - rnd
    assert nk == int(nk) and np.float64(t).view(np.int64) & 0xFFFFFFFF == np.int64(int(nk)) & 0xFFFFFFFF
    r = _fma(nk, lo, _fma(nk, hi, x))
    u = -r
    p = coef[0]
    for c in coef[1:]:
        p = _fma(p, u, c)
    p = p * u
    s = math.ldexp(1.0, int(nk))
    return _fma(s, p, s), -_fma(s, p, s - 1.0)


def test_exp_pair_is_within_an_ulp_of_exp_and_expm1():
    mp.mp.dps = 40
    inv, hi, lo, rnd, coef = _constants(_source())
    assert len(coef) == 11 and rnd == 1.5 * 2 ** 52
    rng = np.random.default_rng(12)
    xs = np.concatenate([10 ** rng.uniform(-300, -1, 300), rng.uniform(0, 2, 500),
                         rng.uniform(0, 40, 300), 10 ** rng.uniform(1, 2.85, 200),
                         [0.0, 5e-324, 1e-17, math.log(2) / 2, math.log(2) * 1.5, 1.0, 700.0, 745.0]])
    we = wm = 0.0
    for x in xs:
        e, m = _exp_pair(float(x), inv, hi, lo, rnd, coef)
        E, M = mp.exp(-mp.mpf(x)), -mp.expm1(-mp.mpf(x))
        if M == 0:
            assert m == 0.0 and e == 1.0
            continue
        wm = max(wm, float(abs(mp.mpf(m) / M - 1)) / ULP)
        if E > 1e-300:  # normal range of e
            we = max(we, float(abs(mp.mpf(e) / E - 1)) / ULP)
    assert we < 0.75 and wm < 1.05, (we, wm)
    # large x: e underflows to zero and m is exactly one; x beyond the clamp too
    for x in (1e4, 1e300, float("inf")):
        assert _exp_pair(x, inv, hi, lo, rnd, coef) == (0.0, 1.0)


def test_exp_pair_polynomial_is_the_remez_solution():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "expm1_minimax", os.path.join(ROOT, "paper_1001_3301_amd", "csrc", "expm1_minimax.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    coef, err = gen.remez()
    assert float(err) < 2e-17
    assert [l.strip() for l in gen.horner_lines(coef)] == [l.strip() for l in _poly_lines(_source())]
