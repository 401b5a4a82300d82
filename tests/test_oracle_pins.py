"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against a fact fixed by the paper or by
mathematics: libm / Python ``math.frexp`` exponents, numpy's direct
float64 -> float16 cast, exact rational arithmetic (``fractions.Fraction``),
``math.fsum``, hand-derived worked examples (``tests/golden``), closed
forms, and the paper's theorems read as inequalities.  No expected value
here comes from the device library.
"""
from __future__ import annotations

import json
import math
import os
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def F(expr: str) -> Fraction:
    """Evaluate an exact expression such as '1 + 2**-6' with Fractions."""
    return eval(expr.replace("2**", "Fraction(2)**"), {"Fraction": Fraction})


def exp_of_fraction(q: Fraction) -> int:
    """floor(log2 |q|) for a nonzero rational, by integer arithmetic."""
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    assert Fraction(2) ** e <= q < Fraction(2) ** (e + 1)
    return e


def py_split(v: float):
    """Exponent / significand via Python's frexp (an independent libm path)."""
    m, e = math.frexp(abs(v))
    return e - 1, m * 2.0


# --------------------------------------------------------------------------
# Building blocks
# --------------------------------------------------------------------------

def test_split_every_exponent_code_and_subnormals():
    vals = []
    for code in range(1, 2047):
        for frac in (0, 1, (1 << 51), (1 << 52) - 1, 0x5555555555555):
            bits = (code << 52) | frac
            vals.append(np.array([bits], dtype=np.uint64).view(np.float64)[0])
    for frac in (1, 2, 3, 0x8000000000000, 0xFFFFFFFFFFFFF, 0x123456789):
        vals.append(np.array([frac], dtype=np.uint64).view(np.float64)[0])
    for v in vals:
        for s in (1.0, -1.0):
            E, m = oracle.split(s * float(v))
            E2, m2 = py_split(s * float(v))
            assert (E, m) == (E2, m2), v
            assert 1.0 <= m < 2.0
            assert Fraction(abs(s * float(v))) == Fraction(m) * Fraction(2) ** E


def test_key_is_exponent_of_product():
    g = workloads.rng(11)
    xs = np.concatenate([
        workloads.log_uniform_pair(3000, 3, -300, 300)[0],
        np.ldexp(g.uniform(1, 2, 500), g.integers(-1074, -1030, 500)),  # subnormal
        1.0 + g.integers(0, 1 << 20, 500) * 2.0 ** -52,                  # near 1
        np.sqrt(2.0) * (1 + g.integers(-64, 64, 500) * 2.0 ** -52),      # m*m ~ 2
    ])
    ys = np.concatenate([
        workloads.log_uniform_pair(3000, 4, -300, 300)[1],
        np.ldexp(g.uniform(1, 2, 500), g.integers(-20, 20, 500)),
        2.0 - g.integers(1, 1 << 20, 500) * 2.0 ** -52,
        np.sqrt(2.0) * (1 + g.integers(-64, 64, 500) * 2.0 ** -52),
    ])
    corner = 0
    for x, y in zip(xs.tolist(), ys.tolist()):
        k = oracle.key(x, y, 0)
        ex = exp_of_fraction(Fraction(x) * Fraction(y))
        # the key is the exponent of the exact product, except where the
        # significand product rounds up to exactly 2 (the key then follows
        # the rounded product, one above)
        if k != ex:
            corner += 1
            assert k == ex + 1
            mx, my = py_split(x)[1], py_split(y)[1]
            assert Fraction(mx) * Fraction(my) < 2 and mx * my == 2.0
        # sum key: E(x) + E(y) from Python's frexp
        assert oracle.key(x, y, 1) == py_split(x)[0] + py_split(y)[0]
    assert corner < 10


def test_key_follows_rounded_product_at_the_carry():
    # Pairs whose significand product is just below 2 but rounds to 2.0: the
    # product key is the IEEE exponent of fl64(x*y), one above the exact one.
    found = 0
    for i in range(1, 4000):
        mx = 1.0 + i * 2.0 ** -12
        my = np.float64(2.0 / mx)
        while Fraction(mx) * Fraction(float(my)) >= 2:
            my = np.nextafter(my, 0.0)
        my = float(my)
        if mx * my != 2.0:
            continue
        found += 1
        for sx, sy, ex, ey in ((1, 1, 0, 0), (-1, 1, 5, -9), (1, -1, -300, 200)):
            x, y = sx * math.ldexp(mx, ex), sy * math.ldexp(my, ey)
            assert oracle.key(x, y, 0) == py_split(x * y)[0] == ex + ey + 1
            assert exp_of_fraction(Fraction(x) * Fraction(y)) == ex + ey
    assert found > 10
    # in general, for normal products the key is the exponent of fl64(x*y)
    x, y = workloads.log_uniform_pair(5000, 12, -100, 100)
    for a, b in zip(x.tolist(), y.tolist()):
        assert oracle.key(a, b, 0) == py_split(a * b)[0]


def test_r16_matches_numpy_float16_cast():
    g = workloads.rng(5)
    base = np.arange(1 << 10, dtype=np.float64)
    ms = [1.0 + base * 2.0 ** -10]                          # representable
    ms.append(1.0 + (base + 0.5) * 2.0 ** -10)              # exact ties
    ms.append(1.0 + (base + 0.5) * 2.0 ** -10 + 2.0 ** -40)  # tie + sticky
    ms.append(1.0 + (base + 0.5) * 2.0 ** -10 - 2.0 ** -52)  # just below tie
    ms.append(1.0 + g.integers(0, 1 << 52, 200000) * 2.0 ** -52)
    ms.append(np.array([2.0 - 2.0 ** -52, 2.0 - 2.0 ** -12, 2.0 - 2.0 ** -11]))
    m = np.concatenate(ms)
    m = m[(m >= 1.0) & (m < 2.0)]
    want = m.astype(np.float16).astype(np.float64) * 1024.0
    got = np.array([oracle.r16(v) for v in m.tolist()])
    np.testing.assert_array_equal(got, want)
    assert oracle.r16(1.0 + 2.0 ** -11) == 1024.0                  # tie -> even
    assert oracle.r16(1.0 + 2.0 ** -11 + 2.0 ** -40) == 1025.0     # above tie


def test_t_exact_against_fractions():
    g = workloads.rng(6)
    cases = [(1, 1e-6), (4, 1e-6), (268, 1e-6), (269, 1e-6), (262, 1e-3),
             (263, 1e-3), (343, 1e-8), (344, 1e-8), (219, 1e-10), (220, 1e-10),
             (209, 1e-4), (210, 1e-4), (1, 5e-324), (4196, 5e-324),
             (3, 2.2250738585072014e-308), (7, 1.7976931348623157e308),
             (1, 1.0), (2, 1.0), (3, 1e3)]
    for _ in range(3000):
        cases.append((int(g.integers(1, 4197)),
                      float(10.0 ** g.uniform(-320, 308))))
    for nb, eps in cases:
        if eps == 0.0:
            continue
        t = oracle.t_of(nb, eps)
        e = Fraction(eps)
        assert nb * Fraction(2) ** t <= e < nb * Fraction(2) ** (t + 1), (nb, eps)


def test_ceil_log2():
    for m in list(range(1, 5000)) + [2 ** 27, 2 ** 27 + 1, 2 ** 40 - 1]:
        assert oracle.ceil_log2(m) == (m - 1).bit_length()


def _min_precision(sigma: int, spare_bits: int) -> int:
    """Lowest precision whose per-bin budget holds (proof of Thm 3.5):
    2^(sigma + t) * eps(pi) <= 2^(t - spare_bits), i.e. sigma + spare <= m_pi,
    searched over perforate (m = 0), half (10), single (23), double (52)."""
    for cls, m in ((oracle.PERF, 0), (oracle.HALF, 10), (oracle.SINGLE, 23),
                   (oracle.DOUBLE, 52)):
        if sigma + spare_bits <= m:
            return cls
    return oracle.DOUBLE  # no precision meets it: stays at input precision


def test_precision_is_the_lowest_one_meeting_the_budget():
    # non-strict reading = lowest precision meeting the budget exactly;
    # strict (printed half-open intervals) = lowest one with a spare bit
    for sigma in range(-40, 80):
        assert oracle.precision(sigma, 1) == _min_precision(sigma, 0), sigma
        assert oracle.precision(sigma, 0) == _min_precision(sigma, 1), sigma


def test_tree64_pairs_adjacent_leaves():
    v = np.zeros(64, dtype=np.float32)
    v[0], v[2], v[3] = 1.0, 2.0 ** -24, 2.0 ** -24
    assert oracle.tree64(v) == 1.0 + 2.0 ** -23      # (1+0) + (2^-24+2^-24)
    v = np.zeros(64, dtype=np.float32)
    v[0], v[1], v[3] = 1.0, 2.0 ** -24, 2.0 ** -24
    assert oracle.tree64(v) == 1.0                   # 1+2^-24 ties to 1, twice
    v = np.zeros(64, dtype=np.float32)
    v[0], v[32], v[33] = 1.0, 2.0 ** -24, 2.0 ** -24
    assert oracle.tree64(v) == 1.0 + 2.0 ** -23      # halves meet at level 6
    v = np.full(64, 3.0, dtype=np.float32)
    assert oracle.tree64(v) == 192.0


def test_exact_sum_matches_fsum_and_fractions():
    g = workloads.rng(7)
    for trial in range(200):
        n = int(g.integers(1, 60))
        v = np.ldexp(g.uniform(-1, 1, n), g.integers(-80, 80, n))
        if trial % 3 == 0:  # heavy cancellation
            v = np.concatenate([v, -v[: n // 2] * (1 + 2.0 ** -52)])
        assert oracle.sum_exact(v) == math.fsum(v.tolist())
        q = sum((Fraction(a) for a in v.tolist()), Fraction(0))
        assert abs(Fraction(oracle.sum_exact(v)) - q) <= abs(
            Fraction(math.fsum(v.tolist())) - q)
    # halfway cases resolved by smaller partials
    assert oracle.sum_exact([1e16, 1.0, 1e-16]) == 1e16 + 2.0
    assert oracle.sum_exact([2.0 ** 53, 1.0, -2.0 ** -60]) == 2.0 ** 53
    assert oracle.sum_exact([]) == 0.0


def test_dot_exact_against_fractions():
    for seed in range(20):
        x, y = workloads.log_uniform_pair(50, 100 + seed, -30, 30)
        q = sum((Fraction(a) * Fraction(b) for a, b in zip(x.tolist(), y.tolist())),
                Fraction(0))
        d = oracle.dot_exact(x, y)
        # correctly rounded: no double is closer
        lo, hi = np.nextafter(d, -np.inf), np.nextafter(d, np.inf)
        assert abs(Fraction(d) - q) <= abs(Fraction(float(lo)) - q)
        assert abs(Fraction(d) - q) <= abs(Fraction(float(hi)) - q)
        qa = sum((abs(Fraction(a) * Fraction(b)) for a, b in zip(x.tolist(), y.tolist())),
                 Fraction(0))
        assert oracle.abs_dot(x, y) == float(qa)  # Fraction -> float rounds to nearest


def test_dot2_within_its_published_bound():
    # Dot2 (Ogita-Rump-Oishi): |dot2 - x.y| <= u |x.y| + gamma_n^2 sum|x_i y_i|,
    # u = 2^-53, gamma_n = n u / (1 - n u); checked against Fractions, also on
    # sums with heavy cancellation, where a plain FP64 dot fails the bound
    u = Fraction(1, 2 ** 53)
    g = workloads.rng(9)
    worst_plain_fails = False
    for trial in range(40):
        n = int(g.integers(2, 400))
        x, y = workloads.log_uniform_pair(n, 200 + trial, -8, 8)
        if trial % 2:
            x = np.concatenate([x, -x])
            y = np.concatenate([y, y * (1 + 2.0 ** -40)])
            n = len(x)
        q = sum((Fraction(a) * Fraction(b) for a, b in zip(x.tolist(), y.tolist())), Fraction(0))
        qa = sum((abs(Fraction(a) * Fraction(b)) for a, b in zip(x.tolist(), y.tolist())),
                 Fraction(0))
        gam = n * u / (1 - n * u)
        bound = u * abs(q) + gam * gam * qa
        assert abs(Fraction(oracle.dot_dot2(x, y)) - q) <= bound, trial
        plain = Fraction(float(np.dot(x, y)))
        worst_plain_fails |= abs(plain - q) > bound
    assert worst_plain_fails  # the cases are hard enough to tell the two apart
    assert oracle.dot_dot2(np.zeros(0), np.zeros(0)) == 0.0


def test_thm34_helper_matches_the_definition():
    x, y = workloads.log_uniform_pair(20000, 43)
    r = oracle.qdot(x, y, 1e-6)
    exact = oracle.dot_exact(x, y)
    b = oracle.bound_thm34(r, exact)
    E = exp_of_fraction(Fraction(exact))
    assert b["hyp"] == (r["e_max"] <= E)
    assert Fraction(b["bound_thm3_rel"]) == Fraction(r["bound_rel"]) * Fraction(2) ** (r["e_max"] - E)
    err = abs(Fraction(r["value"]) - Fraction(exact)) / abs(Fraction(exact))
    assert err <= Fraction(b["bound_thm3_rel"]) * (1 + Fraction(1, 2 ** 20))


# --------------------------------------------------------------------------
# Hand-derived worked examples
# --------------------------------------------------------------------------

def _golden_inputs(case):
    if "x" in case:
        x = np.array([float.fromhex(s) for s in case["x"]])
        y = np.array([float.fromhex(s) for s in case["y"]])
        return x, y, float(case["tol"])
    if "ones" in case:
        n = case["ones"]
        return np.ones(n), np.ones(n), float(case["tol"])
    n = 4160
    x = np.zeros(n)
    y = np.ones(n)
    x[0] = 1.0
    x[64:4158] = 2.0 ** -24
    if case["name"] == "tile_tree_rounds":
        x[1] = x[3] = 2.0 ** -24
    else:
        x[2] = x[3] = 2.0 ** -24
    return x, y, 2.0 ** -20


@pytest.mark.parametrize("name", [c["name"] for c in json.load(open(GOLDEN))["cases"]])
def test_golden_worked_examples(name):
    case = next(c for c in json.load(open(GOLDEN))["cases"] if c["name"] == name)
    x, y, tol = _golden_inputs(case)
    r = oracle.qdot(x, y, tol, want_classes=True, want_keys=True)
    ex = case["expect"]
    assert r["status"] == oracle.OK
    for k in ("count", "n_bins", "e_max", "e_min", "t", "flags", "n_zero"):
        if k in ex:
            assert r[k] == ex[k], k
    if "keys" in ex:
        assert r["keys"].tolist() == ex["keys"]
    if "classes" in ex:
        assert r["classes"].tolist() == ex["classes"]
    if "value" in ex:
        v = ex["value"]
        want = F(v) if isinstance(v, str) else Fraction(v)
        assert Fraction(r["value"]) == want
    if "bound_rel" in ex:
        assert Fraction(r["bound_rel"]) == F(ex["bound_rel"])
    if "exact" in ex:
        assert Fraction(oracle.dot_exact(x, y)) == F(ex["exact"])
    # the one-pass reading: same classes and counts, value summed exactly
    r1 = oracle.qdot(x, y, tol, opt=[0, 0, 0, 1], want_classes=True)
    for k in ("count", "n_bins", "e_max", "e_min", "t", "flags", "n_zero"):
        assert r1[k] == r[k], k
    assert np.array_equal(r1["classes"], r["classes"])
    v1 = ex["value_s1"]
    assert Fraction(r1["value"]) == (F(v1) if isinstance(v1, str) else Fraction(v1))
    # the guaranteed mode (Thm 3.4), where the example works it out
    if "expect_guard" in case:
        eg = case["expect_guard"]
        rg = oracle.qdot(x, y, tol, opt=[0, 0, 0, 0, 1], want_classes=True)
        assert rg["status"] == oracle.OK
        for k in ("count", "flags", "e_ref", "passes"):
            assert rg[k] == eg[k], k
        assert rg["classes"].tolist() == eg["classes"]
        assert Fraction(rg["value"]) == F(eg["value"])
        assert Fraction(rg["bound_rel"]) == F(eg["bound_rel"])
        lo, hi = (F(v) for v in eg["lower_in"])
        assert lo < Fraction(rg["lower"]) <= hi


# --------------------------------------------------------------------------
# Guaranteed mode (Thm 3.4)
# --------------------------------------------------------------------------
GUARD = [0, 0, 0, 0, 1]


def _exact_fraction(x, y) -> Fraction:
    return sum((Fraction(a) * Fraction(b) for a, b in zip(x.tolist(), y.tolist())), Fraction(0))


_cancelling = workloads.cancelling_pair


def test_guard_lower_bound_never_exceeds_the_exact_dot():
    # L 2^e_max <= |x.y| against exact rational arithmetic: on the paper's
    # law, on random-sign paper distribution B, and on cancelling sums
    cases = []
    for s in range(5):
        cases.append(workloads.log_uniform_pair(300, 100 + s))
        xb, yb = workloads.paper_dist_b(300, 9, 200 + s)
        cases.append((xb * np.random.default_rng(s).choice([-1.0, 1.0], 300), yb))
        cases.append(_cancelling(300, 300 + s, 1e-6))
        cases.append(_cancelling(300, 400 + s, 1e-14))
    reselected = 0
    for x, y in cases:
        ex = abs(_exact_fraction(x, y))
        for tol in (1e-1, 1e-3, 1e-6, 1e-10):
            r = oracle.qdot(x, y, tol, opt=GUARD)
            assert r["status"] == oracle.OK
            assert Fraction(r["lower"]) <= ex, (tol, r["lower"], float(ex))
            reselected += bool(r["flags"] & oracle.F_RESELECTED)
    assert reselected > 0


def test_guard_certified_results_meet_tol():
    # certified: the Thm 3.4 bound taken with the true E meets tol, and the
    # observed relative error is within tol
    certified = 0
    for s in range(6):
        for x, y in (workloads.log_uniform_pair(2000, 500 + s), _cancelling(2000, 600 + s, 1e-6)):
            ex = oracle.dot_exact(x, y)
            for tol in (1e-3, 1e-6, 1e-10):
                r = oracle.qdot(x, y, tol, opt=GUARD)
                if r["flags"] & oracle.F_GUARANTEED:
                    certified += 1
                    assert oracle.bound_thm34(r, ex)["bound_thm3_rel"] <= tol
                    assert abs(r["value"] - ex) <= tol * abs(ex)
    assert certified >= 24


def test_guard_reselects_against_a_certified_exponent():
    # sums cancelling to ~3e-4 of their size at tol 1e-4: the selection
    # against e_max misses tol; L > 0, so the classes are selected again
    # against E_lo = e_max + flexp(L) < e_max, and the result meets tol
    by_elo = 0
    for s in range(12):
        x, y = _cancelling(2000, 700 + s, 3e-4)
        ex = oracle.dot_exact(x, y)
        r0 = oracle.qdot(x, y, 1e-4)
        rg = oracle.qdot(x, y, 1e-4, opt=GUARD)
        assert abs(r0["value"] - ex) > 1e-4 * abs(ex)
        assert rg["flags"] & oracle.F_RESELECTED and rg["flags"] & oracle.F_GUARANTEED
        assert rg["passes"] == 2 and rg["e_ref"] < rg["e_max"]
        assert abs(rg["value"] - ex) <= 1e-4 * abs(ex)
        # E_lo is a certified lower bound of flexp(x.y)
        assert rg["e_ref"] <= math.frexp(abs(ex))[1] - 1
        if rg["e_ref"] > rg["e_min"] - rg["t"] - 22 and not rg["flags"] & oracle.F_UNATTAINABLE:
            by_elo += 1
            # Thm 3.5 against the reference: sum_k M_k 2^(k-e_ref+1) eps(k) <= N_bins 2^t
            assert (math.ldexp(rg["bound_rel"], rg["e_max"] - rg["e_ref"])
                    <= rg["n_bins"] * 2.0 ** rg["t"])
    assert by_elo >= 8


def test_guard_makes_every_bin_double_when_the_sum_may_vanish():
    # sums cancelling to 1e-6 of their size at tol 1e-3: after the first
    # sweep |x.y| is not bounded away from 0 (L <= 0), so the reselection
    # makes every bin double (e_ref = e_min - t - 22) and the result meets tol
    for s in range(5):
        x, y = _cancelling(2000, 720 + s, 1e-6)
        ex = oracle.dot_exact(x, y)
        r0 = oracle.qdot(x, y, 1e-3)
        rg = oracle.qdot(x, y, 1e-3, opt=GUARD)
        assert abs(r0["value"] - ex) > 1e-3 * abs(ex)
        assert rg["e_ref"] == rg["e_min"] - rg["t"] - 22
        assert rg["count"][oracle.DOUBLE] == len(x) - rg["n_zero"]
        assert rg["flags"] & oracle.F_RESELECTED and rg["flags"] & oracle.F_GUARANTEED
        assert abs(rg["value"] - ex) <= 1e-3 * abs(ex)


def test_guard_one_signed_products_certify_in_one_sweep():
    # one sign: |x.y| >= max |x_i y_i| >= 2^e_max (the Thm 3.3 hypothesis),
    # so the first selection is certified and nothing else changes
    for s in range(3):
        x = workloads.normal_vector(3000, 800 + s)
        z = np.abs(workloads.normal_vector(3000, 900 + s)) * np.sign(x)
        for y, tol in ((x, 1e-6), (z, 1e-10), (-z, 1e-3)):
            r0 = oracle.qdot(x, y, tol, want_classes=True)
            rg = oracle.qdot(x, y, tol, opt=GUARD, want_classes=True)
            assert rg["flags"] == r0["flags"] | oracle.F_GUARANTEED
            assert rg["passes"] == 1 and rg["e_ref"] == rg["e_max"]
            assert rg["value"] == r0["value"]
            assert np.array_equal(rg["classes"], r0["classes"])
            assert rg["lower"] >= 2.0 ** rg["e_max"]
    # where the rule decides: x = (1, 0.5), y = (1, 1), tol 4.  N_bins = 2,
    # t = floor(log2 2) = 1; scores 0+0-0-1+1 = 0 (half) and 0-1-0-1+1 = -1
    # (perforate).  The sweep gives S = 1 while the error bound holds the
    # whole perforated 0.5 (a > 1), so |S| - a < 0; one sign lifts L to 1,
    # E_lo = e_max, and bound_rel = 2*2^-10 + 1 <= 4 certifies one sweep
    r = oracle.qdot(np.array([1.0, 0.5]), np.ones(2), 4.0, opt=GUARD, want_classes=True)
    assert r["value"] == 1.0 and r["passes"] == 1 and r["e_ref"] == 0 and r["t"] == 1
    assert r["classes"].tolist() == [oracle.HALF, oracle.PERF]
    assert r["flags"] == oracle.F_GUARANTEED and r["lower"] == 1.0


def test_guard_edge_cases():
    for n in (0, 7):  # nothing to sum: +0 is exact
        r = oracle.qdot(np.zeros(n), np.ones(n), 1e-6, opt=GUARD)
        assert r["status"] == oracle.OK and r["value"] == 0.0
        assert r["flags"] == oracle.F_ALL_PERF | oracle.F_GUARANTEED and r["passes"] == 0
    x = np.array([1.0, -0.5])
    y = np.ones(2)
    assert oracle.qdot(x, y, 1e-6, opt=[1, 0, 0, 0, 1])["status"] == oracle.E_INVAL
    assert oracle.qdot(x, y, 1e-6, opt=[0, 0, 0, 1, 1])["status"] == oracle.E_INVAL
    assert oracle.qdot(np.array([np.inf]), np.ones(1), 1e-6, opt=GUARD)["status"] == oracle.E_NONFINITE
    # tol 100 perforates both products (t = 5: scores -4, -5); mixed signs
    # leave |x.y| unbounded from below, so every bin becomes double
    # (e_ref = e_min - t - 22 = -28) and the exact 0.5 comes back
    r0 = oracle.qdot(x, y, 100.0)
    assert r0["value"] == 0.0 and r0["passes"] == 0 and r0["flags"] & oracle.F_ALL_PERF
    r = oracle.qdot(x, y, 100.0, opt=GUARD, want_classes=True)
    assert r["value"] == 0.5 and r["e_ref"] == -28 and r["passes"] == 1
    assert r["classes"].tolist() == [oracle.DOUBLE, oracle.DOUBLE]
    assert r["flags"] == oracle.F_RESELECTED | oracle.F_GUARANTEED


# --------------------------------------------------------------------------
# Single-precision inputs (mu = m_single in eq. (precision-def))
# --------------------------------------------------------------------------

def test_f32_small_integers_give_the_exact_dot():
    # products and tile sums of small integers are exact in FP32, so at a
    # tolerance that keeps everything the value is the integer dot product;
    # every bin scores >= 23, which has no row when mu = m_single: single
    # and flagged
    g = np.random.default_rng(31)
    for n in (1, 63, 64, 1000, 4097):
        x = g.integers(-50, 51, n).astype(np.float32)
        y = g.integers(-50, 51, n).astype(np.float32)
        r = oracle.qdot_f32(x, y, 1e-30, want_classes=True)
        nz = int(np.count_nonzero(x.astype(np.int64) * y.astype(np.int64)))
        assert r["value"] == float(np.dot(x.astype(np.int64), y.astype(np.int64)))
        assert r["count"] == [0, nz, 0, n - nz]
        if nz:
            assert r["flags"] & oracle.F_UNATTAINABLE


def test_f32_hand_example():
    # x = y = (1, 1, 1, 1), tol 1e-9: one bin (key 0, M = 4), t = floor(log2
    # 1e-9) = -30, score 2 + 0 - 0 + 30 + 1 = 33.  Double inputs: double, no
    # flag (33 < 52).  Single inputs: no double row, so single and
    # unattainable (33 >= 23).  Thm 3.6: 0 <= 30 - 23 (double) and
    # 0 <= 30 - 10 (single).  Both values are 4.
    x = np.ones(4)
    rd = oracle.qdot(x, x, 1e-9, want_classes=True)
    rs = oracle.qdot_f32(x.astype(np.float32), x.astype(np.float32), 1e-9, want_classes=True)
    assert rd["classes"].tolist() == [oracle.DOUBLE] * 4 and rd["flags"] == oracle.F_THM_ALL_DOUBLE
    assert rs["classes"].tolist() == [oracle.SINGLE] * 4
    assert rs["flags"] == oracle.F_UNATTAINABLE | oracle.F_THM_ALL_DOUBLE
    assert rd["t"] == rs["t"] == -30 and rd["value"] == rs["value"] == 4.0
    # bound: 4 * 2^1 * 2^-23 with eps(single)
    assert Fraction(rs["bound_rel"]) == Fraction(8, 2 ** 23)


def test_f32_is_the_double_selection_capped_at_single():
    # floats are exact doubles: keys, histogram, t and scores are those of
    # the double path; only the double class becomes single, and where the
    # double path keeps no double bin the two results are identical
    for s, tol in ((41, 1e-3), (42, 1e-6), (43, 1e-12)):
        x, y = workloads.log_uniform_pair(6000, s, -15.0, 15.0)
        xf, yf = x.astype(np.float32), y.astype(np.float32)
        rs = oracle.qdot_f32(xf, yf, tol, want_classes=True, want_hist=True, want_keys=True)
        rd = oracle.qdot(xf.astype(np.float64), yf.astype(np.float64), tol,
                         want_classes=True, want_hist=True, want_keys=True)
        assert np.array_equal(rs["keys"], rd["keys"]) and np.array_equal(rs["hist"], rd["hist"])
        capped = np.where(rd["classes"] == oracle.DOUBLE, oracle.SINGLE, rd["classes"])
        assert np.array_equal(rs["classes"], capped)
        assert rs["t"] == rd["t"] and rs["e_max"] == rd["e_max"]
        if rd["count"][oracle.DOUBLE] == 0:
            assert rs["value"] == rd["value"] and rs["count"] == rd["count"]


def test_f32_bound_on_positive_data():
    # one-signed products: Thm 3.3 holds, error against exact rationals
    for s, tol in ((44, 1e-3), (45, 1e-6), (46, 1e-9)):
        xa, ya = workloads.paper_dist_b(3000, 13, s)
        xf, yf = xa.astype(np.float32), ya.astype(np.float32)
        r = oracle.qdot_f32(xf, yf, tol)
        ex = _exact_fraction(xf.astype(np.float64), yf.astype(np.float64))
        assert abs(Fraction(r["value"]) - ex) <= Fraction(r["bound_rel"]) * abs(ex)
        # Thm 3.5 when every bin met its share.  With N_bins ~ 60, tol 1e-6
        # gives t = -26 and the top bin scores >= 27 >= m_single: single
        # inputs cannot meet it (flagged); tol 1e-3 (t = -16) can
        if tol == 1e-3:
            assert not r["flags"] & oracle.F_UNATTAINABLE and r["bound_rel"] <= tol
        else:
            assert r["flags"] & oracle.F_UNATTAINABLE


def test_f32_one_pass_small_integers_and_shared_classes():
    # the one-pass reading on float inputs: classes and counts of the
    # two-pass reading, kept leaves summed exactly; small-integer products
    # make both exact, and the sum of exactly representable leaves is exact
    g = np.random.default_rng(33)
    x = g.integers(-50, 51, 5000).astype(np.float32)
    y = g.integers(-50, 51, 5000).astype(np.float32)
    r1 = oracle.qdot_f32(x, y, 1e-30, opt=[0, 0, 0, 1])
    assert r1["value"] == float(np.dot(x.astype(np.int64), y.astype(np.int64)))
    xl, yl = workloads.log_uniform_pair(8000, 34, -15.0, 15.0)
    xl, yl = xl.astype(np.float32), yl.astype(np.float32)
    for tol in (1e-2, 1e-5):
        r2 = oracle.qdot_f32(xl, yl, tol, want_classes=True)
        r1 = oracle.qdot_f32(xl, yl, tol, opt=[0, 0, 0, 1], want_classes=True)
        assert np.array_equal(r1["classes"], r2["classes"]) and r1["count"] == r2["count"]
        # S1 = the exactly rounded sum of the same leaves: from the classes,
        # single leaves fl32(x y), half leaves r16 r16 (exact), summed in
        # rationals
        tot = Fraction(0)
        for xi, yi, c in zip(xl.tolist(), yl.tolist(), r1["classes"].tolist()):
            if c == oracle.SINGLE:
                tot += Fraction(float(np.float32(xi) * np.float32(yi)))
            elif c == oracle.HALF:
                mx, ex = math.frexp(abs(xi))
                my, ey = math.frexp(abs(yi))
                hx = float(np.float16(2 * mx)) * 2.0 ** (ex - 1)
                hy = float(np.float16(2 * my)) * 2.0 ** (ey - 1)
                sgn = 1 if (xi < 0) == (yi < 0) else -1
                tot += sgn * Fraction(hx) * Fraction(hy)
        assert Fraction(r1["value"]) == Fraction(float(tot))


def test_f32_guaranteed_mode_hand_example():
    # x = (1.5, -1.5, 2^-10), y = 1, tol 2^-5, as floats.  The first sweep is
    # the double inputs' one (half, half, perforate: value 0, L < 0).  The
    # most precise reselection for single inputs puts every bin at >= m_half:
    # e_ref = e_min - t - 9 = -10 + 6 - 9 = -13, scores 1+0+13+6+1 = 21 and
    # 0-10+13+6+1 = 10, both single.  The FP32 leaves 1.5, -1.5, 2^-10 and
    # their tile sum are exact: value 2^-10.  a is about 2^-19, so L is just
    # below 2^-10, E_lo = -11, and bound_rel 2^11 = (4 + 2^-9) 2^-23 2^11
    # <= 2^-5: certified after two sweeps.
    x = np.array([1.5, -1.5, 2.0 ** -10], dtype=np.float32)
    r = oracle.qdot_f32(x, np.ones(3, dtype=np.float32), 2.0 ** -5, opt=GUARD,
                        want_classes=True)
    assert r["value"] == 2.0 ** -10 and r["e_ref"] == -13 and r["passes"] == 2
    assert r["classes"].tolist() == [oracle.SINGLE] * 3
    assert r["flags"] == oracle.F_RESELECTED | oracle.F_GUARANTEED
    assert Fraction(r["bound_rel"]) == (4 + Fraction(1, 2 ** 9)) / 2 ** 23


def _f32_product_sum(x, y) -> Fraction:
    """Exact sum of the float32-rounded products (numpy float32 multiply: one
    IEEE rounding per product, all normal here)."""
    p = (x.astype(np.float32) * y.astype(np.float32)).astype(np.float64)
    return sum((Fraction(v) for v in p.tolist()), Fraction(0))


def test_f32_bins_held_at_input_precision_sum_the_float_products():
    # Single inputs whose bins score at or above m_single cannot be lowered
    # (no double row): each product is formed in FP32 and added at input
    # precision or better.  With every bin held there (tol 1e-300) the value
    # is the correctly rounded sum of the float32 products, even when the
    # products span far more exponents than one FP32 number can hold
    # (10^+-18 -> keys from -120 to 119, and y = 1 keeps every product
    # exact).
    for seed in range(3):
        x, y = workloads.cancelling_wide_f32(4001, 40 + seed)
        r = oracle.qdot_f32(x, y, 1e-300, want_classes=True)
        assert r["status"] == oracle.OK
        assert r["flags"] & oracle.F_UNATTAINABLE
        assert r["count"][oracle.SINGLE] == 4001
        assert set(r["classes"].tolist()) == {oracle.SINGLE}
        assert Fraction(r["value"]) == Fraction(float(_f32_product_sum(x, y)))
        assert r["part"][oracle.SINGLE] == r["value"] and r["part"][oracle.DOUBLE] == 0.0
    # random operands (products rounded in FP32): the same identity
    g = np.random.default_rng(44)
    x = (g.standard_normal(3000) * 10.0 ** g.uniform(-15, 15, 3000)).astype(np.float32)
    y = (g.standard_normal(3000) * 10.0 ** g.uniform(-15, 15, 3000)).astype(np.float32)
    r = oracle.qdot_f32(x, y, 1e-300)
    assert Fraction(r["value"]) == Fraction(float(_f32_product_sum(x, y)))


def test_f32_guaranteed_mode_on_wide_cancelling_sums():
    # Products spanning 10^+-18 with random signs, cancelling to ~1e-3 of
    # the largest: the first selection holds the top bins at single (no
    # double row) and perforates most others; the sum is not bounded away
    # from 0, so the reselection puts every bin at single or above.  The
    # result is finite, within the rigorous bound, its lower bound never
    # exceeds |x.y| (Fractions), and a certified result meets tol.
    for seed in range(4):
        x, y = workloads.cancelling_wide_f32(4001, 50 + seed)
        ex = _f32_product_sum(x, y)  # y = 1: the float products are exact
        for tol in (1e-3, 1e-6, 1e-10):
            r = oracle.qdot_f32(x, y, tol, opt=GUARD)
            assert r["status"] == oracle.OK and math.isfinite(r["value"]), (seed, tol)
            assert r["flags"] & oracle.F_RESELECTED
            assert abs(Fraction(r["value"]) - ex) <= Fraction(r["bound_rig"])
            assert Fraction(r["lower"]) <= abs(ex)
            if r["flags"] & oracle.F_GUARANTEED:
                assert abs(Fraction(r["value"]) - ex) <= Fraction(tol) * abs(ex)


def test_f32_edges():
    # float subnormals are exact doubles: key of 2^-140 * 1 is -140
    x = np.array([2.0 ** -140, 1.0], dtype=np.float32)
    y = np.array([1.0, 0.0], dtype=np.float32)
    r = oracle.qdot_f32(x, y, 1e-3, want_keys=True)
    assert r["keys"][0] == -140 and r["n_zero"] == 1 and r["value"] == 2.0 ** -140
    x[1] = np.inf
    assert oracle.qdot_f32(x, y, 1e-3)["status"] == oracle.E_NONFINITE


# --------------------------------------------------------------------------
# Binning strategies of Sec. 3.2: ranged and variable-width bins
# --------------------------------------------------------------------------

def _ranged(w):
    return [0, 0, 0, 0, 0, 1, w]


def _variable(s):
    return [0, 0, 0, 0, 0, 2, s]


def test_ranged_and_variable_bins_reduce_to_exact_binning():
    # ranged bins of width 1 are the exact bins; enough splits of the
    # variable-width partition (e_max - e_min) end in singletons too
    for seed in range(3):
        x, y = workloads.log_uniform_pair(5000, 60 + seed)
        x[::53] = 0.0
        for tol in (1e-3, 1e-6, 1e-10):
            e = oracle.qdot(x, y, tol, want_classes=True)
            span = e["e_max"] - e["e_min"]
            for opt in (_ranged(1), _variable(span), _variable(span + 7)):
                r = oracle.qdot(x, y, tol, opt=opt, want_classes=True)
                for k in ("count", "n_bins", "t", "flags", "value", "bound_rel", "bound_rig"):
                    assert r[k] == e[k], (opt, k)
                assert np.array_equal(r["classes"], e["classes"])


def test_binning_worked_example():
    # x = y = (1, 2^-3, 2^-9, 2^-15), tol 1e-6: keys 0, -6, -18, -30, e_max 0,
    # e_min -30 (the exact bins give double, single, half, perforate).
    x = np.array([1.0, 2.0 ** -3, 2.0 ** -9, 2.0 ** -15])
    exact = Fraction(1) + Fraction(2) ** -6 + Fraction(2) ** -18 + Fraction(2) ** -30
    D, S, H, P = oracle.DOUBLE, oracle.SINGLE, oracle.HALF, oracle.PERF
    # Ranged, w = 8: u_k = -30 + 8k - 1 -> (-31,-23] {-30}, (-23,-15] {-18},
    # (-15,-7] empty, (-7,1] {-6, 0}: N_bins 3, t = -22 (2^-22 <= 1e-6/3 <
    # 2^-21).  Scores 1 + 1 - 0 + 22 + 1 = 25 (double), 0 - 15 + 23 = 8
    # (half), 0 - 23 + 23 = 0 (half): nothing perforated, the value is exact.
    r = oracle.qdot(x, x, 1e-6, opt=_ranged(8), want_classes=True)
    assert r["n_bins"] == 3 and r["t"] == -22
    assert r["classes"].tolist() == [D, D, H, H]
    assert Fraction(r["value"]) == exact
    assert Fraction(r["bound_rel"]) == (2 * Fraction(2) ** 2 * Fraction(2) ** -52
                                        + Fraction(2) ** -14 * Fraction(2) ** -10
                                        + Fraction(2) ** -22 * Fraction(2) ** -10)
    # Variable width from (-31, 0]: no split -> one bin, M 4, u 0, N_bins 1,
    # t = -20, score 2 + 0 + 20 + 1 = 23: all double.
    r = oracle.qdot(x, x, 1e-6, opt=_variable(0), want_classes=True)
    assert r["n_bins"] == 1 and r["t"] == -20 and r["classes"].tolist() == [D] * 4
    # one split at m = -31 + 16 = -15: (-31,-15] {-18,-30}, (-15,0] {0,-6};
    # N_bins 2, t = -21; scores 1 + 0 + 21 + 1 = 23 (double), 1 - 15 + 22 = 8
    # (half)
    r = oracle.qdot(x, x, 1e-6, opt=_variable(1), want_classes=True)
    assert r["n_bins"] == 2 and r["t"] == -21 and r["classes"].tolist() == [D, D, H, H]
    # second split: (-15,0] has the larger term (2 * 2^0): (-15,-7] empty and
    # (-7,0]; third: (-7,0] -> (-7,-3] {-6} and (-3,0] {0}.  N_bins 3,
    # t = -22; scores 0 + 0 + 23 = 23 (double), 0 - 3 + 23 = 20 (single),
    # 1 - 15 + 23 = 9 (half)
    r2 = oracle.qdot(x, x, 1e-6, opt=_variable(2), want_classes=True)
    assert r2["n_bins"] == 2 and r2["classes"].tolist() == [D, D, H, H]
    r = oracle.qdot(x, x, 1e-6, opt=_variable(3), want_classes=True)
    assert r["n_bins"] == 3 and r["t"] == -22 and r["classes"].tolist() == [D, S, H, H]
    assert Fraction(r["value"]) == exact


def test_binned_selection_meets_the_per_bin_budget_and_the_bound():
    # On random data: keys of one ranged bin share a class; variable-width
    # selections use at most s + 1 bins; every non-capped bin's Thm 3.5 term
    # M_k 2^(u_k - e_max + 1) eps(k) is <= 2^t (checked via bound_rel <=
    # N_bins 2^t, an exact comparison); the error is within the rigorous bound
    for seed in range(3):
        x, y = workloads.log_uniform_pair(4000, 70 + seed)
        ex = _exact_fraction(x, y)
        for tol in (1e-2, 1e-6, 1e-12):
            for opt in (_ranged(2), _ranged(5), _ranged(16), _ranged(64), _variable(0),
                        _variable(2), _variable(9), _variable(40)):
                r = oracle.qdot(x, y, tol, opt=opt, want_classes=True, want_keys=True)
                assert r["status"] == oracle.OK and sum(r["count"]) == len(x)
                if opt[5] == 1:
                    w = opt[6]
                    grp = {}
                    for kk, c in zip(r["keys"].tolist(), r["classes"].tolist()):
                        grp.setdefault((kk - r["e_min"]) // w, set()).add(c)
                    assert all(len(v) == 1 for v in grp.values())
                else:
                    assert r["n_bins"] <= opt[6] + 1
                if not r["flags"] & oracle.F_UNATTAINABLE:
                    assert Fraction(r["bound_rel"]) <= r["n_bins"] * Fraction(2) ** r["t"]
                assert abs(Fraction(r["value"]) - ex) <= Fraction(r["bound_rig"])


def test_binned_selection_options_and_limits():
    x, y = workloads.log_uniform_pair(300, 80)
    for bad in ([0, 0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 3, 1], [0, 0, 0, 1, 0, 1, 4],
                [0, 0, 0, 0, 1, 2, 4], [0, 0, 0, 0, 0, 2, -1]):
        assert oracle.qdot(x, y, 1e-6, opt=bad)["status"] == oracle.E_INVAL, bad
    # single-precision inputs take the binned selection too
    r = oracle.qdot_f32(x.astype(np.float32), y.astype(np.float32), 1e-4, opt=_ranged(3))
    assert r["status"] == oracle.OK and r["count"][oracle.DOUBLE] == 0
    # wide bins may push FP32 leaves below the normal range: still bounded
    xw, yw = workloads.log_uniform_pair(3000, 81, -60.0, 60.0)
    ex = _exact_fraction(xw, yw)
    for opt in (_ranged(300), _variable(1)):
        r = oracle.qdot(xw, yw, 1e-1, opt=opt)
        assert abs(Fraction(r["value"]) - ex) <= Fraction(r["bound_rig"])


# --------------------------------------------------------------------------
# Histogram, partition, invariants
# --------------------------------------------------------------------------

def test_histogram_matches_counter_of_python_keys():
    x, y = workloads.log_uniform_pair(20000, 21)
    x[::97] = 0.0
    r = oracle.qdot(x, y, 1e-6, want_hist=True, want_keys=True)
    keys = []
    for a, b in zip(x.tolist(), y.tolist()):
        if a == 0.0 or b == 0.0:
            continue
        keys.append(exp_of_fraction(Fraction(a) * Fraction(b)))
    cnt = Counter(keys)
    h = r["hist"]
    for k, c in cnt.items():
        assert h[k - oracle.KMIN] == c
    assert h.sum() == len(keys)
    assert r["n_zero"] == len(x) - len(keys)
    assert r["e_max"] == max(cnt) and r["e_min"] == min(cnt)
    assert r["n_bins"] == len(cnt)
    assert sum(r["count"]) == len(x)


def _per_bin_budget_ok(r, hist):
    """Every bin without the unattainable flag spends at most 2^t of the
    relative budget: M_k 2^(k - e_max + 1) eps(class) <= 2^t (exact)."""
    eps = {oracle.DOUBLE: Fraction(2) ** -52, oracle.SINGLE: Fraction(2) ** -23,
           oracle.HALF: Fraction(2) ** -10, oracle.PERF: Fraction(1)}
    cls_of_key = {}
    for k, c in zip(r["keys"].tolist(), r["classes"].tolist()):
        if k != np.iinfo(np.int32).min:
            cls_of_key.setdefault(k, c)
            assert cls_of_key[k] == c  # one precision per bin
    for k, c in cls_of_key.items():
        M = int(hist[k - oracle.KMIN])
        spent = M * Fraction(2) ** (k - r["e_max"] + 1) * eps[c]
        if not (r["flags"] & oracle.F_UNATTAINABLE):
            assert spent <= Fraction(2) ** r["t"], (k, M, c)
    return cls_of_key


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-10, 1e-16, 1e2])
@pytest.mark.parametrize("law", ["c1", "distA", "distB"])
def test_bounds_and_budget_on_random_data(tol, law):
    if law == "c1":
        x, y = workloads.log_uniform_pair(30000, 31)
    elif law == "distA":
        x, y = workloads.paper_dist_a(30000, 60, 32)
    else:
        x, y = workloads.paper_dist_b(30000, 14, 33)
    r = oracle.qdot(x, y, tol, want_classes=True, want_keys=True, want_hist=True)
    _per_bin_budget_ok(r, r["hist"])
    exact = Fraction(oracle.dot_exact(x, y))  # correctly rounded; the rest is slack
    err = abs(Fraction(r["value"]) - exact)
    # rigorous bound: every rounding counted
    assert err <= Fraction(r["bound_rig"]) + abs(exact) * Fraction(2) ** -52
    # Thm 3.3 / 3.5 when the hypothesis e_max <= flexp(x.y) holds
    E = exp_of_fraction(exact)
    if r["e_max"] <= E and not (r["flags"] & oracle.F_UNATTAINABLE):
        rel = err / abs(exact)
        assert rel <= Fraction(r["bound_rel"]) * (1 + Fraction(1, 2 ** 20))
        assert rel <= Fraction(tol)
    # Thm 3.4 with the exact E always
    if r["e_max"] > E:
        b34 = Fraction(r["bound_rel"]) * Fraction(2) ** (r["e_max"] - E)
        assert err / abs(exact) <= b34 * (1 + Fraction(1, 2 ** 20))


def test_positive_data_satisfies_thm33_hypothesis():
    # all products positive -> e_max <= flexp(x.y) (noted after Thm 3.3)
    x, y = workloads.paper_dist_b(20000, 10, 41)
    r = oracle.qdot(x, y, 1e-8)
    E = exp_of_fraction(Fraction(oracle.dot_exact(x, y)))
    assert r["e_max"] <= E


def test_thm36_early_termination_means_all_double():
    for seed in range(6):
        x, y = workloads.log_uniform_pair(5000, 50 + seed, -1, 1)
        for tol in (1e-16, 1e-14, 1e-12, 1e-9):
            r = oracle.qdot(x, y, tol)
            if r["flags"] & oracle.F_THM_ALL_DOUBLE:
                assert r["count"][oracle.DOUBLE] == len(x)
    r = oracle.qdot(*workloads.log_uniform_pair(5000, 57, -1, 1), 1e-16)
    assert r["flags"] & oracle.F_THM_ALL_DOUBLE


def test_invariants_scaling_sign_swap():
    x, y = workloads.log_uniform_pair(9000, 61)
    r0 = oracle.qdot(x, y, 1e-6, want_classes=True)
    r1 = oracle.qdot(x * 2.0 ** 7, y * 2.0 ** -3, 1e-6, want_classes=True)
    assert np.array_equal(r0["classes"], r1["classes"])
    assert r1["value"] == r0["value"] * 2.0 ** 4
    assert r1["e_max"] == r0["e_max"] + 4
    r2 = oracle.qdot(-x, y, 1e-6, want_classes=True)
    assert r2["value"] == -r0["value"]
    r3 = oracle.qdot(y, x, 1e-6, want_classes=True)
    assert r3["value"] == r0["value"] and np.array_equal(r3["classes"], r0["classes"])
    # permutation: same bins, same classes per component, value moves only by
    # FP32 tile rounding
    p = workloads.rng(3).permutation(len(x))
    r4 = oracle.qdot(x[p], y[p], 1e-6, want_classes=True)
    assert r4["count"] == r0["count"]
    assert np.array_equal(r4["classes"], r0["classes"][p])
    assert abs(r4["value"] - r0["value"]) <= r0["bound_rig"]


def test_raising_tol_never_raises_precision():
    x, y = workloads.log_uniform_pair(8000, 71)
    prev = None
    for tol in [1e-16, 1e-12, 1e-9, 1e-6, 1e-3, 1e-1, 1e1, 1e3]:
        r = oracle.qdot(x, y, tol, want_classes=True)
        if prev is not None:
            assert np.all(r["classes"] >= prev)  # DOUBLE=0 < ... < PERF=3
        prev = r["classes"]


def test_exact_products_all_double_equal_exact_dot():
    # small-integer significands: every product and partial sum exact
    g = workloads.rng(81)
    x = np.ldexp(g.integers(1, 1 << 10, 3000).astype(float), g.integers(-30, 30, 3000))
    y = np.ldexp(g.integers(1, 1 << 10, 3000).astype(float), g.integers(-30, 30, 3000))
    r = oracle.qdot(x, y, 1e-300)
    assert r["count"][oracle.DOUBLE] == 3000
    assert r["value"] == oracle.dot_exact(x, y)


def test_s1_exact_products_all_double_equal_exact_dot():
    g = workloads.rng(82)
    x = np.ldexp(g.integers(1, 1 << 20, 3000).astype(float), g.integers(-40, 40, 3000))
    y = np.ldexp(g.integers(1, 1 << 20, 3000).astype(float), g.integers(-40, 40, 3000))
    y[::3] *= -1.0
    r = oracle.qdot(x, y, 1e-300, opt=[0, 0, 0, 1])
    assert r["count"][oracle.DOUBLE] == 3000
    assert r["value"] == oracle.dot_exact(x, y)


def test_s1_short_significands_sum_kept_products_exactly():
    # with at most 11 significant bits per operand every leaf of every class
    # equals x_i y_i exactly, so the one-pass value is the correctly rounded
    # sum of the kept products (classes taken from the oracle, pinned above)
    g = workloads.rng(83)
    n = 5000
    x = np.ldexp(g.integers(1 << 10, 1 << 11, n).astype(float), g.integers(-60, 20, n))
    y = np.ldexp(g.integers(1 << 10, 1 << 11, n).astype(float), g.integers(-60, 20, n))
    x[g.random(n) < 0.5] *= -1.0
    for tol in (1e-3, 1e-6, 1e-9):
        r = oracle.qdot(x, y, tol, opt=[0, 0, 0, 1], want_classes=True)
        kept = r["classes"] != oracle.PERF
        assert 0 < kept.sum() < n
        exact = sum((Fraction(a) * Fraction(b) for a, b, k in zip(x, y, kept) if k), Fraction(0))
        assert Fraction(r["value"]) == Fraction(float(exact)), tol
        # and the classes mix precisions
        assert len(set(r["classes"][kept].tolist())) >= 2


def test_s1_value_is_permutation_invariant():
    x, y = workloads.log_uniform_pair(30000, 84)
    g = workloads.rng(85)
    a = oracle.qdot(x, y, 1e-6, opt=[0, 0, 0, 1])
    for _ in range(3):
        pm = g.permutation(len(x))
        b = oracle.qdot(x[pm], y[pm], 1e-6, opt=[0, 0, 0, 1])
        assert b["value"] == a["value"] and b["count"] == a["count"]


def test_accum_modes_share_classes():
    x, y = workloads.log_uniform_pair(20000, 91)
    a = oracle.qdot(x, y, 1e-6, opt=[0, 0, 0, 0], want_classes=True)
    b = oracle.qdot(x, y, 1e-6, opt=[0, 0, 0, 1], want_classes=True)
    assert np.array_equal(a["classes"], b["classes"]) and a["count"] == b["count"]
    assert abs(a["value"] - b["value"]) <= a["bound_rig"]


def test_sum_key_and_raw_score_options():
    x, y = workloads.log_uniform_pair(20000, 92)
    ks = oracle.qdot(x, y, 1e-6, opt=[1, 0, 0, 0], want_keys=True)
    for i in range(0, 20000, 37):
        assert ks["keys"][i] == py_split(x[i])[0] + py_split(y[i])[0]
    raw = oracle.qdot(x, y, 1e-6, opt=[0, 1, 0, 0])
    assert raw["t"] == math.floor(math.log2(1e-6))
    adj = oracle.qdot(x, y, 1e-6)
    assert adj["t"] < raw["t"]
    # a larger effective tolerance keeps fewer components at high precision
    assert raw["count"][oracle.PERF] >= adj["count"][oracle.PERF]


# --------------------------------------------------------------------------
# Edge and error cases
# --------------------------------------------------------------------------

def test_edge_cases():
    r = oracle.qdot(np.zeros(0), np.zeros(0), 1e-6)
    assert r["status"] == oracle.OK and r["value"] == 0.0 and r["flags"] & oracle.F_ALL_PERF
    r = oracle.qdot(np.zeros(100), np.ones(100), 1e-6)
    assert r["value"] == 0.0 and r["count"] == [0, 0, 0, 100] and r["n_zero"] == 100
    x = np.ones(10)
    x[3] = np.nan
    assert oracle.qdot(x, np.ones(10), 1e-6)["status"] == oracle.E_NONFINITE
    x[3] = np.inf
    assert oracle.qdot(x, np.ones(10), 1e-6)["status"] == oracle.E_NONFINITE
    for bad in (0.0, -1.0, np.nan, np.inf):
        assert oracle.qdot(np.ones(4), np.ones(4), bad)["status"] == oracle.E_INVAL
    assert oracle.qdot(np.ones(4), np.ones(4), 1e-6, opt=[2, 0, 0, 0])["status"] == oracle.E_INVAL
    # subnormal operands: exact product keys, classes well defined
    sub = np.array([5e-324, 1e-310, -3e-320, 2.5e-308])
    r = oracle.qdot(sub, np.array([1e300, 1e290, 2e300, 1.0]), 1e-12, want_keys=True)
    for i, k in enumerate(r["keys"].tolist()):
        a, b = sub[i], [1e300, 1e290, 2e300, 1.0][i]
        assert k == exp_of_fraction(Fraction(float(a)) * Fraction(b)) or k == \
            exp_of_fraction(Fraction(float(a)) * Fraction(b)) + 1
    # huge tolerance -> everything perforated, value +0
    x, y = workloads.log_uniform_pair(1000, 5)
    r = oracle.qdot(x, y, 1e300)
    assert r["value"] == 0.0 and r["count"][oracle.PERF] == 1000
    # tiny tolerance -> all double
    r = oracle.qdot(x, y, 1e-300)
    assert r["count"][oracle.DOUBLE] == 1000
    # single element, ragged lengths around the tile size
    for n in (1, 63, 64, 65, 127, 129):
        x, y = workloads.log_uniform_pair(n, n)
        r = oracle.qdot(x, y, 1e-6)
        assert sum(r["count"]) == n
        assert abs(r["value"] - oracle.dot_exact(x, y)) <= r["bound_rig"] * (1 + 2 ** -40)


# --------------------------------------------------------------------------
# CG and power method
# --------------------------------------------------------------------------

def test_cg_poisson_converges_within_distinct_eigenvalue_count():
    # 4x4 grid: eigenvalues 4 - 2cos(i pi/5) - 2cos(j pi/5) take at most 10
    # distinct values ((i,j) and (j,i) coincide), so exact-arithmetic CG
    # ends in at most 10 steps.
    rp, col, val = workloads.poisson2d_csr(4)
    b = workloads.normal_vector(16, 1)
    r = oracle.cg(rp, col, val, b, 1e-10, 0.0 + 1e-8, 50, 0)
    assert r["status"] == oracle.OK
    assert r["iters"] <= 11
    assert r["relres_true"] < 1e-9


@pytest.mark.parametrize("m", [16, 32])
def test_cg_qdot_matches_fp64_iteration_count(m):
    rp, col, val = workloads.poisson2d_csr(m)
    b = workloads.normal_vector(m * m, 2)
    a = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 5000, 0)
    q = oracle.cg(rp, col, val, b, 1e-10, 1e-8, 5000, 1, want_trace=True)
    assert a["status"] == oracle.OK and q["status"] == oracle.OK
    assert abs(q["iters"] - a["iters"]) <= 1
    assert q["relres_true"] < 1e-9
    assert len(q["trace"]) == 1 + 2 * q["iters"]


def test_cg_breaks_down_when_everything_is_perforated():
    rp, col, val = workloads.poisson2d_csr(8)
    b = workloads.normal_vector(64, 3)
    r = oracle.cg(rp, col, val, b, 1e-10, 1e300, 100, 1)
    assert r["status"] == oracle.E_BREAKDOWN


def test_power_method_reaches_closed_form_lambda_max():
    m = 4
    rp, col, val = workloads.laplacian3d_csr(m)
    lam_max = 6.0 + 6.0 * math.cos(math.pi / (m + 1))
    x0 = workloads.unit_vector(m ** 3, 9)
    r = oracle.power(rp, col, val, x0, 400, 1e-6, 0)
    assert r["status"] == oracle.OK
    assert abs(r["lambda"] - lam_max) < 1e-9
    q = oracle.power(rp, col, val, x0, 400, 1e-10, 1)
    assert abs(q["lambda"] - lam_max) < 1e-8
    assert np.all(q["trace"] <= lam_max * (1 + 1e-12))


def test_spmv_matches_dense_product():
    rp, col, val = workloads.poisson2d_csr(5)
    A = np.zeros((25, 25))
    for i in range(25):
        for j in range(rp[i], rp[i + 1]):
            A[i, col[j]] = val[j]
    assert np.array_equal(A, A.T)
    np.testing.assert_array_equal(np.diag(A), 4.0)
    x = workloads.normal_vector(25, 4)
    np.testing.assert_allclose(oracle.spmv(rp, col, val, x), A @ x, rtol=0, atol=1e-14)
