"""Pins of the filter / computed-column oracle (oracle/expr.py) against facts
of the arithmetic, not against a second copy of it: exact Pythagorean
triples, integer identities exact in binary64, operand order of the
non-commutative operations, IEEE special values, the stated meaning of
MIN/MAX/SELECT on NaN and signed zeros, De Morgan's laws, and filters with a
known number of survivors."""
import math

import numpy as np

from oracle import expr as E


def prog(*ops):
    return [(o[0], o[1] if len(o) > 1 else 0, o[2] if len(o) > 2 else 0.0) for o in ops]


def col(c):
    return (E.COL, c)


def const(v):
    return (E.CONST, 0, v)


def test_pythagorean_triples_exact():
    x = np.array([3.0, 5.0, 8.0, 20.0, 0.0, 7.0])
    y = np.array([4.0, 12.0, 15.0, 21.0, 9.0, 24.0])
    r = E.evaluate(prog(col(0), col(0), (E.MUL,), col(1), col(1), (E.MUL,), (E.ADD,), (E.SQRT,)), [x, y])
    assert r.tolist() == [5.0, 13.0, 17.0, 29.0, 9.0, 25.0]


def test_operand_order_of_sub_div_and_comparisons():
    a, b = np.array([5.0]), np.array([3.0])
    ev = lambda op: E.evaluate(prog(col(0), col(1), (op,)), [a, b])[0]
    assert ev(E.SUB) == 2.0
    assert ev(E.DIV) == 5.0 / 3.0
    assert (ev(E.LT), ev(E.LE), ev(E.GT), ev(E.GE), ev(E.EQ), ev(E.NE)) == (0, 0, 1, 1, 0, 1)
    assert ev(E.MIN) == 3.0 and ev(E.MAX) == 5.0


def test_integer_identities_exact():
    rng = np.random.default_rng(1)
    a, b, c = (rng.integers(-2**20, 2**20, 1000).astype(np.float64) for _ in range(3))
    # (a + b) * c - a * c - b * c == 0 exactly: every intermediate is an integer below 2^53
    p = prog(col(0), col(1), (E.ADD,), col(2), (E.MUL,), col(0), col(2), (E.MUL,), (E.SUB,),
             col(1), col(2), (E.MUL,), (E.SUB,))
    assert np.all(E.evaluate(p, [a, b, c]) == 0.0)
    assert np.all(E.evaluate(prog(col(0), (E.NEG,), (E.ABS,)), [a]) == np.abs(a))


def test_ieee_special_values():
    x = np.array([1.0, 0.0, -1.0, 4.0, -4.0])
    d = E.evaluate(prog(const(1.0), col(0), (E.DIV,)), [x])
    assert d[0] == 1.0 and d[1] == math.inf and d[2] == -1.0
    s = E.evaluate(prog(col(0), (E.SQRT,)), [x])
    assert s[3] == 2.0 and math.isnan(s[4]) and s[1] == 0.0
    z = E.evaluate(prog(col(0), col(0), (E.SUB,), col(0), col(0), (E.SUB,), (E.DIV,)), [x])
    assert np.all(np.isnan(z))


def test_min_max_select_follow_their_definitions():
    nan = math.nan
    a = np.array([nan, 1.0, -0.0, 0.0, 2.0])
    b = np.array([1.0, nan, 0.0, -0.0, 2.0])
    mn = E.evaluate(prog(col(0), col(1), (E.MIN,)), [a, b])
    mx = E.evaluate(prog(col(0), col(1), (E.MAX,)), [a, b])
    # MIN = (b < a ? b : a), MAX = (a < b ? b : a): a comparison with NaN is false
    assert math.isnan(mn[0]) and mn[1] == 1.0 and math.isnan(mx[0]) and mx[1] == 1.0
    assert math.copysign(1.0, mn[2]) == -1.0 and math.copysign(1.0, mn[3]) == 1.0
    c = np.array([0.0, -0.0, nan, 1.0, -3.0])
    sel = E.evaluate(prog(col(0), const(10.0), const(20.0), (E.SELECT,)), [c])
    assert sel.tolist() == [20.0, 20.0, 10.0, 10.0, 10.0]


def test_logic_is_boolean_and_de_morgan():
    rng = np.random.default_rng(2)
    a = rng.choice([0.0, -0.0, 1.0, -2.5, math.nan], 500)
    b = rng.choice([0.0, 3.0, math.nan, -0.0], 500)
    lhs = E.evaluate(prog(col(0), col(1), (E.AND,), (E.NOT,)), [a, b])
    rhs = E.evaluate(prog(col(0), (E.NOT,), col(1), (E.NOT,), (E.OR,)), [a, b])
    assert np.array_equal(lhs, rhs)
    assert set(np.unique(lhs).tolist()) <= {0.0, 1.0}
    # NaN is true (nonzero), -0.0 is false
    t = E.evaluate(prog(col(0), (E.NOT,), (E.NOT,)), [np.array([math.nan, -0.0, 0.0, 7.0])])
    assert t.tolist() == [1.0, 0.0, 0.0, 1.0]
    lt = E.evaluate(prog(col(0), col(1), (E.LT,)), [a, b])
    ge = E.evaluate(prog(col(0), col(1), (E.GE,)), [a, b])
    ordered = ~(np.isnan(a) | np.isnan(b))
    assert np.all((lt + ge)[ordered] == 1.0) and np.all((lt + ge)[~ordered] == 0.0)


def test_filter_keeps_the_stated_events():
    x = np.concatenate([np.arange(1, 501, dtype=np.float64), -np.arange(1, 301, dtype=np.float64),
                        [0.0, math.nan]])
    y = x * 2.0
    coords, w = E.apply_define({"filter": prog(col(0), const(0.0), (E.GT,)),
                                "weight": prog(col(1), const(0.5), (E.MUL,))}, [x, y], 1)
    assert len(coords[0]) == 500 and np.array_equal(coords[0], np.arange(1, 501, dtype=np.float64))
    assert np.array_equal(w, coords[0])
    coords, w = E.apply_define(None, [x, y], 2)
    assert w is None and np.array_equal(coords[1], y, equal_nan=True)


def test_program_must_leave_one_value():
    import pytest
    with pytest.raises(ValueError):
        E.evaluate(prog(col(0), col(0)), [np.zeros(3)])
