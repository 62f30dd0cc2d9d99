"""Oracle of the event filters and computed columns (test infrastructure).

The paper's analyses put a Filter and a Define in front of every histogram
fill (arXiv:2401.13310 Sec. 3, Listing 1), and its CUDA kernel skips events
marked invalid (Sec. 3.2).  Here a program is a postfix list of operations
(op, col, value) over binary64 columns, with the meaning include/hist.h gives
each operation; this module evaluates it on whole numpy columns, one
operation at a time, and fills the plain oracle histogram with the events a
filter keeps.  Only tests/, the smoke check and the benchmark's CPU legs use
it; it shares no code with the GPU library.
"""
from __future__ import annotations

import numpy as np

# operation codes of the C ABI (hist_opcode)
COL, CONST, ADD, SUB, MUL, DIV, NEG, ABS, SQRT, MIN, MAX = range(11)
LT, LE, GT, GE, EQ, NE, AND, OR, NOT, SELECT = range(11, 21)


def _truth(b):
    return np.where(b, 1.0, 0.0)


def evaluate(ops, columns) -> np.ndarray:
    """Value of a postfix program on every event (binary64, each operation
    rounded once; numpy's + - * / and sqrt are IEEE correctly rounded)."""
    cols = [np.asarray(c, dtype=np.float64) for c in columns]
    n = len(cols[0]) if cols else 0
    stack = []
    with np.errstate(all="ignore"):
        for op, col, value in ops:
            if op == COL:
                stack.append(cols[col])
            elif op == CONST:
                stack.append(np.full(n, float(value)))
            elif op in (NEG, ABS, SQRT, NOT):
                a = stack.pop()
                stack.append(-a if op == NEG else np.abs(a) if op == ABS else
                             np.sqrt(a) if op == SQRT else _truth(a == 0.0))
            elif op == SELECT:
                b = stack.pop()
                a = stack.pop()
                c = stack.pop()
                stack.append(np.where(c != 0.0, a, b))
            else:
                b = stack.pop()
                a = stack.pop()
                if op == ADD:
                    v = a + b
                elif op == SUB:
                    v = a - b
                elif op == MUL:
                    v = a * b
                elif op == DIV:
                    v = a / b
                elif op == MIN:
                    v = np.where(b < a, b, a)
                elif op == MAX:
                    v = np.where(a < b, b, a)
                elif op == LT:
                    v = _truth(a < b)
                elif op == LE:
                    v = _truth(a <= b)
                elif op == GT:
                    v = _truth(a > b)
                elif op == GE:
                    v = _truth(a >= b)
                elif op == EQ:
                    v = _truth(a == b)
                elif op == NE:
                    v = _truth(a != b)
                elif op == AND:
                    v = _truth((a != 0.0) & (b != 0.0))
                elif op == OR:
                    v = _truth((a != 0.0) | (b != 0.0))
                else:
                    raise ValueError("unknown operation %r" % (op,))
                stack.append(v)
    if len(stack) != 1:
        raise ValueError("program leaves %d values" % len(stack))
    return stack[0]


def apply_define(define, columns, dims):
    """(coords, weights) of the events the filter keeps: define is a dict with
    optional 'filter', 'coords' (per axis) and 'weight' programs; an absent
    coordinate is column a, an absent weight is unit (None)."""
    define = define or {}
    cols = [np.asarray(c, dtype=np.float64) for c in columns]
    n = len(cols[0])
    keep = np.ones(n, dtype=bool)
    if define.get("filter"):
        keep = evaluate(define["filter"], cols) != 0.0
    coords = []
    progs = define.get("coords") or []
    for a in range(dims):
        p = progs[a] if a < len(progs) else None
        coords.append((evaluate(p, cols) if p else cols[a])[keep])
    w = None
    if define.get("weight"):
        w = evaluate(define["weight"], cols)[keep]
    return coords, w
