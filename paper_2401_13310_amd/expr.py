"""Postfix programs for the filters and computed columns of ``hist_define``.

``parse("sqrt(x*x + y*y)", ["x", "y", "z"])`` turns an infix expression into
the operation list the C ABI takes (``hist_op`` records); it only rewrites
the text, every value is computed by the kernel.  Grammar, lowest precedence
first: ``||``, ``&&``, comparisons (``< <= > >= == !=``), ``+ -``, ``* /``,
unary ``- !``, then numbers, column names (or ``c0`` .. ``c7``), parentheses
and the functions ``sqrt abs min max select``.
"""
from __future__ import annotations

import re

OPS = {
    "col": 0, "const": 1, "add": 2, "sub": 3, "mul": 4, "div": 5, "neg": 6, "abs": 7,
    "sqrt": 8, "min": 9, "max": 10, "lt": 11, "le": 12, "gt": 13, "ge": 14, "eq": 15,
    "ne": 16, "and": 17, "or": 18, "not": 19, "select": 20,
}

_TOKEN = re.compile(r"\s*(?:(\d+\.?\d*(?:[eE][+-]?\d+)?|\.\d+(?:[eE][+-]?\d+)?)|"
                    r"([A-Za-z_]\w*)|(<=|>=|==|!=|&&|\|\||[-+*/()<>!,]))")
_CMP = {"<": "lt", "<=": "le", ">": "gt", ">=": "ge", "==": "eq", "!=": "ne"}
_FUNCS = {"sqrt": ("sqrt", 1), "abs": ("abs", 1), "min": ("min", 2), "max": ("max", 2),
          "select": ("select", 3)}


def _tokens(text):
    pos, out = 0, []
    text = text.rstrip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise ValueError("cannot read %r at offset %d" % (text, pos))
        num, name, sym = m.groups()
        out.append(("num", float(num)) if num else ("name", name) if name else ("sym", sym))
        pos = m.end()
    return out


def parse(text: str, columns=None) -> list:
    """Postfix operations (op, col, value) for an infix expression."""
    names = {c: i for i, c in enumerate(columns or [])}
    toks = _tokens(text)
    out = []
    i = 0

    def peek():
        return toks[i] if i < len(toks) else (None, None)

    def take(sym=None):
        nonlocal i
        t = peek()
        if sym is not None and t != ("sym", sym):
            raise ValueError("expected %r in %r" % (sym, text))
        i += 1
        return t

    def emit(op, col=0, value=0.0):
        out.append((OPS[op], col, value))

    def primary():
        kind, v = peek()
        if kind == "num":
            take()
            emit("const", value=v)
        elif kind == "name":
            take()
            if v in _FUNCS:
                op, nargs = _FUNCS[v]
                take("(")
                for k in range(nargs):
                    if k:
                        take(",")
                    disjunction()
                take(")")
                emit(op)
            elif v in names:
                emit("col", col=names[v])
            elif re.fullmatch(r"c[0-7]", v):
                emit("col", col=int(v[1]))
            else:
                raise ValueError("unknown name %r in %r" % (v, text))
        elif (kind, v) == ("sym", "("):
            take()
            disjunction()
            take(")")
        else:
            raise ValueError("unexpected %r in %r" % (v, text))

    def unary():
        kind, v = peek()
        if (kind, v) == ("sym", "-"):
            take()
            unary()
            emit("neg")
        elif (kind, v) == ("sym", "!"):
            take()
            unary()
            emit("not")
        else:
            primary()

    def binary(sub, table):
        sub()
        while peek()[0] == "sym" and peek()[1] in table:
            op = table[take()[1]]
            sub()
            emit(op)

    def product():
        binary(unary, {"*": "mul", "/": "div"})

    def total():
        binary(product, {"+": "add", "-": "sub"})

    def comparison():
        total()
        if peek()[0] == "sym" and peek()[1] in _CMP:
            op = _CMP[take()[1]]
            total()
            emit(op)

    def conjunction():
        binary(comparison, {"&&": "and"})

    def disjunction():
        binary(conjunction, {"||": "or"})

    disjunction()
    if i != len(toks):
        raise ValueError("trailing input in %r" % text)
    return out
