"""Readers for the hand-derived fixtures under tests/golden/."""
import os
from fractions import Fraction

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def _num(s):
    return float(Fraction(s))


def mixture_trace(name, C):
    """[(x tuple, [(mu tuple, var, w) or None per rank], B, fg)] for each step."""
    out = []
    for line in _rows(name):
        head, ranks, tail = [p.strip() for p in line.split("|")]
        vals = head.split()
        x = tuple(_num(v) for v in vals[1:1 + C])
        comps = []
        for r in ranks.split(";"):
            r = r.strip()
            if r == "-":
                comps.append(None)
            else:
                v = [_num(t) for t in r.split()]
                comps.append((tuple(v[:C]), v[C], v[C + 1]))
        B, fg = (int(t) for t in tail.split())
        out.append((x, comps, B, fg))
    return out


def fusion_traces():
    out = {}
    for line in _rows("fusion_traces.txt"):
        name, ins, states = [p.strip() for p in line.split("|")]
        inputs = [tuple(int(t) for t in s.split()) for s in ins.split(";")]
        st = [tuple(int(t) for t in s.split()) for s in states.split(";")]
        out[name] = (inputs, st)
    return out
