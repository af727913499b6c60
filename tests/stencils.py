"""Closed-form Q1 stencils read from tests/golden/q1_stencils.txt, applied with
periodic np.roll.  Independent of the oracle (no element loop)."""
import itertools
import os
from fractions import Fraction

import numpy as np

_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "q1_stencils.txt")


def _load():
    out = {}
    for line in open(_GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        name, hp = tok[0], int(tok[1].split("^")[1])
        coef = {tok[i]: float(Fraction(tok[i + 1])) for i in range(2, len(tok), 2)}
        out[name] = (hp, coef)
    return out


STENCILS = _load()
_CLASS2 = {0: "centre", 1: "edge", 2: "corner"}
_CLASS3 = {0: "centre", 1: "face", 2: "edge", 3: "corner"}


def apply(name, u, n, h=1.0):
    """out_i = sum_off coef(off) u_{i+off} on a periodic grid with shape n (x fastest)."""
    hp, coef = STENCILS[name]
    d = len(n)
    U = np.asarray(u, dtype=np.float64).reshape(tuple(reversed(n)))
    out = np.zeros_like(U)
    names = _CLASS2 if d == 2 else _CLASS3
    for off in itertools.product((-1, 0, 1), repeat=d):
        k = sum(1 for o in off if o != 0)
        c = coef.get(names[k], 0.0)
        if c == 0.0:
            continue
        # off is (dx, dy[, dz]); array axes are reversed
        out += c * np.roll(U, shift=tuple(-o for o in reversed(off)), axis=tuple(range(d)))
    return (h ** hp) * out.ravel()
