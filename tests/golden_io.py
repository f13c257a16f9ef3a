"""Parser for tests/golden/worked_examples.txt (hand-derived exact examples)."""
from __future__ import annotations

import math
import os
import re
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(tok: str) -> Fraction:
    tok = tok.strip()
    return Fraction(tok)


def _matrix(val: str):
    val = val.strip()
    m = re.fullmatch(r"diag\((.*)\)", val)
    if m:
        d = [_num(t) for t in m.group(1).split(",")]
        n = len(d)
        return [[d[i] if i == j else Fraction(0) for j in range(n)] for i in range(n)]
    return [[_num(t) for t in row.split(",")] for row in val.split(";")]


def _vector(val: str):
    return [_num(t) for t in val.split(",")]


def _logval(val: str) -> float:
    m = re.fullmatch(r"log\((.*)\)", val.strip())
    return math.log(float(Fraction(m.group(1))))


def worked_examples():
    cases = {}
    cur = None
    with open(os.path.join(GOLDEN, "worked_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            key = key.strip()
            if key == "case":
                cur = {}
                cases[val.strip()] = cur
            elif key in ("A", "L"):
                cur[key] = _matrix(val)
            elif key in ("b", "x"):
                cur[key] = _vector(val)
            elif key == "logdet":
                cur[key] = _logval(val)
    return cases


def as_float(m) -> np.ndarray:
    return np.array([[float(v) for v in row] for row in m]) if isinstance(m[0], list) \
        else np.array([float(v) for v in m])
