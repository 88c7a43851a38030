"""Loader for the hand-derived worked examples in ``tests/golden/``.

The expected values are closed-form rational expressions written by hand
(the clamp, abs and max already resolved); they are evaluated here exactly with
``fractions.Fraction`` through a tiny arithmetic-only parser, so no stored
number comes from any implementation under test.
"""

from __future__ import annotations

import ast
import json
import math
import os
from fractions import Fraction
from typing import Dict, List

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _eval(node, env: Dict[str, Fraction]) -> Fraction:
    if isinstance(node, ast.Expression):
        return _eval(node.body, env)
    if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
        return Fraction(node.value) if isinstance(node.value, int) else Fraction(str(node.value))
    if isinstance(node, ast.Name):
        return env[node.id]
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.USub):
        return -_eval(node.operand, env)
    if isinstance(node, ast.BinOp):
        a, b = _eval(node.left, env), _eval(node.right, env)
        if isinstance(node.op, ast.Add):
            return a + b
        if isinstance(node.op, ast.Sub):
            return a - b
        if isinstance(node.op, ast.Mult):
            return a * b
        if isinstance(node.op, ast.Div):
            return a / b
    raise ValueError(f"unsupported expression element {ast.dump(node)}")


def rational(expr: str, env: Dict[str, Fraction] | None = None) -> Fraction:
    return _eval(ast.parse(expr, mode="eval"), env or {})


def _const(text: str, env: Dict[str, Fraction]) -> Fraction:
    if text.startswith("f32:"):
        return Fraction(float(np.float32(float(text[4:]))))
    return rational(text, env)


def _pixel(text: str) -> float:
    return float("nan") if text == "nan" else float(Fraction(text))


def load_hand_cases() -> List[dict]:
    with open(os.path.join(GOLDEN, "hand_tiles.json")) as fh:
        doc = json.load(fh)
    cases = []
    for c in doc["cases"]:
        env: Dict[str, Fraction] = {}
        for key in ("C1", "C2", "C", "D"):       # D may refer to C1
            env[key] = _const(c["const"][key], env)
        N = c["N"]
        x = np.array([_pixel(v) for v in c["x"]], dtype=np.float32).reshape(N, N)
        y = np.array([_pixel(v) for v in c["y"]], dtype=np.float32).reshape(N, N)
        # every pixel and constant must be exactly representable in float32
        for k in ("C1", "C2", "C", "D"):
            assert Fraction(float(np.float32(float(env[k])))) == env[k], (c["name"], k)
        expect = {k: [rational(e, env) for e in v] for k, v in c["expect"].items()}
        cases.append({"name": c["name"], "N": N, "NT": c["NT"], "x": x, "y": y,
                      "const": env, "expect": expect})
    return cases


def rel_err(got: float, want: Fraction) -> float:
    want_f = float(want)
    if want == 0:
        return abs(got)
    return abs(got - want_f) / abs(want_f)
