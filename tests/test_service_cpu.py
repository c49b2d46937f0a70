"""The constraint language of the decision service against Python's own evaluation of the same
expressions (the paper writes launch-parameter constraints in Python syntax): host code only."""
import numpy as np
import pytest

from paper_1911_02373_amd import klr


@pytest.fixture(scope="module")
def lib():
    return klr.load_library()


def _python(expr, N, L):
    env = {"N": N, "n": N, "D0": N, "bx": L[0], "by": L[1], "bz": L[2], "L0": L[0], "L1": L[1], "L2": L[2],
           "L3": L[3], "T": L[0] * L[1] * L[2] * L[3], "min": min, "max": max, "abs": abs}
    try:
        return 1 if eval(expr, {"__builtins__": {}}, env) else 0
    except ZeroDivisionError:
        return 0


FIXED = [
    "bx < N and by < N", "bx * by <= 1024", "bx*by*bz <= 1024 and bx <= N // 4", "not (bx > 256)",
    "T % 64 == 0", "64 <= T <= 512", "bx <= by < 2 * bx", "N / T >= 4.5", "N // T >= 4 or bx == 1",
    "min(bx, by) >= 8", "max(bx, by, bz) < 512", "abs(bx - by) <= 32", "bx ** 2 <= N", "2 ** 10 >= T",
    "-bx < -8", "N % bx == 0", "(bx + by) * 2 > 64 and not by == 1", "True", "False or bx == 32",
    "N // (by - 32) > 3", "N / (bx - bx) > 0", "1 < 2 < 3 > 2", "bx != by != bz", "-2 ** 2 == -4",
    "2 ** -1 == 0.5", "N >= 1e6", "L3 == 1 and T == bx * by * bz", "7 // -2 == -4 and 7 % -3 == -2",
]


@pytest.mark.parametrize("expr", FIXED)
def test_fixed_expressions_match_python(lib, expr):
    rng = np.random.default_rng(abs(hash(expr)) % (1 << 32))
    for _ in range(200):
        N = int(rng.integers(1, 1 << 24))
        L = [int(1 << rng.integers(0, 11)), int(rng.integers(1, 129)), int(rng.integers(1, 5)), 1]
        assert klr.constraint_check(lib, expr, N, L[:3]) == _python(expr, N, L), (expr, N, L)


def _rand_expr(rng, depth=0):
    if depth > 3 or rng.random() < 0.25:
        return str(rng.choice(["N", "bx", "by", "bz", "T", str(int(rng.integers(0, 300))), "2", "64"]))
    k = rng.integers(0, 8)
    a, b = _rand_expr(rng, depth + 1), _rand_expr(rng, depth + 1)
    if k == 0:
        return f"({a} {rng.choice(['+', '-', '*'])} {b})"
    if k == 1:
        return f"({a} {rng.choice(['//', '%', '/'])} {b})"
    if k == 2:
        return f"({a} {rng.choice(['<', '<=', '>', '>=', '==', '!='])} {b})"
    if k == 3:
        return f"({a} {rng.choice(['and', 'or'])} {b})"
    if k == 4:
        return f"(not {a})"
    if k == 5:
        return f"{rng.choice(['min', 'max'])}({a}, {b})"
    if k == 6:
        return f"(-{a})"
    return f"({a} < {b} <= {_rand_expr(rng, depth + 1)})"


def test_random_expressions_match_python(lib):
    rng = np.random.default_rng(7)
    for _ in range(6000):
        e = _rand_expr(rng)
        N = int(rng.integers(1, 1 << 20))
        L = [int(1 << rng.integers(0, 11)), int(rng.integers(1, 65)), int(rng.integers(1, 3)), 1]
        assert klr.constraint_check(lib, e, N, L[:3]) == _python(e, N, L), (e, N, L)


@pytest.mark.parametrize("bad", ["bx <", "foo < 3", "(bx < 3", "bx < 3)", "min(bx)", "abs(bx, by)", "", "bx $ 3",
                                 "1+(" * 70 + "1" + ")" * 70])
def test_parse_errors_are_reported(lib, bad):
    with pytest.raises(klr.KlrError):
        klr.constraint_check(lib, bad, 1024, [32, 2])
