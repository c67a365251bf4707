"""The lambda pins catch plausible mistakes: each mutant plants one in a copy
of oracle/lambda_sim.py, on the CPU, and at least one pin must fail on it."""
import importlib.util
import inspect
import os

import pytest

import test_lambda_pins as pins
from oracle import lambda_sim

SRC = lambda_sim.__file__

MUTANTS = [
    ("no history-mean term", "C[k] - C[k - H] - (H / n) * C[n]", "C[k] - C[k - H]"),
    ("window one longer", "C[k] - C[k - H] - (H / n) * C[n]", "C[k] - C[k - H - 1] - (H / n) * C[n]"),
    ("normaliser sqrt(H)", ") / math.sqrt(n)", ") / math.sqrt(H)"),
    ("cos in both normals", "r0 * np.sin(2 * np.pi * u[1])", "r0 * np.cos(2 * np.pi * u[1])"),
    ("Box-Muller radius without -2", "r0 = np.sqrt(-2.0 * np.log(u[0]))", "r0 = np.sqrt(-np.log(u[0]))"),
    ("no key bump", "k0, k1 = k0 + W0, k1 + W1", "k0, k1 = k0, k1"),
    ("round words swapped", "c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]",
     "c = [hi0 ^ c[1] ^ k0, lo1, hi1 ^ c[3] ^ k1, lo0]"),
    ("log+ threshold 1", "np.where(t <= math.e, 1.0,", "np.where(t <= 1.0, 1.0,"),
    ("quantile one rank low", "return float(np.sort(S)[quantile_rank(alpha, paths) - 1])",
     "return float(np.sort(S)[quantile_rank(alpha, paths) - 2])"),
]


def pin_cases():
    out = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        if not marks:
            out.append((name, fn, {}))
            continue
        argnames = [a.strip() for a in marks[0].args[0].split(",")]
        for v in marks[0].args[1]:
            out.append((name, fn, dict(zip(argnames, v if isinstance(v, tuple) else (v,)))))
    return out


def load(path, name):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_unmutated_copy_passes_every_pin():
    for name, fn, kw in pin_cases():
        fn(lambda_sim, **kw)


@pytest.mark.parametrize("label,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, label, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old}"
    path = tmp_path / "mut.py"
    path.write_text(src.replace(old, new))
    mod = load(str(path), "lambda_sim_mutant_" + str(abs(hash(label))))
    caught = []
    for name, fn, kw in pin_cases():
        try:
            fn(mod, **kw)
        except (AssertionError, ValueError, IndexError, FloatingPointError):
            caught.append(name)
            break
    assert caught, f"no pin catches the mutant '{label}'"
