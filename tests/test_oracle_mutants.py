"""The pins catch plausible mistakes: each mutant plants one in a copy of the
oracle's source, on the CPU, and at least one pin of test_oracle_pins must fail
against it.  The oracle itself is never modified."""
import inspect
import os
import shutil

import pytest

import test_oracle_pins as pins
from oracle import oracle as orc_mod

SRC = os.path.join(os.path.dirname(orc_mod.__file__), "bfm_oracle.c")

# (name, original text, mutated text): one plausible mistake each.
MUTANTS = [
    ("window one longer (t-h..t)", "for (int w = u - H + 1; w <= u; ++w)", "for (int w = u - H; w <= u; ++w)"),
    ("residual sign yhat - y", "e[u] = y[tv[u] - 1] - yh;", "e[u] = yh - y[tv[u] - 1];"),
    ("MOSUM normaliser sqrt(h)", "double norm = sig * sqrt((double)nv);", "double norm = sig * sqrt((double)H);"),
    ("sigma denominator n", "sig = sqrt(rss / (double)(nv - p));", "sig = sqrt(rss / (double)nv);"),
    ("log+ threshold 1 instead of e", "return x <= M_E ? 1.0 : log(x);", "return x <= 1.0 ? 1.0 : log(x);"),
    ("log base 10", "return x <= M_E ? 1.0 : log(x);", "return x <= M_E ? 1.0 : log10(x);"),
    ("break index off by one", "if (brk < 0 && fabs(mo) > b) brk = tv[u] - n - 1;",
     "if (brk < 0 && fabs(mo) > b) brk = tv[u] - n;"),
    ("last crossing instead of first", "if (brk < 0 && fabs(mo) > b)", "if (fabs(mo) > b)"),
    ("unsigned magnitude", "mag = hi >= -lo ? hi : lo;", "mag = hi >= -lo ? hi : -lo;"),
    ("boundary at original t/n", "double b = boundary(prm->lambda, (double)(u + 1) / (double)nv);",
     "double b = boundary(prm->lambda, (double)tv[u] / (double)n);"),
    ("window from n, not n_v", "int H = prm->h_window > 0 ? prm->h_window : (int)floor(prm->h_frac * (double)nv);",
     "int H = prm->h_window > 0 ? prm->h_window : (int)floor(prm->h_frac * (double)n);"),
    ("0-based trend column", "x[1] = (double)t;", "x[1] = (double)(t - 1);"),
    ("sin and cos swapped", "x[2 * j] = sin(ang);", "x[2 * j] = cos(ang) + 0.0 * sin(ang);"),
    ("harmonic j+1", "double ang = 2.0 * M_PI * fmod((double)j * (double)t, f) / f;",
     "double ang = 2.0 * M_PI * fmod((double)(j + 1) * (double)t, f) / f;"),
    ("angle not reduced", "double ang = 2.0 * M_PI * fmod((double)j * (double)t, f) / f;",
     "double ang = 2.0 * M_PI * (double)j * (double)t / f;"),
    ("refinement subtracted", "for (int j = 0; j < p; ++j) beta[j] += dbeta[j];",
     "for (int j = 0; j < p; ++j) beta[j] -= dbeta[j];"),
    ("reflection not applied to y", "for (int i = j; i < m; ++i) b[i] -= d * A[i * p + j];",
     "for (int i = j; i < m; ++i) b[i] -= 0.5 * d * A[i * p + j];"),
    ("no rank test", "if (norm <= tol) return -1;", "if (norm <= 0.0) return -1;"),
    ("RSS over the first n_v-1 values", "rss += e[u] * e[u];", "rss += u + 1 < nv ? e[u] * e[u] : 0.0;"),
    ("times ignored", "return prm->times ? prm->times[t - 1] : (double)t;", "return (double)t;"),
    ("times one row late", "return prm->times ? prm->times[t - 1] : (double)t;",
     "return prm->times ? prm->times[t < prm->n_obs ? t : t - 1] : (double)t;"),
    ("no forward fill", "            else y[t] = last;\n", "            else y[t] = y[t];\n"),
    ("gap filled from the next value", "            if (isfinite(y[t])) last = y[t];\n            else y[t] = last;",
     "            if (isfinite(y[t])) last = y[t];\n            else y[t] = t + 1 < N && isfinite(y[t + 1]) ? y[t + 1] : last;"),
    ("all-missing series not flagged", "if (N > 0 && !isfinite(y[0])) st = BFO_INSUFFICIENT;", "if (0) st = BFO_INSUFFICIENT;"),
]


def pin_cases():
    """Every pin test with each of its parameter sets."""
    out = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        if not marks:
            out.append((name, fn, {}))
            continue
        argnames, values = marks[0].args[0], marks[0].args[1]
        argnames = [a.strip() for a in argnames.split(",")]
        for v in values:
            v = v if isinstance(v, (tuple, list)) else (v,)
            out.append((name, fn, dict(zip(argnames, v))))
    return out


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_unmutated_copy_passes_every_pin(workdir):
    lib = orc_mod.build(force=True, src=SRC, out=str(workdir / "ref.so"))
    o = orc_mod.Oracle(lib)
    for name, fn, kw in pin_cases():
        fn(o, **kw)


@pytest.mark.parametrize("label,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(workdir, label, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old}"
    path = workdir / (label.replace(" ", "_").replace("/", "_") + ".c")
    path.write_text(src.replace(old, new))
    lib = orc_mod.build(force=True, src=str(path), out=str(path) + ".so")
    o = orc_mod.Oracle(lib)
    caught = []
    for name, fn, kw in pin_cases():
        try:
            fn(o, **kw)
        except (AssertionError, ValueError, IndexError, ZeroDivisionError, FloatingPointError):
            caught.append(name)
    assert caught, f"no pin catches the mutant '{label}'"
