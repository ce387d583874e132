"""Do the oracle's pins catch plausible mistakes?  Each case plants one
mistake in a temporary copy of oracle/oracle.c -- a wrong constant, sign,
index or stream, a dropped term, a transposed operand, an off-by-one --
builds it, and runs the pins of tests/test_oracle_pins.py against it in a
child process: at least one pin must fail.  The oracle itself is never
modified, and an unmutated copy must pass every pin.  CPU only.

Run as a script (python tests/test_oracle_mutants.py LIB ROCRAND_EXE), the
module runs the pins against the oracle library LIB and exits 1 at the
first pin that fails, 0 if none does."""
import itertools
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_SRC = os.path.join(ROOT, "oracle", "oracle.c")
ORACLE_HDR = os.path.join(ROOT, "oracle", "oracle.h")

# (name, text in oracle.c, replacement); each text must occur exactly once
MUTANTS = [
    ("philox multiplier", "#define PHILOX_M0 0xD2511F53u", "#define PHILOX_M0 0xD2511F55u"),
    ("philox weyl constant", "#define PHILOX_W1 0xBB67AE85u", "#define PHILOX_W1 0xBB67AE86u"),
    ("philox transposed product", "uint32_t n0 = hi1 ^ x1 ^ k0;", "uint32_t n0 = hi0 ^ x1 ^ k0;"),
    ("philox nine rounds", "for (round = 0; round < 10; round++)", "for (round = 0; round < 9; round++)"),
    ("philox key bump skipped", "if (round < 9) {", "if (round < 8) {"),
    ("accept counter t and colour swapped", "    ctr[2] = t;\n    ctr[3] = (uint32_t)color;",
     "    ctr[2] = (uint32_t)color;\n    ctr[3] = t;"),
    ("accept block index", "uint64_t block = k >> 2;", "uint64_t block = k >> 1;"),
    ("accept output word", "return out[k & 3];", "return out[(k + 1) & 3];"),
    ("proposal stream", "ctr[3] = (uint32_t)(2 + color);", "ctr[3] = (uint32_t)(1 + color);"),
    ("proposal bit index", "return (int)((out[(k >> 5) & 3] >> (k & 31)) & 1u);",
     "return (int)((out[(k >> 5) & 3] >> ((k + 1) & 31)) & 1u);"),
    ("initial draw stream", "    ctr[2] = 0;\n    ctr[3] = 4;", "    ctr[2] = 0;\n    ctr[3] = 5;"),
    ("lut bit probability", "double p = exp(-4.0 * beta);", "double p = exp(-8.0 * beta);"),
    ("lut pattern probabilities swapped", "prob *= ((k >> j) & 1) ? p : (1.0 - p);",
     "prob *= ((k >> j) & 1) ? (1.0 - p) : p;"),
    ("lut search strict", "if (T[k] <= (uint64_t)u) best = k;", "if (T[k] < (uint64_t)u) best = k;"),
    ("lut stream", "ctr[3] = (uint32_t)(8 + 2 * color + e);", "ctr[3] = (uint32_t)(8 + color + e);"),
    ("threshold rounded", "return (uint32_t)floor(scaled);", "return (uint32_t)floor(scaled + 0.5);"),
    ("threshold sign of exponent", "double p = exp(-beta * dE);", "double p = exp(beta * dE);"),
    ("ising always-flip bound",
     "if (aligned <= 2) {\n            flip = 1;\n        } else {\n            uint32_t u",
     "if (aligned <= 1) {\n            flip = 1;\n        } else {\n            uint32_t u"),
    ("ising thresholds swapped", "flip = (u < (aligned == 3 ? tb->T4 : tb->T8));",
     "flip = (u < (aligned == 3 ? tb->T8 : tb->T4));"),
    ("lut always-flip bound",
     "if (aligned <= 2) {\n            flip = 1;\n        } else {\n            uint64_t g",
     "if (aligned <= 1) {\n            flip = 1;\n        } else {\n            uint64_t g"),
    ("lut bit of the group", "            int j = (int)(k & 3);\n            int exp4",
     "            int j = (int)((k + 1) & 3);\n            int exp4"),
    ("lut exp8 without exp4", "flip = exp8 & exp4;", "flip = exp8;"),
    ("lut three-aligned rule", "                flip = exp4;\n", "                flip = 1 - exp4;\n"),
    ("bc proposal", "return ((idx + 1 + b) % 3) - 1;", "return ((idx + b) % 3) - 1;"),
    ("bc field sign", "return (double)(-h * (s2 - s)) + D * (double)(s2 * s2 - s * s);",
     "return (double)(h * (s2 - s)) + D * (double)(s2 * s2 - s * s);"),
    ("bc crystal field dropped", "return (double)(-h * (s2 - s)) + D * (double)(s2 * s2 - s * s);",
     "return (double)(-h * (s2 - s));"),
    ("bc crystal field linear", "return (double)(-h * (s2 - s)) + D * (double)(s2 * s2 - s * s);",
     "return (double)(-h * (s2 - s)) + D * (double)(s2 - s);"),
    ("neighbour repeated", "nb[3] = at(s, L, x, y - 1);", "nb[3] = at(s, L, x, y + 1);"),
    ("periodic wrap off by one", "    x = ((x % L) + L) % L;", "    x = (((x + 1) % L) + L) % L;"),
    ("colour order", "for (color = 0; color < 2; color++) {\n            int64_t y;",
     "for (color = 1; color >= 0; color--) {\n            int64_t y;"),
    ("sweep index off by one",
     "uint32_t t = (uint32_t)(t0 + it);\n        int color;\n        for (color = 0; color < 2; color++) {\n            int64_t y;",
     "uint32_t t = (uint32_t)(t0 + it + 1);\n        int color;\n        for (color = 0; color < 2; color++) {\n            int64_t y;"),
    ("bond sum term dropped", "b += v * (at(s, L, x + 1, y) + at(s, L, x, y + 1));",
     "b += v * at(s, L, x + 1, y);"),
    ("Q as sum of s", "q += v * v;", "q += v;"),
    ("correlation axes transposed", "sy += v * at(s, L, x, y + d);", "sy += v * at(s, L, x + d, y);"),
    ("sampled sources one axis", "if (sampled && (y % CORR_R) != 0) continue;",
     "if (sampled && (y % 1) != 0) continue;"),
    ("every-source range exclusive", "for (v = 0; v <= half && v <= 2 * CORR_R; v++)",
     "for (v = 0; v <= half && v < 2 * CORR_R; v++)"),
    ("r_c not rounded", "floor(ora_g(L) * sqrt((double)t) + 0.5)", "floor(ora_g(L) * sqrt((double)t))"),
    ("g(L) with log2", "log((double)L / 65536.0)", "log2((double)L / 65536.0)"),
    # (d >= rc instead of d > rc in the log-spaced set is no mistake: a log-spaced
    # d equal to r_c is already the last distance of the linear part)
    ("log-spaced set from 2R", "if (d > rc && d <= half)", "if (d > 2 * CORR_R && d <= half)"),
    ("sigma h histogram sign", "row[v * h + 4]++;", "row[-v * h + 4]++;"),
    # the light-cone window (what the full-size GPU tests compare against)
    ("window ising always-flip bound", "int flip = aligned <= 2;\n                        if (!flip) flip = ora_accept",
     "int flip = aligned <= 1;\n                        if (!flip) flip = ora_accept"),
    ("window neighbour repeated", "nb[3] = patch[(j - 1) * P + i];", "nb[3] = patch[(j + 1) * P + i];"),
    ("window lut exp8 without exp4", "if (aligned == 4 && e4)", "if (aligned == 4)"),
    ("window bc table index", "< tb.thr[sv + 1][b][h + 4];", "< tb.thr[sv + 1][1 - b][h + 4];"),
]

# pins ordered by cost, so that most mutants stop early: the enumerations
# and the Schwinger-Dyson runs (tenths of a second each) after the rest, the
# two that take seconds last
MEDIUM_PINS = ("test_ising_4x4_enumeration", "test_bc_3x3_enumeration", "test_lut_ising_4x4_enumeration",
               "test_schwinger_dyson_identity")
SLOW_PINS = ("test_onsager_yang_at_0p9_tc", "test_bc_4x4_enumeration_energy")


def _cost(name):
    return 2 if name in SLOW_PINS else 1 if name in MEDIUM_PINS else 0


def _pin_calls(rocrand_run):
    """Every pin of test_oracle_pins as (name, call), its parametrize marks
    expanded; the rocRAND fixture is passed in as `rocrand_run`."""
    import inspect

    import test_oracle_pins as pins
    calls = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_") or fn.__module__ != pins.__name__:
            continue
        params = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        grids = []
        for m in params:
            names = [a.strip() for a in (m.args[0].split(",") if isinstance(m.args[0], str) else m.args[0])]
            rows = [v if len(names) > 1 else (v,) for v in m.args[1]]
            grids.append([dict(zip(names, r)) for r in rows])
        for combo in itertools.product(*grids) if grids else [()]:
            kw = {}
            for d in combo:
                kw.update(d)
            if "rocrand_philox" in inspect.signature(fn).parameters:
                kw["rocrand_philox"] = rocrand_run
            calls.append(("%s%s" % (name, sorted(kw.items()) if kw and "rocrand_philox" not in kw else ""),
                          (lambda f=fn, k=kw: f(**k)), fn.__code__.co_firstlineno, _cost(name)))
    calls.sort(key=lambda c: (c[3], c[2]))
    return [(n, f) for n, f, _, _ in calls]


def run_pins(lib_path, rocrand_exe):
    import oracle
    oracle._LIB = lib_path
    oracle._lib = None

    def rocrand_run(rows):
        txt = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
        res = subprocess.run([rocrand_exe], input=txt, capture_output=True, text=True, check=True)
        return [[int(v) for v in line.split()] for line in res.stdout.strip().splitlines()]

    for name, call in _pin_calls(rocrand_run):
        try:
            call()
        except Exception as e:                 # an assertion, or an error the mistake provoked
            print("caught by %s: %s" % (name, type(e).__name__), flush=True)
            return 1
    print("no pin failed", flush=True)
    return 0


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND pin")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-o", out, os.path.join(HERE, "pins", "philox_rocrand.cpp")],
                   check=True, cwd="/tmp", capture_output=True)
    return out


def _run_against(tmp_path, rocrand_exe, source):
    src = tmp_path / "oracle.c"
    src.write_text(source)
    shutil.copy(ORACLE_HDR, tmp_path / "oracle.h")
    lib = str(tmp_path / "liboracle_mutant.so")
    subprocess.run(["gcc", "-std=c99", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", lib, str(src), "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([ROOT, HERE]), OMP_NUM_THREADS="4")
    return subprocess.run([sys.executable, os.path.abspath(__file__), lib, rocrand_exe], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=600)


def test_unmutated_copy_passes_every_pin(tmp_path, rocrand_exe):
    with open(ORACLE_SRC) as f:
        r = _run_against(tmp_path, rocrand_exe, f.read())
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, rocrand_exe, name, old, new):
    with open(ORACLE_SRC) as f:
        text = f.read()
    assert text.count(old) == 1, "mutation site of %r not found once in oracle.c" % name
    r = _run_against(tmp_path, rocrand_exe, text.replace(old, new))
    assert r.returncode == 1, "no pin caught %r:\n%s%s" % (name, r.stdout, r.stderr)


if __name__ == "__main__":
    sys.exit(run_pins(sys.argv[1], sys.argv[2]))
