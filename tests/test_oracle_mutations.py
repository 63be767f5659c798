"""The oracle's pins must catch plausible mistakes. Each case plants one
mistake in a copy of the oracle source (on the CPU, in a temporary
directory), builds it, and runs the pin suite against it: the suite must
fail. The real oracle is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, original text, mistaken text)
MUTANTS = [
    ("fields in list order", "t->fields[order[j]].offset < t->fields[order[j - 1]].offset", "0"),
    ("separately rounded multiply-add", "x = fma(x, a, b);", "x = x * a + b;"),
    ("separately rounded fp32 multiply-add", "x = fmaf(x, af, bf);", "x = x * af + bf;"),
    ("zero-byte objects share an offset", "end = c->objs[i].off + (c->objs[i].bytes ? c->objs[i].bytes : 1);",
     "end = c->objs[i].off + c->objs[i].bytes;"),
    ("relocated to the offset only", "uint64_t q = base + c->objs[j].off;", "uint64_t q = c->objs[j].off;"),
    ("alignment off by one", "static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }",
     "static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a) / a * a; }"),
    ("count multiplier dropped", "*count = (uint64_t)n * f->count_mult;", "*count = (uint64_t)n;"),
    ("elements after the first ignored", "for (uint64_t e = 0; e < o.count; e++) {", "for (uint64_t e = 0; e < 1; e++) {"),
    ("copy back writes pointers", "if (!in_pointer) dst[byte] = src[byte];", "dst[byte] = src[byte];"),
    ("interior pointers accepted", "if (v[i]->host + extent > v[i + 1]->host) {", "if (0) {"),
    ("alias conflict ignored", "if (s->kind != f->kind || s->type != ptype || s->count != count) return OR_E_CONFLICT;",
     "(void)s;"),
    ("chain index not applied", "elem = index[s];\n  }\n  return OR_E_INVAL;", "elem = 0;\n  }\n  return OR_E_INVAL;"),
]

# Mistakes in the later functions, each with the pin file that must catch it.
MUTANTS_MORE = [
    ("unfollowed member walked", "if (!((c->follow[o.type] >> order[k]) & 1u)) continue;", "(void)0;",
     "test_selective.py"),
    ("unfollowed slot kept", "memset(elem + t->fields[k].offset, 0, 8);\n          continue;",
     "continue;", "test_selective.py"),
    ("scalar chain index not applied", "elem = index[s];\n  }\n  const or_type* t", "elem = 0;\n  }\n  const or_type* t",
     "test_scalar_chain.py"),
    ("scalar offset dropped", "*addr = c->base + cur->off + elem * t->size + offset;",
     "*addr = c->base + cur->off + elem * t->size;", "test_scalar_chain.py"),
    ("drift with the old velocity", "          v = fma(f, dt_over_m, v);\n          x = fma(v, dt, x);",
     "          x = fma(v, dt, x);\n          v = fma(f, dt_over_m, v);", "test_kick_drift.py"),
    ("kick scaled by dt", "v = fma(f, dt_over_m, v);", "v = fma(f, dt, v);", "test_kick_drift.py"),
    ("separately rounded kick", "v = fma(f, dt_over_m, v);", "v = f * dt_over_m + v;", "test_kick_drift.py"),
    ("shared arrays accepted", "        if (used[j]) {\n          rc = OR_E_CONFLICT;",
     "        if (0) {\n          rc = OR_E_CONFLICT;", "test_kick_drift.py"),
]


def _run_pins(tmp_path, orig, mut, pin_file):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor not found: {orig}"
    (tmp_path / "oracle.c").write_text(src.replace(orig, mut))
    shutil.copy(os.path.join(ROOT, "oracle", "oracle.h"), tmp_path / "oracle.h")
    lib = tmp_path / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-w", "-o", str(lib),
                    str(tmp_path / "oracle.c"), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib))
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                           os.path.join(ROOT, "tests", pin_file)],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name,orig,mut,pins", MUTANTS_MORE, ids=[m[0] for m in MUTANTS_MORE])
def test_later_pins_catch_planted_mistake(name, orig, mut, pins, tmp_path):
    r = _run_pins(tmp_path, orig, mut, pins)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, orig, mut, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor not found: {orig}"
    (tmp_path / "oracle.c").write_text(src.replace(orig, mut))
    shutil.copy(os.path.join(ROOT, "oracle", "oracle.h"), tmp_path / "oracle.h")
    lib = tmp_path / "liboracle.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-w", "-o", str(lib),
                    str(tmp_path / "oracle.c"), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
