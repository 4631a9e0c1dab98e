"""Checks on the oracle itself (CPU only).

1. The pin suite runs against an AddressSanitizer + UndefinedBehaviorSanitizer
   build of oracle.c, so out-of-bounds accesses and undefined arithmetic in
   the oracle fail the suite instead of passing silently.
2. The beam merge once sized its path buffer as W max(K, 2) while level 1
   creates 2K paths (a heap overflow for W = 1, K > 2); that capacity rule is
   planted back into a copy of oracle.c and the sanitizer run must catch it.
3. Planted mistakes: copies of oracle.c with one plausible error each (a
   dropped term, a wrong sign, swapped operands, a stale optimiser moment,
   a wrong tie order or tie group) must each fail the pin suite. This shows that the pins
   fix every part of the oracle the GPU path is compared with.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")


def _gcc(src, out, sanitize=False):
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wno-unused-function"]
    if sanitize:
        cmd += ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    subprocess.check_call(cmd + [src, "-o", out, "-lm"])


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run_pins(lib, sanitize=None, select=None):
    """Run the pin suite on `lib`; with `sanitize` (a log-file prefix) under
    the sanitizer runtimes, whose reports go to files with that prefix (a
    report on stderr would be lost with pytest's captured output when the
    sanitizer ends the process)."""
    env = dict(os.environ, PQ_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    if sanitize:
        env["LD_PRELOAD"] = ":".join([_runtime("libasan.so"), _runtime("libubsan.so")])
        env["ASAN_OPTIONS"] = f"detect_leaks=0:log_path={sanitize}"
        env["UBSAN_OPTIONS"] = f"halt_on_error=1:print_stacktrace=1:log_path={sanitize}"
    cmd = [sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider"]
    if select:
        cmd += ["-k", select]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def _reports(prefix):
    d, base = os.path.split(prefix)
    return "".join(open(os.path.join(d, f)).read() for f in sorted(os.listdir(d)) if f.startswith(base))


def _mutant(tmp, name, old, new, occurrence=0):
    text = open(SRC).read()
    pos = -1
    for _ in range(occurrence + 1):
        pos = text.find(old, pos + 1)
        assert pos >= 0, f"{name}: the text to replace is not in oracle.c"
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as f:
        f.write(text[:pos] + new + text[pos + len(old):])
    return path


needs_sanitizers = pytest.mark.skipif(not (_runtime("libasan.so") and _runtime("libubsan.so")),
                                      reason="gcc sanitizer runtimes not installed")


@needs_sanitizers
def test_pins_pass_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _gcc(SRC, lib, sanitize=True)
    log = str(tmp_path / "san")
    r = _run_pins(lib, sanitize=log)
    assert r.returncode == 0 and not _reports(log), r.stdout[-3000:] + _reports(log)[-3000:]


@needs_sanitizers
def test_sanitizer_run_catches_the_old_beam_capacity(tmp_path):
    src = _mutant(str(tmp_path), "beam_capacity", "if (cap < 2 * (int64_t)K) cap = 2 * (int64_t)K;",
                  "if (K < 2) cap = W * 2;")
    lib = str(tmp_path / "liboracle_beam.so")
    _gcc(src, lib, sanitize=True)
    log = str(tmp_path / "san")
    r = _run_pins(lib, sanitize=log, select="beam")
    assert r.returncode != 0
    assert "heap-buffer-overflow" in _reports(log)


# (name, text in oracle.c, replacement, which occurrence)
MUTANTS = [
    ("adam_update_stale_moment", "m[i] = b1 * m[i] + (1.0 - b1) * grad[i];", "m[i] = (1.0 - b1) * grad[i];", 0),
    ("adam_update_bias_constant", "c2 = 1.0 - pow(b2, (double)t);", "c2 = 1.0 - pow(b1, (double)t);", 1),
    ("adam_update_eps_inside_sqrt", "(sqrt(v[i] / c2) + eps)", "sqrt(v[i] / c2 + eps)", 1),
    ("adam_solve_stale_moment", "m[i] = b1 * m[i] + (1.0 - b1) * g[i];", "m[i] = (1.0 - b1) * g[i];", 0),
    ("adam_solve_bias_step", "c1 = 1.0 - pow(b1, (double)t)", "c1 = 1.0 - pow(b1, (double)(t + 1))", 0),
    ("mixer_sign", "psi[z | bit] = -I * s * a + c * b;", "psi[z | bit] = I * s * a + c * b;", 0),
    ("cost_sign", "psi[z] *= (cos(phi) - I * sin(phi));", "psi[z] *= (cos(phi) + I * sin(phi));", 0),
    ("init_amplitude", "double a = 1.0 / sqrt((double)dim);", "double a = 1.0 / (double)dim;", 0),
    ("expectation_drops_cut", "t[z] = pr * (double)C[z];", "t[z] = pr;", 0),
    ("gradient_factor", "dgamma[l] = 2.0 * acc;", "dgamma[l] = acc;", 0),
    ("gradient_operands_swapped", "acc += cimag(conj(lam[z]) * psi[z ^ bit]);",
     "acc += cimag(conj(psi[z]) * lam[z ^ bit]);", 0),
    ("cut_table_unit_weight", "if (((z >> u[e]) & 1) != ((z >> v[e]) & 1)) c += weight_of(w, e);",
     "if (((z >> u[e]) & 1) != ((z >> v[e]) & 1)) c += 1;", 0),
    ("cutval_unit_weight", "if (x[u[e]] != x[v[e]]) cut += weight_of(w, e);", "if (x[u[e]] != x[v[e]]) cut += 1;", 0),
    ("topk_tie_group_order", "if (a->rep != b->rep) return a->rep < b->rep;",
     "if (a->rep != b->rep) return a->rep > b->rep;", 0),
    ("topk_tie_rank_order", "return a->rank < b->rank;", "return a->rank > b->rank;", 0),
    ("topk_tie_rank_unmixed", "return xs_step((xs_step(x, m) * 2654435761ull) & mask, m);", "return x & mask;", 0),
    ("free_vertex_zero_weight", "if (weight_of(w, e) > 0) busy", "if (weight_of(w, e) >= 0) busy", 0),
    ("merge_orientation_ignored", "int32_t o = (int32_t)((b & 1u) ^ q->x[start[lvl]]);",
     "int32_t o = (int32_t)(b & 1u);", 0),
    ("merge_tie_order", "return a->digits[i] < b->digits[i] ? -1 : 1;",
     "return a->digits[i] > b->digits[i] ? -1 : 1;", 0),
    ("merge_level_cut_sign", "if (x[c->u[e]] != x[c->v[e]]) s += weight_of(c->w, e);",
     "if (x[c->u[e]] == x[c->v[e]]) s += weight_of(c->w, e);", 0),
    ("partition_stride", "start[i] = i * (N - 1);", "start[i] = i * N;", 0),
    ("mlp_relu_derivative", "d1[j] = h1[j] > 0.0 ? a : 0.0;", "d1[j] = a;", 0),
]


def test_pins_reject_planted_mistakes(tmp_path):
    def one(m):
        name, old, new, occ = m
        src = _mutant(str(tmp_path), name, old, new, occ)
        lib = str(tmp_path / f"lib_{name}.so")
        _gcc(src, lib)
        r = _run_pins(lib)
        return name, r.returncode

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(one, MUTANTS))
    survivors = [name for name, rc in results if rc == 0]
    assert not survivors, f"planted mistakes that every pin accepts: {survivors}"
