"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle source, plants one plausible mistake (a dropped
term, a wrong sign, an off-by-one, a transposed operand, a wrong partition),
builds the copy on the CPU and runs the pin tests against it in a child
process. Every planted mistake has to make at least one pin fail.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "askref.c")

MUTANTS = {
    "dropped_factor_two": ("zi = (zri + zri) + ci;", "zi = zri + ci;"),
    "wrong_sign_real_part": ("zr = (zr2 - zi2) + cr;", "zr = (zr2 + zi2) + cr;"),
    "non_strict_escape": ("if (mag > 4.0)", "if (mag >= 4.0)"),
    "one_iteration_long": ("for (uint32_t k = 1; k <= D; ++k)", "for (uint32_t k = 1; k <= D + 1; ++k)"),
    "count_from_zero": ("for (uint32_t k = 1; k <= D; ++k)", "for (uint32_t k = 0; k <= D; ++k)"),
    "bounded_returns_zero": ("    return D;\n}", "    return 0;\n}"),
    "pixel_corner_not_centre": ("int64_t kx = 2 * (int64_t)px + 1 - (int64_t)W;",
                                "int64_t kx = 2 * (int64_t)px - (int64_t)W;"),
    "axes_pitch_swapped": ("double tx = (double)kx * m[2];", "double tx = (double)kx * m[3];"),
    "rows_flipped": ("*ci = m[1] + ty;", "*ci = m[1] - ty;"),
    "pitch_not_halved": ("m[2] = (x1 - x0) / (2.0 * (double)W);", "m[2] = (x1 - x0) / (double)W;"),
    "ring_wrong_column": ("ring_pixel(c, L, R, R->x + R->w - 1, py,",
                          "ring_pixel(c, L, R, R->x + R->w - 2, py,"),
    "ring_missing_last_row": ("if (py == R->y || py == R->y + R->h - 1) {", "if (py == R->y) {"),
    "uniform_test_wrong": ("} else if (d != *first) {", "} else if (d < *first) {"),
    "leaf_rule_or": ("if (R->w <= c->B && R->h <= c->B) {", "if (R->w <= c->B || R->h <= c->B) {"),
    "ceil_partition": ("return a + (uint32_t)(((uint64_t)j * len) / parts);",
                       "return a + (uint32_t)(((uint64_t)j * len + parts - 1) / parts);"),
    "fill_misses_last_row": (
        "        for (uint32_t py = R->y; py < R->y + R->h; ++py)\n"
        "            for (uint32_t px = R->x; px < R->x + R->w; ++px)\n"
        "                c->out[(uint64_t)py * c->W + px] = v;",
        "        for (uint32_t py = R->y; py + 1 < R->y + R->h; ++py)\n"
        "            for (uint32_t px = R->x; px < R->x + R->w; ++px)\n"
        "                c->out[(uint64_t)py * c->W + px] = v;"),
    "julia_z0_and_c_swapped": ("return askref_dwell_julia(pr, pi, set->cr, set->ci, D);",
                               "return askref_dwell_julia(set->cr, set->ci, pr, pi, D);"),
    "julia_set_ignored": ("if (set && set->julia)", "if (set && !set->julia)"),
    "ring_new_counts_parent_ring": ("if (R->pw == 0 || !on_ring(R->px, R->py, R->pw, R->ph, px, py))",
                                    "if (R->pw == 0 || on_ring(R->px, R->py, R->pw, R->ph, px, py))"),
    # binary64 operation order: one reassociation in each part of z^2 + c
    "reassoc_real": ("zr = (zr2 - zi2) + cr;", "zr = zr2 - (zi2 - cr);"),
    "reassoc_imag": ("zi = (zri + zri) + ci;", "zi = zri + (zri + ci);"),
    "reassoc_real_c_first": ("zr = (zr2 - zi2) + cr;", "zr = (zr2 + cr) - zi2;"),
    # the real part as a product of sum and difference, a common rewriting
    "factored_real_part": ("zr = (zr2 - zi2) + cr;", "zr = (zr + zi) * (zr - zi) + cr;"),
}

# Builds of the unchanged source with other compiler flags: contraction into
# fused multiply-adds changes the rounding of every iteration.
FLAG_MUTANTS = {
    "contracted_build": ("-ffp-contract=fast", "-mfma"),
}

PIN_TESTS = ["tests/test_oracle_dwell.py", "tests/test_oracle_subdiv.py",
             "tests/test_oracle_julia.py"]


def run_mutant(name, tmpdir):
    text = open(SRC).read()
    extra = ("-Wno-error",)  # a planted mistake may leave a value unused
    if name in FLAG_MUTANTS:
        extra += FLAG_MUTANTS[name]
    else:
        old, new = MUTANTS[name]
        assert text.count(old) == 1, name
        text = text.replace(old, new)
    src = os.path.join(tmpdir, "askref_%s.c" % name)
    with open(src, "w") as f:
        f.write(text)
    lib = oracle_build.build(extra=extra, src=src,
                             out=os.path.join(tmpdir, "libaskref_%s.so" % name))
    env = dict(os.environ, ASKREF_LIB=lib)
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:randomly",
                        "-k", "not brute_force", *PIN_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, p.returncode


def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda n: run_mutant(n, str(tmp_path)),
                              sorted(MUTANTS) + sorted(FLAG_MUTANTS)))
    survived = [name for name, rc in results if rc == 0]
    assert not survived, "pins missed planted mistakes: %s" % survived
