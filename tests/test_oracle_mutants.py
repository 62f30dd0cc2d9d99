"""The pins are sensitive: plant plausible mistakes in a copy of the oracle's
C source (on the CPU only), build each mutant, and check that the pin tests
of ``test_oracle_pins`` reject every one of them."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "hist_oracle.c")

# (name, original text, mutated text)
MUTANTS = [
    ("lower_bound_instead_of_upper_bound", "if (x < e[mid])", "if (x <= e[mid])"),
    ("overflow_check_off_by_edge", "if (!(x < xmax))", "if (x > xmax)"),
    ("missing_clamp_below_max", "    if (b > nbins)\n        b = nbins;", ""),
    ("nbins_off_by_one", "double u = (double)nbins * t;", "double u = (double)(nbins + 1) * t;"),
    ("dropped_x_in_second_moment", "wx * x[a]); ++k;", "wx); ++k;"),
    ("cross_term_wrong_index", "(w * x[c]) * x[a]", "(w * x[a]) * x[a]"),
    ("sumw2_not_squared", "double ww = w * w;", "double ww = w;"),
    ("stats_include_flow", "        if (!inside)\n            continue;\n        int k = 0;\n        nadd(&h->stats",
     "        int k = 0;\n        nadd(&h->stats"),
    ("global_bin_wrong_stride", "g = g * (int64_t)(axes[a].nbins + 2) + b[a];",
     "g = g * (int64_t)(axes[a + 1 < dims ? a + 1 : a].nbins + 2) + b[a];"),
    ("weight_sign_flip", "double w = weights ? weights[i] : 1.0;\n        int inside = 1;\n        for (int a = 0; a < d; ++a) {\n            x[a]",
     "double w = weights ? -weights[i] : 1.0;\n        int inside = 1;\n        for (int a = 0; a < d; ++a) {\n            x[a]"),
]

PIN_TESTS = [
    lambda: pins.test_variable_matches_bruteforce_tiny(),
    lambda: pins.test_variable_matches_searchsorted_right(),
    lambda: pins.test_variable_special_cases(),
    lambda: pins.test_uniform_dyadic_exact(),
    lambda: pins.test_uniform_midpoints_and_flow(),
    lambda: pins.test_uniform_monotone(),
    lambda: pins.test_global_bin_round_trip(),
    *[(lambda c=c: pins.test_fill_matches_bruteforce_fsum(c)) for c in range(6)],
    lambda: pins.test_fill_invariants_plain_1d(),
    lambda: pins.test_unit_weights_integer_counts(),
    lambda: pins.test_midpoint_closed_form(),
    lambda: pins.test_accumulate_across_fills(),
    lambda: pins.test_stats_layout_3d_cross_terms(),
]


def _build_mutant(src_text: str, tmpdir: str, name: str) -> str:
    c = os.path.join(tmpdir, name + ".c")
    so = os.path.join(tmpdir, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", so, c, "-lm"], check=True)
    return so


def _failures_in_process(lib_path: str) -> int:
    failed = 0
    with oracle.use_library(lib_path):
        for t in PIN_TESTS:
            try:
                t()
            except AssertionError:
                failed += 1
    return failed


def _failures(lib_path: str) -> int:
    """Runs the pins against ``lib_path`` in a child process: a mutant may
    also crash (a NaN bin used as an index), which counts as caught."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from tests.test_oracle_mutants import _failures_in_process\n"
            "print('FAILED', _failures_in_process(%r))\n" % (root, lib_path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300)
    if r.returncode != 0:
        return 1_000_000
    return int(r.stdout.strip().split()[-1])


def test_unmutated_source_passes_every_pin():
    with tempfile.TemporaryDirectory() as td:
        so = _build_mutant(open(SRC).read(), td, "clean")
        assert _failures(so) == 0


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(name, orig, mut):
    text = open(SRC).read()
    assert text.count(orig) == 1, "mutation anchor must match exactly once: " + name
    with tempfile.TemporaryDirectory() as td:
        so = _build_mutant(text.replace(orig, mut), td, name)
        assert _failures(so) > 0, "no pin caught mutant " + name
