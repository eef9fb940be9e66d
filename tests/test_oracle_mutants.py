"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (on the CPU),
builds it, and runs the pin suite against the mutant in a subprocess: the
suite has to fail. This shows that a dropped term, a wrong index, a transposed
operand, a wrong multiplicity or a wrong rounding cannot slip through, in the
three original kernels and in the Bellman-Ford, TTM and partial-symmetry
definitions.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "systec_oracle.cpp")

MUTANTS = {
    "drops_one_permutation": ("    f(p);\n    ++visited;", "    if (visited > 0) f(p);\n    ++visited;"),
    "output_factor_not_left_out": ("if (t != out_slot) prod *= B[p[t] * R + r];",
                                   "prod *= B[p[t] * R + r];"),
    "ssymv_transposed_operand": ("y[p[0]] += a * x[p[1]];", "y[p[0]] += a * x[p[0]];"),
    "wrong_multiplicity_denominator": ("denom *= factorial(run);", "denom *= run;"),
    "unsorted_tuple_not_sorted": ("    std::sort(c, c + n);\n    k->noncanonical += 1;",
                                  "    k->noncanonical += 1;"),
    "diagonal_prescaled": ("      const double a = val[q];\n      int64_t k = for_each_distinct_permutation(c, 2, [&](const int32_t* p) {\n        if (row_mask",
                           "      const double a = c[0] == c[1] ? 0.5 * val[q] : val[q];\n      int64_t k = for_each_distinct_permutation(c, 2, [&](const int32_t* p) {\n        if (row_mask"),
    "syprd_sign": ("acc += term;", "acc -= term;"),
    "bf16_ties_away": ("std::nearbyint(scaled)", "std::round(scaled)"),
    "bf16_truncates": ("std::nearbyint(scaled)", "std::trunc(scaled)"),
    "bellman_ford_transposed_operand": ("a + d[p[1]]", "a + d[p[0]]"),
    "bellman_ford_max_instead_of_min": ("std::min(y[p[0]], a + d[p[1]])",
                                        "std::max(y[p[0]], a + d[p[1]])"),
    "ttm_contracts_an_output_slot": ("const double* b = B + static_cast<int64_t>(p[0]) * R;",
                                     "const double* b = B + static_cast<int64_t>(p[1]) * R;"),
    "partial_permutes_first_part_only": (
        "} while (std::next_permutation(p + start[q], p + start[q] + size[q]));",
        "} while (q == 0 && std::next_permutation(p + start[q], p + start[q] + size[q]));"),
    "partial_one_factor_for_every_part": (
        "prod *= F[(static_cast<int64_t>(part_of[t]) * dim + a[t]) * R + r];",
        "prod *= F[(static_cast<int64_t>(0) * dim + a[t]) * R + r];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutant = tmp_path / "mutant.cpp"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-fopenmp", "-shared", "-o", str(lib),
                           str(mutant)])
    env = dict(os.environ, SYSTEC_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_next_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
