"""Mutation check of the oracle's pins (CPU): plausible mistakes are planted in
a copy of oracle/gsl_oracle.cpp, the copy is built with g++, and the pin
tests (tests/test_oracle_pins.py) must fail against every mutant.  Takes a
few minutes, so it runs only with GSL_TEST_MUTANTS=1."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gsl_oracle.cpp")

# name: (text in the oracle, planted replacement)
MUTANTS = {
    "self loop votes": ("if (j == i) continue;\n      const int32_t c = C[j];", "const int32_t c = C[j];"),
    "largest label wins ties": ("(s == best_w && c < best)", "(s == best_w && c > best)"),
    "own label wins ties": ("if (best < 0 || s > best_w || (s == best_w && c < best)) {",
                            "if (best < 0 || s > best_w || (s == best_w && (c == C[i] || (best != C[i] && c < best)))) {"),
    "asynchronous reads": ("const int32_t cstar = scan.best_label(i, off, cols, w, C.data());",
                           "const int32_t cstar = scan.best_label(i, off, cols, w, Cn.data());"),
    "strict convergence test": ("(double)dN / (double)n <= tol", "(double)dN / (double)n < tol"),
    "no re-marking": ("for (int64_t e = off[i]; e < off[i + 1]; ++e) next_unprocessed[(size_t)cols[e]] = 1;", ""),
    "split ignores communities": (
        "bfs_visit_for_each(vis, off, cols, i, [&](int64_t j) { return C[j] == c; },\n"
        "                       [&](int64_t j) { Cp[j] = cp; });",
        "bfs_visit_for_each(vis, off, cols, i, [&](int64_t j) { return true; },\n"
        "                       [&](int64_t j) { Cp[j] = cp; });"),
    "sigma counted once": ("if (labels[cols[e]] == c) sigma[(size_t)c] += we;",
                           "if (labels[cols[e]] == c && cols[e] >= i) sigma[(size_t)c] += we;"),
    "weights ignored": ("sum[(size_t)c] += weight_of(w, e);", "sum[(size_t)c] += 1;"),
    "LP without the community test": ("if (C[j] == C[i] && Cp[j] < cmin) cmin = Cp[j];",
                                      "if (Cp[j] < cmin) cmin = Cp[j];"),
    "Alg. 4 off by one": ("if (reached < S[(size_t)c]) D[(size_t)c] = 1;",
                          "if (reached + 1 < S[(size_t)c]) D[(size_t)c] = 1;"),
}

pytestmark = pytest.mark.skipif(os.environ.get("GSL_TEST_MUTANTS") != "1",
                                reason="mutation check runs with GSL_TEST_MUTANTS=1 (a few minutes)")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_the_mutant(name, tmp_path):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert before in src, "the oracle no longer contains the mutated text"
    cpp = tmp_path / "oracle_mutant.cpp"
    lib = tmp_path / "liboracle_mutant.so"
    cpp.write_text(src.replace(before, after))
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-w", str(cpp), "-o", str(lib)])
    env = dict(os.environ, GSL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode != 0, "the pins missed the mutant %r:\n%s" % (name, r.stdout[-2000:])
