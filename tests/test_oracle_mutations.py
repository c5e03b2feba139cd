"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch every one of them (a crash of the mutant also counts as caught).

Runs on the CPU only: each mutant is compiled with the oracle's own flags
into a temporary directory and the pin suite is run against it in a child
process.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lrbg_oracle.c")

MUTANTS = {
    "dense_ts_dropped_first_term": (
        "for (int l = 0; l < k; ++l)\n                s = s + AT(A, i, l, lda)",
        "for (int l = 1; l < k; ++l)\n                s = s + AT(A, i, l, lda)"),
    "dense_ts_transposed_A": ("AT(A, i, l, lda) * AT(U, l, j, ldu)", "AT(A, l, i, lda) * AT(U, l, j, ldu)"),
    "dense_ts_ignores_ldc": ("AT(C, i, j, ldc) = s;", "C[(size_t)i + (size_t)j * (size_t)m] = s;"),
    "inner_wrong_sign": ("s = s + AT(V1, l, i, ldv)", "s = s - AT(V1, l, i, ldv)"),
    "inner_transposed_U2": ("AT(V1, l, i, ldv) * AT(U2, l, j, ldu)", "AT(V1, l, i, ldv) * AT(U2, j % k, l % n, ldu)"),
    "recomp_core_transposed": ("AT(S, i, l, lds) * AT(V2, j, l, ldv)", "AT(S, l, i, lds) * AT(V2, j, l, ldv)"),
    "recomp_basis_not_transposed": ("AT(S, i, l, lds) * AT(V2, j, l, ldv)", "AT(S, i, l, lds) * AT(V2, l % n, j % k, ldv)"),
    "recomp_dropped_last_term": (
        "for (int l = 0; l < k; ++l)\n                s = s + AT(U1, i, l, ldu)",
        "for (int l = 0; l < k - 1; ++l)\n                s = s + AT(U1, i, l, ldu)"),
    "lr_mult_AX_transposed": ("AT(AX, i, l, ldax)", "AT(AX, l, i, ldax)"),
    "lr_mult_BX_transposed": ("AT(BX, l, j, ldbx)", "AT(BX, j, l, ldbx)"),
    "dot2_no_product_error": ("c = c + (ep + es);", "c = c + es;"),
    "qr_wrong_householder_lead": ("x0 <= 0.0 ? x0 - mu :", "x0 <= 0.0 ? x0 + mu :"),
    "qr_beta_missing_factor_two": ("b = 2.0 * v0 * v0 / (sigma + v0 * v0);", "b = v0 * v0 / (sigma + v0 * v0);"),
    "qr_update_skips_pivot_column": ("for (int c = j; c < n; ++c) {", "for (int c = j + 1; c < n; ++c) {"),
    "qr_q_accumulated_forward": ("for (int j = p - 1; j >= 0; --j)", "for (int j = 0; j < p; ++j)"),
    "qr_no_sign_flip": ("b = x0 >= 0.0 ? 0.0 : 2.0;", "b = 0.0;"),
    "qr_norm_includes_pivot": ("for (int i = j + 1; i < m; ++i)\n            sigma = sigma",
                               "for (int i = j; i < m; ++i)\n            sigma = sigma"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "mut.c"
    csrc.write_text(mutated)
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-fopenmp",
                           "-ffp-contract=off", "-fno-fast-math", str(csrc), "-o", str(lib), "-lm"])
    env = dict(os.environ, LRBG_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout[-2000:]}"
