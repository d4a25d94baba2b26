"""Plant plausible mistakes in copies of the oracle (on the CPU) and require the
pins to catch each one.  Shows that the pins are not a retyping of the oracle."""
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "ace_oracle.c")

# (name, original text, mutated text): each is a mistake a reader could make
MUTANTS = [
    ("wrong_w_index", "double prod = xt * (double)wrow[c];",
     "double prod = xt * (double)wrow[(c + 1) % ncols];"),
    ("transposed_bit_table_layout", "const int32_t c = j * K + k;", "const int32_t c = k * L + j;"),
    ("sign_of_zero_is_one", "if (p[c] > 0.0) code |= 1u << k;", "if (p[c] >= 0.0) code |= 1u << k;"),
    ("post_increment_in_running_mean", "S2[j] += 2 * c + 1;", "S2[j] += 2 * c + 3;"),
    ("dropped_square_term", "S2[j] += 2 * c + 1;", "S2[j] += 2 * c;"),
    ("score_reads_wrong_table", "t += counts[j * B + codes[i * L + j]];",
     "t += counts[j * B + codes[i * L + (j + 1) % L]];"),
    ("sigma_missing_m_factor", "const i128 num = (i128)m * (i128)st2 - (i128)sumT * (i128)sumT;",
     "const i128 num = (i128)st2 * (i128)m - (i128)sumT * (i128)sumT / (i128)m;"),
    ("strict_const_threshold", "flags[i] = (uint8_t)(mode == 1 ? (t <= lim) : (t < lim));",
     "flags[i] = (uint8_t)(t < lim);"),
    ("margin_too_small", "return (double)n * u / (1.0 - (double)n * u);", "return u / 1024.0;"),
    ("delete_wrong_sign", "S2[j] -= 2 * c - 1;", "S2[j] -= 2 * c + 1;"),
    ("cube_term_dropped", "s3 += (u128)(3 * c * c + 3 * c + 1);", "s3 += (u128)(3 * c * c + 1);"),
    ("cap_one_too_high", "if (*a >= cap) {", "if (*a > cap) {"),
    ("capped_cube_uses_square", "cube += (u128)(after * after * after - before * before * before);",
     "cube += (u128)(after * after - before * before);"),
    ("zero_vector_pair_never_collides", "p = 0.5;", "p = 0.0;"),
    ("zero_pair_collides_half_the_time", "p = 1.0;", "p = 0.5;"),
    ("mean_divides_by_n_only", "out->mu = n > 0 ? (double)s2tot / ((double)n * (double)L) : 0.0;",
     "out->mu = n > 0 ? (double)s2tot / ((double)n) : 0.0;"),
]


@pytest.fixture(scope="module")
def src_text():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(src_text, name, orig, mut):
    assert src_text.count(orig) >= 1, f"mutation site for {name} not found"
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "m.c")
        so = os.path.join(td, "libm.so")
        with open(c, "w") as f:
            f.write(src_text.replace(orig, mut, 1))
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-o", so, c, "-lm"], check=True)
        failed = []
        with oracle.using_library(so):
            for check in oracle_pins.ALL:
                try:
                    check()
                except AssertionError:
                    failed.append(check.__name__)
        assert failed, f"no pin caught mutant {name}"
