"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source (on
the CPU), builds it, and runs the pin tests against that copy in a child
process; the pins must fail.  The original oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hoszp_ref.c")
PINS = ["tests/test_oracle_paper.py", "tests/test_oracle_invariants.py",
        "tests/test_oracle_exact.py", "tests/test_oracle_next.py"]

MUTANTS = {
    "eq3_sign": ("double shifted = (double)x[i] + eb;", "double shifted = (double)x[i] - eb;"),
    "eq3_truncate": ("double f = floor(scaled);", "double f = (double)(int64_t)scaled;"),
    "lorenzo_from_outlier": ("(int64_t)q[first + k] - (int64_t)q[first + k - 1]",
                             "(int64_t)q[first + k] - (int64_t)q[first]"),
    "sign_of_zero": ("neg[k] = d[k] < 0 ? 1u : 0u;", "neg[k] = d[k] <= 0 ? 1u : 0u;"),
    "lsb_first_bits": ("buf[p >> 3] |= (uint8_t)(0x80u >> (p & 7u));",
                       "buf[p >> 3] |= (uint8_t)(0x01u << (p & 7u));"),
    "width_off_by_one": ("while (width < 32 && (biggest >> width) != 0) ++width;",
                         "while (width < 32 && (biggest >> width) > 1) ++width;"),
    "mean_divisor": ("*mean = ((double)(int64_t)acc.s / (double)g.n) * two_eb;",
                     "*mean = ((double)(int64_t)acc.s / (double)(g.n + 1)) * two_eb;"),
    "var_drops_square_of_sum": ("(i128)g.n * (i128)acc.q - acc.s * acc.s;", "(i128)g.n * (i128)acc.q;"),
    "mul_floor_not_half_up": ("i128 half = (i128)1 << (sh - 1);", "i128 half = 0;"),
    "add_subtracts": ("dz[i] = da[i] + db[i];", "dz[i] = da[i] - db[i];"),
    "negate_keeps_outlier": ("put_u32(out + g.off_o + 4u * b, 0u - o);",
                             "put_u32(out + g.off_o + 4u * b, o);"),
    "decode_ignores_signs": ("d[k] = get_bit(signs, k) ? -m : m;", "d[k] = m;"),
    "dequantize_scale": ("x[i] = (float)((double)q[i] * two_eb);", "x[i] = (float)((double)q[i] * g.eb);"),
    "scalar_bin_without_eps": ("double sum = s + eb;", "double sum = s;"),
    "scalar_sub_adds": ("return shift_outliers(c, c_bytes, s, -1,", "return shift_outliers(c, c_bytes, s, 1,"),
    "scalar_add_shifts_deltas_too": ("    put_u32(out + g.off_o + 4u * b, (uint32_t)(int32_t)(o + sc.delta));",
                                     "    put_u32(out + g.off_o + 4u * b, (uint32_t)(int32_t)(o + sc.delta));\n"
                                     "    out[g.off_p + (b % (g.payload_bytes + 1))] ^= 1u;"),
    "sub_adds": ("int64_t v = (int64_t)qa[i] - (int64_t)qb[i];", "int64_t v = (int64_t)qa[i] + (int64_t)qb[i];"),
    "std_without_sqrt": ("*std = sqrt(var);", "*std = var;"),
    "hadamard_floor_not_half_up": ("i128 rnd = (i128)1 << (sh - 1);", "i128 rnd = 0;"),
    "hadamard_eps_not_doubled": ("const double two_eb = 2.0 * ga.eb;\n  for", "const double two_eb = ga.eb;\n  for"),
    "cov_drops_product_of_means": ("i128 m = (i128)ga.n * p - sa * sb;", "i128 m = (i128)ga.n * p;"),
    "cov_one_scale": ("((2.0 * ga.eb) * (2.0 * gb.eb))", "((2.0 * ga.eb) * (2.0 * ga.eb))"),
    "block_mean_divides_by_block": ("s->means[b] = ((double)sum / (double)len) * s->two_eb;",
                                    "s->means[b] = ((double)sum / 32.0) * s->two_eb;"),
    "constant_block_miscount": ("if (s->widths[b] == 0) s->constant += 1;",
                                "if (s->widths[b] <= 1) s->constant += 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mut = tmp_path / "hoszp_ref.c"
    mut.write_text(src.replace(old, new))
    hdr = os.path.join(ROOT, "oracle", "hoszp_ref.h")
    (tmp_path / "hoszp_ref.h").write_text(open(hdr).read())
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-fPIC", "-shared", "-ffp-contract=off",
                    str(mut), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, HOSZP_REF_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
