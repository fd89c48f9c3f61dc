"""The pins must catch plausible mistakes in the oracle.

Each case copies oracle.c, plants one mistake (a dropped term, a wrong index,
sign or bias, a reversed order, a wrong rounding rule), builds the copy on the
CPU and runs the pin suite against it in a subprocess: the suite must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "int_sum_drops_last_rank": (
        "for (int r = 0; r < P; ++r) acc += (uint32_t)x[r][i];",
        "for (int r = 0; r < P - 1; ++r) acc += (uint32_t)x[r][i];"),
    "int_max_wrong_comparison": (
        "int32_t m = x[0][i];\n    for (int r = 1; r < P; ++r)\n"
        "      if (x[r][i] > m) m = x[r][i];",
        "int32_t m = x[0][i];\n    for (int r = 1; r < P; ++r)\n"
        "      if (x[r][i] < m) m = x[r][i];"),
    "f64_sum_skips_rank0": (
        "for (int r = 0; r < P; ++r) acc += (double)x[r][i];\n    y[i] = acc;"
        "\n  }\n}\n\nvoid orc_sum_f32_f64_omp",
        "for (int r = 1; r < P; ++r) acc += (double)x[r][i];\n    y[i] = acc;"
        "\n  }\n}\n\nvoid orc_sum_f32_f64_omp"),
    "f64_sum_wrong_index": (
        "for (int r = 0; r < P; ++r) acc += (double)x[r][i];\n    y[i] = acc;"
        "\n  }\n}\n\nvoid orc_sum_f32_f64_omp",
        "for (int r = 0; r < P; ++r) acc += (double)x[r][i ^ 1];\n"
        "    y[i] = acc;\n  }\n}\n\nvoid orc_sum_f32_f64_omp"),
    "f32_sum_reversed_order": (
        "float acc = v[0];\n    for (int r = 1; r < P; ++r) acc = acc + v[r];",
        "float acc = v[P - 1];\n    for (int r = P - 2; r >= 0; --r) "
        "acc = acc + v[r];"),
    "twosum_sign_flip": (
        "*e = (a - av) + (b - bv);", "*e = (a - av) - (b - bv);"),
    "sum2_drops_correction": (
        "return isfinite(p) ? p + sigma : p;", "return p;"),
    "bf16_decode_bias": (
        "v = ldexp((double)(128 + f), e - 127 - 7);",
        "v = ldexp((double)(128 + f), e - 128 - 7);"),
    "bf16_encode_ties_away": (
        "if (frac > 0.5 || (frac == 0.5 && fmod(lo, 2.0) != 0.0)) lo += 1.0;",
        "if (frac >= 0.5) lo += 1.0;"),
    "e4m3_decode_bias": (
        "v = ldexp((double)(8 + f), e - 7 - 3);",
        "v = ldexp((double)(8 + f), e - 8 - 3);"),
    "e4m3_no_subnormals": (
        "if (ufp < -6) ufp = -6; /* subnormals: quantum 2^-9 */",
        "if (ufp < -7) ufp = -7;"),
    "e4m3_scale_uses_240": (
        "float s = amax / 448.0f;", "float s = amax / 240.0f;"),
    "e4m3_sum_wrong_block": (
        "acc += orc_e4m3_decode(q[r][i]) * (double)s[r][i / 256];",
        "acc += orc_e4m3_decode(q[r][i]) * (double)s[r][i / 128];"),
    "e4m3_mirror_transposed_scale": (
        "v[r] = (float)orc_e4m3_decode(q[r][i]) * s[r][b];",
        "v[r] = (float)orc_e4m3_decode(q[r][i]) * s[0][b];"),
    "e5m2_decode_bias": (
        "v = ldexp((double)(4 + f), e - 15 - 2);",
        "v = ldexp((double)(4 + f), e - 16 - 2);"),
    "e5m2_no_subnormals": (
        "if (ufp < -14) ufp = -14; /* subnormals: quantum 2^-16 */",
        "if (ufp < -15) ufp = -15;"),
    "e5m2_scale_uses_448": (
        "float s = amax / 57344.0f;", "float s = amax / 448.0f;"),
    "mx_exponent_rounds_down": (
        "while (ldexp(448.0, e) < (double)amax) ++e;",
        "while (ldexp(448.0, e) <= (double)amax) ++e;"),
    "e8m0_bias_128": (
        "return ldexp(1.0, (int)b - 127);", "return ldexp(1.0, (int)b - 128);"),
    "mx_sum_wrong_block": (
        "acc += orc_e4m3_decode(q[r][i]) * orc_e8m0_decode(sb[r][i / 32]);",
        "acc += orc_e4m3_decode(q[r][i]) * orc_e8m0_decode(sb[r][i / 64]);"),
    "mx_pack_multiplies_by_scale": (
        "q[i] = orc_e4m3_encode((double)x[i] / ldexp(1.0, e));",
        "q[i] = orc_e4m3_encode((double)x[i] * ldexp(1.0, e));"),
    "mx_mirror_drops_last_rank_scale": (
        "v[r] = (float)(orc_e4m3_decode(q[r][i]) * orc_e8m0_decode(sb[r][b]));",
        "v[r] = (float)(orc_e4m3_decode(q[r][i]) * orc_e8m0_decode(sb[0][b]));"),
    "bf16_hilo_drops_low_part": (
        "lo[i] = orc_bf16_encode((double)acc - orc_bf16_decode(hi[i]));",
        "lo[i] = orc_bf16_encode(0.0);"),
    "bf16_hilo_low_part_sign": (
        "lo[i] = orc_bf16_encode((double)acc - orc_bf16_decode(hi[i]));",
        "lo[i] = orc_bf16_encode(orc_bf16_decode(hi[i]) - (double)acc);"),
    "max_without_nan_check": (
        "if (isnan(a) || isnan(b)) return NAN;", "/* no NaN check */"),
    "max_keeps_running_value_unless_greater": (
        "if (isnan(a) || isnan(b)) return NAN;\n"
        "  if (a == b) return signbit(a) ? b : a; /* equal values: +0 over -0 */"
        "\n  return a > b ? a : b;",
        "return b > a ? b : a;"),
    "max_signed_zero_keeps_first": (
        "if (a == b) return signbit(a) ? b : a;", "if (a == b) return a;"),
    "max_first_rank_only_compared": (
        "for (int r = 1; r < P; ++r) m = maximum_ieee(m, (double)x[r][i]);",
        "for (int r = 1; r < P - 1; ++r) m = maximum_ieee(m, (double)x[r][i]);"),
    "sum2_corrects_non_finite_sums": (
        "return isfinite(p) ? p + sigma : p;", "return p + sigma;"),
    "bf16_encode_nan_keeps_sign": (
        "if (isnan(v)) return 0x7fc0;",
        "if (isnan(v)) return signbit(v) ? 0xffc0 : 0x7fc0;"),
    "bf16_hilo_low_part_of_infinity": (
        "if (!isfinite(orc_bf16_decode(hi[i]))) {",
        "if (isnan(orc_bf16_decode(hi[i]))) {"),
    "plan_floor_instead_of_ceil": (
        "int64_t psize = (count + nparts - 1) / nparts;",
        "int64_t psize = count / nparts + (count > 0);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as obuild

    old, new = MUTANTS[name]
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, f"mutation site not unique/absent: {name}"
    mut = tmp_path / "oracle_mutant.c"
    mut.write_text(src.replace(old, new))
    lib = str(tmp_path / "liboracle_mutant.so")
    obuild.build(out=lib, src=str(mut))
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
         os.path.join(ROOT, "tests", "test_oracle_pins.py")],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutant {name}:\n{r.stdout}"
