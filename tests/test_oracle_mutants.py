"""Pin strength: plausible mistakes planted in copies of the oracle (on the CPU)
must each fail at least one pin.

Each mutant is the oracle source with one textual edit (a dropped term, a
wrong sign or index, a transposed operand), compiled into a temporary library.
The committed oracle is never modified.
"""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import oracle_pins as pins  # noqa: E402

SRC = os.path.join(os.path.dirname(oracle.__file__), "disc_oracle.c")

# (id, original text, replacement)
MUTANTS = [
    ("row_pass_step", "row[X] = row[X - 1] + 1;", "row[X] = row[X - 1] + 2;"),
    ("row_pass_no_backward", "if (row[X + 1] + 1 < row[X]) row[X] = row[X + 1] + 1;", "(void)0;"),
    ("envelope_denominator", "/ (double)(2 * q - 2 * p)", "/ (double)(q - p)"),
    ("envelope_sign", "(double)(f[q] + (int64_t)q * q) - (double)(f[p] + (int64_t)p * p)",
     "(double)(f[q] - (int64_t)q * q) - (double)(f[p] - (int64_t)p * p)"),
    ("envelope_keep_dominated", "if (s > z[k]) break;", "if (s > z[k] || k > 0) break;"),
    ("envelope_output_offset", "out[q] = d * d + f[v[k]];", "out[q] = d * d + f[q];"),
    ("column_output_shift", "e[(int64_t)(Y - 1) * w + (X - 1)] = (int32_t)res[Y];",
     "e[(int64_t)(Y - 1) * w + (X - 1)] = (int32_t)res[Y - 1];"),
    ("patch_index_transposed", "int64_t p = (int64_t)(y / patch) * gw + (x / patch);",
     "int64_t p = (int64_t)(x / patch) * gh + (y / patch);"),
    ("squared_not_euclidean", "si[p] += (spatial == 0) ? sqrt((double)e[(int64_t)y * w + x]) : 1.0;",
     "si[p] += (spatial == 0) ? (double)e[(int64_t)y * w + x] : 1.0;"),
    ("mean_not_divided", "for (int32_t c = 0; c < C; ++c) mu[c] /= (double)G;", "(void)0;"),
    ("residual_squared", "rr[p] = sqrt(acc);", "rr[p] = acc;"),
    ("D_dropped", "wrow[p] = distinct ? si[p] * D[p] : si[p];", "wrow[p] = si[p];"),
    ("D_inverted", "wrow[p] = distinct ? si[p] * D[p] : si[p];", "wrow[p] = distinct ? si[p] / D[p] : si[p];"),
    ("pool_not_normalised", "for (int32_t c = 0; c < C; ++c) F[c] /= Z;", "(void)0;"),
    ("proj_transposed", "const double* Pc = P + (int64_t)c * E;\n    for (int32_t j = 0; j < E; ++j) y[j] += F[c] * Pc[j];",
     "for (int32_t j = 0; j < E; ++j) y[j] += F[c] * P[(int64_t)j * C + c];"),
    ("output_not_normalised", "out[j] = y[j] / nn;", "out[j] = y[j];"),
    ("no_zero_fallback", "if (Z == 0.0) { /* every touched patch", "if (0) { /* every touched patch"),
    ("e4m3_bias", "v = ldexp(1.0 + man / 8.0, ex - 7);", "v = ldexp(1.0 + man / 8.0, ex - 8);"),
    ("e4m3_subnormal", "v = ldexp((double)man, -9);", "v = ldexp((double)man, -10);"),
    ("query_text_not_normalised", "row[i] = (nt > 0.0 && ny > 0.0) ? d / (nt * ny) : 0.0;",
     "row[i] = (nt > 0.0 && ny > 0.0) ? d / ny : 0.0;"),
    ("query_ties_to_higher_index", "if (!used[i] && (best < 0 || row[i] > row[best])) best = i;",
     "if (!used[i] && (best < 0 || row[i] >= row[best])) best = i;"),
    ("heatmap_D_dropped", "heat[(int64_t)j * G + p] = (nt > 0.0 && ny > 0.0) ? D[p] * (d / (nt * ny)) : 0.0;",
     "heat[(int64_t)j * G + p] = (nt > 0.0 && ny > 0.0) ? (d / (nt * ny)) : 0.0;"),
    ("heatmap_token_norm_dropped", "heat[(int64_t)j * G + p] = (nt > 0.0 && ny > 0.0) ? D[p] * (d / (nt * ny)) : 0.0;",
     "heat[(int64_t)j * G + p] = (nt > 0.0 && ny > 0.0) ? D[p] * (d / nt) : 0.0;"),
    ("heatmap_proj_transposed", "      for (int32_t k = 0; k < E; ++k) y[k] += fc * Pc[k];",
     "      for (int32_t k = 0; k < E; ++k) y[k] += fc * P[(int64_t)k * C + c];"),
    ("dbar_patch_transposed", "acc += D[(int64_t)(y / patch) * gw + (x / patch)];",
     "acc += D[(int64_t)(x / patch) * gh + (y / patch)];"),
    ("angle_sign", "const double c = -(r[0] * n[0] + r[1] * n[1] + r[2] * n[2]);",
     "const double c = (r[0] * n[0] + r[1] * n[1] + r[2] * n[2]);"),
    ("angle_not_averaged", "angle[i] = b > a ? s / (double)(b - a) : 0.0;", "angle[i] = s;"),
    ("size_no_lambda", "double size = lambda * (double)area[i] / ((double)H * (double)W);",
     "double size = (double)area[i] / ((double)H * (double)W);"),
    ("size_no_plateau", "if (size > 1.0) size = 1.0;", "(void)0;"),
    ("sem_not_rectified", "if (sem < 0.0) sem = 0.0;", "(void)0;"),
    ("dist_not_affine", "const double dist = 0.5 + 0.5 * dbar[i];", "const double dist = dbar[i];"),
    ("fuse_ties_to_last", "if (q[i] > map_q[t]) {", "if (q[i] >= map_q[t]) {"),
    ("zero_weight_row_status", "      st = 1;\n    } else {\n      st = pool_project_row(f, G, C, wr, Z",
     "      st = 2;\n    } else {\n      st = pool_project_row(f, G, C, wr, Z"),
    ("zero_weight_row_stale_pooled",
     "    if (Z == 0.0) {\n      for (int32_t j = 0; j < E; ++j) out[(int64_t)i * E + j] = 0.0;\n      for (int32_t c = 0; c < C; ++c) F[c] = 0.0;",
     "    if (Z == 0.0) {\n      for (int32_t j = 0; j < E; ++j) out[(int64_t)i * E + j] = 0.0;"),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


@pytest.mark.parametrize("mid,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, source, mid, old, new):
    assert source.count(old) == 1, f"mutation site for {mid} not found exactly once"
    mutated = source.replace(old, new)
    src = tmp_path / "disc_oracle.c"
    src.write_text(mutated)
    lib = oracle.build(force=True, src=str(src), out=str(tmp_path / f"libmut_{mid}.so"))
    orc = oracle.Oracle(lib)
    caught = []
    for name, check in pins.ALL_PINS:
        try:
            check(orc)
        except AssertionError:
            caught.append(name)
        except Exception:  # a crash or a rejected argument also exposes the mutant
            caught.append(name + "(error)")
        if caught:
            break
    assert caught, f"mutant {mid} passes every pin"
