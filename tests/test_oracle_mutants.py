"""Planted mistakes: each mutant of the oracle source (built on the CPU in a
temporary directory) must fail at least one pin of test_oracle_pins.  This
checks that the pins are strong enough that a plausible slip anywhere in the
oracle -- a stencil window, a weight, a sign, an index, an operation or axis
order, the tie rule, the mask bit order, the padding -- would be noticed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import test_oracle_pins as P

MUTANTS = {
    "w4_window": ("oracle/cz_oracle.c", "int s = clampi(m - 1, 0, h - 4);", "int s = clampi(m - 2, 0, h - 4);"),
    "w4_eval_point": ("oracle/cz_oracle.c", "w[j] = lagrange(x, 4, j, m + 0.5);", "w[j] = lagrange(x, 4, j, m + 0.25);"),
    "w3_below_edge": ("oracle/cz_oracle.c", "(s + i + 1 <= k)", "(s + i + 1 < k)"),
    "w3_window": ("oracle/cz_oracle.c", "int s = clampi(k - 1, 0, h - 3);", "int s = clampi(k, 0, h - 3);"),
    "update_scale": ("oracle/cz_oracle_t.h", "T term = (T)(0.5 * w) * d[m];", "T term = (T)(0.25 * w) * d[m];"),
    "update_sign": ("oracle/cz_oracle_t.h", "s[k] = a[k] + SFX(w4_update)(d, h, k);", "s[k] = a[k] - SFX(w4_update)(d, h, k);"),
    "update_window": ("oracle/cz_oracle.c", "    int s = m - 1;\n    if (k < s || k > s + 3)", "    int s = m - 2;\n    if (k < s || k > s + 3)"),
    "w3_right_child": ("oracle/cz_oracle_t.h", "d[k] = v[2 * k] - SFX(w3_pred)(a, h, k);", "d[k] = v[2 * k + 1] - SFX(w3_pred)(a, h, k);"),
    "w3_inverse_odd": ("oracle/cz_oracle_t.h", "v[2 * k + 1] = (C[k] + C[k]) - a;", "v[2 * k + 1] = C[k] - (a - C[k]);"),
    "dot_order": ("oracle/cz_oracle_t.h", "    T acc = (T)w[0] * x[0];\n    for (int j = 1; j < k; j++)\n        acc = acc + (T)w[j] * x[j];",
                  "    T acc = (T)w[k - 1] * x[k - 1];\n    for (int j = k - 2; j >= 0; j--)\n        acc = acc + (T)w[j] * x[j];"),
    "fwd_axis_order": ("oracle/cz_oracle_t.h", "        SFX(axis_pass)(scheme, 0, 1, N, n, B);\n        SFX(axis_pass)(scheme, 0, 2, N, n, B);",
                       "        SFX(axis_pass)(scheme, 0, 2, N, n, B);\n        SFX(axis_pass)(scheme, 0, 1, N, n, B);"),
    "inv_axis_order": ("oracle/cz_oracle_t.h", "        SFX(axis_pass)(scheme, 1, 2, N, n, B);\n        SFX(axis_pass)(scheme, 1, 1, N, n, B);\n        SFX(axis_pass)(scheme, 1, 0, N, n, B);",
                       "        SFX(axis_pass)(scheme, 1, 0, N, n, B);\n        SFX(axis_pass)(scheme, 1, 1, N, n, B);\n        SFX(axis_pass)(scheme, 1, 2, N, n, B);"),
    "depth_one_short": ("oracle/cz_oracle_t.h", "    for (int n = N; n >= 8; n /= 2) {\n        SFX(axis_pass)(scheme, 0, 0, N, n, B);",
                        "    for (int n = N; n >= 16; n /= 2) {\n        SFX(axis_pass)(scheme, 0, 0, N, n, B);"),
    "tie_rule": ("oracle/cz_oracle_t.h", "fabs((double)C[q]) >= eps", "fabs((double)C[q]) > eps"),
    "threshold_in_T": ("oracle/cz_oracle_t.h", "fabs((double)C[q]) >= eps", "(double)(T)fabs((double)C[q]) >= (double)(T)eps"),
    "corner_not_forced": ("oracle/cz_oracle_t.h", "int coarse = x < 4 && y < 4 && z < 4;", "int coarse = 0;"),
    "mask_msb_first": ("oracle/cz_oracle_t.h", "mask[q >> 3] |= (uint8_t)(1u << (q & 7));", "mask[q >> 3] |= (uint8_t)(0x80u >> (q & 7));"),
    "no_pad_zero": ("oracle/cz_oracle_t.h", "    memset(rec + used, 0, total - used);\n    return total;", "    return total;"),
    "corner_z_short": ("oracle/cz_oracle_t.h", "int coarse = x < 4 && y < 4 && z < 4;", "int coarse = x < 4 && y < 4 && z < 2;"),
    "gather_xy_swap": ("oracle/cz_oracle_t.h", "                B[x + N * (y + N * z)] = field[g];", "                B[y + N * (x + N * z)] = field[g];"),
}


def _pins(o):
    """Run a representative subset of the pins against the oracle module o."""
    P.test_w4_predict_rows_match_fitted_cubic(o, 16)
    P.test_w4_predict_rows_match_fitted_cubic(o, 8)
    P.test_w4li_update_is_half_centred_predict_transpose(o, 16)
    P.test_w3ai_predict_matches_fitted_quadratic_average(o, 16)
    for s in P.SCHEMES:
        P.test_one_level_exact_on_small_integers(o, s, 16)
        P.test_block_n8_exact_rational(o, s)
        P.test_perfect_reconstruction_eps0(o, np.float32, s, 16)
        P.test_stream_invariants_and_decode(o, s, np.float32)
        P.test_inverse_rounding_order(o, np.float32, s)
        P.test_block_rounding_order(o, np.float32, s, 8)
    P.test_w4_details_of_quartic_are_nodal_polynomial(o, 32, 0)
    P.test_w3ai_details_of_cubic(o, 32)
    P.test_threshold_tie_is_kept(o)
    P.test_threshold_compared_in_double(o)
    P.test_constant_field_records(o)


def test_unmutated_passes_subset(oracle):
    _pins(oracle)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch, oracle):
    path, old, new = MUTANTS[name]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for f in ("cz_oracle.c", "cz_oracle_t.h"):
        shutil.copy(os.path.join(root, "oracle", f), tmp_path / f)
    target = tmp_path / os.path.basename(path)
    src = target.read_text()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    target.write_text(src.replace(old, new))
    so = tmp_path / "libczoracle_mutant.so"
    subprocess.run(["gcc", *O.CFLAGS, str(tmp_path / "cz_oracle.c"), "-o", str(so), "-lm"], check=True)
    monkeypatch.setattr(O, "LIB_PATH", str(so))
    monkeypatch.setattr(O, "_lib", None)
    with pytest.raises((AssertionError, O.OracleError)):
        _pins(O)
