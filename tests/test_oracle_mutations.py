"""The pins catch plausible mistakes in the oracle.

Each case compiles a copy of the oracle source with one deliberate mistake
(a dropped term, a flipped sign, an off-by-half bin centre, a transposed
index, a wrong tie rule, ...) into a temporary library, points the oracle
wrapper at it, and runs every pin of test_oracle_pins.py against it: at least
one pin must fail.  Everything happens on the CPU.
"""
import inspect
import os
import subprocess
import sys

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as pins

MUTATIONS = {
    "curvature_sign": ("return -kappa * or_qpt_centre(g, k);", "return kappa * or_qpt_centre(g, k);"),
    "qpt_bin_edge_not_centre": ("return g->qpt_min + ((double)k + 0.5)", "return g->qpt_min + ((double)k + 0.0)"),
    "d0_bin_edge_not_centre": ("return g->d0_min + ((double)l + 0.5)", "return g->d0_min + ((double)l + 0.0)"),
    "drop_2d_term": ("double num = c * (r * r + d * d) + 2.0 * d;\n    double den = 2.0 * r * (1.0 + c * d);\n    double A, K;",
                     "double num = c * (r * r + d * d);\n    double den = 2.0 * r * (1.0 + c * d);\n    double A, K;"),
    "den_sign": ("double den = 2.0 * r * (1.0 + c * d);\n    double A, K;",
                 "double den = 2.0 * r * (1.0 - c * d);\n    double A, K;"),
    "cordic_turn_direction": ("        x = y;\n        y = -tmp;", "        x = -y;\n        y = tmp;"),
    "cordic_constants": ("atan(ldexp(1.0, -i))", "atan(ldexp(1.0, -i - 1))"),
    "cordic_iterations": ("for (i = 0; i < 30; i++) {\n        dx", "for (i = 0; i < 12; i++) {\n        dx"),
    "q16_truncates": ("return (int32_t)llrint(s);", "return (int32_t)s;"),
    "bin_shift": ("& mask) >> F);", "& mask) >> (F + 1));"),
    "angle_bits_off_by_one": ("return or_log2(g->n_phi) + g->frac_bits;", "return or_log2(g->n_phi) + g->frac_bits + 1;"),
    "vote_layout_transposed": ("acc[((int64_t)l * g->n_qpt + k) * g->n_phi + or_bin(phiM[hh], E, M, F)] += 1;",
                               "acc[((int64_t)k * g->n_d0 + l) * g->n_phi + or_bin(phiM[hh], E, M, F)] += 1;"),
    "peaks_precedes_next_bin": ("k2 == k && db == -1);", "k2 == k && db == 1);"),
    "peaks_non_strict": ("if (precedes ? !(v > u) : !(v >= u)) return 0;", "if (!(v >= u)) return 0;"),
    "peaks_no_wrap": ("b2 = (b + db + Np) % Np;", "b2 = b + db; if (b2 < 0 || b2 >= Np) continue;"),
    "peaks_threshold_strict": ("if (v < thr) return 0;", "if (v <= thr) return 0;"),
    "assign_wrong_bin": ("if (or_bin(phiM[h], E, M, F) != bp) continue;",
                         "if (or_bin(phiM[h], E, M, F) != (bp + 1) % g->n_phi) continue;"),
    "assign_order_by_hit_only": ("if (x->rel != y->rel) return x->rel < y->rel ? -1 : 1;", ""),
    "assign_layer_descending": ("for (L = 0; L < g->n_layers; L++) {\n            int32_t E;",
                                "for (L = g->n_layers - 1; L >= 0; L--) {\n            int32_t E;"),
    "zvote_sign": ("int64_t z0 = (int64_t)Z * 65536 - S * C[m] - z0min;", "int64_t z0 = (int64_t)Z * 65536 + S * C[m] - z0min;"),
    "arclen_half": ("s = (2.0 / fabs(c)) * asin(u);", "s = (1.0 / fabs(c)) * asin(u);"),
    "arclen_chord_sign": ("Lc2 = r * r + d * d - 2.0 * d * r * A;", "Lc2 = r * r + d * d + 2.0 * d * r * A;"),
    "zvote_tie_last": ("if (zacc[i] > bestv) {", "if (zacc[i] >= bestv && zacc[i] > 0) {"),
    "fit_det_sign": ("det = sxx * (syy * N - sy * sy) - sxy * (sxy * N - sy * sx)",
                     "det = sxx * (syy * N - sy * sy) + sxy * (sxy * N - sy * sx)"),
    "fit_rhs_sign": ("r0 = -sxz;", "r0 = sxz;"),
    "fit_centre_factor": ("xc = -a / 2.0;", "xc = -a;"),
    "vertex_phi0_bin_edge": ("phi0 = ((uint32_t)b << F) + (1u << (F - 1));", "phi0 = ((uint32_t)b << F);"),
    "vertex_sign": ("v = (phi0 + (uint32_t)E) & mask;", "v = (phi0 - (uint32_t)E) & mask;"),
    "vertex_row_edge": ("return r_min + ((double)j + 0.5)", "return r_min + ((double)j + 0.0)"),
    "cr_round_down": ("*E = (int32_t)((t + ((int64_t)1 << (s - 1))) >> s);", "*E = (int32_t)(t >> s);"),
    "cr_isqrt_step": ("            root = (root >> 1) + bit;", "            root = (root >> 1) + bit + 1;"),
    "cr_layer_radius": ("        r = or_hit_radius(X, Y);", "        r = g->r_cm[layer[h]];"),
    "refine_window_inclusive": ("if (rel[j] >= c0 && rel[j] < c0 + w) {", "if (rel[j] >= c0 && rel[j] <= c0 + w) {"),
    "refine_counts_hits_not_layers": ("for (L = 0; L < NL; L++) nl += (lay_mask >> L) & 1u;", "nl = cnt;"),
    "refine_nearest_to_start": ("dist = 2 * rel[j] - 2 * (int64_t)best_c - w;", "dist = rel[j] - (int64_t)best_c;"),
    "refine_any_hit_of_layer": ("if (layer[h] != L || !(rel[j] >= best_c && rel[j] < (int64_t)best_c + w)) continue;",
                                "if (layer[h] != L) continue;"),
    "cr_assign_layer_radius": ("if (!or_sample_cr(rad[h], c, d, M, &E)) continue;",
                               "if (!or_sample_cr(g->r_cm[L], c, d, M, &E)) continue;"),
    "cr_assign_wrong_bin": ("if (bp != or_bin(phiM[h], E, M, F)) continue;",
                            "if ((bp + 1) % g->n_phi != or_bin(phiM[h], E, M, F)) continue;"),
    "cr_assign_no_angle_order": ("            qsort(mem, (size_t)m, sizeof(or_member_t), or_member_cmp);\n            for (i = 0; i < m; i++) {\n                if (pos < cap_pairs) hit_idx[pos] = mem[i].h;\n                pos++;\n            }\n        }\n    }\n    offsets[n_peaks] = pos;\n    free(phiM);\n    free(rad);",
                                 "            for (i = 0; i < m; i++) {\n                if (pos < cap_pairs) hit_idx[pos] = mem[i].h;\n                pos++;\n            }\n        }\n    }\n    offsets[n_peaks] = pos;\n    free(phiM);\n    free(rad);"),
    "cr_sqrt_operand": ("b = (int64_t)or_isqrt((uint64_t)(((int64_t)1 << 60) - a * a));",
                        "b = (int64_t)or_isqrt((uint64_t)(((int64_t)1 << 60) + a * a));"),
    "vote_columns_transposed": ("int32_t l = cols[2 * i], k = cols[2 * i + 1], hh, E;",
                                "int32_t k = cols[2 * i], l = cols[2 * i + 1], hh, E;"),
    "vote_columns_bin_edge": ("out[(int64_t)i * g->n_phi + or_bin(phiM[hh], E, M, F)] += 1;",
                              "out[(int64_t)i * g->n_phi + (or_bin(phiM[hh], E, M, F) + 1) % g->n_phi] += 1;"),
    "cot_centre_bin_edge": ("double v = g->cot_min + ((double)m + 0.5)", "double v = g->cot_min + ((double)m + 0.0)"),
    "cot_centre_truncates": ("return llrint(v * 65536.0);", "return (int64_t)(v * 65536.0);"),
    "vertex_min_votes_strict": ("if (pk[4 * p + 3] < min_votes) continue;", "if (pk[4 * p + 3] <= min_votes) continue;"),
}

SKIP = {"test_sample_table_vs_mpmath_c2"}  # slow; the c1 and sampled c4 tables run instead


def _pin_functions():
    out = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if name.startswith("test_") and name not in SKIP:
            out.append((name, fn))
    return out


@pytest.fixture(scope="module")
def src_text():
    O.build()
    with open(O.SRC) as f:
        return f.read()


RUNNER = r"""
import inspect, sys
sys.path.insert(0, {root!r})
from oracle import oracle as O
from tests import test_oracle_pins as pins
O.use_library({lib!r})
skip = {skip!r}
for name, fn in inspect.getmembers(pins, inspect.isfunction):
    if not name.startswith("test_") or name in skip:
        continue
    try:
        fn(O) if "oracle_mod" in inspect.signature(fn).parameters else fn()
    except Exception as e:
        print("CAUGHT_BY", name, type(e).__name__, flush=True)
        sys.exit(3)
print("SURVIVED", flush=True)
"""


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, src_text, tmp_path):
    """Run the pins against the mutant in a child process (a mutant may write
    out of bounds or loop; the child's failure or time-out is reported)."""
    old, new = MUTATIONS[name]
    assert src_text.count(old) == 1, f"mutation anchor not unique: {name}"
    src = tmp_path / "mut.c"
    src.write_text(src_text.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", *O.CFLAGS, "-o", str(lib), str(src), "-lm"])
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = RUNNER.format(root=root, lib=str(lib), skip=sorted(SKIP))
    try:
        res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                             env=dict(os.environ, OMP_NUM_THREADS="2"))
        out = res.stdout
        rc = res.returncode
    except subprocess.TimeoutExpired as exc:
        print("child timed out; partial output:", exc.stdout, exc.stderr)
        out, rc = "TIMEOUT", -1
    assert "SURVIVED" not in out and rc != 0, f"no pin caught mutation {name}: {out[-500:]}"


def test_unmutated_source_passes_all_pins(src_text):
    for pname, fn in _pin_functions():
        params = inspect.signature(fn).parameters
        fn(O) if "oracle_mod" in params else fn()
