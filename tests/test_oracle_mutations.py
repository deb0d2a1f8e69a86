"""The oracle's pins have teeth: each plausible mistake planted in a copy of
the oracle source (a wrong constant, sign, index, dropped weight or term) is
caught by at least one pin of test_oracle_pins.py.

Mistakes are planted on the CPU only, in a temporary build of the oracle; the
real oracle is untouched.
"""

from __future__ import annotations

import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "wsm_oracle.c")

# (name, exact text in wsm_oracle.c, planted replacement)
MUTATIONS = [
    ("break_test_2x", "d[(size_t)p * K + t] >= 4.0 * prev", "d[(size_t)p * K + t] >= 2.0 * prev"),
    ("break_test_strict_8x", "d[(size_t)p * K + t] >= 4.0 * prev", "d[(size_t)p * K + t] >= 8.0 * prev"),
    ("tie_prefers_higher_index", "best != p && t < best", "best != p && t > best"),
    ("tie_ignores_previous", "(dist == best_d && best != p && t < best)", "(dist == best_d && t < best)"),
    ("channel_term_swapped", "return d0 * d0 + d1 * d1 + d2 * d2;", "return d0 * d0 + d1 * d0 + d2 * d2;"),
    ("channel_term_dropped", "return d0 * d0 + d1 * d1 + d2 * d2;", "return d0 * d0 + d1 * d1;"),
    ("unweighted_update", "double w = (double)counts[i];", "double w = 1.0;"),
    ("empty_cluster_not_kept", "if (sum[4 * k + 3] > 0.0) {\n            c[3 * k + 0]", "if (1) {\n            c[3 * k + 0]"),
    ("stop_rule_from_first_iter", "(t >= 2 && (prev_sse - sse) / sse <= eps)", "(t >= 1 && (prev_sse - sse) / sse <= eps)"),
    ("stop_rule_sign", "(prev_sse - sse) / sse <= eps)", "(sse - prev_sse) / sse <= eps)"),
    ("reduce_key_channels_swapped", "freq[key] += 1;", "freq[(key & 0xFF00u) | (key >> 16) | ((key & 0xFFu) << 16)] += 1;"),
    ("row_sort_descending", "if (a->d < b->d) return -1;\n    if (a->d > b->d) return 1;",
     "if (a->d < b->d) return 1;\n    if (a->d > b->d) return -1;"),
    ("scan_starts_at_self", "for (int j = 1; j < K; ++j) {\n            int t = M[(size_t)p * K + j];",
     "for (int j = 2; j < K; ++j) {\n            int t = M[(size_t)p * K + j];"),
    ("sse_unweighted", "s += ((double)counts[i] / (double)n_pixels) * min_dist[i];",
     "s += (1.0 / (double)n) * min_dist[i];"),
    ("grad_factor_two_dropped", "double scale = 2.0 * g / (double)n;", "double scale = g / (double)n;"),
    ("grad_sign_flipped", "double diff = x[3 * p + ch] - c[3 * k + ch];",
     "double diff = c[3 * k + ch] - x[3 * p + ch];"),
    ("grad_palette_sign", "grad_c[3 * k + ch] -= scale * diff;", "grad_c[3 * k + ch] += scale * diff;"),
    ("distortion_not_averaged", "    return s / (double)n;\n}\n\nvoid oracle_distortion_grad",
     "    return s;\n}\n\nvoid oracle_distortion_grad"),
]


def _pin_suite():
    """Run a representative subset of the pins; raises on the first failure."""
    for seed in (0, 1):
        pins.test_reduce_matches_numpy_unique(seed)
    pins.test_reduce_hand_cases()
    for ex in pins._golden():
        pins.test_oracle_reproduces_worked_example(ex)
    for seed in range(40):
        pins.test_search_step_equals_exact_brute_force(seed)
    for seed in range(12):
        pins.test_wsm_trajectory_equals_exact_lloyd(seed)
    pins.test_empty_cluster_keeps_its_center()
    pins.test_k1_is_mean_color_and_total_variance()
    pins.test_sq_distance_uses_all_three_channels()
    for seed in range(3):
        pins.test_distortion_gradient_equals_exact_central_difference(seed)
    pins.test_distortion_gradient_vanishes_at_exact_centroids()
    pins.test_distortion_at_nearest_assignment_is_the_map_mse()


def test_unmutated_oracle_passes_the_suite():
    _pin_suite()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new, 1)
    c_path = tmp_path / "mut.c"
    c_path.write_text(mutated)
    hdr = os.path.join(os.path.dirname(SRC), "wsm_oracle.h")
    (tmp_path / "wsm_oracle.h").write_text(open(hdr).read())
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-shared",
                    "-fPIC", str(c_path), "-o", str(so), "-lm"], check=True)
    caught = False
    with oracle.use_library(str(so)):
        try:
            _pin_suite()
        except Exception:
            caught = True
    assert caught, f"planted mistake '{name}' was not caught by any pin"
