"""Plants plausible mistakes in copies of the oracle (on the CPU) and checks
that the pins catch each one: a dropped term, a wrong sign, a wrong
tie-break, a transposed or halved operand, broken synchronous semantics."""
import os
import subprocess

import pytest

import oracle
import pins

MUTANTS = {
    "self_loop_counted_twice_in_degree":
        ("for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e) k[i] += g.w[e];",
         "for (int64_t e = g.off[i]; e < g.off[i + 1]; ++e) k[i] += g.w[e] * (g.col[e] == i ? 2 : 1);"),
    "self_loop_dropped_from_internal_weight":
        ("if (C[u] == C[g.col[e]]) inside += g.w[e];",
         "if (C[u] == C[g.col[e]] && u != g.col[e]) inside += g.w[e];"),
    "stay_gain_sign":
        ("return (i128)two_m * e_iA - (i128)k[i] * (a[A] - k[i]);",
         "return (i128)two_m * e_iA - (i128)k[i] * (a[A] + k[i]);"),
    "gain_factor_two_on_community_degree":
        ("return (i128)two_m * e_ic - (i128)k[i] * a[c];",
         "return (i128)two_m * e_ic - 2 * (i128)k[i] * a[c];"),
    "max_label_tie_break":
        ("if (!have || G > best) { best = G; best_c = kv.first; have = true; }",
         "if (!have || G >= best) { best = G; best_c = kv.first; have = true; }"),
    "singlet_veto_inverted":
        ("size[best_c] == 1 && best_c > A) return A;",
         "size[best_c] == 1 && best_c < A) return A;"),
    "move_on_equal_gain":
        ("if (!have || !(best > stay)) return A;",
         "if (!have || !(best >= stay)) return A;"),
    "asynchronous_updates":
        ("for (size_t t = 0; t < K.size(); ++t) next[t] = decide(K[t], singlet_rule);\n"
         "            for (size_t t = 0; t < K.size(); ++t) {",
         "for (size_t t = 0; t < K.size(); ++t) {\n"
         "                next[t] = decide(K[t], singlet_rule);"),
    "coarse_internal_entry_counted_once":
        ("W[{new_of[C[u]], new_of[C[g.col[e]]]}] += g.w[e];",
         "if (new_of[C[u]] != new_of[C[g.col[e]]] || u <= g.col[e]) W[{new_of[C[u]], new_of[C[g.col[e]]]}] += g.w[e];"),
    "coloring_ascending_priority":
        ("return priority(seed, x) > priority(seed, y); });\n    color.assign(g.n, -1);",
         "return priority(seed, x) < priority(seed, y); });\n    color.assign(g.n, -1);"),
    "coloring_priority_unshifted_seed":
        ("return splitmix64_finalizer((seed << 32) ^ (uint64_t)v);",
         "return splitmix64_finalizer(seed ^ (uint64_t)v);"),
    "vf_leaf_does_not_follow":
        ("map[i] = single[j] ? std::min<int32_t>((int32_t)i, j) : j;",
         "map[i] = single[j] ? std::min<int32_t>((int32_t)i, j) : (int32_t)i;"),
    "loss_kept":
        ("if (N_t < N_prev) {", "if (false && N_t < N_prev) {"),
    "loss_checked_from_second_iteration":
        ("if (N_t < N_prev) {", "if (t >= 2 && N_t < N_prev) {"),
    "threshold_tested_from_first_iteration":
        ("if (t >= 2 && gain_below(N_t, N_prev", "if (t >= 1 && gain_below(N_t, N_prev"),
    "relative_threshold_taken_as_absolute":
        ("u128 ref = mode == 0 ? uabs(before) : (u128)D;", "u128 ref = (u128)D;"),
    "threshold_not_strict":
        ("return h1 < h2 || (h1 == h2 && l1 < l2);", "return h1 < h2 || (h1 == h2 && l1 <= l2);"),
    "colored_phase_uses_theta_final":
        ("int64_t tnum = colored ? P.theta_color_num : P.theta_final_num;\n"
         "        int64_t tden = colored ? P.theta_color_den : P.theta_final_den;",
         "int64_t tnum = P.theta_final_num;\n"
         "        int64_t tden = P.theta_final_den;"),
    "coloring_kept_on_small_phase_gain":
        ("P.color_first_phase_only ||\n"
         "                gain_below(N_t, Q_prev, D, P.theta_color_num, P.theta_color_den, 0))",
         "P.color_first_phase_only)"),
    "first_phase_only_ignored":
        ("n_after == n_before || P.color_first_phase_only ||", "n_after == n_before ||"),
    "colored_no_shrink_ignored":
        ("if (n_after < P.color_cutoff || n_after == n_before ||", "if (n_after < P.color_cutoff ||"),
    "final_no_shrink_ignored":
        ("stop = (n_after == n_before) || (p >= P.max_phases) ||", "stop = (p >= P.max_phases) ||"),
    "color_cutoff_strict":
        ("bool colored = still_coloring && st.g.n >= P.color_cutoff;",
         "bool colored = still_coloring && st.g.n > P.color_cutoff;"),
    "vf_pair_to_larger_id":
        ("map[i] = single[j] ? std::min<int32_t>((int32_t)i, j) : j;",
         "map[i] = single[j] ? std::max<int32_t>((int32_t)i, j) : j;"),
    "chain_vf_without_the_bound":
        ("single[i] = others == 1 && (i128)two_m * w > (i128)k[i] * k[nbr[i]];", "single[i] = others == 1;"),
    "chain_vf_bound_not_strict":
        ("single[i] = others == 1 && (i128)two_m * w > (i128)k[i] * k[nbr[i]];",
         "single[i] = others == 1 && (i128)two_m * w >= (i128)k[i] * k[nbr[i]];"),
    "chain_vf_one_round":
        ("            coarsen_step();\n            ++rounds;\n",
         "            coarsen_step();\n            return 1;\n"),
    "chain_vf_self_loop_rows_excluded":
        ("if (g.col[e] != i) { ++others; nbr[i] = g.col[e]; w = g.w[e]; }",
         "{ ++others; nbr[i] = g.col[e]; w = g.w[e]; }"),
    "chain_vf_pair_to_larger_id":
        ("map[i] = single[to] ? std::min<int32_t>((int32_t)i, to) : to;",
         "map[i] = single[to] ? std::max<int32_t>((int32_t)i, to) : to;"),
    "balance_target_floor":
        ("const int64_t gamma = (g.n + ncolors - 1) / ncolors;", "const int64_t gamma = g.n / ncolors;"),
    "balance_without_room_cap":
        ("                if (moved == room) break;\n", ""),
    "balance_largest_admissible_colour":
        ("for (int32_t d = 0; d < ncolors && to < 0; ++d)", "for (int32_t d = ncolors - 1; d >= 0 && to < 0; --d)"),
    "balance_ascending_priority":
        ("[&](int32_t x, int32_t y) { return priority(seed, x) > priority(seed, y); });\n    int64_t moved_total",
         "[&](int32_t x, int32_t y) { return priority(seed, x) < priority(seed, y); });\n    int64_t moved_total"),
    "rounding_truncates":
        ("if (round_bit && (sticky || (mant & 1))) {",
         "if (false && round_bit && (sticky || (mant & 1))) {"),
}


@pytest.fixture(scope="module")
def src():
    with open(oracle.SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, src, name):
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    path = tmp_path / "mutant.cpp"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", lib, str(path)], check=True)
    O = oracle.Oracle(lib)
    failed = []
    for check in pins.ALL:
        try:
            check(O)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"mutant {name} passed every pin"
