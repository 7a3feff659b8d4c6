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
        ("return priority(seed, x) > priority(seed, y);",
         "return priority(seed, x) < priority(seed, y);"),
    "coloring_priority_unshifted_seed":
        ("return splitmix64_finalizer((seed << 32) ^ (uint64_t)v);",
         "return splitmix64_finalizer(seed ^ (uint64_t)v);"),
    "vf_leaf_does_not_follow":
        ("map[i] = single[j] ? std::min<int32_t>((int32_t)i, j) : j;",
         "map[i] = single[j] ? std::min<int32_t>((int32_t)i, j) : (int32_t)i;"),
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
