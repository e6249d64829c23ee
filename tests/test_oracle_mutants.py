"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, and runs the committed oracle pins against that
build.  The pins must fail (pytest exit status 1: an assertion, not a crash).  A case
that survives names a mistake the pins cannot see.

The mistakes follow the passages they would break: the greedy rule and the fulfillment
transition (Section 3 and 3.1), Algorithm 1's per-pass state reset and cached actions,
the run-form entry state, the noise (Philox4x32-10 and the Gumbel-max rule), the MLP
score (Section 3.2) and the REINFORCE gradient.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "picard_oracle.c")
PINS = [os.path.join(ROOT, "tests", f) for f in
        ("test_oracle_serial.py", "test_oracle_picard.py", "test_oracle_mlp.py",
         "test_oracle_capacity.py")]

# (name, text in the oracle, replacement)
MUTANTS = [
    ("greedy_tie_takes_last",
     "if (best == LOST || c < best_cost)", "if (best == LOST || c <= best_cost)"),
    ("greedy_empty_warehouse_feasible",
     "if (x[w] <= 0) continue;\n            int32_t c",
     "if (x[w] < 0) continue;\n            int32_t c"),
    ("transition_ships_full_quantity",
     "int32_t sh = x[a] < q ? x[a] : q;", "int32_t sh = q;"),
    ("transition_ships_one_unit", "x[a] -= sh;", "x[a] -= sh > 0 ? 1 : 0;"),
    ("alg1_state_not_reset_per_process",
     "memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N); /* every view starts at s_1 */\n    for (int64_t t = 0; t < P->T; ++t) {\n        int32_t *xk = x + (int64_t)P->sku[t] * N;\n        int32_t a;\n        if (!owner || owner[t] == self) {\n            double",
     "if (self == 0) memcpy(x, P->x0, sizeof(int32_t) * (size_t)P->K * N);\n    for (int64_t t = 0; t < P->T; ++t) {\n        int32_t *xk = x + (int64_t)P->sku[t] * N;\n        int32_t a;\n        if (!owner || owner[t] == self) {\n            double"),
    ("alg1_own_steps_not_recorded",
     "            a = policy(P, m, t, xk, &a1, &a2);\n            decided[t] = a;",
     "            a = policy(P, m, t, xk, &a1, &a2);\n            decided[t] = given ? given[t] : a;"),
    # (keeping a cached action whose warehouse has no stock is not listed: it ships
    # min(q, 0) = 0 units, exactly what the lost sale does, so no state or action changes)
    ("alg1_stops_one_pass_early",
     "        if (nch == 0) { rc = 0; break; }",
     "        if (nch <= 1) { rc = 0; break; }"),
    ("runs_consumption_from_current_pass",
     "if (prev[t] != LOST) E[prev[t]] += P->qty[t];",
     "if (next[t] != LOST) E[next[t]] += P->qty[t];"),
    ("runs_consumption_counts_orders",
     "if (prev[t] != LOST) E[prev[t]] += P->qty[t];",
     "if (prev[t] != LOST) E[prev[t]] += 1;"),
    ("runs_own_correction_dropped",
     "int64_t v = (int64_t)x0k[w] - E[w] - D[w];", "int64_t v = (int64_t)x0k[w] - E[w];"),
    ("runs_own_correction_cached_not_removed",
     "if (prev[t] != LOST) D[prev[t]] -= P->qty[t];", ";"),
    ("philox_multiplier_swapped",
     "uint64_t p0 = (uint64_t)M0 * c0;", "uint64_t p0 = (uint64_t)M1 * c0;"),
    ("philox_nine_rounds", "round < 10", "round < 9"),
    ("eval_window_replay_skips_transition",
     "int32_t a = actions[t];\n            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }\n            transition(xk, a, P->qty[t]);",
     "int32_t a = actions[t];\n            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }"),
    ("reinforce_window_replay_skips_transition",
     "/* replay only */\n            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }\n            transition(xk, a, P->qty[t]);",
     "/* replay only */\n            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0)) { rc = -2; break; }"),
    ("policy_at_reads_first_row",
     "choice[i] = policy(P, &m, t, x_rows + i * (int64_t)P->N, &a1, &a2);",
     "choice[i] = policy(P, &m, t, x_rows, &a1, &a2);"),
    ("philox_key_not_bumped", "k1 += W1;", "k1 += 0;"),
    ("uniform_left_edge_of_bin", "(double)(u >> 9) + 0.5", "(double)(u >> 9) + 0.0"),
    ("uniform_same_word_for_all", "uint32_t u = out[w & 3];", "uint32_t u = out[0];"),
    ("gumbel_sign_flipped", "return -log(-log(", "return log(-log("),
    ("learned_runner_up_dropped", "else if (z > top2) top2 = z;", ";"),
    ("mlp_log_instead_of_log1p", "f[1] = log1p(inv);", "f[1] = log(inv + 2.0);"),
    ("mlp_embedding_of_region_zero", "f[2 + i] = m->E[r * 16 + i];",
     "f[2 + i] = m->E[i];"),
    ("mlp_first_relu_dropped", "h1[j] = acc > 0.0 ? acc : 0.0;", "h1[j] = acc;"),
    ("mlp_second_layer_transposed", "acc += m->W2[j * H + i] * h1[i];",
     "acc += m->W2[i * H + j] * h1[i];"),
    ("mlp_output_bias_dropped", "double s = m->b3;", "double s = 0.0;"),
    ("param_pack_without_b2", "n += (int64_t)H * H + H;", "n += (int64_t)H * H;"),
    ("reinforce_logp_without_normaliser", "const double lp = s[a] - lse;",
     "const double lp = s[a] - mx;"),
    ("reinforce_score_sign", "(w == a ? 1.0 : 0.0) - p", "(w == a ? 1.0 : 0.0) + p"),
    ("reinforce_embedding_grad_offset", "m.W1[j * 18 + 2 + i] * dp1[j]",
     "m.W1[j * 18 + 1 + i] * dp1[j]"),
    ("reinforce_w2_grad_transposed", "gW2[j * H + i] += dp2[j] * h1[i];",
     "gW2[i * H + j] += dp2[j] * h1[i];"),
    ("reinforce_second_relu_mask_dropped", "dp2[j] = pre2[j] > 0.0 ? dh[j] : 0.0;",
     "dp2[j] = dh[j];"),
    ("reinforce_state_not_advanced",
     "        transition(xk, a, P->qty[t]);\n    }\n    if (objective)",
     "    }\n    if (objective)"),
    ("eval_at_state_not_advanced",
     "        transition(xk, a, P->qty[t]);\n    }\n    free(x);\n    mlp_free(&m);\n    return rc;",
     "    }\n    free(x);\n    mlp_free(&m);\n    return rc;"),
    # node capacity (Section 3, state (x, c))
    ("cap_greedy_ignores_capacity",
     "if (x[w] <= 0 || c[w] <= 0) continue;\n            const int32_t cw",
     "if (x[w] <= 0) continue;\n            const int32_t cw"),
    ("cap_gamma_ignores_capacity_level", "const int64_t price = glow == 0 ? M - c[w] :",
     "const int64_t price = glow == 0 ? M :"),
    ("cap_gamma_low_prices_every_node", "(c[w] < glow ? (int64_t)glow - c[w] : 0)",
     "((int64_t)glow - c[w])"),
    ("cap_gamma_low_scaled_by_largest_capacity", "int64_t M = glow;\n    if (glow == 0)",
     "int64_t M = 0;\n    if (1)"),
    ("cap_gamma_rank_ties_reversed", "if (cv < cw || (cv == cw && v < w)) ++k;",
     "if (cv < cw || (cv == cw && v > w)) ++k;"),
    ("cap_gamma_max_over_feasible_only", "            if (c[w] > M) M = c[w];",
     "            if (c[w] > M && x[w] > 0) M = c[w];"),
    ("cap_transition_keeps_capacity", "x[a] -= 1;\n    c[a] -= 1;", "x[a] -= 1;"),
    ("cap_bid_stock_price_of_sku_zero",
     "pol->bid_inv ? pol->bid_inv + (int64_t)P->sku[t] * P->N : NULL;",
     "pol->bid_inv ? pol->bid_inv : NULL;"),
    ("cap_bid_capacity_price_ignored", "(pol->bid_cap ? pol->bid_cap[w] : 0);", "0;"),
    ("cap_bid_prices_added_as_rewards", "(int64_t)P->cost[w * R + r] + (bi ? bi[w] : 0) +",
     "(int64_t)P->cost[w * R + r] - (bi ? bi[w] : 0) +"),
    ("cap_bid_ties_to_last", "if (best == LOST || sc < best_s) { best = w; best_s = sc; }\n        }\n        return best;\n    }\n    if (gnum == 0)",
     "if (best == LOST || sc <= best_s) { best = w; best_s = sc; }\n        }\n        return best;\n    }\n    if (gnum == 0)"),
    # (a replayed action that ignores a node's exhausted capacity is not listed: it only
    # lowers that node's stock, and a node without capacity is never chosen again, so
    # every action is unchanged)
    ("cap_blocks_rows_from_initial_stock", "memcpy(xk, x + s * N,", "memcpy(xk, P->x0 + s * N,"),
    ("cap_blocks_capacity_from_initial", "memcpy(cp, c, sizeof(int32_t) * (size_t)N);",
     "memcpy(cp, q->cap0, sizeof(int32_t) * (size_t)N);"),
    ("cap_blocks_replay_of_fresh_actions",
     "            int32_t a = prev[t];\n            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0 || c[a] <= 0))",
     "            int32_t a = next[t];\n            if (a != LOST && (a < 0 || a >= N || xk[a] <= 0 || c[a] <= 0))"),
]


# The inventory-control (OWMR) oracle: its own source, library variable and pins.
OWMR_SRC = os.path.join(ROOT, "oracle", "owmr_oracle.c")
OWMR_PINS = [os.path.join(ROOT, "tests", "test_oracle_owmr.py")]
OWMR_MUTANTS = [
    ("owmr_retailer_receives_full_order",
     "const int64_t got = q < *x0 ? q : *x0;", "const int64_t got = q;"),
    ("owmr_central_not_clamped",
     "*x0 = reset ? P->S0 : (*x0 > q ? *x0 - q : 0);", "*x0 = reset ? P->S0 : *x0 - q;"),
    ("owmr_reset_strict", "const int rs = x0 - qq <= P->s0;", "const int rs = x0 - qq < P->s0;"),
    ("owmr_order_ignores_capacity",
     "const int64_t level = P->S_ret[n] < P->cap[n] ? P->S_ret[n] : P->cap[n];",
     "const int64_t level = P->S_ret[n];"),
    ("owmr_alg1_view_not_reset",
     "for (int n = 0; n < P->N; ++n) c->x[n] = P->x_init[n]; /* every view starts at s_1 */",
     "if (m == 0) for (int n = 0; n < P->N; ++n) c->x[n] = P->x_init[n];"),
    ("owmr_runs_reset_window_off_by_one", "if (c->LR[t] >= a) {", "if (c->LR[t] > a) {"),
    ("owmr_runs_counts_reset_order",
     "const int64_t v = P->S0 - (c->Q[t] - c->Q[r + 1]);",
     "const int64_t v = P->S0 - (c->Q[t] - c->Q[r]);"),
    ("owmr_stops_one_pass_early",
     "        if (same) { rc = 0; break; }", "        if (same || k > 1) { rc = 0; break; }"),
]


def _run_pins_against(name, old, new, workdir, src_path=SRC, env_var="PICARD_ORACLE_LIB",
                      pins=PINS):
    src = open(src_path).read()
    assert src.count(old) == 1, f"{name}: target text must occur once in the oracle"
    csrc = os.path.join(workdir, name + ".c")
    so = os.path.join(workdir, name + ".so")
    open(csrc, "w").write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-w", csrc,
                           "-o", so, "-lm"])
    env = dict(os.environ, **{env_var: so})
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = "\n".join(r.stdout.splitlines()[-6:])
    return r.returncode, tail


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as d:
        with ThreadPoolExecutor(max_workers=4) as pool:
            futs = {name: pool.submit(_run_pins_against, name, old, new, d)
                    for name, old, new in MUTANTS}
            futs.update({name: pool.submit(_run_pins_against, name, old, new, d, OWMR_SRC,
                                           "PICARD_OWMR_ORACLE_LIB", OWMR_PINS)
                         for name, old, new in OWMR_MUTANTS})
            results = {name: f.result() for name, f in futs.items()}
    survivors = {n: t for n, (rc, t) in results.items() if rc == 0}
    crashed = {n: (rc, t) for n, (rc, t) in results.items() if rc not in (0, 1)}
    assert not survivors, f"mistakes no pin catches: {sorted(survivors)}"
    assert not crashed, f"pins crashed instead of failing: {crashed}"


def test_mutant_targets_exist():
    src = open(SRC).read()
    for name, old, _ in MUTANTS:
        assert src.count(old) == 1, name
    src = open(OWMR_SRC).read()
    for name, old, _ in OWMR_MUTANTS:
        assert src.count(old) == 1, name
