"""The oracle's pins catch plausible mistakes: each mutant below plants one
error in a copy of the oracle's C source (a wrong constant, sign, comparison,
tie-break, clamp or dropped term), is built on the CPU, and must fail at
least one test of test_oracle_pins.py."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "gmacop_oracle.c")

MUTANTS = {
    "philox_multiplier": ("0xD2511F53u * c[0]", "0xD2511F55u * c[0]"),
    "isqrt_bound": ("if (mid * mid <= x) lo = mid;", "if (mid * mid < x) lo = mid;"),
    "free_flow_units": ("g->len_dm[e] * 360u / g->speed_kmh[e]", "g->len_dm[e] * 36u / g->speed_kmh[e]"),
    "red_wait_formula": ("red * red / (2 * C)", "red * red / C"),
    "preempt_tie_break": ("load[e] > load[best_edge[v]]", "load[e] >= load[best_edge[v]]"),
    "th_max_comparison": ("load[e] > p->th_max", "load[e] >= p->th_max"),
    "congestion_divisor": ("(uint64_t)t0 * load / theta", "(uint64_t)t0 * load / (theta + 1)"),
    "goal_sign": ("(int64_t)g->x_dm[node] - g->x_dm[dst]", "(int64_t)g->x_dm[node] + g->x_dm[dst]"),
    "eta_scale": ("((uint64_t)1 << 26) / d", "((uint64_t)1 << 25) / d"),
    "roulette_strict": ("if (prefix > target) return j;", "if (prefix >= target) return j;"),
    "visited_ignored": ("if (visited[x]) { wbuf[j] = 0; continue; }", "if (0) { wbuf[j] = 0; continue; }"),
    "deposit_amount": ("const uint64_t d = p->q_deposit / cs;", "const uint64_t d = p->q_deposit / (cs + 1);"),
    "evaporation_factor": ("(uint64_t)tau * (65536u - p->rho_q16) / 65536u",
                           "(uint64_t)tau * (65535u - p->rho_q16) / 65536u"),
    "best_tie": ("(uint32_t)(iter_key >> 32) < *best_cost", "(uint32_t)(iter_key >> 32) <= *best_cost"),
    "load_increment": ("load[path_edges[(size_t)v * S + i]] += 1;", "load[path_edges[(size_t)v * S + i]] += 2;"),
    "counter_swap": ("const uint32_t ctr[4] = {qid, ant, p->iter_offset + iter, step};",
                     "const uint32_t ctr[4] = {ant, qid, p->iter_offset + iter, step};"),
    "word_order": ("return ((uint64_t)x[1] << 32) | x[0];", "return ((uint64_t)x[0] << 32) | x[1];"),
    "goal_exact_weight": ("rw[fill[x]] = t0[e];", "rw[fill[x]] = t0[e] + wf[e];"),
    "goal_exact_cap": ("(dist[v] > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)dist[v])", "((uint32_t)dist[v])"),
    "goal_exact_unreachable": ("h[v] = dist[v] == UINT64_MAX ? U32_MAX :", "h[v] = dist[v] == UINT64_MAX ? 0u :"),
    "goal_exact_row_ignored": ("return hrow ? (int64_t)hrow[x] :", "return hrow ? (int64_t)hrow[dst] :"),
    "goal_exact_forward_roads": (
        """    for (uint32_t e = 0; e < m; ++e) rp[g->col[e] + 1]++;
    for (uint32_t x = 0; x < n; ++x) rp[x + 1] += rp[x];
    uint32_t *fill = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    memcpy(fill, rp, sizeof(uint32_t) * n);
    for (uint32_t u = 0; u < n; ++u)
        for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
            const uint32_t x = g->col[e];
            ru[fill[x]] = u;
            rw[fill[x]] = t0[e];
            fill[x]++;
        }""",
        """    for (uint32_t u = 0; u <= n; ++u) rp[u] = g->row_ptr[u];
    uint32_t *fill = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    for (uint32_t e = 0; e < m; ++e) { ru[e] = g->col[e]; rw[e] = t0[e]; }"""),
    "shortest_route_last_tight": ("if ((uint64_t)t0[e] + h[g->col[e]] == h[u]) { next = e; break; }",
                                  "if ((uint64_t)t0[e] + h[g->col[e]] == h[u]) { next = e; }"),
    "greedy_argmax": ("if (best == U32_MAX || mark[e] < mark[best]) { second = best; best = e; }",
                      "if (best == U32_MAX || mark[e] > mark[best]) { second = best; best = e; }"),
    "greedy_threshold_inclusive": ("choice[v] = (n_t[c] > p->theta && second != U32_MAX)",
                                   "choice[v] = (n_t[c] >= p->theta && second != U32_MAX)"),
    "greedy_no_decrement": ("mark[e] + (int64_t)moves[e] - (int64_t)(m_t[c] - moves[e]);",
                            "mark[e] + (int64_t)moves[e];"),
    "greedy_tie_last": ("else if (second == U32_MAX || mark[e] < mark[second]) second = e;",
                        "else if (second == U32_MAX || mark[e] <= mark[second]) second = e;"),
    "timed_windows_not_accumulated": ("start[e] = (uint32_t)(acc[v] % C);", "start[e] = 0;"),
    "timed_no_cap": ("if (wait > p->t_max_ms) wait = p->t_max_ms;", ""),
    "timed_entry_instead_of_arrival": ("const uint64_t q = ((clock + travel) % C + C - tm->wstart[e]) % C;",
                                       "const uint64_t q = (clock % C + C - tm->wstart[e]) % C;"),
    "timed_preemption_ignored": ("if (C && !tm->pre[e]) {", "if (C) {"),
    "sim_queue_tie_to_last": ("if (Q[e] > 0 && (best[v] == U32_MAX || Q[e] > Q[best[v]])) best[v] = e;",
                              "if (Q[e] > 0 && (best[v] == U32_MAX || Q[e] >= Q[best[v]])) best[v] = e;"),
    "sim_window_ignored": ("if (!green) green = ((t % C + C - ws[e]) % C) < wg[e];", ""),
    "sim_no_t_max": ("if (green || waited[i] >= p->t_max_ms) {", "if (green) {"),
    "sim_no_congestion": ("if (N[e] > p->theta) {\n                v = v * p->theta / N[e];",
                          "if (0) {\n                v = v * p->theta / N[e];"),
    "sim_arrival_at_tick_start": ("const uint64_t a = t + tick_ms;", "const uint64_t a = t;"),
    "sim_own_speed_only": ("uint64_t v = speed_kmh[i] < g->speed_kmh[e] ? speed_kmh[i] : g->speed_kmh[e];",
                           "uint64_t v = speed_kmh[i];"),
    "apply_after_load_update": (
        """            for (uint32_t e = 0; e < m; ++e) tau[e] = orc_apply_tau(p, tau[e], dep[e], load[e]);
            if (!(p->flags & ORC_FLAG_NO_LOAD_UPDATE)) {
                for (uint32_t e = 0; e < m; ++e) load[e] = g->base_load[e];
                for (uint32_t v = 0; v < nv; ++v)
                    for (uint32_t i = 0; i < path_len[v]; ++i) load[path_edges[(size_t)v * S + i]] += 1;
            }""",
        """            if (!(p->flags & ORC_FLAG_NO_LOAD_UPDATE)) {
                for (uint32_t e = 0; e < m; ++e) load[e] = g->base_load[e];
                for (uint32_t v = 0; v < nv; ++v)
                    for (uint32_t i = 0; i < path_len[v]; ++i) load[path_edges[(size_t)v * S + i]] += 1;
            }
            for (uint32_t e = 0; e < m; ++e) tau[e] = orc_apply_tau(p, tau[e], dep[e], load[e]);"""),
}


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, source, name):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut = tmp_path / "gmacop_oracle.c"
    mut.write_text(source.replace(old, new))
    (tmp_path / "gmacop_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "gmacop_oracle.h")).read())
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", str(lib), str(mut)])
    env = dict(os.environ, GMACOP_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
