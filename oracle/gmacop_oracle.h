/*
 * gmacop_oracle.h -- CPU oracle for the GMACO-P routing hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * definition of what the GPU library computes, used to check it.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the GPU library never links, includes or calls it, and the two share no
 * code.
 *
 * Method: Jindal & Bedi, "GMACO-P: GPU assisted Preemptive MACO algorithm for
 * enabling Smart Transportation" (arXiv 2010.14244): the MACO-P vehicle loop
 * (Section 4.1, Fig. 3) and the GMACO-P kernel steps (Section 4.2, Alg. 2:
 * Calc_Dist, Adj_Neigh, Eval_Rout, Calc_Dens, Comp_Thres, Updt_Pher,
 * Evap_Pher).  Where the paper leaves a quantity undefined, the reading used
 * here is stated next to the function that implements it.
 *
 * All arithmetic is integer: pheromone is Q16.16 (65536 = 1.0), times are
 * milliseconds, lengths decimetres, speeds km/h.
 */
#ifndef GMACOP_ORACLE_H
#define GMACOP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t n, m;
    const uint32_t *row_ptr;    /* [n+1] */
    const uint32_t *col;        /* [m] head node */
    const uint32_t *len_dm;     /* [m] */
    const uint16_t *speed_kmh;  /* [m] */
    const uint16_t *green_pm;   /* [m] green share of approach e at head(e), per mille */
    const uint32_t *cycle_ms;   /* [n] 0 = unsignalised */
    const int32_t  *x_dm;       /* [n] */
    const int32_t  *y_dm;       /* [n] */
    const uint32_t *base_load;  /* [m] sensed vehicles per road */
} orc_graph;

typedef struct {
    uint32_t ants, iterations, alpha, beta, max_steps;
    uint32_t rho_q16, tau0_q16, tau_min_q16, tau_max_q16;
    uint64_t q_deposit;
    uint32_t theta, th_max, t_max_ms, vmax_kmh;
    uint32_t mode;          /* 0 = shared pheromone/load, 1 = independent per vehicle */
    uint32_t flags;         /* ORC_FLAG_NO_LOAD_UPDATE: loads frozen at base_load;
                               ORC_FLAG_GOAL_EXACT: exact goal term instead of the straight line */
    uint64_t seed;
    uint32_t iter_offset;
} orc_params;

#define ORC_MODE_SHARED      0u
#define ORC_MODE_INDEPENDENT 1u
#define ORC_FLAG_NO_LOAD_UPDATE 1u
#define ORC_FLAG_GOAL_EXACT 16u   /* goal term = exact shortest free-flow time to dst */
#define ORC_FLAG_SIGNAL_TIMED 64u /* signal waits at the ant's arrival time in the green windows */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* floor(sqrt(x)) for any 64-bit x */
uint64_t orc_isqrt(uint64_t x);

/* Per-road static quantities: free-flow time t0 and fixed-time signal wait wf. */
void orc_edge_static(const orc_graph *g, const orc_params *p, uint32_t *t0, uint32_t *wf);
/* Congestion/preemption cost table for a given per-road load. */
void orc_cost_table(const orc_graph *g, const orc_params *p, const uint32_t *load,
                    const uint32_t *t0, const uint32_t *wf, uint32_t *cost,
                    uint8_t *preempted /* may be NULL */);
/* Goal term h(node) for destination dst (time-to-go lower bound, ms). */
uint64_t orc_goal(const orc_graph *g, const orc_params *p, uint32_t node, uint32_t dst);
/* Exact goal row for destination dst: shortest free-flow time (sum of t0)
 * from every node to dst, min(.., 0xFFFFFFFE); 0xFFFFFFFF = cannot reach dst. */
void orc_goal_exact(const orc_graph *g, const orc_params *p, uint32_t dst, uint32_t *h);
/* Shortest free-flow route src -> dst: first road (road order) on a shortest
 * route at every node; returns its road count, 0 if out of reach, capped or
 * longer than max_len. */
uint32_t orc_shortest_route(const orc_graph *g, const orc_params *p, uint32_t src, uint32_t dst,
                            uint32_t max_len, uint32_t *path);
/* Green windows of the time-dependent signals: per road e, the start (ms, mod
 * the head's cycle) and length of its approach's green. */
void orc_signal_windows(const orc_graph *g, uint32_t *start, uint32_t *green);
/* Cost of road e entered at time `clock` (ms since the call's start) with
 * time-dependent signals, at the sensed loads. */
uint32_t orc_timed_cost(const orc_graph *g, const orc_params *p, uint32_t e, uint64_t clock);
/* Heuristic desirability of a road from its reduced cost. */
uint32_t orc_eta(int64_t delta);
/* Roulette: index chosen among d weights by a 64-bit random word. */
uint32_t orc_roulette(const uint64_t *w, uint32_t d, uint64_t r);
/* One pheromone apply step for a road (evaporate, penalised deposit, clamp). */
uint32_t orc_apply_tau(const orc_params *p, uint32_t tau, uint64_t deposit, uint32_t load);

/* One ant walk under a given pheromone vector and cost table.
 * Returns 1 on arrival at dst, 0 on failure; fills path[0..*len-1] (edges). */
int orc_walk(const orc_graph *g, const orc_params *p, const uint32_t *tau, const uint32_t *cost,
             uint32_t qid, uint32_t src, uint32_t dst, uint32_t ant, uint32_t iter,
             uint32_t *path, uint32_t *len, uint32_t *cost_sum, uint64_t *selections);

/* Whole run (Section 4.2, Alg. 2 steps 3-10 iterated).  Returns 0, or -1 on
 * invalid input.  Outputs: best path per vehicle (edges, row v at
 * path_edges + v*max_steps), its length (0 = none) and cost (UINT32_MAX = none),
 * number of roulette selections, and optionally the final pheromone and load
 * (shared mode: [m]; independent mode: tau [nv*m], load [m]) and the
 * best-so-far cost of each vehicle after every iteration ([iterations*nv]). */
int orc_route(const orc_graph *g, const uint32_t *qid, const uint32_t *src, const uint32_t *dst,
              uint32_t nv, const orc_params *p,
              uint32_t *path_edges, uint32_t *path_len, uint32_t *cost_ms, uint64_t *steps_total,
              uint32_t *tau_out, uint32_t *load_out, uint32_t *best_hist);

/* Literal MACO-P vehicle loop of Fig. 3 in synchronous ticks (least-marker
 * road toward the destination, second least when N_t > theta; markers +1 on
 * the chosen road, -1 on every other road of the city per move).
 * city_of_node: [n] or NULL.  Returns 0, or -1 on invalid input. */
int orc_greedy(const orc_graph *g, const uint32_t *src, const uint32_t *dst, uint32_t nv, const orc_params *p,
               const uint32_t *city_of_node, uint32_t *path_edges, uint32_t *path_len, uint32_t *cost_ms,
               uint64_t *steps_total, uint32_t *marker_out);

/* Traffic simulation of the vehicles' trips along their routes (Section 5):
 * synchronous ticks of tick_ms, congestion slowing a road above theta
 * vehicles, the preemptive signal rule at every signal (green window, longest
 * queue, queue above Th_max, or a wait of T_max).  path: [nv][stride] roads,
 * path_len[nv] (0 = no route), speed_kmh[nv].  Outputs per vehicle: arrival
 * time in ms (UINT32_MAX = no route, or not arrived within max_ticks) and total
 * signal wait; the ticks run.  Returns 0, or -1 on invalid input. */
int orc_simulate(const orc_graph *g, const orc_params *p, const uint32_t *path, uint32_t stride,
                 const uint32_t *path_len, const uint32_t *speed_kmh, uint32_t nv, uint32_t tick_ms,
                 uint32_t max_ticks, uint32_t *arrival_ms, uint32_t *wait_ms, uint32_t *ticks_run);

#ifdef __cplusplus
}
#endif
#endif
