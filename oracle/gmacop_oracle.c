/*
 * gmacop_oracle.c -- CPU oracle for the GMACO-P routing hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see gmacop_oracle.h).  Plain single-threaded C,
 * written for checking by eye against the paper, not for speed.  No blocking,
 * fusion or reordering beyond what each step states.
 *
 * Paper: Jindal & Bedi, arXiv 2010.14244.  Section numbers below refer to it.
 */
#include "gmacop_oracle.h"

#include <stdlib.h>
#include <string.h>

#define U32_MAX 0xFFFFFFFFu
#define COST_CAP (1u << 31)              /* one road never costs more than 2^31 ms */
#define PATH_COST_CAP 0xFFFFFFFEu        /* UINT32_MAX is reserved for "no route" */

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10, counter based (Salmon et al., SC'11).     */
/* The counter of the draw for step s of ant k of vehicle q in iteration t  */
/* is (q, k, t, s); the key is the 64-bit seed split into two words.        */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t out[4];
    out[0] = hi1 ^ c[1] ^ k[0];
    out[1] = lo1;
    out[2] = hi0 ^ c[3] ^ k[1];
    out[3] = lo0;
    memcpy(c, out, sizeof(out));
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {              /* key schedule: Weyl sequence */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

static uint64_t draw64(const orc_params *p, uint32_t qid, uint32_t ant, uint32_t iter, uint32_t step)
{
    const uint32_t ctr[4] = {qid, ant, p->iter_offset + iter, step};
    const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    return ((uint64_t)x[1] << 32) | x[0];
}

/* floor(sqrt(x)) by bisection over [0, 2^32): the largest s with s*s <= x. */
uint64_t orc_isqrt(uint64_t x)
{
    uint64_t lo = 0, hi = (uint64_t)1 << 32;     /* invariant: lo*lo <= x < hi*hi */
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (mid * mid <= x) lo = mid; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* Static per-road quantities.                                              */
/* Free-flow time t0 = len / speed in ms: len_dm * 0.1 m / (speed / 3.6)    */
/* m/s * 1000 = len_dm * 360 / speed.  Floor, at least 1 ms, at most 2^31.  */
/* Fixed-time wait of approach e at its head v (the signal the vehicle      */
/* meets at the end of the road, Section 4.1): with cycle C and red time    */
/* R = C*(1000-green)/1000, an arrival uniform over the cycle waits R^2/(2C) */
/* on average; capped at T_max because a phase waiting longer than T_max   */
/* is given green (Fig. 3, "t_w > T_max").                                  */
/* ------------------------------------------------------------------------ */
void orc_edge_static(const orc_graph *g, const orc_params *p, uint32_t *t0, uint32_t *wf)
{
    for (uint32_t e = 0; e < g->m; ++e) {
        uint64_t t = (uint64_t)g->len_dm[e] * 360u / g->speed_kmh[e];
        if (t < 1) t = 1;
        if (t > COST_CAP) t = COST_CAP;
        t0[e] = (uint32_t)t;

        const uint32_t v = g->col[e];
        const uint64_t C = g->cycle_ms[v];
        if (C == 0) {
            wf[e] = 0;
        } else {
            const uint64_t red = C * (1000u - g->green_pm[e]) / 1000u;
            uint64_t w = red * red / (2 * C);
            if (w > p->t_max_ms) w = p->t_max_ms;
            wf[e] = (uint32_t)w;
        }
    }
}

/* Congestion: a road carrying more than theta vehicles is slowed in        */
/* proportion to its load, floor(t0 * load / theta); below that, t0.        */
static uint64_t travel_ms(uint32_t t0, uint32_t load, uint32_t theta)
{
    return load <= theta ? t0 : (uint64_t)t0 * load / theta;
}

/* ------------------------------------------------------------------------ */
/* Cost table (Section 4.2: Calc_Dens, Comp_Thres, Eval_Rout; Fig. 3).      */
/* A phase of an intersection is one incoming road; its queue is the road's */
/* load.  The preemptive rule gives green to the approach with the longest  */
/* queue (ties: the lowest road id) and to any approach whose queue exceeds */
/* Th_max; an empty queue never takes the green.  A road whose approach has */
/* green costs no signal wait.  Congestion: a road carrying more than the   */
/* threshold theta vehicles is slowed in proportion to its load.            */
/* ------------------------------------------------------------------------ */
void orc_cost_table(const orc_graph *g, const orc_params *p, const uint32_t *load,
                    const uint32_t *t0, const uint32_t *wf, uint32_t *cost, uint8_t *preempted)
{
    /* For every intersection, the approach with the longest non-empty queue. */
    uint32_t *best_edge = (uint32_t *)malloc(sizeof(uint32_t) * (g->n ? g->n : 1));
    for (uint32_t v = 0; v < g->n; ++v) best_edge[v] = U32_MAX;
    for (uint32_t e = 0; e < g->m; ++e) {         /* ascending e: first maximum wins */
        if (load[e] == 0) continue;
        const uint32_t v = g->col[e];
        if (best_edge[v] == U32_MAX || load[e] > load[best_edge[v]]) best_edge[v] = e;
    }
    for (uint32_t e = 0; e < g->m; ++e) {
        const uint32_t v = g->col[e];
        const int green = g->cycle_ms[v] > 0 && load[e] > 0 &&
                          (load[e] > p->th_max || best_edge[v] == e);
        if (preempted) preempted[e] = (uint8_t)green;
        const uint64_t wait = green ? 0 : wf[e];
        uint64_t c = travel_ms(t0[e], load[e], p->theta) + wait;
        if (c > COST_CAP) c = COST_CAP;
        cost[e] = (uint32_t)c;
    }
    free(best_edge);
}

/* ------------------------------------------------------------------------ */
/* Goal term (Section 4.2, Calc_Dist: distance from the current position to */
/* the destination).  Straight-line distance over the fastest speed in the  */
/* network, a lower bound on the remaining travel time:                      */
/*   h = floor(isqrt(dx^2 + dy^2) * k / 2^16),  k = floor(360 * 2^16 / vmax) */
/* vmax = 0 switches the term off.                                           */
/* ------------------------------------------------------------------------ */
uint64_t orc_goal(const orc_graph *g, const orc_params *p, uint32_t node, uint32_t dst)
{
    if (p->vmax_kmh == 0) return 0;
    const int64_t dx = (int64_t)g->x_dm[node] - g->x_dm[dst];
    const int64_t dy = (int64_t)g->y_dm[node] - g->y_dm[dst];
    const uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy);
    const uint64_t k = (uint64_t)360u * 65536u / p->vmax_kmh;
    return orc_isqrt(d2) * k >> 16;
}

/* ------------------------------------------------------------------------ */
/* Exact goal term (Section 4.2, Alg. 2 step 1: Calc_Dist computes the      */
/* distance from any node to the destination over the road network).  Here  */
/* the distance is the shortest free-flow travel time to dst, each road     */
/* weighted by its free-flow time t0 (the static part of its cost, so the   */
/* term never exceeds the true remaining cost).  Dijkstra from dst over the */
/* reversed roads, with a binary heap; sums are exact in 64 bits and        */
/* reported as min(sum, 0xFFFFFFFE); a node from which dst cannot be        */
/* reached gets 0xFFFFFFFF.                                                  */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t d; uint32_t v; } heap_item;

static void heap_push(heap_item *h, uint32_t *n, heap_item x)
{
    uint32_t i = (*n)++;
    h[i] = x;
    while (i > 0) {
        const uint32_t up = (i - 1) / 2;
        if (h[up].d <= h[i].d) break;
        const heap_item t = h[up]; h[up] = h[i]; h[i] = t;
        i = up;
    }
}

static heap_item heap_pop(heap_item *h, uint32_t *n)
{
    const heap_item top = h[0];
    h[0] = h[--(*n)];
    uint32_t i = 0;
    for (;;) {
        const uint32_t a = 2 * i + 1, b = 2 * i + 2;
        uint32_t s = i;
        if (a < *n && h[a].d < h[s].d) s = a;
        if (b < *n && h[b].d < h[s].d) s = b;
        if (s == i) break;
        const heap_item t = h[s]; h[s] = h[i]; h[i] = t;
        i = s;
    }
    return top;
}

void orc_goal_exact(const orc_graph *g, const orc_params *p, uint32_t dst, uint32_t *h)
{
    const uint32_t n = g->n, m = g->m;
    uint32_t *t0 = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *wf = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    orc_edge_static(g, p, t0, wf);
    /* reversed roads: for each node x, the roads u -> x, as (u, t0) */
    uint32_t *rp = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    uint32_t *ru = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *rw = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    for (uint32_t e = 0; e < m; ++e) rp[g->col[e] + 1]++;
    for (uint32_t x = 0; x < n; ++x) rp[x + 1] += rp[x];
    uint32_t *fill = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    memcpy(fill, rp, sizeof(uint32_t) * n);
    for (uint32_t u = 0; u < n; ++u)
        for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
            const uint32_t x = g->col[e];
            ru[fill[x]] = u;
            rw[fill[x]] = t0[e];
            fill[x]++;
        }
    uint64_t *dist = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint8_t *done = (uint8_t *)calloc(n, 1);
    heap_item *heap = (heap_item *)malloc(sizeof(heap_item) * (m + 2));
    uint32_t hn = 0;
    for (uint32_t v = 0; v < n; ++v) dist[v] = UINT64_MAX;
    dist[dst] = 0;
    heap_push(heap, &hn, (heap_item){0, dst});
    while (hn) {
        const heap_item it = heap_pop(heap, &hn);
        if (done[it.v]) continue;
        done[it.v] = 1;
        for (uint32_t i = rp[it.v]; i < rp[it.v + 1]; ++i) {
            const uint32_t u = ru[i];
            const uint64_t nd = it.d + rw[i];
            if (!done[u] && nd < dist[u]) {
                dist[u] = nd;
                heap_push(heap, &hn, (heap_item){nd, u});
            }
        }
    }
    for (uint32_t v = 0; v < n; ++v)
        h[v] = dist[v] == UINT64_MAX ? U32_MAX : (dist[v] > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)dist[v]);
    free(t0); free(wf); free(rp); free(ru); free(rw); free(fill); free(dist); free(done); free(heap);
}

/* Shortest free-flow route from src to dst (the Dijkstra baseline of the    */
/* paper's Table 1): from each node, the first out-road in road order that   */
/* lies on a shortest route, i.e. whose free-flow time equals the drop of   */
/* the exact goal term along it.  Returns the number of roads; 0 when dst    */
/* cannot be reached, when its free-flow time reaches the 2^32-2 cap (the    */
/* drops can no longer be told apart), or when the route has more than      */
/* max_len roads.                                                            */
uint32_t orc_shortest_route(const orc_graph *g, const orc_params *p, uint32_t src, uint32_t dst,
                            uint32_t max_len, uint32_t *path)
{
    uint32_t *h = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    uint32_t *t0 = (uint32_t *)malloc(sizeof(uint32_t) * (g->m + 1));
    uint32_t *wf = (uint32_t *)malloc(sizeof(uint32_t) * (g->m + 1));
    orc_goal_exact(g, p, dst, h);
    orc_edge_static(g, p, t0, wf);
    uint32_t len = 0, u = src;
    const int followable = h[src] < 0xFFFFFFFEu;
    while (followable && u != dst) {
        uint32_t next = U32_MAX;
        for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e)
            if ((uint64_t)t0[e] + h[g->col[e]] == h[u]) { next = e; break; }
        if (len == max_len) { len = 0; break; }
        path[len++] = next;      /* a node with a finite term always has such a road */
        u = g->col[next];
    }
    free(h); free(t0); free(wf);
    return len;
}

/* ------------------------------------------------------------------------ */
/* Time-dependent signals (Section 4.1, Fig. 3 signal block with the phases */
/* run in time).  Green windows: the approaches of an intersection with     */
/* cycle C take their greens in turn, in road order, each for               */
/* floor(C * green / 1000) ms; the first window starts at time 0 (the start */
/* of the call, when every vehicle departs) and each later one where the    */
/* previous ended, modulo C.                                                 */
/* ------------------------------------------------------------------------ */
void orc_signal_windows(const orc_graph *g, uint32_t *start, uint32_t *green)
{
    uint64_t *acc = (uint64_t *)calloc(g->n ? g->n : 1, sizeof(uint64_t));
    for (uint32_t e = 0; e < g->m; ++e) {
        const uint32_t v = g->col[e];
        const uint64_t C = g->cycle_ms[v];
        if (C == 0) { start[e] = green[e] = 0; continue; }
        const uint64_t len = C * g->green_pm[e] / 1000u;
        start[e] = (uint32_t)(acc[v] % C);
        green[e] = (uint32_t)len;
        acc[v] += len;
    }
    free(acc);
}

/* The wait of a vehicle reaching the signal at the end of road e at time   */
/* `arrival` (ms since the call's start): none inside the approach's green  */
/* window, else until the window opens again; an approach that would wait   */
/* longer than T_max is given the green then (Fig. 3, t_w > T_max).  A road */
/* whose approach holds the preemptive green (orc_cost_table) waits 0.       */
typedef struct {
    const uint32_t *travel;     /* [m] travel time of the road at the current loads (no wait) */
    const uint8_t *pre;         /* [m] the approach holds the preemptive green                */
    const uint32_t *wstart, *wgreen;   /* [m] its green window (orc_signal_windows)          */
} orc_timing;

static uint32_t timed_cost(const orc_graph *g, const orc_params *p, const orc_timing *tm, uint32_t e, uint64_t clock)
{
    const uint64_t travel = tm->travel[e];
    const uint64_t C = g->cycle_ms[g->col[e]];
    uint64_t wait = 0;
    if (C && !tm->pre[e]) {
        const uint64_t q = ((clock + travel) % C + C - tm->wstart[e]) % C;   /* phase from the window's opening */
        wait = q < tm->wgreen[e] ? 0 : C - q;
        if (wait > p->t_max_ms) wait = p->t_max_ms;
    }
    const uint64_t c = travel + wait;
    return c > COST_CAP ? COST_CAP : (uint32_t)c;
}

/* Travel part of the cost table: t0 while load <= theta, else floor(t0 * load / theta). */
static void travel_table(const orc_graph *g, const orc_params *p, const uint32_t *load, const uint32_t *t0,
                         uint32_t *travel)
{
    for (uint32_t e = 0; e < g->m; ++e) {
        const uint64_t x = travel_ms(t0[e], load[e], p->theta);
        travel[e] = x > COST_CAP ? COST_CAP : (uint32_t)x;
    }
}

uint32_t orc_timed_cost(const orc_graph *g, const orc_params *p, uint32_t e, uint64_t clock)
{
    const uint32_t m = g->m;
    uint32_t *t0 = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)), *wf = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *cost = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)), *tr = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *ws = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)), *wg = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint8_t *pre = (uint8_t *)malloc(m + 1);
    orc_edge_static(g, p, t0, wf);
    orc_cost_table(g, p, g->base_load, t0, wf, cost, pre);
    travel_table(g, p, g->base_load, t0, tr);
    orc_signal_windows(g, ws, wg);
    const orc_timing tm = {tr, pre, ws, wg};
    const uint32_t c = timed_cost(g, p, &tm, e, clock);
    free(t0); free(wf); free(cost); free(tr); free(ws); free(wg); free(pre);
    return c;
}

/* Desirability of a road from its reduced cost delta = cost + h(head) - h(tail):
 * eta = floor(2^26 / max(delta, 1)), clamped to [1, 65535]. */
uint32_t orc_eta(int64_t delta)
{
    const uint64_t d = delta < 1 ? 1 : (uint64_t)delta;
    uint64_t eta = ((uint64_t)1 << 26) / d;
    if (eta < 1) eta = 1;
    if (eta > 65535) eta = 65535;
    return (uint32_t)eta;
}

static uint64_t ipow(uint64_t b, uint32_t e)
{
    uint64_t r = 1;
    for (uint32_t i = 0; i < e; ++i) r *= b;
    return r;
}

/* Roulette over d weights: target = floor(r * T / 2^64) with T the weight
 * total; the choice is the first index whose inclusive prefix sum exceeds
 * the target.  Zero weights are never chosen. */
uint32_t orc_roulette(const uint64_t *w, uint32_t d, uint64_t r)
{
    uint64_t T = 0;
    for (uint32_t j = 0; j < d; ++j) T += w[j];
    const uint64_t target = (uint64_t)(((unsigned __int128)r * T) >> 64);
    uint64_t prefix = 0;
    for (uint32_t j = 0; j < d; ++j) {
        prefix += w[j];
        if (prefix > target) return j;
    }
    return d;   /* only reached when T == 0 */
}

/* Pheromone apply for one road (Section 4.2, Updt_Pher and Evap_Pher):
 * evaporate by rho (Q16), add the deposit scaled down by theta/load on a
 * congested road (MACO: congested roads attract less), clamp. */
uint32_t orc_apply_tau(const orc_params *p, uint32_t tau, uint64_t deposit, uint32_t load)
{
    const uint64_t dp = load <= p->theta ? deposit
                                         : (uint64_t)(((unsigned __int128)deposit * p->theta) / load);
    const uint64_t evap = (uint64_t)tau * (65536u - p->rho_q16) / 65536u;
    uint64_t t = evap + dp;
    if (t < p->tau_min_q16) t = p->tau_min_q16;
    if (t > p->tau_max_q16) t = p->tau_max_q16;
    return (uint32_t)t;
}

/* ------------------------------------------------------------------------ */
/* One ant (Section 4.2 Alg. 2 steps 4-6; Fig. 3 "else" branch).            */
/* From the current node, the candidates are the out-roads (CSR order) whose */
/* head has not been visited by this ant (Adj_Neigh).  Each has weight       */
/* tau^alpha * eta^beta; the roulette picks one.  No candidates = dead end.  */
/* The walk succeeds on reaching dst and fails after max_steps roads.       */
/* ------------------------------------------------------------------------ */
static uint8_t *g_visited;          /* scratch, n bytes, all zero between walks */
static uint32_t g_visited_n;

/* Goal term of node x: the exact row when the call uses one, else the
 * straight-line estimate. */
static int64_t goal_of(const orc_graph *g, const orc_params *p, const uint32_t *hrow, uint32_t x, uint32_t dst)
{
    return hrow ? (int64_t)hrow[x] : (int64_t)orc_goal(g, p, x, dst);
}

static int walk_impl(const orc_graph *g, const orc_params *p, const uint32_t *tau, const uint32_t *cost,
                     const orc_timing *tm, const uint32_t *hrow, uint32_t qid, uint32_t src, uint32_t dst,
                     uint32_t ant, uint32_t iter, uint32_t *path, uint32_t *len, uint32_t *cost_sum,
                     uint64_t *selections, uint64_t *wbuf)
{
    uint8_t *visited = g_visited;
    uint32_t u = src, s = 0, cs = 0;
    int ok = 0;
    visited[u] = 1;
    int64_t hu = goal_of(g, p, hrow, u, dst);
    for (;;) {
        if (s == p->max_steps) break;
        const uint32_t rs = g->row_ptr[u], d = g->row_ptr[u + 1] - rs;
        uint64_t T = 0;
        for (uint32_t j = 0; j < d; ++j) {
            const uint32_t e = rs + j, x = g->col[e];
            if (visited[x]) { wbuf[j] = 0; continue; }
            /* the road's cost: the table's, or with time-dependent signals the one at this ant's clock */
            const uint32_t ce = tm ? timed_cost(g, p, tm, e, cs) : cost[e];
            const int64_t delta = (int64_t)ce + goal_of(g, p, hrow, x, dst) - hu;
            wbuf[j] = ipow(tau[e], p->alpha) * ipow(orc_eta(delta), p->beta);
            T += wbuf[j];
        }
        if (T == 0) break;                                    /* dead end */
        const uint32_t j = orc_roulette(wbuf, d, draw64(p, qid, ant, iter, s));
        const uint32_t e = rs + j;
        path[s++] = e;
        *selections += 1;
        const uint64_t c = (uint64_t)cs + (tm ? timed_cost(g, p, tm, e, cs) : cost[e]);
        cs = c > PATH_COST_CAP ? PATH_COST_CAP : (uint32_t)c;
        u = g->col[e];
        visited[u] = 1;
        hu = goal_of(g, p, hrow, u, dst);
        if (u == dst) { ok = 1; break; }
    }
    /* clear the visited marks of this walk */
    visited[src] = 0;
    for (uint32_t i = 0; i < s; ++i) visited[g->col[path[i]]] = 0;
    *len = s;
    *cost_sum = cs;
    return ok;
}

static uint32_t max_out_degree(const orc_graph *g)
{
    uint32_t dmax = 0;
    for (uint32_t u = 0; u < g->n; ++u) {
        const uint32_t d = g->row_ptr[u + 1] - g->row_ptr[u];
        if (d > dmax) dmax = d;
    }
    return dmax;
}

static void ensure_visited(uint32_t n)
{
    if (g_visited_n < n) {
        free(g_visited);
        g_visited = (uint8_t *)calloc(n, 1);
        g_visited_n = n;
    }
}

int orc_walk(const orc_graph *g, const orc_params *p, const uint32_t *tau, const uint32_t *cost,
             uint32_t qid, uint32_t src, uint32_t dst, uint32_t ant, uint32_t iter,
             uint32_t *path, uint32_t *len, uint32_t *cost_sum, uint64_t *selections)
{
    ensure_visited(g->n);
    uint64_t *wbuf = (uint64_t *)malloc(sizeof(uint64_t) * (max_out_degree(g) + 1));
    uint32_t *hrow = NULL;
    if (p->flags & ORC_FLAG_GOAL_EXACT) {
        hrow = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
        orc_goal_exact(g, p, dst, hrow);
    }
    /* time-dependent signals: travel times and preemption at the sensed loads */
    uint32_t *t0 = NULL, *wf = NULL, *tc = NULL, *tr = NULL, *ws = NULL, *wg = NULL;
    uint8_t *pre = NULL;
    orc_timing tm_store, *tm = NULL;
    if (p->flags & ORC_FLAG_SIGNAL_TIMED) {
        const uint32_t m = g->m;
        t0 = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)); wf = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
        tc = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)); tr = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
        ws = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)); wg = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
        pre = (uint8_t *)malloc(m + 1);
        orc_edge_static(g, p, t0, wf);
        orc_cost_table(g, p, g->base_load, t0, wf, tc, pre);
        travel_table(g, p, g->base_load, t0, tr);
        orc_signal_windows(g, ws, wg);
        tm_store = (orc_timing){tr, pre, ws, wg};
        tm = &tm_store;
    }
    const int ok = walk_impl(g, p, tau, cost, tm, hrow, qid, src, dst, ant, iter, path, len, cost_sum, selections,
                             wbuf);
    free(wbuf);
    free(hrow);
    free(t0); free(wf); free(tc); free(tr); free(ws); free(wg); free(pre);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Parameter checks: -1 invalid, -2 outside the exact-integer range.        */
/* Every roulette total must fit 64 bits: each weight is below              */
/* 2^(alpha*bits(tau_max) + 16*beta), and a row holds at most 2^ceil(log2 d) */
/* of them.  Deposit totals must stay below 2^63.                           */
/* ------------------------------------------------------------------------ */
static uint32_t bit_length(uint64_t x) { uint32_t b = 0; while (x) { ++b; x >>= 1; } return b; }

static int check(const orc_graph *g, const uint32_t *src, const uint32_t *dst, uint32_t nv,
                 const orc_params *p)
{
    if (p->ants == 0 || p->max_steps == 0 || p->theta == 0) return -1;
    if (p->rho_q16 > 65536u || p->tau_min_q16 == 0) return -1;
    if (p->tau_min_q16 > p->tau0_q16 || p->tau0_q16 > p->tau_max_q16) return -1;
    if (p->mode > 1) return -1;
    for (uint32_t i = 0; i < nv; ++i)
        if (src[i] >= g->n || dst[i] >= g->n || src[i] == dst[i]) return -1;
    const uint32_t dmax = max_out_degree(g);
    const uint32_t lg = dmax <= 1 ? 0 : bit_length(dmax - 1);
    if ((uint64_t)p->alpha * bit_length(p->tau_max_q16) + 16ull * p->beta + lg > 64) return -2;
    const unsigned __int128 dep = (unsigned __int128)(p->mode == ORC_MODE_SHARED ? nv : 1) * p->ants * p->q_deposit;
    if (dep >> 63) return -2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One vehicle, one iteration: all its ants walk on the same pheromone and  */
/* cost table; the iteration-best ant is the successful one with the lowest */
/* (cost, ant index); it replaces the vehicle's best route when strictly    */
/* cheaper (the route output of Alg. 1).  Every successful ant k deposits   */
/* q_deposit / cost_k on each road of its path (Updt_Pher).                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_graph *g;
    const orc_params *p;
    uint32_t S;
    uint32_t *ant_path, *iter_path;
    uint64_t *wbuf;
    uint64_t steps;
    const orc_timing *tm;      /* time-dependent signals, or NULL */
} route_ctx;

static void vehicle_iteration(route_ctx *c, uint32_t qid, uint32_t src, uint32_t dst, uint32_t t,
                              const uint32_t *tau, const uint32_t *cost, const uint32_t *hrow, uint64_t *dep,
                              uint32_t *best_path, uint32_t *best_len, uint32_t *best_cost)
{
    const orc_params *p = c->p;
    uint64_t iter_key = UINT64_MAX;
    uint32_t iter_len = 0;
    for (uint32_t k = 0; k < p->ants; ++k) {
        uint32_t len, cs;
        if (!walk_impl(c->g, p, tau, cost, c->tm, hrow, qid, src, dst, k, t, c->ant_path, &len, &cs, &c->steps,
                       c->wbuf))
            continue;
        const uint64_t key = ((uint64_t)cs << 32) | k;
        if (key < iter_key) {
            iter_key = key;
            iter_len = len;
            memcpy(c->iter_path, c->ant_path, sizeof(uint32_t) * len);
        }
        const uint64_t d = p->q_deposit / cs;
        for (uint32_t i = 0; i < len; ++i) dep[c->ant_path[i]] += d;
    }
    if (iter_key != UINT64_MAX && (uint32_t)(iter_key >> 32) < *best_cost) {
        *best_cost = (uint32_t)(iter_key >> 32);
        *best_len = iter_len;
        memcpy(best_path, c->iter_path, sizeof(uint32_t) * iter_len);
    }
}

/* ------------------------------------------------------------------------ */
/* The whole run (Alg. 2 iterated).  Shared mode: all vehicles share one    */
/* pheromone vector and one load vector; per iteration: cost table from the */
/* load, every ant of every vehicle walks, best routes, deposit, evaporate  */
/* + apply (penalised by the load the ants saw), then the load becomes the  */
/* sensed load plus one for every vehicle whose best route uses the road    */
/* (MACO marker, Fig. 3 "Ph_road++").  Independent mode: each vehicle has a */
/* private pheromone vector and the load stays at the sensed value.         */
/* ------------------------------------------------------------------------ */
int orc_route(const orc_graph *g, const uint32_t *qid, const uint32_t *src, const uint32_t *dst,
              uint32_t nv, const orc_params *p,
              uint32_t *path_edges, uint32_t *path_len, uint32_t *cost_ms, uint64_t *steps_total,
              uint32_t *tau_out, uint32_t *load_out, uint32_t *best_hist)
{
    const int rc = check(g, src, dst, nv, p);
    if (rc) return rc;
    const uint32_t m = g->m, S = p->max_steps;
    ensure_visited(g->n);
    route_ctx c = {g, p, S, NULL, NULL, NULL, 0, NULL};
    c.wbuf = (uint64_t *)malloc(sizeof(uint64_t) * (max_out_degree(g) + 1));
    c.ant_path = (uint32_t *)malloc(sizeof(uint32_t) * S);
    c.iter_path = (uint32_t *)malloc(sizeof(uint32_t) * S);
    uint32_t *t0 = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *wf = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *cost = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *load = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint64_t *dep = (uint64_t *)malloc(sizeof(uint64_t) * (m + 1));
    const int shared = p->mode == ORC_MODE_SHARED;
    const uint32_t n_tau = shared ? 1 : nv;
    uint32_t *tau = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)n_tau * m + 1));

    /* Calc_Dist (Alg. 2 step 1), once per call: the exact goal row of each vehicle */
    uint32_t *hrows = NULL;
    if (p->flags & ORC_FLAG_GOAL_EXACT) {
        hrows = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)nv * g->n + 1));
        for (uint32_t v = 0; v < nv; ++v) orc_goal_exact(g, p, dst[v], hrows + (size_t)v * g->n);
    }
#define HROW(v) (hrows ? hrows + (size_t)(v) * g->n : NULL)

    orc_edge_static(g, p, t0, wf);
    for (uint32_t e = 0; e < m; ++e) load[e] = g->base_load[e];
    /* time-dependent signals: green windows, and per cost table the travel times and preemption */
    uint32_t *tr = NULL, *ws = NULL, *wg = NULL;
    uint8_t *pre = NULL;
    orc_timing tm_store;
    if (p->flags & ORC_FLAG_SIGNAL_TIMED) {
        tr = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)); ws = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
        wg = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1)); pre = (uint8_t *)malloc(m + 1);
        orc_signal_windows(g, ws, wg);
        tm_store = (orc_timing){tr, pre, ws, wg};
        c.tm = &tm_store;
    }
    for (size_t i = 0; i < (size_t)n_tau * m; ++i) tau[i] = p->tau0_q16;
    for (uint32_t v = 0; v < nv; ++v) { path_len[v] = 0; cost_ms[v] = U32_MAX; }

    if (shared) {
        for (uint32_t t = 0; t < p->iterations; ++t) {
            orc_cost_table(g, p, load, t0, wf, cost, pre);
            if (pre) travel_table(g, p, load, t0, tr);
            memset(dep, 0, sizeof(uint64_t) * m);
            for (uint32_t v = 0; v < nv; ++v) {
                vehicle_iteration(&c, qid[v], src[v], dst[v], t, tau, cost, HROW(v), dep,
                                  path_edges + (size_t)v * S, &path_len[v], &cost_ms[v]);
                if (best_hist) best_hist[(size_t)t * nv + v] = cost_ms[v];
            }
            for (uint32_t e = 0; e < m; ++e) tau[e] = orc_apply_tau(p, tau[e], dep[e], load[e]);
            if (!(p->flags & ORC_FLAG_NO_LOAD_UPDATE)) {
                for (uint32_t e = 0; e < m; ++e) load[e] = g->base_load[e];
                for (uint32_t v = 0; v < nv; ++v)
                    for (uint32_t i = 0; i < path_len[v]; ++i) load[path_edges[(size_t)v * S + i]] += 1;
            }
        }
    } else {
        orc_cost_table(g, p, load, t0, wf, cost, pre);
        if (pre) travel_table(g, p, load, t0, tr);
        for (uint32_t v = 0; v < nv; ++v) {
            uint32_t *tv = tau + (size_t)v * m;
            for (uint32_t t = 0; t < p->iterations; ++t) {
                memset(dep, 0, sizeof(uint64_t) * m);
                vehicle_iteration(&c, qid[v], src[v], dst[v], t, tv, cost, HROW(v), dep,
                                  path_edges + (size_t)v * S, &path_len[v], &cost_ms[v]);
                if (best_hist) best_hist[(size_t)t * nv + v] = cost_ms[v];
                for (uint32_t e = 0; e < m; ++e) tv[e] = orc_apply_tau(p, tv[e], dep[e], load[e]);
            }
        }
    }

    *steps_total = c.steps;
    if (tau_out) memcpy(tau_out, tau, sizeof(uint32_t) * (size_t)n_tau * m);
    if (load_out) memcpy(load_out, load, sizeof(uint32_t) * m);
    free(c.wbuf); free(c.ant_path); free(c.iter_path);
    free(t0); free(wf); free(cost); free(load); free(dep); free(tau); free(hrows); free(tr); free(ws); free(wg);
    free(pre);
#undef HROW
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Literal MACO-P vehicle loop (Section 4.1, Fig. 3), read for synchronous  */
/* ticks: at every tick each vehicle still travelling in a city moves one   */
/* road, all of them on the pheromone markers of the tick's start.          */
/*  - Candidates (Fig. 3: the adjacent nodes; the prose: among the paths     */
/*    leading to the destination): the out-roads whose head has a smaller   */
/*    exact goal term (orc_goal_exact) than the current node.  The term     */
/*    drops at every move, so a vehicle never revisits a node and reaches   */
/*    its destination unless the destination is out of reach.              */
/*  - Choice: the candidate with the least marker, ties to the lowest road  */
/*    id; when N_t, the vehicles of the city still travelling at the tick's */
/*    start, exceeds the threshold (theta here), the second least instead   */
/*    (when there are two candidates or more).                              */
/*  - Markers start at the sensed loads.  Every move adds one to the chosen */
/*    road and takes one from every other road of the city (Fig. 3,         */
/*    Ph_road++ and Ph_[N-road]--); with c_e moves along road e among M     */
/*    moves of the tick: marker <- max(0, marker + c_e - (M - c_e)).        */
/*  - A vehicle with no candidate (destination out of reach) stops without  */
/*    a route; after max_steps ticks the vehicles still travelling stop     */
/*    without a route.  Route cost = sum of the cost table at the sensed    */
/*    loads (orc_cost_table), as found.                                     */
/* city_of_node: [n] city of each node, or NULL for one city.  Outputs as   */
/* orc_route; marker_out [m] (may be NULL): markers after the last tick.    */
/* Returns 0, or -1 on invalid input.                                       */
/* ------------------------------------------------------------------------ */
int orc_greedy(const orc_graph *g, const uint32_t *src, const uint32_t *dst, uint32_t nv, const orc_params *p,
               const uint32_t *city_of_node, uint32_t *path_edges, uint32_t *path_len, uint32_t *cost_ms,
               uint64_t *steps_total, uint32_t *marker_out)
{
    const uint32_t n = g->n, m = g->m, S = p->max_steps;
    if (S == 0 || p->theta == 0) return -1;
    for (uint32_t v = 0; v < nv; ++v)
        if (src[v] >= n || dst[v] >= n || src[v] == dst[v]) return -1;
    uint32_t ncity = 1;
    if (city_of_node)
        for (uint32_t x = 0; x < n; ++x)
            if (city_of_node[x] + 1 > ncity) ncity = city_of_node[x] + 1;
    uint32_t *t0 = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *wf = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    uint32_t *cost = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
    uint32_t *moves = (uint32_t *)calloc(m + 1, sizeof(uint32_t));   /* c_e of the tick */
    uint32_t *h = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)nv * n + 1));
    uint32_t *node = (uint32_t *)malloc(sizeof(uint32_t) * (nv + 1));
    uint32_t *choice = (uint32_t *)malloc(sizeof(uint32_t) * (nv + 1));
    uint8_t *travelling = (uint8_t *)malloc(nv + 1);
    uint64_t *csum = (uint64_t *)calloc(nv + 1, sizeof(uint64_t));
    uint32_t *n_t = (uint32_t *)malloc(sizeof(uint32_t) * ncity);
    uint32_t *m_t = (uint32_t *)malloc(sizeof(uint32_t) * ncity);
    orc_edge_static(g, p, t0, wf);
    orc_cost_table(g, p, g->base_load, t0, wf, cost, NULL);
    for (uint32_t e = 0; e < m; ++e) mark[e] = g->base_load[e];
    for (uint32_t v = 0; v < nv; ++v) {
        orc_goal_exact(g, p, dst[v], h + (size_t)v * n);
        node[v] = src[v];
        travelling[v] = 1;
        path_len[v] = 0;
        cost_ms[v] = U32_MAX;
    }
    uint64_t steps = 0;
    for (uint32_t t = 0; t < S; ++t) {
        /* N_t per city: the vehicles still travelling at the tick's start */
        for (uint32_t c = 0; c < ncity; ++c) n_t[c] = m_t[c] = 0;
        uint32_t any = 0;
        for (uint32_t v = 0; v < nv; ++v)
            if (travelling[v]) { n_t[city_of_node ? city_of_node[src[v]] : 0]++; any = 1; }
        if (!any) break;
        /* every travelling vehicle chooses on the markers of the tick's start */
        for (uint32_t v = 0; v < nv; ++v) {
            choice[v] = U32_MAX;
            if (!travelling[v]) continue;
            const uint32_t *hv = h + (size_t)v * n;
            const uint32_t u = node[v], c = city_of_node ? city_of_node[u] : 0;
            uint32_t best = U32_MAX, second = U32_MAX;       /* road ids, ordered by (marker, road id) */
            for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                if (!(hv[g->col[e]] < hv[u])) continue;      /* not leading toward the destination */
                if (best == U32_MAX || mark[e] < mark[best]) { second = best; best = e; }
                else if (second == U32_MAX || mark[e] < mark[second]) second = e;
            }
            if (best == U32_MAX) { travelling[v] = 0; continue; }      /* destination out of reach */
            choice[v] = (n_t[c] > p->theta && second != U32_MAX) ? second : best;
        }
        /* move, count, and update the markers of each city */
        for (uint32_t v = 0; v < nv; ++v) {
            const uint32_t e = choice[v];
            if (e == U32_MAX) continue;
            path_edges[(size_t)v * S + path_len[v]++] = e;
            csum[v] += cost[e];
            moves[e]++;
            m_t[city_of_node ? city_of_node[node[v]] : 0]++;
            steps++;
            node[v] = g->col[e];
            if (node[v] == dst[v]) {
                travelling[v] = 0;
                cost_ms[v] = csum[v] > PATH_COST_CAP ? PATH_COST_CAP : (uint32_t)csum[v];
            }
        }
        for (uint32_t u = 0; u < n; ++u) {
            const uint32_t c = city_of_node ? city_of_node[u] : 0;
            for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                const int64_t x = mark[e] + (int64_t)moves[e] - (int64_t)(m_t[c] - moves[e]);
                mark[e] = x < 0 ? 0 : x;
                moves[e] = 0;
            }
        }
    }
    for (uint32_t v = 0; v < nv; ++v)
        if (travelling[v]) path_len[v] = 0;                  /* still travelling after max_steps ticks */
        else if (cost_ms[v] == U32_MAX) path_len[v] = 0;     /* stopped without a route */
    *steps_total = steps;
    if (marker_out)
        for (uint32_t e = 0; e < m; ++e) marker_out[e] = mark[e] > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)mark[e];
    free(t0); free(wf); free(cost); free(mark); free(moves); free(h); free(node); free(choice); free(travelling);
    free(csum); free(n_t); free(m_t);
    return 0;
}


/* ------------------------------------------------------------------------ */
/* Traffic simulation of the vehicles' trips (Section 5: vehicles drive     */
/* their routes at their own speeds, the preemptive signal rule of Fig. 3   */
/* applied at every signal they meet; the overall travel time).             */
/* Synchronous ticks of tick_ms; every vehicle with a route departs at time */
/* 0 from the start of its first road.  At tick k (t = k * tick_ms), from   */
/* the state at the tick's start, with N_e the vehicles on road e and Q_e   */
/* those stopped at its end:                                                */
/*  - a vehicle stopped at the end of e passes the head's signal when it is */
/*    green for e or when it has waited T_max there, and enters the next    */
/*    road of its route (the pass takes the tick); else it waits the tick;  */
/*  - green for e: the head has no signal, or t lies in e's green window    */
/*    (orc_signal_windows), or Q_e is the largest non-empty queue among the */
/*    head's approaches (ties: the lowest road id), or Q_e > Th_max;        */
/*  - a moving vehicle covers min(its speed, the road's) km/h for tick_ms,  */
/*    slowed to max(1, floor(speed * theta / N_e)) when N_e > theta; at the */
/*    end of its road it stops, or, at the end of its route, arrives at     */
/*    t + tick_ms.                                                          */
/* Positions count 1/360 dm, so v km/h covers v * tick_ms of them a tick.   */
/* ------------------------------------------------------------------------ */
int orc_simulate(const orc_graph *g, const orc_params *p, const uint32_t *path, uint32_t stride,
                 const uint32_t *path_len, const uint32_t *speed_kmh, uint32_t nv, uint32_t tick_ms,
                 uint32_t max_ticks, uint32_t *arrival_ms, uint32_t *wait_ms, uint32_t *ticks_run)
{
    if (tick_ms == 0 || p->theta == 0) return -1;
    uint32_t *tail = (uint32_t *)malloc(sizeof(uint32_t) * (g->m ? g->m : 1));
    for (uint32_t v = 0; v < g->n; ++v)
        for (uint32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) tail[e] = v;
    for (uint32_t i = 0; i < nv; ++i) {   /* routes: roads in range, each starting where the last ended */
        const uint32_t L = path_len[i];
        int ok = L <= stride && (L == 0 || speed_kmh[i] > 0);
        for (uint32_t r = 0; ok && r < L; ++r) {
            const uint32_t e = path[(size_t)i * stride + r];
            ok = e < g->m && (r == 0 || tail[e] == g->col[path[(size_t)i * stride + r - 1]]);
        }
        if (!ok) {
            free(tail);
            return -1;
        }
    }
    uint32_t *ws = (uint32_t *)malloc(sizeof(uint32_t) * (g->m ? g->m : 1));
    uint32_t *wg = (uint32_t *)malloc(sizeof(uint32_t) * (g->m ? g->m : 1));
    orc_signal_windows(g, ws, wg);
    uint32_t *N = (uint32_t *)calloc(g->m ? g->m : 1, sizeof(uint32_t));
    uint32_t *Q = (uint32_t *)calloc(g->m ? g->m : 1, sizeof(uint32_t));
    uint32_t *best = (uint32_t *)malloc(sizeof(uint32_t) * (g->n ? g->n : 1));
    uint32_t *road = (uint32_t *)calloc(nv ? nv : 1, sizeof(uint32_t));      /* index into the route */
    uint64_t *pos = (uint64_t *)calloc(nv ? nv : 1, sizeof(uint64_t));      /* 1/360 dm from the road's start */
    uint8_t *stopped = (uint8_t *)calloc(nv ? nv : 1, 1);
    uint8_t *active = (uint8_t *)calloc(nv ? nv : 1, 1);
    uint32_t *waited = (uint32_t *)calloc(nv ? nv : 1, sizeof(uint32_t));   /* at the current stop */
    uint32_t remaining = 0;
    for (uint32_t i = 0; i < nv; ++i) {
        arrival_ms[i] = U32_MAX;
        wait_ms[i] = 0;
        active[i] = path_len[i] > 0;
        remaining += active[i];
    }
    uint32_t k = 0;
    for (; k < max_ticks && remaining; ++k) {
        const uint64_t t = (uint64_t)k * tick_ms;
        memset(N, 0, sizeof(uint32_t) * g->m);
        memset(Q, 0, sizeof(uint32_t) * g->m);
        for (uint32_t i = 0; i < nv; ++i)
            if (active[i]) {
                const uint32_t e = path[(size_t)i * stride + road[i]];
                N[e]++;
                Q[e] += stopped[i];
            }
        for (uint32_t v = 0; v < g->n; ++v) best[v] = U32_MAX;
        for (uint32_t e = 0; e < g->m; ++e) {   /* ascending e: the first of equal queues wins */
            const uint32_t v = g->col[e];
            if (Q[e] > 0 && (best[v] == U32_MAX || Q[e] > Q[best[v]])) best[v] = e;
        }
        for (uint32_t i = 0; i < nv; ++i) {
            if (!active[i]) continue;
            const uint32_t *route = path + (size_t)i * stride;
            const uint32_t e = route[road[i]], head = g->col[e];
            if (stopped[i]) {
                const uint64_t C = g->cycle_ms[head];
                int green = C == 0 || best[head] == e || Q[e] > p->th_max;
                if (!green) green = ((t % C + C - ws[e]) % C) < wg[e];
                if (green || waited[i] >= p->t_max_ms) {
                    road[i]++;
                    pos[i] = 0;
                    stopped[i] = 0;
                    waited[i] = 0;
                } else {
                    waited[i] += tick_ms;
                    wait_ms[i] += tick_ms;
                }
                continue;
            }
            uint64_t v = speed_kmh[i] < g->speed_kmh[e] ? speed_kmh[i] : g->speed_kmh[e];
            if (N[e] > p->theta) {
                v = v * p->theta / N[e];
                if (v == 0) v = 1;
            }
            pos[i] += v * tick_ms;
            if (pos[i] >= (uint64_t)g->len_dm[e] * 360u) {
                if (road[i] + 1 == path_len[i]) {
                    const uint64_t a = t + tick_ms;
                    arrival_ms[i] = a > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)a;
                    active[i] = 0;
                    remaining--;
                } else {
                    pos[i] = (uint64_t)g->len_dm[e] * 360u;
                    stopped[i] = 1;
                    waited[i] = 0;
                }
            }
        }
    }
    *ticks_run = k;
    free(tail); free(ws); free(wg); free(N); free(Q); free(best); free(road); free(pos); free(stopped);
    free(active); free(waited);
    return 0;
}
