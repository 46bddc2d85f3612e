/*
 * gmacop.h -- C ABI of the GMACO-P routing library for AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Jindal & Bedi, "GMACO-P: GPU assisted Preemptive MACO algorithm
 * for enabling Smart Transportation" (arXiv 2010.14244).  The library runs
 * the data-parallel core of the method on one GPU: ant route construction
 * for every vehicle over a road graph (Section 4.1 Fig. 3 vehicle loop;
 * Section 4.2 Alg. 2 steps 4-6, Adj_Neigh / Eval_Rout), the preemptive
 * signal and congestion cost of every road (Alg. 2 steps 7-8, Calc_Dens /
 * Comp_Thres), and the pheromone and road-load update (Alg. 2 steps 9-10,
 * Updt_Pher / Evap_Pher; Fig. 3 "Ph_road++").  The three calls mirror the
 * host driver of Alg. 1 (allocate and copy in, launch, copy out, free),
 * except that the graph stays resident on the device between calls.
 *
 * Everything crossing this interface is an integer: times in milliseconds,
 * lengths in decimetres, speeds in km/h, pheromone in Q16.16 (65536 = 1.0).
 * Results are deterministic and identical on every run for the same inputs.
 *
 * Return codes: GMACOP_OK (0) or a negative GMACOP_E_* value.  A failed call
 * changes no state; gmacop_last_error() describes the last failure of the
 * calling thread.  "No route found" for a vehicle is a result, not an error.
 */
#ifndef GMACOP_H
#define GMACOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GMACOP_OK            0
#define GMACOP_E_INVAL      -1   /* malformed graph, query or parameter            */
#define GMACOP_E_RANGE      -2   /* parameters exceed the exact 64-bit integer range */
#define GMACOP_E_NOMEM      -3   /* device allocation failed                        */
#define GMACOP_E_DEVICE     -4   /* HIP runtime error                               */
#define GMACOP_E_UNSUPPORTED -5  /* valid input outside what the library handles    */

/* gmacop_params.mode */
#define GMACOP_MODE_SHARED      0u  /* all vehicles share pheromone and road loads      */
#define GMACOP_MODE_INDEPENDENT 1u  /* private pheromone per vehicle, loads frozen      */
#define GMACOP_MODE_GREEDY      2u  /* the literal MACO-P vehicle loop of Fig. 3: no ants;
                                       in synchronous ticks every vehicle still travelling
                                       takes, among the out-roads whose head has a smaller
                                       exact goal term (GMACOP_GOAL_EXACT), the one with
                                       the least marker (ties: lowest road id), or the
                                       second least when more than theta vehicles of its
                                       city are travelling; each move adds 1 to the chosen
                                       road's marker and takes 1 from every other road of
                                       the city (floored at 0); markers start at the
                                       sensed loads.  At most max_steps ticks; ants,
                                       iterations, alpha, beta, rho, tau and q_deposit are
                                       not used.  Route cost = the cost table at the
                                       sensed loads; gmacop_state_get's tau = the final
                                       markers                                          */

/* gmacop_params.flags */
#define GMACOP_NO_LOAD_UPDATE  1u   /* shared mode: keep loads at base_load             */
#define GMACOP_DEVICE_PTRS     2u   /* queries and result buffers are device pointers;
                                       the call returns without synchronising          */
#define GMACOP_TIME_KERNELS    4u   /* record a HIP event pair around every kernel
                                       launch, summed by gmacop_stats_get              */
#define GMACOP_HIP_GRAPH       8u   /* run the call's kernel sequence as a HIP graph,
                                       captured once and replayed while the call's
                                       arguments stay the same; needs a non-null
                                       stream; ignored with GMACOP_TIME_KERNELS        */
#define GMACOP_GOAL_EXACT     16u   /* goal term (Section 4.2, Alg. 2 step 1, Calc_Dist)
                                       = exact shortest free-flow time to the
                                       vehicle's destination (sum of each road's
                                       floor(len * 360 / speed) ms over the best road
                                       sequence; min(d, 2^32 - 2), 2^32 - 1 where the
                                       destination cannot be reached), computed on the
                                       device once per call, instead of the
                                       straight-line term (not in a router);
                                       vmax_kmh is then ignored.  Graphs under 2^24
                                       nodes (GMACOP_E_UNSUPPORTED otherwise)          */

#define GMACOP_RESUME         32u   /* shared mode: start from the pheromone and loads
                                       the graph holds (left by the previous call or
                                       set by gmacop_state_set) instead of tau0 and
                                       base_load, and from the best routes in `out`
                                       (the previous call's results, passed back
                                       unchanged) instead of none; with iter_offset =
                                       the iterations already run, I1 iterations then
                                       I - I1 resumed ones give the result of I in
                                       one call.  GMACOP_E_UNSUPPORTED in independent
                                       mode; GMACOP_E_INVAL for a held route longer
                                       than max_steps or with a road out of range
                                       (host buffers; device buffers are not checked,
                                       such roads are ignored)                          */

#define GMACOP_SIGNAL_TIMED   64u   /* time-dependent signals (Section 4.1, Fig. 3 signal
                                       block run in time): the approaches of an
                                       intersection with cycle C take their greens in
                                       turn, in road order, each for
                                       floor(C * green_pm / 1000) ms, the first from time
                                       0 of the call (every vehicle departs then); an
                                       ant's clock is its cost so far, and a road's cost
                                       is its travel time plus the wait from its arrival
                                       at the head's signal to the next green of its
                                       approach, capped at t_max_ms (Fig. 3
                                       "t_w > T_max"), none for the preemptive green.
                                       Served by the global-memory walker.  Not with
                                       GMACOP_MODE_GREEDY, in a router, or on graphs of
                                       2^24 nodes or more (GMACOP_E_UNSUPPORTED)        */

/* Opaque handle: the graph, its static per-road data and the pheromone / load
 * state on the device.  Owns all of its device memory. */
typedef struct gmacop_graph gmacop_graph;

/* Road network G(N, E) (Fig. 3) in CSR form.  All pointers are host memory,
 * read during gmacop_graph_create only (deep copy); the caller keeps them. */
typedef struct {
    uint32_t n_nodes;            /* n >= 2                                                   */
    uint32_t n_edges;            /* m >= 1                                                   */
    const uint32_t *row_ptr;     /* [n+1] out-roads of u are row_ptr[u] .. row_ptr[u+1]-1;
                                    row_ptr[0] = 0, non-decreasing, row_ptr[n] = m           */
    const uint32_t *col;         /* [m] head node of each road, < n, no self-loops           */
    const uint32_t *len_dm;      /* [m] length in decimetres, >= 1                           */
    const uint16_t *speed_kmh;   /* [m] free-flow speed, >= 1                                */
    const uint16_t *green_pm;    /* [m] green share of road e as an approach of its head
                                    node, per mille, <= 1000                                 */
    const uint32_t *cycle_ms;    /* [n] signal cycle of the node, 0 = no signal              */
    const int32_t *x_dm;         /* [n] planar coordinates, |x|, |y| < 2^30                  */
    const int32_t *y_dm;         /* [n]                                                      */
    const uint32_t *base_load;   /* [m] sensed vehicles on each road (Section 4.2: vehicle
                                    density from road sensors)                               */
    uint32_t n_instances;        /* number of disjoint cities packed in the CSR, >= 1        */
    const uint32_t *inst_node_off; /* [n_instances+1] node range of each city, or NULL when
                                    n_instances == 1; no road may cross two ranges           */
} gmacop_graph_desc;

/* One vehicle (Fig. 3: veh_i.present, veh_i.destin).  qid names the
 * vehicle's random stream: the same qid gives the same draws wherever the
 * vehicle sits in a batch.  qid 0xFFFFFFFF is reserved. */
typedef struct {
    uint32_t qid, src, dst;
} gmacop_od;

typedef struct {
    uint32_t ants;          /* ants per vehicle per iteration, >= 1                         */
    uint32_t iterations;    /* >= 0                                                         */
    uint32_t alpha, beta;   /* integer exponents of pheromone and heuristic                 */
    uint32_t max_steps;     /* roads an ant may take before it gives up, >= 1              */
    uint32_t rho_q16;       /* evaporation, Q16 (32768 = 0.5), <= 65536                     */
    uint32_t tau0_q16;      /* initial pheromone, tau_min <= tau0 <= tau_max                */
    uint32_t tau_min_q16;   /* >= 1                                                         */
    uint32_t tau_max_q16;
    uint64_t q_deposit;     /* deposit numerator, Q16.16 x ms: an ant with path cost c
                               deposits floor(q_deposit / c) on each road of its path       */
    uint32_t theta;         /* congestion threshold (Fig. 3 "N_t > threshold"), >= 1        */
    uint32_t th_max;        /* queue above which an approach takes the green (Fig. 3 Th_max) */
    uint32_t t_max_ms;      /* longest signal wait (Fig. 3 T_max)                           */
    uint32_t vmax_kmh;      /* speed of the straight-line goal term, 0 = off; at least the
                               fastest road speed keeps the term a lower bound              */
    uint32_t mode;          /* GMACOP_MODE_*                                                */
    uint32_t flags;         /* GMACOP_* flags                                               */
    uint64_t seed;          /* Philox key                                                   */
    uint32_t iter_offset;   /* added to the iteration number in every random counter       */
} gmacop_params;

/* Caller-owned outputs (host memory, or device memory with GMACOP_DEVICE_PTRS). */
typedef struct {
    uint32_t *path_edges;   /* [nq * max_steps] best route of vehicle i in row i, as road
                               ids; entries past path_len[i] are unspecified               */
    uint32_t *path_len;     /* [nq] roads on the best route, 0 = no route found            */
    uint32_t *cost_ms;      /* [nq] cost of the best route as found, 0xFFFFFFFF = none      */
    uint64_t *steps_total;  /* [1] roulette selections executed by all ants                 */
} gmacop_result;

/* Build the device-resident graph (Alg. 1 steps 1-2).  Validates the CSR and
 * attributes (GMACOP_E_INVAL), copies everything to the current HIP device
 * and derives each road's free-flow time and fixed-time signal wait on the
 * device.  On success *out owns the graph; on failure *out is NULL. */
int gmacop_graph_create(const gmacop_graph_desc *desc, gmacop_graph **out);

/* Route nq vehicles (Alg. 1 step 3 and Alg. 2, iterated params->iterations
 * times).  Work is ordered on hip_stream (a hipStream_t; NULL = the null
 * stream).  Pheromone starts at tau0 and road loads at base_load on every
 * call.  GMACOP_MODE_SHARED: all vehicles deposit on one pheromone vector and
 * the loads follow the vehicles' best routes.  GMACOP_MODE_INDEPENDENT: every
 * vehicle has its own pheromone, loads stay at base_load, and a vehicle's
 * result does not depend on the other vehicles of the batch (at most 4095
 * iterations).  Without GMACOP_DEVICE_PTRS, q and out are host memory and the call
 * returns once the results are in them (Alg. 1 step 4).  With it, q and out
 * are device memory, the call only enqueues, and the caller synchronises the
 * stream before reading; q must stay valid until then.
 * Errors: GMACOP_E_INVAL (src/dst out of range, src == dst, src and dst in
 * different cities, reserved qid, a parameter outside its documented range),
 * GMACOP_E_RANGE (alpha*bits(tau_max) + 16*beta + ceil(log2(max out-degree))
 * > 64, or the deposit total could reach 2^63), GMACOP_E_UNSUPPORTED (a node
 * with more than 32 out-roads), GMACOP_E_NOMEM, GMACOP_E_DEVICE.
 * One call at a time per graph handle. */
int gmacop_route_batch(gmacop_graph *g, const gmacop_od *q, uint32_t nq, const gmacop_params *p,
                       gmacop_result *out, void *hip_stream);

/* Bytes of device workspace gmacop_route_batch_noalloc may use: one static
 * array of this size per GPU, held from the library's first use of that GPU
 * until the process ends. */
#define GMACOP_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call and the same results as gmacop_route_batch, with every per-call
 * buffer (ant paths, per-vehicle keys and results, the walkers' work lists
 * and visited words, independent-mode pheromone rows) carved out of the
 * library's static per-GPU workspace of GMACOP_NOALLOC_SCRATCH_BYTES.  It
 * calls no hipMalloc, hipFree or other allocating routine; the graph must
 * have been created (and its state allocated) by gmacop_graph_create.
 * Differences from gmacop_route_batch:
 *  - GMACOP_HIP_GRAPH and GMACOP_TIME_KERNELS are rejected (GMACOP_E_INVAL);
 *  - the walkers of one iteration run one after the other on hip_stream;
 *  - a call whose workspace exceeds GMACOP_NOALLOC_SCRATCH_BYTES returns
 *    GMACOP_E_NOMEM and changes nothing (the message gives the size needed);
 *    graphs of 2^24 nodes or more return GMACOP_E_UNSUPPORTED;
 *  - gmacop_vehicle_tau_get is not available after it (GMACOP_E_INVAL).
 * Every call on one GPU, from any graph handle or thread, shares that GPU's
 * workspace and finds the previous call's contents in it; calls that overlap
 * on one GPU (on different streams or threads) race and must not be made.
 * Without GMACOP_DEVICE_PTRS the call synchronises hip_stream before it
 * returns; with it, the results are ready once hip_stream reaches them and
 * the next call on the GPU may reuse the workspace only after that. */
int gmacop_route_batch_noalloc(gmacop_graph *g, const gmacop_od *q, uint32_t nq, const gmacop_params *p,
                               gmacop_result *out, void *hip_stream);

/* Shared-mode state after the last gmacop_route_batch on this graph: the
 * pheromone and road load of every road (host arrays of n_edges entries,
 * either may be NULL).  Synchronises hip_stream. */
int gmacop_state_get(gmacop_graph *g, uint32_t *tau_q16, uint32_t *load, void *hip_stream);

/* Replace the shared-mode state the graph holds (host arrays of n_edges
 * entries; either may be NULL): the pheromone and the current road loads a
 * call with GMACOP_RESUME starts from.  Synchronises hip_stream. */
int gmacop_state_set(gmacop_graph *g, const uint32_t *tau_q16, const uint32_t *load, void *hip_stream);

/* A new epoch of sensed loads (Section 4.2: vehicle densities from road
 * sensors): base_load (host, n_edges entries) replaces the graph's sensed
 * loads for every later gmacop_route_batch call (the loads a call starts
 * from, and the base of its load update).  Synchronises hip_stream. */
int gmacop_set_base_load(gmacop_graph *g, const uint32_t *base_load, void *hip_stream);

/* Independent mode: pheromone of the vehicle at batch position `vehicle` of
 * the last gmacop_route_batch call on this graph, after its last iteration
 * (host array of n_edges entries).  GMACOP_E_INVAL if the last call was not
 * in independent mode or had no such vehicle.  Synchronises hip_stream. */
int gmacop_vehicle_tau_get(gmacop_graph *g, uint32_t vehicle, uint32_t *tau_q16, void *hip_stream);

/* Calc_Dist (Section 4.2, Alg. 2 step 1) on its own: the exact goal term of
 * GMACOP_GOAL_EXACT for nd destinations.  h (host, nd * n_nodes entries) row
 * i gets, for every node, the shortest free-flow time to dst[i] in ms (each
 * road weighted t0 = max(1, min(2^31, floor(len * 360 / speed)))),
 * min(d, 2^32 - 2), and 0xFFFFFFFF for nodes that cannot reach dst[i],
 * including every node of another city.  Synchronous on hip_stream; uses
 * temporary device memory.  GMACOP_E_INVAL for a destination out of range. */
int gmacop_goal_rows(gmacop_graph *g, const uint32_t *dst, uint32_t nd, uint32_t *h, void *hip_stream);

/* The shortest free-flow route of each query (the Dijkstra baseline the paper
 * compares against in Table 1): at every node the first out-road in road
 * order that lies on a shortest route to q[i].dst.  out (host buffers, as in
 * gmacop_route_batch with max_steps entries per row): path_len[i] roads
 * (0 when the destination cannot be reached, its free-flow time reaches
 * 2^32 - 2, or the route has more than max_steps roads), cost_ms[i] its
 * free-flow time (0xFFFFFFFF when path_len is 0), steps_total the sum of
 * path_len.  Errors as gmacop_route_batch's query checks.  Synchronous; uses
 * temporary device memory. */
int gmacop_shortest_routes(gmacop_graph *g, const gmacop_od *q, uint32_t nq, uint32_t max_steps,
                           gmacop_result *out, void *hip_stream);

/* Traffic simulation of trips along given routes (Section 5: vehicles drive
 * their routes at their own speeds and the preemptive signal rule of Fig. 3
 * applies at every signal they meet; the overall travel time of Table 1).
 * Synchronous ticks of tick_ms; every vehicle with a route departs at time 0
 * from the start of its first road.  A moving vehicle covers min(its speed,
 * the road's) km/h per tick, slowed to max(1, floor(v * theta / N)) when its
 * road carries N > p->theta vehicles; at the end of a road it stops, at the
 * end of its route it arrives.  A stopped vehicle passes the next tick when
 * its approach is green -- the head has no signal, or the tick's start time
 * lies in the approach's green window (the windows of GMACOP_SIGNAL_TIMED),
 * or its queue is the largest non-empty one at the intersection (ties: the
 * lowest road id), or its queue exceeds p->th_max -- or once it has waited
 * p->t_max_ms; the crossing takes the tick.  Only theta, th_max and t_max_ms
 * of p are used; the sensed loads are not (the vehicles themselves load the
 * roads).
 *
 * Scenarios: vehicles scen_off[b] .. scen_off[b+1]-1 form scenario b (b <
 * nscen), simulated on their own (one workgroup each), so many runs of the
 * same network go in one call.  Host arrays: path[v * stride + r] the r-th
 * road of vehicle v's route (roads in range, each starting at the node where
 * the previous one ends), path_len[v] <= stride (0: no route, the vehicle
 * stays out), speed_kmh[v] >= 1 when it has a route, scen_off[nscen + 1]
 * (scen_off[0] = 0, non-decreasing).  Outputs (host): arrival_ms[v] (ms;
 * 0xFFFFFFFF without a route or when max_ticks ticks ended first), wait_ms[v]
 * (ms stopped at signals), ticks_run[b].  GMACOP_E_INVAL for any check above,
 * p->theta = 0 or tick_ms = 0, before any device work.  Synchronous on
 * hip_stream; uses temporary device memory (road counts in LDS when 8 bytes
 * per road fit, else nscen * 8 bytes per road, at most 16 GiB:
 * GMACOP_E_NOMEM beyond). */
int gmacop_simulate(gmacop_graph *g, const gmacop_params *p, const uint32_t *path, uint32_t stride,
                    const uint32_t *path_len, const uint32_t *speed_kmh, const uint32_t *scen_off, uint32_t nscen,
                    uint32_t tick_ms, uint32_t max_ticks, uint32_t *arrival_ms, uint32_t *wait_ms,
                    uint32_t *ticks_run, void *hip_stream);

/* Work counters and kernel times accumulated over gmacop_route_batch calls
 * since the last reset.  Kernel index: 0 = walk phase (tour construction and
 * deposit, all walkers of an iteration), 1 = best-route reduction, 2 =
 * pheromone/load update, 3 = signal and cost table, 4 = the LDS walkers of an
 * iteration (cities staged in on-chip memory), 5 = the global-memory walker
 * of an iteration, 6 = the exact goal search of a call (GMACOP_GOAL_EXACT).  ms[] is filled only for calls made with
 * GMACOP_TIME_KERNELS (times from HIP events on the stream each kernel runs
 * on).  walker_*[k]: the same counters per walker kind, k = 0 LDS walkers,
 * 1 global-memory walker, 2 first walker (graphs of 2^24 nodes or more). */
typedef struct {
    uint64_t launches[7];
    double ms[7];
    uint64_t selections;     /* roulette selections (one per road an ant takes)       */
    uint64_t candidates;     /* out-roads examined at those selections                */
    uint64_t arrivals;       /* ants that reached their destination                   */
    uint64_t deposit_roads;  /* roads deposited on by arriving ants                   */
    uint64_t longest_walks;  /* sum over walk launches of the longest ant's road count   */
    uint64_t walker_selections[3];
    uint64_t walker_candidates[3];
    uint64_t walker_arrivals[3];
    uint64_t walker_deposit_roads[3];
} gmacop_stats;

/* Copy the counters into *s (synchronises hip_stream); reset them when reset
 * is non-zero. */
int gmacop_stats_get(gmacop_graph *g, gmacop_stats *s, int reset, void *hip_stream);

/* ---- continuous batching ----
 * A router serves a stream of route queries on a resident graph: every query
 * is an independent-mode run of params->iterations iterations (Section 4.2,
 * Alg. 2 per vehicle), and queries are admitted while others are in flight.
 * Each in-flight query owns a slot (its pheromone, deposits, ant paths and
 * best route on the device); a step admits new queries into free slots,
 * advances every in-flight query by one iteration in one batch of kernels,
 * and returns the queries that completed.  A query's result depends only on
 * the query (its qid keys its random stream): it is identical whatever else
 * is in flight, and identical to gmacop_route_batch in independent mode. */
typedef struct gmacop_server gmacop_server;

/* Create a router on g (which must outlive it).  The number of slots is
 * max_slots, or fewer if the per-slot device memory times the slots would
 * exceed mem_budget_bytes (0: half of the device memory free now); the graph
 * must have fewer than 2^24 nodes.  Loads are frozen at the sensed loads.
 * Of params->flags only GMACOP_TIME_KERNELS is used; GMACOP_GOAL_EXACT is
 * rejected with GMACOP_E_UNSUPPORTED.
 * Errors: GMACOP_E_INVAL / E_RANGE as gmacop_route_batch, GMACOP_E_NOMEM when
 * not even one slot fits, GMACOP_E_UNSUPPORTED for 0 or more than 4095
 * iterations. */
int gmacop_server_create(gmacop_graph *g, const gmacop_params *p, uint32_t max_slots, uint64_t mem_budget_bytes,
                         gmacop_server **out);

/* Slots, slots in use, device bytes per slot (any pointer may be NULL). */
int gmacop_server_info(const gmacop_server *s, uint32_t *slots, uint32_t *active, uint64_t *bytes_per_slot);

/* One step.  On entry *n_admit is the number of queries in admit (host);
 * the first min(*n_admit, free slots) are admitted and *n_admit returns how
 * many.  Every in-flight query then runs one iteration.  Queries that ran
 * their last iteration are returned in order of slot: done_qid[i],
 * done_len[i] (0 = no route), done_cost[i] (0xFFFFFFFF = none) and the route
 * in done_paths[i * max_steps ...] (host buffers of done_cap entries; done_cap
 * must cover every query finishing in the step, at most the slot count);
 * *n_done returns their number.  Synchronous on hip_stream.
 * Argument errors (GMACOP_E_INVAL) are found before anything changes.  A step
 * that fails after them (GMACOP_E_DEVICE, GMACOP_E_NOMEM) drops every query in
 * flight and admits none (*n_admit and *n_done return 0): the router is empty
 * afterwards and the caller resubmits what it still needs. */
int gmacop_server_step(gmacop_server *s, const gmacop_od *admit, uint32_t *n_admit, uint32_t *done_qid,
                       uint32_t *done_len, uint32_t *done_cost, uint32_t *done_paths, uint32_t done_cap,
                       uint32_t *n_done, void *hip_stream);

/* A new epoch of sensed loads for the router (host, n_edges entries): its
 * frozen loads and road costs follow them from the next step on, for the
 * queries in flight as for those admitted later (a query admitted after the
 * call is routed as gmacop_route_batch in independent mode on a graph whose
 * base_load is this array).  The graph's own sensed loads are unchanged.
 * Call between steps; synchronises hip_stream. */
int gmacop_server_set_base_load(gmacop_server *s, const uint32_t *base_load, void *hip_stream);

/* Free the router's device memory (not the graph).  NULL-safe. */
void gmacop_server_release(gmacop_server *s);

/* Free the graph and all of its device memory (Alg. 1 step 5).  NULL-safe. */
void gmacop_release(gmacop_graph *g);

/* Message for the last failed call on this thread ("" if none). */
const char *gmacop_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GMACOP_H */
