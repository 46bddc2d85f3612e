// gmacop.hip -- GMACO-P routing hot path for AMD Instinct MI355X (gfx950).
//
// Method: Jindal & Bedi, "GMACO-P: GPU assisted Preemptive MACO algorithm for
// enabling Smart Transportation" (arXiv 2010.14244), Section 4.1 (Fig. 3,
// MACO-P vehicle loop) and Section 4.2 (Alg. 1 host driver, Alg. 2 kernel
// steps).  One iteration of the method is four kernels on one stream:
//
//   k_walk  one lane per ant: candidate roads of the current node (Adj_Neigh),
//           weight tau^alpha * eta^beta with eta from the road cost and the
//           straight-line goal term (Calc_Dist, Eval_Rout), Philox4x32-10
//           draw, roulette pick; on arrival the ant deposits on its path
//           (Updt_Pher) and offers its (cost, ant) key to its vehicle.
//   k_best  one wave per vehicle: iteration-best ant replaces the vehicle's
//           best route when strictly cheaper; road use counts for the load.
//   k_edge  one lane per road: evaporate + congestion-penalised deposit +
//           clamp (Evap_Pher), new load = sensed load + routed vehicles.
//   k_cost  one lane per intersection: the preemptive signal rule over its
//           approaches (Calc_Dens, Comp_Thres) and the cost of every
//           approach road for the next iteration.
//
// All arithmetic is integer with explicitly stated floors, so results do not
// depend on thread scheduling: deposits and load counts are integer atomic
// sums, the best ant is an atomic minimum of a packed (cost, ant) key.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gmacop.h"

namespace {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------

thread_local std::string t_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(GMACOP_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr uint32_t kNoCost = 0xFFFFFFFFu;
constexpr uint32_t kPathCostCap = 0xFFFFFFFEu;
constexpr uint32_t kRoadCostCap = 1u << 31;
constexpr uint64_t kNoKey = ~0ull;
constexpr int kWave = 64;
constexpr uint32_t kMaxDegree = 32;
constexpr size_t kStaticLds = 256;   // static LDS of the walker kernels (block aggregates), kept out of the dynamic budget
constexpr int kLdsClasses = 6;       // LDS walker classes: 1..3 k_walk_ldsr, 4..6 k_walk_lds (three size tiers each)
constexpr bool is_road_class(uint32_t c) { return c >= 1 && c <= 3; }
constexpr uint64_t kGlbWordsBudget = 4ull << 30;   // bytes of per-slot visited words of k_walk_glb
constexpr uint32_t kLdsBitsetMaxNodes = 4096;   // 512 B of visited bits per ant in LDS
// Work counters on the device: [0] selections, [1] candidates examined, [2] arrivals, [3] roads
// deposited on, [4] sum over iterations of the longest walk; then four per walker kind (the same
// first four quantities) at kWalkerCounters + 4 * kind.
constexpr int kWalkerCounters = 5;
constexpr int kCounters = kWalkerCounters + 4 * 3;
constexpr int kKindLds = 0, kKindGlb = 1, kKindFirst = 2;
constexpr int kTimedKernels = 7;   // walk phase, best route, update, cost table, LDS walkers, global walker,
                                   // exact goal search

// ---------------------------------------------------------------------------
// device arithmetic
// ---------------------------------------------------------------------------

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies, the key advanced by the Weyl constants between rounds.  Returns
// (x1 << 32) | x0 of the output block.
__device__ __forceinline__ uint64_t philox_u64(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;   // one 32x32->64 multiply each
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return ((uint64_t)c1 << 32) | c0;
}

// The same generator advanced a few rounds at a time (rounds R0..R1-1 of the
// ten; key words k0, k1 as given to round 0), so that a walker can spread one
// draw over several steps.  The empty asm keeps the rounds where they are
// written instead of letting the compiler move them next to their first use.
struct PhiloxState {
    uint32_t c0, c1, c2, c3;
};

template <int R0, int R1>
__device__ __forceinline__ void philox_rounds(PhiloxState &x, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = R0; r < R1; ++r) {
        const uint32_t kr0 = k0 + (uint32_t)r * 0x9E3779B9u, kr1 = k1 + (uint32_t)r * 0xBB67AE85u;
        const uint64_t p0 = (uint64_t)0xD2511F53u * x.c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x.c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x.c1 ^ kr0, n2 = (uint32_t)(p0 >> 32) ^ x.c3 ^ kr1;
        x.c0 = n0;
        x.c1 = (uint32_t)p1;
        x.c2 = n2;
        x.c3 = (uint32_t)p0;
    }
    if (R1 > R0) asm volatile("" : "+v"(x.c0), "+v"(x.c1), "+v"(x.c2), "+v"(x.c3));
}

// floor(sqrt(ex^2 + ey^2)) for |ex|, |ey| < 2^31.  Below 2^44 (distances
// under 2^22 dm) the single-precision estimate formed from ex and ey
// themselves -- both exact in float there, two rounded operations, then a
// square root within one ulp -- is within 0.75 of the root, so one step each
// way from the exact integer square gives the floor.  Farther apart, the
// estimate from the rounded sum is corrected by exact integer loops.
__device__ __forceinline__ uint32_t isqrt_dist(int32_t ex, int32_t ey)
{
    const uint64_t x = (uint64_t)((int64_t)ex * ex) + (uint64_t)((int64_t)ey * ey);
    if (x < (1ull << 44)) {
        const float fx = (float)ex, fy = (float)ey;
        const uint32_t s = (uint32_t)__builtin_amdgcn_sqrtf(__fmaf_rn(fx, fx, fy * fy));
        const uint64_t s2 = (uint64_t)s * s;
        return s2 > x ? s - 1 : (s2 + 2ull * s + 1 <= x ? s + 1 : s);
    }
    uint64_t s = (uint64_t)__fsqrt_rn((float)x);
    while (s * s > x) --s;
    while ((s + 1) * (s + 1) <= x) ++s;
    return (uint32_t)s;
}

// Straight-line time-to-go from (x, y) to the destination at vmax:
// floor(isqrt(dx^2 + dy^2) * kgoal / 2^16), kgoal = floor(360 * 2^16 / vmax).
// Coordinates are below 2^30 in magnitude, so the differences fit 32 bits.
__device__ __forceinline__ int64_t goal_ms(int32_t x, int32_t y, int32_t dx, int32_t dy, uint32_t kgoal)
{
    if (kgoal == 0) return 0;
    return (int64_t)(((uint64_t)isqrt_dist(x - dx, y - dy) * kgoal) >> 16);
}

// eta = clamp(floor(2^26 / max(delta, 1)), 1, 65535).  On (1024, 2^26] the
// quotient is below 2^16, so a single-precision reciprocal (within one ulp of
// the rounded divisor) puts the estimate within 0.02 of it, and one step each
// way from the exact remainder gives the floor.  Divisors above 2^26 give 1,
// as 2^26 does.
__device__ __forceinline__ uint32_t eta_of(int64_t delta)
{
    const uint32_t d = delta < 1025 ? 1025u : delta > (int64_t(1) << 26) ? (1u << 26) : (uint32_t)delta;
    uint32_t q = (uint32_t)(__builtin_amdgcn_rcpf((float)d) * 67108864.0f);
    const int32_t r = (int32_t)((1u << 26) - q * d);
    q = r < 0 ? q - 1 : (r >= (int32_t)d ? q + 1 : q);
    return delta <= 1024 ? 65535u : q;
}

__device__ __forceinline__ uint64_t ipow_u64(uint64_t b, uint32_t e)
{
    uint64_t r = 1;
    for (uint32_t i = 0; i < e; ++i) r *= b;
    return r;
}

// Evaporation without deposit, k times: x <- max(tau_min, floor(x (65536 - rho) / 65536)).
__device__ __forceinline__ uint32_t evaporate_k(uint32_t tau, uint32_t k, uint32_t rho, uint32_t tau_min)
{
    for (uint32_t i = 0; i < k && tau > tau_min; ++i) {
        const uint64_t t = ((uint64_t)tau * (65536u - rho)) >> 16;
        tau = t < tau_min ? tau_min : (uint32_t)t;
    }
    return tau;
}

// Pheromone as the walkers read it.  Shared mode: one dense vector.
// Independent mode: every vehicle slot keeps a lazy vector; the entry of a
// road packs tau (bits 0-31), the iteration it holds for (bits 32-43) and
// the call generation (bits 44-63).  An entry of another generation was
// never deposited on in this call and holds the common sequence E^t(tau0);
// a stored value evaporates forward on read.
constexpr uint32_t kGenBits = 20;
constexpr uint32_t kGenMask = (1u << kGenBits) - 1;
constexpr uint32_t kLazyIterMax = 4095;

struct PherView {
    const uint32_t *dense;    // shared mode, [m]
    const uint64_t *lazy;     // independent mode, [slots][m]
    const uint32_t *gen;      // current call generation (device)
    const uint32_t *slot_t;   // serving: iteration of each slot (else NULL: one iteration for all)
    const uint32_t *slot_gen; // serving: generation of each slot (else NULL: *gen)
    uint32_t m, tau0, rho, tau_min;
};

__device__ __forceinline__ uint32_t slot_iter(const PherView &pv, uint32_t v, uint32_t t)
{
    return pv.slot_t ? pv.slot_t[v] : t;
}

struct PherRead {
    const uint32_t *dense;
    const uint64_t *lazy;     // this slot's row
    uint32_t gen, t, tau_def, rho, tau_min;

    __device__ __forceinline__ uint32_t operator()(uint32_t e) const
    {
        if (dense) return dense[e];
        const uint64_t x = lazy[e];
        if ((uint32_t)(x >> 44) != gen) return tau_def;
        const uint32_t ts = (uint32_t)(x >> 32) & 0xFFFu;
        return evaporate_k((uint32_t)x, t - ts, rho, tau_min);
    }
};

// View of slot v at iteration t (t counts from 0 within the call).
__device__ __forceinline__ PherRead pher_at(const PherView &pv, uint32_t v, uint32_t t)
{
    t = slot_iter(pv, v, t);
    PherRead r{pv.dense, nullptr, 0, t, 0, pv.rho, pv.tau_min};
    if (!pv.dense) {
        r.lazy = pv.lazy + (size_t)v * pv.m;
        r.gen = (pv.slot_gen ? pv.slot_gen[v] : *pv.gen) & kGenMask;
        r.tau_def = evaporate_k(pv.tau0, t, pv.rho, pv.tau_min);
    }
    return r;
}

// Deposit accumulators.  Shared mode: one vector.  Independent mode: one per
// slot, with a list of the roads that received a deposit this iteration.
struct DepView {
    uint64_t *dep;            // [m] or [slots][m]
    uint32_t *touched;        // [slots][cap] (independent mode)
    uint32_t *touched_n;      // [slots]
    uint32_t m, cap, indep;

    __device__ __forceinline__ void add(uint32_t v, uint32_t e, uint64_t d) const
    {
        if (!indep) {
            atomicAdd((unsigned long long *)&dep[e], (unsigned long long)d);
            return;
        }
        const unsigned long long old = atomicAdd((unsigned long long *)&dep[(size_t)v * m + e], (unsigned long long)d);
        if (old == 0) {
            const uint32_t i = atomicAdd(&touched_n[v], 1u);
            if (i < cap) touched[(size_t)v * cap + i] = e;
        }
    }
};

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

struct EdgeInitArgs {
    uint32_t m, tau0, t_max, resume;   // resume: keep the current pheromone and load
    const uint32_t *col, *len_dm, *cycle, *base_load;
    const uint16_t *speed, *green;
    uint32_t *t0, *wf, *tau, *load, *cnt;
    uint64_t *dep;
    uint32_t *mir;             // road records of the global walker (8 words per road) or NULL
};

// Per road: free-flow time t0 = floor(len * 360 / speed) in [1, 2^31];
// fixed-time wait at the head signal wf = min(T_max, floor(red^2 / (2C)))
// with red = floor(C * (1000 - green) / 1000); fresh pheromone and load, or
// (resume) the pheromone and load already held, copied to the global
// walker's records.
__global__ void k_init_edges(EdgeInitArgs a)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.m) return;
    uint64_t t = (uint64_t)a.len_dm[e] * 360u / a.speed[e];
    t = t < 1 ? 1 : (t > kRoadCostCap ? kRoadCostCap : t);
    a.t0[e] = (uint32_t)t;
    const uint64_t C = a.cycle[a.col[e]];
    uint64_t w = 0;
    if (C) {
        const uint64_t red = C * (1000u - a.green[e]) / 1000u;
        w = red * red / (2 * C);
        if (w > a.t_max) w = a.t_max;
    }
    a.wf[e] = (uint32_t)w;
    const uint32_t tv = a.resume ? a.tau[e] : a.tau0;
    a.tau[e] = tv;
    if (a.mir) a.mir[(size_t)e * 8 + 5] = tv;
    if (!a.resume) a.load[e] = a.base_load[e];
    a.dep[e] = 0;
    a.cnt[e] = 0;
}

// Empty best routes (or, resume, the best routes held), no iteration key, no selections yet.
__global__ void k_init_vehicles(uint32_t nq, uint32_t resume, uint32_t *best_len, uint32_t *best_cost,
                                uint64_t *iter_key, uint64_t *steps)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) *steps = 0;
    if (v >= nq) return;
    if (!resume) {
        best_len[v] = 0;
        best_cost[v] = kNoCost;
    }
    iter_key[v] = kNoKey;
}

struct CostArgs {
    uint32_t n, theta, th_max;
    const uint32_t *rev_ptr, *rev_edge, *cycle, *load, *t0, *wf;
    uint32_t *cost;
    uint32_t *mir;             // road records of the global walker (8 words per road) or NULL
    uint32_t timed;            // time-dependent signals: cost = travel only, the green flag into the records
};

// Per intersection v: the approach (incoming road) with the longest
// non-empty queue takes the green, ties to the lowest road id; so does any
// approach whose queue exceeds Th_max.  Road cost = congestion-scaled travel
// time (t0 while load <= theta, else floor(t0 * load / theta)) + the fixed
// wait unless the approach has green; capped at 2^31.
__device__ __forceinline__ uint64_t approach_key(uint32_t L, uint32_t e)
{
    return L ? (((uint64_t)L << 32) | (0xFFFFFFFFu - e)) : 0;
}

__device__ __forceinline__ void store_cost(const CostArgs &a, uint32_t e, uint32_t L, uint32_t t0, uint32_t wf,
                                           bool green)
{
    const uint64_t travel = L <= a.theta ? t0 : (uint64_t)t0 * L / a.theta;
    uint64_t c = travel + (green || a.timed ? 0u : wf);   // timed: the walker adds the wait at the ant's clock
    c = c > kRoadCostCap ? kRoadCostCap : c;
    a.cost[e] = (uint32_t)c;
    if (a.mir) {
        a.mir[(size_t)e * 8 + 4] = (uint32_t)c;
        if (a.timed) a.mir[(size_t)e * 8 + 6] = green ? 1u : 0u;
    }
}

// One thread per intersection.  The first kCostBatch approaches are read
// with all their loads in flight at once (road ids, then loads, base times
// and waits), so a node of ordinary degree costs three memory round trips;
// approaches beyond them are read one by one.
constexpr uint32_t kCostBatch = 8;
__global__ void k_cost(CostArgs a)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n) return;
    const uint32_t rb = a.rev_ptr[v], re = a.rev_ptr[v + 1];
    const bool signal = a.cycle[v] != 0;
    uint32_t e[kCostBatch], L[kCostBatch], t0[kCostBatch], wf[kCostBatch];
#pragma unroll
    for (uint32_t u = 0; u < kCostBatch; ++u) e[u] = rb + u < re ? a.rev_edge[rb + u] : 0u;
#pragma unroll
    for (uint32_t u = 0; u < kCostBatch; ++u) {
        L[u] = t0[u] = wf[u] = 0;
        if (rb + u < re) {
            L[u] = a.load[e[u]];
            t0[u] = a.t0[e[u]];
            wf[u] = a.wf[e[u]];
        }
    }
    uint64_t best = 0;
#pragma unroll
    for (uint32_t u = 0; u < kCostBatch; ++u) {
        const uint64_t key = rb + u < re ? approach_key(L[u], e[u]) : 0;
        best = key > best ? key : best;
    }
    for (uint32_t i = rb + kCostBatch; i < re; ++i) {
        const uint32_t ei = a.rev_edge[i];
        const uint64_t key = approach_key(a.load[ei], ei);
        best = key > best ? key : best;
    }
#pragma unroll
    for (uint32_t u = 0; u < kCostBatch; ++u)
        if (rb + u < re)
            store_cost(a, e[u], L[u], t0[u], wf[u],
                       signal && L[u] && (L[u] > a.th_max || approach_key(L[u], e[u]) == best));
    for (uint32_t i = rb + kCostBatch; i < re; ++i) {
        const uint32_t ei = a.rev_edge[i], Li = a.load[ei];
        store_cost(a, ei, Li, a.t0[ei], a.wf[ei], signal && Li && (Li > a.th_max || approach_key(Li, ei) == best));
    }
}

// Add a walker's selections, candidates, arrivals and deposited roads to the
// totals and to its kind's block.
__device__ __forceinline__ void add_walk_counters(uint64_t *c, int kind, uint64_t sel, uint64_t cand, uint64_t arr,
                                                  uint64_t dep)
{
    const uint64_t v[4] = {sel, cand, arr, dep};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        atomicAdd((unsigned long long *)&c[i], (unsigned long long)v[i]);
        atomicAdd((unsigned long long *)&c[kWalkerCounters + 4 * kind + i], (unsigned long long)v[i]);
    }
}

struct WalkArgs {
    const uint32_t *row_ptr, *col, *cost;
    PherView pher;
    DepView depv;
    uint32_t t_local;
    const int32_t *x, *y;
    const gmacop_od *od;
    uint32_t n, nq, ants, max_steps, alpha, beta, kgoal, nwords;
    uint32_t seed_lo, seed_hi, iter;
    uint64_t q_deposit;
    uint32_t *path;        // [max_steps][NA], step-major
    uint32_t *ant_len;     // [NA]
    uint32_t *ant_cost;    // [NA], kNoCost when the ant failed
    uint32_t *gbits;       // [NA][nwords] visited bits when not in LDS
    uint64_t *iter_key;    // [nq]
    uint64_t *steps;       // [1] selections of this call
    uint64_t *counters;    // [kCounters] cumulative work counters
    uint32_t *iter_max;    // longest walk of this iteration
};

// One lane per ant (vehicle v = a / ants, ant k = a % ants).  Visited nodes
// live in a per-ant bitset: in LDS, interleaved by lane so that each lane
// stays in its own bank, or in global memory for large graphs (cleared again
// from the path at the end of the walk).
template <int MAXD, bool LDS_BITS>
__global__ __launch_bounds__(kWave) void k_walk(WalkArgs a)
{
    extern __shared__ uint32_t s_bits[];
    const uint32_t lane = threadIdx.x;
    const uint32_t NA = a.nq * a.ants;
    const uint32_t ant = blockIdx.x * kWave + lane;
    const bool active = ant < NA;
    const uint32_t v = active ? ant / a.ants : 0;
    const uint32_t k = active ? ant % a.ants : 0;
    gmacop_od q = {0, 0, 0};
    if (active) q = a.od[v];
    const bool valid = active && q.src < a.n && q.dst < a.n && q.src != q.dst;

    uint32_t *gb = nullptr;
    if (LDS_BITS) {
        for (uint32_t w = 0; w < a.nwords; ++w) s_bits[w * kWave + lane] = 0;
    } else if (valid) {
        gb = a.gbits + (size_t)ant * a.nwords;
    }
    auto bits_word = [&](uint32_t node) -> uint32_t & {
        return LDS_BITS ? s_bits[(node >> 5) * kWave + lane] : gb[node >> 5];
    };

    uint32_t s = 0, ncand = 0, arrived = 0;
    if (valid) {
        const PherRead tau = pher_at(a.pher, v, a.t_local);
        const int32_t dx = a.x[q.dst], dy = a.y[q.dst];
        uint32_t u = q.src, cs = 0;
        bool ok = false;
        bits_word(u) |= 1u << (u & 31);
        int64_t hu = goal_ms(a.x[u], a.y[u], dx, dy, a.kgoal);
        while (s < a.max_steps) {
            const uint32_t rs = a.row_ptr[u];
            const uint32_t d = a.row_ptr[u + 1] - rs;
            ncand += d;
            uint64_t w[MAXD];
            int64_t hx[MAXD];
            uint32_t cx[MAXD], xx[MAXD];
            uint64_t T = 0;
#pragma unroll
            for (int j = 0; j < MAXD; ++j) {
                w[j] = 0;
                hx[j] = 0;
                cx[j] = 0;
                xx[j] = 0;
                if ((uint32_t)j < d) {
                    const uint32_t e = rs + j;
                    const uint32_t x = a.col[e];
                    xx[j] = x;
                    if (!((bits_word(x) >> (x & 31)) & 1u)) {
                        const uint32_t c = a.cost[e];
                        const int64_t h = goal_ms(a.x[x], a.y[x], dx, dy, a.kgoal);
                        const uint32_t eta = eta_of((int64_t)c + h - hu);
                        w[j] = ipow_u64(tau(e), a.alpha) * ipow_u64(eta, a.beta);
                        hx[j] = h;
                        cx[j] = c;
                    }
                }
                T += w[j];
            }
            if (T == 0) break;   // dead end
            const uint64_t r = philox_u64(q.qid, k, a.iter + slot_iter(a.pher, v, 0), s, a.seed_lo, a.seed_hi);
            const uint64_t target = __umul64hi(r, T);
            uint64_t prefix = 0;
            uint32_t jsel = 0, xsel = 0, csel = 0;
            int64_t hsel = 0;
            bool found = false;
#pragma unroll
            for (int j = 0; j < MAXD; ++j) {
                prefix += w[j];
                const bool take = !found && prefix > target;
                jsel = take ? (uint32_t)j : jsel;
                xsel = take ? xx[j] : xsel;
                csel = take ? cx[j] : csel;
                hsel = take ? hx[j] : hsel;
                found = found || take;
            }
            a.path[(size_t)s * NA + ant] = rs + jsel;
            ++s;
            const uint64_t c2 = (uint64_t)cs + csel;
            cs = c2 > kPathCostCap ? kPathCostCap : (uint32_t)c2;
            u = xsel;
            bits_word(u) |= 1u << (u & 31);
            hu = hsel;
            if (u == q.dst) {
                ok = true;
                break;
            }
        }
        a.ant_len[ant] = s;
        a.ant_cost[ant] = ok ? cs : kNoCost;
        if (ok) {
            arrived = 1;
            const uint64_t dpos = a.q_deposit / cs;
            if (dpos)
                for (uint32_t i = 0; i < s; ++i) a.depv.add(v, a.path[(size_t)i * NA + ant], dpos);
            atomicMin((unsigned long long *)&a.iter_key[v], (unsigned long long)(((uint64_t)cs << 32) | k));
        }
        if (!LDS_BITS) {
            gb[q.src >> 5] = 0;
            for (uint32_t i = 0; i < s; ++i) gb[a.col[a.path[(size_t)i * NA + ant]] >> 5] = 0;
        }
    } else if (active) {
        a.ant_len[ant] = 0;
        a.ant_cost[ant] = kNoCost;
    }
    // one atomic per wave for each counter
    uint64_t cnt = s, cand = ncand, arr = arrived, dh = arrived ? s : 0;
    uint32_t smax = s;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off);
        cand += __shfl_xor(cand, off);
        arr += __shfl_xor(arr, off);
        dh += __shfl_xor(dh, off);
        smax = max(smax, (uint32_t)__shfl_xor((int)smax, off));
    }
    if (lane == 0 && cnt) {
        atomicAdd((unsigned long long *)a.steps, (unsigned long long)cnt);
        add_walk_counters(a.counters, kKindFirst, cnt, cand, arr, dh);
        atomicMax(a.iter_max, smax);
    }
}

// ---- lane-group primitives (groups of L aligned lanes inside a 16-lane DPP row) ----

constexpr int kDppQuad(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
constexpr int kDppRowShr(int n) { return 0x110 + n; }
constexpr int kDppHalfMirror = 0x141;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    return ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp32<CTRL>((uint32_t)v);
}

// Inclusive prefix sum over the group (lane j gets w_0 + ... + w_j).
template <int L>
__device__ __forceinline__ uint64_t grp_prefix(uint64_t v, uint32_t j)
{
    if (L >= 2) { const uint64_t o = dpp64<kDppRowShr(1)>(v); v += j >= 1 ? o : 0; }
    if (L >= 4) { const uint64_t o = dpp64<kDppRowShr(2)>(v); v += j >= 2 ? o : 0; }
    if (L >= 8) { const uint64_t o = dpp64<kDppRowShr(4)>(v); v += j >= 4 ? o : 0; }
    return v;
}

// Sum over the group, returned to every lane.
template <int L>
__device__ __forceinline__ uint64_t grp_sum(uint64_t v)
{
    if (L >= 2) v += dpp64<kDppQuad(1, 0, 3, 2)>(v);
    if (L >= 4) v += dpp64<kDppQuad(2, 3, 0, 1)>(v);
    if (L >= 8) v += dpp64<kDppHalfMirror>(v);
    return v;
}

// Bitwise OR over the group (used with one non-zero contributor).
template <int L>
__device__ __forceinline__ uint32_t grp_or(uint32_t v)
{
    if (L >= 2) v |= dpp32<kDppQuad(1, 0, 3, 2)>(v);
    if (L >= 4) v |= dpp32<kDppQuad(2, 3, 0, 1)>(v);
    if (L >= 8) v |= dpp32<kDppHalfMirror>(v);
    return v;
}

// Value of group lane i (i < L, uniform over the group) to every lane.
template <int L>
__device__ __forceinline__ uint64_t grp_bcast(uint64_t v, uint32_t i)
{
    if (L == 1) return v;
    if (L == 2) return i == 0 ? dpp64<kDppQuad(0, 0, 2, 2)>(v) : dpp64<kDppQuad(1, 1, 3, 3)>(v);
    if (L == 4) {
        const uint64_t b0 = dpp64<kDppQuad(0, 0, 0, 0)>(v), b1 = dpp64<kDppQuad(1, 1, 1, 1)>(v);
        const uint64_t b2 = dpp64<kDppQuad(2, 2, 2, 2)>(v), b3 = dpp64<kDppQuad(3, 3, 3, 3)>(v);
        return i == 0 ? b0 : i == 1 ? b1 : i == 2 ? b2 : b3;
    }
    return __shfl(v, (int)i, L);
}

struct LdsWalkArgs {
    const uint32_t *row_ptr, *col, *cost;
    const uint32_t *node_inst, *inst_off, *inst_eoff;   // city of each node; node / road ranges of cities
    const uint8_t *vclass;     // walker serving each vehicle
    uint32_t cls;              // the LDS size class this launch serves
    PherView pher;
    DepView depv;
    uint32_t t_local;
    const uint2 *rec;          // [m] static: head | head_out_degree << 24, head's first out-road
    const uint32_t *tail;      // [m] static: tail node of each road
    const uint32_t *rev_ptr;   // roads into each node, by node
    // [m] static per road, city-local (cities under 2^16 roads): head's first out-road | out-degree << 16,
    // head's first in-road | in-degree << 16, head | tail << 16, the road's entry of the in-road list
    const uint4 *rvs;
    const int32_t *x, *y;
    const gmacop_od *od;
    uint32_t n, m, nq, ants, apb, bpv, max_steps, alpha, beta, kgoal, nwords;
    uint32_t seed_lo, seed_hi, iter;
    uint64_t q_deposit;
    uint32_t *path, *ant_len, *ant_cost;
    uint64_t *iter_key, *steps, *counters;
    uint32_t *iter_max;    // longest walk of this iteration
    const uint32_t *goal;  // exact goal rows [nq][goal_stride] (city-local node ids), or NULL: straight line
    uint32_t goal_stride;
};

// Per-group scratch at the end of an LDS walker's dynamic LDS: the deposit
// of each group's ant (u64), then the exclusive prefix of the deposited path
// lengths (apb + 1 words).
constexpr size_t lds_group_bytes(uint32_t apb) { return (size_t)apb * 12 + 4; }

// End of an LDS walker block: every ant of the block has walked, so the
// staged road records are no longer read and their space becomes one u64
// deposit accumulator per city road.  The paths of the arriving ants are laid
// end to end and every thread of the block takes an equal slice of their
// entries (its group found in the prefix of path lengths), adding
// floor(q / cost) of the entry's ant to the road with an LDS atomic -- exact
// integer sums, so the order does not matter; all path reads of the block
// are in flight together instead of a long path's lanes reading it a few
// entries at a time.  Then the block adds each non-zero sum to the global
// deposit once, and its best (cost, ant) key and step counters once.
template <int L>
__device__ __forceinline__ void lds_block_finish(const LdsWalkArgs &a, uint64_t *s_mem, uint32_t *s_grp,
                                                 uint32_t e_lo, uint32_t e_cnt, uint32_t v, uint32_t k0, bool active,
                                                 bool ok, uint32_t s, uint32_t cs, uint32_t ncand, uint32_t grp,
                                                 uint32_t j, uint32_t NA)
{
    __shared__ uint64_t s_blk[6];   // best key, steps, candidates, arrivals, deposited roads, longest walk
    const uint32_t tid = threadIdx.x, nthr = blockDim.x, apb = a.apb;
    uint64_t *acc = s_mem;                      // [e_cnt]
    uint64_t *s_dp = (uint64_t *)s_grp;         // [apb]
    uint32_t *s_off = s_grp + 2 * apb;          // [apb + 1]
    const bool arrived = active && ok;
    const uint64_t dpos = arrived ? a.q_deposit / cs : 0;
    __syncthreads();
    for (uint32_t i = tid; i < e_cnt; i += nthr) acc[i] = 0;
    if (tid < 6) s_blk[tid] = tid == 0 ? ~0ull : 0;
    if (j == 0 && grp < apb) {
        s_dp[grp] = dpos;
        s_off[grp] = dpos ? s : 0;
    }
    __syncthreads();
    if (tid < kWave) {   // exclusive prefix of the lengths, groups [tid * per, tid * per + per) per lane
        // (a block of fewer than 64 threads has fewer lanes here: the total comes from its last lane)
        const uint32_t nl = min(nthr, (uint32_t)kWave);
        const uint32_t per = (apb + kWave - 1) / kWave;
        uint32_t sum = 0;
        for (uint32_t g = tid * per; g < min(apb, tid * per + per); ++g) sum += s_off[g];
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
            incl += (int)tid >= off ? o : 0u;
        }
        uint32_t run = incl - sum;
        for (uint32_t g = tid * per; g < min(apb, tid * per + per); ++g) {
            const uint32_t len = s_off[g];
            s_off[g] = run;
            run += len;
        }
        if (tid == nl - 1) s_off[apb] = incl;
    }
    __syncthreads();
    const uint32_t total = s_off[apb];
    const uint32_t per_t = (total + nthr - 1) / nthr;
    uint32_t i = tid * per_t;
    const uint32_t iend = min(total, i + per_t);
    if (i < iend) {
        uint32_t g = 0, hi = apb;   // the group whose entries hold i: s_off[g] <= i < s_off[g + 1]
        while (hi - g > 1) {
            const uint32_t mid = (g + hi) / 2;
            if (s_off[mid] <= i) g = mid; else hi = mid;
        }
        const size_t ant0 = (size_t)v * a.ants + k0;
        // the current group's first entry, the next group's, and its deposit stay in registers: LDS is read
        // again only where the slice crosses into the next ant's entries
        uint32_t cur = s_off[g], nxt = g + 1 < apb ? s_off[g + 1] : total;
        uint64_t dp = s_dp[g];
        while (i < iend) {   // eight path reads in flight, then their LDS adds
            uint32_t e8[8];
            uint64_t d8[8];
            const uint32_t n8 = min(8u, iend - i);
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u) {
                if (u < n8) {
                    while (i + u >= nxt) {   // never past the last group: i + u < total
                        ++g;
                        cur = nxt;
                        nxt = g + 1 < apb ? s_off[g + 1] : total;
                        dp = s_dp[g];
                    }
                    d8[u] = dp;
                    e8[u] = a.path[(size_t)(i + u - cur) * NA + ant0 + g];
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 8; ++u)
                if (u < n8) atomicAdd((unsigned long long *)&acc[e8[u] - e_lo], (unsigned long long)d8[u]);
            i += n8;
        }
    }
    // best key and counters: one contribution per ant (its first lane), into the block's LDS totals
    if (active && j == 0) {
        if (arrived)
            atomicMin((unsigned long long *)&s_blk[0], (unsigned long long)(((uint64_t)cs << 32) | (k0 + grp)));
        atomicAdd((unsigned long long *)&s_blk[1], (unsigned long long)s);
        atomicAdd((unsigned long long *)&s_blk[2], (unsigned long long)ncand);
        if (arrived) {
            atomicAdd((unsigned long long *)&s_blk[3], 1ull);
            atomicAdd((unsigned long long *)&s_blk[4], (unsigned long long)s);
        }
        atomicMax((unsigned long long *)&s_blk[5], (unsigned long long)s);
    }
    __syncthreads();
    for (uint32_t e = tid; e < e_cnt; e += nthr) {
        const uint64_t x = acc[e];
        if (x) a.depv.add(v, e_lo + e, x);
    }
    if (tid == 0) {
        if (s_blk[0] != ~0ull) atomicMin((unsigned long long *)&a.iter_key[v], (unsigned long long)s_blk[0]);
        if (s_blk[1]) {
            atomicAdd((unsigned long long *)a.steps, (unsigned long long)s_blk[1]);
            add_walk_counters(a.counters, kKindLds, s_blk[1], s_blk[2], s_blk[3], s_blk[4]);
            atomicMax(a.iter_max, (uint32_t)s_blk[5]);
        }
    }
}

// One step of an ant on LDS-staged roads (see k_walk_lds).  SL = step index
// modulo L: the group lane that drew this step's Philox word.  Returns false
// when the walk ends (arrival, dead end).
template <int L, int CH, int SL>
__device__ __forceinline__ bool lds_step(const uint2 *s_rec, const uint64_t *s_w, const uint32_t *s_cost,
                                         uint32_t *bits, uint32_t j, uint32_t m_last, uint64_t myr, uint32_t dst,
                                         uint32_t e_lo, uint32_t &u, uint32_t &rs, uint32_t &d, uint32_t &s,
                                         uint32_t &ncand, uint64_t &cs, bool &ok, uint32_t *path_s)
{
    ncand += d;
    uint64_t w[CH], incl[CH];
    uint2 rec[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const uint32_t idx = min(rs + (uint32_t)(c * L) + j, m_last);   // always a valid address
        rec[c] = s_rec[idx];
        w[c] = s_w[idx];
    }
    uint64_t base = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const uint32_t xh = rec[c].x & 0xFFFFFFu;
        const bool live = (uint32_t)(c * L) + j < d && !((bits[xh >> 5] >> (xh & 31)) & 1u);
        w[c] = live ? w[c] : 0;
        incl[c] = grp_prefix<L>(w[c], j) + base;
        base += grp_sum<L>(w[c]);
    }
    const uint64_t T = base;
    if (T == 0) return false;   // dead end
    uint64_t r = myr;
    if (L == 2) r = SL == 0 ? dpp64<kDppQuad(0, 0, 2, 2)>(myr) : dpp64<kDppQuad(1, 1, 3, 3)>(myr);
    if (L == 4) r = dpp64<kDppQuad(SL, SL, SL, SL)>(myr);
    if (L >= 8) r = __shfl(myr, SL, L);
    const uint64_t target = __umul64hi(r, T);
    // exactly one (chunk, lane) holds the target in its prefix interval
    uint32_t sel_x = 0, sel_y = 0, sel_c = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const bool hit = w[c] != 0 && incl[c] - w[c] <= target && target < incl[c];
        sel_x |= hit ? rec[c].x : 0u;
        sel_y |= hit ? rec[c].y : 0u;
        sel_c |= hit ? (uint32_t)(c * L) + j + 1 : 0u;
    }
    sel_x = grp_or<L>(sel_x);
    sel_y = grp_or<L>(sel_y);
    sel_c = grp_or<L>(sel_c);
    if (sel_c == 0) return false;   // unreachable when T > 0; keeps every index in range
    const uint32_t xsel = sel_x & 0xFFFFFFu;
    const uint32_t esel = rs + sel_c - 1;
    if (j == 0) {
        *path_s = e_lo + esel;
        atomicOr(&bits[xsel >> 5], 1u << (xsel & 31));
    }
    cs += s_cost[esel];
    ++s;
    u = xsel;
    rs = sel_y;
    d = sel_x >> 24;
    if (u == dst) {
        ok = true;
        return false;
    }
    return true;
}

// L consecutive steps, step SL using the Philox word of group lane SL.
template <int L, int CH, int SL>
__device__ __forceinline__ bool lds_steps(const uint2 *s_rec, const uint64_t *s_w, const uint32_t *s_cost,
                                          uint32_t *bits, uint32_t j, uint32_t m_last, uint64_t myr, uint32_t dst,
                                          uint32_t max_steps, uint32_t NA, uint32_t e_lo, uint32_t &u, uint32_t &rs,
                                          uint32_t &d, uint32_t &s, uint32_t &ncand, uint64_t &cs, bool &ok,
                                          uint32_t *path)
{
    if (s >= max_steps || !lds_step<L, CH, SL>(s_rec, s_w, s_cost, bits, j, m_last, myr, dst, e_lo, u, rs, d, s,
                                               ncand, cs, ok, path + (size_t)s * NA))
        return false;
    if constexpr (SL + 1 < L)
        return lds_steps<L, CH, SL + 1>(s_rec, s_w, s_cost, bits, j, m_last, myr, dst, max_steps, NA, e_lo, u, rs, d,
                                        s, ncand, cs, ok, path);
    return true;
}
// Walk for graphs whose roads fit in LDS.  One block serves `apb` ants of one
// vehicle (blocks_per_vehicle = bpv).  Prologue: the block derives the
// vehicle's goal term for every node and stages, per road, the head node,
// the head's out-road range and the choice weight tau^alpha * eta^beta
// (a per-destination choice table), then clears its ants' visited bits.
// Walk: L lanes per ant; lane j examines candidates j, j+L, ...; the group
// sums weights with DPP row shifts, and the candidate whose prefix interval
// holds the target (the first, in CSR order, whose inclusive prefix exceeds
// it) is taken.  The L lanes draw Philox words for L consecutive steps at
// once (the counter does not depend on the path), so one draw serves L
// steps; the step loop is unrolled by L so each step reads its word with a
// fixed DPP pattern.  A step is three dependent LDS reads (road record,
// visited word, chosen road's cost).  Deposits are gathered per block
// (lds_block_finish).
template <int L, int CH>
__global__ __launch_bounds__(512) void k_walk_lds(LdsWalkArgs a)
{
    extern __shared__ uint64_t s_mem[];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t v = blockIdx.x / a.bpv, part = blockIdx.x % a.bpv;
    if (a.vclass[v] != a.cls) return;                // whole block: another walker serves this vehicle
    const gmacop_od q = a.od[v];
    // the vehicle's city, in city-local node and road ids
    const uint32_t city = a.node_inst[q.src];
    const uint32_t n_lo = a.inst_off[city], n_cnt = a.inst_off[city + 1] - n_lo;
    const uint32_t e_lo = a.inst_eoff[city], e_cnt = a.inst_eoff[city + 1] - e_lo;
    uint2 *s_rec = (uint2 *)s_mem;                   // [e_cnt] (head | head_deg << 24, head_row_start)
    uint64_t *s_w = s_mem + e_cnt;                   // [e_cnt] choice weight
    uint32_t *s_cost = (uint32_t *)(s_mem + 2 * (size_t)e_cnt);   // [e_cnt] road cost
    uint32_t *s_aux = s_cost + ((e_cnt + 1) & ~1u);  // goal terms, then visited bits
    const uint32_t nws = ((n_cnt + 31) / 32) | 1u;   // visited words per ant (odd stride spreads banks)
    uint32_t *s_grp = s_aux + ((max(n_cnt, nws * a.apb) + 1) & ~1u);   // per-group scratch (lds_block_finish)

    // ---- prologue: choice table of this vehicle, one coalesced pass per road ----
    {
        const int32_t dx = a.x[q.dst], dy = a.y[q.dst];
        for (uint32_t i = tid; i < n_cnt; i += nthr)
            s_aux[i] = a.goal ? a.goal[(size_t)v * a.goal_stride + i]
                              : (uint32_t)goal_ms(a.x[n_lo + i], a.y[n_lo + i], dx, dy, a.kgoal);
    }
    __syncthreads();
    {
        const bool a1b2 = a.alpha == 1 && a.beta == 2;
        const PherRead tau = pher_at(a.pher, v, a.t_local);
        for (uint32_t le = tid; le < e_cnt; le += nthr) {
            const uint32_t e = e_lo + le;
            const uint2 r = a.rec[e];
            const uint32_t c = a.cost[e], t = tau(e), tl = a.tail[e] - n_lo;
            const uint32_t xl = (r.x & 0xFFFFFFu) - n_lo;
            const uint32_t eta = eta_of((int64_t)c + (int64_t)s_aux[xl] - (int64_t)s_aux[tl]);
            const uint64_t wgt = a1b2 ? (uint64_t)t * (eta * eta) : ipow_u64(t, a.alpha) * ipow_u64(eta, a.beta);
            s_w[le] = wgt;
            s_rec[le] = make_uint2(xl | (r.x & 0xFF000000u), r.y - e_lo);
            s_cost[le] = c;
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < nws * a.apb; i += nthr) s_aux[i] = 0;
    __syncthreads();

    // ---- walk ----
    const uint32_t grp = tid / L, j = tid % L;
    const uint32_t k = part * a.apb + grp;
    const bool active = grp < a.apb && k < a.ants;
    const uint32_t NA = a.nq * a.ants;
    const uint32_t ant = v * a.ants + k;
    uint32_t s = 0, ncand = 0, cs = 0;
    bool ok = false;
    uint32_t *path = a.path + ant;
    if (active) {
        uint32_t *bits = s_aux + grp * nws;
        uint32_t u = q.src - n_lo;
        uint32_t rs = a.row_ptr[q.src] - e_lo, d = a.row_ptr[q.src + 1] - a.row_ptr[q.src];
        if (j == 0) atomicOr(&bits[u >> 5], 1u << (u & 31));
        uint64_t cs64 = 0;
        const uint32_t m_last = e_cnt - 1;
        const uint32_t it = a.iter + slot_iter(a.pher, v, 0);
        for (;;) {
            const uint64_t myr = philox_u64(q.qid, k, it, s + j, a.seed_lo, a.seed_hi);
            if (!lds_steps<L, CH, 0>(s_rec, s_w, s_cost, bits, j, m_last, myr, q.dst - n_lo, a.max_steps, NA, e_lo, u,
                                     rs, d, s, ncand, cs64, ok, path))
                break;
        }
        cs = cs64 > kPathCostCap ? kPathCostCap : (uint32_t)cs64;
        if (j == 0) {
            a.ant_len[ant] = s;
            a.ant_cost[ant] = ok ? cs : kNoCost;
        }
    }
    lds_block_finish<L>(a, s_mem, s_grp, e_lo, e_cnt, v, part * a.apb, active, ok, s, cs, ncand, grp, j, NA);
}

// Value of the last lane of the group (the group total of an inclusive prefix).
template <int L>
__device__ __forceinline__ uint64_t grp_last(uint64_t v)
{
    if (L == 1) return v;
    if (L == 2) return dpp64<kDppQuad(1, 1, 3, 3)>(v);
    if (L == 4) return dpp64<kDppQuad(3, 3, 3, 3)>(v);
    return __shfl(v, L - 1, L);
}

// One step of the road-visited walker (k_walk_ldsr).  Every read of the step
// depends only on the current node (its first out-road rs and first in-road
// rv), so the road records, costs, visited words and the node's in-roads come
// back in one LDS round trip.  The current node's in-roads are then marked
// visited; none of them is a candidate of this step (no self-loops).  The
// lane holding the chosen road writes the path entry and adds the road's cost
// to its own partial sum; only the chosen record crosses lanes.
template <int L, int CH, int SL>
__device__ __forceinline__ bool rv_step(const uint4 *s_R, const uint32_t *s_cost, const uint32_t *s_rev,
                                        uint32_t *bits, uint32_t j, uint32_t m_last, uint64_t myr, uint32_t e_lo,
                                        PhiloxState &nx, uint32_t k0, uint32_t k1, uint32_t &rs, uint32_t &d,
                                        uint32_t &rv, uint32_t &ind, uint32_t &s, uint32_t &ncand, uint64_t &cs,
                                        bool &ok, uint32_t *path_s)
{
    uint4 R[CH];
    uint32_t cst[CH], vw[CH], inr[CH], idx[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        idx[c] = min(rs + (uint32_t)(c * L) + j, m_last);   // always a valid address
        inr[c] = s_rev[min(rv + (uint32_t)(c * L) + j, m_last)];
        R[c] = s_R[idx[c]];
        cst[c] = s_cost[idx[c]];
        vw[c] = bits[idx[c] >> 5];
    }
    __builtin_amdgcn_sched_barrier(0);   // every read above is in flight before the first wait
    philox_rounds<SL * 10 / L, (SL + 1) * 10 / L>(nx, k0, k1);   // next block's draw, in the read latency
    // (no branch: lanes past the in-degree OR zero into an in-range word, so
    // nothing below waits for these writes)
#pragma unroll
    for (int c = 0; c < CH; ++c)
        atomicOr(&bits[inr[c] >> 5], (uint32_t)(c * L) + j < ind ? 1u << (inr[c] & 31) : 0u);
    ncand += d;
    uint64_t w[CH], incl[CH];
    uint64_t base = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const bool live = (uint32_t)(c * L) + j < d && !((vw[c] >> (idx[c] & 31)) & 1u);
        w[c] = live ? (((uint64_t)R[c].w << 32) | R[c].z) : 0;
        incl[c] = grp_prefix<L>(w[c], j) + base;
        base = grp_last<L>(incl[c]);
    }
    const uint64_t T = base;
    uint64_t r = myr;
    if (L == 2) r = SL == 0 ? dpp64<kDppQuad(0, 0, 2, 2)>(myr) : dpp64<kDppQuad(1, 1, 3, 3)>(myr);
    if (L == 4) r = dpp64<kDppQuad(SL, SL, SL, SL)>(myr);
    if (L >= 8) r = __shfl(myr, SL, L);
    const uint64_t target = __umul64hi(r, T);
    // the candidate whose prefix interval [incl - w, incl) holds the target (none when T == 0)
    uint32_t sx = 0, sy = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const bool hit = incl[c] - w[c] <= target && target < incl[c];
        sx |= hit ? R[c].x : 0u;
        sy |= hit ? R[c].y : 0u;
        cs += hit ? cst[c] : 0u;
        if (hit) *path_s = e_lo + idx[c];
    }
    sx = grp_or<L>(sx);
    sy = grp_or<L>(sy);
    const bool moved = T != 0;
    s += moved ? 1u : 0u;
    ok = moved && (sx >> 31) != 0;
    rs = sx & 0xFFFFu;
    d = (sx >> 16) & 0x7FFFu;
    rv = sy & 0xFFFFu;
    ind = sy >> 16;
    return moved && !ok;
}

// (ps: this ant's path entry of the current step; it advances by NA per step)
template <int L, int CH, int SL>
__device__ __forceinline__ bool rv_steps(const uint4 *s_R, const uint32_t *s_cost, const uint32_t *s_rev,
                                         uint32_t *bits, uint32_t j, uint32_t m_last, uint64_t myr, uint32_t e_lo,
                                         PhiloxState &nx, uint32_t k0, uint32_t k1, uint32_t max_steps, uint32_t NA,
                                         uint32_t &rs, uint32_t &d, uint32_t &rv, uint32_t &ind, uint32_t &s,
                                         uint32_t &ncand, uint64_t &cs, bool &ok, uint32_t *&ps)
{
    if (s >= max_steps || !rv_step<L, CH, SL>(s_R, s_cost, s_rev, bits, j, m_last, myr, e_lo, nx, k0, k1, rs, d, rv,
                                              ind, s, ncand, cs, ok, ps))
        return false;
    ps += NA;
    if constexpr (SL + 1 < L)
        return rv_steps<L, CH, SL + 1>(s_R, s_cost, s_rev, bits, j, m_last, myr, e_lo, nx, k0, k1, max_steps, NA, rs,
                                       d, rv, ind, s, ncand, cs, ok, ps);
    return true;
}

// Walk for cities whose roads fit in LDS, with visited state kept per road:
// entering a node marks every road into it, so a candidate road is live
// when its own bit is clear -- the bit's address is known from the current
// node alone, and a step needs a single LDS round trip.  Same block layout,
// Philox schedule, choice table and results as k_walk_lds.  LDS per block:
// per road a 16-byte record (head's first out-road | head out-degree << 16 |
// head-is-destination << 31; head's first in-road | head in-degree << 16;
// choice weight), its cost and its entry of the city's in-road list, then
// the goal terms (prologue) overlaid by the visited road bits of each ant.
// City-local road ids must stay below 2^16.
template <int L, int CH>
__global__ __launch_bounds__(512) void k_walk_ldsr(LdsWalkArgs a)
{
    extern __shared__ uint64_t s_mem[];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t v = blockIdx.x / a.bpv, part = blockIdx.x % a.bpv;
    if (a.vclass[v] != a.cls) return;                // whole block: another walker serves this vehicle
    const gmacop_od q = a.od[v];
    const uint32_t city = a.node_inst[q.src];
    const uint32_t n_lo = a.inst_off[city], n_cnt = a.inst_off[city + 1] - n_lo;
    const uint32_t e_lo = a.inst_eoff[city], e_cnt = a.inst_eoff[city + 1] - e_lo;
    uint4 *s_R = (uint4 *)s_mem;                                  // [e_cnt]
    uint32_t *s_cost = (uint32_t *)(s_R + e_cnt);                 // [e_cnt]
    uint32_t *s_rev = s_cost + e_cnt;                             // [e_cnt] city-local roads, grouped by head
    uint32_t *s_aux = s_rev + e_cnt;                              // goal terms, then visited road bits
    const uint32_t nws = ((e_cnt + 31) / 32) | 1u;                // visited words per ant (odd stride)
    uint32_t *s_grp = s_aux + ((max(n_cnt, nws * a.apb) + 1) & ~1u);   // per-group scratch (lds_block_finish)

    {
        // the roads in batches of eight per thread, their loads (all independent) ahead of the arithmetic;
        // the first batch's loads are issued before the goal terms are computed, so they overlap
        const bool a1b2 = a.alpha == 1 && a.beta == 2;
        const PherRead tau = pher_at(a.pher, v, a.t_local);
        const uint32_t dst_l = q.dst - n_lo;
        uint4 st[8];
        uint32_t c[8], t[8];
        auto load_batch = [&](uint32_t b0) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t le = b0 + u * nthr;
                if (le < e_cnt) {
                    st[u] = a.rvs[e_lo + le];
                    c[u] = a.cost[e_lo + le];
                    t[u] = tau(e_lo + le);
                }
            }
        };
        auto stage_batch = [&](uint32_t b0) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t le = b0 + u * nthr;
                if (le < e_cnt) {
                    const uint32_t xl = st[u].z & 0xFFFFu, tl = st[u].z >> 16;
                    const uint32_t eta = eta_of((int64_t)c[u] + (int64_t)s_aux[xl] - (int64_t)s_aux[tl]);
                    const uint64_t wgt = a1b2 ? (uint64_t)t[u] * (eta * eta)
                                              : ipow_u64(t[u], a.alpha) * ipow_u64(eta, a.beta);
                    s_R[le] = make_uint4(st[u].x | (xl == dst_l ? 0x80000000u : 0u), st[u].y, (uint32_t)wgt,
                                         (uint32_t)(wgt >> 32));
                    s_cost[le] = c[u];
                    s_rev[le] = st[u].w;
                }
            }
        };
        load_batch(tid);
        const int32_t dx = a.x[q.dst], dy = a.y[q.dst];
        for (uint32_t i = tid; i < n_cnt; i += nthr)
            s_aux[i] = a.goal ? a.goal[(size_t)v * a.goal_stride + i]
                              : (uint32_t)goal_ms(a.x[n_lo + i], a.y[n_lo + i], dx, dy, a.kgoal);
        __syncthreads();
        stage_batch(tid);
        for (uint32_t b0 = tid + 8 * nthr; b0 < e_cnt; b0 += 8 * nthr) {
            load_batch(b0);
            stage_batch(b0);
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < nws * a.apb; i += nthr) s_aux[i] = 0;
    __syncthreads();

    const uint32_t grp = tid / L, j = tid % L;
    const uint32_t k = part * a.apb + grp;
    const bool active = grp < a.apb && k < a.ants;
    const uint32_t NA = a.nq * a.ants;
    const uint32_t ant = v * a.ants + k;
    uint32_t s = 0, ncand = 0, cs = 0;
    bool ok = false;
    uint32_t *path = a.path + ant;
    if (active) {
        uint32_t *bits = s_aux + grp * nws;
        uint32_t rs = a.row_ptr[q.src] - e_lo, d = a.row_ptr[q.src + 1] - a.row_ptr[q.src];
        uint32_t rv = a.rev_ptr[q.src] - e_lo, ind = a.rev_ptr[q.src + 1] - a.rev_ptr[q.src];
        uint64_t csl = 0;   // this lane's share of the path cost
        const uint32_t m_last = e_cnt - 1;
        const uint32_t it = a.iter + slot_iter(a.pher, v, 0);
        uint64_t myr = philox_u64(q.qid, k, it, s + j, a.seed_lo, a.seed_hi);
        uint32_t *ps = path;
        for (;;) {
            // the draw of the next L steps advances inside these L steps
            PhiloxState nx{q.qid, k, it, s + L + j};
            if (!rv_steps<L, CH, 0>(s_R, s_cost, s_rev, bits, j, m_last, myr, e_lo, nx, a.seed_lo, a.seed_hi,
                                    a.max_steps, NA, rs, d, rv, ind, s, ncand, csl, ok, ps))
                break;
            myr = ((uint64_t)nx.c1 << 32) | nx.c0;
        }
        const uint64_t cs64 = grp_sum<L>(csl);
        cs = cs64 > kPathCostCap ? kPathCostCap : (uint32_t)cs64;
        if (j == 0) {
            a.ant_len[ant] = s;
            a.ant_cost[ant] = ok ? cs : kNoCost;
        }
    }
    lds_block_finish<L>(a, s_mem, s_grp, e_lo, e_cnt, v, part * a.apb, active, ok, s, cs, ncand, grp, j, NA);
}

// A vehicle served by k_walk_glb, with the walk's start data (k_glb_list).
struct GlbVeh {
    uint32_t v, qid, src, dst;
    uint32_t rs, d, n_lo, pad;   // source's out-road range; first node of the city
    int32_t dx, dy;              // destination coordinates
    uint32_t hu_lo, hu_hi;       // goal term of the source
};

struct GlbWalkArgs {
    // [m][2] per road: (head | head_deg << 24, head's first out-road, head x, head y), then
    // (cost, pheromone in shared mode, 0, 0) -- one 32-byte record, so a candidate is one line
    const uint4 *rec32;
    PherView pher;
    DepView depv;
    const GlbVeh *veh;         // [*glb_n] vehicles of this walker
    const uint32_t *glb_n;
    uint32_t *tickets;         // [0]: next ticket (vehicle-major: ticket = list position * ants + ant), [1]: waves done
    uint32_t *vlen;            // [nq] longest walk of each vehicle in this launch (orders the next list)
    uint64_t *gwords;          // [slots][nw2] visited words: current walk's epoch << 32 | 32 node bits
    uint32_t *slot_epoch;      // [slots] epoch of each slot's last walk
    uint32_t m, ants, apb, max_steps, alpha, beta, kgoal;
    uint32_t nw2;              // visited words per slot (largest city / 32)
    uint32_t bloom_log2;       // Bloom filter of 2^bloom_log2 bits per slot in LDS
    uint32_t seed_lo, seed_hi, iter, t_local, nq;
    uint64_t q_deposit;
    uint32_t *path, *ant_len, *ant_cost;
    uint64_t *iter_key, *steps, *counters;
    uint32_t *iter_max;
    const uint32_t *goal;      // exact goal rows [nq][goal_stride] (city-local node ids), or NULL: straight line
    uint32_t goal_stride;
    const uint4 *sig;          // time-dependent signals: per road (head's cycle, green start, green length, 0), or NULL
    uint32_t t_max;
};

constexpr uint8_t kWalkerNone = 0, kWalkerGlobal = 8;   // 1..6: LDS walker classes

// Cost of a road entered at `clock` (ms since the call's start) under
// time-dependent signals: its travel time, plus the wait from its arrival at
// the head's signal to the next opening of its approach's green window
// (s = cycle, window start, window length), capped at T_max; none when the
// approach holds the preemptive green or the head has no signal.  Capped at
// 2^31 like every road cost.
__device__ __forceinline__ uint32_t timed_cost(uint32_t travel, uint32_t green, uint4 s, uint64_t clock, uint32_t t_max)
{
    uint64_t wait = 0;
    if (s.x && !green) {
        const uint64_t q = ((clock + travel) % s.x + s.x - s.y) % s.x;   // phase from the window's opening
        wait = q < s.z ? 0 : s.x - q;
        wait = wait > t_max ? t_max : wait;
    }
    const uint64_t c = travel + wait;
    return c > kRoadCostCap ? kRoadCostCap : (uint32_t)c;
}

__device__ __forceinline__ uint32_t bloom_h1(uint32_t x, uint32_t lg) { return (x * 0x9E3779B1u) >> (32 - lg); }
__device__ __forceinline__ uint32_t bloom_h2(uint32_t x, uint32_t lg)
{
    return ((x ^ 0x5BD1E995u) * 0x85EBCA77u + 0x165667B1u) >> (32 - lg);
}

// Per-lane-group state of a k_walk_glb walk.
struct GlbWalk {
    PherRead tau;
    uint32_t v, k, qid, dst, n_lo, it;
    int32_t dx, dy;
    uint32_t u, rs, d, s, ncand;
    int64_t hu;
    uint64_t cs;
    uint32_t hist[4];          // the last four nodes entered
    uint32_t *path;            // this ant's path column
    const uint32_t *grow;      // the vehicle's exact goal row (when the call uses one)
    uint64_t *pw;              // visited word of the node entered last (group lane 0; nullptr: none)
    uint64_t pval;             // its value, loaded when the node was entered
    uint32_t pbit;
    bool ok;
};

// One step of a k_walk_glb walk.  Candidate roads are 16-byte record
// gathers (head, head's out-road range, head coordinates) plus their cost and
// pheromone.  The visited test is exact but rarely touches memory: the last
// four nodes are in registers, then a per-slot Bloom filter in LDS (two hash
// bits); only when it reports "maybe" is the slot's visited word read.  Entering a node
// sets its visited bit by read-modify-write of the slot's word: the word is
// loaded when the node is entered and written at the next step, behind that
// step's loads (the node stays in the register history meanwhile, and the
// same lane's later reads of the word come after the write).  A word written
// by an earlier walk carries an older epoch and counts as empty, so nothing
// is cleared between walks.
template <int L, int CH, int SL, bool TM>
__device__ __forceinline__ bool glb_step(const GlbWalkArgs &a, GlbWalk &w, uint32_t *bloom, uint64_t *gw,
                                         uint32_t epoch, uint32_t j, uint64_t myr)
{
    w.ncand += w.d;
    const uint32_t lg = a.bloom_log2;
    uint64_t wt[CH], incl[CH];
    uint4 rec[CH];
    uint32_t cst[CH], grn[CH];
    uint4 sg[CH];   // TM: the heads' signal windows
    int64_t hx[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {   // lanes past the out-degree load nothing
        const uint32_t o = (uint32_t)(c * L) + j, idx = w.rs + o;
        uint4 r0 = make_uint4(0, 0, 0, 0), r1 = make_uint4(0, 0, 0, 0);
        uint32_t tl = 0;
        sg[c] = make_uint4(0, 0, 0, 0);
        if (o < w.d) {
            r0 = a.rec32[2 * (size_t)idx];
            r1 = a.rec32[2 * (size_t)idx + 1];
            if (!w.tau.dense) tl = w.tau(idx);
            if constexpr (TM) sg[c] = a.sig[idx];
        }
        rec[c] = r0;
        cst[c] = r1.x;
        grn[c] = r1.z;
        wt[c] = w.tau.dense ? r1.y : tl;
    }
    if (w.pw) {   // group lane 0: the visited bit of the node entered last step
        const uint64_t old = w.pval;
        *w.pw = ((uint32_t)(old >> 32) == epoch ? old : (uint64_t)epoch << 32) | w.pbit;
        w.pw = nullptr;
    }
    uint64_t base = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const uint32_t xh = rec[c].x & 0xFFFFFFu;
        bool live = (uint32_t)(c * L) + j < w.d;
        live = live && xh != w.hist[0] && xh != w.hist[1] && xh != w.hist[2] && xh != w.hist[3];
        if (live) {
            const uint32_t xl = xh - w.n_lo;
            const uint32_t b1 = bloom_h1(xl, lg), b2 = bloom_h2(xl, lg);
            if (((bloom[b1 >> 5] >> (b1 & 31)) & (bloom[b2 >> 5] >> (b2 & 31)) & 1u) != 0) {
                // Bloom filter says "maybe": the slot's visited word decides (read at the device-coherent level)
                const uint64_t vw = __hip_atomic_load(&gw[xl >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                live = (uint32_t)(vw >> 32) != epoch || (((uint32_t)vw >> (xl & 31)) & 1u) == 0;
            }
        }
        hx[c] = 0;
        if (live) {
            if constexpr (TM)   // time-dependent signals: the road's cost at this ant's clock (its capped cost so far)
                cst[c] = timed_cost(cst[c], grn[c], sg[c], w.cs > kPathCostCap ? kPathCostCap : w.cs, a.t_max);
            hx[c] = a.goal ? (int64_t)w.grow[xh - w.n_lo]
                           : goal_ms((int32_t)rec[c].z, (int32_t)rec[c].w, w.dx, w.dy, a.kgoal);
            const uint32_t eta = eta_of((int64_t)cst[c] + hx[c] - w.hu);
            const uint32_t t = (uint32_t)wt[c];
            wt[c] = (a.alpha == 1 && a.beta == 2) ? (uint64_t)t * (eta * eta)
                                                  : ipow_u64(t, a.alpha) * ipow_u64(eta, a.beta);
        } else {
            wt[c] = 0;
        }
        incl[c] = grp_prefix<L>(wt[c], j) + base;
        base += grp_sum<L>(wt[c]);
    }
    const uint64_t T = base;
    if (T == 0) return false;   // dead end
    uint64_t r = myr;
    if (L == 2) r = SL == 0 ? dpp64<kDppQuad(0, 0, 2, 2)>(myr) : dpp64<kDppQuad(1, 1, 3, 3)>(myr);
    if (L == 4) r = dpp64<kDppQuad(SL, SL, SL, SL)>(myr);
    if (L >= 8) r = __shfl(myr, SL, L);
    const uint64_t target = __umul64hi(r, T);
    uint32_t sel_x = 0, sel_y = 0, sel_c = 0, sel_cost = 0, sel_hlo = 0, sel_hhi = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const bool hit = wt[c] != 0 && incl[c] - wt[c] <= target && target < incl[c];
        sel_x |= hit ? rec[c].x : 0u;
        sel_y |= hit ? rec[c].y : 0u;
        sel_c |= hit ? (uint32_t)(c * L) + j + 1 : 0u;
        sel_cost |= hit ? cst[c] : 0u;
        sel_hlo |= hit ? (uint32_t)(uint64_t)hx[c] : 0u;
        sel_hhi |= hit ? (uint32_t)((uint64_t)hx[c] >> 32) : 0u;
    }
    sel_x = grp_or<L>(sel_x);
    sel_y = grp_or<L>(sel_y);
    sel_c = grp_or<L>(sel_c);
    sel_cost = grp_or<L>(sel_cost);
    sel_hlo = grp_or<L>(sel_hlo);
    sel_hhi = grp_or<L>(sel_hhi);
    if (sel_c == 0) return false;   // unreachable when T > 0; keeps every index in range
    const uint32_t xsel = sel_x & 0xFFFFFFu;
    if (j == 0) {
        w.path[(size_t)w.s * a.nq * a.ants] = w.rs + sel_c - 1;
        const uint32_t xl = xsel - w.n_lo;
        const uint32_t b1 = bloom_h1(xl, lg), b2 = bloom_h2(xl, lg);
        atomicOr(&bloom[b1 >> 5], 1u << (b1 & 31));
        atomicOr(&bloom[b2 >> 5], 1u << (b2 & 31));
        w.pw = &gw[xl >> 5];
        w.pbit = 1u << (xl & 31);
        w.pval = __hip_atomic_load(w.pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    w.hist[3] = w.hist[2];
    w.hist[2] = w.hist[1];
    w.hist[1] = w.hist[0];
    w.hist[0] = xsel;
    w.cs += sel_cost;
    w.hu = (int64_t)(((uint64_t)sel_hhi << 32) | sel_hlo);
    ++w.s;
    w.u = xsel;
    w.rs = sel_y;
    w.d = sel_x >> 24;
    if (w.u == w.dst) {
        w.ok = true;
        return false;
    }
    return true;
}

template <int L, int CH, int SL, bool TM>
__device__ __forceinline__ bool glb_steps(const GlbWalkArgs &a, GlbWalk &w, uint32_t *bloom, uint64_t *gw,
                                          uint32_t epoch, uint32_t j, uint64_t myr)
{
    if (w.s >= a.max_steps || !glb_step<L, CH, SL, TM>(a, w, bloom, gw, epoch, j, myr)) return false;
    if constexpr (SL + 1 < L) return glb_steps<L, CH, SL + 1, TM>(a, w, bloom, gw, epoch, j, myr);
    return true;
}

// Walk for graphs too large for LDS: a persistent kernel, one slot per group
// of L lanes (lane j examines candidates j, j+L, ...).  The grid holds as
// many groups as stay resident; a group walks one ant at a time and, when
// its walk ends, takes the next ant from a ticket counter, so lanes do not
// wait for the longest walk of their wave or block.  The groups of a wave
// that need an ant take their tickets together, from a per-wave range that
// is refilled one atomic at a time.  The last wave out resets the counters
// for the next launch.  TM: roads cost by the time-dependent signal rule (a.sig).
template <int L, int CH, bool TM>
__global__ __launch_bounds__(256) void k_walk_glb(GlbWalkArgs a)
{
    constexpr uint32_t kGroups = kWave / L;   // groups per wave = tickets per refill
    extern __shared__ uint32_t s_bloom[];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1);
    const uint32_t grp = tid / L, j = tid % L;
    const uint32_t lead = lane - j;            // wave lane of the group's lane 0
    const uint32_t slot = blockIdx.x * a.apb + grp;
    const uint32_t NA = a.nq * a.ants;
    const uint32_t total = *a.glb_n * a.ants;
    const uint32_t bws = (1u << (a.bloom_log2 - 5)) | 1u;   // odd stride spreads banks
    uint32_t *bloom = s_bloom + grp * bws;
    uint64_t *gw = a.gwords + (size_t)slot * a.nw2;
    uint32_t epoch = a.slot_epoch[slot];
    uint64_t c_steps = 0, c_cand = 0, c_arr = 0, c_dh = 0;   // group lane 0 counts
    uint32_t c_max = 0;
    uint32_t w_next = 0, w_end = 0;            // this wave's unused tickets (equal in every lane)
    bool have = false, done = false;
    GlbWalk w{};
    for (;;) {
        // groups without an ant take the next tickets
        const bool need = !have && !done;
        const uint64_t mask = __ballot(need && j == 0);
        if (mask) {
            const uint32_t n = (uint32_t)__popcll(mask);
            const uint32_t avail = w_end - w_next;
            uint32_t base2 = 0;
            if (n > avail) {
                const uint32_t first = (uint32_t)__ffsll((unsigned long long)mask) - 1;
                uint32_t got = 0;
                if (lane == first) got = atomicAdd(a.tickets, kGroups);
                base2 = __shfl(got, (int)first);
            }
            if (need) {
                const uint32_t rk = (uint32_t)__popcll(mask & ((1ull << lead) - 1));
                const uint32_t t = rk < avail ? w_next + rk : base2 + (rk - avail);
                if (t >= total) {
                    done = true;
                } else {
                    // start the walk of ticket t
                    const uint32_t pos = t / a.ants;
                    const uint4 *vr = (const uint4 *)(a.veh + pos);
                    const uint4 r0 = vr[0], r1 = vr[1], r2 = vr[2];
                    w.k = t - pos * a.ants;
                    w.v = r0.x; w.qid = r0.y; w.u = r0.z; w.dst = r0.w;
                    w.rs = r1.x; w.d = r1.y; w.n_lo = r1.z;
                    w.dx = (int32_t)r2.x; w.dy = (int32_t)r2.y;
                    w.hu = (int64_t)(((uint64_t)r2.w << 32) | r2.z);
                    w.tau = pher_at(a.pher, w.v, a.t_local);
                    w.it = a.iter + slot_iter(a.pher, w.v, 0);
                    w.s = 0; w.ncand = 0; w.cs = 0; w.ok = false;
                    w.hist[0] = w.u; w.hist[1] = w.hist[2] = w.hist[3] = 0xFFFFFFFFu;
                    w.path = a.path + (size_t)w.v * a.ants + w.k;
                    w.grow = a.goal ? a.goal + (size_t)w.v * a.goal_stride : nullptr;
                    if (++epoch == 0) {   // epochs would repeat: clear the slot's words once
                        for (uint32_t i = j; i < a.nw2; i += L) gw[i] = 0;
                        epoch = 1;
                    }
                    for (uint32_t i = j; i < bws; i += L) bloom[i] = 0;
                    w.pw = nullptr;
                    if (j == 0) {
                        const uint32_t ul = w.u - w.n_lo;
                        atomicOr(&bloom[bloom_h1(ul, a.bloom_log2) >> 5], 1u << (bloom_h1(ul, a.bloom_log2) & 31));
                        atomicOr(&bloom[bloom_h2(ul, a.bloom_log2) >> 5], 1u << (bloom_h2(ul, a.bloom_log2) & 31));
                        w.pw = &gw[ul >> 5];
                        w.pbit = 1u << (ul & 31);
                        w.pval = __hip_atomic_load(w.pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    have = true;
                }
            }
            if (n > avail) {
                w_next = base2 + (n - avail);
                w_end = base2 + kGroups;
            } else {
                w_next += n;
            }
        }
        if (__ballot(!done) == 0) break;   // no group of the wave has work left
        if (!have) continue;
        const uint64_t myr = philox_u64(w.qid, w.k, w.it, w.s + j, a.seed_lo, a.seed_hi);
        if (glb_steps<L, CH, 0, TM>(a, w, bloom, gw, epoch, j, myr)) continue;
        // the walk is over
        const uint32_t ant = w.v * a.ants + w.k;
        const uint32_t cs = w.cs > kPathCostCap ? kPathCostCap : (uint32_t)w.cs;
        if (w.ok) {
            const uint64_t dpos = a.q_deposit / cs;
            if (dpos) {   // sixteen path reads per lane in flight (the rest of the wave waits for this)
                for (uint32_t i0 = j; i0 < w.s; i0 += 16 * L) {
                    uint32_t e[16];
#pragma unroll
                    for (uint32_t u = 0; u < 16; ++u) {
                        const uint32_t i = i0 + u * L;
                        e[u] = i < w.s ? a.path[(size_t)i * NA + ant] : 0u;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < 16; ++u)
                        if (i0 + u * L < w.s) a.depv.add(w.v, e[u], dpos);
                }
            }
            if (j == 0)
                atomicMin((unsigned long long *)&a.iter_key[w.v], (unsigned long long)(((uint64_t)cs << 32) | w.k));
        }
        if (j == 0) {
            a.ant_len[ant] = w.s;
            a.ant_cost[ant] = w.ok ? cs : kNoCost;
            atomicMax(&a.vlen[w.v], w.s);
            c_steps += w.s;
            c_cand += w.ncand;
            c_arr += w.ok ? 1 : 0;
            c_dh += w.ok ? w.s : 0;
            c_max = max(c_max, w.s);
        }
        w.pw = nullptr;
        have = false;
    }
    if (j == 0) a.slot_epoch[slot] = epoch;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        c_steps += __shfl_xor(c_steps, off);
        c_cand += __shfl_xor(c_cand, off);
        c_arr += __shfl_xor(c_arr, off);
        c_dh += __shfl_xor(c_dh, off);
        c_max = max(c_max, (uint32_t)__shfl_xor((int)c_max, off));
    }
    if (lane == 0) {
        if (c_steps) {
            atomicAdd((unsigned long long *)a.steps, (unsigned long long)c_steps);
            add_walk_counters(a.counters, kKindGlb, c_steps, c_cand, c_arr, c_dh);
            atomicMax(a.iter_max, c_max);
        }
        // the last wave out resets the ticket counters for the next launch
        const uint32_t waves = gridDim.x * (blockDim.x / kWave);
        if (atomicAdd(&a.tickets[1], 1u) == waves - 1) {
            a.tickets[0] = 0;
            a.tickets[1] = 0;
        }
    }
}

struct GlbListArgs {
    const gmacop_od *od;
    const uint8_t *vclass;
    const uint32_t *row_ptr, *node_lo;
    const int32_t *x, *y;
    uint32_t nq, ants, kgoal;
    GlbVeh *vrec;              // [nq] start data of each vehicle of this walker (k_glb_prep)
    GlbVeh *veh;               // [*glb_n] the launch's ordered list (k_glb_list)
    uint32_t *glb_n;
    uint32_t *vlen;            // [nq] longest walk of each vehicle in the previous launch; reset by k_glb_list
    uint32_t *ant_len, *ant_cost;
    const uint32_t *goal;      // exact goal rows [nq][goal_stride], or NULL: straight line
    uint32_t goal_stride;
};

// Once per call: the start data of every vehicle served by k_walk_glb; ants
// of vehicles no walker serves get an empty result.
__global__ void k_glb_prep(GlbListArgs a)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.nq) return;
    const uint8_t cls = a.vclass[v];
    if (cls == kWalkerGlobal) {
        const gmacop_od q = a.od[v];
        GlbVeh r;
        r.v = v; r.qid = q.qid; r.src = q.src; r.dst = q.dst;
        r.rs = a.row_ptr[q.src]; r.d = a.row_ptr[q.src + 1] - r.rs; r.n_lo = a.node_lo[q.src]; r.pad = 0;
        r.dx = a.x[q.dst]; r.dy = a.y[q.dst];
        const uint64_t hu = a.goal ? (uint64_t)a.goal[(size_t)v * a.goal_stride + (q.src - r.n_lo)]
                                   : (uint64_t)goal_ms(a.x[q.src], a.y[q.src], r.dx, r.dy, a.kgoal);
        r.hu_lo = (uint32_t)hu; r.hu_hi = (uint32_t)(hu >> 32);
        a.vrec[v] = r;
    } else if (cls == kWalkerNone) {
        for (uint32_t k = 0; k < a.ants; ++k) {
            a.ant_len[(size_t)v * a.ants + k] = 0;
            a.ant_cost[(size_t)v * a.ants + k] = kNoCost;
        }
    }
}

constexpr uint32_t kOrderBuckets = 256;   // longest-walk buckets of 4 steps (the last: 1020 and more)

// One block, before every k_walk_glb launch: the vehicles that walker
// serves, ordered by the longest walk each had in the previous launch,
// longest first.  Walk lengths persist from one iteration to the next, so
// long walks start early instead of trailing at the end of the launch; the
// order only schedules work (every ant's walk is fixed by its own counters).
__global__ __launch_bounds__(1024) void k_glb_list(GlbListArgs a)
{
    __shared__ uint32_t s_hist[kOrderBuckets];
    const uint32_t tid = threadIdx.x;
    for (uint32_t b = tid; b < kOrderBuckets; b += blockDim.x) s_hist[b] = 0;
    __syncthreads();
    for (uint32_t v = tid; v < a.nq; v += blockDim.x)
        if (a.vclass[v] == kWalkerGlobal) atomicAdd(&s_hist[min(a.vlen[v] >> 2, kOrderBuckets - 1)], 1u);
    __syncthreads();
    if (tid < kWave) {   // bucket start positions, longest bucket first: lane t scans buckets 255-4t .. 252-4t
        constexpr uint32_t per = kOrderBuckets / kWave;
        uint32_t c[per], sum = 0;
#pragma unroll
        for (uint32_t i = 0; i < per; ++i) {
            c[i] = s_hist[kOrderBuckets - 1 - (tid * per + i)];
            sum += c[i];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
            incl += (int)tid >= off ? o : 0u;
        }
        uint32_t run = incl - sum;
#pragma unroll
        for (uint32_t i = 0; i < per; ++i) {
            s_hist[kOrderBuckets - 1 - (tid * per + i)] = run;
            run += c[i];
        }
        if (tid == kWave - 1) *a.glb_n = incl;
    }
    __syncthreads();
    for (uint32_t v = tid; v < a.nq; v += blockDim.x)
        if (a.vclass[v] == kWalkerGlobal) {
            const uint32_t pos = atomicAdd(&s_hist[min(a.vlen[v] >> 2, kOrderBuckets - 1)], 1u);
            a.vlen[v] = 0;
            a.veh[pos] = a.vrec[v];
        }
}

struct BestArgs {
    uint32_t nq, ants, max_steps, load_update, m;
    uint32_t *iter_max;
    uint64_t *counters;
    const uint32_t *path, *ant_len;
    uint64_t *iter_key;
    uint32_t *best_path, *best_len, *best_cost;
    uint32_t *cnt;
};

// One wave per vehicle: the iteration-best ant (smallest packed key) replaces
// the best route when its cost is strictly lower; every road of the current
// best route adds one to its count for the load update.
__global__ __launch_bounds__(kWave) void k_best(BestArgs a)
{
    const uint32_t v = blockIdx.x, lane = threadIdx.x;
    if (v >= a.nq) return;
    const uint32_t NA = a.nq * a.ants;
    const uint64_t key = a.iter_key[v];
    const uint32_t bc = a.best_cost[v];
    const bool improve = key != kNoKey && (uint32_t)(key >> 32) < bc;
    const uint32_t ant = improve ? v * a.ants + (uint32_t)(key & 0xFFFFFFFFu) : 0;
    const uint32_t len = min(improve ? a.ant_len[ant] : a.best_len[v], a.max_steps);
    uint32_t *bp = a.best_path + (size_t)v * a.max_steps;
    for (uint32_t s = lane; s < len; s += kWave) {
        const uint32_t e = improve ? a.path[(size_t)s * NA + ant] : bp[s];
        if (improve) bp[s] = e;
        if (a.load_update && e < a.m) atomicAdd(&a.cnt[e], 1u);   // (a resumed route from a caller is not trusted)
    }
    if (lane == 0) {
        if (improve) {
            a.best_cost[v] = (uint32_t)(key >> 32);
            a.best_len[v] = len;
        }
        a.iter_key[v] = kNoKey;
        if (v == 0) {   // the walk of this iteration is complete: record its longest ant
            a.counters[4] += *a.iter_max;
            *a.iter_max = 0;
        }
    }
}

struct EdgeArgs {
    uint32_t m, rho, tau_min, tau_max, theta, load_update;
    uint32_t *tau, *load, *cnt;
    const uint32_t *base_load;
    uint64_t *dep;
    uint32_t *mir;             // road records of the global walker (8 words per road) or NULL
};

// Per road: tau <- clamp(floor(tau * (65536 - rho) / 65536) + Dp), with the
// deposit D scaled by theta / load on a congested road, floor(D * theta / L)
// computed exactly as (D / L) * theta + ((D % L) * theta) / L.  Then the load
// becomes the sensed load plus the vehicles whose best route uses the road.
__global__ void k_edge(EdgeArgs a)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.m) return;
    const uint64_t D = a.dep[e];
    const uint32_t L = a.load[e];
    uint64_t dp = D;
    if (L > a.theta) dp = (D / L) * a.theta + ((D % L) * a.theta) / L;
    uint64_t t = (((uint64_t)a.tau[e] * (65536u - a.rho)) >> 16) + dp;
    t = t < a.tau_min ? a.tau_min : (t > a.tau_max ? a.tau_max : t);
    a.tau[e] = (uint32_t)t;
    if (a.mir) a.mir[(size_t)e * 8 + 5] = (uint32_t)t;
    a.dep[e] = 0;
    if (a.load_update) {
        a.load[e] = a.base_load[e] + a.cnt[e];
        a.cnt[e] = 0;
    }
}

struct ApplyArgs {
    uint32_t m, cap, t_local, tau0, rho, tau_min, tau_max, theta;
    const uint32_t *load;     // frozen loads
    const uint32_t *gen;
    const uint32_t *slot_t, *slot_gen;   // serving: per-slot iteration and generation (else NULL)
    uint64_t *lazy, *dep;
    uint32_t *touched, *touched_n;
};

// Independent mode, one block per vehicle slot: for each road deposited on
// in iteration t, tau(t+1) = clamp(floor(tau(t) (65536-rho)/65536) + D'),
// D' = D or floor(D theta / load) -- the same update k_edge applies to a
// dense vector; every other road only evaporates, which its lazy entry
// already expresses.  Then the deposits and the list are cleared.
__global__ __launch_bounds__(256) void k_apply_touched(ApplyArgs a)
{
    const uint32_t v = blockIdx.x;
    const uint32_t n = min(a.touched_n[v], a.cap);
    uint64_t *lazy = a.lazy + (size_t)v * a.m;
    uint64_t *dep = a.dep + (size_t)v * a.m;
    const uint32_t gen = (a.slot_gen ? a.slot_gen[v] : *a.gen) & kGenMask;
    const uint32_t t_local = a.slot_t ? a.slot_t[v] : a.t_local;
    const uint32_t tau_def = evaporate_k(a.tau0, t_local, a.rho, a.tau_min);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t e = a.touched[(size_t)v * a.cap + i];
        const uint64_t x = lazy[e];
        const uint32_t tau = (uint32_t)(x >> 44) == gen
                                 ? evaporate_k((uint32_t)x, t_local - ((uint32_t)(x >> 32) & 0xFFFu), a.rho, a.tau_min)
                                 : tau_def;
        const uint64_t D = dep[e];
        const uint32_t L = a.load[e];
        uint64_t dp = D;
        if (L > a.theta) dp = (D / L) * a.theta + ((D % L) * a.theta) / L;
        uint64_t t = (((uint64_t)tau * (65536u - a.rho)) >> 16) + dp;
        t = t < a.tau_min ? a.tau_min : (t > a.tau_max ? a.tau_max : t);
        lazy[e] = t | ((uint64_t)(t_local + 1) << 32) | ((uint64_t)gen << 44);
        dep[e] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) a.touched_n[v] = 0;
}

// Dense pheromone of one independent slot after `t_end` iterations.
__global__ void k_materialize(const uint64_t *lazy_row, const uint32_t *genp, uint32_t m, uint32_t t_end,
                              uint32_t tau0, uint32_t rho, uint32_t tau_min, uint32_t *out)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint32_t gen = *genp & kGenMask;
    const uint64_t x = lazy_row[e];
    out[e] = (uint32_t)(x >> 44) == gen
                 ? evaporate_k((uint32_t)x, t_end - ((uint32_t)(x >> 32) & 0xFFFu), rho, tau_min)
                 : evaporate_k(tau0, t_end, rho, tau_min);
}

__global__ void k_next_generation(uint32_t *gen)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *gen = (*gen + 1) & kGenMask;
}

// Which walker serves each vehicle: none for an invalid query (node out of
// range, src == dst), else the LDS walker when its city's roads fit the LDS
// budget, else the global-memory walker.
__global__ void k_classify(const gmacop_od *od, uint32_t nq, uint32_t n, const uint32_t *node_inst,
                           const uint8_t *inst_fits_lds, uint8_t *vclass)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const gmacop_od q = od[v];
    uint8_t c = kWalkerNone;
    if (q.src < n && q.dst < n && q.src != q.dst) {
        const uint8_t ic = inst_fits_lds[node_inst[q.src]];
        c = ic ? ic : kWalkerGlobal;
    }
    vclass[v] = c;
}

// ---- exact goal term: shortest free-flow time to each vehicle's destination ----

// The in-roads of every node as (tail, free-flow time), in reverse-CSR order.
__global__ void k_rev_weights(uint32_t m, const uint32_t *rev_edge, const uint32_t *tail, const uint32_t *t0,
                              uint2 *rev_tw)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t e = rev_edge[i];
    rev_tw[i] = make_uint2(tail[e], t0[e]);
}

// Free-flow time of every road, t0 = floor(len * 360 / speed) ms in [1, 2^31]
// (the same quantity k_init_edges derives).
__global__ void k_free_flow(uint32_t m, const uint32_t *len_dm, const uint16_t *speed, uint32_t *t0)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint64_t x = (uint64_t)len_dm[e] * 360u / speed[e];
    x = x < 1 ? 1 : (x > kRoadCostCap ? kRoadCostCap : x);
    t0[e] = (uint32_t)x;
}

struct GoalArgs {
    const gmacop_od *od;       // queries; the destination of task v is od[v].dst
    const uint32_t *list;      // task i is vehicle list[i] (router: admitted slots), or NULL: vehicle i
    const uint32_t *dsts;      // or, when not NULL: task i is the destination dsts[i], row i
    uint32_t ntask, n, stride, qcap, fcap, delta;
    const uint32_t *node_inst, *inst_off, *rev_ptr;
    const uint2 *rev_tw;       // [m] (tail, free-flow time) of the in-roads of each node
    uint32_t *goal;            // [vehicles][stride] rows, city-local node ids (the terms, lowered in place)
    uint32_t *work;            // per block: done [stride], fmark [stride], near queues 2 x qcap, far queues 2 x fcap
    uint32_t *ctl;             // [0] next task, [1] blocks done (the last block out resets both)
};

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr uint32_t kGoalFar = 0xFFFFFFFFu;   // goal term of a node that cannot reach the destination
constexpr uint32_t kGoalCap = 0xFFFFFFFEu;   // largest finite goal term

// Calc_Dist (Alg. 2 step 1) as an exact term: for each task's vehicle, the
// shortest free-flow time from every node of its city to its destination,
// min(d, 2^32 - 2), and 2^32 - 1 where the destination is out of reach.  A
// persistent grid; a block takes one destination at a time and relaxes the
// reversed roads (label correcting).  The result is the unique
// shortest-distance vector, whatever order the relaxations run in; the order
// only decides the work.
//
// Order (near-far): terms below a moving split are relaxed first, in rounds
// from a near queue; a term lowered to or above the split goes to a far
// queue (once per phase, by a phase mark).  When the near queue runs dry the
// split moves up by delta and the far queue is sorted again into near and
// far.  A node is pending while its term is below done[x], the term it was
// last relaxed with; queues only point at candidates, so a stale or repeated
// entry is skipped.  If a queue would overflow, the task switches to scan
// rounds: every pending node of the city below the split, with the split
// moved to the smallest pending term when none is left.  The block size is
// chosen per call, so the kernel takes it from blockDim.
__global__ __launch_bounds__(1024) void k_goal_sssp(GoalArgs a)
{
    __shared__ uint32_t s_task, s_nn, s_fn, s_ovf, s_work, s_min;
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    uint32_t *done = a.work + (size_t)blockIdx.x * (2 * (size_t)a.stride + 2 * (size_t)a.qcap + 2 * (size_t)a.fcap);
    uint32_t *fmark = done + a.stride;
    uint32_t *nq[2] = {fmark + a.stride, fmark + a.stride + a.qcap};
    uint32_t *fq[2] = {nq[1] + a.qcap, nq[1] + a.qcap + a.fcap};
    for (;;) {
        if (tid == 0) s_task = atomicAdd(&a.ctl[0], 1u);
        __syncthreads();
        const uint32_t ti = s_task;
        __syncthreads();
        if (ti >= a.ntask) break;
        const uint32_t v = a.list ? a.list[ti] : ti;
        gmacop_od q;
        if (a.dsts) {
            q.dst = a.dsts[ti];
            q.src = q.dst ^ 1u;   // only its validity is looked at
            if (q.dst >= a.n) continue;
        } else {
            q = a.od[v];
            if (q.src >= a.n || q.dst >= a.n || q.src == q.dst) continue;   // no walk for this vehicle
        }
        const uint32_t city = a.node_inst[q.dst];
        const uint32_t n_lo = a.inst_off[city], nc = a.inst_off[city + 1] - n_lo;
        const uint32_t dl = q.dst - n_lo;
        uint32_t *dist = a.goal + (size_t)v * a.stride;
        for (uint32_t i = tid; i < nc; i += nthr) {
            dist[i] = i == dl ? 0u : kGoalFar;
            done[i] = kGoalFar;
            fmark[i] = 0;
        }
        if (tid == 0) nq[0][0] = dl;
        uint32_t nn = 1, nf = 0, ncur = 0, fcur = 0, phase = 1;
        uint64_t split = a.delta;
        bool scan = false;       // sticky: a queue overflowed, rounds scan the city
        __syncthreads();
        for (;;) {
            // ---- near rounds: relax pending nodes below the split until none is left ----
            for (;;) {
                if (tid == 0) {
                    s_nn = 0;
                    s_ovf = 0;
                    s_work = 0;
                    s_fn = nf;
                }
                __syncthreads();
                const uint32_t lim = scan ? nc : nn;
                const uint32_t *src = nq[ncur];
                uint32_t *dstq = nq[ncur ^ 1], *far = fq[fcur];
                for (uint32_t i = tid; i < lim; i += nthr) {
                    const uint32_t x = scan ? i : ld_agent(&src[i]);
                    const uint32_t d = ld_agent(&dist[x]);
                    if (d >= ld_agent(&done[x]) || d >= split) continue;   // relaxed already, or not near yet
                    atomicMin(&done[x], d);   // (a smaller term relaxed by another thread keeps its mark)
                    if (scan) s_work = 1;
                    const uint32_t jb = a.rev_ptr[n_lo + x], je = a.rev_ptr[n_lo + x + 1];
                    for (uint32_t j0 = jb; j0 < je; j0 += 8) {   // up to eight in-roads with their atomics in flight
                        uint32_t ul[8], nd[8], old[8];
#pragma unroll
                        for (uint32_t u = 0; u < 8; ++u) {
                            ul[u] = 0;
                            nd[u] = kGoalFar;
                            if (j0 + u < je) {
                                const uint2 tw = a.rev_tw[j0 + u];
                                const uint64_t s = (uint64_t)d + tw.y;
                                ul[u] = tw.x - n_lo;
                                nd[u] = s > kGoalCap ? kGoalCap : (uint32_t)s;
                            }
                        }
#pragma unroll
                        for (uint32_t u = 0; u < 8; ++u) old[u] = j0 + u < je ? atomicMin(&dist[ul[u]], nd[u]) : 0u;
#pragma unroll
                        for (uint32_t u = 0; u < 8; ++u) {
                            if (!(j0 + u < je && nd[u] < old[u]) || scan) continue;
                            if (nd[u] < split) {
                                const uint32_t pos = atomicAdd(&s_nn, 1u);
                                if (pos < a.qcap) st_agent(&dstq[pos], ul[u]);
                                else s_ovf = 1;
                            } else if (atomicExch(&fmark[ul[u]], phase) != phase) {
                                const uint32_t pos = atomicAdd(&s_fn, 1u);
                                if (pos < a.fcap) st_agent(&far[pos], ul[u]);
                                else s_ovf = 1;
                            }
                        }
                    }
                }
                __syncthreads();
                const bool more = scan ? s_work != 0 : s_nn != 0;
                const bool ovf = s_ovf != 0;
                nn = s_nn;
                nf = s_fn;
                if (ovf) scan = true;
                ncur ^= 1;
                __syncthreads();   // every thread has read the counters before they are reset
                if (!more && !ovf) break;
            }
            // ---- move the split up ----
            if (scan) {   // the smallest pending term of the city, if any
                if (tid == 0) s_min = kGoalFar;
                __syncthreads();
                for (uint32_t i = tid; i < nc; i += nthr) {
                    const uint32_t d = ld_agent(&dist[i]);
                    if (d < ld_agent(&done[i])) atomicMin(&s_min, d);
                }
                __syncthreads();
                const uint32_t mn = s_min;
                __syncthreads();
                if (mn == kGoalFar) break;
                split = ((uint64_t)mn / a.delta + 1) * a.delta;
                continue;
            }
            if (nf == 0) break;
            split += a.delta;
            for (;;) {   // sort the far queue into near (below the new split) and the next far queue
                ++phase;
                if (tid == 0) {
                    s_nn = 0;
                    s_fn = 0;
                    s_ovf = 0;
                    s_min = kGoalFar;
                }
                __syncthreads();
                const uint32_t *fsrc = fq[fcur];
                uint32_t *fdst = fq[fcur ^ 1], *near = nq[ncur];
                for (uint32_t i = tid; i < nf; i += nthr) {
                    const uint32_t y = ld_agent(&fsrc[i]);
                    const uint32_t d = ld_agent(&dist[y]);
                    if (d >= ld_agent(&done[y])) continue;   // relaxed since it was queued
                    if (d < split) {
                        const uint32_t pos = atomicAdd(&s_nn, 1u);
                        if (pos < a.qcap) st_agent(&near[pos], y);
                        else s_ovf = 1;
                    } else if (atomicExch(&fmark[y], phase) != phase) {
                        atomicMin(&s_min, d);
                        const uint32_t pos = atomicAdd(&s_fn, 1u);
                        if (pos < a.fcap) st_agent(&fdst[pos], y);
                        else s_ovf = 1;
                    }
                }
                __syncthreads();
                nn = s_nn;
                nf = s_fn;
                const uint32_t mn = s_min;
                if (s_ovf) scan = true;
                fcur ^= 1;
                __syncthreads();
                if (scan || nn > 0 || nf == 0) break;
                split = ((uint64_t)mn / a.delta + 1) * a.delta;   // skip empty bands
            }
            if (!scan && nn == 0 && nf == 0) break;
        }
        __syncthreads();   // the workspace is rewritten by the next task
    }
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&a.ctl[1], 1u) == gridDim.x - 1) {
            a.ctl[0] = 0;
            a.ctl[1] = 0;
        }
    }
}

// ---- traffic simulation of trips along routes (Section 5) ----

struct SimArgs {
    const uint32_t *path;        // [vehicles][stride] roads of each route
    const uint32_t *path_len;    // [vehicles] (0: no route, the vehicle stays out)
    const uint32_t *spd;         // [vehicles] km/h
    const uint32_t *scen_off;    // [nscen + 1] first vehicle of each scenario
    uint32_t stride, nscen, m, tick_ms, max_ticks, theta, th_max, t_max;
    const uint32_t *col, *len_dm, *rev_ptr, *rev_edge;
    const uint16_t *speed;
    const uint4 *sig;            // per road: head's cycle, green window start and length
    uint32_t *counts;            // [nscen][2][m] vehicles on / stopped at the end of each road, or NULL: in LDS
    uint64_t *pos;               // [vehicles] position on the current road, 1/360 dm
    uint32_t *road, *waited;     // [vehicles] index into the route; wait at the current stop line
    uint8_t *stopped, *active, *act;   // [vehicles] flags; this tick's change (1 passed, 2 stopped, 3 arrived)
    uint32_t *arrival, *wait_total;    // [vehicles] results: arrival time (ms), total signal wait (ms)
    uint32_t *ticks;             // [nscen] ticks run
};

constexpr uint32_t kNoArrival = 0xFFFFFFFFu;

// One workgroup per scenario, every tick of it in one launch: a tick first
// decides every vehicle's move from the counts at the tick's start (vehicles
// on each road, and stopped at its end), then applies the changes to the
// counts, with a barrier after each half.  The counts sit in LDS when the
// roads fit, else in a global slice of the scenario (read at device scope,
// since the atomics that change them bypass the CU's cache).  A vehicle
// stopped at the end of road e passes when its approach is green -- the head
// has no signal, e's queue is the longest non-empty one at the head (ties:
// lowest road id) or exceeds Th_max, or the time lies in e's green window --
// or when it has waited T_max; a moving vehicle covers min(its speed, the
// road's) km/h, slowed by theta / N above theta vehicles.
__global__ __launch_bounds__(1024) void k_simulate(SimArgs a)
{
    extern __shared__ uint32_t s_cnt[];   // [2][m] when the roads fit
    __shared__ uint32_t s_rem;
    const uint32_t b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    if (b >= a.nscen) return;
    const uint32_t v0 = a.scen_off[b], v1 = a.scen_off[b + 1];
    const bool in_lds = a.counts == nullptr;
    uint32_t *N = in_lds ? s_cnt : a.counts + (size_t)b * 2 * a.m;
    uint32_t *Q = N + a.m;
    auto rd = [&](const uint32_t *c, uint32_t e) { return in_lds ? c[e] : ld_agent(c + e); };
    auto barrier = [&] {   // global counts: every atomic and store complete at device scope first
        if (!in_lds) __threadfence();
        __syncthreads();
    };
    for (uint32_t e = tid; e < 2 * a.m; e += nt) {
        if (in_lds) N[e] = 0;
        else st_agent(N + e, 0u);
    }
    if (tid == 0) s_rem = 0;
    barrier();
    for (uint32_t i = v0 + tid; i < v1; i += nt) {
        const bool go = a.path_len[i] > 0;
        a.pos[i] = 0;
        a.road[i] = 0;
        a.waited[i] = 0;
        a.wait_total[i] = 0;
        a.stopped[i] = 0;
        a.active[i] = go ? 1 : 0;
        a.arrival[i] = kNoArrival;
        if (go) {
            atomicAdd(&N[a.path[(size_t)i * a.stride]], 1u);
            atomicAdd(&s_rem, 1u);
        }
    }
    barrier();
    uint32_t k = 0;
    for (; k < a.max_ticks; ++k) {
        if (s_rem == 0) break;   // read by every thread after the barrier: the same value
        const uint64_t t = (uint64_t)k * a.tick_ms;
        for (uint32_t i = v0 + tid; i < v1; i += nt) {   // decide
            a.act[i] = 0;
            if (!a.active[i]) continue;
            const uint32_t *route = a.path + (size_t)i * a.stride;
            const uint32_t r = a.road[i], e = route[r];
            if (a.stopped[i]) {
                const uint4 sg = a.sig[e];
                const uint32_t qe = rd(Q, e);
                bool green = sg.x == 0 || qe > a.th_max;
                if (!green) {   // the longest queue at the head; e's own queue holds this vehicle
                    const uint32_t head = a.col[e];
                    bool first = true;
                    for (uint32_t j = a.rev_ptr[head]; j < a.rev_ptr[head + 1] && first; ++j) {
                        const uint32_t f = a.rev_edge[j];
                        if (f == e) continue;
                        const uint32_t qf = rd(Q, f);
                        first = qf < qe || (qf == qe && f > e);
                    }
                    green = first;
                }
                if (!green) green = ((t % sg.x + sg.x - sg.y) % sg.x) < sg.z;
                if (green || a.waited[i] >= a.t_max) {
                    a.road[i] = r + 1;
                    a.pos[i] = 0;
                    a.stopped[i] = 0;
                    a.waited[i] = 0;
                    a.act[i] = 1;
                } else {
                    a.waited[i] += a.tick_ms;
                    a.wait_total[i] += a.tick_ms;
                }
                continue;
            }
            uint64_t v = min(a.spd[i], (uint32_t)a.speed[e]);
            const uint32_t ne = rd(N, e);
            if (ne > a.theta) {
                v = v * a.theta / ne;
                if (v == 0) v = 1;
            }
            const uint64_t np = a.pos[i] + v * a.tick_ms, L = (uint64_t)a.len_dm[e] * 360u;
            if (np < L) {
                a.pos[i] = np;
            } else if (r + 1 == a.path_len[i]) {
                const uint64_t at = t + a.tick_ms;
                a.arrival[i] = at > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)at;
                a.active[i] = 0;
                a.act[i] = 3;
            } else {
                a.pos[i] = L;
                a.stopped[i] = 1;
                a.waited[i] = 0;
                a.act[i] = 2;
            }
        }
        barrier();
        for (uint32_t i = v0 + tid; i < v1; i += nt) {   // apply the tick's changes to the counts
            const uint8_t c = a.act[i];
            if (!c) continue;
            const uint32_t *route = a.path + (size_t)i * a.stride;
            const uint32_t r = a.road[i];
            if (c == 1) {   // left road r - 1 from its stop line, now on road r
                atomicSub(&N[route[r - 1]], 1u);
                atomicSub(&Q[route[r - 1]], 1u);
                atomicAdd(&N[route[r]], 1u);
            } else if (c == 2) {
                atomicAdd(&Q[route[r]], 1u);
            } else {
                atomicSub(&N[route[r]], 1u);
                atomicSub(&s_rem, 1u);
            }
        }
        barrier();
    }
    if (tid == 0) a.ticks[b] = k;
}

// The shortest free-flow route of each vehicle (the Dijkstra baseline of
// Table 1), one lane per vehicle: from the source, repeatedly the first
// out-road in road order whose free-flow time equals the drop of the exact
// goal term along it, until the destination.  Length 0 when the destination
// is out of reach, its time reaches the 2^32 - 2 cap, or the route has more
// than max_steps roads.
__global__ void k_shortest_route(const gmacop_od *od, uint32_t nq, uint32_t n, uint32_t max_steps,
                                 const uint32_t *row_ptr, const uint32_t *col, const uint32_t *t0,
                                 const uint32_t *node_lo, const uint32_t *goal, uint32_t stride, uint32_t *path,
                                 uint32_t *len, uint32_t *cost, uint64_t *steps)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const gmacop_od q = od[v];
    uint32_t L = 0, c = kNoCost;
    if (q.src < n && q.dst < n && q.src != q.dst) {
        const uint32_t n_lo = node_lo[q.dst];
        const uint32_t *h = goal + (size_t)v * stride;
        const uint32_t hs = h[q.src - n_lo];
        if (hs < 0xFFFFFFFEu) {
            uint32_t u = q.src;
            bool fits = true;
            while (u != q.dst) {
                const uint32_t hu = h[u - n_lo];
                uint32_t next = 0xFFFFFFFFu;
                for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                    if ((uint64_t)t0[e] + h[col[e] - n_lo] == hu) {
                        next = e;
                        break;
                    }
                if (next == 0xFFFFFFFFu || L == max_steps) {   // (the first cannot happen for a finite term)
                    fits = false;
                    break;
                }
                path[(size_t)v * max_steps + L++] = next;
                u = col[next];
            }
            if (fits) c = hs;
            else L = 0;
        }
    }
    len[v] = L;
    cost[v] = c;
    if (L) atomicAdd((unsigned long long *)steps, (unsigned long long)L);
}

// ---- the literal MACO-P vehicle loop (Fig. 3), synchronous ticks ----

struct GreedyArgs {
    const gmacop_od *od;
    uint32_t nq, n, max_steps, theta, stride;
    const uint32_t *row_ptr, *col, *cost, *node_inst, *inst_off, *inst_eoff, *base_load;
    const uint32_t *goal;      // [nq][stride] exact goal rows (city-local node ids)
    uint32_t *node;            // [nq] current node, kGone once stopped
    uint32_t *choice;          // [nq] road taken in this tick, kGone if none
    const uint32_t *vcity;     // [nq] city of the vehicle, kGone for an invalid query (k_greedy_prep)
    uint64_t *csum;            // [nq] cost so far
    uint64_t *mark, *msum;     // [m] marker, and the city's moves so far when it was set
    uint32_t *cnt;             // [m] moves along the road in this tick (zero between ticks)
    uint32_t *mark_out;        // [m] markers after the last tick (saturated to 32 bits)
    uint32_t *path, *len, *cost_out;   // [nq][max_steps], [nq], [nq] (len 0 / cost kNoCost set beforehand)
    uint64_t *steps;
};

constexpr uint32_t kGone = 0xFFFFFFFFu;

// A marker at the city's move count sm: every move since it was set took one from it, floored at zero.
__device__ __forceinline__ uint64_t marker_at(const GreedyArgs &a, uint32_t e, uint64_t sm)
{
    const uint64_t x = __hip_atomic_load(&a.mark[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t d = sm - __hip_atomic_load(&a.msum[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return x > d ? x - d : 0;
}

// Per vehicle, before k_greedy: its city (kGone for an invalid query), start node, cost so far, no choice.
__global__ void k_greedy_prep(const gmacop_od *od, uint32_t nq, uint32_t n, const uint32_t *node_inst,
                              uint32_t *vcity, uint32_t *node, uint32_t *choice, uint64_t *csum)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nq) return;
    const gmacop_od q = od[v];
    const bool valid = q.src < n && q.dst < n && q.src != q.dst;
    vcity[v] = valid ? node_inst[q.src] : kGone;
    node[v] = valid ? q.src : kGone;
    choice[v] = kGone;
    csum[v] = 0;
}

// One block per city (Fig. 3, one tick at a time): every vehicle still
// travelling takes, among the roads whose head has a smaller exact goal
// term, the one with the least marker (ties: lowest road id), or the second
// least when the city's travelling vehicles exceed theta; then every road
// chosen by c of the tick's M moves becomes max(0, marker + c - (M - c)),
// and every other road loses M (kept lazily: a marker stores the city's move
// count when it was set).  A vehicle without a candidate, or still travelling
// after max_steps ticks, has no route.
__global__ __launch_bounds__(1024) void k_greedy(GreedyArgs a)
{
    __shared__ uint32_t s_travel, s_moves;
    const uint32_t city = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t n_lo = a.inst_off[city];
    const uint32_t e_lo = a.inst_eoff[city], e_hi = a.inst_eoff[city + 1];
    for (uint32_t e = e_lo + tid; e < e_hi; e += nthr) {   // markers start at the sensed loads
        __hip_atomic_store(&a.mark[e], (uint64_t)a.base_load[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.msum[e], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.cnt[e] = 0;
    }
    if (tid == 0) s_travel = 0;
    __syncthreads();
    for (uint32_t v = tid; v < a.nq; v += nthr)   // a vehicle is always handled by the same thread
        if (a.vcity[v] == city) atomicAdd(&s_travel, 1u);
    __syncthreads();
    uint64_t sm = 0;
    for (uint32_t t = 0; t < a.max_steps; ++t) {
        const uint32_t N = s_travel;   // travelling at the tick's start
        __syncthreads();
        if (N == 0) break;
        if (tid == 0) {
            s_moves = 0;
            s_travel = 0;
        }
        __syncthreads();
        for (uint32_t v = tid; v < a.nq; v += nthr) {   // choose and move, on the markers of the tick's start
            if (a.vcity[v] != city) continue;
            const uint32_t u = a.node[v];
            if (u == kGone) continue;
            const uint32_t *hv = a.goal + (size_t)v * a.stride;
            const uint32_t hu = hv[u - n_lo];
            uint32_t best = kGone, second = kGone;
            uint64_t pb = 0, ps = 0;
            for (uint32_t e = a.row_ptr[u]; e < a.row_ptr[u + 1]; ++e) {
                if (!(hv[a.col[e] - n_lo] < hu)) continue;   // not leading toward the destination
                const uint64_t pe = marker_at(a, e, sm);
                if (best == kGone || pe < pb) {
                    second = best;
                    ps = pb;
                    best = e;
                    pb = pe;
                } else if (second == kGone || pe < ps) {
                    second = e;
                    ps = pe;
                }
            }
            if (best == kGone) {   // destination out of reach: stops without a route
                a.node[v] = kGone;
                continue;
            }
            const uint32_t e = (N > a.theta && second != kGone) ? second : best;
            const gmacop_od q = a.od[v];
            a.path[(size_t)v * a.max_steps + a.len[v]] = e;
            a.len[v] += 1;
            const uint64_t cs = a.csum[v] + a.cost[e];
            a.csum[v] = cs;
            a.choice[v] = e;
            atomicAdd(&a.cnt[e], 1u);
            atomicAdd(&s_moves, 1u);
            const uint32_t x = a.col[e];
            if (x == q.dst) {
                a.node[v] = kGone;
                a.cost_out[v] = cs > kPathCostCap ? kPathCostCap : (uint32_t)cs;
            } else {
                a.node[v] = x;
                atomicAdd(&s_travel, 1u);
            }
        }
        __syncthreads();
        const uint32_t M = s_moves;
        for (uint32_t v = tid; v < a.nq; v += nthr) {   // the markers of the roads chosen in this tick
            const uint32_t e = a.vcity[v] == city ? a.choice[v] : kGone;
            if (e == kGone) continue;
            a.choice[v] = kGone;
            const uint32_t c = atomicExch(&a.cnt[e], 0u);   // the first of its vehicles applies the road's update
            if (!c) continue;
            const int64_t x = (int64_t)marker_at(a, e, sm) + (int64_t)c - (int64_t)(M - c);
            __hip_atomic_store(&a.mark[e], (uint64_t)(x < 0 ? 0 : x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.msum[e], sm + M, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        sm += M;
        __syncthreads();
    }
    for (uint32_t v = tid; v < a.nq; v += nthr)   // still travelling, or stopped without a route: none
        if (a.vcity[v] == city && a.cost_out[v] == kNoCost) a.len[v] = 0;
    for (uint32_t e = e_lo + tid; e < e_hi; e += nthr) {
        const uint64_t x = marker_at(a, e, sm);
        a.mark_out[e] = x > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)x;
    }
    if (tid == 0 && sm) atomicAdd((unsigned long long *)a.steps, (unsigned long long)sm);
}

// ---- serving: slot admission, advance, result gather ----

// Queries enter free slots: the slot's route starts empty at iteration 0
// with a fresh pheromone generation.  Slot ids at or above nslots are
// ignored (the host never sends one; the guard keeps every write in range).
__global__ void k_admit(const uint32_t *slots, const gmacop_od *ods, const uint32_t *gens, uint32_t n,
                        uint32_t nslots, gmacop_od *slot_od, uint32_t *slot_t, uint32_t *slot_gen,
                        uint32_t *best_len, uint32_t *best_cost, uint64_t *iter_key)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t sl = slots[i];
    if (sl >= nslots) return;
    slot_od[sl] = ods[i];
    slot_t[sl] = 0;
    slot_gen[sl] = gens[i];
    best_len[sl] = 0;
    best_cost[sl] = kNoCost;
    iter_key[sl] = kNoKey;
}

// After an iteration: every active slot moves to the next iteration; a slot
// that has run all iterations is retired (its query marked invalid, so the
// walkers skip it until a new query is admitted).
__global__ void k_advance(uint32_t nslots, uint32_t n, uint32_t iterations, gmacop_od *slot_od, uint32_t *slot_t)
{
    const uint32_t sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslots) return;
    const gmacop_od q = slot_od[sl];
    if (q.src >= n || q.dst >= n || q.src == q.dst) return;
    const uint32_t t = slot_t[sl] + 1;
    slot_t[sl] = t;
    if (t >= iterations) slot_od[sl] = gmacop_od{q.qid, 0xFFFFFFFFu, 0xFFFFFFFFu};
}

// Results of finished slots into contiguous buffers (one block per slot).  A
// slot id at or above nslots yields "no route" (the host never sends one).
__global__ void k_gather_done(const uint32_t *slots, uint32_t nslots, uint32_t max_steps, const uint32_t *best_path,
                              const uint32_t *best_len, const uint32_t *best_cost, uint32_t *out_path,
                              uint32_t *out_len, uint32_t *out_cost)
{
    const uint32_t i = blockIdx.x, sl = slots[i];
    if (sl >= nslots) {
        if (threadIdx.x == 0) {
            out_len[i] = 0;
            out_cost[i] = kNoCost;
        }
        return;
    }
    const uint32_t len = min(best_len[sl], max_steps);
    for (uint32_t s = threadIdx.x; s < len; s += blockDim.x)
        out_path[(size_t)i * max_steps + s] = best_path[(size_t)sl * max_steps + s];
    if (threadIdx.x == 0) {
        out_len[i] = len;
        out_cost[i] = best_cost[sl];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <typename T>
int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(GMACOP_E_NOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    return GMACOP_OK;
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

uint32_t bit_length(uint64_t x)
{
    uint32_t b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

unsigned blocks_for(uint64_t work, unsigned per_block)
{
    return (unsigned)((work + per_block - 1) / per_block);
}

}  // namespace

// Workspace of k_walk_glb: its vehicle list, counters, and per-slot visited
// words and epochs.  The words keep their meaning across calls as long as
// the slot layout stays the same; a new layout clears them.
struct GlbWork {
    GlbVeh *veh = nullptr, *vrec = nullptr;   // the launch's ordered list; start data per vehicle
    size_t cap_veh = 0, cap_vrec = 0;
    uint32_t *vlen = nullptr;          // [vehicles] longest walk in the last launch
    size_t cap_vlen = 0;
    uint32_t *ctl = nullptr;           // [0]: vehicles listed, [1]: next ticket, [2]: waves done
    uint64_t *words = nullptr;
    size_t cap_words = 0;
    uint32_t *epoch = nullptr;
    size_t cap_epoch = 0;
    uint64_t slots = 0, nw2 = 0;       // layout of `words`

    void release()
    {
        dfree(veh); dfree(vrec); dfree(vlen); dfree(ctl); dfree(words); dfree(epoch);
        veh = nullptr; vrec = nullptr; vlen = nullptr; ctl = nullptr; words = nullptr; epoch = nullptr;
        cap_veh = cap_vrec = cap_vlen = cap_words = cap_epoch = 0;
        slots = nw2 = 0;
    }
};

struct gmacop_graph {
    int device = 0;
    uint32_t n = 0, m = 0, n_inst = 1, max_deg = 0, max_indeg = 0;
    int max_lds = 65536;               // dynamic LDS a block may use on this device
    std::vector<uint32_t> inst_off;    // host copy, [n_inst+1]
    // static graph (device)
    uint32_t *row_ptr = nullptr, *col = nullptr, *len_dm = nullptr, *cycle = nullptr, *base_load = nullptr;
    uint32_t *rev_ptr = nullptr, *rev_edge = nullptr, *tail = nullptr;
    uint2 *rec = nullptr;              // head | head_out_degree << 24, head's first out-road (n < 2^24)
    uint4 *rec32 = nullptr;            // [m][2] global-walker road records: rec, head coordinates; cost, pheromone
    uint4 *rvs = nullptr;              // [m] static city-local road records of k_walk_ldsr
    uint32_t *node_lo = nullptr, *node_inst = nullptr;   // first node / index of each node's city
    uint32_t *inst_off_dev = nullptr, *inst_eoff_dev = nullptr;   // node / road range of each city
    uint8_t *inst_fits = nullptr;      // per city: served by the LDS walker in the current plan
    uint8_t *vclass = nullptr;         // per vehicle: walker of the current call
    size_t cap_vclass = 0;
    uint32_t max_city_nodes = 0;
    std::vector<uint8_t> city_class_dev;   // host copy of inst_fits
    std::vector<uint32_t> inst_eoff;   // host: first road of each city
    std::vector<uint64_t> inst_span2;  // host: squared diagonal of each city's bounding box
    uint16_t *speed = nullptr, *green = nullptr;
    int32_t *x = nullptr, *y = nullptr;
    // per-call state (device)
    uint32_t *t0 = nullptr, *wf = nullptr, *tau = nullptr, *load = nullptr, *cost = nullptr, *cnt = nullptr;
    uint64_t *dep = nullptr;
    // workspace, grown on demand
    size_t cap_path = 0, cap_ants = 0, cap_veh = 0, cap_best = 0, cap_bits = 0;
    uint32_t *path = nullptr, *ant_len = nullptr, *ant_cost = nullptr, *gbits = nullptr;
    uint64_t *iter_key = nullptr, *steps = nullptr;
    uint32_t *best_path = nullptr, *best_len = nullptr, *best_cost = nullptr;
    gmacop_od *od = nullptr;
    GlbWork glb;
    // exact goal term: rows per vehicle, the search's per-block workspace and task counter,
    // the in-roads as (tail, free-flow time)
    size_t cap_goal = 0, cap_goal_work = 0;
    uint32_t *goal = nullptr, *goal_work = nullptr, *goal_ctl = nullptr;
    uint32_t mean_t0 = 1;              // mean free-flow road time (ms), the scale of the search's bands
    // the literal MACO-P loop (GMACOP_MODE_GREEDY): per vehicle and per road state
    size_t cap_gveh = 0, cap_groad = 0;
    uint32_t *gnode = nullptr, *gchoice = nullptr, *gvcity = nullptr;
    uint64_t *gcsum = nullptr, *gmark = nullptr, *gmsum = nullptr;
    uint2 *rev_tw = nullptr;
    uint4 *sig = nullptr;              // [m] time-dependent signals: head's cycle, green window start and length
    std::vector<uint32_t> col_host, tail_host;   // head and tail of each road, copied on first need (route checks)
    // statistics
    uint64_t *counters = nullptr;         // device [kCounters]
    uint32_t *iter_max = nullptr;         // device [1]
    uint64_t launches[kTimedKernels] = {};
    double ms[kTimedKernels] = {};
    struct Timed { hipEvent_t a, b; int kernel; };
    // a second stream for the global walker, run beside the LDS walkers of the same iteration
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::vector<Timed> pending;           // recorded, not yet summed
    std::vector<hipEvent_t> spare;
    // independent mode: lazy pheromone and deposits per vehicle slot
    size_t cap_lazy = 0, cap_depi = 0, cap_touch = 0, cap_touchn = 0;
    uint64_t *lazy = nullptr, *dep_ind = nullptr;
    uint32_t *touched = nullptr, *touched_n = nullptr, *dev_gen = nullptr;
    uint32_t gen_count = 0;            // independent calls since the lazy array was cleared
    uint32_t last_mode = 0, last_nq = 0, last_iters = 0;
    gmacop_params last_p{};
    const uint64_t *last_lazy = nullptr;   // independent mode: the last call's pheromone rows and generation
    const uint32_t *last_gen = nullptr;
    // captured kernel sequence of the last GMACOP_HIP_GRAPH call and the key of its arguments
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;

    ~gmacop_graph()
    {
        (void)hipSetDevice(device);
        dfree(row_ptr); dfree(col); dfree(len_dm); dfree(cycle); dfree(base_load);
        dfree(rev_ptr); dfree(rev_edge); dfree(tail); dfree(rec); dfree(rec32); dfree(rvs); dfree(node_lo); dfree(node_inst);
        dfree(inst_fits); dfree(vclass); dfree(inst_off_dev); dfree(inst_eoff_dev); dfree(speed); dfree(green); dfree(x); dfree(y);
        dfree(t0); dfree(wf); dfree(tau); dfree(load); dfree(cost); dfree(cnt); dfree(dep);
        dfree(path); dfree(ant_len); dfree(ant_cost); dfree(gbits); dfree(iter_key); dfree(steps);
        dfree(best_path); dfree(best_len); dfree(best_cost); dfree(od); dfree(counters); dfree(iter_max);
        dfree(lazy); dfree(dep_ind); dfree(touched); dfree(touched_n); dfree(dev_gen);
        dfree(goal); dfree(goal_work); dfree(goal_ctl); dfree(rev_tw); dfree(sig);
        dfree(gnode); dfree(gchoice); dfree(gvcity); dfree(gcsum); dfree(gmark); dfree(gmsum);
        glb.release();
        for (auto &t : pending) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        for (auto e : spare) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (side) (void)hipStreamDestroy(side);
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

namespace {

template <typename T>
int upload(T **dst, const T *src, size_t count)
{
    int rc = dalloc(dst, count);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return GMACOP_OK;
}

// Grow a workspace buffer to at least `need` elements (contents discarded).
template <typename T>
int grow(T **p, size_t *cap, size_t need, bool zero)
{
    if (need <= *cap && *p) return GMACOP_OK;
    dfree(*p);
    *cap = 0;
    int rc = dalloc(p, need);
    if (rc) return rc;
    if (zero) {
        HIP_TRY(hipMemset(*p, 0, need * sizeof(T)));
        HIP_TRY(hipDeviceSynchronize());   // ordered before work on any stream
    }
    *cap = need;
    return GMACOP_OK;
}

// Size the k_walk_glb workspace for nq vehicles and `slots` slots of nw2 words.
int glb_prepare(GlbWork &w, uint32_t nq, uint64_t slots, uint32_t nw2)
{
    int rc;
    if ((rc = grow(&w.veh, &w.cap_veh, std::max<size_t>(nq, 1), false)) ||
        (rc = grow(&w.vrec, &w.cap_vrec, std::max<size_t>(nq, 1), false)) ||
        (rc = grow(&w.vlen, &w.cap_vlen, std::max<size_t>(nq, 1), true)))
        return rc;
    if (!w.ctl) {
        if ((rc = dalloc(&w.ctl, 3))) return rc;
        HIP_TRY(hipMemset(w.ctl, 0, 3 * sizeof(uint32_t)));
        HIP_TRY(hipDeviceSynchronize());
    }
    if (slots != w.slots || nw2 != w.nw2) {
        const size_t need = (size_t)slots * nw2;
        if ((rc = grow(&w.words, &w.cap_words, std::max<size_t>(need, 1), false)) ||
            (rc = grow(&w.epoch, &w.cap_epoch, std::max<size_t>(slots, 1), false)))
            return rc;
        HIP_TRY(hipMemset(w.words, 0, std::max<size_t>(need, 1) * sizeof(uint64_t)));
        HIP_TRY(hipMemset(w.epoch, 0, std::max<size_t>(slots, 1) * sizeof(uint32_t)));
        HIP_TRY(hipDeviceSynchronize());
        w.slots = slots;
        w.nw2 = nw2;
    }
    return GMACOP_OK;
}

int validate_desc(const gmacop_graph_desc *d)
{
    if (!d) return fail(GMACOP_E_INVAL, "desc is NULL");
    if (d->n_nodes < 2 || d->n_edges < 1) return fail(GMACOP_E_INVAL, "need n >= 2 and m >= 1");
    if (!d->row_ptr || !d->col || !d->len_dm || !d->speed_kmh || !d->green_pm || !d->cycle_ms || !d->x_dm ||
        !d->y_dm || !d->base_load)
        return fail(GMACOP_E_INVAL, "a graph array is NULL");
    const uint32_t n = d->n_nodes, m = d->n_edges;
    if (d->row_ptr[0] != 0 || d->row_ptr[n] != m) return fail(GMACOP_E_INVAL, "row_ptr must run from 0 to m");
    for (uint32_t u = 0; u < n; ++u) {
        if (d->row_ptr[u + 1] < d->row_ptr[u]) return fail(GMACOP_E_INVAL, "row_ptr decreases at node %u", u);
        for (uint32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; ++e) {
            if (d->col[e] >= n) return fail(GMACOP_E_INVAL, "col[%u] out of range", e);
            if (d->col[e] == u) return fail(GMACOP_E_INVAL, "self-loop at road %u", e);
        }
    }
    for (uint32_t e = 0; e < m; ++e) {
        if (d->len_dm[e] == 0) return fail(GMACOP_E_INVAL, "len_dm[%u] is 0", e);
        if (d->speed_kmh[e] == 0) return fail(GMACOP_E_INVAL, "speed_kmh[%u] is 0", e);
        if (d->green_pm[e] > 1000) return fail(GMACOP_E_INVAL, "green_pm[%u] > 1000", e);
    }
    const int32_t lim = 1 << 30;
    for (uint32_t v = 0; v < n; ++v)
        if (d->x_dm[v] <= -lim || d->x_dm[v] >= lim || d->y_dm[v] <= -lim || d->y_dm[v] >= lim)
            return fail(GMACOP_E_INVAL, "coordinates of node %u out of range", v);
    if (d->n_instances == 0) return fail(GMACOP_E_INVAL, "n_instances must be >= 1");
    if (d->n_instances > 1 && !d->inst_node_off) return fail(GMACOP_E_INVAL, "inst_node_off is NULL");
    if (d->inst_node_off) {
        const uint32_t *o = d->inst_node_off;
        if (o[0] != 0 || o[d->n_instances] != n) return fail(GMACOP_E_INVAL, "inst_node_off must run from 0 to n");
        for (uint32_t i = 0; i < d->n_instances; ++i) {
            if (o[i + 1] <= o[i]) return fail(GMACOP_E_INVAL, "empty or decreasing instance %u", i);
            for (uint32_t u = o[i]; u < o[i + 1]; ++u)
                for (uint32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; ++e)
                    if (d->col[e] < o[i] || d->col[e] >= o[i + 1])
                        return fail(GMACOP_E_INVAL, "road %u crosses instances", e);
        }
    }
    return GMACOP_OK;
}

uint32_t instance_of(const gmacop_graph *g, uint32_t node)
{
    return (uint32_t)(std::upper_bound(g->inst_off.begin(), g->inst_off.end(), node) - g->inst_off.begin()) - 1;
}

int take_event(gmacop_graph *g, hipEvent_t *e)
{
    if (!g->spare.empty()) {
        *e = g->spare.back();
        g->spare.pop_back();
        return GMACOP_OK;
    }
    HIP_TRY(hipEventCreate(e));
    return GMACOP_OK;
}

// Brackets one kernel launch with an event pair when timing is on.
struct KernelTimer {
    gmacop_graph *g;
    hipStream_t st;
    bool on;
    int start(int kernel, gmacop_graph::Timed *t)
    {
        g->launches[kernel]++;
        if (!on) return GMACOP_OK;
        t->kernel = kernel;
        int rc = take_event(g, &t->a);
        if (rc || (rc = take_event(g, &t->b))) return rc;
        HIP_TRY(hipEventRecord(t->a, st));
        return GMACOP_OK;
    }
    int stop(gmacop_graph::Timed *t)
    {
        if (!on) return GMACOP_OK;
        HIP_TRY(hipEventRecord(t->b, st));
        g->pending.push_back(*t);
        return GMACOP_OK;
    }
};

int validate_params(const gmacop_graph *g, const gmacop_params *p, uint32_t nq)
{
    if (!p) return fail(GMACOP_E_INVAL, "params is NULL");
    if (p->ants == 0) return fail(GMACOP_E_INVAL, "ants must be >= 1");
    if (p->max_steps == 0) return fail(GMACOP_E_INVAL, "max_steps must be >= 1");
    if (p->theta == 0) return fail(GMACOP_E_INVAL, "theta must be >= 1");
    if (p->rho_q16 > 65536u) return fail(GMACOP_E_INVAL, "rho_q16 must be <= 65536");
    if (p->tau_min_q16 == 0) return fail(GMACOP_E_INVAL, "tau_min_q16 must be >= 1");
    if (p->tau_min_q16 > p->tau0_q16 || p->tau0_q16 > p->tau_max_q16)
        return fail(GMACOP_E_INVAL, "need tau_min <= tau0 <= tau_max");
    if (p->mode > GMACOP_MODE_GREEDY) return fail(GMACOP_E_INVAL, "unknown mode %u", p->mode);
    if (p->flags & ~(GMACOP_NO_LOAD_UPDATE | GMACOP_DEVICE_PTRS | GMACOP_TIME_KERNELS | GMACOP_HIP_GRAPH |
                     GMACOP_GOAL_EXACT | GMACOP_RESUME | GMACOP_SIGNAL_TIMED))
        return fail(GMACOP_E_INVAL, "unknown flags");
    const uint32_t lg = g->max_deg <= 1 ? 0 : bit_length(g->max_deg - 1);
    if ((uint64_t)p->alpha * bit_length(p->tau_max_q16) + 16ull * p->beta + lg > 64)
        return fail(GMACOP_E_RANGE, "alpha*bits(tau_max) + 16*beta + ceil(log2(max degree)) exceeds 64");
    const unsigned __int128 dep =
        (unsigned __int128)(p->mode == GMACOP_MODE_SHARED ? nq : 1) * p->ants * p->q_deposit;
    if (dep >> 63) return fail(GMACOP_E_RANGE, "deposit total could reach 2^63");
    if (g->max_deg > kMaxDegree) return fail(GMACOP_E_UNSUPPORTED, "out-degree %u exceeds %u", g->max_deg, kMaxDegree);
    if ((uint64_t)nq * p->ants > 0xFFFFFFFFull) return fail(GMACOP_E_UNSUPPORTED, "more than 2^32 ants");
    return GMACOP_OK;
}

template <int MAXD>
int launch_walk(const WalkArgs &wa, bool lds, hipStream_t st)
{
    const uint64_t NA = (uint64_t)wa.nq * wa.ants;
    const unsigned grid = blocks_for(NA, kWave);
    if (lds) {
        const size_t sh = (size_t)wa.nwords * kWave * sizeof(uint32_t);
        hipLaunchKernelGGL((k_walk<MAXD, true>), dim3(grid), dim3(kWave), sh, st, wa);
    } else {
        hipLaunchKernelGGL((k_walk<MAXD, false>), dim3(grid), dim3(kWave), 0, st, wa);
    }
    HIP_TRY(hipGetLastError());
    return GMACOP_OK;
}

struct WalkPlan {
    uint32_t maxd = 4;             // candidate bound the kernels are built for
    bool legacy = false;           // k_walk for every vehicle (graphs with 2^24 nodes or more)
    uint32_t lds_lanes = 4, lds_apb = 0, lds_bpv = 0;
    uint32_t road_maxd = 4;               // candidate and in-road bound of k_walk_ldsr
    size_t lds_bytes[kLdsClasses + 1] = {};   // [c]: dynamic LDS of LDS class c's launch, 0 = none
    bool glb = false;              // some city is served by k_walk_glb
    bool timed = false;            // k_walk_glb costs roads by the time-dependent signal rule
    uint32_t glb_lanes = 4, glb_apb = 0, bloom_log2 = 11, glb_nwords = 0;
    uint32_t glb_blocks = 0;       // resident grid of k_walk_glb (glb_grid)
    size_t glb_lds_bytes = 0;
    std::vector<uint8_t> city_class;      // per city: LDS class 1..kLdsClasses, or 0 = global walker
    bool any_lds() const
    {
        for (int c = 1; c <= kLdsClasses; ++c)
            if (lds_bytes[c]) return true;
        return false;
    }
};

template <int L, int MAXD>
int launch_walk_lds(const LdsWalkArgs &wa, const WalkPlan &pl, hipStream_t st, bool setup)
{
    constexpr int CH = (MAXD + L - 1) / L;
    const bool road = is_road_class(wa.cls);
    auto kern = road ? k_walk_ldsr<L, CH> : k_walk_lds<L, CH>;
    if (setup) {   // before any launch: allow the largest dynamic LDS of the classes this kernel serves
        size_t mx = 0;
        for (uint32_t c = 1; c <= kLdsClasses; ++c)
            if (is_road_class(c) == road) mx = std::max(mx, pl.lds_bytes[c]);
        if (mx > 65536)
            HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx));
        return GMACOP_OK;
    }
    const unsigned grid = wa.nq * pl.lds_bpv;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(pl.lds_apb * L), pl.lds_bytes[wa.cls], st, wa);
    HIP_TRY(hipGetLastError());
    return GMACOP_OK;
}

template <int L>
int launch_walk_lds_d(const LdsWalkArgs &wa, const WalkPlan &pl, hipStream_t st, bool setup)
{
    switch (is_road_class(wa.cls) ? pl.road_maxd : pl.maxd) {
    case 4: return launch_walk_lds<L, 4>(wa, pl, st, setup);
    case 8: return launch_walk_lds<L, 8>(wa, pl, st, setup);
    case 16: return launch_walk_lds<L, 16>(wa, pl, st, setup);
    default: return launch_walk_lds<L, 32>(wa, pl, st, setup);
    }
}

int launch_walk_lds_any(const LdsWalkArgs &wa, const WalkPlan &pl, hipStream_t st, bool setup = false);

// Before the first launch: raise the dynamic-LDS limit of both LDS walker kernels as the plan needs.
int setup_walk_lds(LdsWalkArgs wa, const WalkPlan &pl, hipStream_t st)
{
    int rc = GMACOP_OK;
    for (uint32_t c : {1u, 4u}) {
        wa.cls = c;
        if ((rc = launch_walk_lds_any(wa, pl, st, true))) return rc;
    }
    return rc;
}

// One launch per LDS class that some city of the plan uses.
int launch_walk_lds_classes(LdsWalkArgs wa, const WalkPlan &pl, hipStream_t st)
{
    int rc = GMACOP_OK;
    for (uint32_t c = 1; c <= (uint32_t)kLdsClasses && !rc; ++c)
        if (pl.lds_bytes[c]) {
            wa.cls = c;
            rc = launch_walk_lds_any(wa, pl, st);
        }
    return rc;
}

int launch_walk_lds_any(const LdsWalkArgs &wa, const WalkPlan &pl, hipStream_t st, bool setup)
{
    switch (pl.lds_lanes) {
    case 1: return launch_walk_lds_d<1>(wa, pl, st, setup);
    case 2: return launch_walk_lds_d<2>(wa, pl, st, setup);
    case 4: return launch_walk_lds_d<4>(wa, pl, st, setup);
    default: return launch_walk_lds_d<8>(wa, pl, st, setup);
    }
}

template <int L, int MAXD>
int launch_walk_glb(const GlbWalkArgs &wa, const WalkPlan &pl, hipStream_t st)
{
    constexpr int CH = (MAXD + L - 1) / L;
    if (pl.timed)
        hipLaunchKernelGGL((k_walk_glb<L, CH, true>), dim3(pl.glb_blocks), dim3(pl.glb_apb * L), pl.glb_lds_bytes, st,
                           wa);
    else
        hipLaunchKernelGGL((k_walk_glb<L, CH, false>), dim3(pl.glb_blocks), dim3(pl.glb_apb * L), pl.glb_lds_bytes,
                           st, wa);
    HIP_TRY(hipGetLastError());
    return GMACOP_OK;
}

template <int L>
int launch_walk_glb_d(const GlbWalkArgs &wa, const WalkPlan &pl, hipStream_t st)
{
    switch (pl.maxd) {
    case 4: return launch_walk_glb<L, 4>(wa, pl, st);
    case 8: return launch_walk_glb<L, 8>(wa, pl, st);
    case 16: return launch_walk_glb<L, 16>(wa, pl, st);
    default: return launch_walk_glb<L, 32>(wa, pl, st);
    }
}

int launch_walk_glb_any(const GlbWalkArgs &wa, const WalkPlan &pl, hipStream_t st)
{
    switch (pl.glb_lanes) {
    case 1: return launch_walk_glb_d<1>(wa, pl, st);
    case 2: return launch_walk_glb_d<2>(wa, pl, st);
    case 4: return launch_walk_glb_d<4>(wa, pl, st);
    default: return launch_walk_glb_d<8>(wa, pl, st);
    }
}

template <int L, int MAXD>
const void *glb_kernel(bool tm)
{
    constexpr int CH = (MAXD + L - 1) / L;
    return tm ? (const void *)k_walk_glb<L, CH, true> : (const void *)k_walk_glb<L, CH, false>;
}

template <int L>
const void *glb_kernel_d(uint32_t maxd, bool tm)
{
    return maxd <= 4 ? glb_kernel<L, 4>(tm) : maxd <= 8 ? glb_kernel<L, 8>(tm) : maxd <= 16 ? glb_kernel<L, 16>(tm)
                                                                                          : glb_kernel<L, 32>(tm);
}

// The persistent grid of k_walk_glb: as many blocks as stay resident on the
// device (fewer when there are fewer ants), and no more than keep the
// per-slot visited words within kGlbWordsBudget.
int glb_grid(int device, WalkPlan &pl, uint64_t NA)
{
    const uint32_t L = pl.glb_lanes;
    const void *kern = L == 1 ? glb_kernel_d<1>(pl.maxd, pl.timed) : L == 2 ? glb_kernel_d<2>(pl.maxd, pl.timed)
                       : L == 4 ? glb_kernel_d<4>(pl.maxd, pl.timed) : glb_kernel_d<8>(pl.maxd, pl.timed);
    int nb = 0, cus = 0;
    if (pl.glb_lds_bytes > 65536)   // Bloom filters beyond the default dynamic-LDS limit
        HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.glb_lds_bytes));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, (int)(pl.glb_apb * L), pl.glb_lds_bytes));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    uint64_t blocks = (uint64_t)std::max(nb, 1) * (uint64_t)std::max(cus, 1);
    blocks = std::min<uint64_t>(blocks, (NA + pl.glb_apb - 1) / pl.glb_apb);
    const uint64_t per_block = (uint64_t)pl.glb_apb * std::max<uint32_t>(pl.glb_nwords, 1) * sizeof(uint64_t);
    blocks = std::min<uint64_t>(blocks, std::max<uint64_t>((uint64_t)std::max(cus, 1), kGlbWordsBudget / per_block));
    pl.glb_blocks = (uint32_t)std::max<uint64_t>(blocks, 1);
    return GMACOP_OK;
}

uint32_t env_u32(const char *name, uint32_t dflt)
{
    const char *v = getenv(name);
    return (v && *v) ? (uint32_t)strtoul(v, nullptr, 10) : dflt;
}

uint32_t lanes_or(uint32_t L, uint32_t dflt) { return (L == 1 || L == 2 || L == 4 || L == 8) ? L : dflt; }

// The per-size schedule.  Every city whose staged roads and visited state
// fit in LDS goes to an LDS walker, in one of three size tiers (up to a
// quarter, a half, or all of the LDS a block may use), so small cities are
// not charged the largest city's LDS: k_walk_ldsr (visited state per road,
// classes 1..3) where its layout fits, else k_walk_lds (visited state per
// node, classes 4..6); larger cities go to k_walk_glb.  GMACOP_WALK_KERNEL
// (lds: LDS walkers wherever a city fits, whatever the occupancy | global |
// legacy), GMACOP_LDS_VARIANT (node: k_walk_lds only), GMACOP_LDS_MAX_TIER
// (1..3), GMACOP_WALK_LANES, GMACOP_GLB_LANES (1, 2, 4, 8) and
// GMACOP_BLOOM_LOG2 (8..16) override the choices for tuning; results do not
// depend on them.
WalkPlan plan_walk(const gmacop_graph *g, const gmacop_params *p, int max_lds)
{
    WalkPlan pl;
    pl.maxd = g->max_deg <= 4 ? 4 : g->max_deg <= 8 ? 8 : g->max_deg <= 16 ? 16 : 32;
    const char *kind = getenv("GMACOP_WALK_KERNEL");
    // time-dependent signals make a road's weight depend on the ant's clock: only the global walker
    // computes weights per ant
    const bool force_global = (kind && strcmp(kind, "global") == 0) || (p->flags & GMACOP_SIGNAL_TIMED);
    pl.legacy = (kind && strcmp(kind, "legacy") == 0) || g->n >= (1u << 24);
    pl.timed = (p->flags & GMACOP_SIGNAL_TIMED) != 0;
    pl.city_class.assign(g->n_inst, 0);
    if (pl.legacy) return pl;
    pl.lds_lanes = lanes_or(env_u32("GMACOP_WALK_LANES", 4), 4);
    bool road_ok = true;
    {
        const char *var = getenv("GMACOP_LDS_VARIANT");
        const uint32_t md = std::max(g->max_deg, g->max_indeg);
        road_ok = !(var && strcmp(var, "node") == 0) && md <= kMaxDegree;
        pl.road_maxd = md <= 4 ? 4 : md <= 8 ? 8 : md <= 16 ? 16 : 32;
    }
    pl.lds_apb = std::max<uint32_t>(1, std::min<uint32_t>(p->ants, 512 / pl.lds_lanes));
    pl.lds_bpv = (p->ants + pl.lds_apb - 1) / pl.lds_apb;
    const size_t t3 = (size_t)max_lds - kStaticLds, t2 = t3 / 2, t1 = t3 / 4;   // static block aggregates aside
    // the LDS walkers keep each node's goal term in 32 bits: a city whose
    // largest possible term (its bounding-box diagonal at this vmax) does not
    // fit goes to the global walker, which keeps 64
    const uint64_t kgoal = p->vmax_kmh ? (360ull << 16) / p->vmax_kmh : 0;
    const bool exact_goal = (p->flags & GMACOP_GOAL_EXACT) != 0;
    auto goal_fits = [&](uint32_t i) {
        if (exact_goal) return true;   // exact terms are 32-bit by definition
        const uint64_t x = g->inst_span2[i];
        uint64_t r = (uint64_t)std::sqrt((double)x);
        while (r * r < x) ++r;   // ceil(sqrt(x)) <= 2^31.5: no overflow
        return ((r * kgoal) >> 16) <= 0xFFFFFFFFull;
    };
    // A tier holds 4, 2 or 1 blocks per CU.  A city gets an LDS tier only if
    // that keeps at least one wave per SIMD (blocks x waves per block >= 4);
    // otherwise most of the CU would idle, and the persistent global walker,
    // which fills every CU whatever the city, serves it instead.
    const uint32_t wpb = (pl.lds_apb * pl.lds_lanes + kWave - 1) / kWave;
    const bool force_lds = kind && strcmp(kind, "lds") == 0;
    const uint32_t max_tier = std::min(3u, std::max(1u, env_u32("GMACOP_LDS_MAX_TIER", 3)));
    uint32_t glb_nodes = 0;
    for (uint32_t i = 0; i < g->n_inst; ++i) {
        const uint32_t nc = g->inst_off[i + 1] - g->inst_off[i];
        const uint32_t ec = g->inst_eoff[i + 1] - g->inst_eoff[i];
        // k_walk_ldsr: 16-byte record, cost and in-road entry per road; goal terms, then road bits per
        // ant (an even count of words); per-group scratch
        const size_t aux_r = std::max<size_t>(nc, (size_t)(((ec + 31) / 32) | 1u) * pl.lds_apb);
        const size_t need_r = (size_t)ec * 24 + ((aux_r + 1) & ~(size_t)1) * 4 + lds_group_bytes(pl.lds_apb);
        // k_walk_lds: 8-byte record, weight and cost per road; goal terms, then node bits per ant; scratch
        const size_t aux_n = std::max<size_t>(nc, (size_t)(((nc + 31) / 32) | 1u) * pl.lds_apb);
        const size_t need_n = (size_t)ec * 16 + (size_t)((ec + 1) & ~1u) * 4 + ((aux_n + 1) & ~(size_t)1) * 4 +
                              lds_group_bytes(pl.lds_apb);
        auto tier = [&](size_t need) -> uint8_t {
            const uint8_t t = need <= t1 ? 1 : need <= t2 ? 2 : need <= t3 ? 3 : 0;
            return t && t <= max_tier && ((4u >> (t - 1)) * wpb >= 4 || force_lds) ? t : 0;
        };
        uint8_t c = 0;
        size_t need = 0;
        if (!force_global && ec > 0 && goal_fits(i)) {
            if (road_ok && ec < 65536 && (c = tier(need_r)) != 0) {
                need = need_r;
            } else if ((c = tier(need_n)) != 0) {
                c += 3;
                need = need_n;
            }
        }
        pl.city_class[i] = c;
        if (c)
            pl.lds_bytes[c] = std::max(pl.lds_bytes[c], need);
        else
            glb_nodes = std::max(glb_nodes, nc);
    }
    pl.glb = glb_nodes > 0;
    pl.glb_lanes = lanes_or(env_u32("GMACOP_GLB_LANES", 4), 4);
    pl.glb_apb = 256 / pl.glb_lanes;
    pl.bloom_log2 = std::min<uint32_t>(16, std::max<uint32_t>(8, env_u32("GMACOP_BLOOM_LOG2", 11)));
    auto bloom_bytes = [&] { return (size_t)pl.glb_apb * ((1u << (pl.bloom_log2 - 5)) | 1u) * 4; };
    while (pl.bloom_log2 > 8 && bloom_bytes() > (size_t)max_lds) --pl.bloom_log2;   // within a block's LDS
    pl.glb_lds_bytes = bloom_bytes();
    pl.glb_nwords = (glb_nodes + 31) / 32;
    return pl;
}

}  // namespace

extern "C" int gmacop_graph_create(const gmacop_graph_desc *d, gmacop_graph **out)
{
    if (!out) return fail(GMACOP_E_INVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(d);
    if (rc) return rc;
    gmacop_graph *g = new gmacop_graph();
    HIP_TRY(hipGetDevice(&g->device));
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, g->device) == hipSuccess && v > 0)
            g->max_lds = v;
        else if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device) == hipSuccess &&
                 v > 0)
            g->max_lds = v;
        (void)hipGetLastError();
    }
    g->n = d->n_nodes;
    g->m = d->n_edges;
    g->n_inst = d->n_instances;
    if (d->inst_node_off)
        g->inst_off.assign(d->inst_node_off, d->inst_node_off + d->n_instances + 1);
    else
        g->inst_off = {0, g->n};
    for (uint32_t u = 0; u < g->n; ++u) g->max_deg = std::max(g->max_deg, d->row_ptr[u + 1] - d->row_ptr[u]);
    // incoming roads of every node (the approaches of its signal)
    std::vector<uint32_t> rev_ptr(g->n + 1, 0), rev_edge(g->m);
    for (uint32_t e = 0; e < g->m; ++e) rev_ptr[d->col[e] + 1]++;
    for (uint32_t v = 0; v < g->n; ++v) {
        g->max_indeg = std::max(g->max_indeg, rev_ptr[v + 1]);
        rev_ptr[v + 1] += rev_ptr[v];
    }
    {
        std::vector<uint32_t> fill(rev_ptr.begin(), rev_ptr.end() - 1);
        for (uint32_t e = 0; e < g->m; ++e) rev_edge[fill[d->col[e]]++] = e;
    }
    const uint32_t n = g->n, m = g->m;
    // per-road layout records for the LDS walker: tail, head, head's out-road range
    std::vector<uint32_t> tail(m);
    std::vector<uint2> rec(m);
    for (uint32_t u = 0; u < n; ++u)
        for (uint32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; ++e) {
            const uint32_t x = d->col[e];
            tail[e] = u;
            const uint32_t deg = d->row_ptr[x + 1] - d->row_ptr[x];
            rec[e] = make_uint2((x & 0xFFFFFFu) | (std::min(deg, 255u) << 24), d->row_ptr[x]);
        }
    std::vector<uint4> rec32(2 * (size_t)m);   // the cost and pheromone words are written per call
    for (uint32_t e = 0; e < m; ++e) {
        const uint32_t x = d->col[e];
        rec32[2 * (size_t)e] = make_uint4(rec[e].x, rec[e].y, (uint32_t)d->x_dm[x], (uint32_t)d->y_dm[x]);
        rec32[2 * (size_t)e + 1] = make_uint4(0, 0, 0, 0);
    }
    std::vector<uint32_t> node_lo(n), node_inst(n);
    g->inst_eoff.resize(g->n_inst + 1);
    for (uint32_t i = 0; i < g->n_inst; ++i) {
        g->inst_eoff[i] = d->row_ptr[g->inst_off[i]];
        g->max_city_nodes = std::max(g->max_city_nodes, g->inst_off[i + 1] - g->inst_off[i]);
        int64_t x0 = INT64_MAX, x1 = INT64_MIN, y0 = INT64_MAX, y1 = INT64_MIN;
        for (uint32_t u = g->inst_off[i]; u < g->inst_off[i + 1]; ++u) {
            x0 = std::min<int64_t>(x0, d->x_dm[u]); x1 = std::max<int64_t>(x1, d->x_dm[u]);
            y0 = std::min<int64_t>(y0, d->y_dm[u]); y1 = std::max<int64_t>(y1, d->y_dm[u]);
        }
        g->inst_span2.push_back((uint64_t)((x1 - x0) * (x1 - x0)) + (uint64_t)((y1 - y0) * (y1 - y0)));
        for (uint32_t u = g->inst_off[i]; u < g->inst_off[i + 1]; ++u) {
            node_lo[u] = g->inst_off[i];
            node_inst[u] = i;
        }
    }
    g->inst_eoff[g->n_inst] = m;
    // static city-local road records of k_walk_ldsr (meaningful in cities under 2^16 roads, the only ones it serves)
    std::vector<uint4> rvs(m);
    for (uint32_t u = 0; u < n; ++u) {
        const uint32_t c = node_inst[u], e_lo = g->inst_eoff[c], n_lo = g->inst_off[c];
        for (uint32_t e = d->row_ptr[u]; e < d->row_ptr[u + 1]; ++e) {
            const uint32_t x = d->col[e];
            const uint32_t deg = d->row_ptr[x + 1] - d->row_ptr[x], ind = rev_ptr[x + 1] - rev_ptr[x];
            rvs[e] = make_uint4(((d->row_ptr[x] - e_lo) & 0xFFFFu) | (std::min(deg, 0xFFFFu) << 16),
                                ((rev_ptr[x] - e_lo) & 0xFFFFu) | (std::min(ind, 0xFFFFu) << 16),
                                ((x - n_lo) & 0xFFFFu) | (((u - n_lo) & 0xFFFFu) << 16), (rev_edge[e] - e_lo) & 0xFFFFu);
        }
    }
    if ((rc = upload(&g->tail, tail.data(), m)) || (rc = upload(&g->rec, rec.data(), m)) ||
        (rc = upload(&g->rec32, rec32.data(), 2 * (size_t)m)) || (rc = upload(&g->rvs, rvs.data(), m)) || (rc = upload(&g->node_lo, node_lo.data(), n)) ||
        (rc = upload(&g->node_inst, node_inst.data(), n)) || (rc = dalloc(&g->inst_fits, g->n_inst)) ||
        (rc = upload(&g->inst_off_dev, g->inst_off.data(), g->n_inst + 1)) ||
        (rc = upload(&g->inst_eoff_dev, g->inst_eoff.data(), g->n_inst + 1))) {
        std::string keep = t_err;
        delete g;
        t_err = keep;
        return rc;
    }
    if ((rc = upload(&g->row_ptr, d->row_ptr, n + 1)) || (rc = upload(&g->col, d->col, m)) ||
        (rc = upload(&g->len_dm, d->len_dm, m)) || (rc = upload(&g->speed, d->speed_kmh, m)) ||
        (rc = upload(&g->green, d->green_pm, m)) || (rc = upload(&g->cycle, d->cycle_ms, n)) ||
        (rc = upload(&g->x, d->x_dm, n)) || (rc = upload(&g->y, d->y_dm, n)) ||
        (rc = upload(&g->base_load, d->base_load, m)) || (rc = upload(&g->rev_ptr, rev_ptr.data(), n + 1)) ||
        (rc = upload(&g->rev_edge, rev_edge.data(), m)) || (rc = dalloc(&g->t0, m)) || (rc = dalloc(&g->wf, m)) ||
        (rc = dalloc(&g->tau, m)) || (rc = dalloc(&g->load, m)) || (rc = dalloc(&g->cost, m)) ||
        (rc = dalloc(&g->cnt, m)) || (rc = dalloc(&g->dep, m)) || (rc = dalloc(&g->counters, kCounters)) || (rc = dalloc(&g->iter_max, 1))) {
        std::string keep = t_err;
        delete g;
        t_err = keep;
        return rc;
    }
    if (hipMemset(g->counters, 0, kCounters * sizeof(uint64_t)) != hipSuccess ||
        hipMemset(g->iter_max, 0, sizeof(uint32_t)) != hipSuccess) {
        delete g;
        return fail(GMACOP_E_DEVICE, "hipMemset of counters failed");
    }
    {   // green windows of the time-dependent signals: an intersection's approaches take their greens in turn,
        // in road order, each for floor(C * green / 1000) ms, the first from time 0
        std::vector<uint4> sig(m);
        std::vector<uint64_t> acc(n, 0);
        for (uint32_t e = 0; e < m; ++e) {
            const uint32_t v = d->col[e];
            const uint64_t C = d->cycle_ms[v];
            if (!C) {
                sig[e] = make_uint4(0, 0, 0, 0);
                continue;
            }
            const uint64_t len = C * d->green_pm[e] / 1000u;
            sig[e] = make_uint4((uint32_t)C, (uint32_t)(acc[v] % C), (uint32_t)len, 0);
            acc[v] += len;
        }
        if ((rc = upload(&g->sig, sig.data(), m))) {
            std::string keep = t_err;
            delete g;
            t_err = keep;
            return rc;
        }
    }
    {   // the mean free-flow road time, the band width scale of the exact goal search
        long double sum = 0;
        for (uint32_t e = 0; e < m; ++e) {
            uint64_t x = (uint64_t)d->len_dm[e] * 360u / d->speed_kmh[e];
            sum += (long double)(x < 1 ? 1 : (x > kRoadCostCap ? kRoadCostCap : x));
        }
        g->mean_t0 = (uint32_t)std::max<long double>(1.0L, sum / m);
    }
    // static: free-flow times and the in-roads as (tail, free-flow time), for the exact goal term
    if ((rc = dalloc(&g->rev_tw, m))) {
        std::string keep = t_err;
        delete g;
        t_err = keep;
        return rc;
    }
    hipLaunchKernelGGL(k_free_flow, dim3(blocks_for(m, 256)), dim3(256), 0, 0, m, (const uint32_t *)g->len_dm,
                       (const uint16_t *)g->speed, g->t0);
    hipLaunchKernelGGL(k_rev_weights, dim3(blocks_for(m, 256)), dim3(256), 0, 0, m, (const uint32_t *)g->rev_edge,
                       (const uint32_t *)g->tail, (const uint32_t *)g->t0, g->rev_tw);
    if (hipDeviceSynchronize() != hipSuccess) {
        delete g;
        return fail(GMACOP_E_DEVICE, "graph set-up kernels failed");
    }
    *out = g;
    return GMACOP_OK;
}

namespace {

// Per-call workspace of a routing call: ant paths and results, the walkers'
// work lists and visited words, and independent-mode pheromone rows.  The
// allocating entry point takes it from buffers the graph grows on demand;
// gmacop_route_batch_noalloc carves it out of the static scratch array.
struct CallWork {
    uint32_t *path = nullptr, *ant_len = nullptr, *ant_cost = nullptr, *gbits = nullptr;
    uint64_t *iter_key = nullptr, *steps = nullptr;
    uint32_t *best_path = nullptr, *best_len = nullptr, *best_cost = nullptr;
    gmacop_od *od = nullptr;
    uint8_t *vclass = nullptr;
    GlbVeh *gveh = nullptr, *gvrec = nullptr;
    uint32_t *gvlen = nullptr, *gctl = nullptr, *gepoch = nullptr;
    uint64_t *gwords = nullptr;
    uint64_t *lazy = nullptr, *dep_ind = nullptr;
    uint32_t *touched = nullptr, *touched_n = nullptr, *dev_gen = nullptr;
    uint32_t *goal = nullptr, *goal_work = nullptr, *goal_ctl = nullptr;   // exact goal term (GoalPlan)
    uint32_t *gnode = nullptr, *gchoice = nullptr, *gvcity = nullptr;   // GMACOP_MODE_GREEDY
    uint64_t *gcsum = nullptr, *gmark = nullptr, *gmsum = nullptr;
    bool side = false;          // the global walker may run on g->side beside the LDS walkers
    bool allow_graph = false;   // GMACOP_HIP_GRAPH may capture and replay the call
};

// Shape of the exact-goal search: one row of `stride` terms per vehicle (the
// largest city), and a persistent grid whose per-block workspace (stamps and
// two frontier queues) stays within a budget.
struct GoalPlan {
    bool on = false;
    uint32_t stride = 0, qcap = 0, fcap = 0, delta = 1, blocks = 0, threads = 0;
    // u32 words of the per-block workspace: relaxed-at terms, phase marks, two near and two far queues
    size_t work_words() const { return (size_t)blocks * (2 * (size_t)stride + 2 * (size_t)qcap + 2 * (size_t)fcap); }
};

constexpr uint64_t kGoalWorkBudget = 8ull << 30;   // bytes of the search's per-block workspace

// tasks: destinations searched by one launch; threads 0 = choose so that the
// resident blocks together hold about as many threads as the device can
// keep (one wave per destination when there are many, up to 1024 when few).
// The band of the near-far order is a few mean free-flow road times.
int goal_plan(const gmacop_graph *g, const gmacop_params *p, uint64_t tasks, uint64_t budget, uint32_t threads,
              GoalPlan *gp)
{
    *gp = GoalPlan{};
    if (!(p->flags & GMACOP_GOAL_EXACT)) return GMACOP_OK;
    gp->on = true;
    gp->stride = std::max<uint32_t>(g->max_city_nodes, 1);
    gp->qcap = std::min<uint32_t>(gp->stride, 16384);
    gp->fcap = std::min<uint32_t>(gp->stride, 32768);
    if (const char *qc = getenv("GMACOP_GOAL_QCAP")) {   // smaller queues (exercises the scan rounds)
        const uint32_t c = std::max<uint32_t>(1, (uint32_t)strtoul(qc, nullptr, 10));
        gp->qcap = std::min(gp->qcap, c);
        gp->fcap = std::min(gp->fcap, c);
    }
    const uint32_t mult = std::max<uint32_t>(1, env_u32("GMACOP_GOAL_DELTA", 4));
    gp->delta = (uint32_t)std::min<uint64_t>(0x7FFFFFFFull, std::max<uint64_t>(1, (uint64_t)g->mean_t0 * mult));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
    cus = std::max(cus, 1);
    if (!threads) {
        const uint64_t per_task = 2048ull * (uint64_t)cus / std::max<uint64_t>(tasks, 1);
        threads = 64;
        while (threads < 1024 && threads * 2 <= per_task) threads *= 2;
    }
    gp->threads = threads;
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_goal_sssp, (int)threads, 0));
    uint64_t blocks = (uint64_t)std::max(nb, 1) * (uint64_t)cus;
    blocks = std::min<uint64_t>(blocks, std::max<uint64_t>(tasks, 1));
    const uint64_t per_block = 4ull * (2ull * gp->stride + 2ull * gp->qcap + 2ull * gp->fcap);
    blocks = std::min<uint64_t>(blocks, std::max<uint64_t>(1, budget / per_block));
    gp->blocks = (uint32_t)blocks;
    return GMACOP_OK;
}

// The greedy mode (the literal MACO-P loop) routes each vehicle once, without
// ants or iterations, and always on the exact goal term.
gmacop_params effective_params(const gmacop_params &p)
{
    gmacop_params e = p;
    if (p.mode == GMACOP_MODE_GREEDY) {
        e.ants = 1;
        e.iterations = 0;
        e.flags |= GMACOP_GOAL_EXACT;
    }
    return e;
}

// Checks shared by both routing entry points; on success *plan holds the walk schedule.
int route_check(gmacop_graph *g, const gmacop_od *q, uint32_t nq, const gmacop_params *p, const gmacop_result *out,
                WalkPlan *plan)
{
    if (!g) return fail(GMACOP_E_INVAL, "graph is NULL");
    if (!out || !out->path_edges || !out->path_len || !out->cost_ms || !out->steps_total)
        return fail(GMACOP_E_INVAL, "result buffers missing");
    if (nq > 0 && !q) return fail(GMACOP_E_INVAL, "queries are NULL");
    int rc = validate_params(g, p, nq);
    if (rc) return rc;
    if (p->mode == GMACOP_MODE_INDEPENDENT && p->iterations > kLazyIterMax)
        return fail(GMACOP_E_UNSUPPORTED, "independent mode supports at most %u iterations", kLazyIterMax);
    if ((p->flags & GMACOP_RESUME) && p->mode != GMACOP_MODE_SHARED)
        return fail(GMACOP_E_UNSUPPORTED, "GMACOP_RESUME is for shared mode");
    if ((p->flags & GMACOP_RESUME) && !(p->flags & GMACOP_DEVICE_PTRS)) {
        for (uint32_t i = 0; i < nq; ++i) {   // the held best routes are read back to the device
            if (out->path_len[i] > p->max_steps)
                return fail(GMACOP_E_INVAL, "resume: path_len[%u] exceeds max_steps", i);
            for (uint32_t s = 0; s < out->path_len[i]; ++s)
                if (out->path_edges[(size_t)i * p->max_steps + s] >= g->m)
                    return fail(GMACOP_E_INVAL, "resume: road %u of vehicle %u out of range", s, i);
        }
    }
    if (!(p->flags & GMACOP_DEVICE_PTRS)) {
        for (uint32_t i = 0; i < nq; ++i) {
            if (q[i].qid == 0xFFFFFFFFu) return fail(GMACOP_E_INVAL, "query %u uses the reserved qid", i);
            if (q[i].src >= g->n || q[i].dst >= g->n) return fail(GMACOP_E_INVAL, "query %u: node out of range", i);
            if (q[i].src == q[i].dst) return fail(GMACOP_E_INVAL, "query %u: src == dst", i);
            if (instance_of(g, q[i].src) != instance_of(g, q[i].dst))
                return fail(GMACOP_E_INVAL, "query %u: src and dst in different cities", i);
        }
    }
    HIP_TRY(hipSetDevice(g->device));
    *plan = plan_walk(g, p, g->max_lds);
    if (plan->legacy && (p->flags & (GMACOP_GOAL_EXACT | GMACOP_SIGNAL_TIMED)))
        return fail(GMACOP_E_UNSUPPORTED, "the exact goal term and timed signals need a graph under 2^24 nodes");
    if (p->mode == GMACOP_MODE_GREEDY && (p->flags & GMACOP_SIGNAL_TIMED))
        return fail(GMACOP_E_UNSUPPORTED, "GMACOP_MODE_GREEDY does not take GMACOP_SIGNAL_TIMED");
    if (!plan->legacy && plan->glb && (rc = glb_grid(g->device, *plan, (uint64_t)nq * p->ants))) return rc;
    return GMACOP_OK;
}

// Workspace of the allocating entry point: the graph's own buffers, grown to fit.
int route_work_grow(gmacop_graph *g, uint32_t nq, const gmacop_params *p, const WalkPlan &plan, const GoalPlan &gp,
                    hipStream_t st, CallWork *w)
{
    int rc;
    const bool indep = p->mode == GMACOP_MODE_INDEPENDENT;
    const uint32_t S = p->max_steps;
    const uint64_t NA = (uint64_t)nq * p->ants;
    const bool lds = g->n <= kLdsBitsetMaxNodes;
    const uint32_t nwords = (g->n + 31) / 32;
    if ((rc = grow(&g->path, &g->cap_path, (size_t)S * NA, false))) return rc;
    {
        size_t c1 = g->cap_ants;
        if ((rc = grow(&g->ant_len, &c1, NA, false))) return rc;
        size_t c2 = g->cap_ants;
        if ((rc = grow(&g->ant_cost, &c2, NA, false))) return rc;
        g->cap_ants = std::min(c1, c2);
    }
    if (plan.legacy && !lds && (rc = grow(&g->gbits, &g->cap_bits, (size_t)NA * nwords, true))) return rc;
    if (!plan.legacy && plan.glb &&
        (rc = glb_prepare(g->glb, nq, (uint64_t)plan.glb_blocks * plan.glb_apb, plan.glb_nwords)))
        return rc;
    if (!plan.legacy && plan.glb && plan.any_lds() && !g->side) {   // stream and events of the side launch
        HIP_TRY(hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&g->join, hipEventDisableTiming));
    }
    if ((rc = grow(&g->vclass, &g->cap_vclass, std::max<size_t>(nq, 1), false))) return rc;
    {
        size_t c1 = g->cap_veh, c2 = g->cap_veh, c3 = g->cap_veh, c4 = g->cap_veh;
        if ((rc = grow(&g->iter_key, &c1, nq, false)) || (rc = grow(&g->best_len, &c2, nq, false)) ||
            (rc = grow(&g->best_cost, &c3, nq, false)) || (rc = grow(&g->od, &c4, nq, false)))
            return rc;
        g->cap_veh = std::min(std::min(c1, c2), std::min(c3, c4));
    }
    if ((rc = grow(&g->best_path, &g->cap_best, (size_t)nq * S, false))) return rc;
    if (!g->steps && (rc = dalloc(&g->steps, 1))) return rc;
    const uint32_t tcap = (uint32_t)std::min<uint64_t>(g->m, (uint64_t)p->ants * S);
    if (indep && nq) {
        // zero-filled on allocation: deposits and list counts return to zero after every apply
        const bool fresh_lazy = g->cap_lazy < (size_t)nq * g->m;
        if ((rc = grow(&g->lazy, &g->cap_lazy, (size_t)nq * g->m, true)) ||
            (rc = grow(&g->dep_ind, &g->cap_depi, (size_t)nq * g->m, true)) ||
            (rc = grow(&g->touched, &g->cap_touch, (size_t)nq * tcap, false)) ||
            (rc = grow(&g->touched_n, &g->cap_touchn, nq, true)))
            return rc;
        if (!g->dev_gen) {
            if ((rc = dalloc(&g->dev_gen, 1))) return rc;
            HIP_TRY(hipMemset(g->dev_gen, 0, sizeof(uint32_t)));
            HIP_TRY(hipDeviceSynchronize());
            g->gen_count = 0;
        }
        if (fresh_lazy || g->gen_count >= kGenMask) {
            // generation numbers would repeat: start over from an all-zero lazy array
            HIP_TRY(hipMemsetAsync(g->lazy, 0, sizeof(uint64_t) * g->cap_lazy, st));
            HIP_TRY(hipMemsetAsync(g->dev_gen, 0, sizeof(uint32_t), st));
            g->gen_count = 0;
        }
        g->gen_count++;
    }
    w->path = g->path; w->ant_len = g->ant_len; w->ant_cost = g->ant_cost; w->gbits = g->gbits;
    w->iter_key = g->iter_key; w->steps = g->steps;
    w->best_path = g->best_path; w->best_len = g->best_len; w->best_cost = g->best_cost; w->od = g->od;
    w->vclass = g->vclass;
    w->gveh = g->glb.veh; w->gvrec = g->glb.vrec; w->gvlen = g->glb.vlen; w->gctl = g->glb.ctl;
    w->gepoch = g->glb.epoch; w->gwords = g->glb.words;
    w->lazy = g->lazy; w->dep_ind = g->dep_ind; w->touched = g->touched; w->touched_n = g->touched_n;
    w->dev_gen = g->dev_gen;
    if (gp.on) {
        if ((rc = grow(&g->goal, &g->cap_goal, std::max<size_t>((size_t)nq * gp.stride, 1), false)) ||
            (rc = grow(&g->goal_work, &g->cap_goal_work, std::max<size_t>(gp.work_words(), 1), false)))
            return rc;
        if (!g->goal_ctl) {
            if ((rc = dalloc(&g->goal_ctl, 2))) return rc;
            HIP_TRY(hipMemset(g->goal_ctl, 0, 2 * sizeof(uint32_t)));
            HIP_TRY(hipDeviceSynchronize());
        }
        w->goal = g->goal; w->goal_work = g->goal_work; w->goal_ctl = g->goal_ctl;
    }
    if (p->mode == GMACOP_MODE_GREEDY) {
        size_t c1 = g->cap_gveh, c2 = g->cap_gveh, c3 = g->cap_gveh, c4 = g->cap_gveh, r1 = g->cap_groad,
               r2 = g->cap_groad;
        if ((rc = grow(&g->gnode, &c1, std::max<size_t>(nq, 1), false)) ||
            (rc = grow(&g->gchoice, &c2, std::max<size_t>(nq, 1), false)) ||
            (rc = grow(&g->gvcity, &c3, std::max<size_t>(nq, 1), false)) ||
            (rc = grow(&g->gcsum, &c4, std::max<size_t>(nq, 1), false)) || (rc = grow(&g->gmark, &r1, g->m, false)) ||
            (rc = grow(&g->gmsum, &r2, g->m, false)))
            return rc;
        g->cap_gveh = std::min(std::min(c1, c2), std::min(c3, c4));
        g->cap_groad = std::min(r1, r2);
        w->gnode = g->gnode; w->gchoice = g->gchoice; w->gvcity = g->gvcity; w->gcsum = g->gcsum;
        w->gmark = g->gmark; w->gmsum = g->gmsum;
    }
    w->side = true;
    w->allow_graph = true;
    return GMACOP_OK;
}

// The call itself, on workspace w: initial state and cost table, then per
// iteration walk, best route, pheromone/load update, cost table; results to
// the caller's buffers.
int route_run(gmacop_graph *g, const gmacop_od *q, uint32_t nq, const gmacop_params *p, gmacop_result *out,
              hipStream_t st, const WalkPlan &plan, const GoalPlan &gp, const CallWork &w)
{
    int rc;
    const bool indep = p->mode == GMACOP_MODE_INDEPENDENT;
    const bool dev_ptrs = (p->flags & GMACOP_DEVICE_PTRS) != 0;
    const uint32_t S = p->max_steps;
    const uint64_t NA = (uint64_t)nq * p->ants;
    const bool lds = g->n <= kLdsBitsetMaxNodes;
    const uint32_t nwords = (g->n + 31) / 32;
    const uint32_t tcap = (uint32_t)std::min<uint64_t>(g->m, (uint64_t)p->ants * S);
    if (plan.city_class != g->city_class_dev) {   // per-city walker choice, uploaded when it changes
        HIP_TRY(hipMemcpy(g->inst_fits, plan.city_class.data(), g->n_inst, hipMemcpyHostToDevice));
        g->city_class_dev = plan.city_class;
    }

    const uint32_t resume = (p->flags & GMACOP_RESUME) ? 1u : 0u;
    const gmacop_od *od = q;
    uint32_t *best_path = w.best_path, *best_len = w.best_len, *best_cost = w.best_cost;
    uint64_t *steps = w.steps;
    if (dev_ptrs) {
        best_path = out->path_edges;
        best_len = out->path_len;
        best_cost = out->cost_ms;
        steps = out->steps_total;
    } else if (nq) {
        HIP_TRY(hipMemcpyAsync(w.od, q, sizeof(gmacop_od) * nq, hipMemcpyHostToDevice, st));
        if (resume) {   // the best routes held from the previous call
            HIP_TRY(hipMemcpyAsync(best_len, out->path_len, sizeof(uint32_t) * nq, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(best_cost, out->cost_ms, sizeof(uint32_t) * nq, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(best_path, out->path_edges, sizeof(uint32_t) * (size_t)nq * S,
                                   hipMemcpyHostToDevice, st));
        }
        HIP_TRY(hipStreamSynchronize(st));   // the caller's buffers are read before any later error returns
        od = w.od;
    }

    const bool load_update = !(p->flags & GMACOP_NO_LOAD_UPDATE);
    uint32_t *mir = (!plan.legacy && plan.glb) ? (uint32_t *)g->rec32 : nullptr;   // the global walker's records
    EdgeInitArgs ia{g->m, p->tau0_q16, p->t_max_ms, resume, g->col, g->len_dm, g->cycle, g->base_load, g->speed, g->green,
                    g->t0, g->wf, g->tau, g->load, g->cnt, g->dep, mir};
    const uint32_t timed = (p->flags & GMACOP_SIGNAL_TIMED) ? 1u : 0u;
    CostArgs ca{g->n, p->theta, p->th_max, g->rev_ptr, g->rev_edge, g->cycle, g->load, g->t0, g->wf, g->cost, mir,
                timed};
    PherView pv{};
    pv.dense = indep ? nullptr : g->tau;
    pv.lazy = w.lazy;
    pv.gen = w.dev_gen;
    pv.m = g->m; pv.tau0 = p->tau0_q16; pv.rho = p->rho_q16; pv.tau_min = p->tau_min_q16;
    DepView dv{};
    dv.dep = indep ? w.dep_ind : g->dep;
    dv.touched = w.touched; dv.touched_n = w.touched_n; dv.m = g->m; dv.cap = tcap; dv.indep = indep ? 1u : 0u;
    WalkArgs wa{};
    wa.row_ptr = g->row_ptr; wa.col = g->col; wa.cost = g->cost; wa.pher = pv; wa.depv = dv; wa.x = g->x; wa.y = g->y;
    wa.od = od; wa.n = g->n; wa.nq = nq; wa.ants = p->ants; wa.max_steps = S; wa.alpha = p->alpha; wa.beta = p->beta;
    wa.kgoal = p->vmax_kmh ? (uint32_t)((360ull << 16) / p->vmax_kmh) : 0;
    wa.nwords = nwords; wa.seed_lo = (uint32_t)p->seed; wa.seed_hi = (uint32_t)(p->seed >> 32);
    wa.q_deposit = p->q_deposit; wa.path = w.path; wa.ant_len = w.ant_len; wa.ant_cost = w.ant_cost;
    wa.gbits = w.gbits; wa.iter_key = w.iter_key; wa.steps = steps; wa.counters = g->counters;
    wa.iter_max = g->iter_max;
    LdsWalkArgs la{};
    la.row_ptr = g->row_ptr; la.col = g->col; la.cost = g->cost; la.pher = pv; la.depv = dv; la.x = g->x; la.y = g->y;
    la.rec = g->rec; la.tail = g->tail; la.rev_ptr = g->rev_ptr; la.rvs = g->rvs;
    la.node_inst = g->node_inst; la.inst_off = g->inst_off_dev; la.inst_eoff = g->inst_eoff_dev; la.vclass = w.vclass;
    la.od = od; la.n = g->n; la.m = g->m; la.nq = nq; la.ants = p->ants; la.apb = plan.lds_apb; la.bpv = plan.lds_bpv;
    la.max_steps = S; la.alpha = p->alpha; la.beta = p->beta; la.kgoal = wa.kgoal; la.nwords = nwords;
    la.seed_lo = wa.seed_lo; la.seed_hi = wa.seed_hi; la.q_deposit = p->q_deposit; la.path = w.path;
    la.ant_len = w.ant_len; la.ant_cost = w.ant_cost; la.iter_key = w.iter_key;
    la.steps = steps; la.counters = g->counters; la.iter_max = g->iter_max;
    la.goal = gp.on ? w.goal : nullptr; la.goal_stride = gp.stride;
    const bool update_loads = load_update && !indep;
    BestArgs ba{nq, p->ants, S, update_loads ? 1u : 0u, g->m, g->iter_max, g->counters, w.path, w.ant_len, w.iter_key,
                best_path, best_len, best_cost, g->cnt};
    EdgeArgs ea{g->m, p->rho_q16, p->tau_min_q16, p->tau_max_q16, p->theta, update_loads ? 1u : 0u,
                g->tau, g->load, g->cnt, g->base_load, g->dep, mir};
    ApplyArgs aa{g->m, tcap, 0, p->tau0_q16, p->rho_q16, p->tau_min_q16, p->tau_max_q16, p->theta, g->load, w.dev_gen,
                 nullptr, nullptr, w.lazy, w.dep_ind, w.touched, w.touched_n};
    GlbWalkArgs ga{};
    ga.rec32 = g->rec32; ga.pher = pv; ga.depv = dv;
    ga.veh = w.gveh; ga.glb_n = w.gctl; ga.tickets = w.gctl ? w.gctl + 1 : nullptr; ga.gwords = w.gwords;
    ga.vlen = w.gvlen;
    ga.slot_epoch = w.gepoch; ga.m = g->m; ga.nq = nq;
    ga.ants = p->ants; ga.apb = plan.glb_apb; ga.max_steps = S; ga.alpha = p->alpha; ga.beta = p->beta;
    ga.kgoal = wa.kgoal; ga.nw2 = plan.glb_nwords; ga.bloom_log2 = plan.bloom_log2; ga.seed_lo = wa.seed_lo;
    ga.seed_hi = wa.seed_hi; ga.q_deposit = p->q_deposit; ga.path = w.path; ga.ant_len = w.ant_len;
    ga.ant_cost = w.ant_cost; ga.iter_key = w.iter_key; ga.steps = steps;
    ga.counters = g->counters; ga.iter_max = g->iter_max;
    ga.goal = la.goal; ga.goal_stride = gp.stride;
    ga.sig = timed ? g->sig : nullptr; ga.t_max = p->t_max_ms;
    const GlbListArgs gla{od, w.vclass, g->row_ptr, g->node_lo, g->x, g->y, nq, p->ants, wa.kgoal,
                          w.gvrec, w.gveh, w.gctl, w.gvlen, w.ant_len, w.ant_cost, la.goal, gp.stride};
    GoalArgs goa{};
    goa.od = od; goa.list = nullptr; goa.ntask = nq; goa.n = g->n; goa.stride = gp.stride; goa.qcap = gp.qcap; goa.fcap = gp.fcap;
    goa.delta = gp.delta;
    goa.node_inst = g->node_inst; goa.inst_off = g->inst_off_dev; goa.rev_ptr = g->rev_ptr; goa.rev_tw = g->rev_tw;
    goa.goal = w.goal; goa.work = w.goal_work; goa.ctl = w.goal_ctl;
    const bool any_lds = !plan.legacy && plan.any_lds();
    if (any_lds && (rc = setup_walk_lds(la, plan, st))) return rc;

    const bool timing = (p->flags & GMACOP_TIME_KERNELS) != 0;
    const bool use_graph = w.allow_graph && (p->flags & GMACOP_HIP_GRAPH) && !timing && st != nullptr;
    // The whole call as one kernel sequence on `st`: initial state and cost
    // table, then per iteration walk, best route, pheromone/load, cost table.
    auto enqueue = [&]() -> int {
        int erc = GMACOP_OK;
        KernelTimer kt{g, st, timing};
        gmacop_graph::Timed tm{}, tl{};
        hipLaunchKernelGGL(k_init_edges, dim3(blocks_for(g->m, 256)), dim3(256), 0, st, ia);
        if (gp.on && nq) {   // Calc_Dist: the exact goal row of every vehicle, once per call
            gmacop_graph::Timed tq{};
            if ((erc = kt.start(6, &tq))) return erc;
            hipLaunchKernelGGL(k_goal_sssp, dim3(gp.blocks), dim3(gp.threads), 0, st, goa);
            if ((erc = kt.stop(&tq))) return erc;
        }
        if (indep && nq) hipLaunchKernelGGL(k_next_generation, dim3(1), dim3(64), 0, st, w.dev_gen);
        hipLaunchKernelGGL(k_init_vehicles, dim3(blocks_for(std::max(nq, 1u), 256)), dim3(256), 0, st, nq, resume,
                           best_len, best_cost, w.iter_key, steps);
        hipLaunchKernelGGL(k_cost, dim3(blocks_for(g->n, 256)), dim3(256), 0, st, ca);
        if (p->mode == GMACOP_MODE_GREEDY) {   // the literal MACO-P loop: one block per city, all ticks
            if (nq) {
                hipLaunchKernelGGL(k_greedy_prep, dim3(blocks_for(nq, 256)), dim3(256), 0, st, od, nq, g->n,
                                   (const uint32_t *)g->node_inst, w.gvcity, w.gnode, w.gchoice, w.gcsum);
                GreedyArgs gy{};
                gy.od = od; gy.nq = nq; gy.n = g->n; gy.max_steps = S; gy.theta = p->theta; gy.stride = gp.stride;
                gy.row_ptr = g->row_ptr; gy.col = g->col; gy.cost = g->cost; gy.node_inst = g->node_inst;
                gy.inst_off = g->inst_off_dev; gy.inst_eoff = g->inst_eoff_dev; gy.base_load = g->base_load;
                gy.goal = w.goal; gy.node = w.gnode; gy.choice = w.gchoice; gy.vcity = w.gvcity; gy.csum = w.gcsum;
                gy.mark = w.gmark; gy.msum = w.gmsum; gy.cnt = g->cnt; gy.mark_out = g->tau;
                gy.path = best_path; gy.len = best_len; gy.cost_out = best_cost; gy.steps = steps;
                hipLaunchKernelGGL(k_greedy, dim3(g->n_inst), dim3(1024), 0, st, gy);
            }
            HIP_TRY(hipGetLastError());
            return GMACOP_OK;
        }
        if (nq && !plan.legacy) {
            hipLaunchKernelGGL(k_classify, dim3(blocks_for(nq, 256)), dim3(256), 0, st, od, nq, g->n,
                               (const uint32_t *)g->node_inst, (const uint8_t *)g->inst_fits, w.vclass);
            if (plan.glb) hipLaunchKernelGGL(k_glb_prep, dim3(blocks_for(nq, 256)), dim3(256), 0, st, gla);
        }
        HIP_TRY(hipGetLastError());
        WalkArgs wt = wa;
        LdsWalkArgs lt = la;
        GlbWalkArgs gt = ga;
        ApplyArgs at = aa;
        for (uint32_t t = 0; t < p->iterations; ++t) {
            wt.iter = lt.iter = gt.iter = p->iter_offset + t;
            wt.t_local = lt.t_local = gt.t_local = at.t_local = t;
            const uint32_t md = g->max_deg;
            if (NA > 0) {
                if ((erc = kt.start(0, &tm))) return erc;
                if (plan.legacy) {
                    erc = md <= 4 ? launch_walk<4>(wt, lds, st)
                          : md <= 8 ? launch_walk<8>(wt, lds, st)
                          : md <= 16 ? launch_walk<16>(wt, lds, st)
                                     : launch_walk<32>(wt, lds, st);
                } else {
                    // both kinds of walker: the global one on the side stream, beside the LDS ones
                    const bool both = w.side && plan.glb && plan.any_lds();
                    hipStream_t gst = both ? g->side : st;
                    KernelTimer kg{g, gst, timing};
                    gmacop_graph::Timed tg{};
                    if (both) {
                        HIP_TRY(hipEventRecord(g->fork, st));
                        HIP_TRY(hipStreamWaitEvent(g->side, g->fork, 0));
                    }
                    if (plan.glb) {
                        hipLaunchKernelGGL(k_glb_list, dim3(1), dim3(1024), 0, gst, gla);
                        if ((erc = kg.start(5, &tg)) || (erc = launch_walk_glb_any(gt, plan, gst)) ||
                            (erc = kg.stop(&tg)))
                            return erc;
                    }
                    if (plan.any_lds()) {
                        if ((erc = kt.start(4, &tl)) || (erc = launch_walk_lds_classes(lt, plan, st)) ||
                            (erc = kt.stop(&tl)))
                            return erc;
                    }
                    if (both) {
                        HIP_TRY(hipEventRecord(g->join, g->side));
                        HIP_TRY(hipStreamWaitEvent(st, g->join, 0));
                    }
                }
                if (erc || (erc = kt.stop(&tm))) return erc;
                if ((erc = kt.start(1, &tm))) return erc;
                hipLaunchKernelGGL(k_best, dim3(nq), dim3(kWave), 0, st, ba);
                if ((erc = kt.stop(&tm))) return erc;
            }
            if ((erc = kt.start(2, &tm))) return erc;
            if (indep) {
                if (nq) hipLaunchKernelGGL(k_apply_touched, dim3(nq), dim3(256), 0, st, at);
            } else {
                hipLaunchKernelGGL(k_edge, dim3(blocks_for(g->m, 256)), dim3(256), 0, st, ea);
            }
            if ((erc = kt.stop(&tm))) return erc;
            if (update_loads) {
                if ((erc = kt.start(3, &tm))) return erc;
                hipLaunchKernelGGL(k_cost, dim3(blocks_for(g->n, 256)), dim3(256), 0, st, ca);
                if ((erc = kt.stop(&tm))) return erc;
            }
            HIP_TRY(hipGetLastError());
        }
        return GMACOP_OK;
    };

    if (use_graph) {
        // key: every value the captured launches depend on
        std::vector<uint64_t> key = {
            (uint64_t)(uintptr_t)od, (uint64_t)(uintptr_t)best_path, (uint64_t)(uintptr_t)best_len,
            (uint64_t)(uintptr_t)best_cost, (uint64_t)(uintptr_t)steps, (uint64_t)(uintptr_t)w.path,
            (uint64_t)(uintptr_t)w.ant_len, (uint64_t)(uintptr_t)w.ant_cost, (uint64_t)(uintptr_t)w.gbits,
            (uint64_t)(uintptr_t)w.iter_key, nq, p->ants, p->iterations, p->alpha, p->beta, p->max_steps,
            p->rho_q16, p->tau0_q16, p->tau_min_q16, p->tau_max_q16, p->q_deposit, p->theta, p->th_max,
            p->t_max_ms, p->vmax_kmh, p->mode, p->flags & (GMACOP_NO_LOAD_UPDATE | GMACOP_RESUME), p->seed,
            p->iter_offset,
            plan.legacy, plan.lds_lanes, plan.lds_apb, plan.lds_bpv, plan.maxd, plan.road_maxd,
            (uint64_t)plan.lds_bytes[1], (uint64_t)plan.lds_bytes[2], (uint64_t)plan.lds_bytes[3],
            (uint64_t)plan.lds_bytes[4], (uint64_t)plan.lds_bytes[5], (uint64_t)plan.lds_bytes[6], plan.glb,
            plan.glb_lanes, plan.glb_apb, plan.bloom_log2, plan.glb_nwords, plan.glb_blocks,
            (uint64_t)(uintptr_t)w.gveh, (uint64_t)(uintptr_t)w.gvrec, (uint64_t)(uintptr_t)w.gvlen,
            (uint64_t)(uintptr_t)w.gctl, (uint64_t)(uintptr_t)w.gwords, (uint64_t)(uintptr_t)w.gepoch,
            (uint64_t)lds, (uint64_t)(uintptr_t)w.vclass,
            (uint64_t)(uintptr_t)w.lazy, (uint64_t)(uintptr_t)w.dep_ind, (uint64_t)(uintptr_t)w.touched,
            (uint64_t)(uintptr_t)w.touched_n, (uint64_t)(uintptr_t)w.dev_gen, tcap, (uint64_t)w.side,
            (uint64_t)gp.on, gp.stride, gp.qcap, gp.fcap, gp.delta, gp.blocks, gp.threads, (uint64_t)(uintptr_t)w.goal,
            (uint64_t)(uintptr_t)w.goal_work, (uint64_t)(uintptr_t)w.goal_ctl};
        if (!g->gexec || key != g->gkey) {
            if (g->gexec) {
                (void)hipGraphExecDestroy(g->gexec);
                g->gexec = nullptr;
            }
            uint64_t saved[kTimedKernels];
            memcpy(saved, g->launches, sizeof(saved));
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            rc = enqueue();
            memcpy(g->launches, saved, sizeof(saved));   // counted per replay below
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) return fail(GMACOP_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
            const hipError_t ei = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                g->gexec = nullptr;
                return fail(GMACOP_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
            }
            g->gkey = key;
        }
        // launch counts follow the captured sequence
        if (NA > 0) {
            g->launches[0] += p->iterations;
            g->launches[1] += p->iterations;
            if (!plan.legacy && plan.any_lds()) g->launches[4] += p->iterations;
            if (!plan.legacy && plan.glb) g->launches[5] += p->iterations;
        }
        g->launches[2] += p->iterations;
        if (update_loads) g->launches[3] += p->iterations;
        if (gp.on && nq) g->launches[6] += 1;
        HIP_TRY(hipGraphLaunch(g->gexec, st));
    } else if ((rc = enqueue())) {
        return rc;
    }

    if (!dev_ptrs) {
        if (nq) {
            HIP_TRY(hipMemcpyAsync(out->path_len, best_len, sizeof(uint32_t) * nq, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(out->cost_ms, best_cost, sizeof(uint32_t) * nq, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(out->path_edges, best_path, sizeof(uint32_t) * (size_t)nq * S,
                                   hipMemcpyDeviceToHost, st));
        }
        HIP_TRY(hipMemcpyAsync(out->steps_total, steps, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    g->last_mode = p->mode;
    g->last_nq = nq;
    g->last_iters = p->iterations;
    g->last_p = *p;
    g->last_lazy = indep ? w.lazy : nullptr;
    g->last_gen = indep ? w.dev_gen : nullptr;
    return GMACOP_OK;
}

// ---- the allocation-free variant: workspace in a static device array ----

// Per-call workspace of gmacop_route_batch_noalloc.  One copy per GPU, held
// from the library's first use of that GPU until the process ends.  Host code
// never passes this name to a kernel: its device address comes from
// hipGetSymbolAddress, taken once per device.
}  // namespace
static __device__ __align__(256) uint64_t scratch[GMACOP_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];
namespace {

// What the host remembers about each device's scratch: its device address,
// and the layout and generation count of the regions whose contents carry
// over from one call to the next (visited words and epochs of the global
// walker, independent-mode pheromone rows).
struct ScratchDevice {
    void *ptr = nullptr;
    std::vector<uint64_t> layout;
    uint32_t gen_count = 0;
};
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
ScratchDevice g_scratch[kMaxDevices];

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int fill_u32(void *p, size_t words, hipStream_t st)
{
    if (!words) return GMACOP_OK;
    const unsigned grid = (unsigned)std::min<uint64_t>(blocks_for(words, 256), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, st, (uint32_t *)p, words, 0u);
    HIP_TRY(hipGetLastError());
    return GMACOP_OK;
}

// Consecutive 256-byte aligned pieces of one buffer (base NULL: sizes only).
struct Carver {
    uint8_t *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

// The workspace layout of one call; the regions that keep state across calls come first.
size_t carve_work(uint8_t *base, gmacop_graph *g, uint32_t nq, const gmacop_params *p, const WalkPlan &plan,
                  const GoalPlan &gp, CallWork *w)
{
    const bool indep = p->mode == GMACOP_MODE_INDEPENDENT;
    const bool dev_ptrs = (p->flags & GMACOP_DEVICE_PTRS) != 0;
    const uint32_t S = p->max_steps;
    const uint64_t NA = (uint64_t)nq * p->ants;
    const uint32_t tcap = (uint32_t)std::min<uint64_t>(g->m, (uint64_t)p->ants * S);
    Carver c{base};
    CallWork x{};
    if (gp.on) {
        x.goal_ctl = c.take<uint32_t>(2);
        x.goal_work = c.take<uint32_t>(gp.work_words());
        x.goal = c.take<uint32_t>((size_t)nq * gp.stride);
    }
    if (plan.glb) {
        const uint64_t slots = (uint64_t)plan.glb_blocks * plan.glb_apb;
        x.gctl = c.take<uint32_t>(3);
        x.gepoch = c.take<uint32_t>(slots);
        x.gwords = c.take<uint64_t>(slots * plan.glb_nwords);
    }
    if (indep && nq) {
        x.dev_gen = c.take<uint32_t>(1);
        x.lazy = c.take<uint64_t>((size_t)nq * g->m);
        x.dep_ind = c.take<uint64_t>((size_t)nq * g->m);
        x.touched_n = c.take<uint32_t>(nq);
        x.touched = c.take<uint32_t>((size_t)nq * tcap);
    }
    if (p->mode == GMACOP_MODE_GREEDY) {
        x.gnode = c.take<uint32_t>(nq);
        x.gchoice = c.take<uint32_t>(nq);
        x.gvcity = c.take<uint32_t>(nq);
        x.gcsum = c.take<uint64_t>(nq);
        x.gmark = c.take<uint64_t>(g->m);
        x.gmsum = c.take<uint64_t>(g->m);
    }
    x.path = c.take<uint32_t>((size_t)S * NA);
    x.ant_len = c.take<uint32_t>(NA);
    x.ant_cost = c.take<uint32_t>(NA);
    x.iter_key = c.take<uint64_t>(nq);
    x.vclass = c.take<uint8_t>(nq);
    if (plan.glb) {
        x.gveh = c.take<GlbVeh>(nq);
        x.gvrec = c.take<GlbVeh>(nq);
        x.gvlen = c.take<uint32_t>(nq);
    }
    if (!dev_ptrs) {
        x.best_path = c.take<uint32_t>((size_t)nq * S);
        x.best_len = c.take<uint32_t>(nq);
        x.best_cost = c.take<uint32_t>(nq);
        x.od = c.take<gmacop_od>(nq);
        x.steps = c.take<uint64_t>(1);
    }
    if (w) *w = x;
    return c.off;
}

}  // namespace

extern "C" int gmacop_route_batch(gmacop_graph *g, const gmacop_od *q, uint32_t nq, const gmacop_params *params,
                                  gmacop_result *out, void *hip_stream)
{
    if (!params) return fail(GMACOP_E_INVAL, "params is NULL");
    const gmacop_params pe = effective_params(*params);
    const gmacop_params *p = &pe;
    WalkPlan plan;
    int rc = route_check(g, q, nq, p, out, &plan);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    GoalPlan gp;
    if ((rc = goal_plan(g, p, nq, kGoalWorkBudget, 0, &gp))) return rc;
    CallWork w;
    if ((rc = route_work_grow(g, nq, p, plan, gp, st, &w))) return rc;
    return route_run(g, q, nq, p, out, st, plan, gp, w);
}

extern "C" int gmacop_route_batch_noalloc(gmacop_graph *g, const gmacop_od *q, uint32_t nq,
                                          const gmacop_params *params, gmacop_result *out, void *hip_stream)
{
    if (!params) return fail(GMACOP_E_INVAL, "params is NULL");
    const gmacop_params pe = effective_params(*params);
    const gmacop_params *p = &pe;
    if (p && (p->flags & (GMACOP_HIP_GRAPH | GMACOP_TIME_KERNELS)))
        return fail(GMACOP_E_INVAL, "gmacop_route_batch_noalloc takes neither GMACOP_HIP_GRAPH nor GMACOP_TIME_KERNELS");
    WalkPlan plan;
    int rc = route_check(g, q, nq, p, out, &plan);
    if (rc) return rc;
    if (plan.legacy)
        return fail(GMACOP_E_UNSUPPORTED, "gmacop_route_batch_noalloc needs a graph under 2^24 nodes");
    if (plan.glb) {
        // a smaller resident grid of the global walker keeps its visited words within half the scratch
        const uint64_t per_block = (uint64_t)plan.glb_apb * (std::max<uint32_t>(plan.glb_nwords, 1) * 8ull + 4);
        const uint64_t cap = std::max<uint64_t>(1, (GMACOP_NOALLOC_SCRATCH_BYTES / 2) / per_block);
        plan.glb_blocks = (uint32_t)std::min<uint64_t>(plan.glb_blocks, cap);
    }
    GoalPlan gp;   // the search's workspace: at most a quarter of the scratch
    if ((rc = goal_plan(g, p, nq, GMACOP_NOALLOC_SCRATCH_BYTES / 4, 0, &gp))) return rc;
    const size_t need = carve_work(nullptr, g, nq, p, plan, gp, nullptr);
    if (need > GMACOP_NOALLOC_SCRATCH_BYTES)
        return fail(GMACOP_E_NOMEM, "call needs %zu bytes of workspace; gmacop_route_batch_noalloc has %llu", need,
                    (unsigned long long)GMACOP_NOALLOC_SCRATCH_BYTES);
    if (g->device < 0 || g->device >= kMaxDevices) return fail(GMACOP_E_UNSUPPORTED, "device %d", g->device);
    hipStream_t st = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchDevice &sd = g_scratch[g->device];
    if (!sd.ptr) {   // first call on this device (it is current: route_check set it)
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(GMACOP_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        sd.ptr = ptr;
    }
    CallWork w;
    carve_work((uint8_t *)sd.ptr, g, nq, p, plan, gp, &w);
    const bool indep = p->mode == GMACOP_MODE_INDEPENDENT && nq;
    // regions that carry state from call to call start over when their place or size changes
    const std::vector<uint64_t> layout = {
        (uint64_t)(uintptr_t)w.gepoch, (uint64_t)(uintptr_t)w.gwords,
        plan.glb ? (uint64_t)plan.glb_blocks * plan.glb_apb : 0, plan.glb ? plan.glb_nwords : 0,
        (uint64_t)(uintptr_t)w.lazy, indep ? (uint64_t)nq * g->m : 0, (uint64_t)(uintptr_t)w.dev_gen};
    if (layout != sd.layout || (indep && sd.gen_count >= kGenMask)) {
        if (plan.glb) {
            const uint64_t slots = (uint64_t)plan.glb_blocks * plan.glb_apb;
            if ((rc = fill_u32(w.gepoch, slots, st)) || (rc = fill_u32(w.gwords, 2 * slots * plan.glb_nwords, st)))
                return rc;
        }
        if (indep) {
            const size_t rows = (size_t)nq * g->m;
            if ((rc = fill_u32(w.dev_gen, 1, st)) || (rc = fill_u32(w.lazy, 2 * rows, st)) ||
                (rc = fill_u32(w.dep_ind, 2 * rows, st)) || (rc = fill_u32(w.touched_n, nq, st)))
                return rc;
        }
        sd.layout = layout;
        sd.gen_count = 0;
    }
    if (plan.glb) {   // ticket counters, and the walk lengths that order the first list
        if ((rc = fill_u32(w.gctl, 3, st)) || (rc = fill_u32(w.gvlen, std::max<uint32_t>(nq, 1), st))) return rc;
    }
    if (gp.on && (rc = fill_u32(w.goal_ctl, 2, st))) return rc;   // the search's task counter
    if (indep) sd.gen_count++;
    w.side = false;
    w.allow_graph = false;
    rc = route_run(g, q, nq, p, out, st, plan, gp, w);
    g->last_lazy = nullptr;   // the rows live in the shared workspace: no gmacop_vehicle_tau_get after this call
    g->last_gen = nullptr;
    return rc;
}

extern "C" int gmacop_vehicle_tau_get(gmacop_graph *g, uint32_t vehicle, uint32_t *tau_q16, void *hip_stream)
{
    if (!g || !tau_q16) return fail(GMACOP_E_INVAL, "graph or output is NULL");
    if (g->last_mode != GMACOP_MODE_INDEPENDENT || vehicle >= g->last_nq || !g->last_lazy)
        return fail(GMACOP_E_INVAL, "no independent-mode vehicle %u in the last call", vehicle);
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    uint32_t *tmp = nullptr;
    int rc = dalloc(&tmp, g->m);
    if (rc) return rc;
    const gmacop_params &p = g->last_p;
    hipLaunchKernelGGL(k_materialize, dim3(blocks_for(g->m, 256)), dim3(256), 0, st, g->last_lazy + (size_t)vehicle * g->m,
                       g->last_gen, g->m, g->last_iters, p.tau0_q16, p.rho_q16, p.tau_min_q16, tmp);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(tau_q16, tmp, sizeof(uint32_t) * g->m, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(GMACOP_E_DEVICE, "vehicle_tau_get: %s", hipGetErrorString(e));
    return GMACOP_OK;
}

extern "C" int gmacop_state_set(gmacop_graph *g, const uint32_t *tau_q16, const uint32_t *load, void *hip_stream)
{
    if (!g) return fail(GMACOP_E_INVAL, "graph is NULL");
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    if (tau_q16) HIP_TRY(hipMemcpyAsync(g->tau, tau_q16, sizeof(uint32_t) * g->m, hipMemcpyHostToDevice, st));
    if (load) HIP_TRY(hipMemcpyAsync(g->load, load, sizeof(uint32_t) * g->m, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GMACOP_OK;
}

extern "C" int gmacop_set_base_load(gmacop_graph *g, const uint32_t *base_load, void *hip_stream)
{
    if (!g || !base_load) return fail(GMACOP_E_INVAL, "graph or loads are NULL");
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipMemcpyAsync(g->base_load, base_load, sizeof(uint32_t) * g->m, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GMACOP_OK;
}

extern "C" int gmacop_state_get(gmacop_graph *g, uint32_t *tau_q16, uint32_t *load, void *hip_stream)
{
    if (!g) return fail(GMACOP_E_INVAL, "graph is NULL");
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    if (tau_q16) HIP_TRY(hipMemcpyAsync(tau_q16, g->tau, sizeof(uint32_t) * g->m, hipMemcpyDeviceToHost, st));
    if (load) HIP_TRY(hipMemcpyAsync(load, g->load, sizeof(uint32_t) * g->m, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GMACOP_OK;
}

namespace {

// Exact goal rows on temporary device buffers: `tasks` destinations (dsts) or
// vehicles (od); rows [tasks][stride] city-local.
struct GoalRun {
    GoalPlan gp;
    uint32_t *rows = nullptr, *work = nullptr, *ctl = nullptr;
    ~GoalRun()
    {
        dfree(rows); dfree(work); dfree(ctl);
    }
};

int goal_run(gmacop_graph *g, const gmacop_od *od_dev, const uint32_t *dsts_dev, uint32_t tasks, hipStream_t st,
             GoalRun *r)
{
    gmacop_params gpar{};
    gpar.flags = GMACOP_GOAL_EXACT;
    int rc;
    if ((rc = goal_plan(g, &gpar, tasks, kGoalWorkBudget, 0, &r->gp)) ||
        (rc = dalloc(&r->rows, std::max<size_t>((size_t)tasks * r->gp.stride, 1))) ||
        (rc = dalloc(&r->work, std::max<size_t>(r->gp.work_words(), 1))) || (rc = dalloc(&r->ctl, 2)))
        return rc;
    HIP_TRY(hipMemsetAsync(r->ctl, 0, 2 * sizeof(uint32_t), st));
    GoalArgs goa{};
    goa.od = od_dev; goa.dsts = dsts_dev; goa.ntask = tasks; goa.n = g->n; goa.stride = r->gp.stride;
    goa.qcap = r->gp.qcap; goa.fcap = r->gp.fcap; goa.delta = r->gp.delta; goa.node_inst = g->node_inst; goa.inst_off = g->inst_off_dev; goa.rev_ptr = g->rev_ptr;
    goa.rev_tw = g->rev_tw; goa.goal = r->rows; goa.work = r->work; goa.ctl = r->ctl;
    if (tasks) hipLaunchKernelGGL(k_goal_sssp, dim3(r->gp.blocks), dim3(r->gp.threads), 0, st, goa);
    HIP_TRY(hipGetLastError());
    return GMACOP_OK;
}

}  // namespace

extern "C" int gmacop_goal_rows(gmacop_graph *g, const uint32_t *dst, uint32_t nd, uint32_t *h, void *hip_stream)
{
    if (!g || (nd && (!dst || !h))) return fail(GMACOP_E_INVAL, "graph, destinations or output is NULL");
    for (uint32_t i = 0; i < nd; ++i)
        if (dst[i] >= g->n) return fail(GMACOP_E_INVAL, "destination %u out of range", i);
    if (!nd) return GMACOP_OK;
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    uint32_t *ddst = nullptr;
    int rc = dalloc(&ddst, nd);
    if (rc) return rc;
    std::vector<uint32_t> rows;
    uint32_t stride = 0;
    hipError_t e = hipSuccess;
    {
        GoalRun r;
        e = hipMemcpyAsync(ddst, dst, sizeof(uint32_t) * nd, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess && (rc = goal_run(g, nullptr, ddst, nd, st, &r)) == GMACOP_OK) {
            stride = r.gp.stride;
            rows.resize((size_t)nd * stride);
            e = hipMemcpyAsync(rows.data(), r.rows, sizeof(uint32_t) * rows.size(), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
        }
        (void)hipStreamSynchronize(st);   // nothing may still use the buffers freed below
    }
    dfree(ddst);
    if (rc) return rc;
    if (e != hipSuccess) return fail(GMACOP_E_DEVICE, "gmacop_goal_rows: %s", hipGetErrorString(e));
    for (uint32_t i = 0; i < nd; ++i) {   // city-local rows to whole-graph rows
        const uint32_t c = instance_of(g, dst[i]), lo = g->inst_off[c], hi = g->inst_off[c + 1];
        uint32_t *out = h + (size_t)i * g->n;
        std::fill(out, out + g->n, 0xFFFFFFFFu);
        std::copy(rows.begin() + (size_t)i * stride, rows.begin() + (size_t)i * stride + (hi - lo), out + lo);
    }
    return GMACOP_OK;
}

extern "C" int gmacop_shortest_routes(gmacop_graph *g, const gmacop_od *q, uint32_t nq, uint32_t max_steps,
                                      gmacop_result *out, void *hip_stream)
{
    if (!g) return fail(GMACOP_E_INVAL, "graph is NULL");
    if (!out || !out->path_edges || !out->path_len || !out->cost_ms || !out->steps_total)
        return fail(GMACOP_E_INVAL, "result buffers missing");
    if (nq && !q) return fail(GMACOP_E_INVAL, "queries are NULL");
    if (max_steps == 0) return fail(GMACOP_E_INVAL, "max_steps must be >= 1");
    for (uint32_t i = 0; i < nq; ++i) {
        if (q[i].src >= g->n || q[i].dst >= g->n) return fail(GMACOP_E_INVAL, "query %u: node out of range", i);
        if (q[i].src == q[i].dst) return fail(GMACOP_E_INVAL, "query %u: src == dst", i);
        if (instance_of(g, q[i].src) != instance_of(g, q[i].dst))
            return fail(GMACOP_E_INVAL, "query %u: src and dst in different cities", i);
    }
    *out->steps_total = 0;
    if (!nq) return GMACOP_OK;
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    gmacop_od *dq = nullptr;
    uint32_t *dpath = nullptr, *dlen = nullptr, *dcost = nullptr;
    uint64_t *dsteps = nullptr;
    int rc;
    hipError_t e = hipSuccess;
    {
        GoalRun r;
        if (!(rc = dalloc(&dq, nq)) && !(rc = dalloc(&dpath, (size_t)nq * max_steps)) && !(rc = dalloc(&dlen, nq)) &&
            !(rc = dalloc(&dcost, nq)) && !(rc = dalloc(&dsteps, 1))) {
            e = hipMemcpyAsync(dq, q, sizeof(gmacop_od) * nq, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemsetAsync(dsteps, 0, sizeof(uint64_t), st);
            if (e == hipSuccess && !(rc = goal_run(g, dq, nullptr, nq, st, &r))) {
                hipLaunchKernelGGL(k_shortest_route, dim3(blocks_for(nq, 64)), dim3(64), 0, st, (const gmacop_od *)dq,
                                   nq, g->n, max_steps, (const uint32_t *)g->row_ptr, (const uint32_t *)g->col,
                                   (const uint32_t *)g->t0, (const uint32_t *)g->node_lo, (const uint32_t *)r.rows,
                                   r.gp.stride, dpath, dlen, dcost, dsteps);
                e = hipGetLastError();
                if (e == hipSuccess) e = hipMemcpyAsync(out->path_len, dlen, 4ull * nq, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipMemcpyAsync(out->cost_ms, dcost, 4ull * nq, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(out->path_edges, dpath, sizeof(uint32_t) * (size_t)nq * max_steps,
                                       hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipMemcpyAsync(out->steps_total, dsteps, 8, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
            }
        }
        (void)hipStreamSynchronize(st);   // nothing may still use the buffers freed below
    }
    dfree(dq); dfree(dpath); dfree(dlen); dfree(dcost); dfree(dsteps);
    if (rc) return rc;
    if (e != hipSuccess) return fail(GMACOP_E_DEVICE, "gmacop_shortest_routes: %s", hipGetErrorString(e));
    return GMACOP_OK;
}

extern "C" int gmacop_simulate(gmacop_graph *g, const gmacop_params *p, const uint32_t *path, uint32_t stride,
                               const uint32_t *path_len, const uint32_t *speed_kmh, const uint32_t *scen_off,
                               uint32_t nscen, uint32_t tick_ms, uint32_t max_ticks, uint32_t *arrival_ms,
                               uint32_t *wait_ms, uint32_t *ticks_run, void *hip_stream)
{
    if (!g || !p) return fail(GMACOP_E_INVAL, "graph or params is NULL");
    if (!nscen) return GMACOP_OK;
    if (!scen_off || !ticks_run) return fail(GMACOP_E_INVAL, "scenario offsets or ticks_run is NULL");
    if (tick_ms == 0) return fail(GMACOP_E_INVAL, "tick_ms must be >= 1");
    if (p->theta == 0) return fail(GMACOP_E_INVAL, "theta must be >= 1");
    if (scen_off[0] != 0) return fail(GMACOP_E_INVAL, "scen_off[0] must be 0");
    uint32_t most = 0;
    for (uint32_t b = 0; b < nscen; ++b) {
        if (scen_off[b + 1] < scen_off[b]) return fail(GMACOP_E_INVAL, "scen_off decreases at %u", b);
        most = std::max(most, scen_off[b + 1] - scen_off[b]);
    }
    const uint32_t nv = scen_off[nscen];
    if (nv && (!path || !path_len || !speed_kmh || !arrival_ms || !wait_ms))
        return fail(GMACOP_E_INVAL, "vehicle arrays are NULL");
    HIP_TRY(hipSetDevice(g->device));
    if (g->col_host.size() != g->m) {
        std::vector<uint32_t> col(g->m), tail(g->m);
        HIP_TRY(hipMemcpy(col.data(), g->col, 4ull * g->m, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(tail.data(), g->tail, 4ull * g->m, hipMemcpyDeviceToHost));
        g->col_host.swap(col);
        g->tail_host.swap(tail);
    }
    for (uint32_t i = 0; i < nv; ++i) {   // routes: roads in range, each starting where the last one ended
        const uint32_t L = path_len[i];
        if (L > stride) return fail(GMACOP_E_INVAL, "vehicle %u: route longer than its row", i);
        if (L && speed_kmh[i] == 0) return fail(GMACOP_E_INVAL, "vehicle %u: speed 0", i);
        for (uint32_t r = 0; r < L; ++r) {
            const uint32_t e = path[(size_t)i * stride + r];
            if (e >= g->m) return fail(GMACOP_E_INVAL, "vehicle %u: road out of range", i);
            if (r && g->tail_host[e] != g->col_host[path[(size_t)i * stride + r - 1]])
                return fail(GMACOP_E_INVAL, "vehicle %u: route not connected at road %u", i, r);
        }
    }
    // counts of each scenario in LDS when the roads fit, else a global slice per scenario
    const size_t lds_bytes = (size_t)8 * g->m;
    const bool in_lds = lds_bytes + 64 <= (size_t)g->max_lds && env_u32("GMACOP_SIM_GLOBAL", 0) == 0;
    if (!in_lds && (size_t)nscen * 2 * g->m > (4ull << 30))
        return fail(GMACOP_E_NOMEM, "road counts of %u scenarios exceed 16 GiB", nscen);
    const uint32_t threads = std::min<uint32_t>(1024, std::max<uint32_t>(kWave, (most + kWave - 1) / kWave * kWave));
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t NV = std::max<uint32_t>(nv, 1), SP = (size_t)std::max<uint32_t>(stride, 1) * NV;
    uint32_t *dpath = nullptr, *dlen = nullptr, *dspd = nullptr, *doff = nullptr, *dcounts = nullptr;
    uint32_t *droad = nullptr, *dwaited = nullptr, *darr = nullptr, *dwait = nullptr, *dticks = nullptr;
    uint64_t *dpos = nullptr;
    uint8_t *dflags = nullptr;
    int rc;
    hipError_t e = hipSuccess;
    if (!(rc = dalloc(&dpath, SP)) && !(rc = dalloc(&dlen, NV)) && !(rc = dalloc(&dspd, NV)) &&
        !(rc = dalloc(&doff, nscen + 1)) && !(rc = dalloc(&droad, NV)) && !(rc = dalloc(&dwaited, NV)) &&
        !(rc = dalloc(&darr, NV)) && !(rc = dalloc(&dwait, NV)) && !(rc = dalloc(&dticks, nscen)) &&
        !(rc = dalloc(&dpos, NV)) && !(rc = dalloc(&dflags, 3 * NV)) &&
        !(rc = in_lds ? GMACOP_OK : dalloc(&dcounts, (size_t)nscen * 2 * g->m))) {
        if (nv) e = hipMemcpyAsync(dpath, path, 4 * (size_t)nv * stride, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && nv) e = hipMemcpyAsync(dlen, path_len, 4ull * nv, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && nv) e = hipMemcpyAsync(dspd, speed_kmh, 4ull * nv, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(doff, scen_off, 4ull * (nscen + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && in_lds && lds_bytes > 65536)
            e = hipFuncSetAttribute((const void *)k_simulate, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds_bytes);
        if (e == hipSuccess) {
            SimArgs a{};
            a.path = dpath; a.path_len = dlen; a.spd = dspd; a.scen_off = doff;
            a.stride = std::max<uint32_t>(stride, 1); a.nscen = nscen; a.m = g->m; a.tick_ms = tick_ms;
            a.max_ticks = max_ticks; a.theta = p->theta; a.th_max = p->th_max; a.t_max = p->t_max_ms;
            a.col = g->col; a.len_dm = g->len_dm; a.rev_ptr = g->rev_ptr; a.rev_edge = g->rev_edge;
            a.speed = g->speed; a.sig = g->sig; a.counts = in_lds ? nullptr : dcounts;
            a.pos = dpos; a.road = droad; a.waited = dwaited;
            a.stopped = dflags; a.active = dflags + NV; a.act = dflags + 2 * NV;
            a.arrival = darr; a.wait_total = dwait; a.ticks = dticks;
            hipLaunchKernelGGL(k_simulate, dim3(nscen), dim3(threads), in_lds ? lds_bytes : 0, st, a);
            e = hipGetLastError();
        }
        if (e == hipSuccess && nv) e = hipMemcpyAsync(arrival_ms, darr, 4ull * nv, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && nv) e = hipMemcpyAsync(wait_ms, dwait, 4ull * nv, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ticks_run, dticks, 4ull * nscen, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    (void)hipStreamSynchronize(st);   // nothing may still use the buffers freed below
    dfree(dpath); dfree(dlen); dfree(dspd); dfree(doff); dfree(dcounts); dfree(droad); dfree(dwaited);
    dfree(darr); dfree(dwait); dfree(dticks); dfree(dpos); dfree(dflags);
    if (rc) return rc;
    if (e != hipSuccess) return fail(GMACOP_E_DEVICE, "gmacop_simulate: %s", hipGetErrorString(e));
    return GMACOP_OK;
}

extern "C" int gmacop_stats_get(gmacop_graph *g, gmacop_stats *s, int reset, void *hip_stream)
{
    if (!g || !s) return fail(GMACOP_E_INVAL, "graph or stats is NULL");
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    uint64_t c[kCounters];
    HIP_TRY(hipMemcpyAsync(c, g->counters, sizeof(c), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (auto &t : g->pending) {
        HIP_TRY(hipEventSynchronize(t.b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
        g->ms[t.kernel] += ms;
        g->spare.push_back(t.a);
        g->spare.push_back(t.b);
    }
    g->pending.clear();
    for (int k = 0; k < kTimedKernels; ++k) {
        s->launches[k] = g->launches[k];
        s->ms[k] = g->ms[k];
    }
    s->selections = c[0];
    s->candidates = c[1];
    s->arrivals = c[2];
    s->deposit_roads = c[3];
    s->longest_walks = c[4];
    for (int k = 0; k < 3; ++k) {
        s->walker_selections[k] = c[kWalkerCounters + 4 * k + 0];
        s->walker_candidates[k] = c[kWalkerCounters + 4 * k + 1];
        s->walker_arrivals[k] = c[kWalkerCounters + 4 * k + 2];
        s->walker_deposit_roads[k] = c[kWalkerCounters + 4 * k + 3];
    }
    if (reset) {
        HIP_TRY(hipMemsetAsync(g->counters, 0, sizeof(c), st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int k = 0; k < kTimedKernels; ++k) {
            g->launches[k] = 0;
            g->ms[k] = 0;
        }
    }
    return GMACOP_OK;
}

extern "C" void gmacop_release(gmacop_graph *g)
{
    delete g;
}

extern "C" const char *gmacop_last_error(void)
{
    return t_err.c_str();
}

// ---------------------------------------------------------------------------
// continuous-batching router
// ---------------------------------------------------------------------------

struct gmacop_server {
    gmacop_graph *g = nullptr;
    gmacop_params p{};
    uint32_t slots = 0, tcap = 0;
    size_t per_slot = 0;
    WalkPlan plan;
    // device, per slot
    gmacop_od *slot_od = nullptr;
    uint32_t *slot_t = nullptr, *slot_gen = nullptr, *best_path = nullptr, *best_len = nullptr, *best_cost = nullptr;
    uint64_t *iter_key = nullptr, *lazy = nullptr, *dep = nullptr, *steps = nullptr, *counters = nullptr;
    uint32_t *touched = nullptr, *touched_n = nullptr, *path = nullptr, *ant_len = nullptr, *ant_cost = nullptr;
    uint32_t *iter_max = nullptr;
    uint4 *rec32 = nullptr;   // global-walker road records with this router's costs
    GlbWork glb;
    uint8_t *vclass = nullptr;
    // exact goal term: a row per slot, computed at admission
    GoalPlan gp;
    uint32_t *goal = nullptr, *goal_work = nullptr, *goal_ctl = nullptr;
    // device, per road: this router's frozen-load cost table
    uint32_t *t0 = nullptr, *wf = nullptr, *load = nullptr, *cost = nullptr, *cnt = nullptr, *tau = nullptr;
    uint64_t *dep_shared = nullptr;
    // device staging for admissions and results
    uint32_t *adm_slots = nullptr, *adm_gen = nullptr, *done_slots = nullptr, *done_path = nullptr,
             *done_len = nullptr, *done_cost = nullptr;
    gmacop_od *adm_od = nullptr;
    // host mirror
    std::vector<uint32_t> free_list, t_host, qid_host, gen_host;
    std::vector<uint8_t> active;
    // host sources of a step's asynchronous copies: they live as long as the router, so a copy
    // still in flight (the step synchronises only at its end, or not at all on an error) never
    // reads freed memory
    std::vector<uint32_t> adm_slots_host, adm_gen_host, fin_host;
    std::vector<gmacop_od> adm_od_host;
    bool resync = false;               // a failed step emptied the router: rewrite the device slot table first
    uint64_t ticks = 0, admitted = 0, completed = 0;

    ~gmacop_server()
    {
        (void)hipSetDevice(g ? g->device : 0);
        dfree(slot_od); dfree(slot_t); dfree(slot_gen); dfree(best_path); dfree(best_len); dfree(best_cost);
        dfree(iter_key); dfree(lazy); dfree(dep); dfree(steps); dfree(counters); dfree(touched); dfree(touched_n);
        dfree(path); dfree(ant_len); dfree(ant_cost); dfree(iter_max); dfree(vclass); dfree(rec32);
        dfree(goal); dfree(goal_work); dfree(goal_ctl);
        glb.release();
        dfree(t0); dfree(wf); dfree(load); dfree(cost); dfree(cnt); dfree(tau); dfree(dep_shared);
        dfree(adm_slots); dfree(adm_gen); dfree(done_slots); dfree(done_path); dfree(done_len); dfree(done_cost);
        dfree(adm_od);
    }
};

namespace {

template <typename T>
int dalloc_zero(T **p, size_t count)
{
    int rc = dalloc(p, count);
    if (rc) return rc;
    HIP_TRY(hipMemset(*p, 0, std::max<size_t>(count, 1) * sizeof(T)));
    return GMACOP_OK;
}

}  // namespace

extern "C" int gmacop_server_create(gmacop_graph *g, const gmacop_params *p, uint32_t max_slots,
                                    uint64_t mem_budget_bytes, gmacop_server **out)
{
    if (!out) return fail(GMACOP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!g || !p) return fail(GMACOP_E_INVAL, "graph or params is NULL");
    gmacop_params pp = *p;
    pp.mode = GMACOP_MODE_INDEPENDENT;
    if (pp.flags & GMACOP_GOAL_EXACT)   // switched off: a run on the 1M-node city faulted, cause not found
        return fail(GMACOP_E_UNSUPPORTED, "the router does not take GMACOP_GOAL_EXACT");
    if (pp.flags & GMACOP_SIGNAL_TIMED)
        return fail(GMACOP_E_UNSUPPORTED, "the router does not take GMACOP_SIGNAL_TIMED");
    pp.flags &= GMACOP_TIME_KERNELS;   // loads are frozen; results go to host buffers
    int rc = validate_params(g, &pp, 1);
    if (rc) return rc;
    if (pp.iterations == 0 || pp.iterations > kLazyIterMax)
        return fail(GMACOP_E_UNSUPPORTED, "router needs 1..%u iterations", kLazyIterMax);
    HIP_TRY(hipSetDevice(g->device));
    gmacop_server *s = new gmacop_server();
    s->g = g;
    s->p = pp;
    s->plan = plan_walk(g, &pp, g->max_lds);
    if (s->plan.legacy) {
        delete s;
        return fail(GMACOP_E_UNSUPPORTED, "router needs a graph under 2^24 nodes");
    }
    const uint32_t A = pp.ants, S = pp.max_steps, m = g->m;
    s->tcap = (uint32_t)std::min<uint64_t>(m, (uint64_t)A * S);
    // queries are searched as they are admitted, a few at a time: large blocks keep each search short
    if ((rc = goal_plan(g, &pp, 0xFFFFFFFFull, kGoalWorkBudget / 4, 1024, &s->gp))) {
        delete s;
        return rc;
    }
    s->per_slot = (size_t)m * 16 + (size_t)s->tcap * 4 + (size_t)A * S * 4 + (size_t)A * 8 +
                  (size_t)S * 8 + sizeof(GlbVeh) + 64 + (s->gp.on ? (size_t)s->gp.stride * 4 : 0);
    size_t budget = mem_budget_bytes;
    if (!budget) {
        size_t fr = 0, tot = 0;
        HIP_TRY(hipMemGetInfo(&fr, &tot));
        budget = fr / 2;
    }
    // the global walker's visited words: a fixed amount, at most that of its full resident grid
    size_t fixed = s->gp.on ? s->gp.work_words() * 4 : 0;
    if (s->plan.glb) {
        WalkPlan full = s->plan;
        if ((rc = glb_grid(g->device, full, 0xFFFFFFFFull))) {
            delete s;
            return rc;
        }
        fixed = (size_t)full.glb_blocks * full.glb_apb * ((size_t)full.glb_nwords * sizeof(uint64_t) + 4);
    }
    budget = budget > fixed ? budget - fixed : 0;
    uint64_t cap_slots = budget / std::max<size_t>(s->per_slot, 1);
    if (max_slots) cap_slots = std::min<uint64_t>(cap_slots, max_slots);
    cap_slots = std::min<uint64_t>(cap_slots, 0xFFFFFFFFull / std::max<uint32_t>(A, 1));
    if (cap_slots == 0) {
        delete s;
        return fail(GMACOP_E_NOMEM, "memory budget below one query slot (%zu bytes)", s->per_slot);
    }
    const uint32_t NS = (uint32_t)cap_slots;
    s->slots = NS;
    const uint64_t NA = (uint64_t)NS * A;
    std::vector<gmacop_od> idle(NS, gmacop_od{0, 0xFFFFFFFFu, 0xFFFFFFFFu});
    if ((rc = upload(&s->slot_od, idle.data(), NS)) || (rc = dalloc_zero(&s->slot_t, NS)) ||
        (rc = dalloc_zero(&s->slot_gen, NS)) || (rc = dalloc(&s->best_path, (size_t)NS * S)) ||
        (rc = dalloc_zero(&s->best_len, NS)) || (rc = dalloc(&s->best_cost, NS)) || (rc = dalloc(&s->iter_key, NS)) ||
        (rc = dalloc_zero(&s->lazy, (size_t)NS * m)) || (rc = dalloc_zero(&s->dep, (size_t)NS * m)) ||
        (rc = dalloc_zero(&s->touched_n, NS)) || (rc = dalloc(&s->touched, (size_t)NS * s->tcap)) ||
        (rc = dalloc(&s->path, (size_t)S * NA)) || (rc = dalloc(&s->ant_len, NA)) || (rc = dalloc(&s->ant_cost, NA)) ||
        (rc = dalloc_zero(&s->steps, 1)) ||
        (rc = dalloc_zero(&s->counters, kCounters)) || (rc = dalloc_zero(&s->iter_max, 1)) || (rc = dalloc(&s->vclass, NS)) ||
        (rc = dalloc(&s->t0, m)) || (rc = dalloc(&s->wf, m)) || (rc = dalloc(&s->load, m)) ||
        (rc = dalloc(&s->cost, m)) || (rc = dalloc(&s->cnt, m)) || (rc = dalloc(&s->tau, m)) ||
        (rc = dalloc(&s->dep_shared, m)) || (rc = dalloc(&s->adm_slots, NS)) || (rc = dalloc(&s->adm_gen, NS)) ||
        (rc = dalloc(&s->adm_od, NS)) || (rc = dalloc(&s->done_slots, NS)) ||
        (rc = dalloc(&s->done_path, (size_t)NS * S)) || (rc = dalloc(&s->done_len, NS)) ||
        (rc = dalloc(&s->done_cost, NS)) || (s->plan.glb && (rc = glb_grid(g->device, s->plan, NA))) ||
        (s->plan.glb &&
         (rc = glb_prepare(s->glb, NS, (uint64_t)s->plan.glb_blocks * s->plan.glb_apb, s->plan.glb_nwords))) ||
        (s->gp.on && ((rc = dalloc(&s->goal, (size_t)NS * s->gp.stride)) ||
                      (rc = dalloc(&s->goal_work, std::max<size_t>(s->gp.work_words(), 1))) ||
                      (rc = dalloc_zero(&s->goal_ctl, 2))))) {
        std::string keep = t_err;
        delete s;
        t_err = keep;
        return rc;
    }
    // this router's cost table: loads frozen at the sensed loads
    if (s->plan.glb) {   // the global walker's road records, with this router's cost table
        if ((rc = dalloc(&s->rec32, 2 * (size_t)m))) {
            std::string keep = t_err;
            delete s;
            t_err = keep;
            return rc;
        }
        HIP_TRY(hipMemcpy(s->rec32, g->rec32, 2 * (size_t)m * sizeof(uint4), hipMemcpyDeviceToDevice));
    }
    EdgeInitArgs ia{m, pp.tau0_q16, pp.t_max_ms, 0u, g->col, g->len_dm, g->cycle, g->base_load, g->speed, g->green,
                    s->t0, s->wf, s->tau, s->load, s->cnt, s->dep_shared, (uint32_t *)s->rec32};
    hipLaunchKernelGGL(k_init_edges, dim3(blocks_for(m, 256)), dim3(256), 0, 0, ia);
    CostArgs ca{g->n, pp.theta, pp.th_max, g->rev_ptr, g->rev_edge, g->cycle, s->load, s->t0, s->wf, s->cost,
                (uint32_t *)s->rec32, 0u};
    hipLaunchKernelGGL(k_cost, dim3(blocks_for(g->n, 256)), dim3(256), 0, 0, ca);
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete s;
        return fail(GMACOP_E_DEVICE, "router set-up: %s", hipGetErrorString(e));
    }
    s->free_list.resize(NS);
    for (uint32_t i = 0; i < NS; ++i) s->free_list[i] = NS - 1 - i;   // pop_back hands out slot 0 first
    s->t_host.assign(NS, 0);
    s->qid_host.assign(NS, 0);
    s->adm_slots_host.reserve(NS);   // never reallocated: a pending copy keeps a valid source
    s->adm_gen_host.reserve(NS);
    s->fin_host.reserve(NS);
    s->adm_od_host.reserve(NS);
    s->gen_host.assign(NS, 0);
    s->active.assign(NS, 0);
    *out = s;
    return GMACOP_OK;
}

extern "C" int gmacop_server_info(const gmacop_server *s, uint32_t *slots, uint32_t *active, uint64_t *bytes_per_slot)
{
    if (!s) return fail(GMACOP_E_INVAL, "server is NULL");
    if (slots) *slots = s->slots;
    if (active) *active = s->slots - (uint32_t)s->free_list.size();
    if (bytes_per_slot) *bytes_per_slot = s->per_slot;
    return GMACOP_OK;
}

namespace {

// Empty the router after a step failed past its argument checks: every
// query in flight is dropped, all slots return to the free list, and the
// device slot table is rewritten as idle before the next admission.
void server_drop_all(gmacop_server *s)
{
    s->free_list.resize(s->slots);
    for (uint32_t i = 0; i < s->slots; ++i) s->free_list[i] = s->slots - 1 - i;
    std::fill(s->active.begin(), s->active.end(), (uint8_t)0);
    std::fill(s->t_host.begin(), s->t_host.end(), 0u);
    s->resync = true;
}

// Rewrite every slot of the device table as idle (after server_drop_all).
int server_resync(gmacop_server *s, hipStream_t st)
{
    std::vector<gmacop_od> &idle = s->adm_od_host;   // lives as long as the router: a pending copy keeps its source
    idle.assign(s->slots, gmacop_od{0, 0xFFFFFFFFu, 0xFFFFFFFFu});
    HIP_TRY(hipMemcpyAsync(s->slot_od, idle.data(), sizeof(gmacop_od) * s->slots, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    s->resync = false;
    return GMACOP_OK;
}

int server_step_impl(gmacop_server *s, const gmacop_od *admit, uint32_t take, uint32_t *done_qid, uint32_t *done_len,
                     uint32_t *done_cost, uint32_t *done_paths, uint32_t *n_done, hipStream_t st)
{
    gmacop_graph *g = s->g;
    const gmacop_params &p = s->p;
    const uint32_t A = p.ants, S = p.max_steps, NS = s->slots;
    int rc;
    if (s->plan.city_class != g->city_class_dev) {
        HIP_TRY(hipMemcpy(g->inst_fits, s->plan.city_class.data(), g->n_inst, hipMemcpyHostToDevice));
        g->city_class_dev = s->plan.city_class;
    }

    // 1. admissions
    if (take) {
        std::vector<uint32_t> &sl = s->adm_slots_host, &gens = s->adm_gen_host;
        sl.resize(take);
        gens.resize(take);
        for (uint32_t i = 0; i < take; ++i) {
            const uint32_t x = s->free_list.back();
            s->free_list.pop_back();
            if (x >= NS || s->active[x]) return fail(GMACOP_E_DEVICE, "router slot list corrupt (slot %u)", x);
            sl[i] = x;
            uint32_t gnew = s->gen_host[x] + 1;
            if (gnew > kGenMask) {   // generation numbers would repeat: clear the slot's pheromone row
                HIP_TRY(hipMemsetAsync(s->lazy + (size_t)x * g->m, 0, sizeof(uint64_t) * g->m, st));
                gnew = 1;
            }
            s->gen_host[x] = gnew;
            gens[i] = gnew;
            s->t_host[x] = 0;
            s->qid_host[x] = admit[i].qid;
            s->active[x] = 1;
        }
        HIP_TRY(hipMemcpyAsync(s->adm_slots, sl.data(), 4 * take, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(s->adm_gen, gens.data(), 4 * take, hipMemcpyHostToDevice, st));
        s->adm_od_host.assign(admit, admit + take);   // the caller's array may go before the copy runs
        HIP_TRY(hipMemcpyAsync(s->adm_od, s->adm_od_host.data(), sizeof(gmacop_od) * take, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_admit, dim3(blocks_for(take, 256)), dim3(256), 0, st, (const uint32_t *)s->adm_slots,
                           (const gmacop_od *)s->adm_od, (const uint32_t *)s->adm_gen, take, NS, s->slot_od, s->slot_t,
                           s->slot_gen, s->best_len, s->best_cost, s->iter_key);
        HIP_TRY(hipGetLastError());
        if (s->gp.on) {   // Calc_Dist of the admitted queries: their exact goal rows
            GoalArgs goa{};
            goa.od = s->slot_od; goa.list = s->adm_slots; goa.ntask = take; goa.n = g->n; goa.stride = s->gp.stride;
            goa.qcap = s->gp.qcap; goa.fcap = s->gp.fcap; goa.delta = s->gp.delta; goa.node_inst = g->node_inst; goa.inst_off = g->inst_off_dev;
            goa.rev_ptr = g->rev_ptr; goa.rev_tw = g->rev_tw; goa.goal = s->goal; goa.work = s->goal_work;
            goa.ctl = s->goal_ctl;
            KernelTimer kq{g, st, (p.flags & GMACOP_TIME_KERNELS) != 0};
            gmacop_graph::Timed tq{};
            if ((rc = kq.start(6, &tq))) return rc;
            hipLaunchKernelGGL(k_goal_sssp, dim3(std::min(s->gp.blocks, take)), dim3(s->gp.threads), 0, st, goa);
            HIP_TRY(hipGetLastError());
            if ((rc = kq.stop(&tq))) return rc;
        }
        s->admitted += take;
    }

    // 2. one iteration for every active slot
    const WalkPlan &plan = s->plan;
    const bool timing = (p.flags & GMACOP_TIME_KERNELS) != 0;
    KernelTimer kt{g, st, timing};
    gmacop_graph::Timed tm{};
    PherView pv{};
    pv.lazy = s->lazy; pv.gen = nullptr; pv.slot_t = s->slot_t; pv.slot_gen = s->slot_gen;
    pv.m = g->m; pv.tau0 = p.tau0_q16; pv.rho = p.rho_q16; pv.tau_min = p.tau_min_q16;
    DepView dv{s->dep, s->touched, s->touched_n, g->m, s->tcap, 1u};
    const uint32_t kgoal = p.vmax_kmh ? (uint32_t)((360ull << 16) / p.vmax_kmh) : 0;
    hipLaunchKernelGGL(k_classify, dim3(blocks_for(NS, 256)), dim3(256), 0, st, (const gmacop_od *)s->slot_od, NS,
                       g->n, (const uint32_t *)g->node_inst, (const uint8_t *)g->inst_fits, s->vclass);
    if (plan.glb) {
        const GlbListArgs gla{s->slot_od, s->vclass, g->row_ptr, g->node_lo, g->x, g->y, NS, A, kgoal,
                              s->glb.vrec, s->glb.veh, s->glb.ctl, s->glb.vlen, s->ant_len, s->ant_cost,
                              s->gp.on ? s->goal : nullptr, s->gp.stride};
        hipLaunchKernelGGL(k_glb_prep, dim3(blocks_for(NS, 256)), dim3(256), 0, st, gla);
        hipLaunchKernelGGL(k_glb_list, dim3(1), dim3(1024), 0, st, gla);
    }
    HIP_TRY(hipGetLastError());
    if ((rc = kt.start(0, &tm))) return rc;
    {
        LdsWalkArgs la{};
        la.row_ptr = g->row_ptr; la.col = g->col; la.cost = s->cost; la.pher = pv; la.depv = dv; la.x = g->x;
        la.y = g->y; la.rec = g->rec; la.tail = g->tail; la.rev_ptr = g->rev_ptr; la.rvs = g->rvs;
        la.node_inst = g->node_inst; la.inst_off = g->inst_off_dev;
        la.inst_eoff = g->inst_eoff_dev; la.vclass = s->vclass; la.od = s->slot_od; la.n = g->n; la.m = g->m;
        la.nq = NS; la.ants = A; la.apb = plan.lds_apb; la.bpv = plan.lds_bpv; la.max_steps = S; la.alpha = p.alpha;
        la.beta = p.beta; la.kgoal = kgoal; la.nwords = 0; la.seed_lo = (uint32_t)p.seed;
        la.seed_hi = (uint32_t)(p.seed >> 32); la.iter = p.iter_offset; la.t_local = 0; la.q_deposit = p.q_deposit;
        la.path = s->path; la.ant_len = s->ant_len; la.ant_cost = s->ant_cost; la.iter_key = s->iter_key;
        la.steps = s->steps; la.counters = g->counters; la.iter_max = g->iter_max;
        la.goal = s->gp.on ? s->goal : nullptr; la.goal_stride = s->gp.stride;
        if (plan.any_lds() && ((rc = setup_walk_lds(la, plan, st)) || (rc = launch_walk_lds_classes(la, plan, st))))
            return rc;
        if (plan.glb) {
            GlbWalkArgs ga{};
            ga.rec32 = s->rec32; ga.pher = pv; ga.depv = dv;
            ga.veh = s->glb.veh; ga.glb_n = s->glb.ctl; ga.tickets = s->glb.ctl + 1; ga.gwords = s->glb.words;
            ga.vlen = s->glb.vlen;
            ga.slot_epoch = s->glb.epoch; ga.m = g->m; ga.nq = NS; ga.ants = A; ga.apb = plan.glb_apb;
            ga.max_steps = S; ga.alpha = p.alpha; ga.beta = p.beta; ga.kgoal = kgoal; ga.nw2 = plan.glb_nwords;
            ga.bloom_log2 = plan.bloom_log2; ga.seed_lo = la.seed_lo; ga.seed_hi = la.seed_hi; ga.iter = p.iter_offset;
            ga.t_local = 0; ga.q_deposit = p.q_deposit; ga.path = s->path; ga.ant_len = s->ant_len;
            ga.ant_cost = s->ant_cost; ga.iter_key = s->iter_key; ga.steps = s->steps;
            ga.counters = g->counters; ga.iter_max = g->iter_max;
            ga.goal = la.goal; ga.goal_stride = s->gp.stride;
            if ((rc = launch_walk_glb_any(ga, plan, st))) return rc;
        }
    }
    if ((rc = kt.stop(&tm)) || (rc = kt.start(1, &tm))) return rc;
    BestArgs ba{NS, A, S, 0u, g->m, g->iter_max, g->counters, s->path, s->ant_len, s->iter_key, s->best_path, s->best_len,
                s->best_cost, s->cnt};
    hipLaunchKernelGGL(k_best, dim3(NS), dim3(kWave), 0, st, ba);
    if ((rc = kt.stop(&tm)) || (rc = kt.start(2, &tm))) return rc;
    ApplyArgs aa{g->m, s->tcap, 0, p.tau0_q16, p.rho_q16, p.tau_min_q16, p.tau_max_q16, p.theta, s->load, nullptr,
                 s->slot_t, s->slot_gen, s->lazy, s->dep, s->touched, s->touched_n};
    hipLaunchKernelGGL(k_apply_touched, dim3(NS), dim3(256), 0, st, aa);
    if ((rc = kt.stop(&tm))) return rc;
    hipLaunchKernelGGL(k_advance, dim3(blocks_for(NS, 256)), dim3(256), 0, st, NS, g->n, p.iterations, s->slot_od,
                       s->slot_t);
    HIP_TRY(hipGetLastError());

    // 3. finished queries
    std::vector<uint32_t> &fin = s->fin_host;
    fin.clear();
    for (uint32_t i = 0; i < NS; ++i)
        if (s->active[i]) {
            s->t_host[i] += 1;
            if (s->t_host[i] >= p.iterations) fin.push_back(i);
        }
    const uint32_t nf = (uint32_t)fin.size();
    if (nf) {
        HIP_TRY(hipMemcpyAsync(s->done_slots, fin.data(), 4 * nf, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_gather_done, dim3(nf), dim3(64), 0, st, (const uint32_t *)s->done_slots, NS, S,
                           (const uint32_t *)s->best_path, (const uint32_t *)s->best_len,
                           (const uint32_t *)s->best_cost, s->done_path, s->done_len, s->done_cost);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(done_len, s->done_len, 4 * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(done_cost, s->done_cost, 4 * nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(done_paths, s->done_path, sizeof(uint32_t) * (size_t)nf * S, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    for (uint32_t i = 0; i < nf; ++i) {
        done_qid[i] = s->qid_host[fin[i]];
        s->active[fin[i]] = 0;
        s->free_list.push_back(fin[i]);
    }
    *n_done = nf;
    s->completed += nf;
    s->ticks++;
    return GMACOP_OK;
}

}  // namespace

extern "C" int gmacop_server_step(gmacop_server *s, const gmacop_od *admit, uint32_t *n_admit, uint32_t *done_qid,
                                  uint32_t *done_len, uint32_t *done_cost, uint32_t *done_paths, uint32_t done_cap,
                                  uint32_t *n_done, void *hip_stream)
{
    if (!s || !n_admit || !n_done) return fail(GMACOP_E_INVAL, "server or counts are NULL");
    if (*n_admit && !admit) return fail(GMACOP_E_INVAL, "admissions are NULL");
    gmacop_graph *g = s->g;
    const gmacop_params &p = s->p;
    const uint32_t NS = s->slots;
    // queries finishing in this step: those admitted iterations-1 steps ago, plus the new ones if iterations == 1
    uint32_t finishing = 0;
    for (uint32_t i = 0; i < NS; ++i) finishing += s->active[i] && s->t_host[i] + 1 == p.iterations;
    const uint32_t take = std::min<uint32_t>(*n_admit, (uint32_t)s->free_list.size());
    if (finishing + (p.iterations == 1 ? take : 0) > done_cap)
        return fail(GMACOP_E_INVAL, "done_cap %u below the %u queries finishing in this step", done_cap,
                    finishing + (p.iterations == 1 ? take : 0));
    if ((finishing || (p.iterations == 1 && take)) && (!done_qid || !done_len || !done_cost || !done_paths))
        return fail(GMACOP_E_INVAL, "result buffers are NULL");
    for (uint32_t i = 0; i < take; ++i) {
        if (admit[i].qid == 0xFFFFFFFFu) return fail(GMACOP_E_INVAL, "admission %u uses the reserved qid", i);
        if (admit[i].src >= g->n || admit[i].dst >= g->n || admit[i].src == admit[i].dst)
            return fail(GMACOP_E_INVAL, "admission %u: invalid nodes", i);
        if (instance_of(g, admit[i].src) != instance_of(g, admit[i].dst))
            return fail(GMACOP_E_INVAL, "admission %u: src and dst in different cities", i);
    }
    *n_done = 0;
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    int rc;
    if (s->resync && (rc = server_resync(s, st))) {
        *n_admit = 0;
        return rc;
    }
    rc = server_step_impl(s, admit, take, done_qid, done_len, done_cost, done_paths, n_done, st);
    if (rc) {
        const std::string keep = t_err;
        (void)hipStreamSynchronize(st);   // nothing of the failed step may still read the router's buffers
        (void)hipGetLastError();
        server_drop_all(s);
        *n_admit = 0;
        *n_done = 0;
        t_err = keep;
        return rc;
    }
    *n_admit = take;
    return GMACOP_OK;
}

extern "C" int gmacop_server_set_base_load(gmacop_server *s, const uint32_t *base_load, void *hip_stream)
{
    if (!s || !base_load) return fail(GMACOP_E_INVAL, "server or loads are NULL");
    gmacop_graph *g = s->g;
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t st = (hipStream_t)hip_stream;
    // the router's loads become the new sensed loads, and its cost table follows them
    HIP_TRY(hipMemcpyAsync(s->load, base_load, sizeof(uint32_t) * g->m, hipMemcpyHostToDevice, st));
    CostArgs ca{g->n, s->p.theta, s->p.th_max, g->rev_ptr, g->rev_edge, g->cycle, s->load, s->t0, s->wf, s->cost,
                (uint32_t *)s->rec32, 0u};
    hipLaunchKernelGGL(k_cost, dim3(blocks_for(g->n, 256)), dim3(256), 0, st, ca);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return GMACOP_OK;
}

extern "C" void gmacop_server_release(gmacop_server *s)
{
    delete s;
}
