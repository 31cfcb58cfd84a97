// HIP kernels of the CSP solver for gfx950 (CDNA4, wave64).
//
// One wavefront is one search worker.  A worker keeps the domains of its
// current node as word-packed bitsets in LDS (bit a of variable i = value
// lo_i + a), revises constraints to a fixpoint with 64 lanes at a time,
// tests the node with ballots and wave reductions, and backtracks through a
// private trail of domain snapshots in HBM (the paper's per-domain
// save/restore stacks, Sec. 2.2).  Workers take subtrees from a global
// lock-free work queue and donate their shallowest open subtree when others
// are idle, so the whole search stays on the GPU (Sec. 2.1).
//
// Propagation (Sec. 1.1 "constraint propagation", parallelised as in
// Sec. 2.2): every constraint is split into propagators.  A binary
// constraint gives two directed units, each revising its target variable
// against its source; all-different and linear-sum constraints are revised
// by the whole wave.  A round revises every unit whose source changed in the
// previous round; rounds repeat until nothing changes or a domain empties.
// Domain removals are atomic ANDs on LDS words, so units of one round may run
// in any order: all propagators are monotone, and the fixpoint they reach is
// unique, hence identical to the oracle's.
//
// Binary units run in one of two layouts:
//   LANE: one lane per unit; the lane ORs the support rows of the source's
//         live values (rows indexed by source value give the allowed target
//         values) and ANDs the union into the target.
//   SEG:  S = pow2 >= dmax lanes per unit, one lane per target value; each
//         lane tests its value's support row against the source domain and a
//         64-lane ballot assembles the new target words.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cubics_internal.h"
#include "cubics_mlp.h"

// This file is compiled once per domain width (CUBICS_ONLY_WM = 1, 2, 4, 8)
// so that the kernel variants build in parallel; the width-1 object also
// carries the queue-reset kernel and the dispatchers.
#ifndef CUBICS_ONLY_WM
#define CUBICS_ONLY_WM 1
#endif

namespace cubics {

#define DEV __device__ __forceinline__

typedef unsigned long long u64;

DEV int lane_id() { return __lane_id(); }
// Order LDS traffic between the lanes of one wave (compiler barrier + wait).
DEV void wsync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }
DEV int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
DEV uint32_t uniu(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
DEV u64 uni64(u64 x) {
    uint32_t lo = uniu((uint32_t)x), hi = uniu((uint32_t)(x >> 32));
    return ((u64)hi << 32) | lo;
}
DEV long long unill(long long x) { return (long long)uni64((u64)x); }

DEV uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}
DEV int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
DEV long long wave_sum64(long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
DEV u64 wave_sumu64(u64 v) { return (u64)wave_sum64((long long)v); }
DEV uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint32_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// -------------------------------------------------------------- atomics
DEV uint32_t ld_acq(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
DEV uint32_t ld_rlx(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV int ld_rlx_i(int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV u64 ld_rlx_u64(u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void st_rel(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void st_rel_i(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
DEV int add_i(int32_t *p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV uint32_t add_u(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV uint32_t or_u(uint32_t *p, uint32_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void st_rlx(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// device-scope fences: acquire invalidates, release writes back this XCD's L2
DEV void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
DEV void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
// Queue slots move between XCDs through device-coherent (agent-scope)
// accesses only, so handing one over needs no write-back of the producer's
// whole L2 (an agent release) and no invalidation of the consumer's (an agent
// acquire): the producer waits until its slot stores are acknowledged before
// it publishes the slot's sequence word, and the consumer reads the slot only
// after it has claimed that word.  With thousands of hand-overs per second in
// a search's tail, the L2-wide fences stall every worker on the XCD.
DEV void slot_stores_done() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // keeps the compiler's order
    __builtin_amdgcn_s_waitcnt(0);                          // vmcnt(0): stores acknowledged
}
DEV void slot_claimed() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); }
DEV u64 add_u64(u64 *p, u64 v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV bool cas_u32(uint32_t *p, uint32_t *expected, uint32_t desired) {
    return __hip_atomic_compare_exchange_strong(p, expected, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// workgroup-scope words in LDS (the idle-poll token)
DEV bool lds_take(uint32_t *p) {
    uint32_t e = 0u;
    return __hip_atomic_compare_exchange_strong(p, &e, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
}
DEV uint32_t lds_ld(uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
DEV void lds_st(uint32_t *p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
DEV bool cas_i(int32_t *p, int expected, int desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------- bit helpers
template <int WM>
DEV int pop_w(const uint32_t (&d)[WM], int W) {
    int s = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k)
        if (k < W) s += __popc(d[k]);
    return s;
}
template <int WM>
DEV int low_w(const uint32_t (&d)[WM], int W) {  // lowest set index, -1 if empty
    int r = -1;
#pragma unroll
    for (int k = WM - 1; k >= 0; --k)
        if (k < W && d[k]) r = 32 * k + __ffs(d[k]) - 1;
    return r;
}
template <int WM>
DEV int high_w(const uint32_t (&d)[WM], int W) {  // highest set index, -1 if empty
    int r = -1;
#pragma unroll
    for (int k = 0; k < WM; ++k)
        if (k < W && d[k]) r = 32 * k + 31 - __clz(d[k]);
    return r;
}
// mask of indices <= ub (ub may be negative or >= 32W)
DEV uint32_t mask_le(int ub, int k) {
    int t = ub - 32 * k;
    if (t < 0) return 0u;
    if (t >= 31) return 0xFFFFFFFFu;
    return (2u << t) - 1u;
}
// mask of indices >= lb
DEV uint32_t mask_ge(int lb, int k) {
    int t = lb - 32 * k;
    if (t <= 0) return 0xFFFFFFFFu;
    if (t >= 32) return 0u;
    return ~((1u << t) - 1u);
}
DEV uint32_t bit_in_word(int idx, int k) {  // word k of the singleton {idx}; idx may be out of range
    return (idx >= 32 * k && idx < 32 * k + 32) ? (1u << (idx - 32 * k)) : 0u;
}

// ------------------------------------------------------------ counters
struct Counters {
    u64 nodes, fails, sols, steals, tasks;  // wave-uniform, flushed per instance
    u64 rev, bytes;                         // per lane, flushed per instance
    u64 stamp;                              // nodes of this worker, never reset
    u64 ubytes;                             // wave-uniform bytes (trail copies)
    // VAR layout, per lane, folded into rev / bytes at every poll and flush:
    // revisions, revisions that changed the target, and the support rows that
    // table revisions read, one per source value (bytes = 8 rev + 4 chg +
    // 4 rows for one-word domains)
    uint32_t vrev, vchg, vpop;
};

// ------------------------------------------------- binary unit revisions

// Element i of a read-only instance array.  GM: the array lies in global
// memory (instance tables read from HBM), so the load is a global load with
// a uniform base and a 32-bit offset; else it may lie in LDS (an instance
// staged once per workgroup) and goes through a generic pointer.
template <bool GM, class T>
DEV T ldg(const T *p, uint32_t i) {
    if constexpr (GM) return ((const __attribute__((address_space(1))) T *)p)[i];
    else return p[i];
}
template <bool GM>
DEV Unit ld_unit(const Unit *p, uint32_t i) {
    if constexpr (GM) {
        typedef int v4i __attribute__((ext_vector_type(4)));
        const v4i v = ((const __attribute__((address_space(1))) v4i *)p)[i];
        return Unit{v.x, v.y, v.z, v.w};
    } else {
        return p[i];
    }
}

// Rows fetched together by one lane of a LANE table revision: the lane
// gathers up to R live values, then issues all their row loads before it
// uses any, so a revision waits on one memory round trip per batch instead
// of one per row.  Most revisions end within a few rows (the union covers
// the target early), and every slot of a batch costs the whole wave its
// instructions whether or not the lane has a value for it, so batches are
// short: 3 rows for domains of at most two words (measured against 1, 2, 4,
// 6 and 8 on the 4096-instance batch, and against a short first batch
// followed by longer ones).  A missing value reads row -1, the W zero words
// the packer puts before every row block.
#ifndef CUBICS_RB_NARROW
#define CUBICS_RB_NARROW 3
#endif
template <int WM>
constexpr int row_batch() { return WM <= 2 ? CUBICS_RB_NARROW : (WM == 4 ? 4 : 2); }

// Word k of row j - 1 of a row block, j >= 0: rm points at the block's row
// -1 (the zero words before it), stride is the row length in bytes.  One
// unsigned 32 x 32 + 64-bit multiply-add gives a row's address; the words of
// a row then differ only by an immediate offset.
template <bool GM>
DEV uint32_t ld_row(const uint32_t *rm, uint32_t j, uint32_t stride, int k) {
    const char *a = (const char *)rm + (unsigned long long)j * stride;
    if constexpr (GM) return ((const __attribute__((address_space(1))) uint32_t *)a)[k];
    else return ((const uint32_t *)a)[k];
}

// The next R live values of word w of a domain, as value index + 1 (0 once
// the word is exhausted: row -1, the zero row).
template <int R>
DEV void next_values(uint32_t &bits, int w, uint32_t (&j)[R]) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const uint32_t lo = (uint32_t)(__ffs(bits));  // 1-based, 0 when empty
        j[q] = w == 0 ? lo : (bits ? 32u * (uint32_t)w + lo : 0u);
        bits &= bits - 1u;
    }
}

// One batch of the union orientation: OR the rows of the next R source
// values into acc.
template <int R, int WM, bool GM>
DEV void union_batch(const uint32_t *rm, uint32_t stride, uint32_t &bits, int w, int W, uint32_t (&acc)[WM]) {
    uint32_t ix[R];
    next_values<R>(bits, w, ix);
    uint32_t r[R][WM];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < WM; ++k) r[q][k] = k < W ? ld_row<GM>(rm, ix[q], stride, k) : 0u;
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < WM; ++k) acc[k] |= r[q][k];
}

// One batch of the test orientation: keep each of the next R target values
// of word w whose row meets the source domain.
template <int R, int WM, bool GM>
DEV void test_batch(const uint32_t *rm, uint32_t stride, uint32_t &bits, int w, int W, const uint32_t (&ds)[WM],
                    uint32_t &keep) {
    uint32_t ix[R];
    next_values<R>(bits, w, ix);
    uint32_t r[R][WM];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < WM; ++k) r[q][k] = k < W ? ld_row<GM>(rm, ix[q], stride, k) : 0u;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        uint32_t hit = 0u;
#pragma unroll
        for (int k = 0; k < WM; ++k) hit |= r[q][k] & ds[k];
        // ix = 0 reads the zero row: never supported
        if (hit) keep |= 1u << ((ix[q] - 1u) & 31u);
    }
}

// LANE layout: full new target words for one unit.  A table revision first
// ORs the rows of up to RB source values (bits over the target: the values
// of the source's lowest non-empty word); a target value that union covers
// is supported.  If those were all the source's values, the union is exact.
// Otherwise each target value still open has its own row (bits over the
// source) tested against the source domain.  With at most RB target values
// the revision tests them all at once instead.  So a revision reads at most
// RB + (open target values) rows, and most end after one batch: a lane's
// batch costs its wave every slot, so no lane walks a long union for the
// one value it removes.  *rows_read receives the rows read (the algorithmic
// row traffic).
template <int WM, bool GM>
DEV void revise_lane(const InstDev &I, const Unit &u, const uint32_t (&ds)[WM],
                     const uint32_t (&dt)[WM], uint32_t (&nw)[WM], int W, int *rows_read) {
    const int ty = u.tt >> 24;
    constexpr int RB = row_batch<WM>();
#pragma unroll
    for (int k = 0; k < WM; ++k) nw[k] = dt[k];
    *rows_read = 0;
    if (ty == U_TABLE) {
        const int ps = pop_w(ds, W), pt = pop_w(dt, W);
        const uint32_t stride = 4u * (uint32_t)W;
        const uint32_t *rs = I.rows + (uint32_t)u.p1 - W;  // row -1, rows by source value
        const uint32_t *rt = I.rows + (uint32_t)u.p0 - W;  // row -1, rows by target value
        uint32_t acc[WM], keep[WM], open[WM];
#pragma unroll
        for (int k = 0; k < WM; ++k) acc[k] = keep[k] = 0u;
        // the source's lowest non-empty word
        int w0 = 0;
        uint32_t b0 = 0u;
#pragma unroll
        for (int k = WM - 1; k >= 0; --k)
            if (k < W && ds[k]) w0 = k;
#pragma unroll
        for (int k = 0; k < WM; ++k) b0 = (k == w0) ? ds[k] : b0;
        const int n0 = __popc(b0);
        const bool direct = pt <= RB;
        uint32_t ub = direct ? 0u : b0;
        if (ub) union_batch<RB, WM, GM>(rs, stride, ub, w0, W, acc);
        const bool exact = !direct && ub == 0u && n0 == ps;
#pragma unroll
        for (int k = 0; k < WM; ++k) open[k] = exact ? 0u : (dt[k] & ~acc[k]);
        *rows_read = (direct ? 0 : min(n0, RB)) + pop_w(open, W);
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            if (w >= W) break;
            uint32_t bits = open[w];
            while (bits) test_batch<RB, WM, GM>(rt, stride, bits, w, W, ds, keep[w]);
        }
#pragma unroll
        for (int k = 0; k < WM; ++k) nw[k] = (dt[k] & acc[k]) | keep[k];
    } else if (ty == U_NEQ) {
        if (pop_w(ds, W) == 1) {
            int a = low_w(ds, W) + u.p0;
#pragma unroll
            for (int k = 0; k < WM; ++k) nw[k] = dt[k] & ~bit_in_word(a, k);
        }
    } else if (ty == U_LT_UB) {
        int ub = high_w(ds, W) + u.p0 - 1;
#pragma unroll
        for (int k = 0; k < WM; ++k) nw[k] = dt[k] & mask_le(ub, k);
    } else if (ty == U_LT_LB) {
        int lb = low_w(ds, W) - u.p0 + 1;
#pragma unroll
        for (int k = 0; k < WM; ++k) nw[k] = dt[k] & mask_ge(lb, k);
    } else if (ty == U_QUEENS) {
        if (pop_w(ds, W) <= 3) {
            // unsupported = intersection over b in D_src of {b+d, b+d+k, b+d-k}
            uint32_t uns[WM];
#pragma unroll
            for (int k = 0; k < WM; ++k) uns[k] = 0xFFFFFFFFu;
            const int kk = u.p0, dl = u.p1;
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                if (w >= W) break;
                uint32_t bits = ds[w];
                while (bits) {
                    int b = 32 * w + __ffs(bits) - 1 + dl;
                    bits &= bits - 1;
#pragma unroll
                    for (int k = 0; k < WM; ++k)
                        uns[k] &= bit_in_word(b, k) | bit_in_word(b + kk, k) | bit_in_word(b - kk, k);
                }
            }
#pragma unroll
            for (int k = 0; k < WM; ++k) nw[k] = dt[k] & ~uns[k];
        }
    }
}

// SEG layout: is target value index a supported by the source domain?
template <int WM, bool GM>
DEV bool supported_seg(const InstDev &I, const Unit &u, const uint32_t (&ds)[WM], int a, int W) {
    const int ty = u.tt >> 24;
    if (ty == U_TABLE) {
        const uint32_t r0 = (uint32_t)u.p0 + (uint32_t)a * (uint32_t)W;
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k < W) acc |= ldg<GM>(I.rows, r0 + (uint32_t)k) & ds[k];
        return acc != 0;
    } else if (ty == U_NEQ) {
        return !(pop_w(ds, W) == 1 && low_w(ds, W) + u.p0 == a);
    } else if (ty == U_LT_UB) {
        return a <= high_w(ds, W) + u.p0 - 1;
    } else if (ty == U_LT_LB) {
        return a >= low_w(ds, W) - u.p0 + 1;
    } else {  // QUEENS: some b in D_src outside {a-d, a-d-k, a-d+k}
        const int b0 = a - u.p1;
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k < W)
                cnt += __popc(ds[k] & ~(bit_in_word(b0, k) | bit_in_word(b0 - u.p0, k) |
                                        bit_in_word(b0 + u.p0, k)));
        return cnt > 0;
    }
}

// algorithmic bytes of one binary revision: both domains, the support rows
// the revision reads for a table (rows of W words), and the target written
// back if changed
DEV u64 rev_bytes(int W, int rows, bool changed) {
    return 8ull * W + (changed ? 4ull * W : 0ull) + 4ull * (u64)rows * (u64)W;
}

// LDS view of one worker.
struct Lds {
    uint32_t *dom;   // [nmax * wmax]
    u64 *dA, *dB;    // dirty sets [ndw]
    u64 *gp;         // pending globals [ngw]
    uint32_t *fails; // [nmax] failures below each branching variable (policy feature)
    int32_t *trig;   // [nmax + 1] the task's instance's unit ranges per source variable
                     // (staged per task: the fixpoint loop reads two per dirty variable)
    uint32_t *scr;   // 32 words scratch
    float *feat;     // [nmax][4] learned search: the task's static features
    float *vscr;     // [VALUE_LDS_WORDS] learned value order: value features, then scores
};

// Process one chunk of binary units in LANE layout.  Returns wave-uniform fail.
template <int WM, bool GM>
DEV bool chunk_lane(const InstDev &I, const Lds &L, u64 *nxt, int my_u, Counters &C, int lane) {
    const int W = I.W;
    bool changed = false;
    int tgt = 0;
    if (my_u >= 0) {
        const Unit u = ld_unit<GM>(I.units, (uint32_t)my_u);
        tgt = u.tt & 0xFFFFFF;
        uint32_t ds[WM], dt[WM], nw[WM];
#pragma unroll
        for (int k = 0; k < WM; ++k) {
            ds[k] = k < W ? L.dom[u.src * W + k] : 0u;
            dt[k] = k < W ? L.dom[tgt * W + k] : 0u;
        }
        int rows_read = 0;
        revise_lane<WM, GM>(I, u, ds, dt, nw, W, &rows_read);
#pragma unroll
        for (int k = 0; k < WM; ++k) changed |= (k < W) && nw[k] != dt[k];
        C.rev += 1;
        C.bytes += rev_bytes(W, rows_read, changed);
        if (changed) {
#pragma unroll
            for (int k = 0; k < WM; ++k)
                if (k < W && nw[k] != dt[k]) atomicAnd(&L.dom[tgt * W + k], nw[k]);
            atomicOr(&nxt[tgt >> 6], 1ull << (tgt & 63));
        }
    }
    wsync();
    bool empty = false;
    if (changed) {
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k < W) acc |= L.dom[tgt * W + k];
        empty = acc == 0;
    }
    return __ballot(empty) != 0;
}

// Process one chunk of binary units in SEG layout (W <= 2, S lanes per unit).
template <int WM, bool GM>
DEV bool chunk_seg(const InstDev &I, const Lds &L, u64 *nxt, int my_u, int sh, Counters &C, int lane) {
    const int W = I.W;
    const int S = 1 << sh;
    const int slot = lane >> sh, a = lane & (S - 1);
    bool sup = false;
    Unit u = {0, 0, 0, 0};
    uint32_t dt[WM];
#pragma unroll
    for (int k = 0; k < WM; ++k) dt[k] = 0u;
    if (my_u >= 0) {
        u = ld_unit<GM>(I.units, (uint32_t)my_u);
        const int tgt = u.tt & 0xFFFFFF;
        uint32_t ds[WM];
#pragma unroll
        for (int k = 0; k < WM; ++k) {
            ds[k] = k < W ? L.dom[u.src * W + k] : 0u;
            dt[k] = k < W ? L.dom[tgt * W + k] : 0u;
        }
        const bool live = (a < 32 * W) && ((dt[a >> 5] >> (a & 31)) & 1u);
        if (live) sup = supported_seg<WM, GM>(I, u, ds, a, W);
    }
    const u64 m = __ballot(sup);
    bool changed = false;
    int tgt = u.tt & 0xFFFFFF;
    if (my_u >= 0 && a == 0) {
        const u64 seg = sh == 6 ? m : ((m >> (slot << sh)) & ((1ull << S) - 1ull));
        uint32_t nw[WM];
#pragma unroll
        for (int k = 0; k < WM; ++k) nw[k] = k == 0 ? (uint32_t)seg : (k == 1 ? (uint32_t)(seg >> 32) : 0u);
#pragma unroll
        for (int k = 0; k < WM; ++k) changed |= (k < W) && nw[k] != dt[k];
        C.rev += 1;
        // one support row per live target value (each lane reads its own)
        C.bytes += rev_bytes(W, (u.tt >> 24) == U_TABLE ? pop_w(dt, W) : 0, changed);
        if (changed) {
#pragma unroll
            for (int k = 0; k < WM; ++k)
                if (k < W && nw[k] != dt[k]) atomicAnd(&L.dom[tgt * W + k], nw[k]);
            atomicOr(&nxt[tgt >> 6], 1ull << (tgt & 63));
        }
    }
    wsync();
    bool empty = false;
    if (changed) {
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k < W) acc |= L.dom[tgt * W + k];
        empty = acc == 0;
    }
    return __ballot(empty) != 0;
}

// ----------------------------------------------------- global revisions

// value-space shifts of W-word bitsets (bit a -> bit a + s, and back)
template <int WM>
DEV void shl_w(const uint32_t (&d)[WM], int s, uint32_t (&o)[WM]) {
    const int q = s >> 5, r = s & 31;
#pragma unroll
    for (int k = 0; k < WM; ++k) {
        uint32_t hi = 0u, lo = 0u;
#pragma unroll
        for (int j = 0; j < WM; ++j) {
            hi = (j == k - q) ? d[j] : hi;
            lo = (j == k - q - 1) ? d[j] : lo;
        }
        o[k] = r ? ((hi << r) | (lo >> (32 - r))) : hi;
    }
}
template <int WM>
DEV void shr_w(const uint32_t (&d)[WM], int s, uint32_t (&o)[WM]) {
    const int q = s >> 5, r = s & 31;
#pragma unroll
    for (int k = 0; k < WM; ++k) {
        uint32_t lo = 0u, hi = 0u;
#pragma unroll
        for (int j = 0; j < WM; ++j) {
            lo = (j == k + q) ? d[j] : lo;
            hi = (j == k + q + 1) ? d[j] : hi;
        }
        o[k] = r ? ((lo >> r) | (hi << (32 - r))) : lo;
    }
}

// All-different: the values of singleton scope variables are removed from the
// other scope variables (two singletons with one value fail); then the union
// of the scope domains must hold at least k values.  Domains are aligned in
// value space: bit a of variable v stands for value lo_v + a, i.e. bit
// a + (lo_v - base) of the union, with base = the smallest lo of the scope.
template <int WM>
DEV bool revise_alldiff(const InstDev &I, const GDesc &g, const Lds &L, u64 *nxt, Counters &C, int lane) {
    const int W = I.W, k = g.k, base = g.coef_off;
    const int32_t *sc = I.gscope + g.scope_off;
    uint32_t U[WM];
    int nsing = 0;
#pragma unroll
    for (int w = 0; w < WM; ++w) U[w] = 0u;
    for (int t = lane; t < k; t += 64) {
        const int v = sc[t];
        uint32_t d[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
        if (pop_w(d, W) == 1) {
            ++nsing;
            const int sft = I.lo[v] - base;
            if (sft) {
                uint32_t e[WM];
                shl_w(d, sft, e);
#pragma unroll
                for (int w = 0; w < WM; ++w) U[w] |= e[w];
            } else {
#pragma unroll
                for (int w = 0; w < WM; ++w) U[w] |= d[w];
            }
        }
    }
    int upop = 0;
#pragma unroll
    for (int w = 0; w < WM; ++w) {
        if (w < W) {
            U[w] = wave_or(U[w]);
            upop += __popc(U[w]);
        }
    }
    nsing = wave_sum(nsing);
    C.rev += lane == 0 ? 1 : 0;
    C.bytes += lane == 0 ? 4ull * (u64)k * W : 0ull;
    if (upop < nsing) return true;  // two singletons share a value
    uint32_t Un[WM];
    bool emp = false;
#pragma unroll
    for (int w = 0; w < WM; ++w) Un[w] = 0u;
    for (int t = lane; t < k; t += 64) {
        const int v = sc[t];
        const int sft = I.lo[v] - base;
        uint32_t d[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
        if (pop_w(d, W) >= 2) {
            uint32_t Uv[WM];
            if (sft) {
                shr_w(U, sft, Uv);
            } else {
#pragma unroll
                for (int w = 0; w < WM; ++w) Uv[w] = U[w];
            }
            bool ch = false;
            uint32_t any = 0;
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                if (w < W) {
                    uint32_t nd = d[w] & ~Uv[w];
                    ch |= nd != d[w];
                    d[w] = nd;
                    any |= nd;
                }
            }
            if (ch) {
#pragma unroll
                for (int w = 0; w < WM; ++w)
                    if (w < W) L.dom[v * W + w] = d[w];
                atomicOr(&nxt[v >> 6], 1ull << (v & 63));
                C.bytes += 4ull * W;
                emp |= any == 0;
            }
        }
        if (sft) {
            uint32_t e[WM];
            shl_w(d, sft, e);
#pragma unroll
            for (int w = 0; w < WM; ++w) Un[w] |= e[w];
        } else {
#pragma unroll
            for (int w = 0; w < WM; ++w) Un[w] |= d[w];
        }
    }
    int unpop = 0;
#pragma unroll
    for (int w = 0; w < WM; ++w)
        if (w < W) unpop += __popc(wave_or(Un[w]));
    const bool fail = (__ballot(emp) != 0) || unpop < k;
    wsync();
    return fail;
}

// Readlane of a 64-bit lane value from a uniform lane index.
DEV u64 readlane64(u64 v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((u64)hi << 32) | lo;
}

template <int WM>
DEV bool bit_of(const uint32_t (&d)[WM], int v) {
    bool r = false;
#pragma unroll
    for (int w = 0; w < WM; ++w) r |= (w == (v >> 5)) && ((d[w] >> (v & 31)) & 1u);
    return r;
}

// All-different to generalized arc consistency (Regin's method), one lane
// per scope variable (k <= 64), domains aligned in value space.
//  1. A matching covering the scope: for each variable in turn, a
//     breadth-first search for an augmenting path over value bitsets (layer
//     = values reachable through the previous layer's matched variables);
//     none -> the constraint has no solution.
//  2. With M(x) the value of x, value u points to M(x) when u is in D_x.
//     (x, v) belongs to some solution iff v = M(x), or v is reachable from
//     an unmatched value, or v = M(y) with y reachable from x in the graph
//     x -> y when M(x) is in D_y (both ends on one alternating cycle).
// Scratch (LDS bytes): par[32 WM] the variable through which a value was
// reached, then mv[64] the matched value of each variable.
template <int WM>
DEV bool revise_alldiff_gac(const InstDev &I, const GDesc &g, const Lds &L, u64 *nxt, Counters &C, int lane) {
    const int W = I.W, k = g.k, base = g.coef_off;
    const int32_t *sc = I.gscope + g.scope_off;
    uint8_t *par = (uint8_t *)L.scr;
    uint8_t *mv = par + 32 * WM;
    const bool act = lane < k;
    const int v = act ? sc[lane] : 0;
    const int sft = act ? I.lo[v] - base : 0;
    uint32_t d[WM], Dv[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) d[w] = (act && w < W) ? L.dom[v * W + w] : 0u;
    if (sft) {
        shl_w(d, sft, Dv);
    } else {
#pragma unroll
        for (int w = 0; w < WM; ++w) Dv[w] = d[w];
    }
    C.rev += lane == 0 ? 1 : 0;
    C.bytes += lane == 0 ? 4ull * (u64)k * W : 0ull;
    if (__ballot(act && pop_w(Dv, WM) == 0)) return true;

    // ---- 1. matching
    int M = -1;
    uint32_t used[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) used[w] = 0u;
    for (int x = 0; x < k; ++x) {
        uint32_t F[WM], Vis[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            F[w] = (uint32_t)__builtin_amdgcn_readlane((int)Dv[w], x);
            Vis[w] = F[w];
        }
        for (int t = lane; t < 32 * WM; t += 64)
            if (bit_of<WM>(F, t)) par[t] = (uint8_t)x;
        wsync();
        int found = -1;
        for (;;) {
#pragma unroll
            for (int w = WM - 1; w >= 0; --w) {
                const uint32_t fr = F[w] & ~used[w];
                if (fr) found = 32 * w + __ffs(fr) - 1;
            }
            if (found >= 0) break;
            const bool on = act && M >= 0 && bit_of<WM>(F, M);
            uint32_t NF[WM];
            bool any = false;
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                NF[w] = wave_or(on ? (Dv[w] & ~Vis[w]) : 0u);
                any |= NF[w] != 0u;
            }
            if (!any) return true;  // x cannot be matched: no solution
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                uint32_t bits = on ? (Dv[w] & NF[w]) : 0u;
                while (bits) {
                    par[32 * w + __ffs(bits) - 1] = (uint8_t)lane;
                    bits &= bits - 1;
                }
                Vis[w] |= NF[w];
                F[w] = NF[w];
            }
            wsync();
        }
        // augment: walk back from the free value to x, shifting the matches
        int val = found;
        for (;;) {
            const int y = uni((int)par[val]);
            const int prev = __builtin_amdgcn_readlane(M, y);
            if (lane == y) M = val;
            if (y == x) break;
            val = prev;
        }
#pragma unroll
        for (int w = 0; w < WM; ++w)
            if (w == (found >> 5)) used[w] |= 1u << (found & 31);
        wsync();
    }

    // ---- 2. values reachable from unmatched values
    uint32_t R[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) R[w] = wave_or(Dv[w]) & ~used[w];
    for (;;) {
        bool hit = false;
#pragma unroll
        for (int w = 0; w < WM; ++w) hit |= (Dv[w] & R[w]) != 0u;
        const bool add = act && hit && !bit_of<WM>(R, M);
        if (__ballot(add) == 0ull) break;
#pragma unroll
        for (int w = 0; w < WM; ++w) R[w] |= wave_or((add && (M >> 5) == w) ? (1u << (M & 31)) : 0u);
    }
    // ---- 3. reachability between variables (transitive closure)
    u64 inn = 0;  // on lane y: variables a != y with M(a) in D_y
    for (int a = 0; a < k; ++a) {
        const int ma = __builtin_amdgcn_readlane(M, a);
        if (act && a != lane && bit_of<WM>(Dv, ma)) inn |= 1ull << a;
    }
    u64 out = 0;  // on lane x: variables y with x -> y
    for (int y = 0; y < k; ++y) {
        const u64 iy = readlane64(inn, y);
        if ((iy >> lane) & 1ull) out |= 1ull << y;
    }
    for (int z = 0; z < k; ++z) {
        const u64 oz = readlane64(out, z);
        if ((out >> z) & 1ull) out |= oz;
    }
    if (act) mv[lane] = (uint8_t)M;
    wsync();
    // ---- 4. keep = M(x), reachable values, matched values of reachable variables
    uint32_t K[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) K[w] = R[w] | ((act && (M >> 5) == w) ? (1u << (M & 31)) : 0u);
    {
        u64 o = act ? out : 0ull;
        while (o) {
            const int y = __ffsll((long long)o) - 1;
            o &= o - 1;
            const int my = mv[y];
#pragma unroll
            for (int w = 0; w < WM; ++w)
                if (w == (my >> 5)) K[w] |= 1u << (my & 31);
        }
    }
    bool ch = false;
#pragma unroll
    for (int w = 0; w < WM; ++w) {
        const uint32_t nv = Dv[w] & K[w];
        ch |= nv != Dv[w];
        Dv[w] = nv;
    }
    if (act && ch) {
        uint32_t nd[WM];
        if (sft) {
            shr_w(Dv, sft, nd);
        } else {
#pragma unroll
            for (int w = 0; w < WM; ++w) nd[w] = Dv[w];
        }
#pragma unroll
        for (int w = 0; w < WM; ++w)
            if (w < W) L.dom[v * W + w] = nd[w];
        atomicOr(&nxt[v >> 6], 1ull << (v & 63));
        C.bytes += 4ull * W;
    }
    wsync();
    return false;
}

DEV long long floor_div(long long a, long long b) {  // b > 0
    long long q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

// sum a_t x_t <= b (a_t > 0): S = sum a_t * min(D_t); fail if S > b; each
// variable keeps the values v with a_t * v + (S - a_t * min(D_t)) <= b.
template <int WM>
DEV bool revise_linear(const InstDev &I, const GDesc &g, const Lds &L, u64 *nxt, Counters &C, int lane) {
    const int W = I.W, k = g.k;
    const int32_t *sc = I.gscope + g.scope_off;
    const int64_t *co = I.gcoef + g.coef_off;
    const long long b = co[0];
    long long part = 0;
    for (int t = lane; t < k; t += 64) {
        const int v = sc[t];
        uint32_t d[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
        part += (long long)co[1 + t] * (long long)(I.lo[v] + low_w(d, W));
    }
    const long long S = wave_sum64(part);
    C.rev += lane == 0 ? 1 : 0;
    C.bytes += lane == 0 ? 4ull * (u64)k * W : 0ull;
    if (S > b) return true;
    for (int t = lane; t < k; t += 64) {
        const int v = sc[t];
        uint32_t d[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
        const long long at = co[1 + t];
        const long long mn = (long long)I.lo[v] + low_w(d, W);
        const long long slack = b - (S - at * mn);  // >= at * mn, since S <= b
        const long long mx = (long long)I.lo[v] + high_w(d, W);
        // only a variable whose largest value breaks the bound needs the
        // (64-bit) division for its new upper bound
        const long long ubi = at * mx > slack ? floor_div(slack, at) - I.lo[v] : 32LL * W;
        if (ubi < 32LL * W - 1) {
            const int ub = (int)ubi;  // >= the min index, since S <= b
            bool ch = false;
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                if (w < W) {
                    uint32_t nd = d[w] & mask_le(ub, w);
                    ch |= nd != d[w];
                    d[w] = nd;
                }
            }
            if (ch) {
#pragma unroll
                for (int w = 0; w < WM; ++w)
                    if (w < W) L.dom[v * W + w] = d[w];
                atomicOr(&nxt[v >> 6], 1ull << (v & 63));
                C.bytes += 4ull * W;
            }
        }
    }
    wsync();
    return false;
}

// Position (0-based) of the r-th set bit of x, r < popcount(x): halve the
// window by the population of its low half.
DEV int select32(uint32_t x, int r) {
    int pos = 0;
#pragma unroll
    for (int s = 16; s >= 1; s >>= 1) {
        const int c = __popc(x & ((1u << s) - 1u));
        if (r >= c) {
            r -= c;
            x >>= s;
            pos += s;
        }
    }
    return pos;
}

// Keep the values v of x_v (domain d, minimum index mn) with
// a * (lo_v + v) <= slack; the bound never falls below the minimum since the
// caller checked S <= b.
template <int WM>
DEV void linear_cut(const InstDev &I, const Lds &L, u64 *nxt, Counters &C, int v, uint32_t (&d)[WM],
                    long long at, long long slack) {
    const int W = I.W;
    const long long mx = (long long)I.lo[v] + high_w(d, W);
    const long long ubi = at * mx > slack ? floor_div(slack, at) - I.lo[v] : 32LL * W;
    if (ubi < 32LL * W - 1) {
        const int ub = (int)ubi;
        bool ch = false;
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            if (w < W) {
                uint32_t nd = d[w] & mask_le(ub, w);
                ch |= nd != d[w];
                d[w] = nd;
            }
        }
        if (ch) {
#pragma unroll
            for (int w = 0; w < WM; ++w)
                if (w < W) L.dom[v * W + w] = d[w];
            atomicOr(&nxt[v >> 6], 1ull << (v & 63));
            C.bytes += 4ull * W;
        }
    }
}

// sum a_t x_t <= b bounded with the all-different groups inside the scope.
// A group's variables take pairwise different values, so its part of the sum
// is at least L_g = sum_j c_j u_j: c_1 >= c_2 >= ... its coefficients, u_1 <
// u_2 < ... the smallest values of the union of its domains (rearrangement:
// the largest coefficient meets the smallest value).  With P_g the group's
// sum of a_t min D_t,
//   S = sum over ungrouped t of a_t min D_t + sum_g max(P_g, L_g);
// fail if S > b or a group's union holds fewer values than the group has
// variables.  x_t keeps the values v with a_t v + rest_t <= b, rest_t =
// S - a_t min D_t, less max(P_g, L_g) - P_g for t in group g (the rest of the
// group counted by its minima).  One lane per group variable (k_g <= 64);
// lane g keeps group g's excess max(P_g, L_g) - P_g.
template <int WM>
DEV bool revise_linear_ad(const InstDev &I, const GDesc &g, const Lds &L, u64 *nxt, Counters &C, int lane) {
    const int W = I.W, k = g.k;
    const int32_t *sc = I.gscope + g.scope_off, *grp = sc + k;
    const int64_t *co = I.gcoef + g.coef_off;
    const long long b = co[0];
    const int G = (int)co[1 + k];
    long long part = 0;
    for (int t = lane; t < k; t += 64) {
        if (grp[t] >= 0) continue;
        const int v = sc[t];
        uint32_t d[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
        part += (long long)co[1 + t] * (long long)(I.lo[v] + low_w(d, W));
    }
    long long S = wave_sum64(part), excess = 0;
    C.rev += lane == 0 ? 1 : 0;
    C.bytes += lane == 0 ? 4ull * (u64)k * W : 0ull;
    const int32_t *pos = grp + k;
    int off = 2 + k;
    for (int q = 0; q < G; ++q) {
        const int base = (int)co[off], kg = (int)co[off + 1];
        const int64_t *cg = co + off + 2;
        uint32_t U[WM];
        long long pg = 0;
#pragma unroll
        for (int w = 0; w < WM; ++w) U[w] = 0u;
        if (lane < kg) {
            const int t = pos[lane], v = sc[t];
            uint32_t d[WM];
#pragma unroll
            for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
            pg = (long long)co[1 + t] * (long long)(I.lo[v] + low_w(d, W));
            const int sft = I.lo[v] - base;
            if (sft) {
                shl_w(d, sft, U);
            } else {
#pragma unroll
                for (int w = 0; w < WM; ++w) U[w] = d[w];
            }
        }
        int upop = 0;
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            if (w < W) {
                U[w] = wave_or(U[w]);
                upop += __popc(U[w]);
            }
        }
        if (upop < kg) return true;  // wave-uniform
        long long lg = 0;
        if (lane < kg) {
            int r = lane, idx = 0;
            bool found = false;
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                const int pc = __popc(U[w]);
                if (!found && r < pc) {
                    idx = 32 * w + select32(U[w], r);
                    found = true;
                } else if (!found) {
                    r -= pc;
                }
            }
            lg = (long long)cg[lane] * (long long)(base + idx);
        }
        const long long P = wave_sum64(pg), Lg = wave_sum64(lg);
        const long long mx = Lg > P ? Lg : P;
        S += mx;
        excess = lane == q ? mx - P : excess;
        pos += kg;
        off += 2 + kg;
    }
    if (S > b) return true;
    for (int t = lane; t < k; t += 64) {
        if (grp[t] >= 0) continue;
        const int v = sc[t];
        uint32_t d[WM];
#pragma unroll
        for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
        const long long at = co[1 + t];
        const long long mn = (long long)I.lo[v] + low_w(d, W);
        linear_cut<WM>(I, L, nxt, C, v, d, at, b - (S - at * mn));
    }
    pos = grp + k;
    off = 2 + k;
    for (int q = 0; q < G; ++q) {
        const int kg = (int)co[off + 1];
        const long long ex = readlane64((u64)excess, q);
        if (lane < kg) {
            const int t = pos[lane], v = sc[t];
            uint32_t d[WM];
#pragma unroll
            for (int w = 0; w < WM; ++w) d[w] = w < W ? L.dom[v * W + w] : 0u;
            const long long at = co[1 + t];
            const long long mn = (long long)I.lo[v] + low_w(d, W);
            linear_cut<WM>(I, L, nxt, C, v, d, at, b - (S - ex - at * mn));
        }
        pos += kg;
        off += 2 + kg;
    }
    wsync();
    return false;
}

// ------------------------------------------------------------ propagate

// Revise to the fixpoint.  L.dA holds the initially dirty variables.
// Returns true on failure (wave-uniform).
// GLOB: global constraints may occur; SEGC: the SEG layout is compiled in.
template <int WM, bool GLOB, bool SEGC, bool GM>
DEV bool propagate(const InstDev &I, const Lds &L, int layout, Counters &C, int lane) {
    const int n = I.n;
    const int ndw = (n + 63) >> 6, ngw = (I.n_glob + 63) >> 6;
    const bool seg = SEGC && layout == 2 && I.seg_ok;
    const int sh = seg ? (31 - __clz(I.S)) : 0;
    const int CH = seg ? (64 >> sh) : 64;
    const int slot = seg ? (lane >> sh) : lane;
    u64 *cur = L.dA, *nxt = L.dB;
    for (;;) {
        for (int w = lane; w < ndw; w += 64) nxt[w] = 0ull;
        for (int w = lane; w < ngw; w += 64) L.gp[w] = 0ull;
        wsync();
        bool fail = false;
        int cnt = 0, my_u = -1;
        for (int w = 0; w < ndw && !fail; ++w) {
            u64 bits = uni64(cur[w]);
            while (bits && !fail) {
                const int j = w * 64 + __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                int beg = uni(L.trig[j]);
                const int end = uni(L.trig[j + 1]);
                while (beg < end) {
                    const int take = min(end - beg, CH - cnt);
                    if (slot >= cnt && slot < cnt + take) my_u = beg + slot - cnt;
                    cnt += take;
                    beg += take;
                    if (cnt == CH) {
                        fail = (SEGC && seg) ? chunk_seg<WM, GM>(I, L, nxt, my_u, sh, C, lane)
                                             : chunk_lane<WM, GM>(I, L, nxt, my_u, C, lane);
                        cnt = 0;
                        my_u = -1;
                        if (fail) break;
                    }
                }
                if (GLOB && I.n_glob) {
                    const int gb = I.gtrig_off[j], ge = I.gtrig_off[j + 1];
                    for (int t = gb + lane; t < ge; t += 64) {
                        const int g = I.gtrig[t];
                        atomicOr(&L.gp[g >> 6], 1ull << (g & 63));
                    }
                }
            }
        }
        if (!fail && cnt > 0)
            fail = (SEGC && seg) ? chunk_seg<WM, GM>(I, L, nxt, my_u, sh, C, lane)
                                 : chunk_lane<WM, GM>(I, L, nxt, my_u, C, lane);
        if (fail) return true;
        if (GLOB && I.n_glob) {
            wsync();
            for (int w = 0; w < ngw; ++w) {
                u64 bits = uni64(L.gp[w]);
                while (bits) {
                    const int gi = w * 64 + __ffsll((long long)bits) - 1;
                    bits &= bits - 1;
                    const GDesc g = I.gdesc[gi];
                    const bool f = g.type == G_ALLDIFF     ? revise_alldiff<WM>(I, g, L, nxt, C, lane)
                                   : g.type == G_LINEAR    ? revise_linear<WM>(I, g, L, nxt, C, lane)
                                   : g.type == G_LINEAR_AD ? revise_linear_ad<WM>(I, g, L, nxt, C, lane)
                                                           : revise_alldiff_gac<WM>(I, g, L, nxt, C, lane);
                    if (f) return true;
                }
            }
        }
        wsync();
        bool anyn = false;
        for (int w = lane; w < ndw; w += 64) anyn |= nxt[w] != 0ull;
        if (__ballot(anyn) == 0ull) return false;
        u64 *t = cur;
        cur = nxt;
        nxt = t;
    }
}

// Mark every variable dirty (root propagation).
DEV void dirty_all(const Lds &L, int n, int lane) {
    const int ndw = (n + 63) >> 6;
    for (int w = lane; w < ndw; w += 64) {
        const int rem = n - 64 * w;
        L.dA[w] = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    }
    wsync();
}
DEV void dirty_one(const Lds &L, int n, int x, int lane) {
    const int ndw = (n + 63) >> 6;
    for (int w = lane; w < ndw; w += 64) L.dA[w] = (w == (x >> 6)) ? (1ull << (x & 63)) : 0ull;
    wsync();
}

// Node test: 0 open (returns the first-fail variable in *bx), 1 solution,
// 2 failed (an empty domain).
template <int WM>
DEV int node_test(const InstDev &I, const Lds &L, int lane, int *bx) {
    const int n = I.n, W = I.W;
    uint32_t key = 0xFFFFFFFFu;
    bool empty = false;
    for (int i = lane; i < n; i += 64) {
        int p = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k < W) p += __popc(L.dom[i * W + k]);
        empty |= p == 0;
        if (p >= 2) {
            const uint32_t kk = ((uint32_t)p << 16) | (uint32_t)i;
            key = kk < key ? kk : key;
        }
    }
    if (__ballot(empty)) return 2;
    key = wave_min(key);
    if (key == 0xFFFFFFFFu) return 1;
    *bx = (int)(key & 0xFFFFu);
    return 0;
}

// ------------------------------------------------------------- queue

// Bounded MPMC ring (per-cell sequence numbers; Vyukov's bounded queue).
// Called by lane 0 only.  Every poll uses relaxed loads, so idle workers never
// invalidate caches; a successful pop or reserve is followed by one acquire
// fence, and publishing is preceded by one release fence.
// Consumers take tickets: an idle wave claims the next position with one
// fetch-add on the head and waits on that position's own sequence word until
// a producer publishes it.  Compare-and-swap pops made every polling wave
// race for each new task, a storm of atomics on one word per hand-over that
// capped hand-overs at a few 10^4 per second in a search's tail.
// Flags every ring's signal word (lane 0 only): SIG_DONE when an instance's
// done flag was set, SIG_STOP when the whole launch stops.
DEV void signal_rings(const SearchParams &P, uint32_t bit) {
    for (int r = 0; r < P.nrings; ++r) or_u(&P.qb->ring[r].signal, bit);
}
// Stop the launch (lane 0 only): reason 2 time limit, 3 cancelled, 4 trail overflow.
DEV void stop_launch(const SearchParams &P, int reason) {
    P.g->stop_reason = reason;
    st_rel_i(&P.g->stop, 1);
    signal_rings(P, SIG_STOP);
}

DEV bool q_reserve(const SearchParams &P, uint32_t *cell, uint32_t *posout) {
    uint32_t pos = ld_rlx(&P.q->tail);
    for (;;) {
        const uint32_t c = pos & P.qmask;
        const uint32_t s = ld_rlx(&P.qseq[c]);
        const int dif = (int)(s - pos);
        if (dif == 0) {
            if (cas_u32(&P.q->tail, &pos, pos + 1u)) {
                slot_claimed();
                *cell = c;
                *posout = pos;
                return true;
            }
        } else if (dif < 0) {
            return false;
        } else {
            pos = ld_rlx(&P.q->tail);
        }
    }
}

// Push a FRAME task (branch variable x with the remaining values vals over the
// parent snapshot snap, which is nw words in LDS or global memory).
template <int WM>
DEV bool push_frame(const SearchParams &P, int inst, int x, int depth, const uint32_t (&vals)[WM],
                    const uint32_t *snap, int nw, int lane, int side = 0) {
    uint32_t cell = 0, pos = 0;
    int ok = 0;
    if (lane == 0) {
        add_i(&P.g->pending, 1);
        ok = q_reserve(P, &cell, &pos) ? 1 : 0;
        if (!ok) add_i(&P.g->pending, -1);
        // the instance's live tasks count it before it is published
        if (ok && P.nrings > 1) add_i(&P.ctl[inst].live, 1);
    }
    ok = uni(ok);
    if (!ok) return false;
    cell = uniu(cell);
    pos = uniu(pos);
    uint32_t *s = P.qdata + (size_t)cell * P.slot_words;
    if (lane < SLOT_HDR) {  // header word `lane`
        uint32_t h = 0u;
        if (lane == 0) h = (uint32_t)inst;
        if (lane == 1) h = (uint32_t)K_FRAME;
        if (lane == 2) h = (uint32_t)x;
        if (lane == 3) h = (uint32_t)depth;
        if (lane == 12) h = (uint32_t)side;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (lane == 4 + k) h = vals[k];
        st_rlx(s + lane, h);
    }
    for (int t = lane; t < nw; t += 64) st_rlx(s + SLOT_HDR + t, snap[t]);
    slot_stores_done();
    if (lane == 0) st_rlx(&P.qseq[cell], pos + 1u);
    return true;
}

// ------------------------------------------------------------- worker

template <int WM>
struct Frame {  // cached top-of-trail frame
    int x, depth;
    int side;       // 2-way branching: 0 = next child x = min v, 1 = next child x in v
    uint32_t v[WM];
};

// A push beyond the trail's frames: stop the launch with an internal error
// (the host sizes the trail for the deepest path, so this never fires).
DEV bool trail_full(const SearchParams &P, int sp, int lane) {
    if (sp < P.max_frames) return false;
    if (lane == 0) stop_launch(P, 4);
    return true;
}

template <int WM>
DEV void frame_store_meta(uint32_t *f, const Frame<WM> &F, int lane) {
    if (lane == 0) {
        f[0] = (uint32_t)F.x;
        f[1] = (uint32_t)F.depth;
        f[2] = 0u;  // flags: bit 0 = part of the subtree left this worker
        f[3] = (uint32_t)F.side;
    }
    if (lane < WM) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k == lane) v = F.v[k];
        f[4 + lane] = v;
    }
}
template <int WM>
DEV void frame_load_meta(const uint32_t *f, Frame<WM> &F) {
    F.x = uni((int)f[0]);
    F.depth = uni((int)f[1]);
    F.side = uni((int)f[3]);
#pragma unroll
    for (int k = 0; k < WM; ++k) F.v[k] = uniu(f[4 + k]);
}

template <int WM>
DEV void record_solution(const SearchParams &P, const InstDev &I, InstCtl *ctl, const Lds &L,
                         Counters &C, int lane) {
    const int n = I.n, W = I.W;
    if (P.mode == 0) {  // FIRST: one winner stores its assignment
        int won = 0;
        if (lane == 0) won = cas_i(&ctl->found, 0, 1) ? 1 : 0;
        won = uni(won);
        if (won) {
            if (I.sol_buf && I.sol_cap > 0)
                for (int i = lane; i < n; i += 64) {
                    uint32_t d[WM];
#pragma unroll
                    for (int k = 0; k < WM; ++k) d[k] = k < W ? L.dom[i * W + k] : 0u;
                    I.sol_buf[i] = I.lo[i] + low_w(d, W);
                }
            fence_rel();
            if (lane == 0) {
                add_u64(&ctl->count, 1ull);
                ctl->reason = 1;
                st_rel_i(&ctl->done, 1);
                signal_rings(P, SIG_DONE);
            }
        }
        return;
    }
    const bool store = I.sol_buf && I.sol_cap > 0;
    if (store || I.max_solutions) {
        u64 slot = 0;
        if (lane == 0) slot = add_u64(&ctl->n_slots, 1ull);
        slot = uni64(slot);
        if (store && slot < I.sol_cap) {
            int32_t *row = I.sol_buf + slot * (u64)n;
            for (int i = lane; i < n; i += 64) {
                uint32_t d[WM];
#pragma unroll
                for (int k = 0; k < WM; ++k) d[k] = k < W ? L.dom[i * W + k] : 0u;
                row[i] = I.lo[i] + low_w(d, W);
            }
        }
        if (I.max_solutions && slot + 1 >= I.max_solutions && lane == 0) {
            ctl->reason = 3;
            st_rel_i(&ctl->done, 1);
            signal_rings(P, SIG_DONE);
        }
    } else {
        C.sols += 1;
    }
}

// Fold the VAR layout's 32-bit per-lane counters into rev / bytes (done at
// every poll, so they stay far below 2^32: at most 64 * 32 + 1 dirty-variable
// steps per node, each one revision per lane of at most 32 popcount).
DEV void fold_var(Counters &C) {
    C.rev += C.vrev;
    C.bytes += 8ull * C.vrev + 4ull * C.vchg + 4ull * C.vpop;
    C.vrev = C.vchg = C.vpop = 0u;
}

template <int WM>
DEV void flush(InstCtl *ctl, Counters &C, int lane) {
    fold_var(C);
    const u64 rev = wave_sumu64(C.rev), bytes = wave_sumu64(C.bytes) + C.ubytes;
    if (lane == 0) {
        if (C.nodes) add_u64(&ctl->nodes, C.nodes);
        if (C.fails) add_u64(&ctl->fails, C.fails);
        if (C.sols) add_u64(&ctl->count, C.sols);
        if (C.steals) add_u64(&ctl->steals, C.steals);
        if (C.tasks) add_u64(&ctl->tasks, C.tasks);
        if (rev) add_u64(&ctl->revisions, rev);
        if (bytes) add_u64(&ctl->alg_bytes, bytes);
    }
    C.nodes = C.fails = C.sols = C.steals = C.tasks = 0;
    C.rev = C.bytes = C.ubytes = 0;
}

// Nodes between checks of stop flags and donation requests.  Each check may
// donate a frame; in the register layout, where a node costs a fraction of a
// microsecond, checking every 128 nodes split a search's tail into so many
// small tasks that it ran for longer than the rest of the search (RB n=40
// d=16 slice x0=1 with 6144 workers: 19 s at 128, 7.5 s at 512, 3.6 s at
// 2048; checking after 128 nodes and then at doubling intervals brought the
// small tasks back: 19 s).  The LDS layouts keep 128: their many-instance and
// small searches need the faster spreading (13-queens: 20 ms at 128, 66 ms at
// 512).
constexpr int POLL = 128;
constexpr int POLL_VAR = 2048;
// The LDS layouts also poll once POLL_TICKS of wall clock (100 MHz ticks)
// have passed since the last poll, after at least POLL_MIN nodes, and under
// a node budget they count their nodes against it every ACCT_TICKS: when a
// node takes a hundred microseconds (instances of a hundred variables and
// thousands of table revisions per node), 128 nodes are tens of
// milliseconds, during which idle workers wait for a donation, and an
// instance shared by dozens of workers runs thousands of nodes past its
// budget.  (A clock-based poll every 50 us made the fast nodes of small
// count searches donate so often that their tails split into tiny tasks:
// 200 instances of 12-18 variables took 4.7 s instead of 0.6 s.)
constexpr int POLL_MIN = 8;
constexpr long long POLL_TICKS = 100000;
constexpr long long ACCT_TICKS = 5000;


// ------------------------------------------------------ branching policy

// Feature k (0..4) of variable i at a node of depth `depth`: domain fraction,
// static degree / (n-1), mean static tightness, depth / n, log2(1 + fails).
// fs: the instance's static features [n][4] (global or an LDS copy).
DEV float var_feature(const InstDev &I, const float *fs, int i, int k, int depth, int pop, uint32_t fails) {
    switch (k) {
    case 0: return (float)pop * fs[4 * i + 2];
    case 1: return fs[4 * i + 0];
    case 2: return fs[4 * i + 1];
    case 3: return (float)depth / (float)(I.n > 0 ? I.n : 1);
    default: return log2f(1.f + (float)fails);
    }
}

template <int WM>
DEV int var_pop(const InstDev &I, const Lds &L, int i) {
    int p = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k)
        if (k < I.W) p += __popc(L.dom[i * I.W + k]);
    return p;
}

DEV u64 wave_min64(u64 v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const u64 w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

DEV u64 mix64(u64 z) {  // SplitMix64 finalizer (Steele, Lea and Flood 2014)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Learned choice: the candidate (two or more values) with the smallest
// predicted log-size of its subtree; lowest index on ties.  Candidates are
// scored 16 at a time by the MFMA network.
// pol: the network's LDS copy (staged once per workgroup).
template <int WM>
DEV int choose_learned(const PolicyDev &pol, const InstDev &I, const Lds &L, int depth, int lane, int fallback) {
    const int n = I.n;
    const int row = lane & 15, kq = lane >> 4;
    u64 best = ~0ull;
    for (int base = 0; base < n; base += 16) {
        const int i = base + row;
        bf16x4 xT;
        int pop = 0;
        if (i < n) pop = var_pop<WM>(I, L, i);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * kq + j;
            const float f = (i < n && k < POLICY_F) ? var_feature(I, L.feat, i, k, depth, pop, L.fails[i]) : 0.f;
            xT[j] = (short)f2bf(f);
        }
        const f32x4 acc = mlp_tile<true>(pol, xT, lane, nullptr);
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ii = base + 4 * kq + r;
                if (ii < n && var_pop<WM>(I, L, ii) >= 2) {
                    const float y = acc[r] + *pol.b2;
                    const uint32_t u = __float_as_uint(y);
                    const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
                    const u64 key = ((u64)ord << 32) | (u64)ii;
                    best = key < best ? key : best;
                }
            }
        }
    }
    best = wave_min64(best);
    return best == ~0ull ? fallback : (int)(best & 0xFFFFFFFFull);
}

// ------------------------------------------------------- value ordering

// Features of value a of variable x (a live value; lane-parallel over a) at a
// node whose domains are dom ([n][W] words) and whose unit ranges are
// [beg, end) for x, at depth `depth`:
//   g0 = a / d_x (the value's place in the domain),
//   g1 = mean over x's table constraints of the fraction of the other
//        variable's current values that x = a supports (1 without tables),
//   g2 = the smallest of those fractions (1 without tables),
//   g3 = depth / n,
//   g4 = |D_x| / d_x.
// The rows read are those of x's value a in each table (bits over the other
// variable).
template <int WM, bool GM>
DEV void value_features(const InstDev &I, const uint32_t *dom, int beg, int end, int x, int a, int depth,
                        float (&g)[POLICY_F]) {
    const int W = I.W;
    const float inv_d = I.feat_static[4 * x + 2];
    int px = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k)
        if (k < W) px += __popc(dom[x * W + k]);
    float sum = 0.f, mn = 1.f;
    int cnt = 0;
    for (int i = beg; i < end; ++i) {
        const Unit u = ld_unit<GM>(I.units, (uint32_t)i);
        if ((u.tt >> 24) != U_TABLE) continue;
        const int t = u.tt & 0xFFFFFF;
        int pt = 0, hit = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k) {
            if (k < W) {
                const uint32_t dt = dom[t * W + k];
                pt += __popc(dt);
                hit += __popc(dt & ldg<GM>(I.rows, (uint32_t)u.p1 + (uint32_t)a * (uint32_t)W + (uint32_t)k));
            }
        }
        if (pt == 0) continue;
        const float fr = (float)hit / (float)pt;
        sum += fr;
        mn = fr < mn ? fr : mn;
        ++cnt;
    }
    g[0] = (float)a * inv_d;
    g[1] = cnt ? sum / (float)cnt : 1.f;
    g[2] = cnt ? mn : 1.f;
    g[3] = (float)depth / (float)(I.n > 0 ? I.n : 1);
    g[4] = (float)px * inv_d;
}

// Order-preserving key of a float (larger float -> larger key).
DEV uint32_t float_key(float y) {
    const uint32_t u = __float_as_uint(y);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Scores of the live values of x at the node in L.dom (domains of at most
// 64 values: lane a <-> value a): the value network on the value features,
// 16 values per MFMA tile.  Returns this lane's score (lanes of values not
// in D_x: the lowest key).
template <int WM, bool GM>
DEV uint32_t value_scores(const PolicyDev &VP, const InstDev &I, const Lds &L, int x, int depth, int lane) {
    const int W = I.W;
    float *ft = L.vscr;                          // [64][5]
    float *sc = L.vscr + VALUE_MAX * POLICY_F;   // [64]
    const int beg = uni(L.trig[x]), end = uni(L.trig[x + 1]);
    const int a = lane;
    const bool live = a < 32 * W && ((L.dom[x * W + (a >> 5)] >> (a & 31)) & 1u);
    float g[POLICY_F] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) value_features<WM, GM>(I, L.dom, beg, end, x, a, depth, g);
#pragma unroll
    for (int k = 0; k < POLICY_F; ++k) ft[a * POLICY_F + k] = g[k];
    wsync();
    const int row = lane & 15, kq = lane >> 4;
    for (int base = 0; base < 32 * W; base += 16) {
        bf16x4 xT;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * kq + j;
            xT[j] = (short)f2bf(k < POLICY_F ? ft[(base + row) * POLICY_F + k] : 0.f);
        }
        const f32x4 acc = mlp_tile<true>(VP, xT, lane, nullptr);
        if (row == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sc[base + 4 * kq + r] = acc[r] + *VP.b2;
        }
    }
    wsync();
    return live ? float_key(sc[a]) : 0u;
}

// The next child of a d-way branching under the learned value order: the
// remaining value (bit set in v) with the highest score, lowest value on
// ties.  key: this lane's score key (lane = value).
template <int WM>
DEV int pick_value(const uint32_t (&v)[WM], uint32_t key, int lane) {
    bool avail = false;
#pragma unroll
    for (int k = 0; k < WM; ++k) avail |= (k == (lane >> 5)) && ((v[k] >> (lane & 31)) & 1u);
    const u64 m = avail ? (((u64)(~key) << 32) | (u64)lane) : ~0ull;
    return (int)(wave_min64(m) & 0xFFFFFFFFull);
}

// Exploration for trace collection: a uniform pick among the (up to) 4
// candidates with the smallest domains (ties by index).
template <int WM>
DEV int choose_explore(const InstDev &I, const Lds &L, int lane, u64 rnd) {
    uint32_t keys[4];
    int cnt = 0;
    uint32_t prev = 0;
    for (int q = 0; q < 4; ++q) {
        uint32_t key = 0xFFFFFFFFu;
        for (int i = lane; i < I.n; i += 64) {
            const int p = var_pop<WM>(I, L, i);
            if (p >= 2) {
                const uint32_t kk = ((uint32_t)p << 16) | (uint32_t)i;
                if ((q == 0 || kk > prev) && kk < key) key = kk;
            }
        }
        key = wave_min(key);
        if (key == 0xFFFFFFFFu) break;
        keys[q] = key;
        prev = key;
        ++cnt;
    }
    const int pick = (int)(rnd % (u64)(cnt > 0 ? cnt : 1));
    uint32_t kpick = keys[0];
#pragma unroll
    for (int q = 1; q < 4; ++q)
        if (q == pick) kpick = keys[q];
    return (int)(kpick & 0xFFFFu);
}

// Run one task to completion.  FEAT: 0 plain first-fail, 1 learned policy,
// 2 trace recording (each compiled separately to keep the plain kernel's
// register budget).
template <int WM, int FEAT, bool GLOB, bool SEGC, bool GM>
DEV void run_task(const SearchParams &P, const InstDev &I, InstCtl *ctl, int b, int kind,
                  Frame<WM> F0, const Lds &L, uint32_t *trail, Counters &C, int lane,
                  long long t_start, const PolicyDev &LP, const PolicyDev &VP) {
    const int n = I.n, W = I.W, nw = n * W;
    const int layout = P.layout;
    const uint32_t FW = P.frame_words;
    int sp = 0;
    Frame<WM> F;
    bool have_open = false, need_restore = false;
    // register copy of the top frame's snapshot (lane-per-word), so that the
    // siblings under one frame are restored without an HBM round trip
    constexpr int NC = WM <= 2 ? 4 : 1;
    const bool cache_ok = WM <= 2 && nw <= 64 * NC;
    uint32_t snapc[NC];
    bool snap_valid = false;
    int depth = F0.depth;
    int since_poll = 0, polls = 0;
    // clock of the task's last poll (a task starts as if it had just polled)
    long long last_poll = (long long)wall_clock64(), last_acct = last_poll;
    int open_x = 0;
    const bool tracing = FEAT == 2 && P.trace_out != nullptr;
    const bool learned = FEAT == 1 && P.branching == 1;
    // learned value order (d-way): the value network's score keys of the top
    // frame's values (lane = value); each frame keeps its own in its last
    // FRAME_SCORES words
    const bool vorder = FEAT == 1 && P.value_order != 0;
    const uint32_t FS = P.frame_words - FRAME_SCORES;
    uint32_t vkey = 0u;
    if (tracing || learned) {
        for (int i = lane; i < n; i += 64) L.fails[i] = 0u;
        if (learned)
            for (int t = lane; t < 4 * n; t += 64) L.feat[t] = I.feat_static[t];
        wsync();
    }

    if (kind == K_ROOT) {
        // unary constraints restrict the root domains
        for (int t = lane; t < I.n_unary; t += 64) {
            const int v = I.unary[2 * t], off = I.unary[2 * t + 1];
            for (int k = 0; k < W; ++k) atomicAnd(&L.dom[v * W + k], I.rows[off + k]);
        }
        wsync();
        C.nodes += 1;
        C.stamp += 1;
        int bx = 0;
        int st = node_test<WM>(I, L, lane, &bx);
        if (st == 2) { C.fails += 1; return; }
        dirty_all(L, n, lane);
        if (propagate<WM, GLOB, SEGC, GM>(I, L, layout, C, lane)) { C.fails += 1; return; }
        st = node_test<WM>(I, L, lane, &bx);
        if (st == 1) { record_solution<WM>(P, I, ctl, L, C, lane); return; }
        have_open = true;
        open_x = bx;
        depth = 0;
    } else {
        // FRAME task: the snapshot is in L.dom; it becomes trail frame 0
        F = F0;
        for (int t = lane; t < nw; t += 64) trail[FRAME_HDR + t] = L.dom[t];
        if (cache_ok) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (lane + 64 * c < nw) snapc[c] = L.dom[lane + 64 * c];
            snap_valid = true;
        }
        frame_store_meta<WM>(trail, F, lane);
        if (vorder) {
            // the donated frame's node is in L.dom: score its values again
            vkey = value_scores<WM, GM>(VP, I, L, F.x, F.depth, lane);
            trail[FS + lane] = vkey;
        }
        sp = 1;
        need_restore = false;
    }

    for (;;) {
        if (have_open) {
            have_open = false;
            int x = open_x;
            if (tracing && P.explore_pm > 0) {
                const u64 rnd = mix64(((u64)P.seed << 40) ^ ((u64)(blockIdx.x * 16 + (threadIdx.x >> 6)) << 24) ^ C.stamp);
                if ((int)(rnd % 1000ull) < P.explore_pm) x = choose_explore<WM>(I, L, lane, rnd >> 20);
            } else if (learned) {
                x = choose_learned<WM>(LP, I, L, depth, lane, open_x);
            }
            // eager split: hand every child to the queue while the split target is unmet
            bool split = false;
            if (P.split_target > 0) {
                long long prod = 0;
                if (lane == 0) prod = (long long)ld_rlx_u64(&P.g->produced);
                prod = unill(prod);
                if (prod < P.split_target) split = true;
            }
            uint32_t dx[WM];
#pragma unroll
            for (int k = 0; k < WM; ++k) dx[k] = k < W ? uniu(L.dom[x * W + k]) : 0u;
            int side0 = 0;
            if (split) {
                // one FRAME task per child of x, each over this node's domains
                // (d-way: one per value; 2-way: x = min, then x in the rest)
                uint32_t rem[WM];
#pragma unroll
                for (int k = 0; k < WM; ++k) rem[k] = dx[k];
                int pushed = 0;
                if (P.two_way) {
                    int lowk = 0;
#pragma unroll
                    for (int k = WM - 1; k >= 0; --k)
                        if (rem[k]) lowk = k;
                    uint32_t one[WM];
#pragma unroll
                    for (int q = 0; q < WM; ++q) one[q] = q == lowk ? (rem[q] & (0u - rem[q])) : 0u;
                    if (push_frame<WM>(P, b, x, depth, one, L.dom, nw, lane, 0)) {
#pragma unroll
                        for (int q = 0; q < WM; ++q) rem[q] &= ~one[q];
                        ++pushed;
                        side0 = 1;
                        if (push_frame<WM>(P, b, x, depth, rem, L.dom, nw, lane, 1)) {
#pragma unroll
                            for (int q = 0; q < WM; ++q) rem[q] = 0u;
                            ++pushed;
                        }
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < WM; ++k) {
                        while (rem[k]) {
                            const uint32_t lowb = rem[k] & (0u - rem[k]);
                            uint32_t one[WM];
#pragma unroll
                            for (int q = 0; q < WM; ++q) one[q] = q == k ? lowb : 0u;
                            if (!push_frame<WM>(P, b, x, depth, one, L.dom, nw, lane)) break;
                            rem[k] &= ~lowb;
                            ++pushed;
                        }
                    }
                }
                if (lane == 0 && pushed) add_u64(&P.g->produced, (u64)pushed);
                if (tracing && pushed)
                    for (int t = lane; t < sp; t += 64) trail[(size_t)t * FW + 2] = 1u;
                bool left = false;
#pragma unroll
                for (int k = 0; k < WM; ++k) left |= rem[k] != 0u;
                if (!left) goto next_child;
#pragma unroll
                for (int k = 0; k < WM; ++k) dx[k] = rem[k];
            }
            // push a trail frame: snapshot of this node, branch variable x
            {
                if (trail_full(P, sp, lane)) return;
                if (sp > 0 && lane < WM) {
                    // the outgoing top frame keeps its remaining values in HBM
                    uint32_t v = 0;
#pragma unroll
                    for (int k = 0; k < WM; ++k)
                        if (k == lane) v = F.v[k];
                    trail[(size_t)(sp - 1) * FW + 4 + lane] = v;
                }
                if (sp > 0 && lane == 63) trail[(size_t)(sp - 1) * FW + 3] = (uint32_t)F.side;
                uint32_t *f = trail + (size_t)sp * FW;
                for (int t = lane; t < nw; t += 64) f[FRAME_HDR + t] = L.dom[t];
                if (cache_ok) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (lane + 64 * c < nw) snapc[c] = L.dom[lane + 64 * c];
                    snap_valid = true;
                }
                C.ubytes += 4ull * nw;
                F.x = x;
                F.depth = depth;
                F.side = side0;
#pragma unroll
                for (int k = 0; k < WM; ++k) F.v[k] = dx[k];
                frame_store_meta<WM>(f, F, lane);
                if (vorder) {
                    vkey = value_scores<WM, GM>(VP, I, L, x, depth, lane);
                    f[FS + lane] = vkey;
                }
                if (tracing) {
                    const int px = var_pop<WM>(I, L, x);
                    if (lane < POLICY_F) ((float *)f)[16 + lane] = var_feature(I, I.feat_static, x, lane, depth, px, L.fails[x]);
                    if (lane == 0) {
                        f[24] = (uint32_t)C.stamp;
                        f[25] = (uint32_t)(C.stamp >> 32);
                    }
                }
                ++sp;
                need_restore = false;
            }
        }
    next_child:
        // take the next value of the top frame, popping exhausted frames
        for (;;) {
            if (sp == 0) return;
            bool emptyv = true;
#pragma unroll
            for (int k = 0; k < WM; ++k) emptyv &= F.v[k] == 0u;
            if (emptyv) {
                if (tracing) {
                    // the frame's subtree is complete: record (features, log2(1 + nodes below))
                    const uint32_t *f = trail + (size_t)(sp - 1) * FW;
                    const uint32_t flags = uniu(f[2]);
                    const int fdepth = uni((int)f[1]);
                    if (flags == 0u) {
                        const u64 st0 = ((u64)uniu(f[25]) << 32) | uniu(f[24]);
                        u64 idx = 0;
                        if (lane == 0) idx = add_u64((u64 *)P.trace_count, 1ull);
                        idx = uni64(idx);
                        if (idx < P.trace_cap && lane < TRACE_WORDS) {
                            float v = 0.f;
                            if (lane < POLICY_F) v = ((const float *)f)[16 + lane];
                            else if (lane == 5) v = (float)fdepth;
                            else if (lane == 6) v = (float)b;
                            else if (lane == 7) v = log2f(1.f + (float)(C.stamp - st0));
                            P.trace_out[idx * TRACE_WORDS + lane] = v;
                        }
                    }
                }
                --sp;
                if (sp > 0) {
                    frame_load_meta<WM>(trail + (size_t)(sp - 1) * FW, F);
                    if (vorder) vkey = trail[(size_t)(sp - 1) * FW + FS + lane];
                }
                need_restore = true;
                snap_valid = false;
                continue;
            }
            break;
        }
        {
            // the child's domain of x: the smallest remaining value, or (2-way,
            // second child) all the remaining values
            uint32_t cv[WM];
            if (P.two_way && F.side) {
#pragma unroll
                for (int k = 0; k < WM; ++k) {
                    cv[k] = F.v[k];
                    F.v[k] = 0u;
                }
            } else {
                int vi = -1;
                if (vorder) {
                    vi = pick_value<WM>(F.v, vkey, lane);
                } else {
#pragma unroll
                    for (int k = WM - 1; k >= 0; --k)
                        if (F.v[k]) vi = 32 * k + __ffs(F.v[k]) - 1;
                }
#pragma unroll
                for (int k = 0; k < WM; ++k) {
                    cv[k] = bit_in_word(vi, k);
                    F.v[k] &= ~cv[k];
                }
                if (P.two_way) F.side = 1;
            }
            const uint32_t *f = trail + (size_t)(sp - 1) * FW;
            if (need_restore) {
                if (snap_valid) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (lane + 64 * c < nw) L.dom[lane + 64 * c] = snapc[c];
                } else if (cache_ok) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (lane + 64 * c < nw) {
                            snapc[c] = f[FRAME_HDR + lane + 64 * c];
                            L.dom[lane + 64 * c] = snapc[c];
                        }
                    snap_valid = true;
                } else {
                    for (int t = lane; t < nw; t += 64) L.dom[t] = f[FRAME_HDR + t];
                }
                C.ubytes += 4ull * nw;
                wsync();
            }
            need_restore = true;
            if (lane < W) {
                uint32_t w = 0u;
#pragma unroll
                for (int k = 0; k < WM; ++k)
                    if (k == lane) w = cv[k];
                L.dom[F.x * W + lane] = w;
            }
            depth = F.depth + 1;
            dirty_one(L, n, F.x, lane);
        }
        C.nodes += 1;
        C.stamp += 1;
        {
            const bool failed = propagate<WM, GLOB, SEGC, GM>(I, L, layout, C, lane);
            if (failed) {
                C.fails += 1;
                if ((tracing || learned) && lane == 0) L.fails[F.x] += 1u;
            } else {
                int bx = 0;
                const int st = node_test<WM>(I, L, lane, &bx);
                if (st == 1) {
                    record_solution<WM>(P, I, ctl, L, C, lane);
                    if (P.mode == 0) return;  // first mode: one solution ends the instance
                } else {
                    have_open = true;
                    open_x = bx;
                }
            }
        }
        // periodic checks: stop flags and the node budget (every POLL nodes,
        // and under a budget also every POLL_TICKS), then the clock, the
        // cancel flag and donation (every POLL nodes only: donating more
        // often splits a search's tail into too many small tasks)
        ++since_poll;
        bool due = since_poll >= POLL, acct = due;
        if (!due && since_poll >= POLL_MIN) {
            const long long now = (long long)wall_clock64();
            due = now - last_poll >= POLL_TICKS;
            acct = due || (I.max_nodes && now - last_acct >= ACCT_TICKS);
        }
        if (acct) {
            const long long now = (long long)wall_clock64();
            last_acct = now;
            if (due) last_poll = now;
            // one shared word per poll; stop, done and queue words only when
            // it says so
            int stop = 0, want = 0;
            if (lane == 0) {
                const uint32_t sig = ld_rlx(&P.q->signal);
                stop = (sig & SIG_STOP) ? 1 : ((sig & SIG_DONE) ? ld_rlx_i(&ctl->done) : 0);
                // donate while fewer tasks wait unclaimed than waves are idle
                // (a negative difference: tickets waiting for a task)
                const int idle = (int)(sig & SIG_IDLE_MASK);
                if (due && P.donate && idle > 0)
                    want = (int)(ld_rlx(&P.q->tail) - ld_rlx(&P.q->head)) < idle;
            }
            stop = uni(stop);
            if (stop) return;
            if (I.max_nodes) {
                u64 tot = 0;
                if (lane == 0) tot = add_u64(&ctl->nodes, C.nodes) + C.nodes;
                tot = uni64(tot);
                C.nodes = 0;
                if (tot >= I.max_nodes) {
                    if (lane == 0) { ctl->reason = 2; st_rel_i(&ctl->done, 1); signal_rings(P, SIG_DONE); }
                    return;
                }
            }
            if (due) {
            since_poll = 0;
            // the clock and the host's cancel flag (a read over PCIe) every
            // 16th poll
            if ((P.time_ticks || P.cancel) && (++polls & 15) == 0) {
                int st2 = 0;
                if (lane == 0) {
                    if (P.time_ticks && (long long)wall_clock64() - t_start > P.time_ticks) st2 = 2;
                    if (P.cancel && *P.cancel) st2 = 3;
                    if (st2) stop_launch(P, st2);
                }
                if (uni(st2)) return;
            }
            if (uni(want) && sp > 0) {
                // donate the shallowest frame that still has untried values
                int tsel = -1;
                // (frames below the top keep their values in HBM; the top's are in F)
                bool topnz = false;
#pragma unroll
                for (int k = 0; k < WM; ++k) topnz |= F.v[k] != 0u;
                for (int base = 0; base < sp - 1 && tsel < 0; base += 64) {
                    const int t = base + lane;
                    bool nz = false;
                    if (t < sp - 1) {
                        const uint32_t *f = trail + (size_t)t * FW;
                        for (int k = 0; k < W; ++k) nz |= f[4 + k] != 0u;
                    }
                    const u64 m = __ballot(nz);
                    if (m) tsel = base + __ffsll((long long)m) - 1;
                }
                if (tsel < 0 && topnz) tsel = sp - 1;
                if (tsel >= 0) {
                    uint32_t *f = trail + (size_t)tsel * FW;
                    Frame<WM> D;
                    frame_load_meta<WM>(f, D);
                    if (tsel == sp - 1) D = F;
                    if (push_frame<WM>(P, b, D.x, D.depth, D.v, f + FRAME_HDR, nw, lane, D.side)) {
                        if (lane < WM) f[4 + lane] = 0u;
                        if (tracing)
                            for (int t = lane; t <= tsel; t += 64) trail[(size_t)t * FW + 2] = 1u;
                        if (tsel == sp - 1) {
#pragma unroll
                            for (int k = 0; k < WM; ++k) F.v[k] = 0u;
                        }
                        C.steals += 1;
                    }
                }
            }
            }  // due
        }
    }
}


// ------------------------------------------------- VAR layout (n <= 64, W = 1)
//
// One lane per variable: lane i keeps D_i in a register for the whole node.
// A dirty variable j is broadcast with readlane, and every lane t that shares
// a constraint with j revises its own domain against D_j in the same
// instruction (its unit is the dense pair entry [j][t]).  Changes update the
// register at once and feed the next dirty set through a ballot, so a node
// needs no LDS traffic for domains or dirty sets.

// Pair entries (one 32-bit word): type in bits 28..31, parameter in bits
// 0..27 (signed); QUEENS packs k in bits 15..27 and the signed offset
// lo_src - lo_tgt in bits 0..14.
DEV int pair_type(uint32_t e) { return (int)(e >> 28); }
DEV int pair_param(uint32_t e) { return (int)(e << 4) >> 4; }
DEV int pair_qk(uint32_t e) { return (int)((e >> 15) & 0x1FFFu); }
DEV int pair_qdl(uint32_t e) { return (int)(e << 17) >> 17; }

// Support union of the rows of the source values in dj (uniform across the
// wave), four values per step with four row loads in flight.  s_ff1 finds the
// lowest remaining value and s_bitset0 clears it: two scalar instructions per
// value, where the scalar unit is what bounds this layout.  Past the last value
// s_ff1 gives -1 (and s_bitset0 of bit 31 leaves an empty set empty); row -1
// is the zero word the packer puts before every row block.
DEV uint32_t table_union(const uint32_t *rows, uint32_t dj) {
    uint32_t acc = 0u, bits = dj;
    while (bits) {
        int a, b, c, e;
        asm("s_ff1_i32_b32 %0, %1\n\ts_bitset0_b32 %1, %0" : "=&s"(a), "+s"(bits));
        asm("s_ff1_i32_b32 %0, %1\n\ts_bitset0_b32 %1, %0" : "=&s"(b), "+s"(bits));
        asm("s_ff1_i32_b32 %0, %1\n\ts_bitset0_b32 %1, %0" : "=&s"(c), "+s"(bits));
        asm("s_ff1_i32_b32 %0, %1\n\ts_bitset0_b32 %1, %0" : "=&s"(e), "+s"(bits));
        acc |= rows[a] | rows[b] | rows[c] | rows[e];
    }
    return acc;
}

// Revision of target lane t against the broadcast source domain dj (packed
// pair entry e); generic over the unit types.
DEV uint32_t revise_var_generic(const InstDev &I, uint32_t e, uint32_t d, uint32_t dj) {
    const int ty = pair_type(e);
    if (ty == U_TABLE) {
        return d & table_union(I.rows + pair_param(e), dj);
    } else if (ty == U_NEQ) {
        return __popc(dj) == 1 ? d & ~bit_in_word(__ffs(dj) - 1 + pair_param(e), 0) : d;
    } else if (ty == U_LT_UB) {
        return d & mask_le(31 - __clz(dj) + pair_param(e) - 1, 0);
    } else if (ty == U_LT_LB) {
        return d & mask_ge(__ffs(dj) - 1 - pair_param(e) + 1, 0);
    } else if (ty == U_QUEENS) {
        if (__popc(dj) > 3) return d;
        const int kq = pair_qk(e);
        const int dl = pair_qdl(e);
        uint32_t uns = 0xFFFFFFFFu, bits = dj;
        while (bits) {
            const int b = __ffs(bits) - 1 + dl;
            bits &= bits - 1;
            uns &= bit_in_word(b, 0) | bit_in_word(b + kq, 0) | bit_in_word(b - kq, 0);
        }
        return d & ~uns;
    }
    return d;
}

// TYPES: 0 generic, 1 table units only, 2 queens units only (uniform choice).
// The pair matrix has a row stride of 64, so every lane loads its entry
// (lanes >= n read empty entries and hold empty domains).
template <int TYPES>
DEV bool propagate_var_t(const InstDev &I, uint32_t &d, u64 cur, Counters &C, int lane) {
    const int n = I.n;
    const u64 live = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    while (cur) {
        u64 nxt = 0;
        int j = __ffsll((long long)cur) - 1;
        uint32_t e = I.pairs[j * 64 + lane];
        while (cur) {
            cur &= cur - 1;
            // prefetch the pair entry of the next dirty variable
            const int jn = cur ? __ffsll((long long)cur) - 1 : j;
            const uint32_t en = I.pairs[jn * 64 + lane];
            const uint32_t dj = (uint32_t)__builtin_amdgcn_readlane((int)d, j);
            uint32_t nd = d;
            if (TYPES == 1) {
                // every lane revises, without a branch on the lanes: a lane
                // with no constraint to j (e == 0) reads the all-ones rows at
                // offset 0 and keeps its domain
                nd = d & table_union(I.rows + pair_param(e), dj);
                const uint32_t real = e != 0u ? 1u : 0u;
                // the revision reads one row per value of the source
                C.vpop += real * (uint32_t)__popc(dj);
                C.vrev += real;
                C.vchg += nd != d ? 1u : 0u;
            } else if (e != 0u) {
                if (TYPES == 2) {
                    if (__popc(dj) <= 3) {
                        const int kq = pair_qk(e);
                        const int dl = pair_qdl(e);
                        uint32_t uns = 0xFFFFFFFFu, bits = dj;
                        while (bits) {
                            const int b = __ffs(bits) - 1 + dl;
                            bits &= bits - 1;
                            uns &= bit_in_word(b, 0) | bit_in_word(b + kq, 0) | bit_in_word(b - kq, 0);
                        }
                        nd = d & ~uns;
                    }
                } else {
                    nd = revise_var_generic(I, e, d, dj);
                    if (pair_type(e) == U_TABLE) C.vpop += __popc(dj);
                }
                C.vrev += 1u;
                C.vchg += nd != d ? 1u : 0u;
            }
            const u64 chm = __ballot(nd != d);
            d = nd;
            if (chm) {
                if (__ballot(nd == 0u) & live) return true;
                nxt |= chm;
            }
            j = jn;
            e = en;
        }
        cur = nxt;
    }
    return false;
}

DEV bool propagate_var(const InstDev &I, uint32_t &d, u64 cur, Counters &C, int lane) {
    if (I.unit_types == (1 << U_TABLE)) return propagate_var_t<1>(I, d, cur, C, lane);
    if (I.unit_types == (1 << U_QUEENS)) return propagate_var_t<2>(I, d, cur, C, lane);
    return propagate_var_t<0>(I, d, cur, C, lane);
}

// first-fail over the register domains: 0 open (*bx), 1 solution, 2 failed
DEV int node_test_var(int n, uint32_t d, int lane, int *bx) {
    const int pop = __popc(d);  // 0 on lanes >= n
    const u64 live = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    if (__ballot(pop == 0) & live) return 2;
    const u64 open = __ballot(pop >= 2);
    if (!open) return 1;
    for (int p = 2; p <= 32; ++p) {
        const u64 m = __ballot(pop == p);
        if (m) {
            *bx = __ffsll((long long)m) - 1;
            return 0;
        }
    }
    return 1;
}

// The trail of the VAR layout: every frame's domain snapshot (one word per
// lane) goes to HBM, but the frames' branching variable, depth and untried
// values stay in registers, frame f on lane f (at most n <= 64 frames: the
// variables branched on along a path are distinct).  Exhausted frames are
// popped without a memory access; the snapshot of the frame below the top
// is prefetched into a register, so that returning one level needs no wait.
template <int WM>
DEV void run_task_var(const SearchParams &P, const InstDev &I, InstCtl *ctl, int b, int kind,
                      Frame<WM> F0, const Lds &L, uint32_t *trail, Counters &C, int lane,
                      long long t_start) {
    const int n = I.n;
    const uint32_t FW = P.frame_words;
    int sp = 0;
    Frame<WM> F;  // the top frame (sp - 1)
    bool have_open = false, need_restore = false;
    int depth = F0.depth;
    int since_poll = 0, polls = 0;
    // a node budget is checked at every poll: keep it as fine as in the LDS
    // layouts when there is one
    const int poll_iv = I.max_nodes ? POLL : POLL_VAR;
    int open_x = 0;
    uint32_t d = lane < n ? L.dom[lane] : 0u;
    uint32_t snapc = 0u, snapp = 0u;  // snapshots of frames sp - 1 and sp - 2
    bool snap_valid = false, snapp_valid = false;
    int mx = 0, mdep = 0, mside = 0;  // frame `lane` (below the top): variable, depth, side
    uint32_t mval = 0u;               // ... and its untried values

    if (kind == K_ROOT) {
        for (int t = 0; t < I.n_unary; ++t) {
            const int v = I.unary[2 * t], off = I.unary[2 * t + 1];
            if (lane == v) d &= I.rows[off];
        }
        C.nodes += 1;
        C.stamp += 1;
        int bx = 0;
        if (node_test_var(n, d, lane, &bx) == 2) { C.fails += 1; return; }
        const u64 all = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
        if (propagate_var(I, d, all, C, lane)) { C.fails += 1; return; }
        const int st = node_test_var(n, d, lane, &bx);
        if (st == 1) {
            if (lane < n) L.dom[lane] = d;
            wsync();
            record_solution<WM>(P, I, ctl, L, C, lane);
            return;
        }
        have_open = true;
        open_x = bx;
        depth = 0;
    } else {
        F = F0;
        if (lane < n) trail[FRAME_HDR + lane] = d;
        snapc = d;
        snap_valid = true;
        sp = 1;
    }

    for (;;) {
        if (have_open) {
            have_open = false;
            const int x = open_x;
            bool split = false;
            if (P.split_target > 0) {
                long long prod = 0;
                if (lane == 0) prod = (long long)ld_rlx_u64(&P.g->produced);
                prod = unill(prod);
                if (prod < P.split_target) split = true;
            }
            uint32_t dx = (uint32_t)__builtin_amdgcn_readlane((int)d, x);
            int side0 = 0;
            if (split) {
                if (lane < n) L.dom[lane] = d;
                wsync();
                uint32_t rem = dx;
                int pushed = 0;
                if (P.two_way) {
                    uint32_t one[WM];
#pragma unroll
                    for (int q = 0; q < WM; ++q) one[q] = q == 0 ? (rem & (0u - rem)) : 0u;
                    if (push_frame<WM>(P, b, x, depth, one, L.dom, n, lane, 0)) {
                        rem &= ~one[0];
                        ++pushed;
                        side0 = 1;
                        uint32_t rest[WM];
#pragma unroll
                        for (int q = 0; q < WM; ++q) rest[q] = q == 0 ? rem : 0u;
                        if (push_frame<WM>(P, b, x, depth, rest, L.dom, n, lane, 1)) {
                            rem = 0u;
                            ++pushed;
                        }
                    }
                } else {
                    while (rem) {
                        const uint32_t lowb = rem & (0u - rem);
                        uint32_t one[WM];
#pragma unroll
                        for (int q = 0; q < WM; ++q) one[q] = q == 0 ? lowb : 0u;
                        if (!push_frame<WM>(P, b, x, depth, one, L.dom, n, lane)) break;
                        rem &= ~lowb;
                        ++pushed;
                    }
                }
                if (lane == 0 && pushed) add_u64(&P.g->produced, (u64)pushed);
                if (!rem) goto next_child;
                dx = rem;
            }
            {
                if (trail_full(P, sp, lane)) return;
                // the outgoing top frame's meta moves to its lane
                if (sp > 0 && lane == sp - 1) {
                    mx = F.x;
                    mdep = F.depth;
                    mval = F.v[0];
                    mside = F.side;
                }
                uint32_t *f = trail + (size_t)sp * FW;
                if (lane < n) f[FRAME_HDR + lane] = d;
                C.ubytes += 4ull * n;
                snapp = snapc;
                snapp_valid = snap_valid;
                snapc = d;
                snap_valid = true;
                F.x = x;
                F.depth = depth;
                F.side = side0;
                F.v[0] = dx;
#pragma unroll
                for (int k = 1; k < WM; ++k) F.v[k] = 0u;
                ++sp;
                need_restore = false;
            }
        }
    next_child:
        {
            // pop exhausted frames (registers only)
            int popped = 0;
            while (sp > 0 && F.v[0] == 0u) {
                --sp;
                ++popped;
                if (sp > 0) {
                    F.x = __builtin_amdgcn_readlane(mx, sp - 1);
                    F.depth = __builtin_amdgcn_readlane(mdep, sp - 1);
                    F.side = __builtin_amdgcn_readlane(mside, sp - 1);
                    F.v[0] = (uint32_t)__builtin_amdgcn_readlane((int)mval, sp - 1);
                }
            }
            if (sp == 0) return;
            if (popped) {
                need_restore = true;
                if (popped == 1 && snapp_valid) {
                    snapc = snapp;
                    snap_valid = true;
                } else {
                    snap_valid = false;
                }
                // prefetch the snapshot of the frame below the new top
                snapp_valid = false;
                if (sp >= 2) {
                    snapp = lane < n ? trail[(size_t)(sp - 2) * FW + FRAME_HDR + lane] : 0u;
                    snapp_valid = true;
                }
            }
        }
        {
            // the child's domain of x: the smallest remaining value, or (2-way,
            // second child) all the remaining values
            uint32_t cv;
            if (P.two_way && F.side) {
                cv = F.v[0];
                F.v[0] = 0u;
            } else {
                cv = F.v[0] & (0u - F.v[0]);
                F.v[0] &= F.v[0] - 1;
                if (P.two_way) F.side = 1;
            }
            if (need_restore) {
                if (!snap_valid) {
                    const uint32_t *f = trail + (size_t)(sp - 1) * FW;
                    snapc = lane < n ? f[FRAME_HDR + lane] : 0u;
                    snap_valid = true;
                }
                d = snapc;
                C.ubytes += 4ull * n;
            }
            need_restore = true;
            if (lane == F.x) d = cv;
            depth = F.depth + 1;
        }
        C.nodes += 1;
        C.stamp += 1;
        if (propagate_var(I, d, 1ull << F.x, C, lane)) {
            C.fails += 1;
        } else {
            int bx = 0;
            const int st = node_test_var(n, d, lane, &bx);
            if (st == 1) {
                const bool store = P.mode == 0 || (I.sol_buf && I.sol_cap > 0);
                if (store) {
                    if (lane < n) L.dom[lane] = d;
                    wsync();
                }
                record_solution<WM>(P, I, ctl, L, C, lane);
                if (P.mode == 0) return;
            } else {
                have_open = true;
                open_x = bx;
            }
        }
        if (++since_poll >= poll_iv) {
            fold_var(C);
            since_poll = 0;
            // one shared word per poll; stop, done and queue words only when
            // it says so
            int stop = 0, want = 0;
            if (lane == 0) {
                const uint32_t sig = ld_rlx(&P.q->signal);
                stop = (sig & SIG_STOP) ? 1 : ((sig & SIG_DONE) ? ld_rlx_i(&ctl->done) : 0);
                // donate while fewer tasks wait unclaimed than waves are idle
                // (a negative difference: tickets waiting for a task)
                const int idle = (int)(sig & SIG_IDLE_MASK);
                if (P.donate && idle > 0)
                    want = (int)(ld_rlx(&P.q->tail) - ld_rlx(&P.q->head)) < idle;
            }
            if (uni(stop)) return;
            if (I.max_nodes) {
                u64 tot = 0;
                if (lane == 0) tot = add_u64(&ctl->nodes, C.nodes) + C.nodes;
                tot = uni64(tot);
                C.nodes = 0;
                if (tot >= I.max_nodes) {
                    if (lane == 0) { ctl->reason = 2; st_rel_i(&ctl->done, 1); signal_rings(P, SIG_DONE); }
                    return;
                }
            }
            // the clock and the host's cancel flag (a read over PCIe) every
            // 2048 nodes
            if ((P.time_ticks || P.cancel) && (++polls & (poll_iv == POLL ? 15 : 0)) == 0) {
                int st2 = 0;
                if (lane == 0) {
                    if (P.time_ticks && (long long)wall_clock64() - t_start > P.time_ticks) st2 = 2;
                    if (P.cancel && *P.cancel) st2 = 3;
                    if (st2) stop_launch(P, st2);
                }
                if (uni(st2)) return;
            }
            if (uni(want) && sp > 0) {
                // donate the shallowest frame that still has untried values
                const u64 m = __ballot(lane < sp - 1 && mval != 0u);
                int tsel = m ? __ffsll((long long)m) - 1 : -1;
                if (tsel < 0 && F.v[0] != 0u) tsel = sp - 1;
                if (tsel >= 0) {
                    uint32_t *f = trail + (size_t)tsel * FW;
                    Frame<WM> D;
                    if (tsel == sp - 1) {
                        D = F;
                    } else {
                        D.x = __builtin_amdgcn_readlane(mx, tsel);
                        D.depth = __builtin_amdgcn_readlane(mdep, tsel);
                        D.side = __builtin_amdgcn_readlane(mside, tsel);
                        D.v[0] = (uint32_t)__builtin_amdgcn_readlane((int)mval, tsel);
#pragma unroll
                        for (int k = 1; k < WM; ++k) D.v[k] = 0u;
                    }
                    if (push_frame<WM>(P, b, D.x, D.depth, D.v, f + FRAME_HDR, n, lane, D.side)) {
                        if (tsel == sp - 1) F.v[0] = 0u;
                        else if (lane == tsel) mval = 0u;
                        C.steals += 1;
                    }
                }
            }
        }
    }
}

// A copy of an instance descriptor whose array pointers point into `tab`, a
// copy of the instance's packed blob (used to stage one instance in LDS).
DEV InstDev rebase(const InstDev &g, const uint32_t *tab) {
    InstDev I = g;
    const char *b0 = (const char *)g.blob;
    const char *t0 = (const char *)tab;
    I.lo = (const int32_t *)(t0 + ((const char *)g.lo - b0));
    // initial domains may live outside the blob (the copies of a
    // large-neighbourhood search share one blob with their own domains)
    const char *d0 = (const char *)g.dom0;
    I.dom0 = (d0 >= b0 && d0 < b0 + 4 * (size_t)g.blob_words) ? (const uint32_t *)(t0 + (d0 - b0)) : g.dom0;
    I.trig_off = (const int32_t *)(t0 + ((const char *)g.trig_off - b0));
    I.units = (const Unit *)(t0 + ((const char *)g.units - b0));
    I.rows = (const uint32_t *)(t0 + ((const char *)g.rows - b0));
    I.gtrig_off = (const int32_t *)(t0 + ((const char *)g.gtrig_off - b0));
    I.gtrig = (const int32_t *)(t0 + ((const char *)g.gtrig - b0));
    I.gdesc = (const GDesc *)(t0 + ((const char *)g.gdesc - b0));
    I.gscope = (const int32_t *)(t0 + ((const char *)g.gscope - b0));
    I.gcoef = (const int64_t *)(t0 + ((const char *)g.gcoef - b0));
    I.unary = (const int32_t *)(t0 + ((const char *)g.unary - b0));
    I.feat_static = (const float *)(t0 + ((const char *)g.feat_static - b0));
    I.pairs = (const uint32_t *)(t0 + ((const char *)g.pairs - b0));
    I.blob = tab;
    return I;
}

// Waves per SIMD the compiler must leave room for (domains of at most two
// words); it bounds the registers per lane at 512 / CUBICS_LB_WAVES.
#ifndef CUBICS_LB_WAVES
#define CUBICS_LB_WAVES 4
#endif

// Persistent search kernel: every wavefront is a worker that pops tasks from
// the global queue until no task is pending anywhere.  TL: a single-instance
// solve whose packed tables are staged once per workgroup in LDS.
template <int WM, bool TL, int FEAT, bool GLOB, bool SEGC, bool VAR = false>
__global__ __launch_bounds__(512, WM <= 2 ? CUBICS_LB_WAVES : 1) void search_kernel(SearchParams P) {
    extern __shared__ uint32_t lds_raw[];
    // idle_token: 1 while one idle wave of this workgroup polls the global
    // queue; drained: set once that wave saw no task pending anywhere
    __shared__ uint32_t idle_token, drained;
    if (threadIdx.x == 0) {
        idle_token = 0u;
        drained = 0u;
    }
    __syncthreads();
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int wid = blockIdx.x * (blockDim.x >> 6) + wave;
    uint32_t tab_words = 0;
    InstDev IL;
    if (TL) {
        const InstDev G = P.inst[0];
        tab_words = G.blob_words;
        const uint4 *src = (const uint4 *)G.blob;
        uint4 *dst = (uint4 *)lds_raw;
        for (uint32_t t = threadIdx.x; t < tab_words / 4; t += blockDim.x) dst[t] = src[t];
        __syncthreads();
        IL = rebase(G, lds_raw);
    }
    // learned search: the network's weights staged once per workgroup in LDS
    // (every branching reads all of them)
    PolicyDev LP = P.policy, VP = P.vpolicy;
    uint32_t pol_words = 0;
    if (FEAT == 1) {
        // the variable network (learned branching) and the value network
        // (learned value order), each staged when used
        const auto stage = [&](const PolicyDev &src, uint32_t *pw, PolicyDev &dst) {
            const uint32_t *w1g = (const uint32_t *)src.w1;
            const uint32_t *w2g = (const uint32_t *)src.w2;
            for (int t = threadIdx.x; t < POLICY_LDS_WORDS; t += blockDim.x) {
                uint32_t v = 0u;
                if (t < POLICY_LDS_B1) v = w1g[t];
                else if (t < POLICY_LDS_W2) v = __float_as_uint(src.b1[t - POLICY_LDS_B1]);
                else if (t < POLICY_LDS_B2) v = w2g[t - POLICY_LDS_W2];
                else if (t == POLICY_LDS_B2) v = __float_as_uint(*src.b2);
                pw[t] = v;
            }
            dst.w1 = (const uint16_t *)(pw + POLICY_LDS_W1);
            dst.b1 = (const float *)(pw + POLICY_LDS_B1);
            dst.w2 = (const uint16_t *)(pw + POLICY_LDS_W2);
            dst.b2 = (const float *)(pw + POLICY_LDS_B2);
        };
        if (P.branching == 1) stage(P.policy, lds_raw + tab_words, LP);
        if (P.value_order) stage(P.vpolicy, lds_raw + tab_words + POLICY_LDS_WORDS, VP);
        __syncthreads();
        pol_words = 2 * POLICY_LDS_WORDS;
    }
    if (wid >= P.nworkers) return;
    uint32_t *base = lds_raw + tab_words + pol_words + (size_t)wave * P.lds_words;
    Lds L;
    const int ndw = (P.nmax + 63) >> 6, ngw = (P.gmax + 63) >> 6;
    int off = 0;
    L.dom = base;
    off += ((P.nmax * P.wmax) + 1) & ~1;
    L.dA = (u64 *)(base + off);
    off += 2 * ndw;
    L.dB = (u64 *)(base + off);
    off += 2 * ndw;
    L.gp = (u64 *)(base + off);
    off += 2 * (ngw > 0 ? ngw : 1);
    L.fails = base + off;
    off += (P.nmax + 1) & ~1;
    L.trig = (int32_t *)(base + off);
    off += (P.nmax + 2) & ~1;
    L.feat = nullptr;
    L.vscr = nullptr;
    if (FEAT == 1) {  // the learned search's copy of the task's static features
        L.feat = (float *)(base + off);
        off += 4 * P.nmax;
        if (P.value_order) {
            L.vscr = (float *)(base + off);
            off += VALUE_LDS_WORDS;
        }
    }
    L.scr = base + off;  // the rest of the worker's words
    uint32_t *trail = P.trail + (size_t)wid * P.trail_words;
    // the workgroup's ring (with one ring per XCD, workgroup b runs on XCD
    // b % 8, as the hardware deals workgroups out in turn)
    const int ring = P.nrings > 1 ? (int)(blockIdx.x % (unsigned)P.nrings) : 0;
    P.q = &P.qb->ring[ring];
    P.qseq += (size_t)ring * (P.qmask + 1u);
    P.qdata += (size_t)ring * (P.qmask + 1u) * P.slot_words;
    const long long t_start = (long long)wall_clock64();
    Counters C = {};
    bool idle = false;
    // an instance this worker admitted (rings > 1): its ROOT task runs next,
    // on this worker, without passing through the queue
    int direct = -1;
    // Idle waves: only the one holding its workgroup's token takes a ticket
    // and waits on its cell (backing off exponentially, up to ~27 us between
    // polls); the others wait on the token in LDS.  A wave holding a ticket
    // leaves when no task is pending anywhere (no task can appear again), and
    // tells its workgroup through LDS.
    int backoff = 1;
    int poller = 0;  // wave-uniform: this wave holds the token
    int have_ticket = 0, polls = 0;
    uint32_t ticket = 0;
    for (;;) {
        uint32_t cell = 0, pos = 0;
        uint32_t *s = nullptr;
        int b = 0, kind = K_ROOT;
        Frame<WM> F0;
        F0.x = F0.depth = F0.side = 0;
#pragma unroll
        for (int k = 0; k < WM; ++k) F0.v[k] = 0u;
        if (direct >= 0) {
            b = direct;
            direct = -1;
        } else {
            int got = 0, fin = 0;
            if (!poller) {
                int t = 0;
                if (lane == 0) t = lds_take(&idle_token) ? 1 : 0;
                poller = uni(t);
                if (poller) backoff = 1;
            }
            if (poller) {
                if (!have_ticket) {
                    if (lane == 0) ticket = add_u(&P.q->head, 1u);
                    ticket = uniu(ticket);
                    have_ticket = 1;
                    polls = 0;
                }
                if (lane == 0) {
                    got = ld_rlx(&P.qseq[ticket & P.qmask]) == ticket + 1u;
                    if (!got && (++polls & 1) == 0 && ld_rlx_i(&P.g->pending) == 0) {
                        fin = 1;
                        lds_st(&drained, 1u);
                    }
                }
                got = uni(got);
            } else if (lane == 0) {
                fin = lds_ld(&drained) != 0u;
            }
            if (!got) {
                if (lane == 0 && !idle) add_u(&P.q->signal, 1u);
                idle = true;
                if (uni(fin)) break;
                if (poller) {
                    for (int z = 0; z < backoff; ++z) __builtin_amdgcn_s_sleep(32);
                    backoff = backoff < 32 ? backoff * 2 : 32;
                } else {
                    __builtin_amdgcn_s_sleep(16);
                }
                continue;
            }
            slot_claimed();
            pos = ticket;
            cell = ticket & P.qmask;
            have_ticket = 0;
            if (lane == 0) lds_st(&idle_token, 0u);  // hand the token on
            poller = 0;
            backoff = 1;
            if (idle) {
                if (lane == 0) add_u(&P.q->signal, 0xFFFFFFFFu);  // idle - 1
                idle = false;
            }
            s = P.qdata + (size_t)cell * P.slot_words;
            const uint32_t hw = lane < SLOT_HDR ? ld_rlx(s + lane) : 0u;  // header word `lane`
            b = __builtin_amdgcn_readlane((int)hw, 0);
            kind = __builtin_amdgcn_readlane((int)hw, 1);
            F0.x = __builtin_amdgcn_readlane((int)hw, 2);
            F0.depth = __builtin_amdgcn_readlane((int)hw, 3);
            F0.side = __builtin_amdgcn_readlane((int)hw, 12);
#pragma unroll
            for (int k = 0; k < WM; ++k) F0.v[k] = (uint32_t)__builtin_amdgcn_readlane((int)hw, 4 + k);
        }
        const InstDev I = TL ? IL : P.inst[b];
        const int nw = I.n * I.W;
        if (kind == K_ROOT) {
            for (int t = lane; t < nw; t += 64) L.dom[t] = I.dom0[t];
        } else {
            for (int t = lane; t < nw; t += 64) L.dom[t] = ld_rlx(s + SLOT_HDR + t);
        }
        if (!VAR)
            for (int t = lane; t <= I.n; t += 64) L.trig[t] = I.trig_off[t];
        wsync();
        // the slot's words are in LDS now: hand the cell back to producers
        if (s && lane == 0) st_rlx(&P.qseq[cell], pos + P.qmask + 1u);
        InstCtl *ctl = P.ctl + b;
        int skip = 0;
        if (lane == 0) {
            const uint32_t sig = ld_rlx(&P.q->signal);
            skip = (sig & SIG_STOP) ? 1 : ((sig & SIG_DONE) ? ld_rlx_i(&ctl->done) : 0);
        }
        if (!uni(skip)) {
            if (VAR)
                run_task_var<WM>(P, I, ctl, b, kind, F0, L, trail, C, lane, t_start);
            else
                run_task<WM, FEAT, GLOB, SEGC, !TL>(P, I, ctl, b, kind, F0, L, trail, C, lane, t_start, LP, VP);
        }
        C.tasks += 1;
        flush<WM>(ctl, C, lane);
        if (P.nrings > 1) {
            // the instance's last task ended: admit the next instance into
            // this ring (counted as pending before this task's end is)
            int nb = -1;
            if (lane == 0 && add_i(&ctl->live, -1) == 1) {
                const uint32_t a = add_u(&P.g->next_inst, 1u);
                if (a < (uint32_t)P.B) {
                    nb = (int)a;
                    add_i(&P.ctl[nb].live, 1);
                    add_i(&P.g->pending, 1);
                }
            }
            direct = uni(nb);
        }
        if (lane == 0) add_i(&P.g->pending, -1);
    }
    if (lane == 0 && idle) add_u(&P.q->signal, 0xFFFFFFFFu);
}

#if CUBICS_ONLY_WM == 1
// Policy features of every variable at a given node (domains dom[n][W],
// depth), with no failures counted: the same values the branching step and
// the trace records use.
__global__ void features_kernel(const InstDev *inst, const uint32_t *dom, int depth, float *out) {
    const InstDev &I = *inst;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < I.n; i += gridDim.x * blockDim.x) {
        int pop = 0;
        for (int k = 0; k < I.W; ++k) pop += __popc(dom[i * I.W + k]);
        for (int k = 0; k < POLICY_F; ++k) out[i * POLICY_F + k] = var_feature(I, I.feat_static, i, k, depth, pop, 0u);
    }
}

// Value features (value_features) of every value a < 32 W of variable x at a
// node with domains dom [n][W] and the given depth: out[a][5], zeros for
// values not in D_x.  One wavefront; domains of at most 64 values.
__global__ void value_features_kernel(const InstDev *inst, const uint32_t *dom, int depth, int x, float *out) {
    const InstDev &I = *inst;
    const int a = threadIdx.x;
    float g[POLICY_F] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (a < 32 * I.W && ((dom[x * I.W + (a >> 5)] >> (a & 31)) & 1u))
        value_features<2, false>(I, dom, I.trig_off[x], I.trig_off[x + 1], x, a, depth, g);
    if (a < 32 * I.W)
        for (int k = 0; k < POLICY_F; ++k) out[a * POLICY_F + k] = g[k];
}

// Reset the queue and seed it with ROOT tasks: every instance on one ring,
// or, with one ring per XCD, the first `seeded` instances of each ring
// (instance i on ring i % nrings); the rest are admitted as instances end.
__global__ void init_kernel(SearchParams P) {
    const uint32_t cells = P.qmask + 1u;
    const uint32_t R = (uint32_t)P.nrings;
    const uint32_t seeded = R == 1u ? (uint32_t)P.B : min((uint32_t)P.B, R * (uint32_t)P.seeded);
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t c = tid; c < R * cells; c += stride) {
        const uint32_t r = c / cells, local = c % cells;
        const uint32_t on_ring = seeded > r ? (seeded - r + R - 1u) / R : 0u;
        if (local < on_ring) {
            uint32_t *s = P.qdata + (size_t)c * P.slot_words;
            s[0] = local * R + r;
            s[1] = (uint32_t)K_ROOT;
            s[2] = 0;
            s[3] = 0;
            for (int k = 0; k < 8 && 4 + k < SLOT_HDR; ++k) s[4 + k] = 0;
            s[12] = 0;
            P.qseq[c] = local + 1u;
        } else {
            P.qseq[c] = local;
        }
    }
    for (uint32_t b = tid; b < (uint32_t)P.B; b += stride) {
        InstCtl z;
        z.count = z.n_slots = z.nodes = z.fails = z.revisions = z.alg_bytes = z.steals = z.tasks = 0;
        z.done = z.reason = z.found = 0;
        z.live = b < seeded ? 1 : 0;
        P.ctl[b] = z;
    }
    if (tid == 0 && P.trace_count) *P.trace_count = 0ull;
    if (tid < R) {
        P.qb->ring[tid].head = 0;
        P.qb->ring[tid].tail = seeded > tid ? (seeded - tid + R - 1u) / R : 0u;
        P.qb->ring[tid].signal = 0u;
    }
    if (tid == 0) {
        P.g->pending = (int32_t)seeded;
        P.g->produced = 0;
        P.g->stop = 0;
        P.g->stop_reason = 0;
        P.g->next_inst = seeded;
    }
}

#endif

// Root fixpoint of one instance (one wave): writes the domains and the verdict.
template <int WM>
__global__ void root_kernel(SearchParams P, uint32_t *out, int32_t *failed, unsigned long long *revs) {
    extern __shared__ uint32_t lds_raw[];
    const int lane = lane_id();
    const InstDev I = P.inst[0];
    Lds L;
    const int ndw = (P.nmax + 63) >> 6, ngw = (P.gmax + 63) >> 6;
    int off = 0;
    L.dom = lds_raw;
    off += ((P.nmax * P.wmax) + 1) & ~1;
    L.dA = (u64 *)(lds_raw + off);
    off += 2 * ndw;
    L.dB = (u64 *)(lds_raw + off);
    off += 2 * ndw;
    L.gp = (u64 *)(lds_raw + off);
    off += 2 * (ngw > 0 ? ngw : 1);
    L.fails = lds_raw + off;
    off += (P.nmax + 1) & ~1;
    L.trig = (int32_t *)(lds_raw + off);
    off += (P.nmax + 2) & ~1;
    L.scr = lds_raw + off;
    L.feat = nullptr;
    const int n = I.n, W = I.W, nw = n * W;
    for (int t = lane; t < nw; t += 64) L.dom[t] = I.dom0[t];
    for (int t = lane; t <= n; t += 64) L.trig[t] = I.trig_off[t];
    wsync();
    for (int t = lane; t < I.n_unary; t += 64) {
        const int v = I.unary[2 * t], o = I.unary[2 * t + 1];
        for (int k = 0; k < W; ++k) atomicAnd(&L.dom[v * W + k], I.rows[o + k]);
    }
    wsync();
    Counters C = {};
    int bx = 0;
    bool fail = node_test<WM>(I, L, lane, &bx) == 2;
    if (!fail) {
        dirty_all(L, n, lane);
        fail = propagate<WM, true, true, true>(I, L, P.layout, C, lane);
    }
    wsync();
    for (int t = lane; t < nw; t += 64) out[t] = L.dom[t];
    const u64 r = wave_sumu64(C.rev);
    if (lane == 0) {
        *failed = fail ? 1 : 0;
        *revs = r;
    }
}

// -------------------------------------------------- host-side launchers
// Kernel variants: the learned / tracing kernel is general; the plain kernel
// is specialised on the presence of global constraints and on the layout.
template <int WM, bool TL>
static const void *search_fn(int variant) {
    switch (variant) {
    case 0: return (const void *)search_kernel<WM, TL, 0, false, false>;
    case 1: return (const void *)search_kernel<WM, TL, 0, false, true>;
    case 2: return (const void *)search_kernel<WM, TL, 0, true, false>;
    case 3: return (const void *)search_kernel<WM, TL, 0, true, true>;
    case 4: return (const void *)search_kernel<WM, TL, 1, false, false>;
    case 5: return (const void *)search_kernel<WM, TL, 1, false, true>;
    case 6: return (const void *)search_kernel<WM, TL, 1, true, false>;
    case 7: return (const void *)search_kernel<WM, TL, 1, true, true>;
    case 9: return (const void *)search_kernel<WM, TL, 0, false, false, WM == 1>;
    default: return (const void *)search_kernel<WM, TL, 2, true, true>;
    }
}
template <int WM>
static const void *search_fn_t(bool tl, int variant) {
    return tl ? search_fn<WM, true>(variant) : search_fn<WM, false>(variant);
}
template <int WM>
static hipError_t launch_root_t(const SearchParams &P, uint32_t *out, int32_t *failed,
                                unsigned long long *revs, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(root_kernel<WM>, dim3(1), dim3(64), lds, st, P, out, failed, revs);
    return hipGetLastError();
}

#define CUBICS_CAT2(a, b) a##b
#define CUBICS_CAT(a, b) CUBICS_CAT2(a, b)

const void *CUBICS_CAT(search_fn_w, CUBICS_ONLY_WM)(bool tl, int variant) {
    return search_fn_t<CUBICS_ONLY_WM>(tl, variant);
}
hipError_t CUBICS_CAT(launch_root_w, CUBICS_ONLY_WM)(const SearchParams &P, uint32_t *out, int32_t *failed,
                                                      unsigned long long *revs, size_t lds, hipStream_t st) {
    return launch_root_t<CUBICS_ONLY_WM>(P, out, failed, revs, lds, st);
}

#if CUBICS_ONLY_WM == 1
const void *search_fn_w2(bool tl, int variant);
const void *search_fn_w4(bool tl, int variant);
const void *search_fn_w8(bool tl, int variant);
hipError_t launch_root_w2(const SearchParams &, uint32_t *, int32_t *, unsigned long long *, size_t, hipStream_t);
hipError_t launch_root_w4(const SearchParams &, uint32_t *, int32_t *, unsigned long long *, size_t, hipStream_t);
hipError_t launch_root_w8(const SearchParams &, uint32_t *, int32_t *, unsigned long long *, size_t, hipStream_t);

static const void *search_fn_any(int wmax, bool tl, int variant) {
    switch (wmax) {
    case 1: return search_fn_w1(tl, variant);
    case 2: return search_fn_w2(tl, variant);
    case 4: return search_fn_w4(tl, variant);
    default: return search_fn_w8(tl, variant);
    }
}
// variant: 9 = VAR layout (plain); 8 = trace recording; else 4 * learned +
// 2 * globals present + SEG layout
int search_variant(int feat, bool glob, bool seg, bool var) {
    if (feat == 0 && var) return 9;
    return feat == 2 ? 8 : 4 * (feat == 1) + (glob ? 2 : 0) + (seg ? 1 : 0);
}

hipError_t launch_search(int wmax, const SearchParams &P, int blocks, int wpb, size_t lds, bool tl, int variant,
                         hipStream_t st) {
    const void *fn = search_fn_any(wmax, tl, variant);
    if (lds > 64 * 1024) {
        // beyond 64 KiB of dynamic LDS a kernel must opt in (gfx950: 160 KiB)
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    void *args[] = {(void *)&P};
    return hipLaunchKernel(fn, dim3(blocks), dim3(64 * wpb), args, lds, st);
}
hipError_t launch_root(int wmax, const SearchParams &P, uint32_t *out, int32_t *failed,
                       unsigned long long *revs, size_t lds, hipStream_t st) {
    switch (wmax) {
    case 1: return launch_root_w1(P, out, failed, revs, lds, st);
    case 2: return launch_root_w2(P, out, failed, revs, lds, st);
    case 4: return launch_root_w4(P, out, failed, revs, lds, st);
    default: return launch_root_w8(P, out, failed, revs, lds, st);
    }
}
hipError_t launch_init(const SearchParams &P, hipStream_t st) {
    hipLaunchKernelGGL(init_kernel, dim3(256), dim3(256), 0, st, P);
    return hipGetLastError();
}
hipError_t launch_features(const InstDev *inst, const uint32_t *dom, int depth, float *out, int n,
                           hipStream_t st) {
    const int blocks = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
    hipLaunchKernelGGL(features_kernel, dim3(blocks), dim3(256), 0, st, inst, dom, depth, out);
    return hipGetLastError();
}
hipError_t launch_value_features(const InstDev *inst, const uint32_t *dom, int depth, int x, float *out,
                                 hipStream_t st) {
    hipLaunchKernelGGL(value_features_kernel, dim3(1), dim3(64), 0, st, inst, dom, depth, x, out);
    return hipGetLastError();
}
hipError_t search_occupancy(int wmax, int *blocks_per_cu, int wpb, size_t lds, bool tl, int variant) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, search_fn_any(wmax, tl, variant), 64 * wpb, lds);
}
#endif

}  // namespace cubics
