// Internal data layout shared by the host packer (cubics_host.cpp) and the
// HIP kernels (cubics_search.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace cubics {

// Propagator ("unit") types of binary constraints, one unit per direction.
// A unit revises its target variable against its source variable.
enum UnitType : int32_t {
    U_TABLE = 1,   // extensional table, rows in both orientations
    U_NEQ = 2,     // remove a = b + p0 when D_src = {b}
    U_LT_UB = 3,   // keep a <= max(D_src) + p0 - 1
    U_LT_LB = 4,   // keep a >= min(D_src) - p0 + 1
    U_QUEENS = 5,  // p0 = k, p1 = delta: a conflicts with b iff a - b - delta in {0, k, -k}
};
enum GlobalType : int32_t { G_ALLDIFF = 1, G_LINEAR = 2, G_ALLDIFF_GAC = 3, G_LINEAR_AD = 4 };
// A linear <= constraint bounded with the all-different groups inside its
// scope holds at most this many groups, each of at most 64 variables.
constexpr int AD_GROUPS_MAX = 16;
constexpr int GAC_MAX_K = 64;     // variables of one GAC all-different (one lane each)
constexpr int SCRATCH_WORDS = 32;      // per-worker LDS scratch
constexpr int SCRATCH_GAC_WORDS = 96;  // ... when a GAC all-different is present
// VAR layout pair entry, one word (type << 28) | param: TABLE param = word
// offset of the rows indexed by the source value; NEQ / LT param = delta
// (28-bit signed); QUEENS param = k << 15 | (delta & 0x7FFF).
enum TaskKind : int32_t { K_ROOT = 0, K_NODE = 1, K_FRAME = 2 };

// Binary unit (16 B).  tt = target var | type << 24.
// TABLE: p0 = word offset of rows indexed by target value (bits over source),
//        p1 = word offset of rows indexed by source value (bits over target).
struct Unit {
    int32_t tt;
    int32_t src;
    int32_t p0;
    int32_t p1;
};

// Global constraint descriptor (16 B).
struct GDesc {
    int32_t type;
    int32_t k;         // arity
    int32_t scope_off; // into gscope: v_0..v_{k-1}; LINEAR_AD also group[k]
                       // (-1 = ungrouped), then each group's scope positions
    int32_t coef_off;  // into gcoef: b, a_0..a_{k-1} (LINEAR); LINEAR_AD also
                       // G, then per group: base value, k_g, the group's
                       // coefficients in descending order.  ALLDIFF*: the
                       // scope's smallest lo (no gcoef entries)
};

// Per-instance read-only descriptor (device memory).  All pointers are device
// pointers into the problem's packed blob.
struct InstDev {
    int32_t n, W, S, dmax;       // vars, words/domain, SEG lanes per unit, max domain
    int32_t n_units, n_glob, n_unary, seg_ok;
    const int32_t *lo;           // [n]
    const uint32_t *dom0;        // [n*W] declared ranges intersected with init bits
    const int32_t *trig_off;     // [n+1] units sorted by source var
    const Unit *units;           // [n_units]
    const uint32_t *rows;        // table rows (W words per row)
    const int32_t *gtrig_off;    // [n+1]
    const int32_t *gtrig;        // global ids watching each var
    const GDesc *gdesc;          // [n_glob]
    const int32_t *gscope;
    const int64_t *gcoef;
    const int32_t *unary;        // [n_unary][2] {var, row word offset}
    const float *feat_static;    // [n][4] static features for the learned policy
    const uint32_t *pairs;       // [n][64] VAR layout: unit (t <- j) at [j*64 + t], packed
                                 // (type << 28) | param (28-bit signed; QUEENS: k << 15 | offset)
    const uint32_t *blob;        // start of the packed problem (all arrays above lie inside)
    uint32_t blob_words;         // its size in 32-bit words
    int32_t var_ok;              // VAR layout usable: n <= 64, one word per domain,
                                 // binary constraints only, one constraint per pair
    int32_t unit_types;          // bit t set iff some binary unit has type t
    int32_t pad1;
    // per-instance solve settings (written by the host for each solve)
    int32_t *sol_buf;
    uint64_t sol_cap;
    uint64_t max_nodes;
    uint64_t max_solutions;
};

// Per-instance mutable solve state (device memory, zeroed before a solve).
struct InstCtl {
    unsigned long long count, n_slots, nodes, fails, revisions, alg_bytes, steals, tasks;
    int32_t done;     // 1 = stop working on this instance
    int32_t reason;   // 0 none, 1 first found, 2 node limit, 3 cap
    int32_t found;    // FIRST mode winner flag
    int32_t live;     // the instance's tasks queued or running (rings > 1)
};

// Control of one work-queue ring: each hot word on its own 128-byte line.
struct QCtl {
    uint32_t head; uint32_t _p0[31];
    uint32_t tail; uint32_t _p1[31];
    // idle workers of the ring (bits 0..23) | SIG_DONE | SIG_STOP: the one
    // word a busy worker polls; the rest is read only when it is non-zero
    uint32_t signal; int32_t _p3[31];
};
// Launch-wide control.
struct QGlobal {
    int32_t pending; int32_t _p2[31];       // tasks queued or running, all rings
    unsigned long long produced; uint32_t _p4[30];
    int32_t stop; int32_t stop_reason; uint32_t _p5[30];
    uint32_t next_inst; uint32_t _p6[31];   // next instance to admit (rings > 1)
};
// A batch runs on one ring, or on one ring per XCD (workgroup b serves ring
// b % MAX_RINGS; the hardware deals workgroups to the 8 XCDs in turn), each
// ring holding a few instances at a time, so that the tables one XCD's
// workers read stay in that XCD's L2.
constexpr int MAX_RINGS = 8;
struct QBlock {
    QGlobal g;
    QCtl ring[MAX_RINGS];
};

constexpr uint32_t SIG_IDLE_MASK = 0x00FFFFFFu;
constexpr uint32_t SIG_DONE = 1u << 29;  // some instance's done flag is set
constexpr uint32_t SIG_STOP = 1u << 30;  // the whole launch stops

// Queue slot / trail frame header layout (uint32 words).
constexpr int SLOT_HDR = 16;   // [0] inst [1] kind [2] x [3] depth [4..12) vals [12] side
constexpr int FRAME_HDR = 32;  // [0] x [1] depth [2] flags [3] side [4..12) vals [16..21) features [24..26) node stamp

// Learned policy (device).  Parameter vector theta (fp32 master copy):
// W1[64][5] (hidden-major), b1[64], w2[64], b2 -> 449 values.
constexpr int POLICY_F = 5;    // features per variable
constexpr int POLICY_H = 64;   // hidden units
constexpr int POLICY_NP = POLICY_H * POLICY_F + POLICY_H + POLICY_H + 1;
constexpr int OFF_W1 = 0, OFF_B1 = POLICY_H * POLICY_F, OFF_W2 = OFF_B1 + POLICY_H, OFF_B2 = OFF_W2 + POLICY_H;

// LDS copy of the network for the learned search (words): w1 bf16 [64][16]
// (512 words), b1 [64], w2 bf16 [64] (32 words), b2, padded to 16 bytes.
constexpr int POLICY_LDS_W1 = 0, POLICY_LDS_B1 = 512, POLICY_LDS_W2 = 576, POLICY_LDS_B2 = 608;
constexpr int POLICY_LDS_WORDS = 612;

struct PolicyDev {
    const uint16_t *w1;  // [64][16] bf16, inputs >= POLICY_F zero
    const float *b1;     // [64] (inside theta)
    const uint16_t *w2;  // [64] bf16
    const float *b2;     // [1] (inside theta)
};

struct SearchParams {
    const InstDev *inst;
    InstCtl *ctl;
    int32_t B;
    int32_t mode;
    int32_t layout;      // 1 LANE, 2 SEG
    int32_t branching;
    int32_t two_way;     // 2-way branching: x = min D_x, then x != min D_x
    QBlock *qb;
    QCtl *q;             // the worker's ring (the kernel points it at ring b % nrings)
    QGlobal *g;
    int32_t nrings;      // 1, or MAX_RINGS with admission of instances per ring
    int32_t seeded;      // instances queued per ring at launch (rings > 1)
    uint32_t *qseq;      // [nrings][qmask + 1] (the kernel offsets it per ring)
    uint32_t *qdata;     // [nrings][qmask + 1][slot_words]
    uint32_t qmask;      // cells per ring - 1
    uint32_t slot_words;
    uint32_t *trail;
    uint32_t frame_words;
    uint32_t trail_words;  // per worker
    int32_t max_frames;    // frames per worker trail (a push beyond stops the launch)
    int32_t nworkers;
    int32_t donate;
    long long split_target;
    long long time_ticks;  // 0 = none (wall clock ticks)
    const volatile int32_t *cancel;
    int32_t lds_words;     // per worker
    int32_t nmax, wmax, gmax;
    PolicyDev policy;
    PolicyDev vpolicy;     // value network (learned value order; lds copy staged per workgroup)
    int32_t value_order;   // 1 = children of a d-way branching in descending value-network score
    float *trace_out;      // optional trace records [trace_cap][8] (learned policy training)
    unsigned long long *trace_count;
    unsigned long long trace_cap;
    int32_t explore_pm;    // per-mille of branchings that explore among the 4 smallest domains
    uint32_t seed;
};

// Trace record (8 floats): features f0..f4, depth, 0, label = log2(1 + nodes below).
constexpr int TRACE_WORDS = 8;

// Learned value order: per-worker LDS scratch (features of up to 64 values,
// then their scores) and the scores kept in each trail frame.
constexpr int VALUE_MAX = 64;
constexpr int VALUE_LDS_WORDS = VALUE_MAX * POLICY_F + VALUE_MAX;
constexpr int FRAME_SCORES = VALUE_MAX;

}  // namespace cubics
