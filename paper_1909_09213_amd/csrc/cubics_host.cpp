// Host side of libcubics: argument validation, packing of a CSP into the
// device layout (Sec. 2.1: the CPU builds the data structures and moves them
// to GPU memory once), solve orchestration and result readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cubics.h"
#include "cubics_internal.h"

namespace cubics {
hipError_t launch_search(int wmax, const SearchParams &P, int blocks, int wpb, size_t lds, bool tl, int variant,
                         hipStream_t st);
int search_variant(int feat, bool glob, bool seg, bool var);
hipError_t launch_root(int wmax, const SearchParams &P, uint32_t *out, int32_t *failed,
                       unsigned long long *revs, size_t lds, hipStream_t st);
hipError_t launch_init(const SearchParams &P, hipStream_t st);
hipError_t launch_features(const InstDev *inst, const uint32_t *dom, int depth, float *out, int n,
                           hipStream_t st);
hipError_t launch_value_features(const InstDev *inst, const uint32_t *dom, int depth, int x, float *out,
                                 hipStream_t st);
hipError_t search_occupancy(int wmax, int *blocks_per_cu, int wpb, size_t lds, bool tl, int variant);
}  // namespace cubics

using namespace cubics;

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(CUBICS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *cubics_last_error(void) { return g_err.c_str(); }

int cubics_set_error(int code, const char *msg) { return fail(code, "%s", msg); }

// ------------------------------------------------------- device buffers
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap) return 0;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(bytes, 256);
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            return fail(CUBICS_ENOMEM, "hipMalloc(%zu) failed", want);
        }
        cap = want;
        return 0;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct cubics_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    int wall_khz = 100000;
    int lds_max = 64 * 1024;  // LDS bytes one workgroup may allocate (160 KiB on gfx950)
    DevBuf inst, ctl, q, qseq, qdata, trail, rootout, tracecnt;
    DevBuf lnsdom, lnssol;  // large-neighbourhood search: initial domains, solutions
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t *cancel_host = nullptr;  // pinned, polled by the kernel
    struct Tuned {
        int layout;  // revision layout
        int div;     // workers = the occupancy-limited maximum / div
        int gang;    // batches: instances active per XCD ring (0 = one queue)
    };
    std::map<std::string, Tuned> tuned;  // shape bucket -> autotuned choice
    std::map<std::string, hipGraphExec_t> graphs;  // captured launch sequences
    hipStream_t graph_stream = nullptr;  // capture stream when the caller's is the null stream
};

struct cubics_prob {
    cubics_ctx *ctx = nullptr;
    void *blob = nullptr;
    InstDev dev;  // with device pointers into blob
    int n = 0, W = 1, dmax = 1;
    int n_units = 0, n_glob = 0;
    int64_t dsum = 0;  // sum over variables of (dsize - 1): bounds 2-way branchings on a path
    int64_t last_lin_b = -1;  // gcoef index of the bound b of the last LINEAR_LE (or -1)
    bool has_table = false;
    bool has_gac = false;  // a GAC all-different (needs the larger LDS scratch)
    std::string bucket;
};

hipStream_t cubics_ctx_stream(const cubics_ctx *c) { return c->stream; }
int cubics_ctx_device(const cubics_ctx *c) { return c->device; }

// ----------------------------------------------------------------- context
extern "C" int cubics_create(int32_t device, void *hip_stream, cubics_ctx **out) {
    if (!out) return fail(CUBICS_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(CUBICS_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIPCHK(hipSetDevice(device));
    cubics_ctx *c = new cubics_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return fail(CUBICS_EDEVICE, "hipGetDeviceProperties failed");
    }
    c->cu_count = prop.multiProcessorCount;
    if (prop.sharedMemPerBlock >= 64 * 1024) c->lds_max = (int)prop.sharedMemPerBlock;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->wall_khz = khz;
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipHostMalloc((void **)&c->cancel_host, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        cubics_destroy(c);
        return fail(CUBICS_EDEVICE, "event / pinned flag allocation failed");
    }
    *c->cancel_host = 0;
    *out = c;
    return CUBICS_OK;
}

extern "C" void cubics_destroy(cubics_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    c->inst.release(); c->ctl.release(); c->q.release(); c->qseq.release();
    c->qdata.release(); c->trail.release(); c->rootout.release(); c->tracecnt.release();
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->cancel_host) (void)hipHostFree(c->cancel_host);
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->graph_stream) (void)hipStreamDestroy(c->graph_stream);
    delete c;
}

extern "C" int cubics_set_stream(cubics_ctx *c, void *hip_stream) {
    if (!c) return fail(CUBICS_EINVAL, "ctx is NULL");
    c->stream = (hipStream_t)hip_stream;
    return CUBICS_OK;
}

extern "C" void cubics_cancel(cubics_ctx *c) {
    if (c && c->cancel_host) __atomic_store_n(c->cancel_host, 1, __ATOMIC_RELEASE);
}

// -------------------------------------------------------------------- load
namespace {

struct Packer {
    std::vector<uint8_t> bytes;
    size_t add(const void *src, size_t n, size_t align = 256) {
        size_t off = (bytes.size() + align - 1) / align * align;
        bytes.resize(off + n);
        if (n && src) memcpy(bytes.data() + off, src, n);
        return off;
    }
};

inline uint32_t range_word(int d, int k) {
    int nb = d - 32 * k;
    if (nb <= 0) return 0u;
    if (nb >= 32) return 0xFFFFFFFFu;
    return (1u << nb) - 1u;
}

}  // namespace

extern "C" int cubics_load(cubics_ctx *ctx, int32_t n, const int32_t *lo, const int32_t *dsize,
                           const uint32_t *init_bits, int32_t m, const int32_t *type,
                           const int32_t *arity, const int64_t *var_off, const int32_t *vars,
                           const int64_t *par_off, const int64_t *params, const int64_t *tab_off,
                           const uint32_t *tabs, cubics_prob **out) {
    if (!out) return fail(CUBICS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(CUBICS_EINVAL, "ctx is NULL");
    if (n < 0 || m < 0) return fail(CUBICS_EINVAL, "negative n or m");
    if (n > CUBICS_MAX_VARS) return fail(CUBICS_EUNSUPPORTED, "n=%d exceeds %d variables", n, CUBICS_MAX_VARS);
    if (n > 0 && (!lo || !dsize)) return fail(CUBICS_EINVAL, "lo/dsize is NULL");
    if (m > 0 && (!type || !arity || !var_off || !vars || !par_off || !tab_off))
        return fail(CUBICS_EINVAL, "constraint arrays are NULL");
    int dmax = 1;
    for (int i = 0; i < n; ++i) {
        if (dsize[i] < 1) return fail(CUBICS_EINVAL, "dsize[%d]=%d < 1", i, dsize[i]);
        if (dsize[i] > CUBICS_MAX_DOMAIN)
            return fail(CUBICS_EUNSUPPORTED, "dsize[%d]=%d exceeds %d", i, dsize[i], CUBICS_MAX_DOMAIN);
        if (lo[i] < -(1 << 29) || lo[i] > (1 << 29)) return fail(CUBICS_EUNSUPPORTED, "lo[%d] out of range", i);
        dmax = std::max(dmax, (int)dsize[i]);
    }
    // ALLDIFF scopes compare domains in value space: widen W to their spans
    int span_words = 1;
    for (int c = 0; c < m; ++c) {
        if (type[c] != CUBICS_ALLDIFF && type[c] != CUBICS_ALLDIFF_GAC) continue;
        const int k = arity[c];
        if (k < 1 || var_off[c + 1] - var_off[c] != k) continue;  // reported below
        const int32_t *sc = vars + var_off[c];
        bool ok = true;
        for (int t = 0; t < k; ++t) ok &= sc[t] >= 0 && sc[t] < n;
        if (!ok) continue;
        int base = lo[sc[0]], top = lo[sc[0]] + dsize[sc[0]];
        for (int t = 1; t < k; ++t) {
            base = std::min(base, (int)lo[sc[t]]);
            top = std::max(top, (int)(lo[sc[t]] + dsize[sc[t]]));
        }
        if (top - base <= CUBICS_MAX_DOMAIN) span_words = std::max(span_words, (top - base + 31) / 32);
    }
    const int Win = (dmax + 31) / 32;  // words per row of init_bits
    const int W = std::max(Win, span_words);
    if ((int64_t)n * W > 4096) return fail(CUBICS_EUNSUPPORTED, "n*W=%d exceeds 4096 words", n * W);
    if (m > 0 && (var_off[0] != 0 || par_off[0] != 0 || tab_off[0] != 0))
        return fail(CUBICS_EINVAL, "offset arrays must start at 0");

    // ---- domains
    std::vector<uint32_t> dom0((size_t)std::max(n, 1) * W, 0u);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < W; ++k) {
            uint32_t w = range_word(dsize[i], k);
            if (init_bits) w &= k < Win ? init_bits[(size_t)i * Win + k] : 0u;
            dom0[(size_t)i * W + k] = w;
        }

    // ---- constraints
    std::vector<Unit> units;
    // rows start with an all-ones block of 32 words: in the register layout
    // a lane with no constraint to the revised source (pair entry 0, row
    // offset 0) takes the support union of this block and keeps its domain.
    // Row offsets count from that block; the blob holds ROW_PRE zero words
    // before it, so that row -1 of every block, the all-ones one included,
    // lies inside the rows section.
    constexpr int ROW_PRE = 8;
    std::vector<uint32_t> rows(32, 0xFFFFFFFFu);
    std::vector<GDesc> gdesc;
    std::vector<int32_t> gscope;
    std::vector<int64_t> gcoef;
    std::vector<int32_t> unary;
    std::vector<int32_t> deg(std::max(n, 1), 0);
    std::vector<double> tight_sum(std::max(n, 1), 0.0);
    bool has_table = false, has_gac = false;
    int64_t last_lin_b = -1;
    for (int c = 0; c < m; ++c) {
        const int ty = type[c], k = arity[c];
        if (var_off[c + 1] - var_off[c] != k || k < 1)
            return fail(CUBICS_EINVAL, "constraint %d: arity %d does not match its scope", c, k);
        const int32_t *sc = vars + var_off[c];
        for (int t = 0; t < k; ++t) {
            if (sc[t] < 0 || sc[t] >= n) return fail(CUBICS_EINVAL, "constraint %d: variable %d out of range", c, sc[t]);
            for (int u = 0; u < t; ++u)
                if (sc[u] == sc[t]) return fail(CUBICS_EINVAL, "constraint %d: variable %d repeated in scope", c, sc[t]);
        }
        const int64_t npar = par_off[c + 1] - par_off[c];
        const int64_t ntab = tab_off[c + 1] - tab_off[c];
        if (npar < 0 || ntab < 0) return fail(CUBICS_EINVAL, "constraint %d: decreasing offsets", c);
        const int64_t *par = params ? params + par_off[c] : nullptr;
        const uint32_t *tab = tabs ? tabs + tab_off[c] : nullptr;
        if (ty == CUBICS_UNARY) {
            if (k != 1) return fail(CUBICS_EINVAL, "constraint %d: UNARY needs arity 1", c);
            const int i = sc[0], Wi = (dsize[i] + 31) / 32;
            if (ntab != Wi || !tab) return fail(CUBICS_EINVAL, "constraint %d: UNARY table needs %d words", c, Wi);
            unary.push_back(i);
            unary.push_back((int32_t)rows.size());
            for (int w = 0; w < W; ++w) rows.push_back(w < Wi ? (tab[w] & range_word(dsize[i], w)) : 0u);
        } else if (ty >= CUBICS_TABLE2 && ty <= CUBICS_QUEENS) {
            if (k != 2) return fail(CUBICS_EINVAL, "constraint %d: binary type needs arity 2", c);
            const int i = sc[0], j = sc[1];
            const int di = dsize[i], dj = dsize[j];
            deg[i]++; deg[j]++;
            if (ty == CUBICS_TABLE2) {
                const int Wj = (dj + 31) / 32;
                if (ntab != (int64_t)di * Wj || !tab)
                    return fail(CUBICS_EINVAL, "constraint %d: TABLE2 needs %d x %d words", c, di, Wj);
                has_table = true;
                // rows indexed by the value of i (bits over j) and by the value
                // of j (bits over i).  Every block is preceded by W zero words
                // (row -1: the revisions read it for the slots past their last
                // value) and blocks sit at an odd stride: the lanes revising
                // different constraints read row `a` of their own blocks at
                // once, and blocks at a stride of 16 words would put them all
                // in two of the 32 LDS banks.
                const auto block = [&rows, W](size_t words) {
                    rows.resize(rows.size() + W, 0u);
                    const int32_t off = (int32_t)rows.size();
                    rows.resize(rows.size() + words + ((W + words) % 2 == 0 ? 1 : 0), 0u);
                    return off;
                };
                const int32_t off_ij = block((size_t)di * W);
                const int32_t off_ji = block((size_t)dj * W);
                int64_t allowed = 0;
                for (int a = 0; a < di; ++a)
                    for (int b = 0; b < dj; ++b)
                        if ((tab[(size_t)a * Wj + b / 32] >> (b % 32)) & 1u) {
                            rows[off_ij + (size_t)a * W + b / 32] |= 1u << (b % 32);
                            rows[off_ji + (size_t)b * W + a / 32] |= 1u << (a % 32);
                            ++allowed;
                        }
                const double t = 1.0 - (double)allowed / ((double)di * dj);
                tight_sum[i] += t; tight_sum[j] += t;
                units.push_back({i | (U_TABLE << 24), j, off_ij, off_ji});
                units.push_back({j | (U_TABLE << 24), i, off_ji, off_ij});
            } else {
                if (npar != 1 || !par) return fail(CUBICS_EINVAL, "constraint %d: needs 1 parameter", c);
                const int64_t p = par[0];
                if (p < -(1LL << 29) || p > (1LL << 29)) return fail(CUBICS_EUNSUPPORTED, "constraint %d: parameter out of range", c);
                const int32_t dl = (int32_t)((int64_t)lo[j] - lo[i] + (ty == CUBICS_QUEENS ? 0 : p));
                if (ty == CUBICS_NEQ) {
                    // x_i != x_j + p: a = b + dl is removed from i; b = a - dl from j
                    units.push_back({i | (U_NEQ << 24), j, dl, 0});
                    units.push_back({j | (U_NEQ << 24), i, -dl, 0});
                    tight_sum[i] += 1.0 / dj; tight_sum[j] += 1.0 / di;
                } else if (ty == CUBICS_LT) {
                    units.push_back({i | (U_LT_UB << 24), j, dl, 0});
                    units.push_back({j | (U_LT_LB << 24), i, dl, 0});
                    tight_sum[i] += 0.5; tight_sum[j] += 0.5;
                } else {
                    const int32_t kq = (int32_t)p;
                    units.push_back({i | (U_QUEENS << 24), j, kq, (int32_t)(lo[j] - lo[i])});
                    units.push_back({j | (U_QUEENS << 24), i, kq, (int32_t)(lo[i] - lo[j])});
                    tight_sum[i] += 3.0 / dj; tight_sum[j] += 3.0 / di;
                }
            }
        } else if (ty == CUBICS_ALLDIFF || ty == CUBICS_ALLDIFF_GAC || ty == CUBICS_LINEAR_LE ||
                   ty == CUBICS_LINEAR_LE_AD) {
            const bool lin = ty == CUBICS_LINEAR_LE || ty == CUBICS_LINEAR_LE_AD;
            GDesc g;
            g.type = ty == CUBICS_ALLDIFF       ? G_ALLDIFF
                     : ty == CUBICS_ALLDIFF_GAC ? G_ALLDIFF_GAC
                     : ty == CUBICS_LINEAR_LE   ? G_LINEAR
                                                : G_LINEAR_AD;
            if (ty == CUBICS_ALLDIFF_GAC) {
                if (k > GAC_MAX_K)
                    return fail(CUBICS_EUNSUPPORTED, "constraint %d: ALLDIFF_GAC over %d > %d variables", c, k,
                                GAC_MAX_K);
                has_gac = true;
            }
            g.k = k;
            g.scope_off = (int32_t)gscope.size();
            g.coef_off = (int32_t)gcoef.size();
            if (lin) last_lin_b = g.coef_off;
            if (!lin) {
                // the scope's domains are compared in value space: base = the
                // smallest lo; the span must fit the instance's domain words
                int base = lo[sc[0]], top = lo[sc[0]] + dsize[sc[0]];
                for (int t = 1; t < k; ++t) {
                    base = std::min(base, (int)lo[sc[t]]);
                    top = std::max(top, (int)(lo[sc[t]] + dsize[sc[t]]));
                }
                if (top - base > CUBICS_MAX_DOMAIN)
                    return fail(CUBICS_EUNSUPPORTED, "constraint %d: all-different value span %d exceeds %d", c,
                                top - base, CUBICS_MAX_DOMAIN);
                g.coef_off = base;
                for (int t = 0; t < k; ++t) tight_sum[sc[t]] += (double)(k - 1) / dsize[sc[t]];
            } else {
                if (npar != 1 + k || !par) return fail(CUBICS_EINVAL, "constraint %d: LINEAR_LE needs 1+k parameters", c);
                double mag = std::fabs((double)par[0]), vall = 0;
                for (int t = 0; t < k; ++t)
                    vall = std::max(vall, std::max(std::fabs((double)lo[sc[t]]),
                                                   std::fabs((double)lo[sc[t]] + dsize[sc[t]] - 1)));
                for (int t = 0; t < k; ++t) {
                    if (par[1 + t] <= 0) return fail(CUBICS_EINVAL, "constraint %d: non-positive coefficient", c);
                    const double vmax = std::max(std::fabs((double)lo[sc[t]]), std::fabs((double)lo[sc[t]] + dsize[sc[t]] - 1));
                    // a group bound pairs a coefficient with any value of its group
                    mag += (double)par[1 + t] * (ty == CUBICS_LINEAR_LE_AD ? vall : vmax);
                }
                if (mag > 4.0e18) return fail(CUBICS_EUNSUPPORTED, "constraint %d: linear sum may overflow int64", c);
                double maxsum = 0;
                for (int t = 0; t < k; ++t) maxsum += (double)par[1 + t] * ((double)lo[sc[t]] + dsize[sc[t]] - 1);
                const double tt = maxsum > 0 ? std::min(1.0, std::max(0.0, 1.0 - (double)par[0] / maxsum)) : 0.5;
                for (int t = 0; t < k; ++t) tight_sum[sc[t]] += tt;
                for (int t = 0; t <= k; ++t) gcoef.push_back(par[t]);
            }
            for (int t = 0; t < k; ++t) {
                gscope.push_back(sc[t]);
                deg[sc[t]]++;
            }
            if (ty == CUBICS_LINEAR_LE_AD) {
                // groups: the all-different constraints (ALLDIFF, ALLDIFF_GAC)
                // whose variables all lie in the scope, in constraint order,
                // each sharing no variable with a group taken before; at most
                // AD_GROUPS_MAX, each of at most 64 listed variables
                std::vector<int> pos_of(n, -1), grp(k, -1);
                for (int t = 0; t < k; ++t) {
                    if (pos_of[sc[t]] >= 0)
                        return fail(CUBICS_EINVAL, "constraint %d: LINEAR_LE_AD scope repeats variable %d", c, sc[t]);
                    pos_of[sc[t]] = t;
                }
                std::vector<std::vector<int>> groups;
                for (int c2 = 0; c2 < m && (int)groups.size() < AD_GROUPS_MAX; ++c2) {
                    if (type[c2] != CUBICS_ALLDIFF && type[c2] != CUBICS_ALLDIFF_GAC) continue;
                    const int k2 = arity[c2];
                    if (k2 < 1 || k2 > 64 || var_off[c2 + 1] - var_off[c2] != k2) continue;
                    const int32_t *s2 = vars + var_off[c2];
                    std::vector<int> pos;
                    bool ok = true;
                    for (int u = 0; u < k2 && ok; ++u) {
                        const int t = (s2[u] >= 0 && s2[u] < n) ? pos_of[s2[u]] : -1;
                        ok = t >= 0 && grp[t] < 0;
                        if (ok && std::find(pos.begin(), pos.end(), t) == pos.end()) pos.push_back(t);
                    }
                    if (!ok) continue;
                    for (int t : pos) grp[t] = (int)groups.size();
                    groups.push_back(pos);
                }
                for (int t = 0; t < k; ++t) gscope.push_back(grp[t]);
                gcoef.push_back((int64_t)groups.size());
                for (const std::vector<int> &pos : groups) {
                    int base = lo[sc[pos[0]]];
                    std::vector<int64_t> a;
                    for (int t : pos) {
                        base = std::min(base, (int)lo[sc[t]]);
                        a.push_back(par[1 + t]);
                        gscope.push_back(t);
                    }
                    std::sort(a.begin(), a.end(), std::greater<int64_t>());
                    gcoef.push_back(base);
                    gcoef.push_back((int64_t)pos.size());
                    gcoef.insert(gcoef.end(), a.begin(), a.end());
                }
            }
            gdesc.push_back(g);
            if (gdesc.size() > 65535) return fail(CUBICS_EUNSUPPORTED, "more than 65535 global constraints");
        } else {
            return fail(CUBICS_EINVAL, "constraint %d: unknown type %d", c, ty);
        }
    }

    // ---- units sorted by source variable (stable), trigger ranges
    std::vector<int32_t> trig_off(n + 1, 0);
    for (const Unit &u : units) trig_off[u.src + 1]++;
    for (int i = 0; i < n; ++i) trig_off[i + 1] += trig_off[i];
    std::vector<Unit> sorted(units.size());
    {
        std::vector<int32_t> fill(trig_off.begin(), trig_off.end() - 1);
        for (const Unit &u : units) sorted[fill[u.src]++] = u;
    }
    // ---- global trigger lists
    std::vector<int32_t> gtrig_off(n + 1, 0), gtrig;
    for (size_t g = 0; g < gdesc.size(); ++g)
        for (int t = 0; t < gdesc[g].k; ++t) gtrig_off[gscope[gdesc[g].scope_off + t] + 1]++;
    for (int i = 0; i < n; ++i) gtrig_off[i + 1] += gtrig_off[i];
    gtrig.resize(std::max<size_t>(gtrig_off[n], 1));
    {
        std::vector<int32_t> fill(gtrig_off.begin(), gtrig_off.end() - 1);
        for (size_t g = 0; g < gdesc.size(); ++g)
            for (int t = 0; t < gdesc[g].k; ++t) {
                const int v = gscope[gdesc[g].scope_off + t];
                gtrig[fill[v]++] = (int32_t)g;
            }
    }
    // ---- static features of the learned policy: degree/(n-1), mean
    // tightness of the variable's constraints, 1/dsize
    std::vector<float> feat(4 * (size_t)std::max(n, 1), 0.f);
    for (int i = 0; i < n; ++i) {
        feat[4 * i] = n > 1 ? (float)deg[i] / (float)(n - 1) : 0.f;
        feat[4 * i + 1] = deg[i] ? (float)(tight_sum[i] / deg[i]) : 0.f;
        feat[4 * i + 2] = 1.f / (float)dsize[i];
    }

    // ---- VAR layout (one lane per variable): dense pair matrix of units,
    // row stride 64, one packed word per entry
    bool var_ok = n >= 1 && n <= 64 && W == 1 && gdesc.empty();
    std::vector<uint32_t> pairs;
    if (var_ok) {
        pairs.assign((size_t)n * 64, 0u);
        const int32_t P28 = 1 << 27;  // parameters are 28-bit signed
        for (const Unit &u : sorted) {
            const int t = u.tt & 0xFFFFFF, ty = u.tt >> 24, j = u.src;
            uint32_t &e = pairs[(size_t)j * 64 + t];
            if (e != 0u) { var_ok = false; break; }  // two constraints on one pair
            uint32_t prm = 0;
            if (ty == U_QUEENS) {
                if (u.p0 < 0 || u.p0 >= (1 << 13) || u.p1 < -(1 << 14) || u.p1 >= (1 << 14)) { var_ok = false; break; }
                prm = ((uint32_t)u.p0 << 15) | ((uint32_t)u.p1 & 0x7FFFu);
            } else {
                const int32_t v = ty == U_TABLE ? u.p1 : u.p0;
                if (v < -P28 || v >= P28) { var_ok = false; break; }
                prm = (uint32_t)v & 0x0FFFFFFFu;
            }
            e = ((uint32_t)ty << 28) | prm;
        }
    }
    if (!var_ok) pairs.assign(1, 0u);

    // ---- pack and upload
    Packer pk;
    std::vector<int32_t> lov(lo, lo + n);
    if (lov.empty()) lov.push_back(0);
    const size_t o_lo = pk.add(lov.data(), lov.size() * 4);
    const size_t o_dom0 = pk.add(dom0.data(), dom0.size() * 4);
    const size_t o_trig = pk.add(trig_off.data(), trig_off.size() * 4);
    const size_t o_units = pk.add(sorted.data(), std::max<size_t>(sorted.size(), 1) * sizeof(Unit));
    rows.insert(rows.begin(), ROW_PRE, 0u);
    const size_t o_rows = pk.add(rows.data(), rows.size() * 4) + 4 * ROW_PRE;
    const size_t o_gto = pk.add(gtrig_off.data(), gtrig_off.size() * 4);
    const size_t o_gt = pk.add(gtrig.data(), gtrig.size() * 4);
    const size_t o_gd = pk.add(gdesc.data(), std::max<size_t>(gdesc.size(), 1) * sizeof(GDesc));
    if (gscope.empty()) gscope.push_back(0);
    const size_t o_gs = pk.add(gscope.data(), gscope.size() * 4);
    if (gcoef.empty()) gcoef.push_back(0);
    const size_t o_gc = pk.add(gcoef.data(), gcoef.size() * 8);
    if (unary.empty()) { unary.push_back(0); unary.push_back(0); }
    const size_t o_un = pk.add(unary.data(), unary.size() * 4);
    const size_t o_ft = pk.add(feat.data(), feat.size() * 4);
    const size_t o_pairs = pk.add(pairs.data(), pairs.size() * 4);
    pk.add(nullptr, 0, 16);
    pk.bytes.resize((pk.bytes.size() + 15) / 16 * 16, 0);

    HIPCHK(hipSetDevice(ctx->device));
    void *blob = nullptr;
    if (hipMalloc(&blob, pk.bytes.size()) != hipSuccess)
        return fail(CUBICS_ENOMEM, "hipMalloc(%zu) for the problem failed", pk.bytes.size());
    hipError_t e = hipMemcpyAsync(blob, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(blob);
        return fail(CUBICS_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    cubics_prob *p = new cubics_prob();
    p->ctx = ctx;
    p->blob = blob;
    p->n = n;
    p->W = W;
    p->dmax = dmax;
    p->n_units = (int)sorted.size();
    p->n_glob = (int)gdesc.size();
    p->has_table = has_table;
    p->has_gac = has_gac;
    p->last_lin_b = last_lin_b;
    for (int i = 0; i < n; ++i) p->dsum += dsize[i] - 1;
    char *b8 = (char *)blob;
    InstDev &I = p->dev;
    memset(&I, 0, sizeof I);
    I.n = n;
    I.W = W;
    int S = 8;
    while (S < dmax && S < 64) S *= 2;
    I.S = S;
    I.dmax = dmax;
    I.n_units = p->n_units;
    I.n_glob = p->n_glob;
    {
        int nu = 0;
        for (int c = 0; c < m; ++c) nu += type[c] == CUBICS_UNARY;
        I.n_unary = nu;
    }
    I.seg_ok = (dmax <= 64) ? 1 : 0;
    I.lo = (const int32_t *)(b8 + o_lo);
    I.dom0 = (const uint32_t *)(b8 + o_dom0);
    I.trig_off = (const int32_t *)(b8 + o_trig);
    I.units = (const Unit *)(b8 + o_units);
    I.rows = (const uint32_t *)(b8 + o_rows);
    I.gtrig_off = (const int32_t *)(b8 + o_gto);
    I.gtrig = (const int32_t *)(b8 + o_gt);
    I.gdesc = (const GDesc *)(b8 + o_gd);
    I.gscope = (const int32_t *)(b8 + o_gs);
    I.gcoef = (const int64_t *)(b8 + o_gc);
    I.unary = (const int32_t *)(b8 + o_un);
    I.feat_static = (const float *)(b8 + o_ft);
    I.pairs = (const uint32_t *)(b8 + o_pairs);
    I.var_ok = var_ok ? 1 : 0;
    I.unit_types = 0;
    for (const Unit &u : sorted) I.unit_types |= 1 << (u.tt >> 24);
    I.blob = (const uint32_t *)blob;
    I.blob_words = (uint32_t)((pk.bytes.size() + 15) / 16 * 4);
    char key[160];
    snprintf(key, sizeof key, "W%d_d%d_n%d_g%d_t%d", W, (dmax + 7) / 8 * 8, (n + 15) / 16 * 16,
             p->n_glob > 0, has_table ? 1 : 0);
    p->bucket = key;
    *out = p;
    return CUBICS_OK;
}

extern "C" void cubics_free(cubics_prob *p) {
    if (!p) return;
    if (p->blob) {
        (void)hipSetDevice(p->ctx->device);
        (void)hipFree(p->blob);
    }
    delete p;
}

extern "C" int cubics_prob_info(const cubics_prob *p, int32_t *n, int32_t *W, int32_t *n_units, int32_t *n_global) {
    if (!p) return fail(CUBICS_EINVAL, "prob is NULL");
    if (n) *n = p->n;
    if (W) *W = p->W;
    if (n_units) *n_units = p->n_units;
    if (n_global) *n_global = p->n_glob;
    return CUBICS_OK;
}

// ------------------------------------------------------------ solve support
int policy_fill(const cubics_policy *pol, PolicyDev *out);

// ---- static scratch of the allocation-free batch solve
// The buffers of one cubics_solve_batch_static launch (instance descriptors,
// per-instance counters, the work queue and the workers' trail stacks) are
// carved out of this array.  Each GPU the library runs on holds its own copy
// from the first use until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels and copies get the device
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t CUBICS_STATIC_SCRATCH_BYTES = (size_t)CUBICS_STATIC_SCRATCH_MIB << 20;
static __device__ __align__(256) uint8_t scratch[CUBICS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on `device` (which must be current),
// looked up once per device.
int scratch_address(int device, uint8_t **out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(CUBICS_EUNSUPPORTED, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(CUBICS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[device] = (uint8_t *)ptr;
    }
    *out = g_scratch_ptr[device];
    return CUBICS_OK;
}
}  // namespace

namespace {

int pow2_ge(int x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

struct Geometry {
    int nmax = 1, wmax = 1, gmax = 0;
    int lds_words = 0;
    bool gac = false;
};

Geometry geometry(cubics_prob *const *probs, int B) {
    Geometry g;
    int wm = 1;
    for (int b = 0; b < B; ++b) {
        g.nmax = std::max(g.nmax, probs[b]->n);
        wm = std::max(wm, probs[b]->W);
        g.gmax = std::max(g.gmax, probs[b]->n_glob);
        g.gac |= probs[b]->has_gac;
    }
    g.wmax = wm <= 1 ? 1 : wm <= 2 ? 2 : wm <= 4 ? 4 : 8;
    const int ndw = (g.nmax + 63) / 64, ngw = std::max((g.gmax + 63) / 64, 1);
    int words = ((g.nmax * g.wmax) + 1) & ~1;
    words += 2 * ndw + 2 * ndw + 2 * ngw + ((g.nmax + 1) & ~1) + ((g.nmax + 2) & ~1) +
             (g.gac ? SCRATCH_GAC_WORDS : SCRATCH_WORDS);
    g.lds_words = (words + 1) & ~1;
    return g;
}

int choose_layout(cubics_prob *const *probs, int B, int requested) {
    if (requested == CUBICS_LAYOUT_LANE || requested == CUBICS_LAYOUT_SEG || requested == CUBICS_LAYOUT_VAR)
        return requested;
    // AUTO: the autotuned choice of the first instance's shape bucket, else a
    // rule: registers when the instance is small enough, lane-per-value
    // segments once domains are wide
    cubics_ctx *ctx = probs[0]->ctx;
    auto it = ctx->tuned.find(probs[0]->bucket);
    if (it != ctx->tuned.end()) return it->second.layout;
    int dmax = 1;
    bool seg_ok = true, var_ok = true;
    for (int b = 0; b < B; ++b) {
        dmax = std::max(dmax, probs[b]->dmax);
        seg_ok &= probs[b]->dmax <= 64;
        var_ok &= probs[b]->dev.var_ok != 0;
    }
    // registers pay off when the pair matrix and rows are staged in LDS (one
    // instance); from HBM every dirty-variable step waits on a global load
    if (var_ok && B == 1 && probs[0]->dev.blob_words * 4 <= 48 * 1024) return CUBICS_LAYOUT_VAR;
    return (seg_ok && dmax > 24) ? CUBICS_LAYOUT_SEG : CUBICS_LAYOUT_LANE;
}

}  // namespace

// worker_div > 0: use the occupancy-limited worker count divided by it (the
// autotuner's candidates); 0: the caller's count, else the autotuned one for
// an AUTO layout, else the maximum.
// static_scratch: take every device buffer from the static scratch array
// (no allocation; the worker count shrinks until the launch fits).
static int solve_impl(cubics_prob *const *probs, int B, int mode, const cubics_limits *lims,
                      cubics_result *results, int worker_div = 0, bool static_scratch = false) {
    auto t0 = std::chrono::steady_clock::now();
    if (!probs || B < 1 || !results) return fail(CUBICS_EINVAL, "bad batch arguments");
    if (mode < 0 || mode > 2) return fail(CUBICS_EINVAL, "bad mode %d", mode);
    for (int b = 0; b < B; ++b)
        if (!probs[b]) return fail(CUBICS_EINVAL, "prob[%d] is NULL", b);
    cubics_ctx *ctx = probs[0]->ctx;
    for (int b = 1; b < B; ++b)
        if (probs[b]->ctx->device != ctx->device) return fail(CUBICS_EINVAL, "problems on different devices");
    cubics_limits dflt;
    memset(&dflt, 0, sizeof dflt);
    dflt.donate = 1;
    const cubics_limits &L0 = lims ? lims[0] : dflt;
    if (L0.value_policy && L0.two_way)
        return fail(CUBICS_EINVAL, "a learned value order applies to d-way branching (two_way = 0)");
    if (L0.value_policy && (L0.trace_buf || L0.trace_capacity))
        return fail(CUBICS_EINVAL, "a learned value order cannot be combined with trace recording");
    if (L0.branching == CUBICS_BRANCH_LEARNED && !L0.policy)
        return fail(CUBICS_EINVAL, "LEARNED branching needs a policy");
    if (L0.two_way != 0 && L0.two_way != 1) return fail(CUBICS_EINVAL, "two_way must be 0 or 1");
    if (L0.branching != CUBICS_BRANCH_FIRST_FAIL && L0.branching != CUBICS_BRANCH_LEARNED)
        return fail(CUBICS_EINVAL, "bad branching %d", L0.branching);
    if (L0.split_target < 0 || L0.time_ms < 0 || L0.workers < 0)
        return fail(CUBICS_EINVAL, "negative split_target / time_ms / workers");
    for (int b = 0; b < B; ++b) {
        const cubics_limits &Lb = lims ? lims[b] : dflt;
        if (Lb.sol_capacity > 0 && !Lb.sol_buf) return fail(CUBICS_EINVAL, "sol_capacity > 0 with NULL sol_buf");
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (L0.use_graph && st == nullptr) {
        // the null stream cannot be captured: use a blocking stream of the
        // context (it still orders with the null stream)
        if (!ctx->graph_stream) HIPCHK(hipStreamCreate(&ctx->graph_stream));
        st = ctx->graph_stream;
    }
    const Geometry G = geometry(probs, B);
    const int layout = choose_layout(probs, B, L0.layout);
    // trail frames a path can need: one per branching plus a task's frame 0.
    // d-way assigns a variable per branching (<= n + 1 frames); 2-way may
    // branch on a variable again after x != a, at most dsize - 1 times
    int64_t frames = G.nmax + 1;
    if (L0.two_way) {
        frames = 2;
        for (int b = 0; b < B; ++b) frames = std::max<int64_t>(frames, 1 + probs[b]->dsum);
    }

    // ---- workers: fill the device with co-resident wavefronts.  A single
    // instance whose packed tables fit is staged in LDS once per workgroup;
    // the register-resident VAR path uses 8 workers per workgroup to share it.
    const size_t LDS_WG_MAX = (size_t)ctx->lds_max - 256;  // the kernel keeps a few static words
    const bool vorder = L0.value_policy != nullptr;
    if (vorder && G.wmax > 2)
        return fail(CUBICS_EUNSUPPORTED, "a learned value order needs domains of at most 64 values");
    const int feat = (L0.trace_buf && L0.trace_capacity > 0)
                         ? 2
                         : ((L0.branching == CUBICS_BRANCH_LEARNED || vorder) ? 1 : 0);
    bool var_all = G.wmax == 1;
    for (int b = 0; b < B && var_all; ++b) var_all = probs[b]->dev.var_ok != 0;
    // (the VAR layout keeps the frames' meta in lane registers: 64 frames)
    const bool use_var = feat == 0 && layout == CUBICS_LAYOUT_VAR && var_all && frames <= 64;
    const int variant = search_variant(feat, G.gmax > 0, layout == CUBICS_LAYOUT_SEG, use_var);
    int wpb = use_var ? 8 : 4;
    // learned search: each worker also keeps its task's static features [n][4]
    // (placed before the scratch words, which stay last)
    const int lds_words = G.lds_words + (feat == 1 ? 4 * G.nmax + (vorder ? VALUE_LDS_WORDS : 0) : 0);
    const size_t per_wave = (size_t)lds_words * 4;
    const size_t pol_bytes = feat == 1 ? 2 * (size_t)POLICY_LDS_WORDS * 4 : 0;  // network copies
    const size_t tab_bytes = (B == 1) ? (size_t)probs[0]->dev.blob_words * 4 : 0;
    bool tl = B == 1 && L0.tables_in_lds != 2 && tab_bytes + pol_bytes + per_wave <= LDS_WG_MAX;
    size_t lds = (tl ? tab_bytes : 0) + pol_bytes + per_wave * wpb;
    while (wpb > 1 && lds > LDS_WG_MAX) {
        wpb /= 2;
        lds = (tl ? tab_bytes : 0) + pol_bytes + per_wave * wpb;
    }
    if (lds > LDS_WG_MAX) return fail(CUBICS_EUNSUPPORTED, "instance needs %zu bytes of LDS per worker", per_wave);
    int bpc = 0;
    HIPCHK(search_occupancy(G.wmax, &bpc, wpb, lds, tl, variant));
    if (bpc < 1) bpc = 1;
    int div = 1;
    // instances active per XCD ring: the caller's, else (0) the autotuned
    // one for an AUTO layout, else (-1, or nothing tuned) one queue
    int gang = L0.active_per_xcd;
    if (worker_div > 0) {
        div = worker_div;
    } else if (L0.layout == CUBICS_LAYOUT_AUTO) {
        auto it = ctx->tuned.find(probs[0]->bucket);
        if (it != ctx->tuned.end()) {
            div = it->second.div;
            if (gang == 0) gang = it->second.gang;
        }
    }
    if (gang < 0) gang = 0;
    int nworkers = L0.workers > 0 && worker_div == 0 ? L0.workers : std::max(1, bpc * wpb * ctx->cu_count / div);

    // ---- buffers
    // a frame under the learned value order also keeps its values' score keys
    const uint32_t frame_words =
        (uint32_t)((FRAME_HDR + G.nmax * G.wmax + 15) / 16 * 16) + (vorder ? FRAME_SCORES : 0);
    const uint32_t slot_words = (uint32_t)((SLOT_HDR + G.nmax * G.wmax + 15) / 16 * 16);
    const int64_t trail_words64 = (int64_t)frame_words * frames;
    if (trail_words64 > (1LL << 28))
        return fail(CUBICS_EUNSUPPORTED, "a worker's trail would need %lld frames of %u words", (long long)frames,
                    frame_words);
    const uint32_t trail_words = (uint32_t)trail_words64;
    // at most 16 GiB of trail stacks: fewer workers for very deep trails
    nworkers = (int)std::min<int64_t>(nworkers, std::max<int64_t>(1, (16LL << 30) / (4 * trail_words64)));
    // one ring per XCD for a batch when asked for (active_per_xcd > 0) and
    // every ring gets workgroups; else one ring holding every instance
    const auto ring_count = [&](int nw_) {
        return (gang > 0 && B > MAX_RINGS && (nw_ + wpb - 1) / wpb >= MAX_RINGS) ? MAX_RINGS : 1;
    };
    // queue cells per ring for the workers' donations and the eager split
    const auto queue_cells = [&](int nw_) {
        const int R = ring_count(nw_);
        const long long roots = R == 1 ? B : std::min<long long>(B, gang);
        long long want = roots + 2LL * ((nw_ + R - 1) / R) + 2LL * L0.split_target + 1024;
        if (want > (1LL << 26)) want = 1LL << 26;
        uint32_t c = 4096;
        while ((long long)c < want) c *= 2;
        return c;
    };
    const auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    // bytes of the launch's buffers in the static scratch layout
    const auto static_bytes = [&](int nw_) {
        const size_t c = (size_t)queue_cells(nw_) * ring_count(nw_);
        return al(sizeof(InstDev) * (size_t)B) + al(sizeof(InstCtl) * (size_t)B) + al(sizeof(QBlock)) +
               al(4ull * c) + al(4ull * c * slot_words) + 4ull * trail_words * (size_t)nw_;
    };
    if (static_scratch) {
        if (static_bytes(1) > CUBICS_STATIC_SCRATCH_BYTES)
            return fail(CUBICS_EUNSUPPORTED, "the launch needs %zu bytes with one worker; the static scratch holds %zu",
                        static_bytes(1), CUBICS_STATIC_SCRATCH_BYTES);
        // the most workers whose trails fit (the count only shrinks)
        int lo_w = 1, hi_w = nworkers;
        while (lo_w < hi_w) {
            const int mid = lo_w + (hi_w - lo_w + 1) / 2;
            if (static_bytes(mid) <= CUBICS_STATIC_SCRATCH_BYTES) lo_w = mid;
            else hi_w = mid - 1;
        }
        nworkers = lo_w;
    }
    const int blocks = (nworkers + wpb - 1) / wpb;
    const uint32_t cap = queue_cells(nworkers);  // per ring
    const int nrings = ring_count(nworkers);
    const size_t cells = (size_t)cap * nrings;
    void *d_inst, *d_ctl, *d_q, *d_qseq, *d_qdata, *d_trail;
    int rc;
    if (static_scratch) {
        uint8_t *base = nullptr;
        if ((rc = scratch_address(ctx->device, &base))) return rc;
        size_t off = 0;
        const auto take = [&](size_t bytes) {
            void *p_ = base + off;
            off += al(bytes);
            return p_;
        };
        d_inst = take(sizeof(InstDev) * (size_t)B);
        d_ctl = take(sizeof(InstCtl) * (size_t)B);
        d_q = take(sizeof(QBlock));
        d_qseq = take(4ull * cells);
        d_qdata = take(4ull * cells * slot_words);
        d_trail = take(4ull * trail_words * (size_t)nworkers);
    } else {
        if ((rc = ctx->inst.ensure(sizeof(InstDev) * (size_t)B))) return rc;
        if ((rc = ctx->ctl.ensure(sizeof(InstCtl) * (size_t)B))) return rc;
        if ((rc = ctx->q.ensure(sizeof(QBlock)))) return rc;
        if ((rc = ctx->qseq.ensure(4ull * cells))) return rc;
        if ((rc = ctx->qdata.ensure(4ull * cells * slot_words))) return rc;
        if ((rc = ctx->trail.ensure(4ull * trail_words * (size_t)nworkers))) return rc;
        d_inst = ctx->inst.p;
        d_ctl = ctx->ctl.p;
        d_q = ctx->q.p;
        d_qseq = ctx->qseq.p;
        d_qdata = ctx->qdata.p;
        d_trail = ctx->trail.p;
    }

    std::vector<InstDev> inst(B);
    for (int b = 0; b < B; ++b) {
        const cubics_limits &Lb = lims ? lims[b] : dflt;
        inst[b] = probs[b]->dev;
        inst[b].sol_buf = Lb.sol_buf;
        inst[b].sol_cap = Lb.sol_buf ? Lb.sol_capacity : 0;
        inst[b].max_nodes = Lb.max_nodes;
        inst[b].max_solutions = Lb.max_solutions;
        if (mode == CUBICS_MODE_FIRST && inst[b].sol_cap > 1) inst[b].sol_cap = 1;
    }
    HIPCHK(hipMemcpyAsync(d_inst, inst.data(), sizeof(InstDev) * B, hipMemcpyHostToDevice, st));

    SearchParams P;
    memset(&P, 0, sizeof P);
    P.inst = (const InstDev *)d_inst;
    P.ctl = (InstCtl *)d_ctl;
    P.B = B;
    P.mode = mode;
    P.layout = layout;
    P.branching = L0.branching;
    P.two_way = L0.two_way;
    P.qb = (QBlock *)d_q;
    P.q = &P.qb->ring[0];
    P.g = &P.qb->g;
    P.nrings = nrings;
    P.seeded = nrings > 1 ? gang : B;
    P.qseq = (uint32_t *)d_qseq;
    P.qdata = (uint32_t *)d_qdata;
    P.qmask = cap - 1;
    P.slot_words = slot_words;
    P.trail = (uint32_t *)d_trail;
    P.frame_words = frame_words;
    P.trail_words = trail_words;
    P.max_frames = (int32_t)frames;
    P.nworkers = nworkers;
    P.donate = L0.donate ? 1 : 0;
    P.split_target = L0.split_target;
    P.time_ticks = L0.time_ms > 0 ? (long long)L0.time_ms * ctx->wall_khz : 0;
    P.cancel = ctx->cancel_host;
    P.lds_words = lds_words;
    P.nmax = G.nmax;
    P.wmax = G.wmax;
    P.gmax = G.gmax;
    if (L0.policy) policy_fill(L0.policy, &P.policy);
    if (vorder) {
        policy_fill(L0.value_policy, &P.vpolicy);
        P.value_order = 1;
    }
    if (L0.trace_buf && L0.trace_capacity > 0) {
        if ((rc = ctx->tracecnt.ensure(64))) return rc;
        P.trace_out = L0.trace_buf;
        P.trace_count = (unsigned long long *)ctx->tracecnt.p;
        P.trace_cap = L0.trace_capacity;
        P.explore_pm = L0.explore_pm;
        P.seed = L0.seed;
    }
    __atomic_store_n(ctx->cancel_host, 0, __ATOMIC_RELEASE);

    if (L0.use_graph) {
        // queue reset + persistent search as one captured graph, replayed for
        // every later solve with identical launch parameters (the instance
        // descriptors are re-uploaded above, outside the graph)
        std::string key((const char *)&P, sizeof P);
        const int dims[5] = {blocks, wpb, (int)lds, tl ? 1 : 0, G.wmax};
        key.append((const char *)dims, sizeof dims);
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t e1 = launch_init(P, st);
            hipError_t e2 = launch_search(G.wmax, P, blocks, wpb, lds, tl, variant, st);
            hipError_t e3 = hipStreamEndCapture(st, &graph);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(CUBICS_EDEVICE, "graph capture failed");
            }
            hipError_t e4 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e4 != hipSuccess) return fail(CUBICS_EDEVICE, "graph instantiation failed");
            it = ctx->graphs.emplace(key, exec).first;
        }
        HIPCHK(hipEventRecord(ctx->ev0, st));
        HIPCHK(hipGraphLaunch(it->second, st));
        HIPCHK(hipEventRecord(ctx->ev1, st));
    } else {
        HIPCHK(launch_init(P, st));
        HIPCHK(hipEventRecord(ctx->ev0, st));
        HIPCHK(launch_search(G.wmax, P, blocks, wpb, lds, tl, variant, st));
        HIPCHK(hipEventRecord(ctx->ev1, st));
    }
    std::vector<InstCtl> ctl(B);
    QGlobal qh;
    unsigned long long ntraces = 0;
    if (P.trace_out) HIPCHK(hipMemcpyAsync(&ntraces, ctx->tracecnt.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctl.data(), d_ctl, sizeof(InstCtl) * B, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&qh, &((QBlock *)d_q)->g, sizeof(QGlobal), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float kms = 0.f;
    HIPCHK(hipEventElapsedTime(&kms, ctx->ev0, ctx->ev1));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

    for (int b = 0; b < B; ++b) {
        const cubics_limits &Lb = lims ? lims[b] : dflt;
        const InstCtl &c = ctl[b];
        cubics_result &r = results[b];
        memset(&r, 0, sizeof r);
        r.nodes = c.nodes;
        r.fails = c.fails;
        r.revisions = c.revisions;
        r.steals = c.steals;
        r.alg_bytes = c.alg_bytes;
        r.tasks = c.tasks;
        r.ms = ms;
        r.kernel_ms = kms;
        r.traces = std::min<unsigned long long>(ntraces, P.trace_cap);
        if (qh.stop_reason == 4) return fail(CUBICS_EDEVICE, "internal error: trail overflow");
        const bool stopped = qh.stop != 0;
        const int stop_verdict = qh.stop_reason == 3 ? CUBICS_CANCELLED : CUBICS_LIMIT;
        if (mode == CUBICS_MODE_FIRST) {
            if (c.found) {
                r.verdict = CUBICS_SAT;
                r.count = 1;
                r.n_written = inst[b].sol_cap > 0 ? 1 : 0;
            } else if (c.reason == 2) {
                r.verdict = CUBICS_LIMIT;
            } else if (stopped) {
                r.verdict = stop_verdict;
            } else {
                r.verdict = CUBICS_UNSAT;
            }
        } else {
            uint64_t count = c.count + c.n_slots;
            r.n_written = std::min<uint64_t>(c.n_slots, inst[b].sol_cap);
            r.truncated = (inst[b].sol_cap > 0 && c.n_slots > inst[b].sol_cap) ? 1 : 0;
            if (c.reason == 3 || (Lb.max_solutions && count >= Lb.max_solutions)) {
                count = std::min<uint64_t>(count, Lb.max_solutions);
                r.verdict = CUBICS_LIMIT;
            } else if (c.reason == 2) {
                r.verdict = CUBICS_LIMIT;
            } else if (stopped) {
                r.verdict = stop_verdict;
            } else {
                r.verdict = count > 0 ? CUBICS_SAT : CUBICS_UNSAT;
            }
            r.count = count;
        }
    }
    return CUBICS_OK;
}

extern "C" int cubics_autotune(cubics_prob *const *probs, int32_t B, int32_t mode, const cubics_limits *limits,
                               int64_t time_ms, int32_t *chosen, int32_t *chosen_div, int32_t *chosen_active,
                               double *rates) {
    if (!probs || B < 1 || !probs[0] || time_ms < 1) return fail(CUBICS_EINVAL, "bad autotune arguments");
    bool seg_ok = true, var_ok = true;
    for (int b = 0; b < B; ++b) {
        if (!probs[b]) return fail(CUBICS_EINVAL, "prob[%d] is NULL", b);
        seg_ok &= probs[b]->dmax <= 64;
        var_ok &= probs[b]->dev.var_ok != 0;
    }
    std::vector<cubics_limits> lim(B);
    for (int b = 0; b < B; ++b) {
        if (limits) lim[b] = limits[b];
        else { memset(&lim[b], 0, sizeof(cubics_limits)); lim[b].donate = 1; }
        lim[b].sol_buf = nullptr;
        lim[b].sol_capacity = 0;
        lim[b].trace_buf = nullptr;
        lim[b].trace_capacity = 0;
        lim[b].use_graph = 0;
    }
    lim[0].time_ms = time_ms;
    lim[0].active_per_xcd = -1;  // layouts and worker counts are compared on one queue
    std::vector<cubics_result> res(B);
    if (rates)
        for (int k = 0; k < 3 * CUBICS_AUTOTUNE_DIVS; ++k) rates[k] = 0.0;
    cubics_ctx::Tuned best = {CUBICS_LAYOUT_LANE, 1, 0};
    const int tune_mode = mode == CUBICS_MODE_FIRST ? CUBICS_MODE_FIRST : CUBICS_MODE_COUNT;
    double best_rate = -1.0;
    int cands[3], nc = 0;
    cands[nc++] = CUBICS_LAYOUT_LANE;
    if (seg_ok) cands[nc++] = CUBICS_LAYOUT_SEG;
    if (var_ok) cands[nc++] = CUBICS_LAYOUT_VAR;
    static const int divs[CUBICS_AUTOTUNE_DIVS] = {1, 2, 4};
    for (int ci = 0; ci < nc; ++ci) {
        lim[0].layout = cands[ci];
        for (int di = 0; di < CUBICS_AUTOTUNE_DIVS; ++di) {
            // a warm-up run, then the timed one
            for (int rep = 0; rep < 2; ++rep) {
                int rc = solve_impl(probs, B, tune_mode, lim.data(), res.data(), divs[di]);
                if (rc) return rc;
            }
            uint64_t nodes = 0;
            for (int b = 0; b < B; ++b) nodes += res[b].nodes;
            const double rate = (double)nodes / std::max(res[0].kernel_ms, 1e-3);
            if (rates) rates[(cands[ci] - 1) * CUBICS_AUTOTUNE_DIVS + di] = rate;
            // fewer workers must be clearly faster (5%) to win: rates within
            // run-to-run noise keep the fuller launch
            const double need = (best_rate > 0 && di > 0 && cands[ci] == best.layout) ? 1.05 : 1.0;
            if (rate > best_rate * need) {
                best_rate = rate;
                best = {cands[ci], divs[di], 0};
            }
        }
    }
    // batches: one ring per XCD with a few instances active on each, for
    // the chosen layout and worker count (5% better than one queue to win).
    // Rings pay off over a whole launch (their instances first spread over
    // an XCD's workers), so when every instance has a node budget each
    // candidate runs to completion instead of for time_ms.
    if (B > MAX_RINGS) {
        bool budgeted = true;
        for (int b = 0; b < B; ++b) budgeted &= lim[b].max_nodes > 0;
        static const int gangs[] = {-1, 4, 8, 16, 32};
        lim[0].layout = best.layout;
        if (budgeted) lim[0].time_ms = 0;
        double base_rate = 0.0;
        for (int g : gangs) {
            lim[0].active_per_xcd = g;
            for (int rep = 0; rep < (budgeted ? 1 : 2); ++rep) {
                int rc = solve_impl(probs, B, tune_mode, lim.data(), res.data(), best.div);
                if (rc) return rc;
            }
            uint64_t nodes = 0;
            for (int b = 0; b < B; ++b) nodes += res[b].nodes;
            const double rate = (double)nodes / std::max(res[0].kernel_ms, 1e-3);
            if (g < 0) {
                base_rate = best_rate = rate;
            } else if (rate > std::max(best_rate, 1.05 * base_rate)) {
                best_rate = rate;
                best.gang = g;
            }
        }
    }
    probs[0]->ctx->tuned[probs[0]->bucket] = best;
    if (chosen) *chosen = best.layout;
    if (chosen_div) *chosen_div = best.div;
    if (chosen_active) *chosen_active = best.gang;
    return CUBICS_OK;
}

extern "C" int cubics_solve(cubics_prob *prob, int32_t mode, const cubics_limits *limits, cubics_result *result) {
    if (!prob) return fail(CUBICS_EINVAL, "prob is NULL");
    cubics_prob *arr[1] = {prob};
    return solve_impl(arr, 1, mode, limits, result);
}

extern "C" int cubics_solve_batch(cubics_prob *const *probs, int32_t B, int32_t mode, const cubics_limits *limits,
                                  cubics_result *results) {
    return solve_impl(probs, B, mode, limits, results);
}

extern "C" int cubics_solve_batch_static(cubics_prob *const *probs, int32_t B, int32_t mode,
                                         const cubics_limits *limits, cubics_result *results) {
    if (limits && limits[0].use_graph)
        return fail(CUBICS_EINVAL, "cubics_solve_batch_static: use_graph is not available (a graph allocates)");
    if (limits && (limits[0].trace_buf || limits[0].trace_capacity))
        return fail(CUBICS_EINVAL, "cubics_solve_batch_static: trace recording is not available");
    return solve_impl(probs, B, mode, limits, results, 0, true);
}

extern "C" int cubics_features(cubics_prob *p, const uint32_t *dom_bits, int32_t depth, float *out) {
    if (!p || !out) return fail(CUBICS_EINVAL, "NULL argument");
    if (depth < 0) return fail(CUBICS_EINVAL, "negative depth");
    cubics_ctx *ctx = p->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const size_t n = (size_t)std::max(p->n, 0), nw = std::max<size_t>(n * p->W, 1);
    int rc;
    if ((rc = ctx->inst.ensure(sizeof(InstDev)))) return rc;
    if ((rc = ctx->rootout.ensure(nw * 4 + n * POLICY_F * 4 + 64))) return rc;
    if (n == 0) return CUBICS_OK;
    uint32_t *ddom = (uint32_t *)ctx->rootout.p;
    float *dout = (float *)((char *)ctx->rootout.p + nw * 4);
    HIPCHK(hipMemcpyAsync(ctx->inst.p, &p->dev, sizeof(InstDev), hipMemcpyHostToDevice, ctx->stream));
    if (dom_bits)
        HIPCHK(hipMemcpyAsync(ddom, dom_bits, n * p->W * 4, hipMemcpyHostToDevice, ctx->stream));
    else
        HIPCHK(hipMemcpyAsync(ddom, p->dev.dom0, n * p->W * 4, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(launch_features((const InstDev *)ctx->inst.p, ddom, depth, dout, (int)n, ctx->stream));
    HIPCHK(hipMemcpyAsync(out, dout, n * POLICY_F * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CUBICS_OK;
}

extern "C" int cubics_value_features(cubics_prob *p, const uint32_t *dom_bits, int32_t depth, int32_t x,
                                     float *out) {
    if (!p || !out) return fail(CUBICS_EINVAL, "NULL argument");
    if (depth < 0) return fail(CUBICS_EINVAL, "negative depth");
    if (x < 0 || x >= p->n) return fail(CUBICS_EINVAL, "variable %d out of range", x);
    if (p->W > 2) return fail(CUBICS_EUNSUPPORTED, "value features need domains of at most 64 values");
    cubics_ctx *ctx = p->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    const size_t n = (size_t)p->n, nw = n * p->W, nv = 32 * (size_t)p->W;
    int rc;
    if ((rc = ctx->inst.ensure(sizeof(InstDev)))) return rc;
    if ((rc = ctx->rootout.ensure(nw * 4 + nv * POLICY_F * 4 + 64))) return rc;
    uint32_t *ddom = (uint32_t *)ctx->rootout.p;
    float *dout = (float *)((char *)ctx->rootout.p + nw * 4);
    HIPCHK(hipMemcpyAsync(ctx->inst.p, &p->dev, sizeof(InstDev), hipMemcpyHostToDevice, ctx->stream));
    if (dom_bits)
        HIPCHK(hipMemcpyAsync(ddom, dom_bits, nw * 4, hipMemcpyHostToDevice, ctx->stream));
    else
        HIPCHK(hipMemcpyAsync(ddom, p->dev.dom0, nw * 4, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(launch_value_features((const InstDev *)ctx->inst.p, ddom, depth, x, dout, ctx->stream));
    HIPCHK(hipMemcpyAsync(out, dout, nv * POLICY_F * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CUBICS_OK;
}

extern "C" int cubics_root(cubics_prob *p, int32_t layout, uint32_t *out_bits, int32_t *failed) {
    if (!p || !out_bits || !failed) return fail(CUBICS_EINVAL, "NULL argument");
    cubics_ctx *ctx = p->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    cubics_prob *arr[1] = {p};
    const Geometry G = geometry(arr, 1);
    const size_t nw = (size_t)std::max(p->n, 1) * p->W;
    int rc;
    if ((rc = ctx->inst.ensure(sizeof(InstDev)))) return rc;
    if ((rc = ctx->rootout.ensure(nw * 4 + 64))) return rc;
    HIPCHK(hipMemcpyAsync(ctx->inst.p, &p->dev, sizeof(InstDev), hipMemcpyHostToDevice, ctx->stream));
    SearchParams P;
    memset(&P, 0, sizeof P);
    P.inst = (const InstDev *)ctx->inst.p;
    P.layout = choose_layout(arr, 1, layout);
    P.lds_words = G.lds_words;
    P.nmax = G.nmax;
    P.wmax = G.wmax;
    P.gmax = G.gmax;
    uint32_t *dout = (uint32_t *)ctx->rootout.p;
    int32_t *dfail = (int32_t *)((char *)ctx->rootout.p + nw * 4);
    unsigned long long *drev = (unsigned long long *)((char *)ctx->rootout.p + nw * 4 + 8);
    HIPCHK(launch_root(G.wmax, P, dout, dfail, drev, (size_t)G.lds_words * 4, ctx->stream));
    HIPCHK(hipMemcpyAsync(out_bits, dout, (size_t)p->n * p->W * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(failed, dfail, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return CUBICS_OK;
}

// ------------------------------------------------ large-neighbourhood search
//
// Minimise sum_i c_i x_i (c_i >= 0) over the solutions of a CSP: the
// instance is loaded once with one more constraint, sum c_i x_i <= UB, whose
// bound is rewritten in the device copy every round.  A round solves B
// neighbourhoods of the incumbent in one persistent launch (find-first, a
// node budget each): neighbourhood 0 frees every variable (its UNSAT proves
// the incumbent optimal), the others fix a random part of the variables to
// the incumbent's values.  All neighbourhoods share the packed constraints;
// only their initial domains differ.

namespace {
uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

extern "C" int cubics_lns(cubics_ctx *ctx, int32_t n, const int32_t *lo, const int32_t *dsize,
                          const uint32_t *init_bits, int32_t m, const int32_t *type, const int32_t *arity,
                          const int64_t *var_off, const int32_t *vars, const int64_t *par_off,
                          const int64_t *params, const int64_t *tab_off, const uint32_t *tabs,
                          const int64_t *obj, const cubics_lns_params *lp, int32_t *best,
                          cubics_lns_result *res) {
    auto t0 = std::chrono::steady_clock::now();
    if (!ctx || !obj || !lp || !best || !res) return fail(CUBICS_EINVAL, "NULL argument");
    if (n < 1) return fail(CUBICS_EINVAL, "n must be >= 1");
    if (lp->neighborhoods < 1 || lp->neighborhoods > 65536) return fail(CUBICS_EINVAL, "neighborhoods out of 1..65536");
    if (lp->relax_pm < 1 || lp->relax_pm > 1000) return fail(CUBICS_EINVAL, "relax_pm out of 1..1000");
    if (lp->rounds < 0 || lp->time_ms < 0) return fail(CUBICS_EINVAL, "negative rounds / time_ms");
    memset(res, 0, sizeof *res);
    // ---- the instance plus sum c_i x_i <= UB (variables with c_i > 0)
    std::vector<int32_t> ob_vars;
    std::vector<int64_t> ob_par(1, INT64_MAX / 4);
    for (int i = 0; i < n; ++i) {
        if (obj[i] < 0) return fail(CUBICS_EUNSUPPORTED, "objective coefficient %d is negative", i);
        if (obj[i] > 0) {
            ob_vars.push_back(i);
            ob_par.push_back(obj[i]);
        }
    }
    if (ob_vars.empty()) return fail(CUBICS_EINVAL, "the objective has no positive coefficient");
    const int M = m + 1, k = (int)ob_vars.size();
    std::vector<int32_t> ty(type, type + m), ar(arity, arity + m), vv(vars, vars + (m ? var_off[m] : 0));
    std::vector<int64_t> vo(var_off, var_off + m + 1), po(par_off, par_off + m + 1), pa(params, params + (m ? par_off[m] : 0));
    std::vector<int64_t> to(tab_off, tab_off + m + 1);
    if (m == 0) { vo.assign(1, 0); po.assign(1, 0); to.assign(1, 0); }
    ty.push_back(CUBICS_LINEAR_LE);
    ar.push_back(k);
    vv.insert(vv.end(), ob_vars.begin(), ob_vars.end());
    vo.push_back((int64_t)vv.size());
    pa.insert(pa.end(), ob_par.begin(), ob_par.end());
    po.push_back((int64_t)pa.size());
    to.push_back(to.back());
    cubics_prob *base = nullptr;
    int rc = cubics_load(ctx, n, lo, dsize, init_bits, M, ty.data(), ar.data(), vo.data(), vv.data(), po.data(),
                         pa.data(), to.data(), tabs, &base);
    if (rc) return rc;
    std::unique_ptr<cubics_prob, void (*)(cubics_prob *)> guard(base, cubics_free);
    const int W = base->W, B = lp->neighborhoods;
    int64_t *d_bound = (int64_t *)base->dev.gcoef + base->last_lin_b;
    std::vector<uint32_t> dom0((size_t)n * W);
    hipStream_t st = ctx->stream;  // every copy runs on the context's stream
    HIPCHK(hipMemcpyAsync(dom0.data(), base->dev.dom0, dom0.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if ((rc = ctx->lnsdom.ensure(4ull * (size_t)B * n * W))) return rc;
    if ((rc = ctx->lnssol.ensure(4ull * (size_t)B * n))) return rc;
    // neighbourhoods: views of the base problem with their own initial domains
    std::vector<cubics_prob> views(B, *base);
    std::vector<cubics_prob *> vp(B);
    for (int b = 0; b < B; ++b) {
        views[b].blob = nullptr;  // not owned
        views[b].dev.dom0 = (const uint32_t *)ctx->lnsdom.p + (size_t)b * n * W;
        vp[b] = &views[b];
    }
    std::vector<cubics_limits> lim(B);
    std::vector<cubics_result> out(B);
    std::vector<uint32_t> hdom((size_t)B * n * W);
    std::vector<int32_t> sols((size_t)B * n), cur(n);
    uint64_t rng = 0x5DEECE66Dull ^ ((uint64_t)lp->seed << 17);
    auto objective = [&](const int32_t *x) {
        int64_t f = 0;
        for (int i = 0; i < n; ++i) f += obj[i] * (int64_t)x[i];
        return f;
    };
    auto elapsed_ms = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    int64_t incumbent = 0;
    bool have = false;
    for (int round = 0;; ++round) {
        // bound: strictly better than the incumbent (none yet: unbounded)
        const int64_t ub = have ? incumbent - 1 : INT64_MAX / 4;
        HIPCHK(hipMemcpyAsync(d_bound, &ub, sizeof ub, hipMemcpyHostToDevice, st));
        const int nb = have ? B : 1;  // the first round looks for any solution
        for (int b = 0; b < nb; ++b) {
            uint32_t *d = hdom.data() + (size_t)b * n * W;
            memcpy(d, dom0.data(), dom0.size() * 4);
            if (b == 0) continue;  // neighbourhood 0: every variable free
            for (int i = 0; i < n; ++i) {
                if ((int)(splitmix(rng) % 1000ull) < lp->relax_pm) continue;  // freed
                const int a = cur[i] - lo[i];
                for (int w = 0; w < W; ++w) d[(size_t)i * W + w] = (w == a / 32) ? (1u << (a % 32)) : 0u;
            }
        }
        HIPCHK(hipMemcpyAsync(ctx->lnsdom.p, hdom.data(), 4ull * nb * n * W, hipMemcpyHostToDevice, st));
        // the host buffers are reused next round: wait for the copies
        HIPCHK(hipStreamSynchronize(st));
        for (int b = 0; b < nb; ++b) {
            memset(&lim[b], 0, sizeof(cubics_limits));
            lim[b].max_nodes = lp->max_nodes;
            lim[b].donate = 1;
            lim[b].sol_buf = (int32_t *)ctx->lnssol.p + (size_t)b * n;
            lim[b].sol_capacity = 1;
        }
        if (lp->time_ms > 0) lim[0].time_ms = std::max<int64_t>(1, lp->time_ms - (int64_t)elapsed_ms());
        if ((rc = solve_impl(vp.data(), nb, CUBICS_MODE_FIRST, lim.data(), out.data()))) return rc;
        HIPCHK(hipMemcpyAsync(sols.data(), ctx->lnssol.p, 4ull * nb * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        res->rounds = round + 1;
        int pick = -1;
        int64_t fbest = 0;
        for (int b = 0; b < nb; ++b) {
            res->nodes += out[b].nodes;
            if (out[b].verdict != CUBICS_SAT) continue;
            const int64_t f = objective(sols.data() + (size_t)b * n);
            if (pick < 0 || f < fbest) { pick = b; fbest = f; }
        }
        if (pick >= 0 && (!have || fbest < incumbent)) {
            memcpy(cur.data(), sols.data() + (size_t)pick * n, sizeof(int32_t) * n);
            if (have) res->improvements += 1;
            incumbent = fbest;
            have = true;
        }
        if (!have && out[0].verdict == CUBICS_UNSAT) break;        // the CSP has no solution
        if (have && round > 0 && out[0].verdict == CUBICS_UNSAT && pick < 0) {
            res->optimal = 1;  // no solution better than the incumbent exists
            break;
        }
        if (!have && out[0].verdict != CUBICS_SAT) break;         // no solution within the budget
        if (lp->rounds > 0 && round + 1 >= lp->rounds) break;
        if (lp->time_ms > 0 && elapsed_ms() >= lp->time_ms) break;
    }
    res->found = have ? 1 : 0;
    res->objective = incumbent;
    if (have) memcpy(best, cur.data(), sizeof(int32_t) * n);
    res->ms = elapsed_ms();
    return CUBICS_OK;
}
