// C ABI of the RaftGP hot path: argument checks, workspace planning and the
// stage sequence (projection -> GCN -> k-means grid -> scores -> selection).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/raftgp.h"
#include "kernels.h"

using namespace raft;

struct raft_ctx {
    int device = 0;
    void* scratch = nullptr;       // this device's copy of the fixed scratch array
    std::string autotune_cache;    // path of the tuner's cache file ("" = none)
    std::map<std::string, int> tuned;   // tuner choices: workload key -> choice
    int num_cu = 256;
    size_t lds_max = 65536;
    std::string err;
    int32_t* d_status = nullptr;   // device status word
    int32_t* h_pinned = nullptr;   // pinned host scratch (4096 ints)
    // pinned staging of raft_graph_create (row pointers, row order): grown on
    // demand; every use ends with a synchronisation of its stream, so no copy
    // from it is in flight when the next call regrows it
    char* stage = nullptr;
    size_t stage_bytes = 0;
    double stage_ms[5] = {0, 0, 0, 0, 0};
    hipEvent_t ev[6] = {};
    hipEvent_t poll_ev[2] = {};    // convergence polls of the Lloyd loop (no timing)
    // per-kernel-class event timing (raft_profile_enable)
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used = 0;
    std::vector<std::pair<int, size_t>> prof_recs;
    double prof_ms[RAFT_PROF_CLASSES] = {};
    int64_t prof_n[RAFT_PROF_CLASSES] = {};
};

struct raft_graph {
    raft_ctx* ctx = nullptr;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t* rp = nullptr;
    int32_t* ci = nullptr;
    int32_t* deg = nullptr;
    float* s = nullptr;
    float* sh = nullptr;
    float* dcoef = nullptr;
    int32_t* order = nullptr;   // rows by degree class, heaviest first (stable)
    // heavy[b]: the rows with at least b 16-edge batches (b <= 16; the last
    // class holds every longer row), which lead the order
    int32_t heavy[17] = {};
    bool owns = true;           // false: the arrays belong to a stream
    GraphView view() const {
        GraphView v;
        v.n = n;
        v.nnz = nnz;
        v.rp = rp;
        v.ci = ci;
        v.deg = deg;
        v.s = s;
        v.sh = sh;
        v.dcoef = dcoef;
        v.order = order;
        return v;
    }
};

void tuner_load(raft_ctx* ctx);   // reads the context's tuner cache file

// Fixed scratch for the allocation-free entry point (raft_spmm_noalloc):
// one copy of this array per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel: the device address of each
// GPU's copy is looked up once per device (hipGetSymbolAddress, with that
// device current) when the first context on it is created.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

namespace {

// Brackets one launch with a pair of pooled events when its class is enabled.
struct ProfScope {
    raft_ctx* c;
    int kind;
    hipStream_t st;
    size_t idx = (size_t)-1;
    ProfScope(raft_ctx* c_, int kind_, hipStream_t st_) : c(c_), kind(kind_), st(st_) {
        if (!(c->prof_mask & (1u << kind))) return;
        if (c->prof_used + 2 > c->prof_pool.size()) {
            for (int i = 0; i < 256; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                c->prof_pool.push_back(e);
            }
        }
        idx = c->prof_used;
        c->prof_used += 2;
        (void)hipEventRecord(c->prof_pool[idx], st);
    }
    ~ProfScope() {
        if (idx == (size_t)-1) return;
        (void)hipEventRecord(c->prof_pool[idx + 1], st);
        c->prof_recs.push_back({kind, idx});
    }
};

// An event pair for one kernel launch that records them itself (the launch
// packet's own start and end times, hipExtLaunchKernel): no extra packets
// between kernels, where a recorded event costs a few microseconds of gap.
// Null events when the class is not being profiled.
struct ProfLaunch {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfLaunch(raft_ctx* c, int kind) {
        if (!(c->prof_mask & (1u << kind))) return;
        if (c->prof_used + 2 > c->prof_pool.size()) {
            for (int i = 0; i < 256; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                c->prof_pool.push_back(e);
            }
        }
        const size_t idx = c->prof_used;
        c->prof_used += 2;
        e0 = c->prof_pool[idx];
        e1 = c->prof_pool[idx + 1];
        c->prof_recs.push_back({kind, idx});
    }
};

// Folds finished event pairs into the per-class totals (after a sync).
void prof_collect(raft_ctx* c) {
    for (auto& r : c->prof_recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->prof_pool[r.second], c->prof_pool[r.second + 1]) ==
            hipSuccess) {
            c->prof_ms[r.first] += ms;
            c->prof_n[r.first] += 1;
        }
    }
    c->prof_recs.clear();
    c->prof_used = 0;
}

raft_status fail(raft_ctx* ctx, raft_status code, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIP_TRY(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), RAFT_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define RAFT_TRY(call)                 \
    do {                               \
        raft_status s_ = (call);       \
        if (s_ != RAFT_OK) return s_;  \
    } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Feature widths: powers of two from 16 to 4096 (the paper's widths, Table I).
bool width_ok(int v) { return v >= 16 && v <= 4096 && (v & (v - 1)) == 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bump allocator over the caller's workspace (or a size-only dry run).
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += align256(count * sizeof(T));
        return p;
    }
};

struct Grid {
    std::vector<int32_t> ks, koff16, koff, cand_of;
    int Kc = 0, KP = 0, SK = 0, k_max = 0;
};

Grid make_grid(int k_min, int k_max, int k_step) {
    Grid g;
    for (int k = k_min; k <= k_max; k += k_step) g.ks.push_back(k);
    g.Kc = (int)g.ks.size();
    for (int k : g.ks) {
        g.koff16.push_back(g.KP);
        g.koff.push_back(g.SK);
        const int pad = (k + 15) / 16 * 16;
        for (int r = 0; r < pad; ++r) g.cand_of.push_back((int)g.koff16.size() - 1);
        g.KP += pad;
        g.SK += k;
        g.k_max = std::max(g.k_max, k);
    }
    return g;
}

// Work lists over the candidates still active: alist holds their ids;
// agrp splits alist into groups of about 256 padded centres (assignment),
// ugrp into groups whose clusters fit the update kernel's LDS budget.
struct Lists {
    std::vector<int32_t> alist, agrp, ugrp, uwi0, ulen, cranges;
    int uwork = 0;
};

// Length of the dynamic work lists (see pack_lists).
constexpr int kDynLen(int Kc) { return 6 * Kc + 3; }

// Point ranges per update group are capped so the partial buffers stay
// bounded, and at 256 so each of the finishing kernel's 4 waves folds at most
// 64 ranges (one per lane).
int update_ranges_max(int n, int num_cu) {
    return std::max(1, std::min(std::min(num_cu, 256), (n + 63) / 64));
}

Lists make_lists(const Grid& G, const int32_t* active, int ucap, int n, int num_cu) {
    Lists l;
    for (int k = 0; k < G.Kc; ++k)
        if (!active || active[k]) l.alist.push_back(k);
    l.agrp.push_back(0);
    int acc = 0;
    // groups of about 256 padded centres, at most kAssignMaxGroup
    // candidates (the assignment keeps a label row per candidate in LDS)
    int in_group = 0;
    for (size_t t = 0; t < l.alist.size(); ++t) {
        acc += (G.ks[l.alist[t]] + 15) / 16 * 16;
        ++in_group;
        if ((acc >= 256 || in_group == kAssignMaxGroup) && t + 1 < l.alist.size()) {
            in_group = 0;
            l.agrp.push_back((int32_t)t + 1);
            acc = 0;
        }
    }
    l.agrp.push_back((int32_t)l.alist.size());
    l.ugrp.push_back(0);
    acc = 0;
    int cnt = 0;
    for (size_t t = 0; t < l.alist.size(); ++t) {
        const int rows = kmeans_update_rows(G.ks[l.alist[t]]);
        if (cnt > 0 && (acc + rows > ucap || cnt >= kmeans_update_max_candidates())) {
            l.ugrp.push_back((int32_t)t);
            acc = 0;
            cnt = 0;
        }
        acc += rows;
        ++cnt;
    }
    l.ugrp.push_back((int32_t)l.alist.size());
    // work items: about 3 per CU in total, split over the groups in
    // proportion to their candidate counts (the update's work per point)
    const int ug = (int)l.ugrp.size() - 1;
    const int total_c = std::max<int>(1, (int)l.alist.size());
    const int max_r = update_ranges_max(n, num_cu);
    l.cranges.assign(G.Kc, 1);
    l.uwi0.push_back(0);
    for (int gi = 0; gi < ug; ++gi) {
        const int c = l.ugrp[gi + 1] - l.ugrp[gi];
        int r = (int)((3LL * num_cu * c) / total_c);
        r = std::max(1, std::min(r, max_r));
        const int len = ((n + r - 1) / r + 63) / 64 * 64;
        r = (n + len - 1) / len;
        l.ulen.push_back(len);
        l.uwi0.push_back(l.uwi0.back() + r);
        for (int t = l.ugrp[gi]; t < l.ugrp[gi + 1]; ++t) l.cranges[l.alist[t]] = r;
    }
    l.uwork = l.uwi0.back();
    return l;
}

// LDS budget of one update work-group: three work-groups per CU, as many as
// its registers allow (n50k: 47.4 -> 50.2 graphs/s against two of 72 KB;
// four of 36 KB: 49.4).
constexpr size_t kUpdateLdsBudget = 48 * 1024;

int update_cap(const Grid& G, int d) {
    const size_t fixed = kmeans_update_lds(0, d);
    const size_t per = kmeans_update_lds(1, d) - fixed;
    int most = 0;
    for (int k : G.ks) most = std::max(most, kmeans_update_rows(k));
    return std::max<int>(most, (int)((kUpdateLdsBudget - fixed) / per));
}

int embed_dim(const raft_config* c) {
    return c->n_layers > 0 ? c->layer_dims[c->n_layers - 1] : c->proj_dim;
}

int max_width(const raft_config* c) {
    int m = c->proj_dim;
    for (int k = 0; k < c->n_layers; ++k) m = std::max(m, c->layer_dims[k]);
    return m;
}

raft_status check_config(raft_ctx* ctx, const raft_graph* g, const raft_config* c) {
    if (!c) return fail(ctx, RAFT_E_INVAL, "config is null");
    if (c->abi_version != RAFT_ABI_VERSION)
        return fail(ctx, RAFT_E_INVAL, "abi_version %d != %d", c->abi_version, RAFT_ABI_VERSION);
    if (c->op < RAFT_X_NCUT || c->op > RAFT_X_MOD_REDUCED)
        return fail(ctx, RAFT_E_INVAL, "op %d not a projection operator", c->op);
    if (!width_ok(c->proj_dim)) return fail(ctx, RAFT_E_UNSUPPORTED, "proj_dim %d", c->proj_dim);
    if (c->q < 1) return fail(ctx, RAFT_E_INVAL, "q must be >= 1");
    if (c->n_layers < 0 || c->n_layers > RAFT_MAX_LAYERS)
        return fail(ctx, RAFT_E_INVAL, "n_layers %d", c->n_layers);
    int lin = c->proj_dim;
    for (int k = 0; k < c->n_layers; ++k) {
        if (!width_ok(c->layer_dims[k]) || !dense_supported(lin, c->layer_dims[k]))
            return fail(ctx, RAFT_E_UNSUPPORTED, "layer %d width %d", k + 1, c->layer_dims[k]);
        lin = c->layer_dims[k];
    }
    if (c->k_step < 1 || c->k_min < 1 || c->k_min > c->k_max || c->k_max > RAFT_MAX_K)
        return fail(ctx, RAFT_E_INVAL, "candidate grid %d..%d step %d", c->k_min, c->k_max,
                    c->k_step);
    if (g && c->k_max > g->n) return fail(ctx, RAFT_E_INVAL, "k_max %d exceeds N", c->k_max);
    if (c->kmeans_max_iter < 1) return fail(ctx, RAFT_E_INVAL, "kmeans_max_iter < 1");
    if (c->kmeans_prune < 0 || c->kmeans_prune > 2)
        return fail(ctx, RAFT_E_INVAL, "kmeans_prune %d (0, 1 or 2)", c->kmeans_prune);
    return RAFT_OK;
}

// Workspace layout shared by every staged call.
struct Plan {
    int L = 0, d = 0, Lmax = 0, spmm_grid_ = 0, score_grid_ = 0, S = 0, race_grid = 0;
    Grid grid;
    Lists lists;
    int ucap = 0;
    int ranges_max = 0;
    int share = 0;   // CUs the result-invariant shapes are sized for
    // projection / embedding
    float *y0, *y1, *pbuf, *yout, *zout, *wbuf;
    double *cpart, *c64;
    float* cvec;
    // k-means
    KmeansPlan km;
    int32_t* meta;   // ks, koff16, koff, cand_of, alist, agrp, ugrp packed
    int32_t* dyn;    // alist, agrp, ugrp (rewritten at convergence polls)
    // scores
    ScorePlan sc;
    uint8_t* lab_pm;
    double *mod_int, *ncut_int;
    int32_t* ksel_int;
    int32_t* picks_int;
    int32_t* iters_int;
    size_t bytes = 0;
};

// `features` = false leaves out the N x L feature buffers (a batch keeps them
// packed for all its graphs).  `share` (0 = every CU) is the number of CUs the
// result-invariant launch shapes are sized for: the update's point ranges, the
// edge-score and race grids.  Centre sums and score counts are exact integers
// and the race is a lexicographic argmin, so these shapes never change a
// result; a batch gives each graph a share of the chip (see the tuner).
void plan_layout(raft_ctx* ctx, const raft_graph* g, const raft_config* c, char* base, Plan& P,
                 bool features = true, int share = 0) {
    const int cu = share > 0 ? std::min(share, ctx->num_cu) : ctx->num_cu;
    P.share = cu;
    const int n = g->n;
    P.L = c->proj_dim;
    P.d = embed_dim(c);
    P.Lmax = max_width(c);
    P.grid = make_grid(c->k_min, c->k_max, c->k_step);
    P.spmm_grid_ = spmm_grid(n, P.Lmax, ctx->num_cu, nullptr);
    // every width uses the same grid formula (it does not depend on L)
    P.score_grid_ = score_grid(n, cu);
    P.S = (P.grid.Kc + 7) / 8 * 8;
    P.ucap = update_cap(P.grid, P.d);
    P.lists = make_lists(P.grid, nullptr, P.ucap, n, cu);
    P.race_grid = kmeans_race_grid(n, cu);
    Arena a;
    a.base = base;
    const size_t nL = features ? (size_t)n * P.Lmax : 0;
    P.y0 = a.take<float>(nL);
    P.y1 = a.take<float>(nL);
    P.pbuf = a.take<float>(nL);
    P.yout = a.take<float>(features ? (size_t)n * P.L : 0);
    P.zout = a.take<float>(features ? (size_t)n * P.d : 0);
    if (!features) P.y0 = P.y1 = P.pbuf = P.yout = P.zout = nullptr;
    size_t wmax = 1;
    int lin = P.L;
    for (int k = 0; k < c->n_layers; ++k) {
        wmax = std::max(wmax, (size_t)lin * c->layer_dims[k]);
        lin = c->layer_dims[k];
    }
    P.wbuf = a.take<float>(wmax);
    P.cpart = a.take<double>(((size_t)spmm_grid(n, P.L, ctx->num_cu, nullptr) + kColsumStageRows) * P.L);
    P.c64 = a.take<double>(P.Lmax);
    P.cvec = a.take<float>(P.Lmax);
    // k-means
    const Grid& G = P.grid;
    const size_t meta_n = (size_t)3 * G.Kc + G.KP + (size_t)kDynLen(G.Kc);
    P.meta = a.take<int32_t>(meta_n);
    P.dyn = P.meta ? P.meta + 3 * G.Kc + G.KP : nullptr;
    KmeansPlan& km = P.km;
    km.n = n;
    km.d = P.d;
    km.Kc = G.Kc;
    km.k_max = G.k_max;
    km.KP = G.KP;
    km.SK = G.SK;
    km.agroups = (int)P.lists.agrp.size() - 1;
    km.ugroups = (int)P.lists.ugrp.size() - 1;
    km.usk_max = P.ucap;
    P.ranges_max = update_ranges_max(n, cu);
    km.uwork = P.lists.uwork;
    km.race_grid = P.race_grid;
    km.ks = P.meta;
    km.koff16 = P.meta ? P.meta + G.Kc : nullptr;
    km.koff = P.meta ? P.meta + 2 * G.Kc : nullptr;
    km.cand_of = P.meta ? P.meta + 3 * G.Kc : nullptr;
    km.alist = P.dyn;
    km.agrp = P.dyn ? P.dyn + G.Kc : nullptr;
    km.ugrp = P.dyn ? P.dyn + 2 * G.Kc + 1 : nullptr;
    km.uwi0 = P.dyn ? P.dyn + 3 * G.Kc + 2 : nullptr;
    km.ulen = P.dyn ? P.dyn + 4 * G.Kc + 3 : nullptr;
    km.cranges = P.dyn ? P.dyn + 5 * G.Kc + 3 : nullptr;
    km.active = a.take<int32_t>(G.Kc);
    km.changes = a.take<int32_t>(G.Kc);
    P.iters_int = a.take<int32_t>(G.Kc);
    km.iters = P.iters_int;
    km.active_count = a.take<int32_t>(1);
    km.C = a.take<float>((size_t)G.KP * P.d);
    km.cnorm = a.take<float>(G.KP);
    km.split = kmeans_split_supported(P.d) ? 1 : 0;
    // points (split halves or FP32) beyond 64 MB: assignment blocks of one
    // point tile run together (see the assignment kernels' block order)
    km.group_major = (size_t)n * P.d * 4 > ((size_t)64 << 20) ? 1 : 0;
    km.zh = a.take<uint16_t>(km.split ? (size_t)n * P.d : 1);
    km.zl = a.take<uint16_t>(km.split ? (size_t)n * P.d : 1);
    km.ch = a.take<uint16_t>(km.split ? (size_t)G.KP * P.d : 1);
    km.cl = a.take<uint16_t>(km.split ? (size_t)G.KP * P.d : 1);
    km.S64 = a.take<long long>((size_t)G.KP * P.d);
    km.N32 = a.take<int32_t>(G.KP);
    km.pdelta = a.take<long long>((size_t)P.ranges_max * G.KP * P.d);
    km.pcnt = a.take<int32_t>((size_t)P.ranges_max * G.KP);
    km.pdirty = a.take<uint8_t>((size_t)P.ranges_max * G.KP);
    km.zmax_bits = a.take<uint32_t>(1);
    km.w = a.take<float>(n);
    km.race_val = a.take<double>((size_t)2 * P.race_grid);
    km.race_idx = a.take<int32_t>((size_t)2 * P.race_grid);
    P.picks_int = a.take<int32_t>(G.k_max);
    km.picks = P.picks_int;
    km.lab_cm = a.take<uint8_t>((size_t)G.Kc * n);
    km.lab_old = a.take<uint8_t>((size_t)G.Kc * n);
    km.nchunks = (int)(((int64_t)n + 63) / 64);
    km.moved_it = a.take<int32_t>((size_t)km.nchunks * G.Kc);
    // bound-pruned assignment: graphs on their own (a batch assigns every
    // point), split-fp16 operands, bounded running sums, tables that fit in
    // LDS.  Scoring a listed point gathers its row (4 d bytes) for one
    // candidate, where the full assignment reads each point once per group
    // of candidates; the saving is in the MFMA work, which grows with K: by
    // default only grids with a mean K of 64 or more are pruned (measured:
    // N = 1M, K = 50..150 step 5, d = 128: 217 -> 145..165 ms per run;
    // N = 50k, K = 2..80, d = 64: 8.4..11.5 -> 8.6..12.2 ms).
    const int nranges = (int)((n + kPruneRange - 1) / kPruneRange);
    const bool prune_pays = c->kmeans_prune == 1 || (c->kmeans_prune == 0 && G.SK >= 64 * G.Kc);
    km.prune = features && km.split && prune_pays && c->kmeans_max_iter <= 65536 &&
                       list_lds_bytes(P.d, (G.k_max + 15) / 16, G.Kc * nranges) <=
                           (size_t)kPruneDynLdsMax
                   ? 1
                   : 0;
    if (km.prune) {
        km.hu = a.take<float>((size_t)G.Kc * n);
        km.hl = a.take<float>((size_t)G.Kc * n);
        km.cum = a.take<double>(G.KP);
        km.cmx = a.take<double>(G.Kc);
        km.dmx = a.take<double>((size_t)2 * G.Kc);
        km.zn2 = a.take<float>(n);
        km.pe = a.take<float>(n);
        km.plist = a.take<int32_t>((size_t)G.Kc * n);
        km.scnt = a.take<int32_t>((size_t)G.Kc * nranges);
        km.nranges = nranges;
        km.znmax_bits = a.take<uint32_t>(1);
        km.list_tiles = (G.k_max + 15) / 16;
    }
    km.status = ctx->d_status;
    km.seed = c->seed;
    km.zoff = 0;
    // scores
    ScorePlan& sc = P.sc;
    sc.n = n;
    sc.Kc = G.Kc;
    sc.S = P.S;
    sc.SK = G.SK;
    sc.grid = P.score_grid_;
    sc.heavy = g->heavy[score_split_batches(P.S)];
    sc.nnz = g->nnz;
    sc.ks = km.ks;
    sc.koff = km.koff;
    sc.lpart = a.take<int32_t>((size_t)P.score_grid_ * G.SK);
    sc.vpart = a.take<int32_t>((size_t)P.score_grid_ * G.SK);
    sc.l64 = a.take<int64_t>(G.SK);
    sc.v64 = a.take<int64_t>(G.SK);
    P.mod_int = a.take<double>(G.Kc);
    P.ncut_int = a.take<double>(G.Kc);
    sc.mod = P.mod_int;
    sc.ncut = P.ncut_int;
    sc.best = a.take<int32_t>(1);
    sc.first = a.take<int32_t>(RAFT_MAX_K + 1);
    sc.remap = a.take<int32_t>(RAFT_MAX_K + 1);
    sc.status = ctx->d_status;
    P.ksel_int = a.take<int32_t>(4);
    P.lab_pm = a.take<uint8_t>((size_t)n * P.S);
    P.bytes = a.off;
}

// Packs the dynamic lists at fixed offsets: alist [Kc], agrp [Kc+1],
// ugrp [Kc+1], uwi0 [Kc+1], ulen [Kc], cranges [Kc].
void pack_lists(const Lists& l, int Kc, int32_t* out) {
    std::fill(out, out + kDynLen(Kc), 0);
    std::copy(l.alist.begin(), l.alist.end(), out);
    std::copy(l.agrp.begin(), l.agrp.end(), out + Kc);
    std::copy(l.ugrp.begin(), l.ugrp.end(), out + 2 * Kc + 1);
    std::copy(l.uwi0.begin(), l.uwi0.end(), out + 3 * Kc + 2);
    std::copy(l.ulen.begin(), l.ulen.end(), out + 4 * Kc + 3);
    std::copy(l.cranges.begin(), l.cranges.end(), out + 5 * Kc + 3);
}

raft_status upload_meta(raft_ctx* ctx, const Plan& P, hipStream_t st) {
    const Grid& G = P.grid;
    std::vector<int32_t> meta;
    meta.insert(meta.end(), G.ks.begin(), G.ks.end());
    meta.insert(meta.end(), G.koff16.begin(), G.koff16.end());
    meta.insert(meta.end(), G.koff.begin(), G.koff.end());
    meta.insert(meta.end(), G.cand_of.begin(), G.cand_of.end());
    const size_t at = meta.size();
    meta.resize(at + (size_t)kDynLen(G.Kc));
    pack_lists(P.lists, G.Kc, meta.data() + at);
    HIP_TRY(ctx, hipMemcpyAsync(P.meta, meta.data(), meta.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st));
    // pageable source: wait so the host vector may go out of scope
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return RAFT_OK;
}

raft_status check_ws(raft_ctx* ctx, void* ws, size_t ws_bytes, size_t need) {
    if (!ws) return fail(ctx, RAFT_E_INVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(ctx, RAFT_E_INVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(ctx, RAFT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);
    return RAFT_OK;
}

raft_status check_graph(raft_ctx* ctx, const raft_graph* g) {
    if (!ctx) return RAFT_E_INVAL;
    if (!g) return fail(ctx, RAFT_E_INVAL, "graph is null");
    if (g->ctx != ctx) return fail(ctx, RAFT_E_INVAL, "graph belongs to another context");
    return RAFT_OK;
}

raft_status launch_check(raft_ctx* ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, RAFT_E_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return RAFT_OK;
}

// Y = X^q Theta into `out` using the plan's ping-pong buffers.
raft_status do_project(raft_ctx* ctx, const raft_graph* g, const raft_config* c, Plan& P,
                       float* out, hipStream_t st) {
    const int L = P.L;
    const GraphView gv = g->view();
    float* src = P.y0;
    launch_gaussian(c->seed, 0x10, g->n, L, 1.0 / std::sqrt((double)L), src, st);
    const bool mod_full = c->op == RAFT_X_MOD_FULL;
    if (mod_full) {
        launch_colsum_partials(gv, L, src, P.cpart, ctx->num_cu, st);
        launch_colsum_finish(P.cpart, spmm_grid(g->n, L, ctx->num_cu, nullptr), L, P.c64, P.cvec,
                             st);
    }
    for (int t = 1; t <= c->q; ++t) {
        float* dst = (t == c->q) ? out : (src == P.y0 ? P.y1 : P.y0);
        const bool need_cs = mod_full && t < c->q;
        {
            ProfScope ps(ctx, RAFT_PROF_SPMM, st);
            launch_spmm(gv, c->op, L, src, dst, P.cvec, need_cs ? P.cpart : nullptr, ctx->num_cu,
                        st);
        }
        if (need_cs)
            launch_colsum_finish(P.cpart, spmm_grid(g->n, L, ctx->num_cu, nullptr), L, P.c64,
                                 P.cvec, st);
        src = dst;
    }
    return launch_check(ctx);
}

raft_status do_embed(raft_ctx* ctx, const raft_graph* g, const raft_config* c, Plan& P,
                     const float* Y, float* Z, hipStream_t st) {
    const GraphView gv = g->view();
    const float* h = Y;
    int lin = P.L;
    if (c->n_layers == 0) {
        if (Z != Y)
            HIP_TRY(ctx, hipMemcpyAsync(Z, Y, (size_t)g->n * lin * sizeof(float),
                                        hipMemcpyDeviceToDevice, st));
        if (c->normalize_input) launch_rownorm(Z, g->n, lin, st);
        return launch_check(ctx);
    }
    if (c->normalize_input) {
        HIP_TRY(ctx, hipMemcpyAsync(P.y1, Y, (size_t)g->n * lin * sizeof(float),
                                    hipMemcpyDeviceToDevice, st));
        launch_rownorm(P.y1, g->n, lin, st);
        h = P.y1;
    }
    for (int k = 1; k <= c->n_layers; ++k) {
        const int lout = c->layer_dims[k - 1];
        launch_gaussian(c->seed, 0x10 + (uint64_t)k, lin, lout, 1.0 / std::sqrt((double)lin),
                        P.wbuf, st);
        {
            ProfScope ps(ctx, RAFT_PROF_SPMM, st);
            launch_spmm(gv, kOpGcn, lin, h, P.pbuf, nullptr, nullptr, ctx->num_cu, st);
        }
        float* dst = (k == c->n_layers) ? Z : (h == P.y0 ? P.y1 : P.y0);
        {
            ProfScope ps(ctx, RAFT_PROF_DENSE, st);
            launch_dense_layer(P.pbuf, P.wbuf, dst, g->n, lin, lout, false, ctx->d_status,
                               ctx->num_cu, st);
        }
        h = dst;
        lin = lout;
    }
    return launch_check(ctx);
}

static int live_polled(const int32_t* active, int Kc) {
    int live = 0;
    for (int k = 0; k < Kc; ++k) live += active[k] != 0;
    return live;
}

raft_status do_partition(raft_ctx* ctx, const raft_graph* g, const raft_config* c, Plan& P,
                         const float* Z, raft_outputs* out, hipStream_t st, bool timed) {
    KmeansPlan km = P.km;
    if (out && out->picks) km.picks = out->picks;
    if (out && out->iters) km.iters = out->iters;
    ScorePlan sc = P.sc;
    if (out && out->mod) sc.mod = out->mod;
    if (out && out->ncut) sc.ncut = out->ncut;
    int32_t* ksel = (out && out->k_selected) ? out->k_selected : P.ksel_int;
    const int t_max = c->kmeans_max_iter;
    const int check = c->check_every > 0 ? c->check_every : 4;
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[2], st));
    launch_kmeans_reset(km, st);
    launch_zmax(km, Z, ctx->num_cu, st);
    if (km.split) launch_split_points(km, Z, st);
    if (km.prune) launch_prune_init(km, Z, st);
    for (int t = 0; t < km.k_max; ++t) {
        ProfScope ps(ctx, RAFT_PROF_RACE, st);
        launch_race_pick(km, Z, t, st);
    }
    launch_init_centres(km, Z, st);
    RAFT_TRY(launch_check(ctx));
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[3], st));
    const int Kc = P.grid.Kc;
    // Convergence polls without stalling the GPU: at every `check`-th
    // iteration the active flags are copied to pinned host memory behind an
    // event, and the host acts on the copy of the previous poll (the GPU is
    // past it and still has the iterations since queued).  The work lists
    // built from it are one poll stale: they may still hold candidates that
    // retired since, which every kernel skips, so results do not change.
    // Two pinned slots each for the flags and the packed lists: a slot is
    // rewritten only after the event of the poll that last used it.
    int32_t* h_active[2] = {ctx->h_pinned + 16, ctx->h_pinned + 16 + (RAFT_MAX_K + 1)};
    int32_t* h_lists[2] = {ctx->h_pinned + 16 + 2 * (RAFT_MAX_K + 1),
                           ctx->h_pinned + 16 + 2 * (RAFT_MAX_K + 1) + kDynLen(RAFT_MAX_K)};
    static_assert(16 + 2 * (RAFT_MAX_K + 1) + 2 * kDynLen(RAFT_MAX_K) <= 4096,
                  "poll slots exceed the pinned scratch");
    int poll = 0;
    int nact = (int)P.lists.alist.size();   // candidates of alist (the kernels skip retired ones)
    int live_listed = Kc;                   // live candidates when the lists were built
    for (int it = 1; it <= t_max; ++it) {
        km.it = it;
        {
            const ProfLaunch pl(ctx, RAFT_PROF_ASSIGN);
            if (km.prune && it >= kPruneFrom)
                launch_assign_pruned(km, nact, ctx->num_cu, st, pl.e0, pl.e1);
            else
                launch_assign(km, Z, ctx->num_cu, st, pl.e0, pl.e1);
        }
        if (it == t_max) {
            launch_iter_finalize(km, it, t_max, st);
            break;
        }
        {
            ProfScope ps(ctx, RAFT_PROF_UPDATE, st);
            launch_update(km, Z, ctx->lds_max, it, t_max, st);
        }
        if (it % check == 0) {
            const int32_t* ha = h_active[(poll - 1) & 1];
            int live = live_listed;
            if (poll > 0) {
                HIP_TRY(ctx, hipEventSynchronize(ctx->poll_ev[(poll - 1) & 1]));
                live = live_polled(ha, Kc);
                if (live == 0) break;
            }
            // compact the work lists to the candidates still iterating (a
            // candidate never resumes, so the same count is the same set)
            if (live != live_listed) {
                live_listed = live;
                const Lists l = make_lists(P.grid, ha, P.ucap, g->n, ctx->num_cu);
                int32_t* hl = h_lists[poll & 1];
                pack_lists(l, Kc, hl);
                HIP_TRY(ctx, hipMemcpyAsync(P.dyn, hl, (size_t)kDynLen(Kc) * sizeof(int32_t),
                                            hipMemcpyHostToDevice, st));
                km.agroups = (int)l.agrp.size() - 1;
                km.ugroups = (int)l.ugrp.size() - 1;
                km.uwork = l.uwork;
                nact = (int)l.alist.size();
            }
            HIP_TRY(ctx, hipMemcpyAsync(h_active[poll & 1], km.active, Kc * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, st));
            HIP_TRY(ctx, hipEventRecord(ctx->poll_ev[poll & 1], st));
            ++poll;
        }
    }
    RAFT_TRY(launch_check(ctx));
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[4], st));
    if (out && out->centres) launch_copy_centres(km, out->centres, st);
    launch_transpose_labels(km.lab_cm, g->n, P.grid.Kc, P.lab_pm, P.S, st);
    {
        ProfScope ps(ctx, RAFT_PROF_SCORE, st);
        launch_edge_score(g->view(), sc, P.lab_pm, st);
    }
    launch_score_finish(sc, st);
    launch_select(sc, P.lab_pm, out ? out->labels : nullptr, ksel, st);
    if (out && out->labels_all)
        launch_copy_labels(P.lab_pm, g->n, P.grid.Kc, P.S, out->labels_all, st);
    if (timed) HIP_TRY(ctx, hipEventRecord(ctx->ev[5], st));
    return launch_check(ctx);
}

raft_status plan_for(raft_ctx* ctx, const raft_graph* g, const raft_config* c, void* ws,
                     size_t ws_bytes, Plan& P) {
    RAFT_TRY(check_config(ctx, g, c));
    plan_layout(ctx, g, c, nullptr, P);
    const int d = embed_dim(c);
    if (!kmeans_supported(d)) return fail(ctx, RAFT_E_UNSUPPORTED, "embedding width %d", d);
    if (kmeans_update_lds(P.ucap, d) > ctx->lds_max)
        return fail(ctx, RAFT_E_UNSUPPORTED, "k_max %d too large for width %d", P.grid.k_max, d);
    if (!score_supported(P.grid.Kc, P.grid.SK))
        return fail(ctx, RAFT_E_UNSUPPORTED, "%d candidates with sum of K %d (at most 256 and 16384)",
                    P.grid.Kc, P.grid.SK);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, P.bytes));
    plan_layout(ctx, g, c, reinterpret_cast<char*>(ws), P);
    return RAFT_OK;
}

}  // namespace

extern "C" {

int32_t raft_abi_version(void) { return RAFT_ABI_VERSION; }

const char* raft_status_string(raft_status s) {
    switch (s) {
        case RAFT_OK: return "ok";
        case RAFT_E_INVAL: return "invalid argument";
        case RAFT_E_CSR: return "malformed CSR";
        case RAFT_E_NOEDGES: return "graph has no edges";
        case RAFT_E_WORKSPACE: return "workspace too small";
        case RAFT_E_NOMEM: return "out of device memory";
        case RAFT_E_DEVICE: return "HIP runtime error";
        case RAFT_E_NUMERIC: return "non-finite value";
        case RAFT_E_UNSUPPORTED: return "unsupported size";
        default: return "unknown status";
    }
}

raft_status raft_ctx_create(int device, const char* autotune_cache, raft_ctx** out) {
    if (!out) return RAFT_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return RAFT_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return RAFT_E_DEVICE;
    if (device >= kMaxDevices) return RAFT_E_UNSUPPORTED;
    void* scratch_ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
                return RAFT_E_DEVICE;
            g_scratch_ptr[device] = p;
        }
        scratch_ptr = g_scratch_ptr[device];
    }
    raft_ctx* c = new raft_ctx();
    c->device = device;
    c->scratch = scratch_ptr;
    if (autotune_cache) c->autotune_cache = autotune_cache;
    tuner_load(c);
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cu > 0)
        c->num_cu = cu;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeSharedMemPerBlockOptin, device) ==
            hipSuccess &&
        lds > 0)
        c->lds_max = (size_t)lds;
    else if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
                 hipSuccess &&
             lds > 0)
        c->lds_max = (size_t)lds;
    if (hipMalloc(&c->d_status, 256) != hipSuccess ||
        hipHostMalloc((void**)&c->h_pinned, 16384, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return RAFT_E_NOMEM;
    }
    if (hipMemset(c->d_status, 0, 256) != hipSuccess) {
        delete c;
        return RAFT_E_DEVICE;
    }
    for (auto& e : c->ev) (void)hipEventCreate(&e);
    for (auto& e : c->poll_ev) (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    *out = c;
    return RAFT_OK;
}

void raft_ctx_destroy(raft_ctx* ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->poll_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->prof_pool) (void)hipEventDestroy(e);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    delete ctx;
}

size_t raft_last_error(raft_ctx* ctx, char* buf, size_t n) {
    if (!ctx) return 0;
    if (buf && n) {
        const size_t m = std::min(n - 1, ctx->err.size());
        memcpy(buf, ctx->err.data(), m);
        buf[m] = 0;
    }
    return ctx->err.size();
}

raft_status raft_sync_status(raft_ctx* ctx, void* stream) {
    if (!ctx) return RAFT_E_INVAL;
    hipStream_t st = as_stream(stream);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_pinned, ctx->d_status, sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    const int32_t s = ctx->h_pinned[0];
    if (s) {
        HIP_TRY(ctx, hipMemsetAsync(ctx->d_status, 0, sizeof(int32_t), st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        if (s & kStatusNumeric) return fail(ctx, RAFT_E_NUMERIC, "non-finite value (status %#x)", s);
        if (s & kStatusLabel) return fail(ctx, RAFT_E_INVAL, "label out of range (status %#x)", s);
        return fail(ctx, RAFT_E_CSR, "device status %#x", s);
    }
    return RAFT_OK;
}

raft_status raft_graph_create(raft_ctx* ctx, const void* row_ptr, int row_ptr_is_int64,
                              const int32_t* col_idx, int64_t n, int64_t nnz,
                              int inputs_on_device, void* stream, raft_graph** out) {
    if (!ctx) return RAFT_E_INVAL;
    if (!out) return fail(ctx, RAFT_E_INVAL, "out is null");
    *out = nullptr;
    if (!row_ptr || (nnz > 0 && !col_idx)) return fail(ctx, RAFT_E_INVAL, "null CSR array");
    if (n < 1 || n >= INT32_MAX) return fail(ctx, RAFT_E_INVAL, "n = %lld", (long long)n);
    if (nnz < 0) return fail(ctx, RAFT_E_INVAL, "nnz = %lld", (long long)nnz);
    if (nnz >= INT32_MAX)
        return fail(ctx, RAFT_E_UNSUPPORTED, "nnz = %lld does not fit the int32 CSR",
                    (long long)nnz);
    hipStream_t st = as_stream(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // row_ptr is checked on the host before any kernel indexes col_idx with
    // it; an int64 row_ptr is narrowed to int32 after the checks.  Host
    // copies go through the context's pinned staging (one DMA each, where
    // pageable memory is copied in many small pieces):
    // [raw row_ptr (n+1) x elem][int32 row_ptr (n+1)][row order n]
    const size_t elem = row_ptr_is_int64 ? sizeof(int64_t) : sizeof(int32_t);
    const size_t raw_bytes = ((size_t)n + 1) * elem;
    const size_t raw_pad = (raw_bytes + 255) / 256 * 256;
    const size_t rp_pad = (((size_t)n + 1) * sizeof(int32_t) + 255) / 256 * 256;
    const size_t need = raw_pad + rp_pad + (size_t)n * sizeof(int32_t);
    if (ctx->stage_bytes < need) {
        if (ctx->stage) (void)hipHostFree(ctx->stage);
        ctx->stage = nullptr;
        ctx->stage_bytes = 0;
        if (hipHostMalloc((void**)&ctx->stage, need) != hipSuccess) {
            ctx->stage = nullptr;
            return fail(ctx, RAFT_E_NOMEM, "pinned staging of %zu bytes", need);
        }
        ctx->stage_bytes = need;
    }
    int32_t* h_rp = reinterpret_cast<int32_t*>(ctx->stage + raw_pad);
    int32_t* order = reinterpret_cast<int32_t*>(ctx->stage + raw_pad + rp_pad);
    {
        const char* raw = reinterpret_cast<const char*>(row_ptr);
        if (inputs_on_device) {
            HIP_TRY(ctx, hipMemcpyAsync(ctx->stage, row_ptr, raw_bytes, hipMemcpyDeviceToHost, st));
            HIP_TRY(ctx, hipStreamSynchronize(st));
            raw = ctx->stage;
        }
        if (row_ptr_is_int64) {
            const int64_t* r64 = reinterpret_cast<const int64_t*>(raw);
            if (r64[0] != 0 || r64[n] != nnz)
                return fail(ctx, RAFT_E_CSR, "row_ptr must start at 0 and end at nnz");
            for (int64_t i = 0; i < n; ++i)
                if (r64[i + 1] < r64[i])
                    return fail(ctx, RAFT_E_CSR, "row_ptr decreases at %lld", (long long)i);
            // non-decreasing from 0 to nnz < INT32_MAX: every entry fits int32
            for (int64_t i = 0; i <= n; ++i) h_rp[i] = (int32_t)r64[i];
        } else {
            memcpy(h_rp, raw, raw_bytes);
        }
    }
    if (h_rp[0] != 0 || h_rp[n] != nnz)
        return fail(ctx, RAFT_E_CSR, "row_ptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < n; ++i)
        if (h_rp[i + 1] < h_rp[i]) return fail(ctx, RAFT_E_CSR, "row_ptr decreases at %lld", (long long)i);
    if (nnz % 2) return fail(ctx, RAFT_E_CSR, "odd nnz cannot be a symmetric loop-free CSR");
    raft_graph* g = new raft_graph();
    g->ctx = ctx;
    g->n = (int32_t)n;
    g->nnz = nnz;
    bool ok = hipMalloc(&g->rp, sizeof(int32_t) * (n + 1)) == hipSuccess &&
              hipMalloc(&g->ci, sizeof(int32_t) * std::max<int64_t>(nnz, 1)) == hipSuccess &&
              hipMalloc(&g->deg, sizeof(int32_t) * n) == hipSuccess &&
              hipMalloc(&g->s, sizeof(float) * n) == hipSuccess &&
              hipMalloc(&g->sh, sizeof(float) * n) == hipSuccess &&
              hipMalloc(&g->dcoef, sizeof(float) * n) == hipSuccess &&
              hipMalloc(&g->order, sizeof(int32_t) * n) == hipSuccess;
    if (!ok) {
        raft_graph_destroy(g);
        return fail(ctx, RAFT_E_NOMEM, "graph allocation failed");
    }
    const hipMemcpyKind kind = inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpyAsync(g->rp, h_rp, sizeof(int32_t) * (n + 1),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz > 0)
        e = hipMemcpyAsync(g->ci, col_idx, sizeof(int32_t) * nnz, kind, st);
    // Row order of the row-split kernels (SpMM, edge scores): a stable
    // partition by the number of 16-edge batches a row needs (at most 16
    // classes), heaviest first, so the rows a wave takes side by side have
    // similar lengths and the longest start first.  Only the schedule
    // changes: every row is summed in its own edge order.
    {
        constexpr int kClasses = 17;
        auto cls = [&](int64_t i) {
            const int64_t b = (h_rp[i + 1] - h_rp[i] + 15) / 16;
            return (int)(kClasses - 1 - std::min<int64_t>(b, kClasses - 1));
        };
        int64_t start[kClasses + 1] = {};
        for (int64_t i = 0; i < n; ++i) ++start[cls(i) + 1];
        for (int c = 0; c < kClasses; ++c) start[c + 1] += start[c];
        for (int64_t i = 0; i < n; ++i) order[start[cls(i)]++] = (int32_t)i;
        // after the fill start[c] is the end of class c: the rows with at
        // least b batches are those of classes 0 .. 16 - b
        g->heavy[0] = (int32_t)n;
        for (int b = 1; b < kClasses; ++b) g->heavy[b] = (int32_t)start[kClasses - 1 - b];
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->order, order, sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->d_status, 0, sizeof(int32_t), st);
    if (e != hipSuccess) {
        raft_graph_destroy(g);
        return fail(ctx, RAFT_E_DEVICE, "graph upload: %s", hipGetErrorString(e));
    }
    launch_validate_csr(g->rp, g->ci, g->n, ctx->d_status, ctx->num_cu, st);
    launch_degrees(g->rp, g->n, nnz, g->deg, g->s, g->sh, g->dcoef, st);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_pinned, ctx->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        raft_graph_destroy(g);
        return fail(ctx, RAFT_E_DEVICE, "graph validation: %s", hipGetErrorString(e));
    }
    const int32_t status = ctx->h_pinned[0];
    if (status) {
        (void)hipMemsetAsync(ctx->d_status, 0, sizeof(int32_t), st);
        (void)hipStreamSynchronize(st);
        raft_graph_destroy(g);
        return fail(ctx, RAFT_E_CSR, "CSR invalid (%s%s%s%s%s)",
                    (status & kStatusCsrRange) ? "range " : "",
                    (status & kStatusCsrOrder) ? "order " : "",
                    (status & kStatusCsrLoop) ? "self-loop " : "",
                    (status & kStatusCsrSym) ? "asymmetric " : "",
                    (status & kStatusCsrRowPtr) ? "row_ptr " : "");
    }
    *out = g;
    return RAFT_OK;
}

void raft_graph_destroy(raft_graph* g) {
    if (!g || !g->owns) return;
    (void)hipDeviceSynchronize();
    if (g->rp) (void)hipFree(g->rp);
    if (g->ci) (void)hipFree(g->ci);
    if (g->deg) (void)hipFree(g->deg);
    if (g->s) (void)hipFree(g->s);
    if (g->sh) (void)hipFree(g->sh);
    if (g->dcoef) (void)hipFree(g->dcoef);
    if (g->order) (void)hipFree(g->order);
    delete g;
}

raft_status raft_graph_degrees(const raft_graph* g, int32_t* deg_out, void* stream) {
    if (!g || !deg_out) return RAFT_E_INVAL;
    raft_ctx* ctx = g->ctx;
    HIP_TRY(ctx, hipMemcpyAsync(deg_out, g->deg, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice,
                                as_stream(stream)));
    return RAFT_OK;
}

raft_status raft_graph_size(const raft_graph* g, int64_t* n, int64_t* nnz) {
    if (!g) return RAFT_E_INVAL;
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    return RAFT_OK;
}

raft_status raft_graph_csr(const raft_graph* g, int32_t* row_ptr, int32_t* col_idx, void* stream) {
    if (!g || !row_ptr || (g->nnz > 0 && !col_idx)) return RAFT_E_INVAL;
    raft_ctx* ctx = g->ctx;
    hipStream_t st = as_stream(stream);
    HIP_TRY(ctx, hipMemcpyAsync(row_ptr, g->rp, sizeof(int32_t) * ((size_t)g->n + 1),
                                hipMemcpyDeviceToDevice, st));
    if (g->nnz > 0)
        HIP_TRY(ctx, hipMemcpyAsync(col_idx, g->ci, sizeof(int32_t) * (size_t)g->nnz,
                                    hipMemcpyDeviceToDevice, st));
    return RAFT_OK;
}

raft_status raft_workspace_size(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                                size_t* bytes) {
    RAFT_TRY(check_graph(ctx, g));
    if (!bytes) return fail(ctx, RAFT_E_INVAL, "bytes is null");
    RAFT_TRY(check_config(ctx, g, cfg));
    Plan P;
    plan_layout(ctx, g, cfg, nullptr, P);
    *bytes = P.bytes;
    return RAFT_OK;
}

raft_status raft_gaussian(raft_ctx* ctx, uint64_t seed, uint64_t stream_id, int64_t rows,
                          int64_t cols, double sigma, float* out, void* stream) {
    if (!ctx) return RAFT_E_INVAL;
    if (rows < 0 || cols < 0) return fail(ctx, RAFT_E_INVAL, "negative size");
    if (rows * cols > 0 && !out) return fail(ctx, RAFT_E_INVAL, "out is null");
    if (!std::isfinite(sigma)) return fail(ctx, RAFT_E_INVAL, "sigma not finite");
    launch_gaussian(seed, stream_id, rows, cols, sigma, out, as_stream(stream));
    return launch_check(ctx);
}

// Layout of raft_score's workspace: candidate table, stride-S labels,
// per-work-group partial counts, int64 totals.
static size_t score_ws_bytes(raft_ctx* ctx, const raft_graph* g, int Kc, int SK) {
    const int S = (Kc + 7) / 8 * 8;
    const int grid = score_grid(g->n, ctx->num_cu);
    Arena a;
    a.take<int32_t>(2 * (size_t)Kc);
    a.take<uint8_t>((size_t)g->n * S);
    a.take<int32_t>((size_t)grid * SK);
    a.take<int32_t>((size_t)grid * SK);
    a.take<int64_t>(SK);
    a.take<int64_t>(SK);
    return a.off;
}

static size_t spmm_ws_bytes(raft_ctx* ctx, const raft_graph* g, int L) {
    const int grid = spmm_grid(g->n, L, ctx->num_cu, nullptr);
    return align256(((size_t)grid + kColsumStageRows) * L * sizeof(double)) + align256(L * sizeof(double)) +
           align256(L * sizeof(float));
}

static raft_status spmm_checks(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                               const float* Y_in, const float* Y_out) {
    RAFT_TRY(check_graph(ctx, g));
    if (op < RAFT_X_NCUT || op > RAFT_X_GCN) return fail(ctx, RAFT_E_INVAL, "op %d", op);
    if (!spmm_supported(L)) return fail(ctx, RAFT_E_UNSUPPORTED, "width %d", L);
    if (!Y_in || !Y_out || Y_in == Y_out) return fail(ctx, RAFT_E_INVAL, "bad Y buffers");
    if ((op == RAFT_X_MOD_FULL || op == RAFT_X_MOD_REDUCED) && g->nnz == 0)
        return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    return RAFT_OK;
}

// One sparse step; `ws` holds MOD_FULL's column-sum partials (already checked
// to be large enough), unused for the other operators.
static raft_status spmm_body(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                             const float* Y_in, float* Y_out, void* ws, hipStream_t st) {
    const GraphView gv = g->view();
    if (op == RAFT_X_MOD_FULL) {
        Arena a;
        a.base = reinterpret_cast<char*>(ws);
        const int grid = spmm_grid(g->n, L, ctx->num_cu, nullptr);
        double* cpart = a.take<double>(((size_t)grid + kColsumStageRows) * L);
        double* c64 = a.take<double>(L);
        float* cvec = a.take<float>(L);
        launch_colsum_partials(gv, L, Y_in, cpart, ctx->num_cu, st);
        launch_colsum_finish(cpart, grid, L, c64, cvec, st);
        launch_spmm(gv, op, L, Y_in, Y_out, cvec, nullptr, ctx->num_cu, st);
    } else {
        launch_spmm(gv, op, L, Y_in, Y_out, nullptr, nullptr, ctx->num_cu, st);
    }
    return launch_check(ctx);
}

raft_status raft_spmm(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                      const float* Y_in, float* Y_out, void* ws, size_t ws_bytes, void* stream) {
    RAFT_TRY(spmm_checks(ctx, g, op, L, Y_in, Y_out));
    if (op == RAFT_X_MOD_FULL) RAFT_TRY(check_ws(ctx, ws, ws_bytes, spmm_ws_bytes(ctx, g, L)));
    return spmm_body(ctx, g, op, L, Y_in, Y_out, ws, as_stream(stream));
}

raft_status raft_spmm_noalloc(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                              const float* Y_in, float* Y_out, void* stream) {
    RAFT_TRY(spmm_checks(ctx, g, op, L, Y_in, Y_out));
    if (op == RAFT_X_MOD_FULL) {
        const size_t need = spmm_ws_bytes(ctx, g, L);
        if (need > kNoAllocScratchBytes)
            return fail(ctx, RAFT_E_WORKSPACE,
                        "N = %d at width %d needs %zu bytes of scratch; the fixed scratch holds "
                        "%zu (use raft_spmm with a workspace)",
                        g->n, L, need, kNoAllocScratchBytes);
        if (!ctx->scratch) return fail(ctx, RAFT_E_DEVICE, "scratch address not resolved");
    }
    // every partial and stage row is written before it is read, so stale
    // contents from an earlier call need no clearing
    return spmm_body(ctx, g, op, L, Y_in, Y_out, ctx->scratch, as_stream(stream));
}

raft_status raft_spmm_merge_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t op,
                                           int32_t L, size_t* bytes) {
    RAFT_TRY(check_graph(ctx, g));
    if (!bytes) return fail(ctx, RAFT_E_INVAL, "bytes is null");
    if (op < RAFT_X_NCUT || op > RAFT_X_GCN) return fail(ctx, RAFT_E_INVAL, "op %d", op);
    if (!spmm_supported(L) || L > 256) return fail(ctx, RAFT_E_UNSUPPORTED, "width %d", L);
    *bytes = align256(spmm_merge_ws_bytes(g->n, g->nnz, L, op)) +
             (op == RAFT_X_MOD_FULL ? spmm_ws_bytes(ctx, g, L) : 0);
    return RAFT_OK;
}

raft_status raft_spmm_merge(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                            const float* Y_in, float* Y_out, void* ws, size_t ws_bytes,
                            void* stream) {
    RAFT_TRY(spmm_checks(ctx, g, op, L, Y_in, Y_out));
    size_t need = 0;
    RAFT_TRY(raft_spmm_merge_workspace_size(ctx, g, op, L, &need));
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, need));
    hipStream_t st = as_stream(stream);
    const GraphView gv = g->view();
    char* w = reinterpret_cast<char*>(ws);
    const float* cvec = nullptr;
    if (op == RAFT_X_MOD_FULL) {
        Arena a;
        a.base = w + align256(spmm_merge_ws_bytes(g->n, g->nnz, L, op));
        const int grid = spmm_grid(g->n, L, ctx->num_cu, nullptr);
        double* cpart = a.take<double>(((size_t)grid + kColsumStageRows) * L);
        double* c64 = a.take<double>(L);
        float* cv = a.take<float>(L);
        launch_colsum_partials(gv, L, Y_in, cpart, ctx->num_cu, st);
        launch_colsum_finish(cpart, grid, L, c64, cv, st);
        cvec = cv;
    }
    launch_spmm_merge(gv, op, L, Y_in, Y_out, cvec, w, st);
    return launch_check(ctx);
}

raft_status raft_project(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg, void* ws,
                         size_t ws_bytes, float* Y_out, void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!Y_out) return fail(ctx, RAFT_E_INVAL, "Y_out is null");
    if (cfg && cfg->op != RAFT_X_NCUT && g->nnz == 0)
        return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    Plan P;
    RAFT_TRY(plan_for(ctx, g, cfg, ws, ws_bytes, P));
    return do_project(ctx, g, cfg, P, Y_out, as_stream(stream));
}

raft_status raft_gcn_layer(raft_ctx* ctx, const raft_graph* g, int32_t L_in, int32_t L_out,
                           const float* H_in, const float* W, int32_t linear, float* H_out,
                           float* P_out, void* ws, size_t ws_bytes, void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!dense_supported(L_in, L_out) || !spmm_supported(L_in))
        return fail(ctx, RAFT_E_UNSUPPORTED, "widths %d -> %d", L_in, L_out);
    if (!H_in || !W || !H_out) return fail(ctx, RAFT_E_INVAL, "null buffer");
    hipStream_t st = as_stream(stream);
    float* P = P_out;
    if (!P) {
        const size_t need = align256((size_t)g->n * L_in * sizeof(float));
        RAFT_TRY(check_ws(ctx, ws, ws_bytes, need));
        P = reinterpret_cast<float*>(ws);
    }
    launch_spmm(g->view(), kOpGcn, L_in, H_in, P, nullptr, nullptr, ctx->num_cu, st);
    launch_dense_layer(P, W, H_out, g->n, L_in, L_out, linear != 0, ctx->d_status, ctx->num_cu,
                       st);
    return launch_check(ctx);
}

raft_status raft_embed(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg, const float* Y,
                       void* ws, size_t ws_bytes, float* Z_out, void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!Y || !Z_out) return fail(ctx, RAFT_E_INVAL, "null buffer");
    Plan P;
    RAFT_TRY(plan_for(ctx, g, cfg, ws, ws_bytes, P));
    return do_embed(ctx, g, cfg, P, Y, Z_out, as_stream(stream));
}

raft_status raft_partition(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                           const float* Z, void* ws, size_t ws_bytes, raft_outputs* out,
                           void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!Z) return fail(ctx, RAFT_E_INVAL, "Z is null");
    if (g->nnz == 0) return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    Plan P;
    RAFT_TRY(plan_for(ctx, g, cfg, ws, ws_bytes, P));
    hipStream_t st = as_stream(stream);
    RAFT_TRY(upload_meta(ctx, P, st));
    return do_partition(ctx, g, cfg, P, Z, out, st, false);
}

raft_status raft_score(raft_ctx* ctx, const raft_graph* g, const uint8_t* labels_all, int32_t Kc,
                       const int32_t* ks, double* mod, double* ncut, void* ws, size_t ws_bytes,
                       void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!labels_all || !ks || !mod || !ncut || Kc < 1)
        return fail(ctx, RAFT_E_INVAL, "bad score arguments");
    if (g->nnz == 0) return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    std::vector<int32_t> koff(Kc);
    int SK = 0;
    for (int k = 0; k < Kc; ++k) {
        if (ks[k] < 1 || ks[k] > RAFT_MAX_K) return fail(ctx, RAFT_E_INVAL, "ks[%d] = %d", k, ks[k]);
        koff[k] = SK;
        SK += ks[k];
    }
    if (!score_supported(Kc, SK))
        return fail(ctx, RAFT_E_UNSUPPORTED, "%d labelings with sum of K %d (at most 256 and 16384)",
                    Kc, SK);
    const int S = (Kc + 7) / 8 * 8;
    const int grid = score_grid(g->n, ctx->num_cu);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, score_ws_bytes(ctx, g, Kc, SK)));
    Arena a;
    a.base = reinterpret_cast<char*>(ws);
    a.off = 0;
    hipStream_t st = as_stream(stream);
    int32_t* meta = a.take<int32_t>(2 * (size_t)Kc);
    uint8_t* pm = a.take<uint8_t>((size_t)g->n * S);
    ScorePlan sc;
    sc.n = g->n;
    sc.Kc = Kc;
    sc.S = S;
    sc.SK = SK;
    sc.grid = grid;
    sc.heavy = g->heavy[score_split_batches(S)];
    sc.nnz = g->nnz;
    sc.ks = meta;
    sc.koff = meta + Kc;
    sc.lpart = a.take<int32_t>((size_t)grid * SK);
    sc.vpart = a.take<int32_t>((size_t)grid * SK);
    sc.l64 = a.take<int64_t>(SK);
    sc.v64 = a.take<int64_t>(SK);
    sc.mod = mod;
    sc.ncut = ncut;
    sc.best = nullptr;
    sc.first = nullptr;
    sc.remap = nullptr;
    sc.status = ctx->d_status;
    std::vector<int32_t> hm(ks, ks + Kc);
    hm.insert(hm.end(), koff.begin(), koff.end());
    HIP_TRY(ctx, hipMemcpyAsync(meta, hm.data(), hm.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    // dense point-major [n x Kc] -> stride-S layout
    if (S == Kc) {
        HIP_TRY(ctx, hipMemcpyAsync(pm, labels_all, (size_t)g->n * S, hipMemcpyDeviceToDevice, st));
    } else {
        HIP_TRY(ctx, hipMemset2DAsync(pm, S, 0, S, g->n, st));
        HIP_TRY(ctx, hipMemcpy2DAsync(pm, S, labels_all, Kc, Kc, g->n, hipMemcpyDeviceToDevice, st));
    }
    launch_edge_score(g->view(), sc, pm, st);
    launch_score_finish(sc, st);
    return launch_check(ctx);
}

raft_status raft_spmm_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                                    size_t* bytes) {
    RAFT_TRY(check_graph(ctx, g));
    if (!bytes) return fail(ctx, RAFT_E_INVAL, "bytes is null");
    if (op < RAFT_X_NCUT || op > RAFT_X_GCN) return fail(ctx, RAFT_E_INVAL, "op %d", op);
    if (!spmm_supported(L)) return fail(ctx, RAFT_E_UNSUPPORTED, "width %d", L);
    *bytes = op == RAFT_X_MOD_FULL ? spmm_ws_bytes(ctx, g, L) : 0;
    return RAFT_OK;
}

raft_status raft_score_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t Kc,
                                     const int32_t* ks, size_t* bytes) {
    RAFT_TRY(check_graph(ctx, g));
    if (!bytes || !ks || Kc < 1) return fail(ctx, RAFT_E_INVAL, "bad score arguments");
    int SK = 0;
    for (int k = 0; k < Kc; ++k) {
        if (ks[k] < 1 || ks[k] > RAFT_MAX_K) return fail(ctx, RAFT_E_INVAL, "ks[%d] = %d", k, ks[k]);
        SK += ks[k];
    }
    if (!score_supported(Kc, SK))
        return fail(ctx, RAFT_E_UNSUPPORTED, "%d labelings with sum of K %d (at most 256 and 16384)",
                    Kc, SK);
    *bytes = score_ws_bytes(ctx, g, Kc, SK);
    return RAFT_OK;
}

raft_status raft_confusion(raft_ctx* ctx, const int32_t* a, const int32_t* b, int64_t n,
                           int32_t ka, int32_t kb, int64_t* counts, void* stream) {
    if (!ctx) return RAFT_E_INVAL;
    if (n < 0 || ka < 1 || kb < 1 || !counts || (n > 0 && (!a || !b)))
        return fail(ctx, RAFT_E_INVAL, "bad confusion arguments");
    if ((int64_t)ka * kb > ((int64_t)1 << 31))
        return fail(ctx, RAFT_E_UNSUPPORTED, "table %d x %d too large", ka, kb);
    launch_confusion(a, b, n, ka, kb, counts, ctx->d_status, ctx->num_cu, as_stream(stream));
    return launch_check(ctx);
}

raft_status raft_nmi_from_counts(const int64_t* counts, int32_t ka, int32_t kb, double* nmi) {
    if (!counts || !nmi || ka < 1 || kb < 1) return RAFT_E_INVAL;
    // marginals, then I(a;b) and the two entropies in natural log, each
    // summed in row-major order
    std::vector<int64_t> ra(ka, 0), cb(kb, 0);
    int64_t total = 0;
    for (int r = 0; r < ka; ++r)
        for (int c = 0; c < kb; ++c) {
            const int64_t v = counts[(size_t)r * kb + c];
            if (v < 0) return RAFT_E_INVAL;
            ra[r] += v;
            cb[c] += v;
            total += v;
        }
    if (total == 0) return RAFT_E_INVAL;
    const double nt = (double)total;
    double ha = 0.0, hb = 0.0, mi = 0.0;
    for (int r = 0; r < ka; ++r)
        if (ra[r] > 0) {
            const double p = (double)ra[r] / nt;
            ha -= p * std::log(p);
        }
    for (int c = 0; c < kb; ++c)
        if (cb[c] > 0) {
            const double p = (double)cb[c] / nt;
            hb -= p * std::log(p);
        }
    if (ha + hb == 0.0) {
        *nmi = 1.0;
        return RAFT_OK;
    }
    for (int r = 0; r < ka; ++r)
        for (int c = 0; c < kb; ++c) {
            const int64_t v = counts[(size_t)r * kb + c];
            if (v > 0) {
                const double pj = (double)v / nt;
                const double pp = ((double)ra[r] / nt) * ((double)cb[c] / nt);
                mi += pj * std::log(pj / pp);
            }
        }
    *nmi = 2.0 * mi / (ha + hb);
    return RAFT_OK;
}

raft_status raft_run(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg, void* ws,
                     size_t ws_bytes, raft_outputs* out, void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (g->nnz == 0) return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    Plan P;
    RAFT_TRY(plan_for(ctx, g, cfg, ws, ws_bytes, P));
    hipStream_t st = as_stream(stream);
    RAFT_TRY(upload_meta(ctx, P, st));
    float* Y = (out && out->Y) ? out->Y : P.yout;
    float* Z = (out && out->Z) ? out->Z : P.zout;
    HIP_TRY(ctx, hipEventRecord(ctx->ev[0], st));
    RAFT_TRY(do_project(ctx, g, cfg, P, Y, st));
    HIP_TRY(ctx, hipEventRecord(ctx->ev[1], st));
    RAFT_TRY(do_embed(ctx, g, cfg, P, Y, Z, st));
    RAFT_TRY(do_partition(ctx, g, cfg, P, Z, out, st, true));
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev[5]));
    prof_collect(ctx);
    float ms = 0;
    for (int s = 0; s < 5; ++s) {
        if (hipEventElapsedTime(&ms, ctx->ev[s], ctx->ev[s + 1]) == hipSuccess)
            ctx->stage_ms[s] = ms;
    }
    return RAFT_OK;
}

// ---- training -------------------------------------------------------------

namespace {

bool train_width_ok(int v) { return v == 16 || v == 32 || v == 64 || v == 128; }

struct TrainWs {
    float *P, *U, *Ga, *Gb, *WT, *wpart, *S2;
    double* dpart;
    size_t bytes = 0;
};

raft_status train_check(raft_ctx* ctx, const raft_graph* g, int32_t n_layers, const int32_t* dims) {
    RAFT_TRY(check_graph(ctx, g));
    if (n_layers < 1 || n_layers > RAFT_MAX_LAYERS || !dims)
        return fail(ctx, RAFT_E_INVAL, "n_layers %d", n_layers);
    for (int k = 0; k <= n_layers; ++k)
        if (!train_width_ok(dims[k])) return fail(ctx, RAFT_E_UNSUPPORTED, "width %d", dims[k]);
    for (int k = 0; k < n_layers; ++k)
        if (!wgrad_supported(dims[k], dims[k + 1]) || !dense_supported(dims[k], dims[k + 1]) ||
            !dense_supported(dims[k + 1], dims[k]))
            return fail(ctx, RAFT_E_UNSUPPORTED, "layer %d: %d x %d", k + 1, dims[k], dims[k + 1]);
    return RAFT_OK;
}

void train_layout(raft_ctx* ctx, const raft_graph* g, int n_layers, const int32_t* dims, int K,
                  char* base, TrainWs& t) {
    int lmax = K;
    for (int k = 0; k <= n_layers; ++k) lmax = std::max(lmax, (int)dims[k]);
    Arena a;
    a.base = base;
    const size_t nl = (size_t)g->n * lmax;
    t.P = a.take<float>(nl);
    t.U = a.take<float>(nl);
    t.Ga = a.take<float>(nl);
    t.Gb = a.take<float>(nl);
    t.S2 = a.take<float>(nl);
    t.WT = a.take<float>((size_t)lmax * lmax);
    t.wpart = a.take<float>((size_t)wgrad_parts(g->n) * lmax * lmax);
    // column-sum partials (+ stage) for the rank-1 term of B S, and loss partials
    const size_t cs = ((size_t)spmm_grid(g->n, K, ctx->num_cu, nullptr) + kColsumStageRows) * K + 2 * (size_t)K;
    t.dpart = a.take<double>(std::max<size_t>(cs, (size_t)rowdot_parts((int64_t)g->n * K)) + 64);
    t.bytes = a.off;
}

// B S into out (column sums through the workspace's FP64 partials).
void apply_b(raft_ctx* ctx, const raft_graph* g, const float* S, int K, float* out, double* dpart,
             hipStream_t st) {
    const GraphView gv = g->view();
    const int grid = spmm_grid(g->n, K, ctx->num_cu, nullptr);
    double* c64 = dpart + ((size_t)grid + kColsumStageRows) * K;
    float* cvec = reinterpret_cast<float*>(c64 + K);
    launch_colsum_partials(gv, K, S, dpart, ctx->num_cu, st);
    launch_colsum_finish(dpart, grid, K, c64, cvec, st);
    launch_spmm(gv, kOpModFull, K, S, out, cvec, nullptr, ctx->num_cu, st);
}

}  // namespace

raft_status raft_train_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t n_layers,
                                      const int32_t* dims, int32_t K, size_t* bytes) {
    RAFT_TRY(train_check(ctx, g, n_layers, dims));
    if (!bytes || !train_width_ok(K)) return fail(ctx, RAFT_E_INVAL, "bad K or bytes");
    TrainWs t;
    train_layout(ctx, g, n_layers, dims, K, nullptr, t);
    *bytes = t.bytes;
    return RAFT_OK;
}

raft_status raft_gcn_forward(raft_ctx* ctx, const raft_graph* g, int32_t n_layers,
                             const int32_t* dims, const float* H0, const float* const* W,
                             float* const* H_saved, float* U_out, void* ws, size_t ws_bytes,
                             void* stream) {
    RAFT_TRY(train_check(ctx, g, n_layers, dims));
    if (!H0 || !W || !U_out || (n_layers > 1 && !H_saved))
        return fail(ctx, RAFT_E_INVAL, "null buffer");
    TrainWs t;
    train_layout(ctx, g, n_layers, dims, dims[n_layers], nullptr, t);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, t.bytes));
    train_layout(ctx, g, n_layers, dims, dims[n_layers], reinterpret_cast<char*>(ws), t);
    hipStream_t st = as_stream(stream);
    const GraphView gv = g->view();
    const float* h = H0;
    for (int k = 0; k < n_layers; ++k) {
        launch_spmm(gv, kOpGcn, dims[k], h, t.P, nullptr, nullptr, ctx->num_cu, st);
        const bool last = k == n_layers - 1;
        float* out = last ? U_out : H_saved[k];
        if (!out || !W[k]) return fail(ctx, RAFT_E_INVAL, "null layer buffer");
        launch_dense_layer(t.P, W[k], out, g->n, dims[k], dims[k + 1], last, ctx->d_status,
                           ctx->num_cu, st);
        h = out;
    }
    return launch_check(ctx);
}

raft_status raft_gcn_backward(raft_ctx* ctx, const raft_graph* g, int32_t n_layers,
                              const int32_t* dims, const float* H0, const float* const* W,
                              const float* const* H_saved, const float* G_U, float* const* G_W,
                              float* G_H0, void* ws, size_t ws_bytes, void* stream) {
    RAFT_TRY(train_check(ctx, g, n_layers, dims));
    if (!H0 || !W || !G_U || !G_W || (n_layers > 1 && !H_saved))
        return fail(ctx, RAFT_E_INVAL, "null buffer");
    TrainWs t;
    train_layout(ctx, g, n_layers, dims, dims[n_layers], nullptr, t);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, t.bytes));
    train_layout(ctx, g, n_layers, dims, dims[n_layers], reinterpret_cast<char*>(ws), t);
    hipStream_t st = as_stream(stream);
    const GraphView gv = g->view();
    const float* gcur = G_U;        // gradient w.r.t. this layer's output
    float* gnext = t.Ga;
    for (int k = n_layers - 1; k >= 0; --k) {
        const int li = dims[k], lo = dims[k + 1];
        const float* hin = k == 0 ? H0 : H_saved[k - 1];
        launch_spmm(gv, kOpGcn, li, hin, t.P, nullptr, nullptr, ctx->num_cu, st);   // recompute P
        const float* gu = gcur;
        if (k != n_layers - 1) {
            // recompute the pre-activation, then back through normalisation and tanh
            launch_dense_layer(t.P, W[k], t.U, g->n, li, lo, true, ctx->d_status, ctx->num_cu,
                               st);
            launch_tanh_norm_backward(t.U, const_cast<float*>(gcur), g->n, lo, st);
        }
        launch_wgrad(t.P, gu, g->n, li, lo, t.wpart, G_W[k], st);
        if (k > 0 || G_H0) {
            launch_transpose(W[k], li, lo, t.WT, st);
            launch_dense_layer(gu, t.WT, t.Gb, g->n, lo, li, true, ctx->d_status, ctx->num_cu,
                               st);   // G_P
            float* dst = (k == 0) ? G_H0 : gnext;
            launch_spmm(gv, kOpGcn, li, t.Gb, dst, nullptr, nullptr, ctx->num_cu, st);   // A_hat_n G_P
            gcur = dst;
            gnext = (gnext == t.Ga) ? t.S2 : t.Ga;
        }
    }
    return launch_check(ctx);
}

raft_status raft_modloss_forward(raft_ctx* ctx, const raft_graph* g, const float* U, int32_t K,
                                 float* S_out, double* loss, void* ws, size_t ws_bytes,
                                 void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!U || !S_out || !loss || !train_width_ok(K)) return fail(ctx, RAFT_E_INVAL, "bad arguments");
    if (g->nnz == 0) return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    const int32_t dims[2] = {K, K};
    TrainWs t;
    train_layout(ctx, g, 1, dims, K, nullptr, t);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, t.bytes));
    train_layout(ctx, g, 1, dims, K, reinterpret_cast<char*>(ws), t);
    hipStream_t st = as_stream(stream);
    launch_softmax_rows(U, S_out, g->n, K, st);
    apply_b(ctx, g, S_out, K, t.U, t.dpart, st);
    launch_modloss_value(S_out, t.U, (int64_t)g->n * K, (double)g->nnz, t.dpart, loss, st);
    return launch_check(ctx);
}

raft_status raft_modloss_backward(raft_ctx* ctx, const raft_graph* g, const float* S, int32_t K,
                                  const float* scale, float* G_U, void* ws, size_t ws_bytes,
                                  void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!S || !G_U || !train_width_ok(K)) return fail(ctx, RAFT_E_INVAL, "bad arguments");
    if (g->nnz == 0) return fail(ctx, RAFT_E_NOEDGES, "modularity needs e > 0");
    const int32_t dims[2] = {K, K};
    TrainWs t;
    train_layout(ctx, g, 1, dims, K, nullptr, t);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, t.bytes));
    train_layout(ctx, g, 1, dims, K, reinterpret_cast<char*>(ws), t);
    hipStream_t st = as_stream(stream);
    apply_b(ctx, g, S, K, t.U, t.dpart, st);
    launch_modloss_grad(S, t.U, g->n, K, 2.0 / (double)g->nnz, scale, G_U, st);
    return launch_check(ctx);
}

raft_status raft_adam_step(raft_ctx* ctx, float* w, float* m, float* v, const float* grad,
                           int64_t n, float lr, float beta1, float beta2, float eps, int32_t step,
                           void* stream) {
    if (!ctx) return RAFT_E_INVAL;
    if (n < 0 || (n > 0 && (!w || !m || !v || !grad)) || step < 1)
        return fail(ctx, RAFT_E_INVAL, "bad Adam arguments");
    launch_adam(w, m, v, grad, n, lr, beta1, beta2, eps, step, as_stream(stream));
    return launch_check(ctx);
}

raft_status raft_profile_enable(raft_ctx* ctx, uint32_t mask) {
    if (!ctx) return RAFT_E_INVAL;
    HIP_TRY(ctx, hipDeviceSynchronize());
    prof_collect(ctx);
    ctx->prof_mask = mask & ((1u << RAFT_PROF_CLASSES) - 1);
    return RAFT_OK;
}

raft_status raft_profile_read(raft_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx || !ms || !launches) return RAFT_E_INVAL;
    HIP_TRY(ctx, hipDeviceSynchronize());
    prof_collect(ctx);
    for (int k = 0; k < RAFT_PROF_CLASSES; ++k) {
        ms[k] = ctx->prof_ms[k];
        launches[k] = ctx->prof_n[k];
        ctx->prof_ms[k] = 0;
        ctx->prof_n[k] = 0;
    }
    return RAFT_OK;
}

raft_status raft_get_stage_times(raft_ctx* ctx, double* ms5) {
    if (!ctx || !ms5) return RAFT_E_INVAL;
    for (int s = 0; s < 5; ++s) ms5[s] = ctx->stage_ms[s];
    return RAFT_OK;
}

}  // extern "C"

// ---- batches of graphs (block-diagonal CSR, one launch per stage) --------

struct raft_batch {
    raft_ctx* ctx = nullptr;
    int G = 0;
    raft_config cfg{};
    std::vector<raft_graph> shadow;      // n and nnz of each graph (plan sizes)
    std::vector<uint64_t> seeds;
    std::vector<int32_t> base;           // first row of graph g in the packed CSR
    std::vector<int64_t> ebase;          // first stored entry of graph g
    int32_t N = 0;
    int64_t NNZ = 0;
    int32_t *rp = nullptr, *ci = nullptr, *deg = nullptr, *order = nullptr;
    float *s = nullptr, *sh = nullptr, *dcoef = nullptr;
    // the captured embedding + seeding launches, valid for one workspace
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* exec_ws = nullptr;
    // pinned host memory of the convergence polls: two slots of the dynamic
    // control part and two of the active flags, allocated once
    char* h_poll = nullptr;
    size_t dyn_bytes = 0, flag_bytes = 0;
    hipEvent_t poll_ev[2] = {};
    double stage_ms[3] = {0, 0, 0};
    hipEvent_t ev[4] = {};
    // tuner: share multiplier of the result-invariant shapes (0 = not chosen)
    int factor = 0;
    int graph_factor = -1;            // factor the recorded HIP graph was built for
    std::vector<std::pair<int, double>> tune_ms;
};

namespace {

// Work-group table of one batched launch kind (host side).
struct HostTable {
    std::vector<int32_t> start, count;
    int grid = 0;
    size_t off = 0;   // offset in the control block
};

HostTable make_table(const std::vector<int>& counts) {
    HostTable t;
    const int G = (int)counts.size();
    t.start.assign(G + 1, 0);
    t.count.assign(G, 0);
    for (int g = 0; g < G; ++g) {
        t.count[g] = counts[g];
        t.start[g + 1] = t.start[g] + (counts[g] + 7) / 8 * 8;
    }
    t.grid = t.start[G];
    return t;
}

enum BatchTab {
    bt_one, bt_gtheta, bt_cpart, bt_cslices, bt_spmm_proj, bt_dense, bt_rownorm, bt_reset,
    bt_zmax, bt_split, bt_race, bt_init, bt_ufinish, bt_transpose, bt_edge, bt_reduce,
    bt_sfinal, bt_first, bt_apply, bt_copy, bt_gw0, bt_spmm_layer0 = bt_gw0 + RAFT_MAX_LAYERS,
    bt_static_end = bt_spmm_layer0 + RAFT_MAX_LAYERS
};

// Per-run layout of a batch: the control block (per-graph plans, launch
// items and tables, uploaded from the host), the packed feature buffers, and
// one single-graph partition layout per graph.
struct BatchLayout {
    int Kc = 0, KP = 0, SK = 0, L = 0, d = 0, Lmax = 0, S = 0;
    std::vector<Plan> P;
    std::vector<GraphView> gv;
    std::vector<KmeansPlan> km;
    std::vector<ScorePlan> sc;
    std::vector<HostTable> tab;          // static tables, index BatchTab
    HostTable tab_assign, tab_update;
    // control block offsets
    size_t off_meta = 0, off_gv = 0, off_sc = 0, off_spmm = 0, off_cs = 0, off_ga = 0,
           off_de = 0, off_dyn = 0, off_km = 0, off_lists = 0, off_ta = 0, off_tu = 0,
           off_flags = 0, ctl_upload = 0, ctl_bytes = 0;
    // feature buffers (device)
    float *Y0 = nullptr, *Y1 = nullptr, *PB = nullptr, *YO = nullptr, *Zp = nullptr;
    char* ctl = nullptr;
    size_t bytes = 0;
    std::vector<char> host;              // the uploaded part of the control block
};

template <typename T>
T* at(char* base, size_t off) {
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
}

BatchTable dev_table(char* ctl, const HostTable& t, int G) {
    BatchTable b;
    b.start = at<int32_t>(ctl, t.off);
    b.count = at<int32_t>(ctl, t.off + sizeof(int32_t) * (size_t)(G + 1));
    b.G = G;
    return b;
}

size_t table_bytes(int G) { return sizeof(int32_t) * (size_t)(2 * G + 1); }

void put_table(std::vector<char>& host, const HostTable& t) {
    memcpy(host.data() + t.off, t.start.data(), sizeof(int32_t) * t.start.size());
    memcpy(host.data() + t.off + sizeof(int32_t) * t.start.size(), t.count.data(),
           sizeof(int32_t) * t.count.size());
}

int width_in(const raft_config* c, int k) { return k == 0 ? c->proj_dim : c->layer_dims[k - 1]; }

// Builds the layout for workspace `ws` (nullptr: sizes only) and the host
// image of the control block.
// CUs graph g's result-invariant shapes are sized for: its part of the chip
// by node count times the tuner's factor (factor <= 0: the whole chip, the
// single-graph shapes, which also bound the workspace).
int batch_share(const raft_batch* b, int g, int factor) {
    const int cu = b->ctx->num_cu;
    if (factor <= 0) return cu;
    const double part = (double)cu * factor * b->shadow[g].n / std::max<int64_t>(1, b->N);
    return (int)std::max<double>(8.0, std::min<double>(cu, std::ceil(part)));
}

void batch_layout(raft_batch* b, char* ws, raft_outputs* outs, BatchLayout& B, int factor) {
    raft_ctx* ctx = b->ctx;
    const raft_config* c = &b->cfg;
    const int G = b->G;
    const Grid grid = make_grid(c->k_min, c->k_max, c->k_step);
    B.Kc = grid.Kc;
    B.KP = grid.KP;
    B.SK = grid.SK;
    B.L = c->proj_dim;
    B.d = embed_dim(c);
    B.Lmax = max_width(c);
    B.S = (grid.Kc + 7) / 8 * 8;
    const int nl = c->n_layers;
    // control block
    Arena a;
    a.base = ws;
    B.ctl = ws;
    B.off_meta = a.off;
    a.take<int32_t>((size_t)3 * B.Kc + B.KP);
    B.off_gv = a.off;
    a.take<GraphView>(G);
    B.off_sc = a.off;
    a.take<ScorePlan>(G);
    B.off_spmm = a.off;
    a.take<SpmmItem>((size_t)(nl + 1) * G);
    B.off_cs = a.off;
    a.take<ColsumItem>(G);
    B.off_ga = a.off;
    a.take<GaussItem>((size_t)(nl + 1) * G);
    B.off_de = a.off;
    a.take<DenseItem>((size_t)(nl + 1) * G);
    B.tab.assign(bt_static_end, HostTable());
    std::vector<size_t> tab_off(bt_static_end);
    for (int t = 0; t < bt_static_end; ++t) {
        tab_off[t] = a.off;
        a.take<char>(table_bytes(G));
    }
    // the dynamic part, rewritten at every convergence poll
    B.off_dyn = a.off;
    B.off_km = a.off;
    a.take<KmeansPlan>(G);
    B.off_lists = a.off;
    a.take<int32_t>((size_t)G * kDynLen(B.Kc));
    B.off_ta = a.off;
    a.take<char>(table_bytes(G));
    B.off_tu = a.off;
    a.take<char>(table_bytes(G));
    B.ctl_upload = a.off;
    // device-written active flags of every candidate of every graph
    B.off_flags = a.off;
    a.take<int32_t>((size_t)G * B.Kc);
    B.ctl_bytes = a.off;
    // packed features
    const size_t NL = (size_t)b->N * B.Lmax;
    B.Y0 = a.take<float>(NL);
    B.Y1 = a.take<float>(NL);
    B.PB = a.take<float>(NL);
    B.YO = a.take<float>((size_t)b->N * B.L);
    B.Zp = a.take<float>((size_t)b->N * B.d);
    // per graph: the single-graph layout without feature buffers
    B.P.assign(G, Plan());
    B.gv.assign(G, GraphView());
    B.km.assign(G, KmeansPlan());
    B.sc.assign(G, ScorePlan());
    for (int g = 0; g < G; ++g) {
        raft_config cg = *c;
        cg.seed = b->seeds[g];
        char* sub = ws ? ws + a.off : nullptr;
        plan_layout(ctx, &b->shadow[g], &cg, sub, B.P[g], false, batch_share(b, g, factor));
        a.off += align256(B.P[g].bytes);
    }
    B.bytes = a.off;
    if (!ws) return;
    // ---- host image of the control block ----
    B.host.assign(B.ctl_upload, 0);
    char* H = B.host.data();
    char* D = ws;
    {
        int32_t* m = reinterpret_cast<int32_t*>(H + B.off_meta);
        std::copy(grid.ks.begin(), grid.ks.end(), m);
        std::copy(grid.koff16.begin(), grid.koff16.end(), m + B.Kc);
        std::copy(grid.koff.begin(), grid.koff.end(), m + 2 * B.Kc);
        std::copy(grid.cand_of.begin(), grid.cand_of.end(), m + 3 * B.Kc);
    }
    const int32_t* d_meta = at<int32_t>(D, B.off_meta);
    int32_t* d_lists = at<int32_t>(D, B.off_lists);
    int32_t* d_flags = at<int32_t>(D, B.off_flags);
    std::vector<std::vector<int>> cnt(bt_static_end, std::vector<int>(G, 0));
    for (int g = 0; g < G; ++g) {
        Plan& P = B.P[g];
        const raft_graph& sg = b->shadow[g];
        raft_outputs* o = outs ? &outs[g] : nullptr;
        GraphView v;
        v.n = sg.n;
        v.nnz = sg.nnz;
        v.rp = b->rp;
        v.ci = b->ci;
        v.deg = b->deg;
        v.s = b->s;
        v.sh = b->sh;
        v.dcoef = b->dcoef;
        v.order = b->order + b->base[g];
        v.base = b->base[g];
        B.gv[g] = v;
        KmeansPlan km = P.km;
        km.ks = d_meta;
        km.koff16 = d_meta + B.Kc;
        km.koff = d_meta + 2 * B.Kc;
        km.cand_of = d_meta + 3 * B.Kc;
        int32_t* dl = d_lists + (size_t)g * kDynLen(B.Kc);
        km.alist = dl;
        km.agrp = dl + B.Kc;
        km.ugrp = dl + 2 * B.Kc + 1;
        km.uwi0 = dl + 3 * B.Kc + 2;
        km.ulen = dl + 4 * B.Kc + 3;
        km.cranges = dl + 5 * B.Kc + 3;
        km.active = d_flags + (size_t)g * B.Kc;
        if (o && o->picks) km.picks = o->picks;
        if (o && o->iters) km.iters = o->iters;
        km.zoff = b->base[g];
        km.seed = b->seeds[g];
        B.km[g] = km;
        pack_lists(P.lists, B.Kc,
                   reinterpret_cast<int32_t*>(H + B.off_lists) + (size_t)g * kDynLen(B.Kc));
        ScorePlan sc = P.sc;
        sc.ks = d_meta;
        sc.koff = d_meta + 2 * B.Kc;
        if (o && o->mod) sc.mod = o->mod;
        if (o && o->ncut) sc.ncut = o->ncut;
        sc.lab = P.lab_pm;
        sc.lab_cm = km.lab_cm;
        sc.ksel_out = (o && o->k_selected) ? o->k_selected : P.ksel_int;
        sc.labels_out = o ? o->labels : nullptr;
        sc.labels_all_out = o ? o->labels_all : nullptr;
        B.sc[g] = sc;
        // launch items
        const int n = sg.n;
        for (int k = 0; k <= c->n_layers; ++k) {
            // item k: the projection (k = 0) or the aggregation of layer k,
            // whose SpMM runs at the layer's input width
            const int w = width_in(c, k);
            const int wsp = k == 0 ? B.L : width_in(c, k - 1);
            SpmmItem it;
            it.g = v;
            it.cvec = P.cvec;
            it.cpart = P.cpart;
            it.R = 0;
            it.nrb = 0;
            const int gridk = spmm_launch_shape(n, wsp, ctx->num_cu, &it.R, &it.nrb);
            cnt[k == 0 ? bt_spmm_proj : bt_spmm_layer0 + k - 1][g] = gridk;
            reinterpret_cast<SpmmItem*>(H + B.off_spmm)[(size_t)k * G + g] = it;
            GaussItem ga;
            ga.seed = b->seeds[g];
            if (k == 0) {
                ga.stream = 0x10;
                ga.rows = n;
                ga.cols = B.L;
                ga.sigma = 1.0 / std::sqrt((double)B.L);
                ga.out = B.Y0 + (size_t)b->base[g] * B.L;
                cnt[bt_gtheta][g] = gaussian_blocks(n, B.L);
            } else {
                const int lin = width_in(c, k - 1);
                ga.stream = 0x10 + (uint64_t)k;
                ga.rows = lin;
                ga.cols = w;
                ga.sigma = 1.0 / std::sqrt((double)lin);
                ga.out = P.wbuf;
                cnt[bt_gw0 + k - 1][g] = gaussian_blocks(lin, w);
            }
            reinterpret_cast<GaussItem*>(H + B.off_ga)[(size_t)k * G + g] = ga;
        }
        ColsumItem cs;
        cs.g = v;
        cs.part = P.cpart;
        int rpw = 0;
        cs.parts = spmm_grid(n, B.L, ctx->num_cu, &rpw);
        cs.rpw = rpw;
        cs.c64 = P.c64;
        cs.cvec = P.cvec;
        reinterpret_cast<ColsumItem*>(H + B.off_cs)[g] = cs;
        cnt[bt_cpart][g] = cs.parts;
        cnt[bt_cslices][g] = cs.parts > 0 ? kColsumSliceBlocks : 0;
        cnt[bt_one][g] = 1;
        cnt[bt_dense][g] = dense_blocks(n);
        cnt[bt_rownorm][g] = rownorm_blocks(n);
        cnt[bt_reset][g] = kmeans_blocks(km, kKmReset, ctx->num_cu);
        cnt[bt_zmax][g] = kmeans_blocks(km, kKmZmax, ctx->num_cu);
        cnt[bt_split][g] = km.split ? kmeans_blocks(km, kKmSplit, ctx->num_cu) : 0;
        cnt[bt_race][g] = kmeans_blocks(km, kKmRace, ctx->num_cu);
        cnt[bt_init][g] = kmeans_blocks(km, kKmInit, ctx->num_cu);
        // rows walked grid-stride (k_update_finish_b): two work-groups per
        // CU of the graph's share of the chip, and at most 16 rows per
        // work-group (every graph has the grid's full row count, however
        // small its share)
        cnt[bt_ufinish][g] = std::min(kmeans_blocks(km, kKmUpdateFinish, ctx->num_cu),
                                      std::max(2 * P.share, (km.KP + 1 + 15) / 16));
        cnt[bt_transpose][g] = score_blocks(sc, kScTranspose);
        cnt[bt_edge][g] = score_blocks(sc, kScEdge);
        cnt[bt_reduce][g] = score_blocks(sc, kScReduce);
        cnt[bt_sfinal][g] = score_blocks(sc, kScFinalize);
        cnt[bt_first][g] = score_blocks(sc, kScFirst);
        cnt[bt_apply][g] = sc.labels_out ? score_blocks(sc, kScApply) : 0;
        cnt[bt_copy][g] = sc.labels_all_out ? score_blocks(sc, kScCopy) : 0;
    }
    // dense items: layer k reads PB, writes the layer's destination buffer
    {
        DenseItem* de = reinterpret_cast<DenseItem*>(H + B.off_de);
        const float* h = B.YO;
        float* hbuf = c->normalize_input ? B.Y1 : nullptr;
        if (hbuf) h = hbuf;
        for (int g = 0; g < G; ++g) {
            DenseItem it;
            it.P = nullptr;
            it.W = nullptr;
            it.H = (c->n_layers == 0 ? B.Zp : B.Y1) + (size_t)b->base[g] * B.L;
            it.n = b->shadow[g].n;
            de[(size_t)c->n_layers * G + g] = it;      // row normalisation of the input
        }
        for (int k = 1; k <= c->n_layers; ++k) {
            const int lin = width_in(c, k - 1), lout = width_in(c, k);
            float* dst = (k == c->n_layers) ? B.Zp : (h == B.Y0 ? B.Y1 : B.Y0);
            for (int g = 0; g < G; ++g) {
                DenseItem it;
                it.P = B.PB + (size_t)b->base[g] * lin;
                it.W = B.P[g].wbuf;
                it.H = dst + (size_t)b->base[g] * lout;
                it.n = b->shadow[g].n;
                de[(size_t)(k - 1) * G + g] = it;
            }
            h = dst;
        }
    }
    for (int t = 0; t < bt_static_end; ++t) {
        B.tab[t] = make_table(cnt[t]);
        B.tab[t].off = tab_off[t];
        put_table(B.host, B.tab[t]);
    }
    memcpy(H + B.off_gv, B.gv.data(), sizeof(GraphView) * G);
    memcpy(H + B.off_sc, B.sc.data(), sizeof(ScorePlan) * G);
}

// Dynamic tables from the plans' current work lists (0 for a graph whose
// candidates have all stopped), written with the plans into the host image.
void batch_dynamic(raft_batch* b, BatchLayout& B, char* H, const std::vector<int>& live) {
    const int G = b->G;
    std::vector<int> ca(G), cu(G);
    for (int g = 0; g < G; ++g) {
        ca[g] = live[g] ? kmeans_blocks(B.km[g], kKmAssign, b->ctx->num_cu) : 0;
        cu[g] = live[g] ? kmeans_blocks(B.km[g], kKmUpdate, b->ctx->num_cu) : 0;
    }
    B.tab_assign = make_table(ca);
    B.tab_assign.off = B.off_ta - B.off_dyn;
    B.tab_update = make_table(cu);
    B.tab_update.off = B.off_tu - B.off_dyn;
    memcpy(H + (B.off_km - B.off_dyn), B.km.data(), sizeof(KmeansPlan) * G);
    const HostTable* ts[2] = {&B.tab_assign, &B.tab_update};
    for (const HostTable* t : ts) {
        memcpy(H + t->off, t->start.data(), sizeof(int32_t) * t->start.size());
        memcpy(H + t->off + sizeof(int32_t) * t->start.size(), t->count.data(),
               sizeof(int32_t) * t->count.size());
    }
    B.tab_assign.off = B.off_ta;
    B.tab_update.off = B.off_tu;
}

// Host check of a batch layout before anything is launched: every array a
// kernel of graph g indexes (at the extent its single-graph launch uses)
// lies inside the graph's own part of the workspace, the control block or
// the packed feature buffers, the parts do not overlap, and every table
// gives each graph at least its count of work-groups.
struct Span {
    const char* lo;
    size_t len;
};

bool span_in(const void* p, size_t bytes, const char* lo, size_t len) {
    const char* q = reinterpret_cast<const char*>(p);
    return q >= lo && bytes <= len && (size_t)(q - lo) <= len - bytes;
}

raft_status batch_check(raft_ctx* ctx, const raft_batch* b, const BatchLayout& B,
                        size_t ws_bytes) {
    const int G = b->G;
    const char* ws = B.ctl;
    if (B.bytes > ws_bytes) return fail(ctx, RAFT_E_WORKSPACE, "batch layout exceeds workspace");
    const char* ctl = ws;
    const size_t NL = (size_t)b->N * B.Lmax * sizeof(float);
    auto bad = [&](int g, const char* what) {
        return fail(ctx, RAFT_E_INVAL, "batch layout check: graph %d, %s", g, what);
    };
    std::vector<Span> subs;
    size_t off = 0;
    {
        // the per-graph parts follow the features, in graph order
        off = (size_t)(reinterpret_cast<const char*>(B.Zp) - ws) +
              align256((size_t)b->N * B.d * sizeof(float));
    }
    for (int g = 0; g < G; ++g) {
        const Plan& P = B.P[g];
        const char* lo = ws + off;
        const size_t len = P.bytes;
        if (off + len > B.bytes) return bad(g, "part beyond the layout");
        off += align256(len);
        const KmeansPlan& k = B.km[g];
        const ScorePlan& c = B.sc[g];
        const size_t n = (size_t)b->shadow[g].n, d = (size_t)B.d, KP = (size_t)B.KP;
        const size_t Kc = (size_t)B.Kc;
        const size_t rmax = (size_t)update_ranges_max(b->shadow[g].n, P.share);
        struct Need {
            const void* p;
            size_t bytes;
            const char* name;
        } own[] = {
            {k.C, KP * d * 4, "C"}, {k.cnorm, KP * 4, "cnorm"},
            {k.S64, KP * d * 8, "S64"}, {k.N32, KP * 4, "N32"},
            {k.pdelta, rmax * KP * d * 8, "pdelta"}, {k.pcnt, rmax * KP * 4, "pcnt"},
            {k.pdirty, rmax * KP, "pdirty"}, {k.zmax_bits, 4, "zmax"}, {k.w, n * 4, "w"},
            {k.race_val, (size_t)2 * k.race_grid * 8, "race_val"},
            {k.race_idx, (size_t)2 * k.race_grid * 4, "race_idx"},
            {k.lab_cm, Kc * n, "lab_cm"}, {k.lab_old, Kc * n, "lab_old"},
            {k.moved_it, (size_t)k.nchunks * Kc * 4, "moved_it"},
            {k.changes, Kc * 4, "changes"}, {k.active_count, 4, "active_count"},
            {c.lpart, (size_t)c.grid * B.SK * 4, "lpart"},
            {c.vpart, (size_t)c.grid * B.SK * 4, "vpart"}, {c.l64, (size_t)B.SK * 8, "l64"},
            {c.v64, (size_t)B.SK * 8, "v64"}, {c.best, 4, "best"},
            {c.first, (RAFT_MAX_K + 1) * 4, "first"}, {c.remap, (RAFT_MAX_K + 1) * 4, "remap"},
            {c.lab, n * (size_t)B.S, "lab"},
            {P.cpart, ((size_t)spmm_grid((int32_t)n, B.L, ctx->num_cu, nullptr) + kColsumStageRows) *
                          B.L * 8, "cpart"},
            {P.c64, (size_t)B.L * 8, "c64"}, {P.cvec, (size_t)B.L * 4, "cvec"},
        };
        for (const Need& q : own)
            if (!span_in(q.p, q.bytes, lo, len)) return bad(g, q.name);
        if (k.split && (!span_in(k.zh, n * d * 2, lo, len) || !span_in(k.zl, n * d * 2, lo, len) ||
                        !span_in(k.ch, KP * d * 2, lo, len) || !span_in(k.cl, KP * d * 2, lo, len)))
            return bad(g, "split halves");
        // outputs may be caller memory; internal defaults must be in the part
        if (k.n != (int)n || k.d != (int)d || k.Kc != B.Kc || k.KP != B.KP) return bad(g, "plan sizes");
        if (!span_in(k.active, Kc * 4, ctl + B.off_flags, (size_t)G * Kc * 4)) return bad(g, "flags");
        if (!span_in(k.alist, (size_t)kDynLen(B.Kc) * 4, ctl + B.off_lists,
                     (size_t)G * kDynLen(B.Kc) * 4))
            return bad(g, "lists");
        if ((size_t)k.zoff + n > (size_t)b->N || b->base[g] != k.zoff) return bad(g, "zoff");
        if (B.gv[g].base != b->base[g] || B.gv[g].n != (int)n) return bad(g, "view");
        // widths of the layers: W buffer and row ranges of the packed features
        size_t wmax = 1;
        for (int l = 1; l <= b->cfg.n_layers; ++l)
            wmax = std::max(wmax, (size_t)width_in(&b->cfg, l - 1) * width_in(&b->cfg, l));
        if (!span_in(P.wbuf, wmax * 4, lo, len)) return bad(g, "W");
        for (int l = 0; l <= b->cfg.n_layers; ++l)
            if (((size_t)b->base[g] + n) * width_in(&b->cfg, l) * 4 > NL) return bad(g, "features");
        for (int t = 0; t < bt_static_end; ++t) {
            const HostTable& h = B.tab[t];
            if (h.start[g + 1] - h.start[g] < h.count[g] || h.start[g] % 8) return bad(g, "table");
        }
    }
    for (int t = 0; t < bt_static_end; ++t)
        if (B.tab[t].grid != B.tab[t].start[G]) return fail(ctx, RAFT_E_INVAL, "table grid");
    if (off > B.bytes) return fail(ctx, RAFT_E_INVAL, "parts beyond the layout");
    return RAFT_OK;
}

// The fixed launch sequence before the Lloyd loop: projection, GCN, k-means
// reset, scales and the k-means++ race.  Recorded into a HIP graph.
raft_status batch_prefix(raft_batch* b, BatchLayout& B, hipStream_t st) {
    raft_ctx* ctx = b->ctx;
    const raft_config* c = &b->cfg;
    const int G = b->G;
    char* D = B.ctl;
    auto T = [&](int k) { return dev_table(D, B.tab[k], G); };
    auto grid = [&](int k) { return B.tab[k].grid; };
    const SpmmItem* sp = at<SpmmItem>(D, B.off_spmm);
    const GaussItem* ga = at<GaussItem>(D, B.off_ga);
    const DenseItem* de = at<DenseItem>(D, B.off_de);
    const ColsumItem* cs = at<ColsumItem>(D, B.off_cs);
    const KmeansPlan* km = at<KmeansPlan>(D, B.off_km);
    const int L = B.L;
    // projection
    launch_gaussian_batched(ga, T(bt_gtheta), grid(bt_gtheta), st);
    const bool mod_full = c->op == RAFT_X_MOD_FULL;
    float* src = B.Y0;
    if (mod_full) {
        launch_colsum_partials_batched(cs, L, src, T(bt_cpart), grid(bt_cpart), st);
        launch_colsum_finish_batched(cs, L, T(bt_cslices), grid(bt_cslices), T(bt_one),
                                     grid(bt_one), st);
    }
    for (int t = 1; t <= c->q; ++t) {
        float* dst = (t == c->q) ? B.YO : (src == B.Y0 ? B.Y1 : B.Y0);
        const bool need_cs = mod_full && t < c->q;
        launch_spmm_batched(sp, c->op, L, src, dst, need_cs, T(bt_spmm_proj), grid(bt_spmm_proj),
                            st);
        if (need_cs)
            launch_colsum_finish_batched(cs, L, T(bt_cslices), grid(bt_cslices), T(bt_one),
                                         grid(bt_one), st);
        src = dst;
    }
    // GCN
    const float* h = B.YO;
    if (c->n_layers == 0) {
        HIP_TRY(ctx, hipMemcpyAsync(B.Zp, B.YO, (size_t)b->N * L * sizeof(float),
                                    hipMemcpyDeviceToDevice, st));
        if (c->normalize_input)
            launch_rownorm_batched(de, L, T(bt_rownorm), grid(bt_rownorm), st);
    } else {
        if (c->normalize_input) {
            HIP_TRY(ctx, hipMemcpyAsync(B.Y1, B.YO, (size_t)b->N * L * sizeof(float),
                                        hipMemcpyDeviceToDevice, st));
            launch_rownorm_batched(de + (size_t)c->n_layers * G, L, T(bt_rownorm),
                                   grid(bt_rownorm), st);
            h = B.Y1;
        }
        int lin = L;
        for (int k = 1; k <= c->n_layers; ++k) {
            const int lout = c->layer_dims[k - 1];
            launch_gaussian_batched(ga + (size_t)k * G, T(bt_gw0 + k - 1), grid(bt_gw0 + k - 1),
                                    st);
            launch_spmm_batched(sp + (size_t)k * G, kOpGcn, lin, h, B.PB, false,
                                T(bt_spmm_layer0 + k - 1), grid(bt_spmm_layer0 + k - 1), st);
            launch_dense_layer_batched(de + (size_t)(k - 1) * G, lin, lout, false, ctx->d_status,
                                       T(bt_dense), grid(bt_dense), st);
            h = (k == c->n_layers) ? B.Zp : (h == B.Y0 ? B.Y1 : B.Y0);
            lin = lout;
        }
    }
    // k-means reset, scales, seeding
    const int d = B.d;
    const bool split = B.P[0].km.split != 0;
    const int kmax = B.P[0].km.k_max;
    launch_kmeans_batched(kKmReset, km, d, split, B.Zp, 0, 0, 0, 0, T(bt_reset), grid(bt_reset),
                          st);
    launch_kmeans_batched(kKmZmax, km, d, split, B.Zp, 0, 0, 0, 0, T(bt_zmax), grid(bt_zmax), st);
    if (split)
        launch_kmeans_batched(kKmSplit, km, d, split, B.Zp, 0, 0, 0, 0, T(bt_split),
                              grid(bt_split), st);
    for (int t = 0; t < kmax; ++t)
        launch_kmeans_batched(kKmRace, km, d, split, B.Zp, t, 0, 0, 0, T(bt_race), grid(bt_race),
                              st);
    launch_kmeans_batched(kKmRaceFinal, km, d, split, B.Zp, 0, 0, 0, 0, T(bt_one), grid(bt_one),
                          st);
    launch_kmeans_batched(kKmInit, km, d, split, B.Zp, 0, 0, 0, 0, T(bt_init), grid(bt_init), st);
    return launch_check(ctx);
}

}  // namespace

extern "C" {

raft_status raft_batch_create(raft_ctx* ctx, int32_t G, const raft_graph* const* graphs,
                              const uint64_t* seeds, const raft_config* cfg, raft_batch** out) {
    if (!ctx) return RAFT_E_INVAL;
    if (!out) return fail(ctx, RAFT_E_INVAL, "out is null");
    *out = nullptr;
    if (G < 1 || !graphs) return fail(ctx, RAFT_E_INVAL, "batch of %d graphs", G);
    RAFT_TRY(check_config(ctx, nullptr, cfg));
    const int d = embed_dim(cfg);
    if (!kmeans_supported(d)) return fail(ctx, RAFT_E_UNSUPPORTED, "embedding width %d", d);
    if (max_width(cfg) > 256)
        return fail(ctx, RAFT_E_UNSUPPORTED, "batches take widths up to 256 (widest %d)",
                    max_width(cfg));
    int64_t N = 0, NNZ = 0;
    for (int g = 0; g < G; ++g) {
        RAFT_TRY(check_graph(ctx, graphs[g]));
        if (graphs[g]->nnz == 0) return fail(ctx, RAFT_E_NOEDGES, "graph %d has no edges", g);
        if (cfg->k_max > graphs[g]->n)
            return fail(ctx, RAFT_E_INVAL, "k_max %d exceeds N of graph %d", cfg->k_max, g);
        N += graphs[g]->n;
        NNZ += graphs[g]->nnz;
    }
    if (N >= INT32_MAX || NNZ >= INT32_MAX)
        return fail(ctx, RAFT_E_UNSUPPORTED, "batch of %lld rows, %lld entries exceeds int32",
                    (long long)N, (long long)NNZ);
    {
        Plan P;
        plan_layout(ctx, graphs[0], cfg, nullptr, P);
        if (kmeans_update_lds(P.ucap, d) > ctx->lds_max)
            return fail(ctx, RAFT_E_UNSUPPORTED, "k_max %d too large for width %d", P.grid.k_max, d);
        if (!score_supported(P.grid.Kc, P.grid.SK))
            return fail(ctx, RAFT_E_UNSUPPORTED,
                        "%d candidates with sum of K %d (at most 256 and 16384)", P.grid.Kc,
                        P.grid.SK);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    raft_batch* b = new raft_batch();
    b->ctx = ctx;
    b->G = G;
    b->cfg = *cfg;
    b->N = (int32_t)N;
    b->NNZ = NNZ;
    b->shadow.resize(G);
    b->seeds.resize(G);
    b->base.resize(G);
    b->ebase.resize(G);
    int64_t r = 0, e = 0;
    for (int g = 0; g < G; ++g) {
        b->shadow[g].ctx = ctx;
        b->shadow[g].n = graphs[g]->n;
        b->shadow[g].nnz = graphs[g]->nnz;
        std::copy(graphs[g]->heavy, graphs[g]->heavy + 17, b->shadow[g].heavy);
        b->seeds[g] = seeds ? seeds[g] : cfg->seed;
        b->base[g] = (int32_t)r;
        b->ebase[g] = e;
        r += graphs[g]->n;
        e += graphs[g]->nnz;
    }
    auto cleanup = [&](raft_status st, const char* what) {
        raft_batch_destroy(b);
        return fail(ctx, st, "%s", what);
    };
    bool ok = hipMalloc(&b->rp, sizeof(int32_t) * ((size_t)N + 1)) == hipSuccess &&
              hipMalloc(&b->ci, sizeof(int32_t) * (size_t)NNZ) == hipSuccess &&
              hipMalloc(&b->deg, sizeof(int32_t) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->order, sizeof(int32_t) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->s, sizeof(float) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->sh, sizeof(float) * (size_t)N) == hipSuccess &&
              hipMalloc(&b->dcoef, sizeof(float) * (size_t)N) == hipSuccess;
    if (!ok) return cleanup(RAFT_E_NOMEM, "batch allocation failed");
    // pack the graphs: block g of the block-diagonal CSR is graph g with its
    // rows at base[g], its columns shifted by base[g], its entries at ebase[g]
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return cleanup(RAFT_E_DEVICE, "stream creation failed");
    b->cap_stream = st;
    hipError_t err = hipSuccess;
    for (int g = 0; g < G && err == hipSuccess; ++g) {
        const raft_graph* gr = graphs[g];
        const size_t off = (size_t)b->base[g];
        launch_offset_copy(gr->rp, b->rp + off, (int64_t)gr->n + 1, (int32_t)b->ebase[g], st);
        launch_offset_copy(gr->ci, b->ci + b->ebase[g], gr->nnz, b->base[g], st);
        launch_offset_copy(gr->order, b->order + off, gr->n, b->base[g], st);
        err = hipMemcpyAsync(b->deg + off, gr->deg, sizeof(int32_t) * gr->n,
                             hipMemcpyDeviceToDevice, st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(b->s + off, gr->s, sizeof(float) * gr->n, hipMemcpyDeviceToDevice,
                                 st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(b->sh + off, gr->sh, sizeof(float) * gr->n,
                                 hipMemcpyDeviceToDevice, st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(b->dcoef + off, gr->dcoef, sizeof(float) * gr->n,
                                 hipMemcpyDeviceToDevice, st);
        if (err == hipSuccess) err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) return cleanup(RAFT_E_DEVICE, "batch packing failed");
    // pinned poll buffers
    BatchLayout B;
    batch_layout(b, nullptr, nullptr, B, 0);
    b->dyn_bytes = B.ctl_upload - B.off_dyn;
    b->flag_bytes = sizeof(int32_t) * (size_t)G * B.Kc;
    if (hipHostMalloc((void**)&b->h_poll, 2 * (b->dyn_bytes + b->flag_bytes),
                      hipHostMallocDefault) != hipSuccess)
        return cleanup(RAFT_E_NOMEM, "pinned poll buffer");
    for (auto& ev : b->poll_ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return cleanup(RAFT_E_DEVICE, "event creation failed");
    for (auto& ev : b->ev)
        if (hipEventCreate(&ev) != hipSuccess) return cleanup(RAFT_E_DEVICE, "event creation failed");
    *out = b;
    return RAFT_OK;
}

void raft_batch_destroy(raft_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (auto& ev : b->poll_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto& ev : b->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (b->h_poll) (void)hipHostFree(b->h_poll);
    int32_t* ip[] = {b->rp, b->ci, b->deg, b->order};
    for (int32_t* q : ip)
        if (q) (void)hipFree(q);
    float* fp[] = {b->s, b->sh, b->dcoef};
    for (float* q : fp)
        if (q) (void)hipFree(q);
    delete b;
}

raft_status raft_batch_workspace_size(raft_ctx* ctx, const raft_batch* b, size_t* bytes) {
    if (!ctx) return RAFT_E_INVAL;
    if (!b || !bytes) return fail(ctx, RAFT_E_INVAL, "null argument");
    if (b->ctx != ctx) return fail(ctx, RAFT_E_INVAL, "batch belongs to another context");
    BatchLayout B;
    batch_layout(const_cast<raft_batch*>(b), nullptr, nullptr, B, 0);   // the largest shapes
    *bytes = B.bytes;
    return RAFT_OK;
}

raft_status raft_batch_set_capture(raft_batch* b, int32_t enable) {
    if (!b) return RAFT_E_INVAL;
    b->use_graph = enable != 0;
    return RAFT_OK;
}

}  // extern "C"

namespace {

raft_status batch_run_once(raft_ctx* ctx, raft_batch* b, void* ws, size_t ws_bytes,
                           raft_outputs* outs, void* stream, int factor) {
    const int G = b->G;
    const raft_config* c = &b->cfg;
    BatchLayout B;
    batch_layout(b, nullptr, nullptr, B, factor);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, B.bytes));
    batch_layout(b, reinterpret_cast<char*>(ws), outs, B, factor);
    RAFT_TRY(batch_check(ctx, b, B, ws_bytes));
    hipStream_t st = as_stream(stream);
    // control block: static part and the initial dynamic part
    {
        std::vector<int> live(G, 1);
        batch_dynamic(b, B, B.host.data() + B.off_dyn, live);
        HIP_TRY(ctx, hipMemcpyAsync(B.ctl, B.host.data(), B.ctl_upload, hipMemcpyHostToDevice, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));   // pageable source
        // both pinned slots start from this image (the last run ended with a
        // synchronisation, so no copy from them is in flight)
        for (int q = 0; q < 2; ++q)
            memcpy(b->h_poll + q * b->dyn_bytes, B.host.data() + B.off_dyn, b->dyn_bytes);
    }
    HIP_TRY(ctx, hipEventRecord(b->ev[0], st));
    if (b->use_graph) {
        if (!b->exec || b->exec_ws != ws || b->graph_factor != factor) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
            HIP_TRY(ctx, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
            const raft_status ps = batch_prefix(b, B, b->cap_stream);
            hipGraph_t gr = nullptr;
            const hipError_t ce = hipStreamEndCapture(b->cap_stream, &gr);
            if (ps != RAFT_OK) {
                if (gr) (void)hipGraphDestroy(gr);
                return ps;
            }
            if (ce != hipSuccess)
                return fail(ctx, RAFT_E_DEVICE, "graph capture: %s", hipGetErrorString(ce));
            b->graph = gr;
            HIP_TRY(ctx, hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0));
            b->exec_ws = ws;
            b->graph_factor = factor;
        }
        HIP_TRY(ctx, hipGraphLaunch(b->exec, st));
    } else {
        RAFT_TRY(batch_prefix(b, B, st));
    }
    HIP_TRY(ctx, hipEventRecord(b->ev[1], st));
    // Lloyd over every candidate of every graph: one launch per kernel and
    // iteration; convergence polls as in the single-graph loop (the host acts
    // on the flags of the previous poll), with all graphs' flags in one copy
    char* D = B.ctl;
    const KmeansPlan* kmd = at<KmeansPlan>(D, B.off_km);
    const int d = B.d;
    const bool split = B.P[0].km.split != 0;
    const size_t ulds = kmeans_update_lds(B.P[0].ucap, d);
    const int t_max = c->kmeans_max_iter;
    const int check = c->check_every > 0 ? c->check_every : 4;
    const Grid grid = make_grid(c->k_min, c->k_max, c->k_step);
    char* h_dyn[2] = {b->h_poll, b->h_poll + b->dyn_bytes};
    int32_t* h_flags[2] = {reinterpret_cast<int32_t*>(b->h_poll + 2 * b->dyn_bytes),
                           reinterpret_cast<int32_t*>(b->h_poll + 2 * b->dyn_bytes + b->flag_bytes)};
    std::vector<int> live(G, 1);
    int poll = 0;
    for (int it = 1; it <= t_max; ++it) {
        launch_kmeans_batched(kKmAssign, kmd, d, split, B.Zp, it, t_max, ctx->lds_max, ulds,
                              dev_table(D, B.tab_assign, G), B.tab_assign.grid, st);
        if (it == t_max) {
            launch_kmeans_batched(kKmFinalize, kmd, d, split, B.Zp, it, t_max, 0, 0,
                                  dev_table(D, B.tab[bt_one], G), B.tab[bt_one].grid, st);
            break;
        }
        launch_kmeans_batched(kKmUpdate, kmd, d, split, B.Zp, it, t_max, ctx->lds_max, ulds,
                              dev_table(D, B.tab_update, G), B.tab_update.grid, st);
        launch_kmeans_batched(kKmUpdateFinish, kmd, d, split, B.Zp, it, t_max, 0, 0,
                              dev_table(D, B.tab[bt_ufinish], G), B.tab[bt_ufinish].grid, st);
        if (it % check == 0) {
            if (poll > 0) {
                HIP_TRY(ctx, hipEventSynchronize(b->poll_ev[(poll - 1) & 1]));
                const int32_t* ha = h_flags[(poll - 1) & 1];
                int total = 0;
                for (int g = 0; g < G; ++g) {
                    const int32_t* hg = ha + (size_t)g * B.Kc;
                    int lg = 0;
                    for (int k = 0; k < B.Kc; ++k) lg += hg[k] != 0;
                    live[g] = lg;
                    total += lg;
                }
                if (total == 0) break;
                char* hd = h_dyn[poll & 1];
                int32_t* hl = reinterpret_cast<int32_t*>(hd + (B.off_lists - B.off_dyn));
                for (int g = 0; g < G; ++g) {
                    if (!live[g]) continue;
                    const Lists l = make_lists(grid, ha + (size_t)g * B.Kc, B.P[g].ucap,
                                               b->shadow[g].n, B.P[g].share);
                    pack_lists(l, B.Kc, hl + (size_t)g * kDynLen(B.Kc));
                    B.km[g].agroups = (int)l.agrp.size() - 1;
                    B.km[g].ugroups = (int)l.ugrp.size() - 1;
                    B.km[g].uwork = l.uwork;
                }
                // a stopped graph keeps the lists the slot held (no kernel
                // reads them: its assignment and update get no work-groups)
                batch_dynamic(b, B, hd, live);
                HIP_TRY(ctx, hipMemcpyAsync(D + B.off_dyn, hd, b->dyn_bytes, hipMemcpyHostToDevice,
                                            st));
            }
            HIP_TRY(ctx, hipMemcpyAsync(h_flags[poll & 1], D + B.off_flags, b->flag_bytes,
                                        hipMemcpyDeviceToHost, st));
            HIP_TRY(ctx, hipEventRecord(b->poll_ev[poll & 1], st));
            ++poll;
        }
    }
    RAFT_TRY(launch_check(ctx));
    HIP_TRY(ctx, hipEventRecord(b->ev[2], st));
    // scores, selection and outputs of every graph
    const GraphView* gvd = at<GraphView>(D, B.off_gv);
    const ScorePlan* scd = at<ScorePlan>(D, B.off_sc);
    const int sk[] = {bt_transpose, bt_edge, bt_reduce, bt_sfinal, bt_one, bt_first, bt_one,
                      bt_apply, bt_copy};
    const int kinds[] = {kScTranspose, kScEdge, kScReduce, kScFinalize, kScSelect, kScFirst,
                         kScRank, kScApply, kScCopy};
    for (int q = 0; q < 9; ++q)
        launch_score_batched(kinds[q], gvd, scd, B.S, B.SK, dev_table(D, B.tab[sk[q]], G),
                             B.tab[sk[q]].grid, st);
    for (int g = 0; g < G && outs; ++g) {
        const size_t r0 = (size_t)b->base[g];
        const size_t n = (size_t)b->shadow[g].n;
        if (outs[g].Y)
            HIP_TRY(ctx, hipMemcpyAsync(outs[g].Y, B.YO + r0 * B.L, n * B.L * sizeof(float),
                                        hipMemcpyDeviceToDevice, st));
        if (outs[g].Z)
            HIP_TRY(ctx, hipMemcpyAsync(outs[g].Z, B.Zp + r0 * d, n * d * sizeof(float),
                                        hipMemcpyDeviceToDevice, st));
        if (outs[g].centres) launch_copy_centres(B.km[g], outs[g].centres, st);
    }
    RAFT_TRY(launch_check(ctx));
    HIP_TRY(ctx, hipEventRecord(b->ev[3], st));
    HIP_TRY(ctx, hipEventSynchronize(b->ev[3]));
    float ms = 0;
    for (int s2 = 0; s2 < 3; ++s2)
        if (hipEventElapsedTime(&ms, b->ev[s2], b->ev[s2 + 1]) == hipSuccess) b->stage_ms[s2] = ms;
    return RAFT_OK;
}

std::string batch_key(const raft_batch* b) {
    const raft_config* c = &b->cfg;
    char buf[256];
    snprintf(buf, sizeof buf, "batch G=%d N=%d L=%d d=%d q=%d layers=%d K=%d..%d/%d op=%d cu=%d",
             b->G, b->N, c->proj_dim, embed_dim(c), c->q, c->n_layers, c->k_min, c->k_max,
             c->k_step, c->op, b->ctx->num_cu);
    return buf;
}

void tuner_save(raft_ctx* ctx) {
    if (ctx->autotune_cache.empty()) return;
    const std::string tmp = ctx->autotune_cache + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        for (const auto& kv : ctx->tuned) f << kv.first << '\t' << kv.second << '\n';
    }
    (void)std::rename(tmp.c_str(), ctx->autotune_cache.c_str());
}

}  // namespace

void tuner_load(raft_ctx* ctx) {
    if (ctx->autotune_cache.empty()) return;
    std::ifstream f(ctx->autotune_cache);
    std::string line;
    while (std::getline(f, line)) {
        const size_t tab = line.rfind('\t');
        if (tab == std::string::npos) continue;
        ctx->tuned[line.substr(0, tab)] = std::atoi(line.c_str() + tab + 1);
    }
}

extern "C" {

// Share multipliers the tuner times (0: the single-graph shapes).
static const int kTuneFactors[] = {1, 2, 4, 8, 0};

raft_status raft_batch_run(raft_ctx* ctx, raft_batch* b, void* ws, size_t ws_bytes,
                           raft_outputs* outs, void* stream) {
    if (!ctx) return RAFT_E_INVAL;
    if (!b) return fail(ctx, RAFT_E_INVAL, "batch is null");
    if (b->ctx != ctx) return fail(ctx, RAFT_E_INVAL, "batch belongs to another context");
    if (b->factor == 0) {
        // The tuner: the launch shapes it chooses among give identical
        // results, so the choice is made by running the batch once per
        // candidate (after one warm-up run) and keeping the fastest by GPU
        // time; the choice is cached per workload key in the context and,
        // when the context names a cache file, in that file.
        const std::string key = batch_key(b);
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) {
            b->factor = it->second;
        } else {
            RAFT_TRY(batch_run_once(ctx, b, ws, ws_bytes, outs, stream, kTuneFactors[0]));
            double best = 1e300;
            int choice = kTuneFactors[0];
            b->tune_ms.clear();
            for (int f : kTuneFactors) {
                RAFT_TRY(batch_run_once(ctx, b, ws, ws_bytes, outs, stream, f));
                const double t = b->stage_ms[0] + b->stage_ms[1] + b->stage_ms[2];
                b->tune_ms.push_back({f, t});
                if (t < best) {
                    best = t;
                    choice = f;
                }
            }
            ctx->tuned[key] = choice;
            tuner_save(ctx);
            b->factor = choice;
        }
        if (b->factor == 0) b->factor = -1;   // the single-graph shapes
    }
    return batch_run_once(ctx, b, ws, ws_bytes, outs, stream, b->factor < 0 ? 0 : b->factor);
}

raft_status raft_batch_tuning(const raft_batch* b, int32_t* factor, double* ms, int32_t cap,
                              int32_t* count) {
    if (!b || !factor || !count) return RAFT_E_INVAL;
    *factor = b->factor < 0 ? 0 : b->factor;
    *count = (int32_t)b->tune_ms.size();
    for (int i = 0; i < cap && i < *count; ++i) {
        ms[2 * i] = b->tune_ms[i].first;
        ms[2 * i + 1] = b->tune_ms[i].second;
    }
    return RAFT_OK;
}

raft_status raft_batch_plan_check(int32_t G, const int32_t* n, const int64_t* nnz,
                                  const raft_config* cfg, int32_t num_cu, char* msg,
                                  size_t msg_len) {
    if (G < 1 || !n || !nnz || !cfg || num_cu < 1) return RAFT_E_INVAL;
    raft_ctx ctx;
    ctx.num_cu = num_cu;
    raft_status st = check_config(&ctx, nullptr, cfg);
    raft_batch b;
    b.ctx = &ctx;
    b.G = G;
    b.cfg = *cfg;
    b.shadow.resize(G);
    b.seeds.assign(G, cfg->seed);
    b.base.resize(G);
    b.ebase.resize(G);
    int64_t r = 0, e = 0;
    for (int g = 0; g < G && st == RAFT_OK; ++g) {
        if (n[g] < 1 || nnz[g] < 1 || cfg->k_max > n[g]) st = RAFT_E_INVAL;
        b.shadow[g].n = n[g];
        b.shadow[g].nnz = nnz[g];
        b.base[g] = (int32_t)r;
        b.ebase[g] = e;
        r += n[g];
        e += nnz[g];
    }
    if (st == RAFT_OK && (r >= INT32_MAX || e >= INT32_MAX)) st = RAFT_E_UNSUPPORTED;
    if (st == RAFT_OK) {
        b.N = (int32_t)r;
        b.NNZ = e;
        // stand-in addresses: the check only compares ranges
        b.rp = b.ci = b.deg = b.order = reinterpret_cast<int32_t*>((uintptr_t)1 << 44);
        b.s = b.sh = b.dcoef = reinterpret_cast<float*>((uintptr_t)1 << 44);
        BatchLayout B;
        batch_layout(&b, nullptr, nullptr, B, 0);
        const size_t bytes = B.bytes;   // the workspace size the library reports
        for (int f : kTuneFactors) {
            BatchLayout B2;
            char* fake = reinterpret_cast<char*>((uintptr_t)1 << 40);
            batch_layout(&b, fake, nullptr, B2, f);
            std::vector<int> live(G, 1);
            std::vector<char> dyn(B2.ctl_upload - B2.off_dyn);
            batch_dynamic(&b, B2, dyn.data(), live);
            st = batch_check(&ctx, &b, B2, bytes);
            if (st != RAFT_OK) break;
        }
    }
    if (msg && msg_len) {
        const size_t m = std::min(msg_len - 1, ctx.err.size());
        memcpy(msg, ctx.err.data(), m);
        msg[m] = 0;
    }
    b.rp = b.ci = b.deg = b.order = nullptr;
    b.s = b.sh = b.dcoef = nullptr;
    return st;
}

raft_status raft_batch_stage_times(const raft_batch* b, double* ms3) {
    if (!b || !ms3) return RAFT_E_INVAL;
    for (int s2 = 0; s2 < 3; ++s2) ms3[s2] = b->stage_ms[s2];
    return RAFT_OK;
}

}  // extern "C"

// ---- hierarchical model selection (Alg. 1) --------------------------------

namespace {

struct HierLayout {
    int n = 0, d = 0, max_sets = 0, max_slots = 0;
    int32_t *perm, *perm_next, *setid, *setid_next, *leaf, *pick, *ridx, *rlow, *n32, *active,
        *changed, *iters, *live, *cursor, *block_of, *meta;
    int8_t* side;
    double* rval;
    float *C, *cnorm;
    long long *S64, *counts;
    uint32_t* zmax;
    size_t bytes = 0;
};

// Points per work-group of the level kernels.
constexpr int kHierPts = 256;

void hier_layout(int n, int d, char* base, HierLayout& H) {
    H.n = n;
    H.d = d;
    // the sets of a level are disjoint and non-empty: at most n of them; a
    // set has at most ceil(cnt / kHierPts) race work-groups, at most
    // sets + n / kHierPts in total
    H.max_sets = n + 2;
    H.max_slots = H.max_sets + n / kHierPts + 1;
    Arena a;
    a.base = base;
    H.perm = a.take<int32_t>(n);
    H.perm_next = a.take<int32_t>(n);
    H.setid = a.take<int32_t>(n);
    H.setid_next = a.take<int32_t>(n);
    H.leaf = a.take<int32_t>(n);
    H.side = a.take<int8_t>(n);
    H.pick = a.take<int32_t>((size_t)2 * H.max_sets);
    H.rval = a.take<double>(H.max_slots);
    H.ridx = a.take<int32_t>(H.max_slots);
    H.rlow = a.take<int32_t>(H.max_slots);
    H.C = a.take<float>((size_t)2 * H.max_sets * d);
    H.cnorm = a.take<float>((size_t)2 * H.max_sets);
    H.S64 = a.take<long long>((size_t)2 * H.max_sets * d);
    H.n32 = a.take<int32_t>((size_t)2 * H.max_sets);
    H.active = a.take<int32_t>(H.max_sets);
    H.changed = a.take<int32_t>(H.max_sets);
    H.iters = a.take<int32_t>(H.max_sets);
    H.live = a.take<int32_t>(1);
    H.counts = a.take<long long>((size_t)7 * H.max_sets);
    H.cursor = a.take<int32_t>(H.max_sets);
    H.zmax = a.take<uint32_t>(1);
    // per level: beg, cnt, need, tnode [max_sets each], child [2 max_sets],
    // two tables [2 (2 max_sets + 1)]
    H.meta = a.take<int32_t>((size_t)6 * H.max_sets + 2 * (2 * (size_t)H.max_sets + 1));
    // block number of every tree node (at most 2 n tree nodes)
    H.block_of = a.take<int32_t>((size_t)2 * n + 1);
    H.bytes = a.off;
}

HostTable make_table_unpadded(const std::vector<int>& counts) {
    HostTable t;
    const int G = (int)counts.size();
    t.start.assign(G + 1, 0);
    t.count = counts;
    for (int g = 0; g < G; ++g) t.start[g + 1] = t.start[g] + counts[g];
    t.grid = t.start[G];
    return t;
}

// Eq. 7 in FP64 from integer counts, blocks in order (m: intra edges, v:
// G-volumes), left to right as written.
double lmod_fp64(const int64_t* m, const int64_t* v, int k) {
    int64_t two_e = 0;
    for (int r = 0; r < k; ++r) two_e += v[r];
    const double e = (double)two_e / 2.0;
    double total = 0.0;
    for (int r = 0; r < k; ++r) {
        const double t = (double)v[r] / (double)two_e;
        total = total + ((double)m[r] / e - t * t);
    }
    return total;
}

}  // namespace

extern "C" {

raft_status raft_hier_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t d,
                                     size_t* bytes) {
    RAFT_TRY(check_graph(ctx, g));
    if (!bytes) return fail(ctx, RAFT_E_INVAL, "bytes is null");
    if (!kmeans_supported(d)) return fail(ctx, RAFT_E_UNSUPPORTED, "width %d", d);
    HierLayout H;
    hier_layout(g->n, d, nullptr, H);
    *bytes = H.bytes;
    return RAFT_OK;
}

raft_status raft_hier_partition(raft_ctx* ctx, const raft_graph* g, const float* Z, int32_t d,
                                const raft_hier_config* cfg, void* ws, size_t ws_bytes,
                                int32_t* labels, int32_t* n_blocks, raft_hier_node* tree,
                                int32_t tree_cap, int32_t* n_tree, int32_t* node_trace,
                                int32_t trace_depth, void* stream) {
    RAFT_TRY(check_graph(ctx, g));
    if (!Z || !cfg || !labels || !n_blocks) return fail(ctx, RAFT_E_INVAL, "null argument");
    if (!kmeans_supported(d)) return fail(ctx, RAFT_E_UNSUPPORTED, "width %d", d);
    if (cfg->eps < 0 || cfg->t_max < 1) return fail(ctx, RAFT_E_INVAL, "eps %d t_max %d", cfg->eps, cfg->t_max);
    if (node_trace && trace_depth < 0) return fail(ctx, RAFT_E_INVAL, "trace_depth");
    const int n = g->n;
    HierLayout H;
    hier_layout(n, d, nullptr, H);
    RAFT_TRY(check_ws(ctx, ws, ws_bytes, H.bytes));
    hier_layout(n, d, reinterpret_cast<char*>(ws), H);
    hipStream_t st = as_stream(stream);
    const GraphView gv = g->view();
    int64_t* hbuf = reinterpret_cast<int64_t*>(ctx->h_pinned);   // pinned scratch (16 KiB)
    // setup: identity permutation, one set, scale of the fixed-point sums
    launch_hier_setup(Z, (int64_t)n * d, H.zmax, H.perm, H.setid, H.setid_next, H.side, H.leaf,
                      n, st);
    if (node_trace && trace_depth > 0) launch_fill_i32(node_trace, (int64_t)trace_depth * n, -1, st);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_pinned, H.zmax, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    int fexp = 0;
    {
        float zmax;
        memcpy(&zmax, ctx->h_pinned, sizeof zmax);
        if (zmax > 0.f) {
            int ez;
            std::frexp(zmax, &ez);
            fexp = 30 - ez;
        }
    }
    struct SetInfo {
        int beg, cnt, tnode;
    };
    std::vector<raft_hier_node> nodes;
    nodes.push_back(raft_hier_node{0, n, -1, {-1, -1}, -1, 0, {0, 0}, NAN, NAN});
    std::vector<SetInfo> sets = {{0, n, 0}};
    const int eps = cfg->eps;
    int depth = 0;
    std::vector<int32_t> meta;
    std::vector<int64_t> cnt_host;
    while (!sets.empty()) {
        const int ns = (int)sets.size();
        if (ns > H.max_sets) return fail(ctx, RAFT_E_INVAL, "hierarchy level of %d sets", ns);
        // per-set arrays and the two launch tables of the level
        std::vector<int> ck(ns), ca(ns);
        meta.assign((size_t)6 * H.max_sets + 2 * (2 * (size_t)H.max_sets + 1), 0);
        int32_t* m_beg = meta.data();
        int32_t* m_cnt = m_beg + H.max_sets;
        int32_t* m_need = m_cnt + H.max_sets;
        int32_t* m_tnode = m_need + H.max_sets;
        int32_t* m_child = m_tnode + H.max_sets;   // 2 max_sets
        int32_t* m_tk = m_child + 2 * H.max_sets;  // table of the KMeans kernels
        int32_t* m_ta = m_tk + 2 * H.max_sets + 1; // table of the per-node kernels
        bool any_need = false;
        for (int s2 = 0; s2 < ns; ++s2) {
            m_beg[s2] = sets[s2].beg;
            m_cnt[s2] = sets[s2].cnt;
            m_tnode[s2] = sets[s2].tnode;
            const bool need = sets[s2].cnt > 2 * eps + 1;
            m_need[s2] = need;
            any_need |= need;
            ca[s2] = (sets[s2].cnt + kHierPts - 1) / kHierPts;
            ck[s2] = need ? ca[s2] : 0;
            m_child[2 * s2] = m_child[2 * s2 + 1] = -1;
        }
        const HostTable tk = make_table_unpadded(ck), ta = make_table_unpadded(ca);
        if (tk.grid > H.max_slots) return fail(ctx, RAFT_E_INVAL, "race slots");
        std::copy(tk.start.begin(), tk.start.end(), m_tk);
        std::copy(tk.count.begin(), tk.count.end(), m_tk + ns + 1);
        std::copy(ta.start.begin(), ta.start.end(), m_ta);
        std::copy(ta.count.begin(), ta.count.end(), m_ta + ns + 1);
        HIP_TRY(ctx, hipMemcpyAsync(H.meta, meta.data(), meta.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, st));
        HierPlan h;
        h.Z = Z;
        h.d = d;
        h.seed = cfg->seed;
        h.depth = depth;
        h.fexp = fexp;
        h.beg = H.meta;
        h.cnt = H.meta + H.max_sets;
        h.need = H.meta + 2 * H.max_sets;
        h.tnode = H.meta + 3 * H.max_sets;
        h.child = H.meta + 4 * H.max_sets;
        h.perm = (depth & 1) ? H.perm_next : H.perm;
        h.perm_next = (depth & 1) ? H.perm : H.perm_next;
        h.setid = (depth & 1) ? H.setid_next : H.setid;
        h.setid_next = (depth & 1) ? H.setid : H.setid_next;
        h.side = H.side;
        h.leaf = H.leaf;
        h.pick = H.pick;
        h.rval = H.rval;
        h.ridx = H.ridx;
        h.rlow = H.rlow;
        h.C = H.C;
        h.cnorm = H.cnorm;
        h.S64 = H.S64;
        h.n32 = H.n32;
        h.active = H.active;
        h.changed = H.changed;
        h.iters = H.iters;
        h.live = H.live;
        h.counts = H.counts;
        h.cursor = H.cursor;
        BatchTable btk{H.meta + 6 * H.max_sets, H.meta + 6 * H.max_sets + ns + 1, ns};
        BatchTable bta{H.meta + 6 * H.max_sets + 2 * H.max_sets + 1,
                       H.meta + 6 * H.max_sets + 2 * H.max_sets + 1 + ns + 1, ns};
        launch_fill_i64(H.counts, (int64_t)7 * ns, st);
        launch_fill_i32(H.iters, ns, 0, st);
        if (any_need) {
            for (int t = 0; t < 2; ++t) {
                launch_hier(kHierRace, h, gv, d, t, 0, ns, btk, tk.grid, st);
                launch_hier(kHierPick, h, gv, d, t, 0, ns, btk, 0, st);
            }
            launch_hier(kHierInit, h, gv, d, 0, 0, ns, btk, 0, st);
            for (int it = 1; it <= cfg->t_max; ++it) {
                launch_fill_i32(H.live, 1, 0, st);
                launch_hier(kHierAssign, h, gv, d, it, cfg->t_max, ns, btk, tk.grid, st);
                launch_hier(kHierUpdate, h, gv, d, it, cfg->t_max, ns, btk, 0, st);
                HIP_TRY(ctx, hipMemcpyAsync(ctx->h_pinned, H.live, sizeof(int32_t),
                                            hipMemcpyDeviceToHost, st));
                HIP_TRY(ctx, hipStreamSynchronize(st));
                if (ctx->h_pinned[0] == 0) break;
            }
        }
        launch_hier(kHierCounts, h, gv, d, 0, 0, ns, bta, ta.grid, st);
        RAFT_TRY(launch_check(ctx));
        cnt_host.resize((size_t)8 * ns);
        HIP_TRY(ctx, hipMemcpyAsync(cnt_host.data(), H.counts, sizeof(int64_t) * 7 * ns,
                                    hipMemcpyDeviceToHost, st));
        std::vector<int32_t> its(ns);
        HIP_TRY(ctx, hipMemcpyAsync(its.data(), H.iters, sizeof(int32_t) * ns,
                                    hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        // decisions (Alg. 1), children and the next level's sets
        std::vector<SetInfo> next;
        std::vector<int32_t> cursor;
        for (int s2 = 0; s2 < ns; ++s2) {
            const int64_t* c = cnt_host.data() + (size_t)7 * s2;
            raft_hier_node& nd = nodes[sets[s2].tnode];
            const int64_t vol[2] = {c[5], c[6]};
            const int64_t volU = vol[0] + vol[1];
            const int64_t mU = c[0] / 2;
            bool split = false;
            if (volU > 0) {
                const int64_t mv[1] = {mU}, vv[1] = {volU};
                nd.m1 = lmod_fp64(mv, vv, 1);
            }
            if (m_need[s2] && volU > 0) {
                const int64_t ms[2] = {c[1] / 2, c[2] / 2};
                nd.m2 = lmod_fp64(ms, vol, 2);
                nd.sizes[0] = (int32_t)c[3];
                nd.sizes[1] = (int32_t)c[4];
                nd.kmeans_iters = its[s2];
                split = !(c[3] <= eps || c[4] <= eps || nd.m1 > nd.m2);
            } else if (m_need[s2]) {
                nd.sizes[0] = (int32_t)c[3];
                nd.sizes[1] = (int32_t)c[4];
                nd.kmeans_iters = its[s2];
            }
            if (!split) continue;
            for (int a2 = 0; a2 < 2; ++a2) {
                const int tn = (int)nodes.size();
                const int beg = sets[s2].beg + (a2 ? (int)c[3] : 0);
                const int cnt2 = (int)c[3 + a2];
                nodes.push_back(raft_hier_node{depth + 1, cnt2, sets[s2].tnode, {-1, -1}, -1, 0,
                                               {0, 0}, NAN, NAN});
                nodes[sets[s2].tnode].child[a2] = tn;
                m_child[2 * s2 + a2] = (int)next.size();
                next.push_back({beg, cnt2, tn});
                cursor.push_back(beg);
            }
        }
        if (next.size() > (size_t)H.max_sets) return fail(ctx, RAFT_E_INVAL, "next level sets");
        HIP_TRY(ctx, hipMemcpyAsync(H.meta + 4 * H.max_sets, m_child, sizeof(int32_t) * 2 * ns,
                                    hipMemcpyHostToDevice, st));
        if (!cursor.empty())
            HIP_TRY(ctx, hipMemcpyAsync(H.cursor, cursor.data(), sizeof(int32_t) * cursor.size(),
                                        hipMemcpyHostToDevice, st));
        if (node_trace && depth < trace_depth)
            launch_hier_trace(h, node_trace + (size_t)depth * n, bta, ta.grid, st);
        launch_hier(kHierScatter, h, gv, d, 0, 0, ns, bta, ta.grid, st);
        RAFT_TRY(launch_check(ctx));
        HIP_TRY(ctx, hipStreamSynchronize(st));   // meta / cursor sources are host vectors
        sets.swap(next);
        ++depth;
    }
    // blocks in the order Alg. 1 adds them: depth first, U_1 before U_2
    std::vector<int32_t> block_of(nodes.size(), -1);
    int nb = 0;
    std::vector<int> stack = {0};
    while (!stack.empty()) {
        const int t = stack.back();
        stack.pop_back();
        if (nodes[t].child[0] < 0) {
            nodes[t].block = nb;
            block_of[t] = nb++;
            continue;
        }
        stack.push_back(nodes[t].child[1]);
        stack.push_back(nodes[t].child[0]);
    }
    if (nodes.size() > (size_t)2 * n + 1) return fail(ctx, RAFT_E_INVAL, "tree size");
    HIP_TRY(ctx, hipMemcpyAsync(H.block_of, block_of.data(), sizeof(int32_t) * block_of.size(),
                                hipMemcpyHostToDevice, st));
    launch_hier_labels(H.leaf, H.block_of, n, labels, st);
    RAFT_TRY(launch_check(ctx));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    (void)hbuf;
    *n_blocks = nb;
    if (n_tree) *n_tree = (int32_t)nodes.size();
    if (tree)
        for (size_t t = 0; t < nodes.size() && (int)t < tree_cap; ++t) tree[t] = nodes[t];
    return RAFT_OK;
}

// ---------------------------------------------------------------------------
// Alg. 2: sampling from the degree-corrected SBM.  The host groups the nodes
// by block (increasing id), accumulates each block's theta prefix left to
// right in FP64 and lists the block pairs r <= s with both blocks non-empty;
// every row of every pair is one device thread.  A counting pass, a scan and
// a writing pass give the edge list, which becomes a symmetric sorted CSR and
// then a graph handle (validated like any other).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
struct DeviceAllocs {
    std::vector<void*> p;
    ~DeviceAllocs() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    bool get(T** out, size_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
        p.push_back(q);
        *out = static_cast<T*>(q);
        return true;
    }
};
}  // namespace

extern "C" {

raft_status raft_sbm_sample(raft_ctx* ctx, int64_t n, int32_t k, const double* theta,
                            const int32_t* blocks, const double* omega, uint64_t seed,
                            void* stream, raft_graph** out) {
    if (!ctx) return RAFT_E_INVAL;
    if (!out) return fail(ctx, RAFT_E_INVAL, "out is null");
    *out = nullptr;
    if (!theta || !blocks || !omega) return fail(ctx, RAFT_E_INVAL, "null argument");
    if (n < 1 || n >= INT32_MAX) return fail(ctx, RAFT_E_INVAL, "n = %lld", (long long)n);
    if (k < 1 || k > kSbmMaxBlocks)
        return fail(ctx, RAFT_E_INVAL, "k = %d outside 1..%d", k, kSbmMaxBlocks);
    for (int64_t i = 0; i < n; ++i) {
        if (blocks[i] < 0 || blocks[i] >= k)
            return fail(ctx, RAFT_E_INVAL, "blocks[%lld] = %d outside 0..%d", (long long)i,
                        blocks[i], k - 1);
        if (!std::isfinite(theta[i]) || theta[i] < 0)
            return fail(ctx, RAFT_E_INVAL, "theta[%lld] not finite and >= 0", (long long)i);
    }
    for (int64_t q = 0; q < (int64_t)k * k; ++q)
        if (!std::isfinite(omega[q]) || omega[q] < 0)
            return fail(ctx, RAFT_E_INVAL, "omega entry %lld not finite and >= 0", (long long)q);
    for (int r = 0; r < k; ++r)
        for (int s = r + 1; s < k; ++s)
            if (omega[(size_t)r * k + s] != omega[(size_t)s * k + r])
                return fail(ctx, RAFT_E_INVAL, "omega not symmetric at (%d, %d)", r, s);
    // blocks, members in increasing id (a stable counting sort), prefixes
    std::vector<int32_t> bcount(k, 0), boff(k, 0), members((size_t)n);
    for (int64_t i = 0; i < n; ++i) ++bcount[blocks[i]];
    for (int r = 1; r < k; ++r) boff[r] = boff[r - 1] + bcount[r - 1];
    {
        std::vector<int32_t> cur(boff);
        for (int64_t i = 0; i < n; ++i) members[cur[blocks[i]]++] = (int32_t)i;
    }
    std::vector<double> pref((size_t)n + k);
    for (int s = 0; s < k; ++s) {
        double* ps = pref.data() + boff[s] + s;
        double acc = 0.0;
        ps[0] = 0.0;
        for (int y = 0; y < bcount[s]; ++y) {
            acc = acc + theta[members[(size_t)boff[s] + y]];
            ps[y + 1] = acc;
        }
    }
    std::vector<int32_t> pair_r, pair_s;
    std::vector<int64_t> rowoff = {0};
    for (int r = 0; r < k; ++r)
        for (int s = r; s < k; ++s)
            if (bcount[r] > 0 && bcount[s] > 0) {
                pair_r.push_back(r);
                pair_s.push_back(s);
                rowoff.push_back(rowoff.back() + bcount[r]);
            }
    const int npairs = (int)pair_r.size();
    const int64_t nrows = rowoff.back();
    hipStream_t st = as_stream(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    DeviceAllocs A;
    SbmPlan P{};
    double *d_theta, *d_omega, *d_pref;
    int32_t *d_members, *d_boff, *d_bcount, *d_pr, *d_ps;
    int64_t *d_rowoff, *cnt, *off, *bsum, *total;
    const int64_t nb_rows = (nrows + 1023) / 1024 + 1, nb_n = ((int64_t)n + 1 + 1023) / 1024 + 1;
    if (!A.get(&d_theta, n) || !A.get(&d_omega, (size_t)k * k) || !A.get(&d_pref, n + k) ||
        !A.get(&d_members, n) || !A.get(&d_boff, k) || !A.get(&d_bcount, k) ||
        !A.get(&d_pr, npairs) || !A.get(&d_ps, npairs) || !A.get(&d_rowoff, npairs + 1) ||
        !A.get(&cnt, nrows) || !A.get(&off, nrows) ||
        !A.get(&bsum, std::max(nb_rows, nb_n)) || !A.get(&total, 1))
        return fail(ctx, RAFT_E_NOMEM, "sampler allocation failed (%lld rows)", (long long)nrows);
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t e = up(d_theta, theta, sizeof(double) * n);
    if (e == hipSuccess) e = up(d_omega, omega, sizeof(double) * k * k);
    if (e == hipSuccess) e = up(d_pref, pref.data(), sizeof(double) * pref.size());
    if (e == hipSuccess) e = up(d_members, members.data(), sizeof(int32_t) * n);
    if (e == hipSuccess) e = up(d_boff, boff.data(), sizeof(int32_t) * k);
    if (e == hipSuccess) e = up(d_bcount, bcount.data(), sizeof(int32_t) * k);
    if (e == hipSuccess) e = up(d_pr, pair_r.data(), sizeof(int32_t) * npairs);
    if (e == hipSuccess) e = up(d_ps, pair_s.data(), sizeof(int32_t) * npairs);
    if (e == hipSuccess) e = up(d_rowoff, rowoff.data(), sizeof(int64_t) * rowoff.size());
    if (e != hipSuccess) return fail(ctx, RAFT_E_DEVICE, "sampler upload: %s", hipGetErrorString(e));
    P.k = k;
    P.npairs = npairs;
    P.nrows = nrows;
    P.seed = seed;
    P.theta = d_theta;
    P.omega = d_omega;
    P.members = d_members;
    P.boff = d_boff;
    P.bcount = d_bcount;
    P.pref = d_pref;
    P.rowoff = d_rowoff;
    P.pair_r = d_pr;
    P.pair_s = d_ps;
    // pass 1: edges per row; offsets by the scan; the total read back
    launch_sbm_rows(P, false, cnt, nullptr, nullptr, nullptr, st);
    launch_scan_i64(cnt, nrows, off, bsum, total, st);
    RAFT_TRY(launch_check(ctx));
    int64_t ne = 0;
    int64_t* h_total = reinterpret_cast<int64_t*>(ctx->h_pinned);
    HIP_TRY(ctx, hipMemcpyAsync(h_total, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    ne = h_total[0];
    if (ne < 0) return fail(ctx, RAFT_E_DEVICE, "edge count %lld", (long long)ne);
    if (2 * ne >= INT32_MAX)
        return fail(ctx, RAFT_E_UNSUPPORTED, "%lld sampled edges exceed the int32 CSR",
                    (long long)ne);
    // pass 2: the same draws, edges stored; then the CSR
    int32_t *src, *dst, *col;
    int64_t *deg, *rp, *cursor;
    if (!A.get(&src, ne) || !A.get(&dst, ne) || !A.get(&col, 2 * ne) || !A.get(&deg, n + 1) ||
        !A.get(&rp, n + 1) || !A.get(&cursor, n))
        return fail(ctx, RAFT_E_NOMEM, "sampler edge buffers (%lld edges)", (long long)ne);
    launch_sbm_rows(P, true, nullptr, off, src, dst, st);
    HIP_TRY(ctx, launch_sbm_csr(src, dst, ne, (int)n, deg, rp, cursor, bsum, total, col, st));
    RAFT_TRY(launch_check(ctx));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return raft_graph_create(ctx, rp, 1, col, n, 2 * ne, 1, stream, out);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Streaming update (Sec. III-D).  The stream keeps every level of the
// embedding: Theta, Y_1..Y_q, the input of layer 1 (Y_q or its row-normalised
// copy) and the layer outputs H_1..H_n.  New edges are merged into a new CSR
// (the degree arrays recomputed by the same kernel as at graph creation, the
// row schedule kept from the previous graph: it only orders work), and under
// the NCut operator level t is recomputed on the rows within t hops of the
// new edges' endpoints (layer k on q + k hops) by the same row kernels as a
// full pass, so every row equals a full recomputation on the new graph bit
// for bit.  The modularity operators carry 1/2e in every entry, so there
// every level is recomputed in full.
// ---------------------------------------------------------------------------
struct raft_stream {
    raft_ctx* ctx = nullptr;
    raft_graph gr[2];                      // current and next graph (stream-owned arrays)
    int cur = 0;
    int64_t ci_cap[2] = {0, 0};
    raft_config cfg{};
    int n = 0, L = 0, R = 0, lmax = 0;
    std::vector<int> lin, lout;            // per layer
    std::vector<float*> y;                 // q + 1 levels, y[0] = Theta
    float* h0 = nullptr;                   // normalised input (normalize_input only)
    std::vector<float*> h, w;              // layer outputs and weights
    float *pbuf = nullptr, *gin = nullptr, *gout = nullptr;
    double *cpart = nullptr, *c64 = nullptr;
    float* cvec = nullptr;
    int32_t *dist = nullptr, *lists = nullptr, *mstatus = nullptr;
    int64_t *flag = nullptr, *pos = nullptr, *bsum = nullptr, *totals = nullptr;
    int64_t *add_cnt = nullptr, *add_off = nullptr;
    int32_t* edges = nullptr;              // staging: rows, cols, V' (3 x edge_cap)
    int64_t edge_cap = 0;
    std::vector<void*> mem;
    raft_graph* g() { return &gr[cur]; }
    const float* input() const { return h0 ? h0 : y[cfg.q]; }
    const float* z() const { return cfg.n_layers ? h[cfg.n_layers - 1] : input(); }
};

namespace {

template <typename T>
bool stream_alloc(raft_stream* s, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    s->mem.push_back(q);
    *p = static_cast<T*>(q);
    return true;
}

// Replaces *p (a stream allocation, or null) by a larger one; the old
// contents are not kept.
template <typename T>
bool stream_realloc(raft_stream* s, T** p, size_t count) {
    if (*p) {
        auto it = std::find(s->mem.begin(), s->mem.end(), (void*)*p);
        if (it != s->mem.end()) s->mem.erase(it);
        (void)hipFree(*p);
        *p = nullptr;
    }
    return stream_alloc(s, p, count);
}

// Level t is run over all rows once its ball holds more than half of them:
// rows outside the ball recompute to their previous values, and a full
// launch needs no row gather and scatter.
bool stream_level_full(const raft_stream* s, const int64_t* counts, int t) {
    return 2 * counts[t - 1] > (int64_t)s->n;
}

// Every level from scratch, in the order and with the kernels of
// raft_project and raft_embed.
raft_status stream_full(raft_stream* s, hipStream_t st) {
    raft_ctx* ctx = s->ctx;
    const GraphView gv = s->g()->view();
    const raft_config& c = s->cfg;
    const int n = s->n, L = s->L;
    const bool mod_full = c.op == RAFT_X_MOD_FULL;
    const int grid = spmm_grid(n, L, ctx->num_cu, nullptr);
    if (mod_full) {
        launch_colsum_partials(gv, L, s->y[0], s->cpart, ctx->num_cu, st);
        launch_colsum_finish(s->cpart, grid, L, s->c64, s->cvec, st);
    }
    for (int t = 1; t <= c.q; ++t) {
        const bool need_cs = mod_full && t < c.q;
        launch_spmm(gv, c.op, L, s->y[t - 1], s->y[t], s->cvec, need_cs ? s->cpart : nullptr,
                    ctx->num_cu, st);
        if (need_cs) launch_colsum_finish(s->cpart, grid, L, s->c64, s->cvec, st);
    }
    if (s->h0) {
        HIP_TRY(ctx, hipMemcpyAsync(s->h0, s->y[c.q], (size_t)n * L * sizeof(float),
                                    hipMemcpyDeviceToDevice, st));
        launch_rownorm(s->h0, n, L, st);
    }
    const float* hin = s->input();
    for (int k = 0; k < c.n_layers; ++k) {
        launch_spmm(gv, kOpGcn, s->lin[k], hin, s->pbuf, nullptr, nullptr, ctx->num_cu, st);
        launch_dense_layer(s->pbuf, s->w[k], s->h[k], n, s->lin[k], s->lout[k], false,
                           ctx->d_status, ctx->num_cu, st);
        hin = s->h[k];
    }
    return launch_check(ctx);
}

// Level t on lists[t - 1] (counts[t - 1] rows), or on all rows once the
// ball is most of the graph; NCut operator.
raft_status stream_incremental(raft_stream* s, const int64_t* counts, hipStream_t st) {
    raft_ctx* ctx = s->ctx;
    const raft_config& c = s->cfg;
    const int n = s->n, L = s->L;
    const GraphView all = s->g()->view();
    auto sub = [&](int t) {
        if (stream_level_full(s, counts, t)) return all;
        GraphView v = all;
        v.order = s->lists + (size_t)(t - 1) * n;
        v.n = (int32_t)counts[t - 1];
        return v;
    };
    for (int t = 1; t <= c.q; ++t)
        launch_spmm(sub(t), kOpNcut, L, s->y[t - 1], s->y[t], nullptr, nullptr, ctx->num_cu, st);
    if (s->h0) {
        if (stream_level_full(s, counts, c.q)) {
            HIP_TRY(ctx, hipMemcpyAsync(s->h0, s->y[c.q], (size_t)n * L * sizeof(float),
                                        hipMemcpyDeviceToDevice, st));
            launch_rownorm(s->h0, n, L, st);
        } else {
            const int32_t* lq = s->lists + (size_t)(c.q - 1) * n;
            const int32_t cq = (int32_t)counts[c.q - 1];
            launch_stream_rows(true, lq, cq, L, s->y[c.q], s->gin, st);
            launch_rownorm(s->gin, cq, L, st);
            launch_stream_rows(false, lq, cq, L, s->gin, s->h0, st);
        }
    }
    const float* hin = s->input();
    for (int k = 0; k < c.n_layers; ++k) {
        const int t = c.q + k + 1;
        launch_spmm(sub(t), kOpGcn, s->lin[k], hin, s->pbuf, nullptr, nullptr, ctx->num_cu, st);
        if (stream_level_full(s, counts, t)) {
            launch_dense_layer(s->pbuf, s->w[k], s->h[k], n, s->lin[k], s->lout[k], false,
                               ctx->d_status, ctx->num_cu, st);
        } else {
            const int32_t* lt = s->lists + (size_t)(t - 1) * n;
            const int32_t ct = (int32_t)counts[t - 1];
            launch_stream_rows(true, lt, ct, s->lin[k], s->pbuf, s->gin, st);
            launch_dense_layer(s->gin, s->w[k], s->gout, ct, s->lin[k], s->lout[k], false,
                               ctx->d_status, ctx->num_cu, st);
            launch_stream_rows(false, lt, ct, s->lout[k], s->gout, s->h[k], st);
        }
        hin = s->h[k];
    }
    return launch_check(ctx);
}

}  // namespace

extern "C" {

void raft_stream_destroy(raft_stream* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (void* q : s->mem) (void)hipFree(q);
    delete s;
}

raft_status raft_stream_create(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                               void* stream, raft_stream** out) {
    RAFT_TRY(check_graph(ctx, g));
    if (!out) return fail(ctx, RAFT_E_INVAL, "out is null");
    *out = nullptr;
    RAFT_TRY(check_config(ctx, g, cfg));
    if (cfg->q + cfg->n_layers > kStreamMaxLevels)
        return fail(ctx, RAFT_E_UNSUPPORTED, "q + n_layers = %d exceeds %d",
                    cfg->q + cfg->n_layers, kStreamMaxLevels);
    hipStream_t st = as_stream(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    raft_stream* s = new raft_stream();
    s->ctx = ctx;
    s->cfg = *cfg;
    s->n = g->n;
    s->L = cfg->proj_dim;
    s->R = cfg->q + cfg->n_layers;
    s->lmax = s->L;
    int l = s->L;
    for (int k = 0; k < cfg->n_layers; ++k) {
        s->lin.push_back(l);
        s->lout.push_back(cfg->layer_dims[k]);
        l = cfg->layer_dims[k];
        s->lmax = std::max(s->lmax, l);
    }
    auto cleanup = [&](raft_status code, const char* what) {
        raft_stream_destroy(s);
        return fail(ctx, code, "stream: %s", what);
    };
    const size_t n = (size_t)s->n;
    bool ok = true;
    // two graphs: the current one (a copy of g) and the next one
    for (int b = 0; b < 2; ++b) {
        raft_graph& G = s->gr[b];
        G.ctx = ctx;
        G.n = g->n;
        G.nnz = g->nnz;
        std::copy(g->heavy, g->heavy + 17, G.heavy);
        G.owns = false;
        s->ci_cap[b] = std::max<int64_t>(g->nnz + g->nnz / 4, 1024);
        ok = ok && stream_alloc(s, &G.rp, n + 1) && stream_alloc(s, &G.ci, s->ci_cap[b]) &&
             stream_alloc(s, &G.deg, n) && stream_alloc(s, &G.s, n) && stream_alloc(s, &G.sh, n) &&
             stream_alloc(s, &G.dcoef, n) && stream_alloc(s, &G.order, n);
    }
    s->y.assign(cfg->q + 1, nullptr);
    s->h.assign(cfg->n_layers, nullptr);
    s->w.assign(cfg->n_layers, nullptr);
    for (auto& p : s->y) ok = ok && stream_alloc(s, &p, n * s->L);
    if (cfg->normalize_input) ok = ok && stream_alloc(s, &s->h0, n * s->L);
    for (int k = 0; k < cfg->n_layers; ++k)
        ok = ok && stream_alloc(s, &s->h[k], n * s->lout[k]) &&
             stream_alloc(s, &s->w[k], (size_t)s->lin[k] * s->lout[k]);
    const int grid = spmm_grid(s->n, s->L, ctx->num_cu, nullptr);
    ok = ok && stream_alloc(s, &s->pbuf, n * s->lmax) && stream_alloc(s, &s->gin, n * s->lmax) &&
         stream_alloc(s, &s->gout, n * s->lmax) &&
         stream_alloc(s, &s->cpart, ((size_t)grid + kColsumStageRows) * s->L) &&
         stream_alloc(s, &s->c64, (size_t)s->L) && stream_alloc(s, &s->cvec, (size_t)s->L) &&
         stream_alloc(s, &s->dist, n) && stream_alloc(s, &s->lists, n * s->R) &&
         stream_alloc(s, &s->flag, n) && stream_alloc(s, &s->pos, n) &&
         stream_alloc(s, &s->bsum, (n + 1 + 1023) / 1024 + 1) &&
         stream_alloc(s, &s->totals, (size_t)kStreamMaxLevels + 1) &&
         stream_alloc(s, &s->add_cnt, n + 1) && stream_alloc(s, &s->add_off, n + 1) &&
         stream_alloc(s, &s->mstatus, 1);
    if (!ok) return cleanup(RAFT_E_NOMEM, "device allocation failed");
    raft_graph& G = s->gr[0];
    const hipMemcpyKind dd = hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(G.rp, g->rp, sizeof(int32_t) * (n + 1), dd, st);
    if (e == hipSuccess && g->nnz > 0)
        e = hipMemcpyAsync(G.ci, g->ci, sizeof(int32_t) * g->nnz, dd, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G.deg, g->deg, sizeof(int32_t) * n, dd, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G.s, g->s, sizeof(float) * n, dd, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G.sh, g->sh, sizeof(float) * n, dd, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G.dcoef, g->dcoef, sizeof(float) * n, dd, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G.order, g->order, sizeof(int32_t) * n, dd, st);
    if (e != hipSuccess) return cleanup(RAFT_E_DEVICE, "graph copy");
    launch_gaussian(cfg->seed, 0x10, s->n, s->L, 1.0 / std::sqrt((double)s->L), s->y[0], st);
    for (int k = 0; k < cfg->n_layers; ++k)
        launch_gaussian(cfg->seed, 0x10 + (uint64_t)(k + 1), s->lin[k], s->lout[k],
                        1.0 / std::sqrt((double)s->lin[k]), s->w[k], st);
    const raft_status r = stream_full(s, st);
    if (r == RAFT_OK && hipStreamSynchronize(st) != hipSuccess)
        return cleanup(RAFT_E_DEVICE, "initial levels");
    if (r != RAFT_OK) {
        raft_stream_destroy(s);
        return r;
    }
    *out = s;
    return RAFT_OK;
}

raft_status raft_stream_graph(const raft_stream* s, const raft_graph** g) {
    if (!s || !g) return RAFT_E_INVAL;
    *g = &s->gr[s->cur];
    return RAFT_OK;
}

raft_status raft_stream_embedding(const raft_stream* s, float* Y, float* Z, void* stream) {
    if (!s) return RAFT_E_INVAL;
    raft_ctx* ctx = s->ctx;
    hipStream_t st = as_stream(stream);
    const size_t n = (size_t)s->n;
    if (Y)
        HIP_TRY(ctx, hipMemcpyAsync(Y, s->y[s->cfg.q], n * s->L * sizeof(float),
                                    hipMemcpyDeviceToDevice, st));
    if (Z) {
        const int d = s->cfg.n_layers ? s->lout.back() : s->L;
        HIP_TRY(ctx, hipMemcpyAsync(Z, s->z(), n * d * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    return RAFT_OK;
}

raft_status raft_stream_add_edges(raft_stream* s, const int32_t* src, const int32_t* dst,
                                  int64_t m, void* stream, int64_t* rows_per_level) {
    if (!s) return RAFT_E_INVAL;
    raft_ctx* ctx = s->ctx;
    if (m < 0 || (m > 0 && (!src || !dst))) return fail(ctx, RAFT_E_INVAL, "edge arrays");
    const int n = s->n;
    if (m == 0) {
        if (rows_per_level) std::fill(rows_per_level, rows_per_level + s->R, (int64_t)0);
        return RAFT_OK;
    }
    raft_graph* g = s->g();
    if (g->nnz + 2 * m >= INT32_MAX)
        return fail(ctx, RAFT_E_UNSUPPORTED, "%lld entries do not fit the int32 CSR",
                    (long long)(g->nnz + 2 * m));
    // both directions of every edge sorted by (row, col); V' = the rows
    std::vector<std::pair<int32_t, int32_t>> dir;
    dir.reserve((size_t)2 * m);
    for (int64_t e = 0; e < m; ++e) {
        const int32_t a = src[e], b = dst[e];
        if (a < 0 || a >= n || b < 0 || b >= n)
            return fail(ctx, RAFT_E_INVAL, "edge %lld (%d, %d) out of range", (long long)e, a, b);
        if (a == b) return fail(ctx, RAFT_E_INVAL, "edge %lld is a self pair (%d)", (long long)e, a);
        dir.emplace_back(a, b);
        dir.emplace_back(b, a);
    }
    std::sort(dir.begin(), dir.end());
    for (size_t q = 1; q < dir.size(); ++q)
        if (dir[q] == dir[q - 1])
            return fail(ctx, RAFT_E_INVAL, "edge (%d, %d) given twice", dir[q].first,
                        dir[q].second);
    const int64_t m2 = (int64_t)dir.size(), nnz2 = g->nnz + m2;
    std::vector<int32_t> host((size_t)3 * m2);
    int32_t* rows = host.data();
    int32_t* cols = rows + m2;
    int32_t* vp = cols + m2;
    int nv = 0;
    for (int64_t q = 0; q < m2; ++q) {
        rows[q] = dir[q].first;
        cols[q] = dir[q].second;
        if (q == 0 || rows[q] != rows[q - 1]) vp[nv++] = rows[q];
    }
    hipStream_t st = as_stream(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int nxt = 1 - s->cur;
    raft_graph* g2 = &s->gr[nxt];
    if (s->edge_cap < m2) {
        if (!stream_realloc(s, &s->edges, (size_t)3 * m2)) {
            s->edge_cap = 0;
            return fail(ctx, RAFT_E_NOMEM, "stream edge staging");
        }
        s->edge_cap = m2;
    }
    if (s->ci_cap[nxt] < nnz2) {
        const int64_t cap = std::min<int64_t>(nnz2 + nnz2 / 4, INT32_MAX);
        if (!stream_realloc(s, &g2->ci, cap)) {
            s->ci_cap[nxt] = 0;
            return fail(ctx, RAFT_E_NOMEM, "stream graph growth");
        }
        s->ci_cap[nxt] = cap;
    }
    int32_t* d_rows = s->edges;
    int32_t* d_cols = d_rows + m2;
    int32_t* d_vp = d_cols + m2;
    HIP_TRY(ctx, hipMemcpyAsync(d_rows, host.data(), sizeof(int32_t) * (2 * m2 + nv),
                                hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemsetAsync(s->mstatus, 0, sizeof(int32_t), st));
    launch_stream_merge(g->rp, g->ci, n, d_rows, d_cols, m2, s->add_cnt, s->add_off, s->bsum,
                        s->totals, g2->rp, g2->ci, s->mstatus, st);
    HIP_TRY(ctx, hipMemcpyAsync(g2->order, g->order, sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                                st));
    std::copy(g->heavy, g->heavy + 17, g2->heavy);
    launch_degrees(g2->rp, n, nnz2, g2->deg, g2->s, g2->sh, g2->dcoef, st);
    const bool local = s->cfg.op == RAFT_X_NCUT;
    if (local)
        launch_stream_balls(g2->rp, g2->ci, n, d_vp, nv, s->R, s->dist, s->flag, s->pos, s->bsum,
                            s->totals, s->lists, st);
    RAFT_TRY(launch_check(ctx));
    // status and the ball sizes in one read-back (the pageable staging
    // vector above is also released by this wait)
    int32_t* h_status = ctx->h_pinned;
    int64_t* h_counts = reinterpret_cast<int64_t*>(ctx->h_pinned + 2);
    HIP_TRY(ctx, hipMemcpyAsync(h_status, s->mstatus, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (local)
        HIP_TRY(ctx, hipMemcpyAsync(h_counts, s->totals, sizeof(int64_t) * s->R,
                                    hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (h_status[0])
        return fail(ctx, RAFT_E_CSR, "stream update: an edge is already in the graph; nothing changed");
    std::vector<int64_t> counts(s->R, n);
    if (local) std::copy(h_counts, h_counts + s->R, counts.begin());
    g2->nnz = nnz2;
    s->cur = nxt;
    const raft_status r = local ? stream_incremental(s, counts.data(), st) : stream_full(s, st);
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (rows_per_level) std::copy(counts.begin(), counts.end(), rows_per_level);
    return r;
}

}  // extern "C"
