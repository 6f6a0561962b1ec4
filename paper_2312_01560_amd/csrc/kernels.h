// Kernel launchers of the HIP path (internal interface between the C ABI and
// the .hip translation units).  All launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace raft {

// ---- graph.hip -----------------------------------------------------------
void launch_validate_csr(const int32_t* rp, const int32_t* ci, int32_t n, int32_t* status,
                         int num_cu, hipStream_t st);
void launch_degrees(const int32_t* rp, int32_t n, int64_t nnz, int32_t* deg, float* s, float* sh,
                    float* dcoef, hipStream_t st);
void launch_offset_copy(const int32_t* src, int32_t* dst, int64_t n, int32_t add, hipStream_t st);

// ---- gauss.hip -----------------------------------------------------------
void launch_gaussian(uint64_t seed, uint64_t stream_id, int64_t rows, int64_t cols, double sigma,
                     float* out, hipStream_t st);

// Batched launches (many graphs in one launch) take per-graph items in device
// memory and a BatchTable (common.h) whose counts come from the *_blocks
// functions below.
struct GaussItem {
    uint64_t seed, stream;
    int64_t rows, cols;
    double sigma;
    float* out;
};
int gaussian_blocks(int64_t rows, int64_t cols);
void launch_gaussian_batched(const GaussItem* items, const BatchTable& t, int grid,
                             hipStream_t st);

// ---- spmm.hip ------------------------------------------------------------
enum SpmmOp { kOpNcut = 0, kOpModFull = 1, kOpModReduced = 2, kOpGcn = 3 };

struct GraphView {
    int32_t n;
    int64_t nnz;
    const int32_t* rp;
    const int32_t* ci;
    const int32_t* deg;
    const float* s;      // D^-1/2 (0 for isolated nodes)
    const float* sh;     // (D+1)^-1/2
    const float* dcoef;  // d_i / 2e
    const int32_t* order;  // [n] rows by degree class, heaviest first (row-split schedules)
    // Global id of the graph's node 0: 0 for a graph on its own; in a batch,
    // where the graphs form one block-diagonal CSR, the graph's first row.
    // rp, ci, order and the per-node arrays hold global ids; kernels that walk
    // the graph's rows by local index add base.
    int32_t base = 0;
};

// Grid size (work-groups) of one SpMM launch; colsum partial buffers hold
// spmm_grid(...) * L doubles.
int spmm_grid(int32_t n, int L, int num_cu, int* rows_per_wave);
bool spmm_supported(int L);
// y = X x for operator op.  cvec: FP32 d^T x (MOD_FULL only).  If colsum_part
// is non-null, also writes per-work-group FP64 partials of d^T y.
void launch_spmm(const GraphView& g, int op, int L, const float* x, float* y, const float* cvec,
                 double* colsum_part, int num_cu, hipStream_t st);
// FP64 partials of d^T x over row blocks (grid = spmm_grid(...)).
void launch_colsum_partials(const GraphView& g, int L, const float* x, double* part, int num_cu,
                            hipStream_t st);
// c = sum of `parts` partial rows (fixed order), cvec = FP32(c).  The partial
// buffer must hold kColsumStageRows more rows after the partials (stage).
constexpr int kColsumStageRows = 64;
void launch_colsum_finish(const double* part, int parts, int L, double* c64, float* cvec,
                          hipStream_t st);

// Merge-path SpMM (work split evenly over row ends + stored entries):
// workspace bytes for (n, nnz, L, op) and the launch (a range pass and a
// fix-up pass).  No column-sum epilogue.
int spmm_merge_ranges(int32_t n, int64_t nnz);
size_t spmm_merge_ws_bytes(int32_t n, int64_t nnz, int L, int op);
void launch_spmm_merge(const GraphView& g, int op, int L, const float* x, float* y,
                       const float* cvec, void* ws, hipStream_t st);

// Grid of one graph's SpMM launch; R = rows per row block, nrb = row blocks.
int spmm_launch_shape(int32_t n, int L, int num_cu, int* R, int* nrb);
struct SpmmItem {
    GraphView g;
    const float* cvec;   // MOD_FULL: the graph's FP32 d^T x
    double* cpart;       // the graph's colsum partials (with the epilogue)
    int32_t R, nrb;
};
void launch_spmm_batched(const SpmmItem* items, int op, int L, const float* x, float* y, bool cs,
                         const BatchTable& t, int grid, hipStream_t st);
struct ColsumItem {
    GraphView g;
    double* part;        // [parts + kColsumStageRows] x L
    int32_t parts, rpw;
    double* c64;
    float* cvec;
};
void launch_colsum_partials_batched(const ColsumItem* items, int L, const float* x,
                                    const BatchTable& t, int grid, hipStream_t st);
// kColsumSlices blocks per graph (t_slices), then one per graph (t_one).
void launch_colsum_finish_batched(const ColsumItem* items, int L, const BatchTable& t_slices,
                                  int grid_slices, const BatchTable& t_one, int grid_one,
                                  hipStream_t st);
constexpr int kColsumSliceBlocks = 64;

// ---- dense.hip -----------------------------------------------------------
bool dense_supported(int lin, int lout);
// H = rownorm(tanh(P W)) (or U = P W when linear), P [n x lin], W [lin x lout].
void launch_dense_layer(const float* P, const float* W, float* H, int32_t n, int lin, int lout,
                        bool linear, int32_t* status, int num_cu, hipStream_t st);
// Row L2 normalisation in place (x / max(||x||, 1e-12)).
void launch_rownorm(float* x, int32_t n, int L, hipStream_t st);

struct DenseItem {
    const float* P;      // [n x lin] (the graph's rows)
    const float* W;      // [lin x lout] (the graph's own weights)
    float* H;            // [n x lout]
    int32_t n;
};
int dense_blocks(int32_t n);
void launch_dense_layer_batched(const DenseItem* items, int lin, int lout, bool linear,
                                int32_t* status, const BatchTable& t, int grid, hipStream_t st);
int rownorm_blocks(int32_t n);
// Normalises items[g].H (n rows of width L) in place.
void launch_rownorm_batched(const DenseItem* items, int L, const BatchTable& t, int grid,
                            hipStream_t st);

// ---- kmeans.hip ----------------------------------------------------------
struct KmeansPlan {
    int32_t n, d, Kc, k_max;
    int32_t KP;          // padded centre rows (sum of ceil16(K))
    int32_t SK;          // real centre count (sum of K)
    int32_t agroups;     // candidate groups of the assignment kernel (over alist)
    int32_t ugroups;     // candidate groups of the update kernel (over alist)
    int32_t usk_max;     // bound on the accumulator rows of an update group (LDS sizing)
    int32_t uwork;       // update work items (group, point range)
    int32_t race_grid;
    // device arrays
    const int32_t* ks;       // [Kc]
    const int32_t* koff16;   // [Kc] padded centre offsets
    const int32_t* koff;     // [Kc] real offsets (score tables)
    const int32_t* cand_of;  // [KP] candidate of each padded centre row
    const int32_t* alist;    // [Kc] candidates still active at the last poll
    const int32_t* agrp;     // [agroups + 1] offsets into alist
    const int32_t* ugrp;     // [ugroups + 1] offsets into alist
    const int32_t* uwi0;     // [ugroups + 1] first work item of each update group
    const int32_t* ulen;     // [ugroups] point range length of each update group
    const int32_t* cranges;  // [Kc] point ranges of each candidate's update group
    int32_t* active;         // [Kc]
    int32_t* changes;        // [Kc] non-zero when a label of the candidate changed
    int32_t* iters;          // [Kc]
    int32_t* active_count;   // [1]
    float* C;                // [KP x d]
    float* cnorm;            // [KP]
    // Split-fp16 operands of the assignment (split != 0): x 2^s = hi + lo,
    // s = 10 - (exponent of the largest |z|), both halves fp16 bit patterns.
    int32_t split;
    int32_t group_major;     // assignment block order: candidate group fastest (large N)
    uint16_t* zh;            // [n x d]
    uint16_t* zl;            // [n x d]
    uint16_t* ch;            // [KP x d]
    uint16_t* cl;            // [KP x d]
    long long* S64;          // [KP x d] centre sums, fixed point (z * 2^e as int32, summed)
    int32_t* N32;            // [KP] cluster sizes
    long long* pdelta;       // [max ranges x KP x d] per-range changes of S64 (flagged rows)
    int32_t* pcnt;           // [max ranges x KP] per-range changes of N32
    uint8_t* pdirty;         // [max ranges x KP] a point moved into or out of the row
    uint32_t* zmax_bits;     // [1] largest |z| (float bits), sets the fixed-point scale
    float* w;                // [n]
    double* race_val;        // [2 x race_grid] per-group minima, by launch parity
    int32_t* race_idx;       // [2 x race_grid]
    int32_t* picks;          // [k_max]
    uint8_t* lab_cm;         // [Kc x n] candidate-major labels
    uint8_t* lab_old;        // [Kc x n] labels before the last assignment (0xFF: none)
    // Last iteration in which a label of the 64-point chunk changed, per
    // candidate: written by the assignment, read by the update of the same
    // iteration to skip chunks no point of a candidate left or entered.
    int32_t* moved_it;       // [nchunks x Kc]
    int32_t nchunks;         // ceil(n / 64)
    int32_t it;              // Lloyd iteration of the launch (1-based)
    int32_t* status;
    uint64_t seed;           // Philox key word 0 of the race
    int32_t zoff = 0;        // in a batch: first row of the graph's points in the packed Z
    // Bound-pruned assignment (single graphs, split-fp16; prune != 0): from
    // iteration kPruneFrom on, k_prune_test lists the points whose distance
    // bounds do not prove their label and k_prune_score scores them.  Bounds per (candidate,
    // point), with Cum the summed drift of a
    // centre and CumMax the summed largest drift of the candidate's centres:
    //   hu = u - Cum_a   (u >= distance to the own centre a, rounded up)
    //   hl = l + CumMax  (l <= distance to every other centre, rounded down)
    // as of the point's last scoring; null and 0 when not pruning.
    int32_t prune = 0;
    float* hu = nullptr;        // [Kc x n]
    float* hl = nullptr;        // [Kc x n]
    double* cum = nullptr;      // [KP] summed drift of each centre row
    double* cmx = nullptr;      // [Kc] summed largest drift, updates before the previous one
    double* dmx = nullptr;      // [Kc x 2] largest drift of an update, slot = iteration & 1
    float* zn2 = nullptr;       // [n] |z|^2, rounded up
    float* pe = nullptr;        // [n] bound on the error of a computed score, rounded up
    int32_t* plist = nullptr;   // [Kc x n] listed points, each range in its own slots
    int32_t* scnt = nullptr;    // [Kc x nranges] listed points per range
    int32_t nranges = 0;        // ceil(n / kPruneRange)
    int32_t lists_nact = 0;     // alist positions k_prune_score's LDS holds (set per launch)
    int32_t list_tiles = 0;     // centre tiles of the largest candidate (LDS of k_prune_score)
    uint32_t* znmax_bits = nullptr;   // [1] largest |z| (float bits)
};

// Points per work-group of the pruned assignment (bound tests, then scoring).
constexpr int kPruneRange = 2048;
// First Lloyd iteration whose assignment is pruned (the first two move the
// centres too far for the bounds to hold many points).
constexpr int kPruneFrom = 3;

bool kmeans_supported(int d);
int kmeans_race_grid(int32_t n, int num_cu);
// LDS bytes of one update work-group whose candidates total sum_rows
// accumulator rows (kmeans_update_rows(K) per candidate).
size_t kmeans_update_lds(int sum_rows, int d);
int kmeans_update_rows(int K);
// Candidates one update work-group can hold.
int kmeans_update_max_candidates();
void launch_kmeans_reset(const KmeansPlan& p, hipStream_t st);
void launch_zmax(const KmeansPlan& p, const float* Z, int num_cu, hipStream_t st);
// Pick t of the race (launch t resolves pick t-1; the launch of the last
// pick also resolves it).
void launch_race_pick(const KmeansPlan& p, const float* Z, int t, hipStream_t st);
void launch_init_centres(const KmeansPlan& p, const float* Z, hipStream_t st);
// e0 / e1 (nullable): events the launch records itself at its start and end.
void launch_assign(const KmeansPlan& p, const float* Z, int num_cu, hipStream_t st,
                   hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Split-fp16 assignment is available for d multiple of 32.
bool kmeans_split_supported(int d);
// Pruned assignment: bounds and the fills they start from (once per
// partition, after the points are split); then per iteration from
// kPruneFrom on, one launch over the `nact` candidates of alist.  e0 / e1 as
// for launch_assign.
void launch_prune_init(const KmeansPlan& p, const float* Z, hipStream_t st);
size_t list_lds_bytes(int d, int tiles, int lists);
// Dynamic LDS the scoring kernel may use (its static LDS stays below 8 KB).
constexpr int kPruneDynLdsMax = 152 * 1024;
void launch_assign_pruned(const KmeansPlan& p, int nact, int num_cu, hipStream_t st,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// zh/zl from Z (after launch_zmax).
void launch_split_points(const KmeansPlan& p, const float* Z, hipStream_t st);
void launch_iter_finalize(const KmeansPlan& p, int it, int t_max, hipStream_t st);
// Update of iteration `it` followed by the end-of-iteration bookkeeping
// (what launch_iter_finalize does, fused into the finishing kernel).
void launch_update(const KmeansPlan& p, const float* Z, size_t lds_max, int it, int t_max,
                   hipStream_t st);
// Real centre rows of every candidate, compacted: out [SK x d] (grid order).
void launch_copy_centres(const KmeansPlan& p, float* out, hipStream_t st);

// Launch kinds of the k-means stage, their grid per graph, and the batched
// launch of one kind over all graphs (`it` is the pick index for kKmRace and
// the Lloyd iteration otherwise).
enum KmeansKind {
    kKmReset, kKmZmax, kKmSplit, kKmRace, kKmRaceFinal, kKmInit, kKmAssign, kKmFinalize,
    kKmUpdate, kKmUpdateFinish, kKmKinds
};
// Candidates of one assignment group at most (each has at least 16 padded
// centre rows and a group closes at 256 rows, so groups stay below this).
constexpr int kAssignMaxGroup = 16;
// Waves per work-group of the split-fp16 assignment at d <= 64 (measured at
// N = 50k, d = 64: 2 waves 70.4 us, 4 waves 48.8 us, 8 waves 53.4 us).
constexpr int kAssignWavesSmallD = 4;
int kmeans_blocks(const KmeansPlan& p, int kind, int num_cu);
void launch_kmeans_batched(int kind, const KmeansPlan* plans, int d, bool split, const float* Z,
                           int it, int t_max, size_t lds_max, size_t update_lds,
                           const BatchTable& t, int grid, hipStream_t st);

// ---- score.hip -----------------------------------------------------------
struct ScorePlan {
    int32_t n, Kc, S;     // S = row stride of point-major labels (multiple of 8)
    int32_t SK;           // sum of K
    int32_t grid;
    int32_t heavy = 0;    // leading rows of the row order whose edges a wave splits
    int64_t nnz;
    const int32_t* ks;
    const int32_t* koff;
    int32_t* lpart;       // [grid x SK]
    int32_t* vpart;       // [grid x SK]
    int64_t* l64;         // [SK]
    int64_t* v64;         // [SK]
    double* mod;          // [Kc]
    double* ncut;         // [Kc]
    int32_t* best;        // [1]
    int32_t* first;       // [RAFT_MAX_K + 1]
    int32_t* remap;       // [RAFT_MAX_K + 1]
    int32_t* status;
    // batched launches only (a single graph passes these as arguments)
    uint8_t* lab = nullptr;              // [n x S] point-major labels of the graph
    const uint8_t* lab_cm = nullptr;     // [Kc x n] candidate-major labels (k-means)
    int32_t* ksel_out = nullptr;         // [3] K*, K_eff, index of K*
    int32_t* labels_out = nullptr;       // [n] canonical labels of K* (nullable)
    uint8_t* labels_all_out = nullptr;   // [n x Kc] (nullable)
};

int score_grid(int32_t n, int num_cu);
bool score_supported(int Kc, int SK);   // Kc <= 256 labelings, sum of K <= 16384
// Rows with at least this many 16-edge batches are split over the row groups
// of a wave by the edge-score kernel (for label row stride S).
int score_split_batches(int S);
void launch_transpose_labels(const uint8_t* cm, int32_t n, int Kc, uint8_t* pm, int S,
                             hipStream_t st);
void launch_edge_score(const GraphView& g, const ScorePlan& p, const uint8_t* lab_pm,
                       hipStream_t st);
void launch_score_finish(const ScorePlan& p, hipStream_t st);
// Selection of K* (first maximum of Mod) and canonical relabelling.
void launch_select(const ScorePlan& p, const uint8_t* lab_pm, int32_t* labels_out,
                   int32_t* k_selected, hipStream_t st);
// Copy point-major labels [n x S] into a dense [n x Kc] output.
void launch_copy_labels(const uint8_t* pm, int32_t n, int Kc, int S, uint8_t* out, hipStream_t st);

// Launch kinds of the score stage, their grid per graph, and the batched
// launch of one kind over all graphs (S, SK: shared by every graph).
enum ScoreKind {
    kScTranspose, kScEdge, kScReduce, kScFinalize, kScSelect, kScFirst, kScRank, kScApply,
    kScCopy, kScKinds
};
int score_blocks(const ScorePlan& p, int kind);
void launch_score_batched(int kind, const GraphView* views, const ScorePlan* plans, int S, int SK,
                          const BatchTable& t, int grid, hipStream_t st);

// ---- hier.hip ------------------------------------------------------------
// State of one level of the hierarchical model selection (Alg. 1): the sets
// being partitioned, each a segment [beg, beg + cnt) of the node permutation.
struct HierPlan {
    const float* Z;          // [n x d]
    int32_t d;
    uint64_t seed;           // Philox key word 0 of the K = 2 race
    int32_t depth;           // level of the sets in the tree (race counter word 2)
    int32_t fexp;            // fixed-point exponent of the centre sums
    const int32_t* beg;      // [nsets]
    const int32_t* cnt;      // [nsets]
    const int32_t* need;     // [nsets] 1: run KMeans (|U| > 2 eps + 1)
    const int32_t* child;    // [2 nsets] next-level set of each side, -1: U is a block
    const int32_t* tnode;    // [nsets] tree node of the set
    int32_t* perm;           // [n] this level's segments
    int32_t* perm_next;      // [n]
    int32_t* setid;          // [n] set of each node at this level (-1: in a block)
    int32_t* setid_next;     // [n]
    int8_t* side;            // [n] side of each node in its set's split
    int32_t* leaf;           // [n] tree node of the block holding the node
    int32_t* pick;           // [2 nsets]
    double* rval;            // [race grid] per-work-group race minima
    int32_t* ridx;           // [race grid]
    int32_t* rlow;           // [race grid] lowest node id other than pick 0
    float* C;                // [nsets x 2 x d]
    float* cnorm;            // [nsets x 2]
    long long* S64;          // [nsets x 2 x d] fixed-point sums of the sides
    int32_t* n32;            // [nsets x 2]
    int32_t* active;         // [nsets]
    int32_t* changed;        // [nsets]
    int32_t* iters;          // [nsets]
    int32_t* live;           // [1] sets still iterating after an update
    long long* counts;       // [nsets x 7] integer counts of Eq. 7
    int32_t* cursor;         // [next nsets] fill positions of the children's segments
};
enum HierKind { kHierRace, kHierPick, kHierInit, kHierAssign, kHierUpdate, kHierCounts,
                kHierScatter };
void launch_hier(int kind, const HierPlan& h, const GraphView& g, int d, int t, int t_max,
                 int nsets, const BatchTable& tb, int grid, hipStream_t st);
void launch_hier_trace(const HierPlan& h, int32_t* out, const BatchTable& tb, int grid,
                       hipStream_t st);
void launch_hier_labels(const int32_t* leaf, const int32_t* block_of, int n, int32_t* labels,
                        hipStream_t st);
// zmax_bits = bits of the largest |Z| (zeroed first); perm = 0..n-1,
// setid = setid_next = 0, side = 0, leaf = -1.
void launch_hier_setup(const float* Z, int64_t total, uint32_t* zmax_bits, int32_t* perm,
                       int32_t* setid, int32_t* setid_next, int8_t* side, int32_t* leaf, int n,
                       hipStream_t st);
// Clears count arrays of the level (a kernel, no memset).
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_fill_i64(long long* p, int64_t n, hipStream_t st);

// ---- sampler.hip -----------------------------------------------------------
// One level of rows of the fast SBM sampler: row x of block pair (r, s),
// r <= s, is node members[boff[r] + x] against block s.
constexpr int kSbmMaxBlocks = 4096;
struct SbmPlan {
    int32_t k, npairs;
    int64_t nrows;
    uint64_t seed;
    const double* theta;     // [n]
    const double* omega;     // [k x k]
    const int32_t* members;  // [n] nodes grouped by block, increasing id in a block
    const int32_t* boff;     // [k] first member of each block
    const int32_t* bcount;   // [k]
    const double* pref;      // [n + k] per block: 0, theta sums left to right (n_s + 1 values)
    const int64_t* rowoff;   // [npairs + 1] first row of each pair
    const int32_t* pair_r;   // [npairs]
    const int32_t* pair_s;   // [npairs]
};
void launch_sbm_rows(const SbmPlan& p, bool write, int64_t* cnt, const int64_t* off,
                     int32_t* src, int32_t* dst, hipStream_t st);
// Exclusive scan (out[i] = sum of v[0..i)); bsum holds ceil(n / 1024) values,
// total the sum of all.
void launch_scan_i64(const int64_t* v, int64_t n, int64_t* out, int64_t* bsum, int64_t* total,
                     hipStream_t st);
// Symmetric CSR of the edge list (both directions, rows sorted): deg [n + 1],
// rp [n + 1], cursor [n], bsum [ceil((n + 1) / 1024)], total [1], col [2 ne].
hipError_t launch_sbm_csr(const int32_t* src, const int32_t* dst, int64_t ne, int n,
                          int64_t* deg, int64_t* rp, int64_t* cursor, int64_t* bsum,
                          int64_t* total, int32_t* col, hipStream_t st);

// ---- stream.hip ------------------------------------------------------------
constexpr int kStreamMaxLevels = 64;   // q + GCN layers of a stream
// Merged CSR of a graph and m directed new entries (rows, cols) sorted by
// (row, col): add_cnt / add_off [n + 1], bsum [ceil((n + 1) / 1024)],
// total [1], rp_new [n + 1], ci_new [nnz + m].  A new entry already in the
// graph sets kStatusCsrSym.
void launch_stream_merge(const int32_t* rp, const int32_t* ci, int32_t n, const int32_t* rows,
                         const int32_t* cols, int64_t m, int64_t* add_cnt, int64_t* add_off,
                         int64_t* bsum, int64_t* total, int32_t* rp_new, int32_t* ci_new,
                         int32_t* status, hipStream_t st);
// Hop distances from vprime (radius + 1 beyond radius) and, for t = 1..radius,
// lists[(t - 1) n ..] = the rows within t hops in increasing id, totals[t - 1]
// their number.  flag / pos [n], bsum [ceil(n / 1024)].
void launch_stream_balls(const int32_t* rp, const int32_t* ci, int32_t n, const int32_t* vprime,
                         int32_t nv, int radius, int32_t* dist, int64_t* flag, int64_t* pos,
                         int64_t* bsum, int64_t* totals, int32_t* lists, hipStream_t st);
// Row gather (dst[r] = src[list[r]]) or scatter (dst[list[r]] = src[r]).
void launch_stream_rows(bool gather, const int32_t* list, int32_t c, int L, const float* src,
                        float* dst, hipStream_t st);

// ---- confusion.hip -------------------------------------------------------
// counts [ka x kb] int64 (zeroed here) = joint histogram of labels a, b [n];
// a label out of range sets kStatusLabel and is not counted.
void launch_confusion(const int32_t* a, const int32_t* b, int64_t n, int ka, int kb,
                      int64_t* counts, int32_t* status, int num_cu, hipStream_t st);

// ---- train.hip -----------------------------------------------------------
void launch_softmax_rows(const float* U, float* S, int n, int K, hipStream_t st);
int rowdot_parts(int64_t total);
// loss = -sum(S o BS) / m2 in FP64 (part: rowdot_parts(total) doubles)
void launch_modloss_value(const float* S, const float* BS, int64_t total, double m2, double* part,
                          double* loss, hipStream_t st);
void launch_modloss_grad(const float* S, const float* BS, int n, int K, double inv_e,
                         const float* scale, float* GU, hipStream_t st);
void launch_tanh_norm_backward(const float* U, float* G, int n, int L, hipStream_t st);
void launch_transpose(const float* W, int rows, int cols, float* WT, hipStream_t st);
int wgrad_parts(int n);
bool wgrad_supported(int li, int lo);
// GW = P^T GU (part: wgrad_parts(n) * li * lo floats)
void launch_wgrad(const float* P, const float* GU, int n, int li, int lo, float* part, float* GW,
                  hipStream_t st);
void launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                 float b2, float eps, int step, hipStream_t st);

}  // namespace raft
