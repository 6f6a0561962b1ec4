/*
 * raftgp.h -- C ABI of the MI355X (gfx950) implementation of the RaftGP hot
 * path (Gao et al., "RaftGP: Random Fast Graph Partitioning", IEEE HPEC 2023).
 *
 * Problem statement (Sec. II): an undirected, unweighted graph G = (V, E) with
 * symmetric adjacency A in {0,1}^{N x N} is partitioned into K disjoint
 * blocks, K not given.  The method (Sec. III) is
 *   1. random feature extraction   Y = X^q Theta   (Sec. III-A, Eq. 5),
 *      X = M = D^-1/2 A D^-1/2 (NCut, Eq. 2) or the modularity matrix
 *      (Eq. 4; full B = A - d d^T/2e applied in low-rank form, or the paper's
 *      edge-masked reduced matrix Q~);
 *   2. random embedding            Z = GCN(Y) with untrained random weights
 *      (Sec. III-B, Eq. 6, tanh, row L2 normalisation);
 *   3. model selection             k-means on Z for every candidate K of a
 *      grid, scored by modularity (Eq. 3) and NCut (Eq. 1); K* = argmax Mod.
 *
 * Conventions for every call:
 *   - Return value: raft_status, RAFT_OK (0) or a negative error code.
 *     Nothing aborts or throws.  raft_last_error() gives a message.
 *   - Device pointers are HIP device (or managed) memory on the context's
 *     device; the caller owns every buffer it passes in.  Dense matrices are
 *     row-major FP32.
 *   - `stream` is a hipStream_t (NULL = default stream).  Compute calls are
 *     asynchronous on that stream unless documented otherwise; argument
 *     errors are reported synchronously before anything is enqueued.
 *   - Device-detected errors (non-finite values, invalid CSR) are latched in
 *     a status word and returned by raft_sync_status().
 *   - A context is used by one host thread at a time.  Graph handles are
 *     immutable after creation.
 */
#ifndef RAFTGP_H
#define RAFTGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAFT_ABI_VERSION 4

typedef int32_t raft_status;
#define RAFT_OK             0
#define RAFT_E_INVAL       -1   /* bad argument (null pointer, size, range)   */
#define RAFT_E_CSR         -2   /* CSR not symmetric/sorted/unique/loop-free   */
#define RAFT_E_NOEDGES     -3   /* e = 0: modularity (Eq. 3) divides by e      */
#define RAFT_E_WORKSPACE   -4   /* workspace smaller than raft_workspace_size  */
#define RAFT_E_NOMEM       -5   /* device allocation failed                    */
#define RAFT_E_DEVICE      -6   /* HIP runtime error                           */
#define RAFT_E_NUMERIC     -7   /* non-finite value detected on the device     */
#define RAFT_E_UNSUPPORTED -8   /* width / K outside the compiled kernels      */

/* Structural operator X of the random projection (Sec. III-A). */
#define RAFT_X_NCUT        0    /* M = D^-1/2 A D^-1/2 (Eq. 2); D^-1/2 = 0 for isolated nodes */
#define RAFT_X_MOD_FULL    1    /* B = A - d d^T / 2e (Eq. 4), never formed                 */
#define RAFT_X_MOD_REDUCED 2    /* Q~: B masked to the edge set (Sec. III-A)                */
#define RAFT_X_GCN         3    /* D^-1/2 (A + I) D^-1/2 with D = deg + 1 (Eq. 6)           */

/* Feature / embedding widths supported by the kernels. */
#define RAFT_MAX_LAYERS 8
#define RAFT_MAX_K      255     /* labels are stored as bytes                */

typedef struct raft_ctx raft_ctx;
typedef struct raft_graph raft_graph;

typedef struct {
    int32_t  abi_version;              /* must be RAFT_ABI_VERSION                    */
    int32_t  op;                       /* RAFT_X_NCUT / MOD_FULL / MOD_REDUCED        */
    int32_t  proj_dim;                 /* L, a power of two 16..4096 (batches: <= 256) */
    int32_t  q;                        /* propagation steps, >= 1 (q = 1 is Eq. 5)    */
    int32_t  n_layers;                 /* GCN layers, 0..RAFT_MAX_LAYERS               */
    int32_t  layer_dims[RAFT_MAX_LAYERS]; /* L_1..L_n, powers of two 16..4096 (a layer
                                          * wider than 128 x 256 needs L_k >= 128); the
                                          * embedding width d = last <= 256            */
    int32_t  normalize_input;          /* row-normalise Y before layer 1 (default 0)  */
    int32_t  k_min, k_max, k_step;     /* candidate grid, 1 <= k_min <= k_max <= min(N, 255) */
    int32_t  kmeans_max_iter;          /* T_max (assignments per candidate), >= 1     */
    int32_t  check_every;              /* host convergence poll period (0 = 4)        */
    int32_t  kmeans_prune;             /* Lloyd assignments from the third on may skip
                                        * the points whose distance bounds prove their
                                        * label cannot change (single graphs, split-fp16
                                        * path): 0 (default) where it pays, when the
                                        * grid's mean K is at least 64; 1 whenever
                                        * supported; 2 never.  Labels, centres and
                                        * iteration counts are the same in every mode. */
    uint64_t seed;                     /* Philox key word 0 for Theta, W and the race */
} raft_config;

/* Output buffers of raft_partition / raft_run (device memory, caller-owned).
 * Kc = number of candidates in the grid, K_max = the largest candidate. */
typedef struct {
    float*   Y;            /* [N x L] projected features (nullable)                  */
    float*   Z;            /* [N x d] embedding (nullable in raft_run)               */
    int32_t* labels;       /* [N] labels of K*, relabelled by first occurrence       */
    int32_t* k_selected;   /* [3]: K*, K_eff (non-empty blocks), index of K* in grid */
    double*  mod;          /* [Kc] modularity per candidate (nullable)               */
    double*  ncut;         /* [Kc] NCut per candidate (nullable)                     */
    uint8_t* labels_all;   /* [N x Kc] labels of every candidate, point-major (nullable) */
    int32_t* picks;        /* [K_max] k-means++ picks (nullable)                     */
    int32_t* iters;        /* [Kc] Lloyd assignments performed (nullable)            */
    float*   centres;      /* [sum of K x d] final centres, candidate after candidate in
                            * grid order, K rows each (nullable).  A candidate that
                            * converged has each non-empty centre equal to the mean of
                            * its points; an empty cluster keeps its last centre.     */
} raft_outputs;

/* ---- context and errors ------------------------------------------------- */

/* Create a context on HIP device `device`.  *out receives the handle.
 * autotune_cache (nullable): path of a text file in which the launch-shape
 * tuner keeps its measured choices (read at creation when it exists,
 * rewritten when a choice is added); NULL keeps the choices in memory only. */
raft_status raft_ctx_create(int device, const char* autotune_cache, raft_ctx** out);
void        raft_ctx_destroy(raft_ctx* ctx);
const char* raft_status_string(raft_status s);
/* Copies the last error message of this context into buf (NUL-terminated);
 * returns the full message length. */
size_t      raft_last_error(raft_ctx* ctx, char* buf, size_t n);
int32_t     raft_abi_version(void);
/* Synchronises `stream` and returns RAFT_E_NUMERIC if a kernel flagged a
 * non-finite value since the last call (the flag is then cleared). */
raft_status raft_sync_status(raft_ctx* ctx, void* stream);

/* ---- graph (Sec. II: undirected unweighted A, CSR) ----------------------- */

/* Copies a CSR (row_ptr[n+1], col_idx[nnz] int32) into library-owned device
 * memory, validates it on the device (sorted unique columns, no self loops,
 * symmetric, in range) and computes degrees, 2e and the scale vectors
 * D^-1/2 and (D+1)^-1/2.  row_ptr holds int32 entries, or int64 entries
 * when row_ptr_is_int64 != 0; int64 offsets are checked (0 first, nnz last,
 * non-decreasing) and narrowed to the library's int32 CSR, and nnz >= 2^31 - 1
 * returns RAFT_E_UNSUPPORTED.  `inputs_on_device` != 0 means the two arrays
 * are device pointers.  Synchronous: returns after validation (RAFT_E_CSR on
 * a malformed graph).  The caller may free its arrays on return. */
raft_status raft_graph_create(raft_ctx* ctx, const void* row_ptr, int row_ptr_is_int64,
                              const int32_t* col_idx, int64_t n, int64_t nnz,
                              int inputs_on_device, void* stream, raft_graph** out);
void        raft_graph_destroy(raft_graph* g);
/* Device copies of the degree vector (int32 [N]) and of the CSR (for tests). */
raft_status raft_graph_degrees(const raft_graph* g, int32_t* deg_out, void* stream);
/* N and nnz (stored entries, 2|E|) of a graph; either pointer may be NULL. */
raft_status raft_graph_size(const raft_graph* g, int64_t* n, int64_t* nnz);
/* Device-to-device copy of the library's CSR: row_ptr int32 [N + 1],
 * col_idx int32 [nnz] (sorted rows), asynchronous on `stream`. */
raft_status raft_graph_csr(const raft_graph* g, int32_t* row_ptr, int32_t* col_idx, void* stream);

/* ---- streaming graphs (Sec. III-D) ------------------------------------------ */

/* A stream holds a graph and every level of its embedding (Theta, Y_1..Y_q,
 * the input of layer 1 and the GCN layer outputs, all in library-owned device
 * memory, about (q + n_layers + 4) x N x max width floats) and updates them
 * when edges arrive.  New edges change the degrees of their endpoints V'
 * only; under the NCut operator M (Eq. 2) and the GCN operator (Eq. 6) an
 * entry depends on its two endpoints' degrees, so level t of Y = X^q Theta
 * can change only within t hops of V' and GCN layer k within q + k hops (the
 * multi-hop neighbourhood V'' of the section).  raft_stream_add_edges
 * recomputes each level on that ball only, with the row kernels of a full
 * pass, so the result equals raft_project + raft_embed on the new graph bit
 * for bit.  Under the modularity operators (Eq. 4, Q~) every entry carries
 * 1/2e, which any new edge changes: there every level is recomputed in full.
 * Model selection (raft_partition, raft_hier_partition) runs on the stream's
 * current graph and embedding; it is not incremental.
 *
 * raft_stream_create: copies g, computes every level with cfg (op, proj_dim,
 * q, layers, normalize_input, seed; the candidate grid is checked as for
 * raft_run but not used); q + n_layers <= 64.  Synchronous. */
typedef struct raft_stream raft_stream;
raft_status raft_stream_create(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                               void* stream, raft_stream** out);
void        raft_stream_destroy(raft_stream* s);
/* Adds the m undirected edges (src[e], dst[e]) (host int32 arrays, either
 * order).  RAFT_E_INVAL on an endpoint out of range, a self pair or an edge
 * given twice, RAFT_E_CSR on an edge already in the graph: in both cases
 * nothing changes.  rows_per_level (nullable, q + n_layers entries) receives
 * the number of rows within each level's hop ball (N everywhere for the
 * modularity operators); a level whose ball holds more than half of the rows
 * is run over all rows (rows outside the ball recompute to their previous
 * values).  The stream keeps two graph buffers and alternates between them,
 * so a handle from raft_stream_graph must be fetched again after each update.
 * Synchronous.  After RAFT_E_DEVICE the stream must be destroyed. */
raft_status raft_stream_add_edges(raft_stream* s, const int32_t* src, const int32_t* dst,
                                  int64_t m, void* stream, int64_t* rows_per_level);
/* The current graph (owned by the stream, never passed to
 * raft_graph_destroy; valid until the next raft_stream_add_edges or
 * raft_stream_destroy). */
raft_status raft_stream_graph(const raft_stream* s, const raft_graph** g);
/* Device copies of the current Y = X^q Theta [N x L] and Z [N x d] (either
 * pointer may be NULL), asynchronous on `stream`. */
raft_status raft_stream_embedding(const raft_stream* s, float* Y, float* Z, void* stream);

/* ---- graph sampling (Sec. IV, Alg. 2: fast degree-corrected SBM) --------- */

/* Samples an undirected graph from the degree-corrected SBM (Sec. II, SBM
 * definition): i and j are joined with probability 1 - exp(-lambda_ij),
 * lambda_ij = theta_i theta_j Omega_{c_i c_j}, independently over the pairs
 * i < j.  Alg. 2's jump: the possible edges between blocks r <= s form a
 * |C_r| x |C_s| table (C_r = the nodes of block r in increasing id); each row
 * x of it (node C_r[x] against C_s; for r = s only columns y > x) is one
 * device thread that jumps from one sampled entry to the next: from column m
 * it draws E = -ln u, u the first word of Philox4x64-10 with key (seed, 0x30)
 * and counter (r K + s, x, jump number, 0) as a 52-bit uniform in (0, 1),
 * stops when E >= lambda_row (P_s[|C_s|] - P_s[m]), and otherwise takes the
 * smallest t >= m with lambda_row (P_s[t + 1] - P_s[m]) > E (binary search;
 * P_s = the FP64 theta prefix of block s accumulated left to right,
 * lambda_row = Omega_rs theta_{C_r[x]}).  FP64 throughout; the result is a
 * function of (theta, blocks, omega, seed) alone, bit for bit.
 *   theta  [n] host FP64, finite, >= 0;  blocks [n] host int32 in 0..k-1;
 *   omega  [k x k] host FP64 row-major, symmetric, finite, >= 0;
 *   1 <= k <= 4096, 1 <= n < 2^31 - 1.
 * *out receives a graph handle as from raft_graph_create (validated; the
 * sampled nnz = 2|E| must stay below 2^31 - 1, else RAFT_E_UNSUPPORTED).
 * Device memory: O(n + k^2 + number of table rows + |E|) temporaries, freed
 * before return.  Synchronous. */
raft_status raft_sbm_sample(raft_ctx* ctx, int64_t n, int32_t k, const double* theta,
                            const int32_t* blocks, const double* omega, uint64_t seed,
                            void* stream, raft_graph** out);

/* ---- workspace ----------------------------------------------------------- */

/* Bytes of device workspace raft_project / raft_embed / raft_partition /
 * raft_run need for this graph and config (256-byte aligned base). */
raft_status raft_workspace_size(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                                size_t* bytes);

/* ---- stage A1: seeded Gaussian matrices (Sec. III-A Eq. 5, Sec. III-B) ---- */

/* out[rows x cols] = FP32(sigma * N(0,1)) drawn from Philox4x64-10 with key
 * (seed, stream_id), counter (row, col/4, 0, 0): each counter gives four
 * Box-Muller normals for columns 4*(col/4)..+3.  Theta uses stream 0x10 and
 * sigma = L^-1/2; GCN layer k (1-based) uses 0x10 + k and sigma = L_{k-1}^-1/2. */
raft_status raft_gaussian(raft_ctx* ctx, uint64_t seed, uint64_t stream_id, int64_t rows,
                          int64_t cols, double sigma, float* out, void* stream);

/* ---- stages A2/A3: one sparse step and the projection -------------------- */

/* Workspace bytes raft_spmm needs for (op, L): the FP64 column-sum
 * partials of MOD_FULL's rank-1 term; 0 for the other operators. */
raft_status raft_spmm_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                                    size_t* bytes);

/* Y_out = X Y_in for one operator X (RAFT_X_*), Y_in/Y_out [N x L] row-major,
 * distinct buffers.  MOD_FULL needs workspace for the column sums d^T Y_in
 * (raft_spmm_workspace_size); the other operators take ws = NULL.  */
raft_status raft_spmm(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                      const float* Y_in, float* Y_out, void* ws, size_t ws_bytes, void* stream);

/* raft_spmm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, bit for bit, with MOD_FULL's column-sum partials
 * kept in a fixed scratch array of 16 MiB that the library holds on each GPU
 * it runs on until the process ends.  Nothing is allocated or freed.  The
 * caller passes inputs and outputs as for raft_spmm.  MOD_FULL needs
 * raft_spmm_workspace_size(...) <= 16 MiB (about 2 million rows at L = 256,
 * 8 million at L = 64), else RAFT_E_WORKSPACE with a message.  Every call on
 * one GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (two streams, two host threads) race and must be serialised by the caller. */
raft_status raft_spmm_noalloc(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                              const float* Y_in, float* Y_out, void* stream);

/* raft_spmm with the work split by the merge path of the CSR (Merrill and
 * Garland 2016) instead of by rows: the N row ends and nnz stored entries
 * are cut into equal ranges of 256 path items, whatever the row lengths, so
 * heavy-tailed degrees cost no imbalance; rows cut by a range boundary are
 * finished by a fix-up pass that adds their pieces in range order
 * (deterministic).  Same operators and layouts as raft_spmm; results equal
 * raft_spmm's up to FP32 summation order.  Workspace: the range partials
 * (raft_spmm_merge_workspace_size), plus the column sums for MOD_FULL. */
raft_status raft_spmm_merge_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t op,
                                           int32_t L, size_t* bytes);
raft_status raft_spmm_merge(raft_ctx* ctx, const raft_graph* g, int32_t op, int32_t L,
                            const float* Y_in, float* Y_out, void* ws, size_t ws_bytes,
                            void* stream);

/* Y = X^q Theta (Sec. III-A, Eq. 5 with q powers), Theta drawn as in
 * raft_gaussian with cfg->seed.  Y_out [N x L]. */
raft_status raft_project(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                         void* ws, size_t ws_bytes, float* Y_out, void* stream);

/* ---- stage A4: random GCN (Sec. III-B, Eq. 6) ----------------------------- */

/* One layer: H_out = rownorm(tanh((A_hat_n H_in) W)), W [L_in x L_out]
 * row-major (device).  With `linear` != 0 the tanh and the normalisation are
 * skipped (U = A_hat_n H_in W).  P_out (nullable, [N x L_in]) receives
 * A_hat_n H_in. */
raft_status raft_gcn_layer(raft_ctx* ctx, const raft_graph* g, int32_t L_in, int32_t L_out,
                           const float* H_in, const float* W, int32_t linear, float* H_out,
                           float* P_out, void* ws, size_t ws_bytes, void* stream);

/* Z = GCN(Y) with W^(k) drawn as in raft_gaussian (seed cfg->seed). */
raft_status raft_embed(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                       const float* Y, void* ws, size_t ws_bytes, float* Z_out, void* stream);

/* ---- stages A5-A7: model selection --------------------------------------- */

/* k-means for every candidate K of the grid (nested k-means++ exponential
 * race, Lloyd to a fixed point or T_max), scores per candidate, selection of
 * K* by modularity.  Z [N x d], d = last layer width (or L when n_layers = 0).
 * Polls convergence from the host every cfg->check_every iterations, so the
 * call synchronises `stream`. */
raft_status raft_partition(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                           const float* Z, void* ws, size_t ws_bytes, raft_outputs* out,
                           void* stream);

/* Stage A7 alone: Mod (Eq. 3) and NCut (Eq. 1) of Kc labelings given as
 * point-major bytes labels_all[N x Kc]; ks[Kc] (host) are the block counts.
 * mod/ncut are device arrays [Kc].  At most 256 labelings with a sum of
 * block counts of at most 16384 (RAFT_E_UNSUPPORTED beyond); a label not
 * below its labeling's K is not counted and latches a status that
 * raft_sync_status returns as RAFT_E_INVAL. */
raft_status raft_score(raft_ctx* ctx, const raft_graph* g, const uint8_t* labels_all,
                       int32_t Kc, const int32_t* ks, double* mod, double* ncut,
                       void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes raft_score needs for Kc labelings with block counts
 * ks[Kc] (host array). */
raft_status raft_score_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t Kc,
                                     const int32_t* ks, size_t* bytes);

/* ---- comparison of partitions (normalised mutual information) ----------- */

/* Contingency counts of two labelings of the same n nodes: counts[r*kb + c]
 * (device int64 [ka x kb], overwritten) = #{i : a[i] = r, b[i] = c}.  a, b
 * are device int32 [n] with labels in [0, ka) and [0, kb); a label out of
 * range is not counted and latches a status that raft_sync_status returns as
 * RAFT_E_INVAL.  Integer counts, exact and independent of scheduling. */
raft_status raft_confusion(raft_ctx* ctx, const int32_t* a, const int32_t* b, int64_t n,
                           int32_t ka, int32_t kb, int64_t* counts, void* stream);
/* Host-side finish: NMI = 2 I(a;b) / (H(a) + H(b)) in natural log from a
 * HOST copy of the counts (1 when both entropies are 0). */
raft_status raft_nmi_from_counts(const int64_t* counts, int32_t ka, int32_t kb, double* nmi);

/* A1-A7: projection, embedding and model selection (synchronises `stream`). */
raft_status raft_run(raft_ctx* ctx, const raft_graph* g, const raft_config* cfg,
                     void* ws, size_t ws_bytes, raft_outputs* out, void* stream);

/* ---- batches of graphs ---------------------------------------------------
 * Many graphs of uneven size through the whole path (A1-A7, as raft_run) at
 * once.  raft_batch_create packs the graphs into one block-diagonal CSR on
 * the device (graph g's rows after those of graphs 0..g-1, its column ids and
 * stored entries shifted to match; a library-owned copy, so the graph handles
 * may be destroyed afterwards).  Every stage then runs as one launch over all
 * graphs and all candidate K of the grid, each graph's work-groups doing what
 * its own launch would; the fixed launch sequence before the Lloyd loop
 * (projection, GCN, k-means++ race) is recorded once into a HIP graph per
 * workspace and replayed.  All graphs share `cfg` (operator, widths, q,
 * candidate grid, T_max); graph g draws Theta, W and the race with seeds[g]
 * (cfg->seed when seeds is NULL).  Graph g's outputs are those of raft_run on
 * graph g with cfg->seed = seeds[g], bit for bit.  Errors: RAFT_E_NOEDGES for
 * a graph without edges, RAFT_E_INVAL when k_max exceeds a graph's N,
 * RAFT_E_UNSUPPORTED when the packed CSR exceeds int32 indices. */
typedef struct raft_batch raft_batch;
raft_status raft_batch_create(raft_ctx* ctx, int32_t G, const raft_graph* const* graphs,
                              const uint64_t* seeds, const raft_config* cfg, raft_batch** out);
void        raft_batch_destroy(raft_batch* b);
/* Workspace bytes of raft_batch_run (caller-owned device memory, 256-byte
 * aligned).  The HIP graph recorded for a workspace stays valid while the
 * same workspace pointer is passed. */
raft_status raft_batch_workspace_size(raft_ctx* ctx, const raft_batch* b, size_t* bytes);
/* per_graph[G]: the outputs of each graph as for raft_run (any field
 * nullable).  Polls convergence from the host and synchronises `stream`. */
raft_status raft_batch_run(raft_ctx* ctx, raft_batch* b, void* ws, size_t ws_bytes,
                           raft_outputs* per_graph, void* stream);
/* enable = 0 launches the prefix directly instead of replaying the HIP graph
 * (same results; default 1). */
raft_status raft_batch_set_capture(raft_batch* b, int32_t enable);
/* Host-only check of the batch planner (no device needed): lays out a batch
 * of G graphs with n[g] rows and nnz[g] stored entries for `cfg` on a device
 * with num_cu compute units, at stand-in addresses, and verifies that every
 * array each graph's kernels index lies inside that graph's part of the
 * workspace, the control block or the packed features, and that every launch
 * table gives each graph its work-groups.  RAFT_OK or an error with the
 * reason in msg.  raft_batch_run runs the same check on its real layout. */
raft_status raft_batch_plan_check(int32_t G, const int32_t* n, const int64_t* nnz,
                                  const raft_config* cfg, int32_t num_cu, char* msg,
                                  size_t msg_len);
/* The batch's launch-shape tuner.  The edge-score and k-means++ race grids
 * and the update's point ranges of each graph are sized for a share of the
 * chip (its node count over the batch's, times a factor); these shapes never
 * change a result (integer counts and sums, a lexicographic argmin).  On the
 * first raft_batch_run of a workload not in the context's tuner cache, the
 * batch runs once per candidate factor (after one warm-up run) and keeps the
 * fastest by GPU time; the choice is kept per workload key in the context
 * and written to the context's autotune_cache file when one was given.
 * factor receives the choice (0 = the single-graph shapes); ms[2 i], ms[2 i +
 * 1] the i-th candidate and its time in ms (up to cap candidates); count the
 * number of candidates timed by this batch (0 when the cache held the key). */
raft_status raft_batch_tuning(const raft_batch* b, int32_t* factor, double* ms, int32_t cap,
                              int32_t* count);
/* GPU time of the last raft_batch_run: [0] projection + GCN + seeding,
 * [1] Lloyd, [2] scores and outputs (ms). */
raft_status raft_batch_stage_times(const raft_batch* b, double* ms3);

/* ---- hierarchical model selection (Sec. III-C, Alg. 1) --------------------
 * Partitions the embedding Z [N x d] (device) of graph g by Alg. 1: a set U
 * (the root is V) with local modularity m_1 = LMod(U; G) (Eq. 7) is split by
 * KMeans with K = 2 into (U_1, U_2) with m_2 = LMod(U_1, U_2; G); U becomes a
 * block when |U_1| <= eps or |U_2| <= eps or m_1 > m_2, otherwise U_1 and U_2
 * are partitioned the same way.  Readings: a set of at most 2 eps + 1 nodes
 * is a block without KMeans (one side would have at most eps nodes); a set
 * with zero G-volume is a block (Eq. 7 is undefined); KMeans K = 2 is
 * k-means++ by the exponential race with draws -ln u of Philox4x64-10 key
 * (seed, 0x21), counter (node id, pick, depth, 0), then Lloyd to a fixed point
 * or t_max assignments, ties to U_1 (the side of the first pick); blocks are
 * numbered in the order Alg. 1 adds them (depth first, U_1 before U_2).
 * All sets of one depth are split at once on the GPU; LMod is finished in
 * FP64 on the host from exact integer counts, in the order r = 1, 2. */
typedef struct {
    int32_t eps;          /* stopping threshold (the paper uses 5)                   */
    int32_t t_max;        /* Lloyd assignments per split (>= 1)                       */
    uint64_t seed;        /* Philox key word 0 of the race                            */
} raft_hier_config;
typedef struct {
    int32_t depth;        /* level of the set (root 0)                                */
    int32_t size;         /* |U|                                                      */
    int32_t parent;       /* tree node of the parent set (-1 for the root)            */
    int32_t child[2];     /* tree nodes of U_1, U_2 (-1 when U is a block)            */
    int32_t block;        /* block number when U is a block, else -1                  */
    int32_t kmeans_iters; /* Lloyd assignments of the split (0: no KMeans ran)        */
    int32_t sizes[2];     /* |U_1|, |U_2| of the KMeans split (0 when none ran)       */
    double m1, m2;        /* LMod(U; G), LMod(U_1, U_2; G) (NaN when not computed)    */
} raft_hier_node;
/* Workspace bytes of raft_hier_partition for graph g and embedding width d. */
raft_status raft_hier_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t d,
                                     size_t* bytes);
/* labels [N] (device) receive block numbers; *n_blocks the number of blocks.
 * tree (host, nullable, tree_cap records) receives the visited sets in tree
 * node order (the root first, then level by level), *n_tree their number.
 * node_trace (device, nullable, [trace_depth x N] int32) receives for each
 * depth < trace_depth and node 2 t + a, t the tree node of the node's set at
 * that depth and a its side in that set's KMeans split (0 when none ran), or
 * -1 once the node is in a block of a smaller depth.  Synchronises `stream`. */
raft_status raft_hier_partition(raft_ctx* ctx, const raft_graph* g, const float* Z, int32_t d,
                                const raft_hier_config* cfg, void* ws, size_t ws_bytes,
                                int32_t* labels, int32_t* n_blocks, raft_hier_node* tree,
                                int32_t tree_cap, int32_t* n_tree, int32_t* node_trace,
                                int32_t trace_depth, void* stream);

/* ---- training the GCN weights (optional; the method itself keeps them random) ----
 * Relaxed modularity: with hard memberships H, tr(H^T B H)/2e is the
 * modularity of Eq. 3 (matrix form Eq. 4); replacing H by row-softmax
 * assignments S gives the loss -tr(S^T B S)/2e.  The model is the GCN of
 * Eq. 6 with trainable W^(k): hidden layers tanh + row normalisation, the
 * last layer linear (its output U are the logits of S).
 * Widths dims[0..n_layers] each in {16, 32, 64, 128}, dims[k]*dims[k+1] <=
 * 8192.  W[k] are device pointers to [dims[k] x dims[k+1]] row-major.
 * Buffers are device memory owned by the caller; pointer arrays are host
 * arrays of device pointers. */

/* Workspace bytes for raft_gcn_forward/backward and raft_modloss_* with
 * logits width K. */
raft_status raft_train_workspace_size(raft_ctx* ctx, const raft_graph* g, int32_t n_layers,
                                      const int32_t* dims, int32_t K, size_t* bytes);
/* U_out [N x dims[n_layers]] = logits; H_saved[k] (k = 0..n_layers-2)
 * receive the output of hidden layer k+1, i.e. the input of layer k+2, kept
 * for the backward pass (pre-activations are recomputed there). */
raft_status raft_gcn_forward(raft_ctx* ctx, const raft_graph* g, int32_t n_layers,
                             const int32_t* dims, const float* H0, const float* const* W,
                             float* const* H_saved, float* U_out, void* ws, size_t ws_bytes,
                             void* stream);
/* Adjoint of raft_gcn_forward: G_W[k] = dL/dW^(k) from G_U = dL/dU; G_H0
 * (nullable) = dL/dH0.  Recomputes A_hat_n H and the pre-activations. */
raft_status raft_gcn_backward(raft_ctx* ctx, const raft_graph* g, int32_t n_layers,
                              const int32_t* dims, const float* H0, const float* const* W,
                              const float* const* H_saved, const float* G_U, float* const* G_W,
                              float* G_H0, void* ws, size_t ws_bytes, void* stream);
/* S_out = softmax_rows(U) [N x K]; *loss (device double) = -tr(S^T B S)/2e. */
raft_status raft_modloss_forward(raft_ctx* ctx, const raft_graph* g, const float* U, int32_t K,
                                 float* S_out, double* loss, void* ws, size_t ws_bytes,
                                 void* stream);
/* G_U = scale * dloss/dU for S = softmax(U) (B S recomputed from S);
 * scale: device float (nullable = 1). */
raft_status raft_modloss_backward(raft_ctx* ctx, const raft_graph* g, const float* S, int32_t K,
                                  const float* scale, float* G_U, void* ws, size_t ws_bytes,
                                  void* stream);
/* One Adam step (Kingma & Ba) on n parameters; step counts from 1. */
raft_status raft_adam_step(raft_ctx* ctx, float* w, float* m, float* v, const float* grad,
                           int64_t n, float lr, float beta1, float beta2, float eps, int32_t step,
                           void* stream);

/* ---- measurement ---------------------------------------------------------- */

/* Kernel classes timed by raft_profile_enable (bit k of the mask = class k). */
#define RAFT_PROF_SPMM    0   /* sparse products of the projection and GCN aggregation */
#define RAFT_PROF_DENSE   1   /* GCN dense layer (MFMA)                               */
#define RAFT_PROF_RACE    2   /* k-means++ race pick                                  */
#define RAFT_PROF_ASSIGN  3   /* k-means assignment over all candidates (MFMA)        */
#define RAFT_PROF_UPDATE  4   /* k-means centre update                                */
#define RAFT_PROF_SCORE   5   /* per-edge candidate scores                            */
#define RAFT_PROF_CLASSES 6

/* Brackets every later launch of the enabled kernel classes with HIP events
 * on the launch stream (mask 0 disables).  Synchronises the device. */
raft_status raft_profile_enable(raft_ctx* ctx, uint32_t mask);
/* Accumulated device milliseconds and launch counts per class since the last
 * read (ms[RAFT_PROF_CLASSES], launches[RAFT_PROF_CLASSES]); resets them.
 * Synchronises the device. */
raft_status raft_profile_read(raft_ctx* ctx, double* ms, int64_t* launches);

/* Per-stage device times (ms) of the last raft_run on this context:
 * [0] project, [1] embed, [2] seeding, [3] Lloyd, [4] scores+select. */
raft_status raft_get_stage_times(raft_ctx* ctx, double* ms5);

#ifdef __cplusplus
}
#endif
#endif /* RAFTGP_H */
