/*
 * sbp.h -- C-ABI of the MI355X (gfx950) stochastic block partitioning library.
 *
 * The library computes, on one GPU, the hot path of stochastic block
 * partitioning (SBP) on the degree-corrected stochastic blockmodel as framed
 * by Wanye et al., "Exact Distributed Stochastic Block Partitioning"
 * (arXiv 2305.18663):
 *   - the blockmodel matrix M and block degrees ............ Sec. II-A
 *   - the description length DL ............................ Eq. 1, Eq. 2
 *   - Metropolis-Hastings vertex moves in asynchronous-Gibbs
 *     batches (the MCMC phase) ............................. Alg. 2, Sec. II-B, Alg. 5
 *   - block merge scoring and application .................. Alg. 1, Alg. 4
 *   - the whole method with its golden-ratio search ........ Sec. II-B
 *
 * Problem statement (Sec. I, Eq. 2): given a directed graph G, find a block
 * count C and an assignment b of vertices to blocks minimising DL.
 *
 * Conventions
 *   - Every pointer is a DEVICE pointer unless marked [host].
 *   - Calls enqueue work on `stream` (a hipStream_t passed as void*, NULL =
 *     the default stream) and return before the work completes, unless
 *     marked SYNC.
 *   - The library never allocates device memory.  Callers provide blockmodel
 *     storage and workspace sized by the *_bytes queries; every region must
 *     be 256-byte aligned.
 *   - Return value: SBP_OK (0) or a negative SBP_E_* code; the thread-local
 *     message of the last failure is returned by sbp_last_error().
 *   - Every output is a pure function of the inputs (graph, assignment,
 *     block count, parameters including the seed).  It does not depend on the
 *     stream, on other work on the device, or on which other graphs share a
 *     batched launch.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC 2011), key = seed
 *     (low word, high word), counters given per call below; four 64-bit
 *     words W0..W3 come from two blocks (a, b, base, tag), (a, b, base+1, tag)
 *     with W0 = out0 | out1<<32, W1 = out2 | out3<<32 of the first block,
 *     W2, W3 likewise of the second.  An index in [0, n) is floor(W n / 2^64).
 */
#ifndef SBP_H
#define SBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBP_OK 0
#define SBP_E_ARG (-1)    /* null pointer, n < 1, C < 1, C > n, bad parameter */
#define SBP_E_GRAPH (-2)  /* malformed CSR/CSC (from sbp_validate_graph)      */
#define SBP_E_LABEL (-3)  /* assignment outside [0, C)                        */
#define SBP_E_SPACE (-4)  /* blockmodel or workspace too small / full engine  */
#define SBP_E_HIP (-5)    /* a HIP runtime call failed                        */
#define SBP_E_LIMIT (-6)  /* size beyond the library limits below             */

/* Limits: e < 2^30, n < 2^30, and no vertex with more than SBP_MAX_DEGREE
 * edge ends (out + in). */
#define SBP_MAX_DEGREE 16384
/* Block counts up to this value use the dense blockmodel tier. */
#define SBP_DENSE_MAX_C 64

/* A directed graph (Sec. II-A: V vertices, E directed edges): CSR of the
 * out-edges and CSC of the in-edges of the same edge multiset, neighbour ids
 * ascending within each row, multi-edges repeated, self-loops allowed.
 * All arrays are int32 device arrays owned by the caller. */
typedef struct sbp_graph {
    int32_t n;               /* vertices */
    int32_t e;               /* directed edges */
    const int32_t *out_ptr;  /* [n+1] */
    const int32_t *out_idx;  /* [e] targets of out-edges */
    const int32_t *in_ptr;   /* [n+1] */
    const int32_t *in_idx;   /* [e] sources of in-edges */
} sbp_graph;

/* One sweep of vertex moves (Alg. 2).  Vertex v draws words from counter
 * (v, sweep, 0, 0).  Batch j = {v : v mod n_batches = j}; each batch is
 * evaluated against the blockmodel at its start and its accepted moves are
 * then applied (n_batches = 1: all vertices against one snapshot;
 * n_batches = n: sequential Alg. 2). */
typedef struct sbp_sweep_params {
    uint64_t seed;
    uint32_t sweep;     /* sweep index used in the random-number counter */
    int32_t n_batches;  /* >= 1; values above n are clamped to n */
    double beta;        /* inverse temperature of the acceptance test (> 0) */
    int32_t eps;        /* proposal mixing weight (>= 0), integer */
    int32_t n_hubs;     /* hybrid sweep (Sec. II-B): the n_hubs vertices of highest
                         * degree (out + in edge ends, ties by smaller id) first
                         * move one at a time in that order, each evaluated
                         * against the state the previous ones left, then the
                         * others in the n_batches snapshot batches.  0 = all
                         * asynchronous; 0..min(n, 4096), else SBP_E_ARG.  The
                         * dense tier runs the hubs in one workgroup; the
                         * sparse tier (C > 64) takes each hub as a batch of its
                         * own with a blockmodel rebuild in between (slow: about
                         * one rebuild per hub). */
} sbp_sweep_params;

/* Sweep totals, written to device memory. */
typedef struct sbp_sweep_stats {
    int64_t proposals;       /* vertices evaluated */
    int64_t self_proposals;  /* proposals of the vertex's own block (no-ops) */
    int64_t accepted;
    int64_t near_ties;       /* proposals (not no-ops) whose margin (see the
                              * trace) is within 1e-9 of zero: decisions a
                              * differently ordered FP64 sum could flip */
    double sum_dS_accepted;  /* sum of DL changes of accepted moves */
    double dl_after;         /* DL of the assignment after the sweep */
} sbp_sweep_stats;

/* Optional per-vertex trace of a sweep; each pointer may be NULL. */
typedef struct sbp_sweep_trace {
    int32_t *prop;    /* [n] proposed block */
    double *dS;       /* [n] DL change of the proposed move (0 for no-ops) */
    double *lnH;      /* [n] log Hastings ratio ln q(s->r) - ln q(r->s) */
    double *margin;   /* [n] (-beta dS + lnH) - ln u; accepted iff > 0 */
    int8_t *accept;   /* [n] 1 if the move was applied */
} sbp_sweep_trace;

/* Block merge scoring (Alg. 1).  Block c draws words from counter
 * (c, phase, 2j, 1) for proposal j < proposals. */
typedef struct sbp_merge_params {
    uint64_t seed;
    uint32_t phase;
    int32_t proposals;  /* x of Alg. 1, >= 1 */
    int32_t eps;
    int32_t reserved;
} sbp_merge_params;

/* The whole method (Sec. II-B). */
typedef struct sbp_partition_params {
    uint64_t seed;
    double beta;
    int32_t eps;
    int32_t merge_proposals;  /* x of Alg. 1 */
    int32_t max_sweeps;       /* x of Alg. 2 */
    int32_t n_batches;        /* batches per sweep */
    double t_pre;             /* MCMC stop tolerance before the golden bracket exists */
    double t_post;            /* ... and after */
    double merge_rate;        /* fraction of blocks merged before the bracket exists */
    int32_t max_iters;        /* cap on merge+MCMC iterations */
    int32_t n_hubs;           /* hybrid sweeps: the n_hubs highest-degree vertices move one at a time
                                 first in every sweep (as sbp_sweep_params.n_hubs; clamped to n) */
} sbp_partition_params;

/* ------------------------------------------------------------------ */
/* Size queries (host)                                                 */
/* ------------------------------------------------------------------ */
enum { SBP_OP_VALIDATE = 0, SBP_OP_BUILD = 1, SBP_OP_SWEEP = 2, SBP_OP_MERGE = 3 };

/* Bytes of blockmodel storage for a graph with n vertices, e edges and C
 * blocks.  C <= SBP_DENSE_MAX_C selects the dense tier, else the sparse one. */
size_t sbp_blockmodel_bytes(int32_t n, int32_t e, int32_t C);
/* Bytes of workspace for one of the SBP_OP_* calls. */
size_t sbp_workspace_bytes(int32_t op, int32_t n, int32_t e, int32_t C);

/* ------------------------------------------------------------------ */
/* Graph ingest and check (SYNC)                                       */
/* ------------------------------------------------------------------ */
/* Builds the graph arrays of sbp_graph from a list of e directed edges
 * (src[i] -> dst[i], device arrays, multi-edges and self-loops allowed):
 * out_ptr[n+1]/out_idx[e] sorted by (source, target) and in_ptr[n+1]/
 * in_idx[e] sorted by (target, source), all caller-owned device arrays
 * (Sec. II-A: the directed graph of V vertices and E edges).  Returns
 * SBP_E_GRAPH if an endpoint lies outside [0, n), SBP_E_SPACE if the
 * workspace (sbp_graph_workspace_bytes) is too small. */
size_t sbp_graph_workspace_bytes(int32_t n, int32_t e);
int sbp_graph_from_edges(int32_t n, int32_t e, const int32_t *src, const int32_t *dst, int32_t *out_ptr,
                         int32_t *out_idx, int32_t *in_ptr, int32_t *in_idx, void *ws, size_t ws_bytes,
                         void *stream);

/* Checks monotone pointers, ptr[0] = 0, ptr[n] = e, ids in [0, n), equal
 * edge counts, and the degree limit.  Returns SBP_OK or SBP_E_GRAPH/LIMIT. */
int sbp_validate_graph(const sbp_graph *g /*[host]*/, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Blockmodel (Sec. II-A; Eq. 1)                                       */
/* ------------------------------------------------------------------ */
/* Builds M (M_ab = number of edges from block a to block b), the block
 * degrees d_a^out = sum_b M_ab, d_b^in = sum_a M_ab, and the proposal tables
 * into `bm` for assignment `assign` [n] with labels in [0, C).
 * Errors: SBP_E_ARG, SBP_E_SPACE (bm_bytes or ws_bytes too small),
 * SBP_E_LIMIT.  Labels are not range-checked here (sbp_check_labels). */
int sbp_build_blockmodel(const sbp_graph *g /*[host]*/, const int32_t *assign, int32_t C,
                         void *bm, size_t bm_bytes, void *ws, size_t ws_bytes, void *stream);

/* SYNC.  SBP_OK if every label lies in [0, C), else SBP_E_LABEL. */
int sbp_check_labels(int32_t n, const int32_t *assign, int32_t C, void *ws, size_t ws_bytes, void *stream);

/* Reads the blockmodel of (g, C) back as sorted coordinates (rows, cols,
 * vals) plus degrees.  Outputs are device arrays of capacity max(e, C*C)
 * (entries) and C (degrees); *nnz [host] receives the entry count.  SYNC. */
int sbp_blockmodel_coo(const sbp_graph *g /*[host]*/, int32_t C, const void *bm, int32_t *rows, int32_t *cols,
                       int32_t *vals, int32_t *dout, int32_t *din, int64_t *nnz /*[host]*/, void *stream);

/* ------------------------------------------------------------------ */
/* Description length (Eq. 1, Eq. 2)                                   */
/* ------------------------------------------------------------------ */
/* DL = E h(C^2/E) + N ln C - L(G|B), natural log, written as
 * f(E+C^2) - f(E) - f(C^2) + N ln C - [sum f(M_ab) - sum f(d_a^out) - sum f(d_b^in)]
 * with f(x) = x ln x, f(0) = 0, and C the label count of the blockmodel.
 * The value is computed (fixed reduction order) whenever the blockmodel is
 * built or updated by a sweep; this call writes it to dl (one device double). */
int sbp_description_length(const sbp_graph *g /*[host]*/, int32_t C, const void *bm, double *dl, void *stream);

/* ------------------------------------------------------------------ */
/* MCMC sweep (Alg. 2 in asynchronous-Gibbs batches)                   */
/* ------------------------------------------------------------------ */
/* One sweep over all vertices.  For vertex v in block r: with k its edge
 * ends (out-edges in CSR order, then in-edges in CSC order), if k = 0 the
 * proposal is s = idx(W2, C); otherwise the end j = idx(W0, k) gives the
 * neighbour block t, and s = idx(W2, C) if idx(W1, d_t + eps C) < eps C,
 * else the smallest s whose running sum of e_ts (e = M + M^T) in ascending
 * s exceeds idx(W2, d_t), d_t = d_t^out + d_t^in.  s = r is a no-op.  The
 * move is scored by its exact DL change dS over the changed entries of M
 * and the block degrees, and accepted iff
 *   ln u < -beta dS + ln H,  u = ((W3 >> 11) + 0.5) 2^-53,
 * where H = q(s->r)/q(r->s) and q(r->s) = sum_t (k_t/k)(e_ts + eps)/(d_t + eps C)
 * (the reverse law evaluated after the move).
 * `assign` [n] (in/out) and `bm` (in/out, built for `assign` and C) are
 * updated to the state after the sweep; `stats` (device, nullable) receives
 * totals; `trace` [host] (nullable) points at optional per-vertex arrays.
 * Errors: SBP_E_ARG, SBP_E_SPACE. */
int sbp_nodal_sweep(const sbp_graph *g /*[host]*/, int32_t *assign, int32_t C, void *bm, size_t bm_bytes,
                    const sbp_sweep_params *p /*[host]*/, sbp_sweep_stats *stats,
                    const sbp_sweep_trace *trace /*[host]*/, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free variant of sbp_nodal_sweep, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * semantics and results as sbp_nodal_sweep without ws/ws_bytes; its
 * scratch (the per-vertex decisions and per-workgroup partials) is a
 * file-scope device array of the library, about 4.2 MB on every GPU it runs
 * on, held until the process ends.  Limits: dense tier only (C <=
 * SBP_DENSE_MAX_C, else SBP_E_ARG), n_hubs = 0 (else SBP_E_ARG), n <=
 * SBP_STATIC_MAX_VERTICES (else SBP_E_LIMIT); every check happens before any
 * work is enqueued.  It calls no allocating routine.  All calls on one GPU
 * share the array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
#define SBP_STATIC_MAX_VERTICES (1 << 20)
int sbp_nodal_sweep_static(const sbp_graph *g /*[host]*/, int32_t *assign, int32_t C, void *bm, size_t bm_bytes,
                           const sbp_sweep_params *p /*[host]*/, sbp_sweep_stats *stats,
                           const sbp_sweep_trace *trace /*[host]*/, void *stream);

/* Replayable sweep (Alg. 2 batches captured once as a HIP graph).
 * sbp_sweep_graph_create records one sweep of sbp_nodal_sweep with the
 * given arguments (no trace) and instantiates it; nothing runs on the GPU.
 * Each sbp_sweep_graph_launch then runs exactly that sweep on `stream`,
 * except that the sweep index of the random stream is read from
 * *sweep_index (one device uint32, set by the caller before the first
 * launch) and the launch adds one to it when the sweep ends, so k launches
 * equal k calls of sbp_nodal_sweep with sweep = s, s+1, ..., s+k-1 (same
 * assign/bm/stats results, bit for bit).  `stats` (device) is required and
 * rewritten by every launch.  The graph holds the addresses of g's arrays,
 * assign, bm, sweep_index, stats and ws: they must stay allocated and
 * unmoved, and the graph is used with the same C, until destroy.  Launches
 * are ordered on their stream like kernels; launches of one graph on
 * different streams, or of graphs sharing ws, race unless the caller orders
 * them.  Limits: dense tier only (C <= SBP_DENSE_MAX_C, else SBP_E_ARG).
 * The library allocates no device memory for the graph.  Errors: SBP_E_ARG,
 * SBP_E_SPACE, SBP_E_HIP (capture or instantiation failed; *out = NULL). */
typedef struct sbp_sweep_graph sbp_sweep_graph;
int sbp_sweep_graph_create(const sbp_graph *g /*[host]*/, int32_t *assign, int32_t C, void *bm, size_t bm_bytes,
                           const sbp_sweep_params *p /*[host]*/, uint32_t *sweep_index, sbp_sweep_stats *stats,
                           void *ws, size_t ws_bytes, sbp_sweep_graph **out /*[host]*/);
/* ASYNC on stream.  SBP_E_ARG for a NULL handle or a device other than the
 * one current at creation. */
int sbp_sweep_graph_launch(sbp_sweep_graph *graph, void *stream);
/* Frees the graph (the caller orders this after its last launch ends). */
int sbp_sweep_graph_destroy(sbp_sweep_graph *graph);

/* ------------------------------------------------------------------ */
/* Block merges (Alg. 1)                                               */
/* ------------------------------------------------------------------ */
/* For every block c: `proposals` candidate partners c' (d_c = 0: uniform
 * over the other blocks; else t drawn from e_c. with idx(W0, d_c), then a
 * uniform block != c if idx(W1, d_t + eps C) < eps C, else c' drawn from
 * e_t. with idx(W2, d_t); c' = c is invalid).  Each valid candidate is
 * scored by dS_local = -(change of L when c and c' become one block); the
 * candidate with the smallest floor(dS_local 2^20) is kept (first on ties).
 * Outputs [C]: partner (or -1), dS = dS_local + model-term change C -> C-1
 * (the full DL change after compaction; +inf without a candidate), and
 * dS_local (nullable).  bm must be built for (assign, C). */
int sbp_merge_scores(const sbp_graph *g /*[host]*/, const int32_t *assign, int32_t C, const void *bm,
                     const sbp_merge_params *p /*[host]*/, int32_t *partner, double *dS, double *dS_local,
                     void *ws, size_t ws_bytes, void *stream);

/* Applies up to n_merges merges (Alg. 1 bottom; pointer-based tracking of
 * Sec. III-A (d)): candidates in ascending (floor(dS_local 2^20), c); each
 * joins the group of c with the group of partner[c] unless they are already
 * one group or partner[c] = -1; stops after n_merges joins.  map [C]
 * receives the new label of every old block: groups numbered in ascending
 * order of their smallest member.  *C_new [host] receives the group count.
 * SYNC. */
int sbp_merge_apply(int32_t C, const int32_t *partner, const double *dS_local, int32_t n_merges,
                    int32_t *map, int32_t *C_new /*[host]*/, void *ws, size_t ws_bytes, void *stream);

/* assign[v] <- map[assign[v]] for all v. */
int sbp_relabel(int32_t n, int32_t *assign, const int32_t *map, void *stream);

/* Drops empty labels keeping the order of the others; *C_new [host]. SYNC. */
int sbp_compact(int32_t n, int32_t *assign, int32_t C, int32_t *C_new /*[host]*/, void *ws,
                size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* The whole method (Sec. II-B) and its batched / continuous form       */
/* ------------------------------------------------------------------ */
/* Agglomerative SBP: start from assign_in (labels < C_in, compacted) or,
 * when assign_in is NULL, from every vertex in its own block; alternate a
 * merge phase (Alg. 1) down to a target count and an MCMC phase (Alg. 2,
 * stopped when |DL_prev - DL| < t DL or after max_sweeps sweeps) at that
 * count, while a golden-ratio search over C keeps three (C, DL, assignment)
 * results, each stored at the count its merge phase produced (blocks the
 * MCMC phase emptied stay as empty labels and count in C of Eq. 2): before a
 * bracket exists the next target is C_mid - floor(C_mid merge_rate) from the
 * best result; afterwards the larger of the segments (C_hi - C_mid) and
 * (C_mid - C_lo) is split 0.382 of its length away from mid (upper: merged
 * down from the hi result; lower: from the best result).  Stops when
 * C_hi - C_lo <= 2 (C_mid - C_lo <= 1 without hi), when no merge is
 * possible, or after max_iters iterations; returns the best result with
 * its empty labels dropped (C_out non-empty blocks) and its DL at C_out.
 * Merge phase k uses phase index k; sweeps are numbered across the run.
 * Workspace: sbp_partition_workspace_bytes.  SYNC. */
size_t sbp_partition_workspace_bytes(int32_t n_graphs, const int32_t *n /*[host]*/, const int32_t *e /*[host]*/);
int sbp_partition(const sbp_graph *g /*[host]*/, const int32_t *assign_in, int32_t C_in,
                  const sbp_partition_params *p /*[host]*/, int32_t *assign_out, int32_t *C_out /*[host]*/,
                  double *dl_out /*[host]*/, void *ws, size_t ws_bytes, void *stream);

/* n_graphs independent partitions in shared launches; graph i's result is
 * bit-identical to sbp_partition on graph i alone.  SYNC. */
int sbp_partition_batch(int32_t n_graphs, const sbp_graph *graphs /*[host]*/,
                        const sbp_partition_params *params /*[host], one per graph*/,
                        int32_t *const *assign_out /*[host] array of device pointers*/,
                        int32_t *C_out /*[host]*/, double *dl_out /*[host]*/,
                        void *ws, size_t ws_bytes, void *stream);

/* Per-iteration record of a finished graph (host): rows of [C_start,
 * C_target, C_after_merge, sweeps, C_stored] and the DL of each stored
 * result.  `tag` is the engine tag (-1 for sbp_partition).  The record is
 * removed once read.  Returns the number of rows written (0 if none). */
int sbp_partition_trace(int64_t tag, int64_t *rows /*[host] 5*cap*/, double *dl /*[host] cap*/, int32_t cap);

/* ------------------------------------------------------------------ */
/* Divide-and-conquer SBP (Sec. II-C, Alg. 3)                          */
/* ------------------------------------------------------------------ */
/* The vertices are split round robin into n_sub subgraphs (vertex v goes to
 * subgraph v mod n_sub; a subgraph keeps the edges between its own
 * vertices, renumbered in ascending order).  Every subgraph is partitioned
 * by the whole method (as sbp_partition, with seed p->seed + 1 + r for
 * subgraph r), all in one batched run.  While more than four partial
 * results remain they are combined in pairs (0,1), (2,3), ... (an odd last
 * one passes on): on the graph the pair's vertices induce, with the second
 * result's labels after the first's, every community of the second joins
 * the community of the first whose merge changes DL least (compared on
 * floor(dS_local 2^20) as in sbp_merge_scores, the lowest on ties), all
 * choices made before any is applied; the result is compacted.  The
 * remaining results are concatenated (labels of result k after those of
 * results 0..k-1) and the whole method continues on the full graph from that
 * assignment with p (as sbp_partition with assign_in).
 * Outputs: assign_out [n] (device), *C_out, *dl_out [host]; sub_C [host,
 * nullable] receives the block count found for each subgraph [n_sub].
 * 1 <= n_sub <= n, else SBP_E_ARG.  Workspace: sbp_dcsbp_workspace_bytes.
 * SYNC. */
size_t sbp_dcsbp_workspace_bytes(int32_t n, int32_t e, int32_t n_sub);
int sbp_dcsbp(const sbp_graph *g /*[host]*/, int32_t n_sub, const sbp_partition_params *p /*[host]*/,
              int32_t *assign_out, int32_t *C_out /*[host]*/, double *dl_out /*[host]*/, int32_t *sub_C /*[host]*/,
              void *ws, size_t ws_bytes, void *stream);

/* Continuous batching engine.  Graphs are admitted while their footprint
 * fits the engine's workspace; every sbp_engine_step advances each admitted
 * graph by one step of its own partition (a merge phase, one sweep batch,
 * or a compaction) in shared launches; finished graphs leave and free their
 * space for new admissions.  The engine object is host memory; all device
 * memory comes from ws. */
typedef struct sbp_engine sbp_engine;
size_t sbp_engine_workspace_bytes(int64_t max_vertices, int64_t max_edges, int32_t max_graphs);
int sbp_engine_create(void *ws, size_t ws_bytes, int64_t max_vertices, int64_t max_edges, int32_t max_graphs,
                      void *stream, sbp_engine **out /*[host]*/);
/* Admits a graph (assign_out [n] receives the final assignment).  With
 * C_init = 0 the partition starts from every vertex in its own block; with
 * C_init > 0 assign_out must already hold a compact assignment with labels
 * 0..C_init-1 (every label used).  Returns
 * SBP_OK, or SBP_E_SPACE if it does not fit right now (try again after
 * steps), or another error. `tag` identifies the graph in sbp_engine_poll. */
int sbp_engine_admit(sbp_engine *eng, const sbp_graph *g /*[host]*/, const sbp_partition_params *p /*[host]*/,
                     int32_t *assign_out, int32_t C_init, int64_t tag);
/* One step for all admitted graphs (SYNC).  *active [host] receives the
 * number of graphs still running. */
int sbp_engine_step(sbp_engine *eng, int32_t *active /*[host]*/);
/* Pops one finished graph: returns 1 and fills tag, C, DL, or returns 0. */
int sbp_engine_poll(sbp_engine *eng, int64_t *tag, int32_t *C, double *dl);
/* Bytes the graph would occupy in the engine (its admission footprint). */
size_t sbp_engine_graph_bytes(int32_t n, int32_t e);
int sbp_engine_destroy(sbp_engine *eng);

/* Launch-shape tuning (results do not depend on it).  Keys:
 *   "dense_eval_workgroups"  workgroups of the dense sweep-evaluation grid
 *                            (0 = one per chunk, capped at the workgroups
 *                            a CU holds)
 *   "dense_delta_workgroups" workgroups of the dense block-matrix update
 *   "dense_update_moved_share" a one-batch dense sweep updates M and the end
 *                            bytes from the moved vertices alone when at
 *                            most value/1024 of the vertices moved (default
 *                            64; 0..1024, or -1 for never), otherwise by a
 *                            pass over every edge end
 *   "engine_dense_max_c"     engine sweep batches at C <= value (0..64) run on
 *                            the dense kernels (default 64; 0 = never)
 *   "table_max_c"            sparse sweeps at C <= value (0..2048) read M from
 *                            a C x C lookup table (default 2048; 0 = never)
 *   "table_build"            engine steps count M into the tables: 0 never,
 *                            1 when the tables are small against the edges
 *                            (default), 2 whenever every graph's table fits
 *   "batches_in_step"        1 (default): the hubs and batches of a sweep after
 *                            its first run in the same engine step, each on a
 *                            blockmodel rebuilt after the one before, without
 *                            a host round trip; 0: one a step
 * Returns SBP_E_ARG for an unknown key or a value out of range. */
int sbp_tune(const char *key, int64_t value);

/* Kernel timing for measurement.  on = 0 disables it; on = k >= 1 attaches
 * HIP events to the start and end of every k-th launch of the
 * sweep-evaluation kernel ("sweep_eval"; dense and sparse tiers), counting
 * from the first launch after the call (k = 1: every launch).  Each pair of
 * attached events costs the GPU a few microseconds, so a sampling stride
 * k > 1 keeps a timed loop close to its unprofiled speed.
 * sbp_profile_read synchronises on those events and returns the summed
 * milliseconds and the number of timed launches since the last reset;
 * reset = 1 clears the record.  Host-side bookkeeping only; returns
 * SBP_E_ARG for on < 0 or an unknown kernel name. */
int sbp_profile_enable(int32_t on);
int sbp_profile_read(const char *kernel, double *ms /*[host]*/, int64_t *launches /*[host]*/, int32_t reset);

const char *sbp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SBP_H */
