/*
 * libsimrank: incremental all-pairs SimRank on one MI355X (gfx950) GPU.
 *
 * Method: Yu, Lin, Zhang, McCann, "Dynamical SimRank Search on Time-Varying Networks".
 * SimRank is the unique fixed point of  S = C Q S Q^T + (1 - C) I  (section 3.1, eq (03a)),
 * Q the backward transition matrix (Q[a][x] = 1/indeg(a) for an edge x -> a). A link update
 * changes Q by a rank-one term (Theorems 1 and 9) and S by Delta S = M + M^T, where M solves
 * a rank-one Sylvester equation (Theorem 2, eq (14)); the library evaluates M by K sparse
 * matrix-vector products (eq (16a)), restricts the work to the affected areas of Theorem 4,
 * handles edges that bring new nodes (section 6, cases C1-C3), batches of edges grouped by
 * shared sink (section 8, Table 2, Algorithm 6), and a column-by-column mode that never
 * stores S (section 7, Algorithm 7).
 *
 * Conventions for every entry point:
 *  - An edge (i, j) means i -> j; j is the sink whose row of Q changes.
 *  - Node ids are int32 in [0, n). New nodes take the next ids n, n+1, ... (section 6 remark).
 *  - Host arrays passed in are borrowed for the duration of the call only.
 *  - Device pointers passed in are owned by the caller and must stay valid until the
 *    context's stream has executed the work (synchronise the stream or call sr_synchronize).
 *  - All work is enqueued on the HIP stream given to init_simrank and is asynchronous,
 *    except where a call says it synchronises.
 *  - Errors are status codes; nothing is thrown across the ABI. A validation error
 *    (SR_EINVAL .. SR_EMODE) leaves the context unchanged. SR_EHIP (a HIP runtime error)
 *    poisons the context: every later call except sr_destroy returns SR_EHIP.
 *  - Matrices are row-major. S is symmetric, so row x of S is also column x.
 */
#ifndef LIBSIMRANK_SIMRANK_H
#define LIBSIMRANK_SIMRANK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sr_ctx sr_ctx;

typedef enum sr_status {
  SR_OK = 0,
  SR_EINVAL = -1,     /* malformed argument (null pointer, bad config, bad op)          */
  SR_ERANGE = -2,     /* node id out of range, or new node ids not dense                */
  SR_EEXIST = -3,     /* insertion of an edge that exists                               */
  SR_ENOENT = -4,     /* deletion of an edge that does not exist                        */
  SR_ESELF = -5,      /* self-loop                                                      */
  SR_ECAPACITY = -6,  /* node or edge capacity, or scratch capacity, exceeded           */
  SR_ENOMEM = -7,     /* device or host allocation failed                               */
  SR_EMODE = -8,      /* call not available in this context's mode or precision        */
  SR_EHIP = -9        /* HIP runtime error; the context is poisoned                     */
} sr_status;

/* Storage of the dense S. */
enum {
  SR_S_FP64 = 0,       /* float64                                                         */
  SR_S_FP32_HILO = 1,  /* float32 value + float32 compensation, adjacent per entry; updates
                          add in float64                                                   */
  SR_S_FP32 = 2        /* plain float32 (no compensation), for precision comparisons      */
};
/* Context mode. */
enum { SR_DENSE = 0, SR_COLUMN = 1 };
/* Which gamma formula a unit or block update uses (section 4). */
enum {
  SR_GAMMA_CLOSED = 0, /* Theorem 3 / Theorem 9 / Table 2 closed form (2 columns of S)     */
  SR_GAMMA_DIRECT = 1  /* Theorem 2 direct form w = Q S v + (v^T S v / 2) u                */
};
/* Arithmetic of the fused batch passes (the low-rank update of S by many blocks at once). */
enum {
  SR_UPDATE_FP64 = 0, /* float64 matrix cores                                               */
  SR_UPDATE_FP32 = 1  /* float32 matrix cores: the panel rounded to float, products and sums
                         in float, added to S in float64 (the value + compensation store
                         keeps the sum); the series vectors and gamma stay float64          */
};
/* What query_column returns. */
enum { SR_COL_S = 0, SR_COL_DELTA = 1 };

typedef struct sr_config {
  double C;              /* damping factor, 0 < C < 1 (paper default 0.6)                  */
  int32_t K;             /* iterations: the series keeps K + 1 terms, k = 0..K (Alg. 1)     */
  int32_t K_ps;          /* PartialSim depth in column mode (section 7); 0 means K          */
  int32_t s_prec;        /* SR_S_FP64 | SR_S_FP32_HILO | SR_S_FP32 (dense mode)             */
  int32_t mode;          /* SR_DENSE | SR_COLUMN                                            */
  int32_t gamma_form;    /* SR_GAMMA_CLOSED | SR_GAMMA_DIRECT                               */
  int32_t prune;         /* 1: restrict the S update to the affected areas (Theorem 4)      */
  int64_t node_cap;      /* maximum node count over the context's life (>= n); 0 means n    */
  int64_t edge_cap;      /* maximum edge count (>= m); 0 means 2 m + 1024                   */
  double init_tol;       /* fixed-point step tolerance of the initial S (max-abs)           */
  int32_t init_max_iter; /* iteration cap of the initial fixed point                        */
  int32_t batch_chunk;   /* low-rank blocks per fused pass of apply_batch, or per
                            accumulate pass of apply_batch_columns (at most 65,535; more is
                            SR_EINVAL, as in sr_set_tuning); 0: the mode's default,
                            64 in dense mode, ceil(512 / (2 (K + 1))) in column mode
                            (passes bounded by arithmetic, not by the output's traffic, with
                            a panel of at most 512 + 2 (K + 1) columns of n doubles)       */
  int32_t fused_batch;   /* 1: apply_batch defers low-rank blocks into fused passes;
                            0: each block updates S on its own                              */
  int32_t split_rows;    /* graph rows (in- or out-lists) with more entries are traversed in
                            chunks of 4096 entries, one workgroup each, whose partial sums a
                            second small launch adds; rows of 2049 .. split_rows entries take
                            one workgroup. 0 means 8192; otherwise at least 2048             */
  int32_t profile;       /* 1: time the S-update launches from creation on (as sr_profile(1)),
                            so that those inside init_simrank_tree are counted too          */
  int32_t graphs;        /* 1: fused batches capture each block's K-step series chain as a HIP
                            graph (one per panel slot of a chunk, kept while the node count
                            and the graph's row tiers stay) and replay it; 0: plain launches */
  int32_t update_prec;   /* SR_UPDATE_FP64 | SR_UPDATE_FP32: the fused passes' arithmetic    */
  int32_t block_store;   /* 1 (init_simrank_partitioned only, dense mode): keep S as Example
                            1.1 does, per pair of partition blocks: the diagonal blocks S_Gi
                            of the blocks' own edges, and for the cross-block edges only the
                            block pairs their Delta S reaches, each a dense sub-matrix
                            allocated when first reached; no n x n store. Such a context
                            serves query_column (SR_COL_S), query_columns, query_topk,
                            sr_gather_pairs and sr_copy_S, and takes apply_batch batches of
                            insertions and deletions between existing nodes (fused passes
                            into the reached pairs); other updates, backward and
                            query_topk_noalloc return SR_EMODE. 0: one dense store          */
  int32_t tile_skip;     /* 1: a dense fused pass skips, per 128 x 128 tile of the square of
                            its reached nodes, the k-steps (panel columns 4 g .. 4 g + 3) of
                            each block whose xi_2g and xi_2g+1 vanish on both of the tile's
                            row ranges (xi_k lives on the nodes k out-steps from the sink,
                            Theorem 4's A_k); those products are exact zeros, so S is bit for
                            bit the same as with 0, every k-step of every tile               */
} sr_config;

/* Per-update statistics (filled when a non-null pointer is passed; the call then
 * synchronises the stream). */
typedef struct sr_update_stats {
  int32_t case_id;     /* 0 both ends existing, 1 new sink, 2 new source, 3 both new       */
  int32_t op;          /* +1 insert, -1 delete                                             */
  int64_t d_j;         /* in-degree of the sink before the update                          */
  int64_t n_after;     /* node count after the update                                      */
  int64_t aff_A;       /* |A_hat| (union of the A_k of Theorem 4)                          */
  int64_t aff_B;       /* |B_hat|                                                          */
  int64_t aff_AB;      /* |A_hat & B_hat|                                                  */
  int64_t pairs;       /* S entries written: |A_hat x B_hat u B_hat x A_hat|, or n^2       */
  double bound;        /* truncation bound 2 C^(K+2)/(1-C) |u|_inf |w|_inf of Delta S      */
} sr_update_stats;

typedef struct sr_batch_stats {
  int64_t edges_in;       /* edges passed in                                               */
  int64_t edges_net;      /* edges left after insert/delete cancellation                   */
  int64_t blocks;         /* similar-sink blocks processed                                 */
  int64_t blocks_case[4]; /* blocks per case C0..C3                                        */
  int64_t lowrank_blocks; /* blocks that produced a low-rank Delta S (C0 and C2)           */
  int64_t n_after;        /* node count after the batch                                    */
  int64_t pairs;          /* S entries updated, summed over low-rank blocks, plus border
                             and diagonal writes of C1 / C2 / C3 blocks; a fused pass counts
                             the square of the nodes it reaches (those with a nonzero panel
                             row), per deferred block; with block_store, the entries of the
                             block pairs the pass reaches, per deferred block              */
  int32_t fused_passes;   /* passes over S made by the fused apply                         */
  int32_t series_replays; /* K-step series chains replayed from captured HIP graphs        */
  int64_t pass_entries;   /* dense fused passes: distinct entries (a <= b) of S that their
                             GEMMs computed, summed over the passes' low-rank blocks (a
                             pass covers the square of the nodes its blocks reach)          */
  int64_t pass_skipped;   /* of those, entry k-steps skipped by tile_skip: summed over the
                             blocks and their k-steps (4 panel columns, 8 flop per entry),
                             the distinct entries of the tiles that skipped the k-step; the
                             passes' arithmetic is 8 (pass_entries ceil((K + 1) / 2) -
                             pass_skipped) flop                                            */
} sr_batch_stats;

/* Fills *cfg with defaults: C = 0.6, K = 15, K_ps = 30, SR_S_FP64, SR_DENSE,
 * SR_GAMMA_CLOSED, prune = 1, capacities 0 (derived), init_tol = 1e-15, init_max_iter = 400,
 * batch_chunk = 0 (the mode's default), fused_batch = 1, graphs = 1, tile_skip = 1. */
sr_status sr_default_config(sr_config* cfg);

/* Creates a context for the digraph with n nodes and m edges src[e] -> dst[e] (host arrays,
 * no self-loops, no duplicates). weight: host float64 per edge (> 0), or NULL for an
 * unweighted graph; Q is row-normalised, Q[x][y] = w(y -> x) / W_x. A weighted graph
 * supports unit updates in dense mode (apply_edge_update, apply_weight_update), queries and
 * backward; its batches and column-mode updates return SR_EMODE. S0: NULL to compute the initial S on the device by the
 * fixed-point iteration of eq (03a) until the max-abs step is <= cfg->init_tol; otherwise a
 * device pointer to an n x n float64 row-major S (leading dimension n), which is copied.
 * In column mode S is never stored and S0 must be NULL. hip_stream: a hipStream_t (NULL for
 * the null stream). Synchronises the stream before returning. On success *out owns every
 * device allocation of the context. */
sr_status init_simrank(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                       const int32_t* dst, const double* weight, const sr_config* cfg,
                       const void* S0, void* hip_stream);

/* All-pairs SimRank seeded from a spanning forest (Example 1.2): builds the breadth-first
 * spanning forest of the digraph (nodes without in-edges are roots first, then any node not
 * reached yet, both in ascending id; out-neighbours are scanned in ascending id), creates a
 * dense-mode context on the forest's edges with S set by the example's closed form (for a, b
 * at one depth H whose lowest common ancestor is lambda edges up,
 * S[a][b] = C^lambda (1 - C^(H - lambda + 1)); 0 across depths and across trees), then
 * applies every other edge, in the caller's order, as one apply_batch of insertions. The
 * result is S of the whole graph up to the K-term truncation of each block's series.
 * src, dst: host arrays of m edges (no self-loops, no duplicates); cfg: as init_simrank, mode
 * must be SR_DENSE (SR_EMODE otherwise), edge_cap 0 means 2 m + 1024. Unweighted only.
 * stats: NULL, or the batch's statistics. On any error nothing is returned (*out = NULL). */
sr_status init_simrank_tree(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                            const int32_t* dst, const sr_config* cfg, void* hip_stream,
                            sr_batch_stats* stats);

/* Graph partitioner for init_simrank_partitioned (host only, no GPU work): blocks of at most
 * ceil(n / parts) nodes grown breadth first over the undirected graph. A block starts at the
 * smallest unassigned id and scans neighbours in ascending id; a full block stops at once, and
 * one whose search runs dry continues from the smallest unassigned id. part_out: host array
 * of n block labels 0, 1, ... SR_EINVAL for parts < 1, SR_ERANGE for an edge out of range. */
sr_status sr_partition(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       int32_t parts, int32_t* part_out);

/* All-pairs SimRank over a partitioned graph (Example 1.1): with part[v] the block of node v
 * (host array, any labels in [0, n), e.g. from sr_partition), S of the edges inside blocks is
 * block diagonal; each block's S is computed on its own nodes (the fixed point of eq (03a),
 * float64) and placed on the diagonal of the store, then the edges across blocks are applied,
 * in the caller's order, as one apply_batch of insertions. The result is S of the whole graph
 * up to the K-term truncation of each block of the batch. cfg: as init_simrank, mode must be
 * SR_DENSE (SR_EMODE otherwise), edge_cap 0 means 2 m + 1024; with cfg->block_store = 1 the
 * store is the block pairs (see sr_config; labels must be below 4096, SR_ECAPACITY
 * otherwise). Unweighted only. stats: NULL, or the batch's statistics. On any error nothing
 * is returned (*out = NULL). */
sr_status init_simrank_partitioned(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                                   const int32_t* dst, const int32_t* part,
                                   const sr_config* cfg, void* hip_stream,
                                   sr_batch_stats* stats);

/* Applies one edge update, op = +1 insert or -1 delete (Algorithms 1 and 2, Theorem 9;
 * node insertions: Algorithms 3, 4, 5 with the new ids i == n (C2), j == n (C1), or
 * i == n, j == n + 1 (C3)). Dense mode updates S. Column mode (Algorithm 7) stores no S: it
 * computes the columns the update needs by PartialSim on the current graph (S[:, i] and
 * S[:, j] for C0, S[:, i] for C1, S[:, j] for C2) and keeps this update's Delta S in factored
 * form for query_columns / query_column(SR_COL_DELTA): the series panel (C0, C2), the new
 * sink's column (C1), the new diagonals (C3). Deletions are between existing nodes (C0).
 * stats: NULL, or filled after synchronising. */
sr_status apply_edge_update(sr_ctx* ctx, int32_t i, int32_t j, int32_t op,
                            sr_update_stats* stats);

/* Weighted graphs: sets the weight of edge i -> j to w >= 0, as one rank-one update of the
 * row-normalised Q, the weighted analogue of Theorems 1 and 9 (Delta Q = e_j a (e_i -
 * Q[j, :])^T with a = dw / (W_j + dw), dw the weight change, W_j j's in-weight sum; the
 * forms of an empty row before or after are the unweighted ones), solved like
 * apply_edge_update with Theorem 3's closed form in a (it rests only on the fixed-point
 * identity of eq (33)). w > 0 on a missing edge inserts it (new nodes as apply_edge_update:
 * j == n, i == n, or i == n and j == n + 1), w == 0 deletes an existing edge, any other w
 * changes its weight; w equal to the current weight changes nothing. apply_edge_update on
 * a weighted graph inserts with weight 1. SR_EMODE for an unweighted context or in column
 * mode, SR_EINVAL for a negative or non-finite w, SR_ENOENT for w == 0 on a missing edge;
 * otherwise as apply_edge_update. stats: NULL, or filled after synchronising. */
sr_status apply_weight_update(sr_ctx* ctx, int32_t i, int32_t j, double w,
                              sr_update_stats* stats);

/* Applies a batch of cnt edge updates (host arrays; op[e] = +1 or -1) by Algorithm 6:
 * cancellation of insert/delete pairs, similar-sink partition, deletion blocks, then
 * insertion blocks split by whether their sources already exist, each by the Table 2
 * formula of its case. New node ids in the batch must be exactly n .. n + N - 1.
 * A net count outside {-1, 0, +1} for an edge, an insertion of an existing edge or a
 * deletion of a missing one rejects the whole batch before any change. Dense mode only.
 * stats: NULL, or filled after synchronising. */
sr_status apply_batch(sr_ctx* ctx, int64_t cnt, const int32_t* src, const int32_t* dst,
                      const int8_t* op, sr_batch_stats* stats);

/* Column mode: applies a batch of edge insertions and deletions between existing nodes and
 * returns the columns of its Delta S, memory-efficiently: Algorithm 6's plan (as
 * apply_batch) with the column method of Algorithm 7 inside every block (PartialSim of
 * S[:, I] and S[:, j] on the graph as the earlier blocks left it, Table 2 row C0, the K-step
 * series of eq (16a)), and eq (71) summed over the blocks:
 *   out_dev[t * ld_out + a] = Delta S[a][cols[t]]   (float64, t < ncols, a < n).
 * cols: host array of node ids (< n); out_dev: device, ncols x ld_out float64, ld_out >= n,
 * overwritten (entries past n of a row are set to zero). Memory: O(K n + m) besides the output: batch_chunk
 * deferred blocks of n x 2(K+1) doubles each (packed in slabs of 16 columns; at most
 * 512 + 2(K+1) columns at the default chunk), then one FP64 matrix-core pass over them per
 * chunk. SR_EMODE outside column mode, for a weighted graph, or when an edge would create
 * a node; SR_ERANGE for a column id out of range; otherwise as apply_batch (validation errors
 * change nothing). stats: NULL, or filled after synchronising. */
sr_status apply_batch_columns(sr_ctx* ctx, int64_t cnt, const int32_t* src,
                              const int32_t* dst, const int8_t* op, const int32_t* cols,
                              int32_t ncols, double* out_dev, int64_t ld_out,
                              sr_batch_stats* stats);

/* Writes column x as n float64 values to out_dev (device). what = SR_COL_S: the current
 * S[:, x] (dense mode). what = SR_COL_DELTA: Delta S[:, x] of the last apply_edge_update
 * (both modes): eq (71), M_K[:, x] + M_K[x, :]^T, for C0 and C2 (with the new source's own
 * column (1 - C) e_i), the new sink's column and border entry for C1 (Theorem 8), the new
 * diagonals for C3; n is the node count after the update and a new node's old column counts
 * as zero. SR_EMODE when the last call was not a unit update. */
sr_status query_column(sr_ctx* ctx, int32_t x, int32_t what, double* out_dev);

/* Writes ncols columns as float32 to out_dev (device), column c at out_dev + c * ld_out,
 * ld_out >= n. cols: host array of node ids. Column mode: Delta S[:, cols] of the last
 * apply_edge_update, as query_column(SR_COL_DELTA) (eq (71) for all columns at once in the
 * low-rank cases). Dense mode: S[:, cols]. */
sr_status query_columns(sr_ctx* ctx, const int32_t* cols, int32_t ncols, float* out_dev,
                        int64_t ld_out);

/* Top-k single-source search after any updates: for each query x = q[t] (host array of nq
 * ids < n), the k nodes b with the largest S[x][b], best first, ties to the smaller id, x
 * itself left out when exclude_self is nonzero: idx_dev[t * k + r] (int32, device) and
 * val_dev[t * k + r] (float64, device), r < k. Dense mode reads the stored row of x (S is
 * symmetric) once per query; column mode computes S[:, x] by PartialSim (section 7, depth
 * K_ps) two queries at a time first. 1 <= k <= 3072 and k <= n - (exclude_self ? 1 : 0),
 * else SR_EINVAL; SR_ERANGE for a query id out of range. */
sr_status query_topk(sr_ctx* ctx, const int32_t* q, int32_t nq, int32_t k,
                     int32_t exclude_self, int32_t* idx_dev, double* val_dev);

/* query_topk for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same selection, bit for bit, but
 * the query ids are staged in a static per-GPU device array of 65,536 ids (256 KiB, held until
 * the process ends) instead of a buffer the context allocates; the call neither allocates nor
 * frees memory and does not synchronise the stream itself. q: host array of nq ids, copied to
 * the array by a copy enqueued on the context's stream: keep it unchanged until that stream
 * has run the call's work. SR_ECAPACITY for nq > 65536 (nothing is launched); otherwise as
 * query_topk. Every call on a
 * GPU shares that GPU's array: calls on different streams of one GPU that overlap in time
 * race on it (calls on one stream are ordered). */
sr_status query_topk_noalloc(sr_ctx* ctx, const int32_t* q, int32_t nq, int32_t k,
                             int32_t exclude_self, int32_t* idx_dev, double* val_dev);

/* Gathers S[a[p], b[p]] for npairs pairs into out_dev (float64); a_dev, b_dev device int32.
 * Dense mode. */
sr_status sr_gather_pairs(sr_ctx* ctx, int64_t npairs, const int32_t* a_dev,
                          const int32_t* b_dev, double* out_dev);

/* Reverse-mode derivative of a loss L(S) with respect to the edge weights of the current
 * graph (weighted or unweighted; an unweighted graph has all weights 1), using the stored S
 * (after updates: the incrementally maintained one). Inputs: npairs pairs
 * (a_dev[p], b_dev[p]) with dL/dS[a,b] = g_dev[p] (all device arrays; ids outside [0, n) are
 * SR_ERANGE before any launch, which synchronises the stream). Solves the transposed
 * Sylvester equation Lam = G + C Q^T Lam Q to the init tolerance and writes dL/dw for every
 * current edge to dL_dw_dev (device, m float64, m the current edge count) in the order of
 * sr_edges: init_simrank's edge order until the first update, sinks ascending after it.
 * Dense mode (SR_EMODE otherwise). Allocates four n x n float64 work matrices for the call. */
sr_status backward(sr_ctx* ctx, int64_t npairs, const int32_t* a_dev, const int32_t* b_dev,
                   const double* g_dev, double* dL_dw_dev);

/* Affected-area sets of the last dense apply_edge_update with pruning: level = -1 gives
 * A_hat and B_hat, level k in 0..K gives A_k and B_k (Theorem 4, eq (41)), as ascending
 * int32 lists written to A_dev / B_dev (device, capacity n each; NULL to only count).
 * Synchronises; *nA, *nB receive the sizes. */
sr_status sr_get_aff(sr_ctx* ctx, int32_t level, int32_t* A_dev, int64_t* nA, int32_t* B_dev,
                     int64_t* nB);

/* Copies S[0:n, 0:n] as float64 into out_dev (device) with leading dimension ld >= n.
 * Dense mode. */
sr_status sr_copy_S(sr_ctx* ctx, double* out_dev, int64_t ld);

/* The current edges: src[e] -> dst[e] with weight w[e] (1 for an unweighted graph), host
 * arrays of capacity cap (any may be NULL), in the order backward reports dL/dw: the edge
 * arrays given to init_simrank until the first update, then by sink ascending (slot order
 * within a sink). *m receives the edge count; nothing is written when cap < *m. */
sr_status sr_edges(sr_ctx* ctx, int32_t* src, int32_t* dst, double* w, int64_t cap,
                   int64_t* m);

/* Current node and edge counts. */
sr_status sr_sizes(sr_ctx* ctx, int64_t* n, int64_t* m);

/* The context's configuration as resolved at init (defaults filled in: capacities,
 * batch_chunk) and as changed since by sr_set_tuning. SR_EINVAL for a NULL argument. */
sr_status sr_get_config(sr_ctx* ctx, sr_config* out);

/* Bytes of the context's store of S: the dense n x n store (node_cap rows of its leading
 * dimension), or with block_store the sub-matrices of the block pairs held (pairs: their
 * count; 0 for a dense store); 0 in column mode. bytes, pairs: NULL or filled. SR_EINVAL
 * for an invalid context. */
sr_status sr_store_bytes(sr_ctx* ctx, int64_t* bytes, int64_t* pairs);

/* Device memory the library holds now, over all contexts of the process (S, panels, graph
 * arrays, work buffers; not the caller's buffers, not the static no-allocation scratch), and
 * the peak since the last reset: held, peak: NULL or filled, in bytes; reset_peak != 0 sets
 * the peak to the bytes held now after reading it. Always SR_OK. */
sr_status sr_device_bytes(int64_t* held, int64_t* peak, int32_t reset_peak);

/* The block plan of the last apply_batch, as int32 records
 * [case, op, j, d_j, delta, i_1, ..., i_delta] concatenated, into out (host, capacity cap).
 * *len receives the number of int32 values (also when out is NULL or cap is too small). */
sr_status sr_last_plan(sr_ctx* ctx, int32_t* out, int64_t cap, int64_t* len);

/* Waits for all work enqueued by the context. */
sr_status sr_synchronize(sr_ctx* ctx);

/* Releases every allocation of the context; ctx may be NULL. */
sr_status sr_destroy(sr_ctx* ctx);

/* Static description of a status code. */
const char* sr_strerror(sr_status status);

/* Diagnostics: kernel timing of the S-update launches. enable = 1 records a pair of HIP events
 * on the context's stream around every launch of a call's dominant kernel: the S update
 * (single-update and fused-batch kernels), the column output of query_columns in column
 * mode, and the dense Q^T X products of backward; 0 stops recording. */
sr_status sr_profile(sr_ctx* ctx, int32_t enable);

/* Synchronises, then returns the summed elapsed milliseconds of the recorded launches (*ms)
 * and their count (*launches); reset = 1 clears the record. */
sr_status sr_profile_read(sr_ctx* ctx, double* ms, int64_t* launches, int32_t reset);

/* Tuning: times the fused pass of apply_batch at the context's current node count with the
 * GEMM tile variant `variant` (0 .. 3: float64 matrix cores with panel columns per LDS chunk
 * and LDS pitch in doubles, (16, 18), (16, 20), (32, 34), (32, 36); 4: float32 matrix cores,
 * as SR_UPDATE_FP32) over `blocks` deferred blocks, and the incremental
 * corrections one deferred block makes for blocks / 2 later slots of its chunk: *gemm_ms and
 * *corr_ms are the mean of `reps` launches after one warm-up. The pass runs on a zero panel,
 * so S keeps its values, through the reached-node form of apply_batch's passes with every
 * node listed. Dense mode; allocates a zero panel of n x blocks 2(K+1) (rounded up to 32)
 * doubles and the node list for the call; synchronises. */
sr_status sr_time_fused(sr_ctx* ctx, int32_t variant, int32_t blocks, int32_t reps,
                        double* gemm_ms, double* corr_ms);

/* Tuning: sets the context's batch_chunk (blocks per fused pass, 1 .. 65,535, else SR_EINVAL)
 * and the fused GEMM's tile variant (as sr_time_fused). A new chunk frees the batch panel and
 * correction buffers, which the next batch allocates again (synchronises). SR_ERANGE for an
 * unknown variant. */
sr_status sr_set_tuning(sr_ctx* ctx, int32_t batch_chunk, int32_t variant);

/* Diagnostics: runs one v_mfma_f64_16x16x4_f64 on a single wave with lane l supplying
 * a_dev[l] and b_dev[l] (64 device doubles each) and writes the four accumulator values held
 * by lane l to out_dev[4 l .. 4 l + 3] (256 device doubles). Used by the tests to confirm the
 * operand and accumulator lane layout the update kernel assumes. Asynchronous on hip_stream. */
sr_status sr_mfma_layout_probe(const double* a_dev, const double* b_dev, double* out_dev,
                               void* hip_stream);

/* Diagnostics: the same for v_mfma_f32_16x16x4f32 with float operands and accumulators (the
 * float32 fused pass relies on its layout). */
sr_status sr_mfma_layout_probe_f32(const float* a_dev, const float* b_dev, float* out_dev,
                                   void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LIBSIMRANK_SIMRANK_H */
