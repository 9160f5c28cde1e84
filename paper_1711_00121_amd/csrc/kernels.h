// Host-side launchers of the HIP kernels of libsimrank. Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sr {

// ---------------------------------------------------------------------------------------
// Graph patches: small in-place edits of the device slotted CSR, passed by value.
struct Patch {
  static constexpr int MAX = 30;
  int32_t count;
  int32_t array[MAX];  // index into the pointer table below
  int32_t index[MAX];
  int32_t value[MAX];
};
// Pointer table order: in_start, in_len, in_idx, out_start, out_len, out_idx.
struct AdjPtrs {
  int32_t* p[6];
};
hipError_t launch_patch(const AdjPtrs& t, const Patch& p, hipStream_t s);
// Weight patches of a weighted graph: slot weights of the in- and out-lists and the in-weight
// sums W, passed by value.
struct WPatch {
  static constexpr int MAX = 24;
  int32_t count;
  int32_t array[MAX];  // 0 in-list slot weights, 1 out-list slot weights, 2 W
  int32_t index[MAX];
  double value[MAX];
};
struct WPtrs {
  double* p[3];
};
hipError_t launch_patch_w(const WPtrs& t, const WPatch& p, hipStream_t s);

// A list of node ids (the sources I of a block). Up to MAX ids travel by value in the
// kernel arguments; a longer list lives in device memory (dev, count entries), so a block of
// any size is one launch sequence. Kernels read entry t with at(t).
struct IdList {
  static constexpr int MAX = 60;
  int32_t count = 0;
  int32_t id[MAX];
  const int32_t* dev = nullptr;  // device ids when count > MAX, else null
  __host__ __device__ int32_t at(int t) const { return dev ? dev[t] : id[t]; }
};

// ---------------------------------------------------------------------------------------
// Sparse traversals. Rows with more than kLight entries are listed by the host: "medium"
// rows (at most kMedium entries) are handled by one wave each, "heavy" rows (up to a split
// threshold, kSplitRows by default) by a workgroup, and "huge" rows are cut into chunks of
// kChunk entries, one workgroup per chunk, whose partial sums a second small launch adds up
// in chunk order. The second launch costs a few microseconds, about what a workgroup takes for
// one or two more rounds of a row's loads, so only long rows gain from it: splitting above two
// chunks' worth measured +3% on batches at n = 58k-92k (the hubs' rows, up to ~34k entries,
// trail every series step otherwise), the same as splitting above one chunk, while at
// n = 20k, whose one row above a chunk holds 5.5k entries, splitting it cost 10% of the
// forest-seeded pipeline.
constexpr int kLight = 64;
constexpr int kMedium = 2048;
constexpr int kSplitRows = 8192;
constexpr int kChunk = 4096;
struct HeavyArgs {
  const int32_t* med;    // medium row ids (device), ascending
  int32_t nmed;
  const int32_t* heavy;  // heavy row ids (device), ascending
  int32_t nheavy;
  const int32_t* huge;   // huge row ids (device), ascending
  int32_t nhuge;
  const int2* chunk;     // (row, first entry) per chunk, grouped by huge row in list order
  int32_t nchunk;
  const int32_t* hfirst;  // chunks of huge row h: [hfirst[h], hfirst[h + 1])
  double2* part;          // per chunk: partial sums (scratch, nchunk entries)
  uint32_t* pflag;        // per chunk: affected-area bits (scratch)
};
// Pull form of one affected-area level (Theorem 4): out bit b is set when some in-neighbour x
// of b (new graph) has (s0 | s1)(x). Null sets are empty.
struct AffLevel {
  const uint32_t* a0;
  const uint32_t* a1;
  uint32_t* aout;
  const uint32_t* b0;
  const uint32_t* b1;
  uint32_t* bout;
  int64_t nwords;  // words per bitmap (covers every node id that can appear in the lists)
};
// y[a] = post * (base[a] + scale * (Q x)[a]) for a < n (base may be null). When fout is set,
// bit a of fout is also set if some in-neighbour x of a has bit x of fin (old-graph F1);
// nwords as in AffLevel.
hipError_t launch_spmv_q(const DevQ& q, const HeavyArgs& h, int64_t n, const double* x,
                         double* y, double scale, hipStream_t s, const double* base = nullptr,
                         double post = 1.0, const uint32_t* fin = nullptr,
                         uint32_t* fout = nullptr, int64_t nwords = 0);
// y[b] = scale * (Q^T x)[b] = scale * sum_{a in out(b)} Q[a][b] x[a] (h: heavy out-rows).
// The input comes pre-divided by the row weight of Q, xd[a] = x[a] / d[a] (d = in-degree, or
// the in-weight sum when weighted; 0 where d[a] = 0), so an entry costs one gather; the
// output is written both plain (y) and divided (yd) for the next product.
hipError_t launch_spmv_qt(const DevQ& q, const DevAdj& out, const HeavyArgs& h, int64_t n,
                          const double* xd, double* y, double* yd, double scale,
                          hipStream_t s);
// The same two products on two vectors at once, stored as pairs (node a at 2 a): the gathers of
// both vectors share one cache line. launch_spmv_q2 writes y2, or, with ya and yb set, the two
// halves to ya and yb (base2 may alias y2: each row reads its base before writing).
hipError_t launch_spmv_q2(const DevQ& q, const HeavyArgs& h, int64_t n, const double* x2,
                          double* y2, double scale, hipStream_t s, const double* base2 = nullptr,
                          double post = 1.0, double* ya = nullptr, double* yb = nullptr);
hipError_t launch_spmv_qt2(const DevQ& q, const DevAdj& out, const HeavyArgs& h, int64_t n,
                           const double* xd2, double* y2, double* yd2, double scale,
                           hipStream_t s);
// The same step with explicit places: reads the (xi_k, eta_k) pair of row x at src + x * sld,
// writes the new pair of row a to wbase + a * wld (and to cdst + 2 a when cdst is set).
hipError_t launch_series_step_to(const DevQ& q, const HeavyArgs& h, int64_t n, double* wbase,
                                 int wld, const double* src, int sld, double* cdst, double sx,
                                 double sy, hipStream_t s);
// One step of eq (16a) on the panel P (row a holds (xi_k, eta_k) pairs for k = 0..K, pld
// doubles per row): xi_{k+1} = sx * Q xi_k, eta_{k+1} = sy * Q eta_k; optionally one
// affected-area level in the same pass.
// pairs (optional): 2 x pairs_cap x 2 doubles of scratch; step k writes its pairs compactly
// to half k % 2 and step k + 1 gathers from there instead of from the panel.
hipError_t launch_series_step(const DevQ& q, const HeavyArgs& h, int64_t n, double* P, int pld,
                              int k, double sx, double sy, const AffLevel* aff, hipStream_t s,
                              double* pairs = nullptr, int64_t pairs_cap = 0);

// ---------------------------------------------------------------------------------------
// Dense S helpers.
// SI[a] = sum_{i in I} S[i][a] (accumulate when acc != 0), suppI |= (S[i][a] != 0);
// when j >= 0 also Sj[a] = S[j][a], suppJ bit = (S[j][a] != 0).
// cI / cJ (optional): corrections added to SI / Sj after the supports are taken.
hipError_t launch_gather_rows(SView S, int64_t n, const IdList& I, int acc, int32_t j,
                              double* SI, double* Sj, uint32_t* suppI, uint32_t* suppJ,
                              hipStream_t s, const double* cI = nullptr,
                              const double* cJ = nullptr);
// out[a] = sum_{x in in_old(j)} S[x][a] (rows of S for the in-neighbours of j).
hipError_t launch_gather_inrows(SView S, int64_t n, const DevQ& q, int32_t j, double* out,
                                hipStream_t s);

// Scalars and coefficients of one block update, shared by the gamma kernels.
struct GammaArgs {
  int32_t kind;     // 0 closed form (C0), 1 direct form (C0), 2 C2 z of eq (60) / Table 2,
                    // 3 closed form of a weighted edge change (one source, scale alpha)
  int32_t op;       // +1 insert, -1 delete
  int32_t j;
  int32_t delta;
  int64_t dj;       // in-degree of j before the block
  double C;
  double xi0;       // xi_0 = xi0 * e_j
  double alpha;     // weighted graphs: kind 3's scale a = dw / (W_j + dw) of
                    // Delta Q = e_j a (e_i - Q[j, :])^T; kind 2 with alpha > 0 uses it for
                    // 1 / (d_j + 1) (a new source of weight w: a = w / (W_j + w))
  IdList I;         // sources (for S_II and the direct form's v)
  // When set, the sum over I of the closed form's S[:, I] (kind 0: S_II) or of the direct
  // form's z (kind 1), precomputed by launch_sum_at; long lists use it so that no thread
  // loops over I.
  const double* sumI;
};
// Writes column 0 of the panel: (xi_0, eta_0) = (xi0 e_j, gamma). Inputs: SI = S[:, I],
// Sj = S[:, j], QSI = Q_old S[:, I]; the direct form also needs zsum = sum over in_old(j)
// of S rows and Qz = Q_old z (computed by the caller from zbuf). maxabs receives
// max|gamma| bits (atomicMax on the IEEE pattern of a nonnegative double).
hipError_t launch_gamma(const GammaArgs& g, int64_t n, const double* SI, const double* Sj,
                        const double* QSI, const double* zbuf, const double* Qz, double* P,
                        int pld, unsigned long long* maxabs, hipStream_t s);
// mm[0] = min, mm[1] = max over the ids a[p], b[p], p < np (device int32 arrays); with
// np = 0, mm = (INT32_MAX, INT32_MIN).
hipError_t launch_ids_range(const int32_t* a, const int32_t* b, int64_t np, int32_t* mm,
                            hipStream_t s);
// out[0] = sum_{t < I.count} v[I.at(t)] in a fixed order (one wave).
hipError_t launch_sum_at(const double* v, const IdList& I, double* out, hipStream_t s);
// Direct form step 1: z = S v into zbuf, from SI and zsum (see Theorem 2, eq (20)).
hipError_t launch_direct_z(const GammaArgs& g, int64_t n, const double* SI,
                           const double* zsum, double* zbuf, hipStream_t s);

// C1 border (Theorem 8, Table 2 row C1): S[j][a] = S[a][j] = y[a] for a < n_old,
// S[j][j] = corner = (C/delta^2) S_II + 1 - C (S_II read from SI at the sources, or from
// *sumI when set).
hipError_t launch_c1_border(SView S, int64_t n_old, int32_t j, const double* y,
                            const double* SI, const IdList& I, double C, hipStream_t s,
                            const double* sumI = nullptr);
// y[j] = (C / delta^2) S_II + 1 - C (S_II from SI at the sources, or *sumI when set).
hipError_t launch_c1_corner(double* y, int32_t j, const double* SI, const IdList& I, double C,
                            hipStream_t s, const double* sumI = nullptr);
// Delta S columns of the last node insertion in column mode, for the list rows (device, nrows
// columns; or the single column x when rows is null): kind 1 (C1) from the new sink's column y,
// kind 3 (C3) from the new diagonals vi, vj, kind 2 (C2) only sets entry i of column i to vi
// (after the panel product). Output float32 (out32) or float64 (out64), row t at t * ld.
hipError_t launch_node_cols(const int32_t* rows, int32_t x, int32_t nrows, int64_t n, int kind,
                            int32_t i, int32_t j, const double* y, double vi, double vj,
                            float* out32, double* out64, int64_t ld, hipStream_t s);
// Writes S[id][id] = val[t] for a short list (new-node diagonals).
struct DiagList {
  static constexpr int MAX = 30;
  int32_t count;
  int32_t id[MAX];
  double val[MAX];
};
hipError_t launch_set_diag(SView S, const DiagList& d, hipStream_t s);

// Initial S by the fixed point of eq (03a), in float64 with leading dimension n.
// Y[a][:] = scale * (Q X)[a][:]  (+ add_diag on Y[a][a]); when prev != null also
// maxdiff = max |Y - prev| (atomicMax on the IEEE bits).
hipError_t launch_spmm_rows(const DevQ& q, int64_t n, const double* X, double* Y,
                            double scale, double add_diag, const double* prev,
                            unsigned long long* maxdiff, hipStream_t s);
hipError_t launch_transpose(int64_t n, const double* X, double* Y, hipStream_t s);
// dst (store format, leading dim ld) = src (float64, leading dim n), rows/cols < n; with
// srcT = src^T, dst = (src + src^T) / 2, which is exactly symmetric.
hipError_t launch_to_store(SView dst, int64_t n, const double* src, hipStream_t s,
                           const double* srcT = nullptr);
hipError_t launch_from_store(SView src, int64_t n, double* dst, int64_t ld_dst,
                             hipStream_t s);
hipError_t launch_copy_row(SView S, int64_t n, int32_t x, double* out, hipStream_t s);
hipError_t launch_gather_pairs(SView S, int64_t np, const int32_t* a, const int32_t* b,
                               double* out, hipStream_t s);
hipError_t launch_rows_to_f32(SView S, int64_t n, const int32_t* rows, int32_t nrows,
                              float* out, int64_t ld_out, hipStream_t s);

// ---------------------------------------------------------------------------------------
// Affected areas (Theorem 4). Bitmaps of W words per level; A and B hold K+1 levels each.
struct AffArgs {
  int64_t n;
  int32_t W;       // words per bitmap
  int32_t K;
  uint32_t* A;     // (K+1) * W words
  uint32_t* B;
};
// Level 0 (after F1 = out_old(supp S[I, :]) was or-ed into B_0 by the Q S[:, I] product):
// B_0 |= supp S[j, :] when f2, and j joins A_0 and B_0.
hipError_t launch_aff_level0(const AffArgs& a, const uint32_t* suppJ, int f2, int32_t j,
                             hipStream_t s);
// A_hat = A_0 | A_K, B_hat = B_0 | B_K into Ahat/Bhat; rows = ascending list of the rows the
// streaming update takes, entry (node << 2) | (in A_hat << 1) | (in B_hat): A_hat | B_hat, or,
// when the smaller set X of the two has at most n / 16 nodes, X alone, with the other set's
// nodes outside X listed in mrows for launch_aff_mirror.
// cnt[0..3] = |A_hat|, |B_hat|, |A_hat & B_hat|, |rows|; cnt[6] = |mrows| (0: none).
hipError_t launch_aff_compact(const AffArgs& a, uint32_t* Ahat, uint32_t* Bhat,
                              int32_t* rows, int32_t* mrows, int64_t* cnt, hipStream_t s);
// After the streaming update of the listed rows: S[y][x] = S[x][y] for the listed x and the
// mirrored y (nothing when cnt[6] == 0).
hipError_t launch_aff_mirror(SView S, const int32_t* rows, const int32_t* mrows,
                             const int64_t* cnt, hipStream_t s);
// Ascending list of the set bits of bm (n bits) into out; *cnt receives the count.
hipError_t launch_bits_to_list(const uint32_t* bm, int64_t n, int32_t W, int32_t* out,
                               int64_t* cnt, hipStream_t s);
// Or-combination helper: dst = a | b (W words).
hipError_t launch_bits_or(const uint32_t* a, const uint32_t* b, uint32_t* dst, int32_t W,
                          hipStream_t s);

// ---------------------------------------------------------------------------------------
// Low-rank update of S (the hot kernel):
//   for each listed row a (rows[t], t < nrows; with a mask the entries are packed as
//   (node << 2) | (in Ahat << 1) | (in Bhat)) and column b < ncols where the pair is in
//   Ahat x Bhat u Bhat x Ahat (all pairs when Ahat is null):
//       S[a][b] += sum_{c < r} P[a][c] * P[b][c ^ 1]
// P rows hold (xi_k, eta_k) pairs, so the sum is sum_k xi_k[a] eta_k[b] + eta_k[a] xi_k[b].
// For several blocks the panel holds their pairs side by side (r = 2 (K+1) * blocks).
// Fused passes (fused = 1, no row list or mask) run as a GEMM over the upper triangle of
// 128 x 128 tiles, whatever r; it then needs nrows == ncols, r and pld multiples of 32,
// p_rows >= nrows rounded up to 128, with panel rows [nrows, p_rows) zero.
// Column-output form (out != null): out[t][b] = sum_c P[rows[t]][c] * P[b][c ^ 1] as float32
// (row t of out at out + t * ld_out), no mask; S is not touched.
struct LowRankArgs {
  SView S;
  const double* P;
  int32_t pld;        // doubles per panel row (multiple of 4)
  int32_t r;          // columns of the panel used (multiple of 2)
  const int32_t* rows;
  int64_t nrows;      // used when nrows_dev is null
  const int64_t* nrows_dev;
  int64_t ncols;
  const uint32_t* Ahat;
  const uint32_t* Bhat;
  float* out;
  int64_t ld_out;
  int64_t p_rows;     // rows allocated in P (rows past the written ones are zero)
  int64_t gstride;    // doubles between consecutive groups of pld columns (block-major
                      // batch panel); column c of row a is at (c / pld) gstride + a pld + c % pld
  double* acc_out;    // launch_lowrank_acc: float64 output, ld_out doubles per row
  int32_t fused;      // 1: a fused batch pass, always the symmetric GEMM (even at r = 32)
  // Fused passes: when set, the pass covers only the nodes act[0 .. *act_n) (ascending; the
  // nodes with a nonzero panel row in the pass, see launch_pass_rows): the others' rows and
  // columns of the update are exact zeros. The count is read on the device.
  const int32_t* act;
  const int64_t* act_n;
  int32_t variant;    // fused GEMM: tile variant (0 .. kGemmVariants - 1): float64 matrix
                      // cores with panel columns per LDS chunk and LDS pitch (16, 18),
                      // (16, 20), (32, 34), (32, 36); kGemmF32: float32 matrix cores
  // Fused passes over an active list, float64 matrix cores: when set, tflags[b tf_ld + t]
  // (launch_tile_flags) has bit g set when block b's columns 4 g and 4 g + 2 (xi_2g, xi_2g+1)
  // hold a nonzero on list positions 128 t .. 128 t + 127. The tile (I, J) then skips block
  // b's k-step g (its panel columns 4 g .. 4 g + 3) when neither tile has the bit: each of its
  // products has a zero xi factor.
  const uint32_t* tflags;
  int64_t tf_ld;
};
constexpr int kGemmF32 = 4;
constexpr int kGemmVariants = 5;
constexpr int kTileRows = 128;  // rows (list positions) of a fused-pass tile
hipError_t launch_lowrank(const LowRankArgs& a, hipStream_t s);
// Tile flags of a fused pass over the active list act[0 .. *act_n) (see LowRankArgs::tflags):
// for each of the q panel segments (gstride doubles apart, pld per row, pld / 4 <= 32 k-steps)
// and each tile t < ceil(*act_n / 128), flags[b tf_ld + t] gets bit g when xi_2g or xi_2g+1
// (columns 4 g, 4 g + 2) is nonzero on one of the tile's positions; for the first `steps`
// k-steps, skip[b steps + g] (zeroed by the caller) gains the positions of the tiles whose bit
// g is clear. n_max bounds *act_n; tf_ld >= ceil(n_max / 128).
hipError_t launch_tile_flags(const double* P, int pld, int64_t gstride, int q,
                             const int32_t* act, const int64_t* act_n, int64_t n_max,
                             uint32_t* flags, int64_t tf_ld, int32_t* skip, int steps,
                             hipStream_t s);
// The nodes a fused pass reaches: bit a of bm (ceil(n / 32) words, zeroed by the caller) is set
// when row a of any of the q panel segments (gstride doubles apart, pld per row) has a nonzero
// entry among its first w columns.
hipError_t launch_pass_rows(const double* P, int pld, int64_t gstride, int q, int w, int64_t n,
                            uint32_t* bm, hipStream_t s);
// Column mode, batches: acc_out[p][a] += sum_{c < r} P[rows[p]][c] P[a][c ^ 1] for list
// positions p < nrows and nodes a < ncols (the deferred blocks' Delta S[a][rows[p]], eq (71)),
// on FP64 matrix cores. P is block-major (gstride); r and pld multiples of 16; P holds at least
// ncols rounded up to 128 rows.
hipError_t launch_lowrank_acc(const LowRankArgs& a, hipStream_t s);
// Fused batches, incremental form. The blocks of a chunk that read columns of S take slots;
// slot s reads the sum of the columns I_s and the column j_s (j_s < 0: none), and keeps two
// correction vectors of the chunk's deferred terms, corr[2 (s - base)] and
// corr[2 (s - base) + 1], ldc doubles each. After a deferred block has written its panel
// segment Pseg (n rows of pld doubles; columns at or past 2(K+1) zero), slots s0 .. s1 - 1
// receive its part of those columns (eq (71) per column):
//   corr[2 (s - base)][a]     += sum_c Pseg[a][c] sum_{i in I_s} Pseg[i][c ^ 1]
//   corr[2 (s - base) + 1][a] += sum_c Pseg[a][c] Pseg[j_s][c ^ 1]
// pld must be 32 or 64 (other widths: hipErrorInvalidValue; the caller then corrects from
// the whole panel with launch_panel_correct). The caller caps the slots of a chunk.
struct CorrSlots {
  const int32_t* rstart;  // rows of slot s: rows[rstart[s] .. rstart[s + 1])
  const int32_t* rows;
  const int32_t* sink;    // j_s or -1
  double* corr;
  int64_t ldc;
  int32_t base;           // first slot of the chunk
  double* w;              // scratch: 2 (s1 - s0) pld doubles
};
hipError_t launch_corr_update(const double* Pseg, int pld, int64_t n, const CorrSlots& c,
                              int s0, int s1, hipStream_t s);
// Fused batches: the columns S_t[:, c] of the current S are the stored S plus the deferred
// blocks' terms sum_{col < r} P[:, col] P[c, col ^ 1]. wts[col] = sum_{i in I} P[i][col ^ 1]
// and wts[r + col] = P[j][col ^ 1] (j < 0: no second vector), then
// SI[a] += sum_col P[a][col] wts[col] (when I nonempty), Sj[a] += sum_col P[a][col] wts[r+col].
// P is block-major: column col of row a at (col / pld) gstride + a pld + col % pld.
hipError_t launch_panel_correct(const double* P, int pld, int64_t gstride, int r, int64_t n,
                                const IdList& I, int32_t j, double* wts, double* SI,
                                double* Sj, hipStream_t s);
// out[a] = sum_{c < r} P[a][c] * P[x][c ^ 1] for a < n (Delta S[:, x], eq (71)), float64.
hipError_t launch_delta_col(const double* P, int pld, int r, int64_t n, int32_t x, double* out,
                            hipStream_t s);

// ---------------------------------------------------------------------------------------
// Adjoint (edge-weight gradient). Dense matrices use leading dimension round_up(n, 64).
// G[a][b] += g and G[b][a] += g for every pair (the symmetric part of dL/dS, doubled).
hipError_t launch_scatter_pairs_sym(double* G, int64_t n, int64_t np, const int32_t* a,
                                    const int32_t* b, const double* g, hipStream_t s);
// Y[b][:] = scale * (Q^T X)[b][:] (+ Gadd[b][:] when Gadd != null); maxdiff vs prev as above.
// qv: the values Q[a][b] of the out-list slots (launch_qt_values).
hipError_t launch_spmm_qt_rows(const DevAdj& out, const double* qv, int64_t n, const double* X,
                               double* Y, double scale, const double* Gadd, const double* prev,
                               unsigned long long* maxdiff, hipStream_t s);
// qv[p] = Q[a][b] for every out-list slot p of the rows b < n (a the slot's node).
hipError_t launch_qt_values(const DevQ& q, const DevAdj& out, int64_t n, double* qv,
                            hipStream_t s);
// Per sink x and in-list slot p (source y): dq[p] = C * <Sig[x, :], T[y, :]>, then
// dw[slot_edge[p]] = (dq[p] - sum_p' Q[x][y_p'] dq[p']) / W_x (W_x = in-degree unweighted).
hipError_t launch_edge_grad(const DevQ& q, int64_t n, const double* Sig, const double* T,
                            double C, const int32_t* slot_edge, double* dq, double* dw,
                            hipStream_t s);
// Small helpers.
// x = sum of e_i over the ids (distinct); with dq, also xd[a] = x[a] / d[a], d the in-degree
// (or the in-weight sum when weighted), 0 where d[a] = 0.
hipError_t launch_indicator(double* x, int64_t n, const IdList& ids, hipStream_t s,
                            const DevQ* dq = nullptr, double* xd = nullptr);
// Pairs (indicator of a, indicator of b) at x2[2 v], x2[2 v + 1], and x2 / d at xd2.
hipError_t launch_indicator2(double* x2, int64_t n, const IdList& a, const IdList& b,
                             hipStream_t s, const DevQ& dq, double* xd2);
// Top-k of S row q[t] (or of vecs + t * ldv when vecs is set), ties to the smaller id, x
// itself left out with exclude_self: out_idx / out_val[t * k + r], r < k, best first.
constexpr int kTopkMax = 3072;
hipError_t launch_topk(const SView& S, const double* vecs, int64_t ldv, const int32_t* q,
                       int nq, int64_t n, int k, int exclude_self, int32_t* out_idx,
                       double* out_val, hipStream_t s);
// Places a block's float64 S at its nodes' rows and columns of the store.
hipError_t launch_place_block(SView S, const int32_t* gid, int64_t nb, const double* Sb,
                              int64_t ldb, hipStream_t s);
// Writes S of a spanning forest (parent[v] = -1 for a root; depth[v] its level) into the
// n x n block of the store by Example 1.2's closed form.
hipError_t launch_tree_init(SView S, int64_t n, const int32_t* parent, const int32_t* depth,
                            double C, hipStream_t s);
// ---------------------------------------------------------------------------------------
// Block store (Example 1.1): S kept per pair of partition blocks instead of as one n x n
// matrix. Block p holds the nodes mem[mem_off[p] .. mem_off[p] + mem_n[p]) (ascending ids);
// part[a] is a's block and loc[a] its position there. pairs[p * np + q] (p <= q) is the
// dense mem_n[p] x mem_n[q] sub-matrix S[mem_p][mem_q] (row-major, ld = mem_n[q], the
// store's precision), or a view with null pointers when the pair holds no nonzero entry;
// entries with p > q are read from pair (q, p), transposed. The diagonal pairs hold S_old's
// blocks S_Gi; the others only the Delta S of cross-block updates.
struct BlockStore {
  const SView* pairs;
  int32_t np;
  const int32_t* part;
  const int32_t* loc;
  const int32_t* mem;
  const int64_t* mem_off;
  const int32_t* mem_n;
};
// One 128 x 128 tile (ti, tj) of pair (p, q), p <= q (ti <= tj when p == q).
struct BsItem {
  int32_t p, q, ti, tj;
};
// SI[a] = sum over I of S[i][a] (+ cI[a]), Sj[a] = S[j][a] (+ cJ[a]), a < n (j < 0: none).
hipError_t launch_bs_gather_rows(const BlockStore& B, int64_t n, const IdList& I, int32_t j,
                                 double* SI, double* Sj, const double* cI, const double* cJ,
                                 hipStream_t s);
// Rows of S as dense vectors: out[t * ld_out + a] = S[rows[t]][a] (float64, or float32 when
// out32 is set), t < nrows, a < n.
hipError_t launch_bs_rows(const BlockStore& B, int64_t n, const int32_t* rows, int64_t nrows,
                          double* out, float* out32, int64_t ld_out, hipStream_t s);
// out[t] = S[a[t]][b[t]], t < cnt.
hipError_t launch_bs_pairs(const BlockStore& B, int64_t cnt, const int32_t* a,
                           const int32_t* b, double* out, hipStream_t s);
// Which blocks the deferred blocks of a fused pass reach: for deferred block d < q (panel
// segment d, gstride doubles apart, pld doubles per row, columns 2k = xi_k, 2k + 1 = eta_k,
// k < nk) and node a < n with a nonzero xi_k (eta_k) entry,
// flags[((d * np + part[a]) * nk + k) * 2] ([... + 1]) is set to 1. flags must hold
// q * np * nk * 2 words, zeroed by the caller.
hipError_t launch_bs_touch(const double* P, int pld, int64_t gstride, int q, int nk, int64_t n,
                           const int32_t* part, int32_t np, uint32_t* flags, hipStream_t s);
// Writes a block's float64 S (nb x nb, ld ldb) into its diagonal pair view.
hipError_t launch_bs_place(SView dst, const double* Sb, int64_t ldb, int64_t nb,
                           hipStream_t s);
// Fused pass into the block store: for every listed tile, S[mem_p rows][mem_q cols] +=
// sum_{c < r} P[a][c] P[b][c ^ 1] over the panel a.P (block-major, a.pld, a.gstride; r a
// multiple of 16), mirrored inside diagonal pairs so that they stay exactly symmetric.
hipError_t launch_bs_gemm(const LowRankArgs& a, const BlockStore& B, const BsItem* items,
                          int64_t nitems, hipStream_t s);

hipError_t launch_fill_diag(double* A, int64_t n, int64_t ld, double v, hipStream_t s);
hipError_t launch_diag_range(SView S, int64_t lo, int64_t hi, double v, hipStream_t s);
hipError_t launch_mfma_probe(const double* a, const double* b, double* out, hipStream_t s);
hipError_t launch_mfma_probe_f32(const float* a, const float* b, float* out, hipStream_t s);

}  // namespace sr
