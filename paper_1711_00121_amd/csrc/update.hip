// The S update of the incremental method: S <- S + M_K + M_K^T restricted to the affected
// areas (Algorithm 1 final line; Algorithm 2 with the union-rectangle reading), where
// M_K = sum_k xi_k eta_k^T (eq (16a)). Entry (a, b) receives
//     sum_k xi_k[a] eta_k[b] + eta_k[a] xi_k[b] = sum_c P[a][c] P[b][c ^ 1]
// with panel rows P[a] = (xi_0[a], eta_0[a], xi_1[a], eta_1[a], ...). Several blocks of a batch
// stack their pairs along c, so the same product applies a rank-2(K+1)B update in one pass.
//
// Three kernels, all on v_mfma_f64_16x16x4_f64 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator slot v of lane l is D[4v + l/16][l%16]):
//  - lowrank_strip_kernel, one block (r <= 32): bound by HBM. S streams through once; the
//    S loads of the next row tile are in flight while the current tile multiplies and stores.
//  - lowrank_cols_kernel, columns of Delta S for the column-by-column method (r <= 32, float32
//    output): bound by FP64 matrix throughput and the output writes.
//  - lowrank_gemm_kernel, fused batches (r = 32 B): bound by FP64 matrix throughput. Only
//    the upper triangle of tiles is computed (the update is symmetric). xi_k vanishes outside
//    the nodes k out-steps from the block's sink (the A_k of Theorem 4), so over a pass's
//    reached nodes a tile skips the early k-steps of the blocks whose xi columns are zero on
//    both of its row ranges (tile_flags_kernel marks them).
#include "kernels.h"

namespace sr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TR = 64;    // tile rows (positions in the row list)
constexpr int RC = 32;    // panel columns staged per pass
constexpr int LP = RC + 1;  // LDS row pitch in doubles (odd pitch spreads banks)
constexpr int NT = 256;

// An S entry as loaded (no arithmetic on it until it is needed, so that the load can stay in
// flight): FP64 value, or FP32 value and compensation.
template <int PREC>
struct Raw {
  double d;
  float2 hl;
  float h;
};

// NT: non-temporal store (S entries that one launch writes exactly once).
typedef float nt_float2 __attribute__((ext_vector_type(2)));

template <int PREC>
__device__ __forceinline__ void sload(const SView& S, int64_t off, Raw<PREC>& x) {
  if constexpr (PREC == PREC_FP64) {
    x.d = S.d[off];
  } else if constexpr (PREC == PREC_HILO) {
    x.hl = S.hl[off];
  } else {
    x.h = S.hi[off];
  }
}

template <int PREC>
__device__ __forceinline__ double sval(const Raw<PREC>& x) {
  if constexpr (PREC == PREC_FP64) return x.d;
  else if constexpr (PREC == PREC_HILO) return (double)x.hl.x + (double)x.hl.y;
  else return (double)x.h;
}

template <int PREC, bool NT = false>
__device__ __forceinline__ void sput(const SView& S, int64_t off, double t) {
  if constexpr (PREC == PREC_FP64) {
    if constexpr (NT) __builtin_nontemporal_store(t, S.d + off);
    else S.d[off] = t;
  } else if constexpr (PREC == PREC_HILO) {
    const float h = (float)t;
    const float l = (float)(t - (double)h);
    if constexpr (NT) {
      const nt_float2 v = {h, l};
      __builtin_nontemporal_store(v, reinterpret_cast<nt_float2*>(S.hl + off));
    } else {
      S.hl[off] = make_float2(h, l);
    }
  } else {
    if constexpr (NT) __builtin_nontemporal_store((float)t, S.hi + off);
    else S.hi[off] = (float)t;
  }
}

// Stores an entry back exactly as it was loaded.
template <int PREC, bool NT = false>
__device__ __forceinline__ void sraw(const SView& S, int64_t off, const Raw<PREC>& x) {
  if constexpr (PREC == PREC_FP64) {
    if constexpr (NT) __builtin_nontemporal_store(x.d, S.d + off);
    else S.d[off] = x.d;
  } else if constexpr (PREC == PREC_HILO) {
    if constexpr (NT) {
      const nt_float2 v = {x.hl.x, x.hl.y};
      __builtin_nontemporal_store(v, reinterpret_cast<nt_float2*>(S.hl + off));
    } else {
      S.hl[off] = x.hl;
    }
  } else {
    if constexpr (NT) __builtin_nontemporal_store(x.h, S.hi + off);
    else S.hi[off] = x.h;
  }
}

// Streaming update for one block (r <= RC panel columns). Workgroup = strip of SC columns whose
// panel rows live in LDS for the whole strip; the workgroup walks row tiles of TR listed rows,
// wave w taking rows [16 w, 16 w + 16) of each tile against the strip's SC columns (ST
// accumulators of 16 x 16). Per tile a wave first issues the A fragments and S loads of its
// NEXT tile and the row-list entries of the tile after that, then runs the MFMAs and stores
// the current tile from values loaded one iteration earlier. Each wave thus keeps a tile of
// S loads in flight while it computes and stores, which HBM latency at full bandwidth needs;
// and since the waits count loads in issue order, waiting for the current tile's operands
// never waits for the next tile's.
// Every load is unconditional from an in-bounds address (rows past the list read row 0;
// columns past n stay inside the padded leading dimension, a multiple of SC) and selected
// afterwards: a load under a branch is followed by a full wait and serialises the tile.
constexpr int SC = 64;
constexpr int ST = SC / 16;
// The updated entries are stored non-temporally (measured: 8% faster at n = 20k and 50k);
// non-temporal loads of the same entries were 30-50% slower.
constexpr bool kStripNTStore = true;

template <int PREC, bool MASK, bool HASROWS, bool FULL = false>
__global__ __launch_bounds__(NT) void lowrank_strip_kernel(LowRankArgs g) {
  __shared__ double lcol[SC * LP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * SC;

  {
    double2 vv[SC * (RC / 2) / NT];
#pragma unroll
    for (int u = 0; u < SC * (RC / 2) / NT; ++u) {
      const int e = tid + u * NT;
      const int rr = e / (RC / 2), cc = (e % (RC / 2)) * 2;
      const int64_t b = c0 + rr;
      const bool ok = b < g.ncols && cc < g.r;
      vv[u] = *reinterpret_cast<const double2*>(g.P + (ok ? b * g.pld + cc : 0));
      if (!ok) vv[u] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < SC * (RC / 2) / NT; ++u) {
      const int e = tid + u * NT;
      const int rr = e / (RC / 2), cc = (e % (RC / 2)) * 2;
      lcol[rr * LP + cc] = vv[u].x;
      lcol[rr * LP + cc + 1] = vv[u].y;
    }
  }
  // Column flags of this lane's 16-column slices, one bit per slice t.
  int cin = 0, cA = 0, cB = 0;
#pragma unroll
  for (int t = 0; t < ST; ++t) {
    const int64_t b = c0 + t * 16 + l16;
    const int in = b < g.ncols;
    cin |= in << t;
    if (MASK) {
      const int64_t bb = in ? b : 0;
      const uint32_t wa = g.Ahat[bb >> 5], wb = g.Bhat[bb >> 5];
      cA |= (int)((wa >> (bb & 31)) & 1u) << t;
      cB |= (int)((wb >> (bb & 31)) & 1u) << t;
    }
  }
  if (!MASK) cA = cB = (1 << ST) - 1;
  __syncthreads();

  const int64_t nrows = g.nrows_dev ? *g.nrows_dev : g.nrows;
  const int64_t nrt = (nrows + TR - 1) / TR;
  const int64_t gy = gridDim.y;
  const int64_t last = nrows > 0 ? nrows - 1 : 0;
  // Row-list entries of a tile: [0] the A-operand row (rbase + l16), [1..4] the accumulator
  // rows (rbase + 4 v + lk). Positions past the list read the last entry (any in-bounds row).
  auto fetch = [&](int64_t rt, int32_t (&e)[5]) {
    const int64_t rbase = rt * TR + wave * 16;
    const int64_t p0 = rbase + l16;
    e[0] = HASROWS ? g.rows[p0 < nrows ? p0 : last] : (int32_t)p0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t pc = rbase + v * 4 + lk;
      e[1 + v] = HASROWS ? g.rows[pc < nrows ? pc : last] : (int32_t)pc;
    }
  };
  // Output row of accumulator slot v: the node (with a mask the entry is packed as
  // (node << 2) | (in A_hat << 1) | in B_hat).
  auto out_row = [&](int64_t rt, const int32_t (&e)[5], int v) -> int64_t {
    const int64_t pc = rt * TR + wave * 16 + v * 4 + lk;
    const int64_t rr = MASK ? ((int64_t)e[1 + v] >> 2) : (int64_t)e[1 + v];
    return pc < nrows ? rr : 0;
  };
  auto load_tile = [&](int64_t rt, const int32_t (&e)[5], Raw<PREC> (&x)[ST][4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t base = out_row(rt, e, v) * g.S.ld + c0 + l16;
#pragma unroll
      for (int t = 0; t < ST; ++t) sload<PREC>(g.S, base + t * 16, x[t][v]);
    }
  };

  // A operand of a tile: row (rbase + l16) of the panel; k-step ks of lane group lk uses
  // panel column 4 ks + lk, so only ceil(r / 4) k-steps run (r = 22 at K = 10). No select is
  // applied: positions past the list read row 0 and their output rows are never stored, and
  // panel columns at or past r meet zeros on the B side (staged above).
  auto load_a = [&](int64_t rt, const int32_t (&e)[5], double (&av)[RC / 4]) {
    const int64_t p0 = rt * TR + wave * 16 + l16;
    const int64_t arow = p0 < nrows ? ((int64_t)e[0] >> (MASK ? 2 : 0)) : 0;
    const double* src = g.P + arow * g.pld + lk;
#pragma unroll
    for (int ks = 0; ks < RC / 4; ++ks) av[ks] = src[4 * ks];
  };
  const int ksteps = (g.r + 3) / 4;

  // Pipeline: iteration rt holds the entries, S values and A operand of tile rt (loaded one
  // iteration earlier) and issues those of tile rt + gy (entries: rt + 2 gy) before its MFMAs.
  int32_t e0[5], e1[5], e2[5];
  Raw<PREC> x0[ST][4], x1[ST][4];
  double a0[RC / 4], a1[RC / 4];
  int64_t rt = blockIdx.y;
  fetch(rt, e0);
  load_tile(rt, e0, x0);
  load_a(rt, e0, a0);
  fetch(rt + gy, e1);
  for (; rt < nrt; rt += gy) {
    const int64_t rbase = rt * TR + wave * 16;
    load_a(rt + gy, e1, a1);
    load_tile(rt + gy, e1, x1);
    fetch(rt + 2 * gy, e2);
    dbl4 acc[ST];
#pragma unroll
    for (int t = 0; t < ST; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < RC / 4; ++ks) {
      if (ks >= ksteps) break;  // uniform
      const int c = (4 * ks + lk) ^ 1;
#pragma unroll
      for (int t = 0; t < ST; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[ks], lcol[(t * 16 + l16) * LP + c],
                                                      acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t pc = rbase + v * 4 + lk;
      const int64_t row = out_row(rt, e0, v);
      const int rok = pc < nrows;
      const int rA = MASK ? ((e0[1 + v] >> 1) & 1) : 1;
      const int rB = MASK ? (e0[1 + v] & 1) : 1;
      // pairs in A_hat x B_hat u B_hat x A_hat, as a bit per slice
      const int on = (rok ? cin : 0) & ((rA ? cB : 0) | (rB ? cA : 0));
      if constexpr (FULL) {
        // a slice with any pair of this row is written whole: its other entries go back
        // exactly as loaded, so each row's line is written in full
        int whole = 0;
#pragma unroll
        for (int t = 0; t < ST; ++t) {
          const uint64_t bal = __ballot((on >> t) & 1);
          whole |= (((bal >> (16 * lk)) & 0xFFFFull) != 0 ? 1 : 0) << t;
        }
        whole &= (rok ? cin : 0);
#pragma unroll
        for (int t = 0; t < ST; ++t) {
          if (!((whole >> t) & 1)) continue;
          const int64_t off = row * g.S.ld + c0 + t * 16 + l16;
          if ((on >> t) & 1)
            sput<PREC, kStripNTStore>(g.S, off, sval<PREC>(x0[t][v]) + acc[t][v]);
          else
            sraw<PREC, kStripNTStore>(g.S, off, x0[t][v]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < ST; ++t) {
          if (!((on >> t) & 1)) continue;
          const int64_t b = c0 + t * 16 + l16;
          sput<PREC, kStripNTStore>(g.S, row * g.S.ld + b, sval<PREC>(x0[t][v]) + acc[t][v]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      e0[q] = e1[q];
      e1[q] = e2[q];
    }
#pragma unroll
    for (int q = 0; q < RC / 4; ++q) a0[q] = a1[q];
#pragma unroll
    for (int t = 0; t < ST; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) x0[t][v] = x1[t][v];
  }
}

// Fused batch pass (any r that is a multiple of GC, all rows and columns, no mask):
// S += P swap(P)^T as a GEMM with inner dimension r. The product is symmetric
// (sum_c P[a][c] P[b][c^1] = sum_c P[b][c] P[a][c^1]), so only tiles (I, J) with I <= J of the
// 128 x 128 tiling are computed: a diagonal tile adds its product to S[I][I], an
// off-diagonal tile adds it to S[I][J] and its transpose to S[J][I]. That halves the matrix
// work and keeps S exactly symmetric. Wave (wr, wc) owns a 64 x 64 quarter (4 x 4
// accumulators of 16 x 16). Panel columns are staged through LDS GC at a time, double
// buffered: the global loads of chunk c + 1 are issued before the MFMAs of chunk c and land
// in LDS after them. The global panel loads are unconditional (the panel holds zero rows up
// to a multiple of GT and zero columns up to a multiple of GC), so the loop has no branch.
// With GC = 16 two workgroups share a CU (74 KB of LDS and at most 256 registers each), so
// one workgroup's barrier and LDS staging overlap the other's MFMAs; with GC = 32 a
// workgroup takes a CU alone and waits at half as many barriers. The chunk width GC and the
// LDS pitch GP are template parameters chosen at run time among the instantiated variants
// (kGemmVariants; the autotuner times them).
// Workgroups are dealt to the 8 XCDs round-robin; workgroup w takes triangle tile
// (w % 8) * per + w / 8, so each XCD walks a contiguous run of tiles (mostly one tile row)
// and shares that row's panel in its L2. The column panels are not shared: measured at
// n = 58k-92k, the fabric fetch per pass is ~20x the algorithmic bytes (S once, panel once),
// ~2.9 TB/s beside 0.86 of the FP64 matrix peak. An order in 8 x 8 super-tiles, which cuts
// the panel slices per XCD from ~65 to 16, measured 2.4% slower: the pass is bound by the
// matrix cores, not by these re-reads.
constexpr int GT = 128;       // tile rows = tile cols
constexpr int GC = 16;        // panel columns per chunk of the default variant (and of kRect, kBlk)
// LDS pitch in doubles. A wave reads 16 rows x 4 columns per operand; with 64 four-byte banks
// a half-wave (16 rows x 2 columns) touches 32 distinct doubles when 18 * row mod 32 spreads
// the rows over the even double slots, so the reads are free of bank conflicts.
constexpr int GP = 18;
constexpr int NXCD = 8;

// Tile t of the upper triangle of a T x T tiling, row by row: row I holds (I, I..T-1) and
// starts at I T - I (I - 1) / 2.
__device__ __forceinline__ void tri_tile(int64_t t, int64_t T, int64_t& I, int64_t& J) {
  const double b = 2.0 * (double)T + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  i = i < 0 ? 0 : (i > T - 1 ? T - 1 : i);
  while (i > 0 && i * T - i * (i - 1) / 2 > t) --i;
  while (i + 1 < T && (i + 1) * T - (i + 1) * i / 2 <= t) ++i;
  I = i;
  J = i + (t - (i * T - i * (i - 1) / 2));
}

constexpr int64_t kRectGroup = 8;

// Modes of lowrank_gemm_kernel.
constexpr int kSym = 0;   // fused pass into the dense S (upper triangle of tiles, mirrored)
constexpr int kRect = 1;  // column-mode batches: accumulate into a float64 output
constexpr int kBlk = 2;   // fused pass into the block store
constexpr int kSymAct = 3;  // kSym over the nodes of an active list (LowRankArgs::act)

// kRect (column mode, batches): a rectangular product accumulated into a float64 output,
//     acc_out[p][a] += sum_{c < r} P[rows[p]][c] P[a][c ^ 1]   (p < nrows, a < ncols),
// over T row tiles (list positions) x TJ column tiles (nodes), without the symmetry; A rows
// are gathered through the list (positions past it read its last entry, not stored).
// kBlk: one workgroup per listed tile (ti, tj) of a block pair (p, q); A rows are the members
// of block p from 128 ti on, B rows those of block q from 128 tj on (positions past a
// block read its last member and are not stored), and the product is added to the pair's
// sub-matrix; inside a diagonal pair (p == q, ti <= tj) the mirrored entry is written from
// the same sum, and a diagonal tile stores a <= b only, as the symmetric mode does.
// GCt: panel columns per LDS chunk; GPt: LDS row pitch in doubles; WPC: workgroups per CU.
template <int PREC, int MODE = kSym, int GCt = GC, int GPt = GP, int WPC = 2>
__global__ __launch_bounds__(NT, WPC) void lowrank_gemm_kernel(LowRankArgs g, int64_t T,
                                                            int64_t per, int64_t TJ = 0,
                                                            BlockStore bs = {},
                                                            const BsItem* items = nullptr) {
  constexpr int GL = GT * (GCt / 2) / NT;  // double2 loads per thread per side per chunk
  constexpr int GR = NT / (GCt / 2);       // rows staged per load round
  __shared__ double As[2][GT * GPt];
  __shared__ double Bs[2][GT * GPt];
  const int64_t w = blockIdx.x;
  const int64_t t = (w % NXCD) * per + w / NXCD;
  int64_t I, J;
  [[maybe_unused]] int32_t bp = 0, bq = 0;
  [[maybe_unused]] int64_t cnt = 0;
  if constexpr (MODE == kSymAct) {
    // the triangle of the list's tiles, dealt to the XCDs as in kSym (the grid is sized for
    // the whole node range; workgroups past the list's share return)
    cnt = *g.act_n;
    const int64_t Ta = (cnt + GT - 1) / GT;
    const int64_t tiles = Ta * (Ta + 1) / 2;
    const int64_t pa = (tiles + NXCD - 1) / NXCD;
    if (w / NXCD >= pa) return;
    const int64_t ta = (w % NXCD) * pa + w / NXCD;
    if (ta >= tiles) return;
    tri_tile(ta, Ta, I, J);
  } else if constexpr (MODE == kBlk) {
    if (t >= T) return;  // T: the number of listed tiles
    const BsItem it = items[t];
    bp = it.p;
    bq = it.q;
    I = it.ti;
    J = it.tj;
  } else if constexpr (MODE == kRect) {
    // Tiles in groups of kRectGroup row tiles, column-major inside a group: the workgroups
    // running together on one XCD share one column tile (a slice of the panel, read from HBM
    // once per group) and the group's row tiles (gathered rows, small enough to stay cached).
    if (t >= T * TJ) return;
    const int64_t gsz = kRectGroup * TJ;
    const int64_t grp = t / gsz, in = t % gsz;
    const int64_t gm = (T - grp * kRectGroup) < kRectGroup ? (T - grp * kRectGroup) : kRectGroup;
    I = grp * kRectGroup + in % gm;
    J = in / gm;
  } else {
    if (t >= T * (T + 1) / 2) return;
    tri_tile(t, T, I, J);
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  const int64_t r0 = I * GT;
  const int64_t c0 = J * GT;
  const int nch = g.r / GCt;

  // This thread stages rows lrow + GR u, columns lcol + {0, 1} of each chunk.
  const int lrow = tid / (GCt / 2), lcol = 2 * (tid % (GCt / 2));
  const double* pa = g.P + (r0 + lrow) * (int64_t)g.pld + lcol;
  const double* pb = g.P + (c0 + lrow) * (int64_t)g.pld + lcol;
  const int64_t ustep = GR * (int64_t)g.pld;
  // kRect: the A rows of this thread, gathered through the list; kBlk: the A and B rows,
  // gathered through the two blocks' member lists
  constexpr bool GA = MODE != kSym;
  constexpr bool GB = MODE == kBlk || MODE == kSymAct;
  int64_t arow[GA ? GL : 1], brow[GB ? GL : 1];
  [[maybe_unused]] int64_t na = 0, nb = 0;
  if constexpr (MODE == kRect) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int64_t p = r0 + lrow + GR * u;
      arow[u] = (int64_t)g.rows[p < g.nrows ? p : g.nrows - 1] * g.pld + lcol;
    }
  } else if constexpr (MODE == kSymAct) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int64_t p = r0 + lrow + GR * u, q = c0 + lrow + GR * u;
      arow[u] = (int64_t)g.act[p < cnt ? p : cnt - 1] * g.pld + lcol;
      brow[u] = (int64_t)g.act[q < cnt ? q : cnt - 1] * g.pld + lcol;
    }
  } else if constexpr (MODE == kBlk) {
    const int32_t* ma = bs.mem + bs.mem_off[bp];
    const int32_t* mb = bs.mem + bs.mem_off[bq];
    na = bs.mem_n[bp];
    nb = bs.mem_n[bq];
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int64_t p = r0 + lrow + GR * u, q = c0 + lrow + GR * u;
      arow[u] = (int64_t)ma[p < na ? p : na - 1] * g.pld + lcol;
      brow[u] = (int64_t)mb[q < nb ? q : nb - 1] * g.pld + lcol;
    }
  }
  double2 ra[GL], rb[GL];
  auto load = [&](int ch) {
    // chunk ch: columns [ch GCt, ch GCt + GCt) lie in column group (ch GCt) / pld
    const int64_t cb = (int64_t)((ch * GCt) / g.pld) * g.gstride + (ch * GCt) % g.pld;
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      if constexpr (GA)
        ra[u] = *reinterpret_cast<const double2*>(g.P + arow[u] + cb);
      else
        ra[u] = *reinterpret_cast<const double2*>(pa + u * ustep + cb);
      if constexpr (GB)
        rb[u] = *reinterpret_cast<const double2*>(g.P + brow[u] + cb);
      else
        rb[u] = *reinterpret_cast<const double2*>(pb + u * ustep + cb);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int o = (lrow + GR * u) * GPt + lcol;
      As[buf][o] = ra[u].x;
      As[buf][o + 1] = ra[u].y;
      Bs[buf][o] = rb[u].x;
      Bs[buf][o + 1] = rb[u].y;
    }
  };

  dbl4 acc[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[s][q] = dbl4{0.0, 0.0, 0.0, 0.0};

  // kSymAct with tile flags: the k-steps of a block whose xi factors vanish on both tiles are
  // skipped (exact zeros, so the sums are bit for bit those of the full loop)
  [[maybe_unused]] const uint32_t* tfI = nullptr;
  [[maybe_unused]] const uint32_t* tfJ = nullptr;
  if constexpr (MODE == kSymAct) {
    if (g.tflags) {
      tfI = g.tflags + I;
      tfJ = g.tflags + J;
    }
  }

  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    // the last chunk reloads itself (uniform, harmless) so the loop body has no branch
    load(ch + 1 < nch ? ch + 1 : ch);
    uint32_t live = ~0u;  // bit u: k-step u of this chunk runs
    if constexpr (MODE == kSymAct) {
      if (tfI) {
        const int64_t o = (int64_t)((ch * GCt) / g.pld) * g.tf_ld;
        live = (tfI[o] | tfJ[o]) >> (((ch * GCt) % g.pld) / 4);
        live = __builtin_amdgcn_readfirstlane(live);
      }
    }
    auto step = [&](int k4) {
      const int c = k4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) av[s] = As[buf][(wr * 64 + s * 16 + l16) * GPt + c];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Bs[buf][(wc * 64 + q * 16 + l16) * GPt + (c ^ 1)];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[s][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[q], acc[s][q], 0, 0, 0);
    };
    // (a second, branch-free copy of the loop for chunks with every k-step live spilled
    // accumulators to scratch inside the loop)
#pragma unroll
    for (int k4 = 0; k4 < GCt; k4 += 4)
      if ((live >> (k4 / 4)) & 1u) step(k4);
    // keep the staging stores (and their wait for the global loads) after the MFMAs
    __builtin_amdgcn_sched_barrier(0);
    store(buf ^ 1);
    __syncthreads();
  }

  if constexpr (MODE == kBlk) {
    // the pair's sub-matrix += acc, one row sub-tile at a time (loads first, then stores);
    // inside a diagonal pair the mirrored entry goes with it
    const SView o = bs.pairs[(int64_t)bp * bs.np + bq];
    const bool mir = bp == bq;
    const bool diag = mir && I == J;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      Raw<PREC> x[4][4], y[4][4];
      int on[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t a = r0 + wr * 64 + s * 16 + v * 4 + lk;
          const int64_t b = c0 + wc * 64 + q * 16 + l16;
          on[q][v] = a < na && b < nb;
          sload<PREC>(o, on[q][v] ? a * o.ld + b : 0, x[q][v]);
          if (mir) sload<PREC>(o, on[q][v] ? b * o.ld + a : 0, y[q][v]);
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (!on[q][v]) continue;
          const int64_t a = r0 + wr * 64 + s * 16 + v * 4 + lk;
          const int64_t b = c0 + wc * 64 + q * 16 + l16;
          const double d = acc[s][q][v];
          if (!diag || a <= b) sput<PREC>(o, a * o.ld + b, sval<PREC>(x[q][v]) + d);
          if (mir && (!diag || a < b)) sput<PREC>(o, b * o.ld + a, sval<PREC>(y[q][v]) + d);
        }
    }
    return;
  }

  if constexpr (MODE == kRect) {
    // acc_out[p][a] += acc, one row sub-tile at a time (loads first, then the stores)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double x[4][4];
      int on[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t p = r0 + wr * 64 + s * 16 + v * 4 + lk;
          const int64_t b = c0 + wc * 64 + q * 16 + l16;
          on[q][v] = p < g.nrows && b < g.ncols;
          x[q][v] = g.acc_out[on[q][v] ? p * g.ld_out + b : 0];
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (!on[q][v]) continue;
          const int64_t p = r0 + wr * 64 + s * 16 + v * 4 + lk;
          const int64_t b = c0 + wc * 64 + q * 16 + l16;
          g.acc_out[p * g.ld_out + b] = x[q][v] + acc[s][q][v];
        }
    }
    return;
  }

  // S[a][b] += acc and S[b][a] += acc, one row sub-tile at a time: the direct and the
  // mirrored loads of a sub-tile are issued together (one memory round trip per sub-tile),
  // then both stores. A diagonal tile computes both (a, b) and (b, a), whose sums the matrix
  // cores may round differently; there only a <= b is stored, with its mirror, so S stays
  // exactly symmetric. Loads are unconditional from clamped addresses; out-of-range entries
  // are not stored.
  // (kSymAct: positions in the list; the entries are those of the listed nodes, and since the
  // list ascends, position order is node order for the diagonal rule.)
  const bool diag = I == J;
  const int64_t lim_r = MODE == kSymAct ? cnt : g.nrows;
  const int64_t lim_c = MODE == kSymAct ? cnt : g.ncols;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    Raw<PREC> x[4][4], y[4][4];
    int on[4][4];
    int64_t an[4], bn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t p = r0 + wr * 64 + s * 16 + v * 4 + lk;
      an[v] = MODE == kSymAct ? (int64_t)g.act[p < cnt ? p : 0] : p;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p = c0 + wc * 64 + q * 16 + l16;
      bn[q] = MODE == kSymAct ? (int64_t)g.act[p < cnt ? p : 0] : p;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t pr = r0 + wr * 64 + s * 16 + v * 4 + lk;
        const int64_t pc = c0 + wc * 64 + q * 16 + l16;
        on[q][v] = pr < lim_r && pc < lim_c;
        const int64_t da = on[q][v] ? an[v] * g.S.ld + bn[q] : 0;
        const int64_t ma = on[q][v] ? bn[q] * g.S.ld + an[v] : 0;
        sload<PREC>(g.S, da, x[q][v]);
        sload<PREC>(g.S, ma, y[q][v]);
      }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (!on[q][v]) continue;
        const int64_t pr = r0 + wr * 64 + s * 16 + v * 4 + lk;
        const int64_t pc = c0 + wc * 64 + q * 16 + l16;
        const double d = acc[s][q][v];
        if (!diag || pr <= pc) sput<PREC>(g.S, an[v] * g.S.ld + bn[q], sval<PREC>(x[q][v]) + d);
        if (!diag || pr < pc) sput<PREC>(g.S, bn[q] * g.S.ld + an[v], sval<PREC>(y[q][v]) + d);
      }
  }
}

// Fused batch pass on the FP32 matrix cores (tile variant kGemmF32): the same tiling and
// symmetric epilogue as lowrank_gemm_kernel, with the panel rounded to float when it is
// staged (32 columns per chunk, LDS pitch 33 floats: a half-wave's 16 rows x 2 columns fall on
// 32 distinct banks) and v_mfma_f32_16x16x4f32, whose accumulator slot v of lane l holds row
// 4 (l / 16) + v of the 16 x 16 block (the float64 instruction's is 4 v + l / 16). The float
// sum is added to the stored value in float64 and stored as the store's precision keeps it
// (value + compensation re-split), so long streams accumulate without loss, but each pass
// carries the rounding of float products and sums.
constexpr int GCF = 32;
constexpr int GPF = GCF + 1;
typedef float fl4 __attribute__((ext_vector_type(4)));

template <int PREC, bool ACT = false>
__global__ __launch_bounds__(NT, 2) void lowrank_gemm_f32_kernel(LowRankArgs g, int64_t T,
                                                              int64_t per) {
  constexpr int GL = GT * (GCF / 2) / NT;  // double2 loads per thread per side per chunk (8)
  constexpr int GR = NT / (GCF / 2);       // rows staged per load round (16)
  __shared__ float As[2][GT * GPF];
  __shared__ float Bs[2][GT * GPF];
  const int64_t w = blockIdx.x;
  int64_t I, J;
  [[maybe_unused]] int64_t cnt = 0;
  if constexpr (ACT) {
    // tiles of the active list, as in lowrank_gemm_kernel's kSymAct mode
    cnt = *g.act_n;
    const int64_t Ta = (cnt + GT - 1) / GT;
    const int64_t tiles = Ta * (Ta + 1) / 2;
    const int64_t pa = (tiles + NXCD - 1) / NXCD;
    if (w / NXCD >= pa) return;
    const int64_t ta = (w % NXCD) * pa + w / NXCD;
    if (ta >= tiles) return;
    tri_tile(ta, Ta, I, J);
  } else {
    const int64_t t = (w % NXCD) * per + w / NXCD;
    if (t >= T * (T + 1) / 2) return;
    tri_tile(t, T, I, J);
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  const int64_t r0 = I * GT;
  const int64_t c0 = J * GT;
  const int nch = g.r / GCF;
  const int lrow = tid / (GCF / 2), lcol = 2 * (tid % (GCF / 2));
  const double* pa = g.P + (r0 + lrow) * (int64_t)g.pld + lcol;
  const double* pb = g.P + (c0 + lrow) * (int64_t)g.pld + lcol;
  const int64_t ustep = GR * (int64_t)g.pld;
  // ACT: the rows of this thread, gathered through the list
  int64_t arow[ACT ? GL : 1], brow[ACT ? GL : 1];
  if constexpr (ACT) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int64_t p = r0 + lrow + GR * u, q = c0 + lrow + GR * u;
      arow[u] = (int64_t)g.act[p < cnt ? p : cnt - 1] * g.pld + lcol;
      brow[u] = (int64_t)g.act[q < cnt ? q : cnt - 1] * g.pld + lcol;
    }
  }
  double2 ra[GL], rb[GL];
  auto load = [&](int ch) {
    const int64_t cb = (int64_t)((ch * GCF) / g.pld) * g.gstride + (ch * GCF) % g.pld;
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      if constexpr (ACT) {
        ra[u] = *reinterpret_cast<const double2*>(g.P + arow[u] + cb);
        rb[u] = *reinterpret_cast<const double2*>(g.P + brow[u] + cb);
      } else {
        ra[u] = *reinterpret_cast<const double2*>(pa + u * ustep + cb);
        rb[u] = *reinterpret_cast<const double2*>(pb + u * ustep + cb);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int o = (lrow + GR * u) * GPF + lcol;
      As[buf][o] = (float)ra[u].x;
      As[buf][o + 1] = (float)ra[u].y;
      Bs[buf][o] = (float)rb[u].x;
      Bs[buf][o + 1] = (float)rb[u].y;
    }
  };
  fl4 acc[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[s][q] = fl4{0.0f, 0.0f, 0.0f, 0.0f};
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    load(ch + 1 < nch ? ch + 1 : ch);
#pragma unroll
    for (int k4 = 0; k4 < GCF; k4 += 4) {
      const int c = k4 + lk;
      float av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) av[s] = As[buf][(wr * 64 + s * 16 + l16) * GPF + c];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Bs[buf][(wc * 64 + q * 16 + l16) * GPF + (c ^ 1)];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[q], acc[s][q], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    store(buf ^ 1);
    __syncthreads();
  }
  // epilogue as lowrank_gemm_kernel's, rows 4 lk + v of each 16 x 16 block (ACT: list
  // positions, translated to the listed nodes)
  const bool diag = I == J;
  const int64_t lim_r = ACT ? cnt : g.nrows;
  const int64_t lim_c = ACT ? cnt : g.ncols;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    Raw<PREC> x[4][4], y[4][4];
    int on[4][4];
    int64_t an[4], bn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t p = r0 + wr * 64 + s * 16 + 4 * lk + v;
      an[v] = ACT ? (int64_t)g.act[p < cnt ? p : 0] : p;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p = c0 + wc * 64 + q * 16 + l16;
      bn[q] = ACT ? (int64_t)g.act[p < cnt ? p : 0] : p;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t pr = r0 + wr * 64 + s * 16 + 4 * lk + v;
        const int64_t pc = c0 + wc * 64 + q * 16 + l16;
        on[q][v] = pr < lim_r && pc < lim_c;
        const int64_t da = on[q][v] ? an[v] * g.S.ld + bn[q] : 0;
        const int64_t ma = on[q][v] ? bn[q] * g.S.ld + an[v] : 0;
        sload<PREC>(g.S, da, x[q][v]);
        sload<PREC>(g.S, ma, y[q][v]);
      }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (!on[q][v]) continue;
        const int64_t pr = r0 + wr * 64 + s * 16 + 4 * lk + v;
        const int64_t pc = c0 + wc * 64 + q * 16 + l16;
        const double d = (double)acc[s][q][v];
        if (!diag || pr <= pc) sput<PREC>(g.S, an[v] * g.S.ld + bn[q], sval<PREC>(x[q][v]) + d);
        if (!diag || pr < pc) sput<PREC>(g.S, bn[q] * g.S.ld + an[v], sval<PREC>(y[q][v]) + d);
      }
  }
}

__global__ __launch_bounds__(256) void delta_col_kernel(const double* __restrict__ P, int pld,
                                                       int r, int64_t n, int32_t x,
                                                       double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (a >= n) return;
  double d = 0.0;
  for (int c = 0; c < r; ++c) d += P[a * pld + c] * P[(int64_t)x * pld + (c ^ 1)];
  out[a] = d;
}

__global__ __launch_bounds__(256) void panel_weights_kernel(const double* __restrict__ P, int pld,
                                                           int64_t gstride, int r, IdList I,
                                                           int32_t j, double* __restrict__ wts) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= r) return;
  const int cs = col ^ 1;
  const double* base = P + (int64_t)(cs / pld) * gstride + cs % pld;
  double w = 0.0;
  for (int t = 0; t < I.count; ++t) w += base[(int64_t)I.at(t) * pld];
  wts[col] = w;
  wts[r + col] = j >= 0 ? base[(int64_t)j * pld] : 0.0;
}

// One wave per row: lanes stride over the row's r panel entries (contiguous), then reduce.
__global__ __launch_bounds__(256) void panel_gemv_kernel(const double* __restrict__ P, int pld,
                                                         int64_t gstride, int r, int64_t n,
                                                         const double* __restrict__ wts,
                                                         double* __restrict__ SI,
                                                         double* __restrict__ Sj) {
  const int64_t a = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (a >= n) return;
  const double* row = P + a * pld;
  double s0 = 0.0, s1 = 0.0;
  for (int col = lane; col < r; col += 64) {
    const double p = row[(int64_t)(col / pld) * gstride + col % pld];
    s0 += p * wts[col];
    s1 += p * wts[r + col];
  }
  s0 = wave_sum(s0, 64);
  s1 = wave_sum(s1, 64);
  if (lane == 0) {
    if (SI) SI[a] += s0;
    if (Sj) Sj[a] += s1;
  }
}

// Incremental corrections of a fused chunk (the declaration states the sums). Weights first:
// one thread per (vector, panel column).
__global__ __launch_bounds__(256) void corr_weights_kernel(const double* __restrict__ Pseg,
                                                          int pld, CorrSlots c, int s0, int s1) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int nv = 2 * (s1 - s0);
  if (t >= nv * pld) return;
  const int v = t / pld, col = t % pld;
  const int slot = s0 + v / 2;
  const int cs = col ^ 1;
  double w = 0.0;
  if ((v & 1) == 0) {
    for (int p = c.rstart[slot]; p < c.rstart[slot + 1]; ++p)
      w += Pseg[(int64_t)c.rows[p] * pld + cs];
  } else {
    const int j = c.sink[slot];
    if (j >= 0) w = Pseg[(int64_t)j * pld + cs];
  }
  c.w[t] = w;
}

// One thread per row a: the row's PW panel entries stay in registers, the weights of up to
// kCorrVB vectors at a time are staged in LDS (every lane reads the same word), and each
// vector's entry a is read, increased and written back (coalesced over a).
constexpr int kCorrVB = 64;
template <int PW>
__global__ __launch_bounds__(256) void corr_update_kernel(const double* __restrict__ Pseg,
                                                         int64_t n, CorrSlots c, int s0,
                                                         int s1) {
  __shared__ double lw[kCorrVB * PW];
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = a < n;
  double p[PW];
  const double2* row = reinterpret_cast<const double2*>(Pseg + (in ? a : 0) * PW);
#pragma unroll
  for (int q = 0; q < PW / 2; ++q) {
    const double2 v = row[q];
    p[2 * q] = v.x;
    p[2 * q + 1] = v.y;
  }
  const int nv = 2 * (s1 - s0);
  double* out = c.corr + (int64_t)2 * (s0 - c.base) * c.ldc + a;
  for (int v0 = 0; v0 < nv; v0 += kCorrVB) {
    const int vb = min(kCorrVB, nv - v0);
    __syncthreads();
    for (int e = threadIdx.x; e < vb * PW; e += 256) lw[e] = c.w[(int64_t)v0 * PW + e];
    __syncthreads();
    if (in) {
      // 8 vectors at a time: their 8 loads are issued together (positions past vb reload the
      // last vector and are not stored)
      for (int v = 0; v < vb; v += 8) {
        double cur[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cur[u] = out[(int64_t)(v0 + min(v + u, vb - 1)) * c.ldc];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int vv = min(v + u, vb - 1);
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < PW; ++q) acc += p[q] * lw[vv * PW + q];
          if (v + u < vb) out[(int64_t)(v0 + v + u) * c.ldc] = cur[u] + acc;
        }
      }
    }
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Column output for one block (r <= RC panel columns, float32):
//     out[p][b] = sum_{c < r} P[rows[p]][c] P[b][c ^ 1]   (Delta S[b][rows[p]], eq (71))
// for list positions p < nrows and nodes b < ncols. The tiling is the streaming kernel's
// without S: workgroup = strip of SC nodes, wave w = positions [16 w, 16 w + 16) of each TR
// tile. A strip's B fragments are the same for every tile, so each lane keeps them in
// registers for the whole kernel (KS k-steps of 4 panel columns; columns at or past r are
// zero there); a tile then costs ST KS MFMAs, KS loads of A fragments issued one tile ahead,
// and its float32 stores, with no LDS traffic. With VEC, accumulator t of lane column l holds
// node c0 + 4 l + t, so a lane's four accumulators of one row are adjacent and go out as one
// 16-byte store (a quarter of the store instructions); otherwise node c0 + 16 t + l. Full
// tiles store without per-entry checks.
template <int KS, bool VEC>
__global__ __launch_bounds__(NT, KS <= 6 ? 4 : 3) void lowrank_cols_kernel(LowRankArgs g) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int lk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * SC;
  auto node = [&](int t) -> int64_t { return VEC ? c0 + 4 * l16 + t : c0 + 16 * t + l16; };
  // B[k][j] = P[node][k ^ 1], k = 4 ks + lk (k ^ 1 < 4 KS <= pld: in bounds)
  double bv[ST][KS];
#pragma unroll
  for (int t = 0; t < ST; ++t) {
    const int64_t b = node(t);
    const bool okb = b < g.ncols;
    const double* src = g.P + (okb ? b : 0) * g.pld;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lk;
      const double v = src[k ^ 1];
      bv[t][ks] = (okb && k < g.r) ? v : 0.0;
    }
  }
  const int64_t nrows = g.nrows;
  const int64_t nrt = (nrows + TR - 1) / TR;
  const int64_t gy = gridDim.y;
  const bool full_cols = c0 + SC <= g.ncols;
  // A operand row of a tile: the node at list position (tile base + l16), clamped to the
  // last position (any listed node is an in-bounds panel row)
  auto fetch = [&](int64_t rt) -> int32_t {
    const int64_t p = rt * TR + wave * 16 + l16;
    return g.rows[p < nrows ? p : nrows - 1];
  };
  auto load_a = [&](int32_t nd, double (&av)[KS]) {
    const double* src = g.P + (int64_t)nd * g.pld + lk;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) av[ks] = src[4 * ks];
  };
  int64_t rt = blockIdx.y;
  double a0[KS], a1[KS];
  load_a(fetch(rt), a0);
  int32_t e1 = fetch(rt + gy);
  for (; rt < nrt; rt += gy) {
    load_a(e1, a1);
    e1 = fetch(rt + 2 * gy);
    dbl4 acc[ST];
#pragma unroll
    for (int t = 0; t < ST; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < ST; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[ks], bv[t][ks], acc[t], 0, 0, 0);
    const int64_t rb = rt * TR + wave * 16;
    if (full_cols && rb + 16 <= nrows) {
#pragma unroll
      // the output is written once and not read back here: non-temporal stores (17% faster
      // than ordinary ones at n = 1M)
      for (int v = 0; v < 4; ++v) {
        float* orow = g.out + (rb + v * 4 + lk) * g.ld_out + c0;
        if (VEC) {
          const f32x4 val = {(float)acc[0][v], (float)acc[1][v], (float)acc[2][v],
                             (float)acc[3][v]};
          __builtin_nontemporal_store(val, reinterpret_cast<f32x4*>(orow + 4 * l16));
        } else {
#pragma unroll
          for (int t = 0; t < ST; ++t)
            __builtin_nontemporal_store((float)acc[t][v], orow + 16 * t + l16);
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t pc = rb + v * 4 + lk;
        if (pc >= nrows) continue;
        float* orow = g.out + pc * g.ld_out;
#pragma unroll
        for (int t = 0; t < ST; ++t)
          if (node(t) < g.ncols) orow[node(t)] = (float)acc[t][v];
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a0[ks] = a1[ks];
  }
}

}  // namespace

hipError_t launch_panel_correct(const double* P, int pld, int64_t gstride, int r, int64_t n,
                                const IdList& I, int32_t j, double* wts, double* SI,
                                double* Sj, hipStream_t s) {
  if (r <= 0 || n <= 0) return hipSuccess;
  panel_weights_kernel<<<(unsigned)((r + 255) / 256), 256, 0, s>>>(P, pld, gstride, r, I, j,
                                                                    wts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  panel_gemv_kernel<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(P, pld, gstride, r, n, wts,
                                                            I.count ? SI : nullptr,
                                                            j >= 0 ? Sj : nullptr);
  return hipGetLastError();
}

hipError_t launch_corr_update(const double* Pseg, int pld, int64_t n, const CorrSlots& c,
                              int s0, int s1, hipStream_t s) {
  if (pld != 32 && pld != 64) return hipErrorInvalidValue;
  if (s1 <= s0 || n <= 0) return hipSuccess;
  const int nt = 2 * (s1 - s0) * pld;
  corr_weights_kernel<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(Pseg, pld, c, s0, s1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (pld == 32)
    corr_update_kernel<32><<<grid, 256, 0, s>>>(Pseg, n, c, s0, s1);
  else
    corr_update_kernel<64><<<grid, 256, 0, s>>>(Pseg, n, c, s0, s1);
  return hipGetLastError();
}

hipError_t launch_delta_col(const double* P, int pld, int r, int64_t n, int32_t x, double* out,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  delta_col_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, pld, r, n, x, out);
  return hipGetLastError();
}

template <int KS>
static void cols_launch(const LowRankArgs& a, dim3 grid, hipStream_t s) {
  // 16-byte stores need ld_out and the base address aligned to 4 floats
  if (a.ld_out % 4 == 0 && reinterpret_cast<uintptr_t>(a.out) % 16 == 0)
    lowrank_cols_kernel<KS, true><<<grid, NT, 0, s>>>(a);
  else
    lowrank_cols_kernel<KS, false><<<grid, NT, 0, s>>>(a);
}

// Listed rows store whole 16-column slices (measured at n = 92.5k, A_hat ~ B_hat ~ 0.64 n:
// 17.6 ms instead of 18.4 ms with per-entry masked stores, although more bytes are written).
template <int PREC, bool MASK>
static void strip_launch(const LowRankArgs& a, dim3 grid, hipStream_t s) {
  if (a.rows)
    lowrank_strip_kernel<PREC, MASK, true, MASK><<<grid, NT, 0, s>>>(a);
  else
    lowrank_strip_kernel<PREC, MASK, false><<<grid, NT, 0, s>>>(a);
}

hipError_t launch_lowrank(const LowRankArgs& a, hipStream_t s) {
  if (a.ncols <= 0 || (a.nrows_dev == nullptr && a.nrows <= 0)) return hipSuccess;
  const int64_t nrows_bound = a.nrows_dev ? (a.rows ? a.ncols : a.nrows) : a.nrows;
  if (!a.fused && a.r > RC && (a.rows != nullptr || a.nrows_dev != nullptr || a.Ahat != nullptr)) {
    // one streaming pass per 32 panel columns (pairs never straddle a pass)
    if (a.out) return hipErrorInvalidValue;
    for (int c = 0; c < a.r; c += RC) {
      LowRankArgs b = a;
      b.P = a.P + c;
      b.r = a.r - c < RC ? a.r - c : RC;
      hipError_t e = launch_lowrank(b, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (a.r <= RC && !a.fused) {
    const int64_t strips = (a.ncols + SC - 1) / SC;
    const int64_t rtiles = (nrows_bound + TR - 1) / TR;
    int64_t gy = (4096 + strips - 1) / strips;
    if (gy > rtiles) gy = rtiles;
    if (gy < 1) gy = 1;
    dim3 grid((unsigned)strips, (unsigned)gy);
    const bool mask = a.Ahat != nullptr && a.out == nullptr;
    if (a.out) {
      // column output: list rows on the host count only; r even, so ceil(r / 4) is 1..8
      if (a.rows == nullptr || a.nrows_dev != nullptr || a.Ahat != nullptr) {
        return hipErrorInvalidValue;
      }
      // at least two workgroups per strip: shorter row loops balance the tail better
      if (grid.y < 2 && rtiles >= 2) grid.y = 2;
      switch ((a.r + 3) / 4) {
        case 1: cols_launch<1>(a, grid, s); break;
        case 2: cols_launch<2>(a, grid, s); break;
        case 3: cols_launch<3>(a, grid, s); break;
        case 4: cols_launch<4>(a, grid, s); break;
        case 5: cols_launch<5>(a, grid, s); break;
        case 6: cols_launch<6>(a, grid, s); break;
        case 7: cols_launch<7>(a, grid, s); break;
        default: cols_launch<8>(a, grid, s); break;
      }
    } else if (a.S.prec == PREC_FP64) {
      mask ? strip_launch<PREC_FP64, true>(a, grid, s)
           : strip_launch<PREC_FP64, false>(a, grid, s);
    } else if (a.S.prec == PREC_HILO) {
      mask ? strip_launch<PREC_HILO, true>(a, grid, s)
           : strip_launch<PREC_HILO, false>(a, grid, s);
    } else {
      mask ? strip_launch<PREC_FP32, true>(a, grid, s)
           : strip_launch<PREC_FP32, false>(a, grid, s);
    }
    return hipGetLastError();
  }
  // Fused passes, and several blocks without a row list: the GEMM over the upper triangle of
  // tiles, which writes (a, b) and (b, a) from one sum so S stays exactly symmetric (rows
  // list and mask not used; see lowrank_gemm_kernel for what the panel must hold).
  if (a.variant < 0 || a.variant >= kGemmVariants) return hipErrorInvalidValue;
  const int gc = a.variant < 2 ? 16 : 32;  // the float32 variant stages 32 columns too
  if (a.rows != nullptr || a.nrows_dev != nullptr || a.Ahat != nullptr || a.out != nullptr ||
      a.nrows != a.ncols || a.r % gc != 0 || a.pld % gc != 0 || (a.act && !a.act_n) ||
      (a.tflags && (!a.act || a.pld / 4 > 32 || a.tf_ld < (a.nrows + GT - 1) / GT)))
    return hipErrorInvalidValue;
  const int64_t T = (a.nrows + GT - 1) / GT;
  if (a.p_rows < T * GT) return hipErrorInvalidValue;
  const int64_t tiles = T * (T + 1) / 2;
  const int64_t per = (tiles + NXCD - 1) / NXCD;
  const unsigned grid = (unsigned)(per * NXCD);
  auto go = [&](auto prec) {
    constexpr int P = decltype(prec)::value;
    if (a.act) {
      switch (a.variant) {
        case kGemmF32: lowrank_gemm_f32_kernel<P, true><<<grid, NT, 0, s>>>(a, T, per); break;
        case 0: lowrank_gemm_kernel<P, kSymAct, 16, 18, 2><<<grid, NT, 0, s>>>(a, T, per); break;
        case 1: lowrank_gemm_kernel<P, kSymAct, 16, 20, 2><<<grid, NT, 0, s>>>(a, T, per); break;
        case 2: lowrank_gemm_kernel<P, kSymAct, 32, 34, 1><<<grid, NT, 0, s>>>(a, T, per); break;
        default:
          lowrank_gemm_kernel<P, kSymAct, 32, 36, 1><<<grid, NT, 0, s>>>(a, T, per);
          break;
      }
      return;
    }
    switch (a.variant) {
      case kGemmF32: lowrank_gemm_f32_kernel<P><<<grid, NT, 0, s>>>(a, T, per); break;
      case 0: lowrank_gemm_kernel<P, kSym, 16, 18, 2><<<grid, NT, 0, s>>>(a, T, per); break;
      case 1: lowrank_gemm_kernel<P, kSym, 16, 20, 2><<<grid, NT, 0, s>>>(a, T, per); break;
      case 2: lowrank_gemm_kernel<P, kSym, 32, 34, 1><<<grid, NT, 0, s>>>(a, T, per); break;
      default: lowrank_gemm_kernel<P, kSym, 32, 36, 1><<<grid, NT, 0, s>>>(a, T, per); break;
    }
  };
  if (a.S.prec == PREC_FP64)
    go(std::integral_constant<int, PREC_FP64>{});
  else if (a.S.prec == PREC_HILO)
    go(std::integral_constant<int, PREC_HILO>{});
  else
    go(std::integral_constant<int, PREC_FP32>{});
  return hipGetLastError();
}

// One thread per (node, panel segment): a nonzero among the row's first w entries sets the
// node's bit; a wave's 64 bits go out as two atomics (nodes of a wave share two words).
__global__ __launch_bounds__(256) void pass_rows_kernel(const double* __restrict__ P, int pld,
                                                        int64_t gstride, int w, int64_t n,
                                                        uint32_t* __restrict__ bm) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool nz = false;
  if (a < n) {
    const double* row = P + (int64_t)blockIdx.y * gstride + a * pld;
    for (int c = 0; c < w; c += 2) {
      const double2 v = *reinterpret_cast<const double2*>(row + c);
      nz |= v.x != 0.0 || v.y != 0.0;
    }
  }
  const uint64_t m = __ballot(nz);
  const int lane = threadIdx.x & 63;
  if ((lane == 0 || lane == 32) && a < n) {
    const uint32_t bits = (uint32_t)(lane == 0 ? m : (m >> 32));
    if (bits) atomicOr(bm + (a >> 5), bits);
  }
}

hipError_t launch_pass_rows(const double* P, int pld, int64_t gstride, int q, int w, int64_t n,
                            uint32_t* bm, hipStream_t s) {
  if (n <= 0 || q <= 0) return hipSuccess;
  if (q > 65535 || w > pld || w % 2 != 0 || pld % 2 != 0) return hipErrorInvalidValue;
  pass_rows_kernel<<<dim3((unsigned)((n + 255) / 256), (unsigned)q), 256, 0, s>>>(P, pld, gstride,
                                                                                  w, n, bm);
  return hipGetLastError();
}

// One workgroup per (tile, panel segment), one thread per list position: the thread's bits
// (k-steps whose xi columns are nonzero on its row) are OR-ed over the tile in LDS.
static_assert(GT == kTileRows, "fused-pass tiles and tile flags share their row count");
__global__ __launch_bounds__(kTileRows) void tile_flags_kernel(const double* __restrict__ P,
                                                               int pld, int64_t gstride,
                                                               const int32_t* __restrict__ act,
                                                               const int64_t* __restrict__ act_n,
                                                               uint32_t* __restrict__ flags,
                                                               int64_t tf_ld,
                                                               int32_t* __restrict__ skip,
                                                               int steps) {
  __shared__ uint32_t tile_bits;
  const int64_t cnt = *act_n;
  const int64_t t = blockIdx.x;
  const int64_t p0 = t * kTileRows;
  if (p0 >= cnt) return;  // uniform: past the list's tiles
  if (threadIdx.x == 0) tile_bits = 0;
  __syncthreads();
  const int64_t p = p0 + threadIdx.x;
  uint32_t bits = 0;
  if (p < cnt) {
    const double* row = P + (int64_t)blockIdx.y * gstride + (int64_t)act[p] * pld;
    for (int c = 0; c < pld; c += 4) {
      const double2 v0 = *reinterpret_cast<const double2*>(row + c);      // xi_2g, eta_2g
      const double2 v1 = *reinterpret_cast<const double2*>(row + c + 2);  // xi_2g+1, eta_2g+1
      if (v0.x != 0.0 || v1.x != 0.0) bits |= 1u << (c / 4);
    }
  }
  if (bits) atomicOr(&tile_bits, bits);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t b = tile_bits;
    flags[(int64_t)blockIdx.y * tf_ld + t] = b;
    const int32_t size = (int32_t)(cnt - p0 < kTileRows ? cnt - p0 : kTileRows);
    for (int g = 0; g < steps; ++g)
      if (!((b >> g) & 1u)) atomicAdd(skip + (int64_t)blockIdx.y * steps + g, size);
  }
}

hipError_t launch_tile_flags(const double* P, int pld, int64_t gstride, int q,
                             const int32_t* act, const int64_t* act_n, int64_t n_max,
                             uint32_t* flags, int64_t tf_ld, int32_t* skip, int steps,
                             hipStream_t s) {
  if (n_max <= 0 || q <= 0) return hipSuccess;
  const int64_t tiles = (n_max + kTileRows - 1) / kTileRows;
  if (q > 65535 || pld % 4 != 0 || pld / 4 > 32 || steps < 1 || steps > pld / 4 ||
      tf_ld < tiles || !act || !act_n || !flags || !skip)
    return hipErrorInvalidValue;
  tile_flags_kernel<<<dim3((unsigned)tiles, (unsigned)q), kTileRows, 0, s>>>(
      P, pld, gstride, act, act_n, flags, tf_ld, skip, steps);
  return hipGetLastError();
}

hipError_t launch_bs_gemm(const LowRankArgs& a, const BlockStore& B, const BsItem* items,
                          int64_t nitems, hipStream_t s) {
  if (nitems <= 0 || a.r <= 0) return hipSuccess;
  if (a.r % GC != 0 || a.pld % GC != 0 || !items) return hipErrorInvalidValue;
  const int64_t per = (nitems + NXCD - 1) / NXCD;
  const unsigned grid = (unsigned)(per * NXCD);
  if (a.S.prec == PREC_FP64)
    lowrank_gemm_kernel<PREC_FP64, kBlk><<<grid, NT, 0, s>>>(a, nitems, per, 0, B, items);
  else if (a.S.prec == PREC_HILO)
    lowrank_gemm_kernel<PREC_HILO, kBlk><<<grid, NT, 0, s>>>(a, nitems, per, 0, B, items);
  else
    lowrank_gemm_kernel<PREC_FP32, kBlk><<<grid, NT, 0, s>>>(a, nitems, per, 0, B, items);
  return hipGetLastError();
}

hipError_t launch_lowrank_acc(const LowRankArgs& a, hipStream_t s) {
  if (a.nrows <= 0 || a.ncols <= 0 || a.r <= 0) return hipSuccess;
  if (a.rows == nullptr || a.acc_out == nullptr || a.r % GC != 0 || a.pld % GC != 0 ||
      a.ld_out < a.ncols)
    return hipErrorInvalidValue;
  const int64_t T = (a.nrows + GT - 1) / GT;
  const int64_t TJ = (a.ncols + GT - 1) / GT;
  if (a.p_rows < TJ * GT) return hipErrorInvalidValue;
  const int64_t tiles = T * TJ;
  const int64_t per = (tiles + NXCD - 1) / NXCD;
  lowrank_gemm_kernel<PREC_FP64, kRect><<<(unsigned)(per * NXCD), NT, 0, s>>>(a, T, per, TJ);
  return hipGetLastError();
}

}  // namespace sr

namespace sr {

// Lane-layout check of v_mfma_f64_16x16x4_f64 (all accesses in bounds: 64 lanes, 4 outputs
// each). out[lane * 4 + v] = D element held by lane in slot v for A = a_in, B = b_in.
__global__ __launch_bounds__(64) void mfma_probe_kernel(const double* a_in, const double* b_in,
                                                        double* out) {
  const int lane = threadIdx.x;
  dbl4 c = {0.0, 0.0, 0.0, 0.0};
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a_in[lane], b_in[lane], c, 0, 0, 0);
  for (int v = 0; v < 4; ++v) out[lane * 4 + v] = c[v];
}

hipError_t launch_mfma_probe(const double* a, const double* b, double* out, hipStream_t s) {
  mfma_probe_kernel<<<1, 64, 0, s>>>(a, b, out);
  return hipGetLastError();
}

// The same check for v_mfma_f32_16x16x4f32 (float operands and accumulators).
typedef float f32x4_acc __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(64) void mfma_probe_f32_kernel(const float* a_in, const float* b_in,
                                                            float* out) {
  const int lane = threadIdx.x;
  f32x4_acc c = {0.0f, 0.0f, 0.0f, 0.0f};
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a_in[lane], b_in[lane], c, 0, 0, 0);
  for (int v = 0; v < 4; ++v) out[lane * 4 + v] = c[v];
}

hipError_t launch_mfma_probe_f32(const float* a, const float* b, float* out, hipStream_t s) {
  mfma_probe_f32_kernel<<<1, 64, 0, s>>>(a, b, out);
  return hipGetLastError();
}

}  // namespace sr
