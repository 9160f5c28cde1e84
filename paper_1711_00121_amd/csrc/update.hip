// The S update of the incremental method: S <- S + M_K + M_K^T restricted to the affected
// areas (Algorithm 1 final line; Algorithm 2 with the union-rectangle reading), where
// M_K = sum_k xi_k eta_k^T (eq (16a)). Entry (a, b) receives
//     sum_k xi_k[a] eta_k[b] + eta_k[a] xi_k[b] = sum_c P[a][c] P[b][c ^ 1]
// with panel rows P[a] = (xi_0[a], eta_0[a], xi_1[a], eta_1[a], ...). Several blocks of a batch
// stack their pairs along c, so the same kernel applies a rank-2(K+1)B update in one pass.
//
// Mapping to gfx950: each 256-thread workgroup owns a 64 x 128 tile of (listed rows) x
// (columns) and stages the tile's panel rows in LDS; each wave computes a 32 x 64 sub-tile
// with v_mfma_f64_16x16x4_f64 (2 x 4 accumulators of 16 x 16). The wave issues its S loads
// before the MFMA loop, so HBM latency overlaps the matrix work, then adds, re-splits (hi/lo)
// and stores. S is read and written once per update; the kernel is bound by HBM bandwidth
// for one block and by FP64 matrix throughput for large batches.
#include "kernels.h"

namespace sr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TR = 64;    // tile rows (positions in the row list)
constexpr int RC = 32;    // panel columns staged per pass
constexpr int LP = RC + 1;  // LDS row pitch in doubles (odd pitch spreads banks)
constexpr int NT = 256;

__device__ __forceinline__ bool pair_in(const uint32_t* Ah, const uint32_t* Bh, bool ra, bool rb,
                                        int64_t b) {
  if (!Ah) return true;
  const bool ca = bit_get(Ah, b), cb = bit_get(Bh, b);
  return (ra && cb) || (rb && ca);
}

template <int PREC>
__device__ __forceinline__ double sget(const SView& S, int64_t off) {
  if (PREC == PREC_FP64) return S.d[off];
  if (PREC == PREC_HILO) return (double)S.hi[off] + (double)S.lo[off];
  return (double)S.hi[off];
}

template <int PREC>
__device__ __forceinline__ void sput(const SView& S, int64_t off, double t) {
  if (PREC == PREC_FP64) {
    S.d[off] = t;
  } else if (PREC == PREC_HILO) {
    const float h = (float)t;
    S.hi[off] = h;
    S.lo[off] = (float)(t - (double)h);
  } else {
    S.hi[off] = (float)t;
  }
}

// Streaming update for one block (r <= RC panel columns). Workgroup = strip of SC columns whose
// panel rows live in LDS for the whole strip; the workgroup walks row tiles of TR listed rows,
// wave w taking rows [16 w, 16 w + 16) of each tile against the strip's SC columns (SC / 16
// accumulators). Per tile a wave issues its A-fragment loads and all its S loads before the
// MFMAs, so the S latency overlaps the matrix work of this and the other resident waves.
// Every load is unconditional from an in-bounds address (rows past the list read row 0;
// columns past n stay inside the padded leading dimension, a multiple of SC) and selected
// afterwards: a load under a branch is followed by a full wait and serialises the tile.
constexpr int SC = 64;
constexpr int ST = SC / 16;

template <int PREC, bool MASK, bool COLOUT, bool HASROWS>
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
  bool cin[ST], cA[ST], cB[ST];
#pragma unroll
  for (int t = 0; t < ST; ++t) {
    const int64_t b = c0 + t * 16 + l16;
    cin[t] = b < g.ncols;
    if (MASK) {
      const int64_t bb = cin[t] ? b : 0;
      const uint32_t wa = g.Ahat[bb >> 5], wb = g.Bhat[bb >> 5];
      cA[t] = (wa >> (bb & 31)) & 1u;
      cB[t] = (wb >> (bb & 31)) & 1u;
    } else {
      cA[t] = cB[t] = true;
    }
  }
  __syncthreads();

  const int64_t nrows = g.nrows_dev ? *g.nrows_dev : g.nrows;
  const int64_t nrt = (nrows + TR - 1) / TR;
  const int ksteps = RC / 4;  // columns past r are zero on both sides
  // Row-list entries of a tile: [0] the A-operand row (rbase + l16), [1..4] the accumulator
  // rows (rbase + 4 v + lk). They are fetched one tile ahead so the S addresses of a tile do
  // not wait on a list load.
  auto fetch = [&](int64_t rt, int32_t (&e)[5]) {
    const int64_t rbase = rt * TR + wave * 16;
    const int64_t last = nrows > 0 ? nrows - 1 : 0;
    const int64_t p0 = rbase + l16;
    e[0] = HASROWS ? g.rows[p0 < nrows ? p0 : last] : (int32_t)p0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t pc = rbase + v * 4 + lk;
      e[1 + v] = HASROWS ? g.rows[pc < nrows ? pc : last] : (int32_t)pc;
    }
  };
  int32_t cur[5], nxt[5];
  if ((int64_t)blockIdx.y < nrt) fetch(blockIdx.y, cur);
  for (int64_t rt = blockIdx.y; rt < nrt; rt += gridDim.y) {
    const int64_t rbase = rt * TR + wave * 16;
    // A operand. The inner sum over panel columns is order-free, so k-step ks of lane group
    // lk uses column 8 lk + ks (same permutation on the B side): each lane's 8 A values are
    // contiguous. With a mask the row list holds (node << 2) | (in A_hat << 1) | in B_hat.
    const bool pa_ok = rbase + l16 < nrows;
    const int64_t arow = pa_ok ? ((int64_t)cur[0] >> (MASK ? 2 : 0)) : 0;
    double av[RC / 4];
    {
      const double2* src = reinterpret_cast<const double2*>(g.P + arow * g.pld + 8 * lk);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const double2 v = src[h];
        av[2 * h] = v.x;
        av[2 * h + 1] = v.y;
      }
#pragma unroll
      for (int ks = 0; ks < RC / 4; ++ks)
        if (!pa_ok || 8 * lk + ks >= g.r) av[ks] = 0.0;
    }
    // accumulator rows of this lane: rbase + 4 v + lk
    int64_t crow[4];
    bool rok[4], rA[4], rB[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t pc = rbase + v * 4 + lk;
      rok[v] = pc < nrows;
      const int32_t packed = cur[1 + v];
      // column output: the output row is the position in the query list, not the node
      const int64_t rr = COLOUT ? pc : (MASK ? (packed >> 2) : packed);
      crow[v] = rok[v] ? rr : 0;
      rA[v] = MASK ? ((packed >> 1) & 1) : true;
      rB[v] = MASK ? (packed & 1) : true;
    }
    if (rt + gridDim.y < nrt) fetch(rt + gridDim.y, nxt);
    bool on[ST][4];
#pragma unroll
    for (int t = 0; t < ST; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        on[t][v] = rok[v] && cin[t] && ((rA[v] && cB[t]) || (rB[v] && cA[t]));
    double old[ST][4];
    if (!COLOUT) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t base = crow[v] * g.S.ld + c0 + l16;
#pragma unroll
        for (int t = 0; t < ST; ++t) old[t][v] = sget<PREC>(g.S, base + t * 16);
      }
    }
    dbl4 acc[ST];
#pragma unroll
    for (int t = 0; t < ST; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < RC / 4; ++ks) {
      if (ks < ksteps) {
        const int c = (8 * lk + ks) ^ 1;
#pragma unroll
        for (int t = 0; t < ST; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], lcol[(t * 16 + l16) * LP + c],
                                                        acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int t = 0; t < ST; ++t) {
        if (!on[t][v]) continue;
        const int64_t b = c0 + t * 16 + l16;
        if (COLOUT) {
          g.out[crow[v] * g.ld_out + b] = (float)acc[t][v];
        } else {
          sput<PREC>(g.S, crow[v] * g.S.ld + b, old[t][v] + acc[t][v]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) cur[q] = nxt[q];
  }
}

// Fused batch pass (any r, all rows and columns, no mask): S += P swap(P)^T as a GEMM with
// inner dimension r. 128 x 128 tiles; wave (wr, wc) owns a 64 x 64 quarter (4 x 4 accumulators
// of 16 x 16). Panel columns are staged through LDS 16 at a time, double buffered: the global
// loads of chunk c + 1 are in flight while the MFMAs of chunk c run.
constexpr int GT = 128;       // tile rows = tile cols
constexpr int GC = 16;        // panel columns per chunk
constexpr int GP = GC + 1;    // LDS pitch (doubles)
constexpr int GL = GT * (GC / 2) / NT;  // double2 loads per thread per side per chunk (4)

template <int PREC>
__global__ __launch_bounds__(NT) void lowrank_gemm_kernel(LowRankArgs g) {
  __shared__ double As[2][GT * GP];
  __shared__ double Bs[2][GT * GP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.y * GT;
  const int64_t c0 = (int64_t)blockIdx.x * GT;
  const int64_t nrows = g.nrows;
  const int nch = (g.r + GC - 1) / GC;

  double2 ra[GL], rb[GL];
  auto load = [&](int ch) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int e = tid + u * NT;
      const int rr = e / (GC / 2), cc = ch * GC + (e % (GC / 2)) * 2;
      const int64_t a = r0 + rr, b = c0 + rr;
      const bool oka = a < nrows && cc < g.r, okb = b < g.ncols && cc < g.r;
      ra[u] = *reinterpret_cast<const double2*>(g.P + (oka ? a * g.pld + cc : 0));
      rb[u] = *reinterpret_cast<const double2*>(g.P + (okb ? b * g.pld + cc : 0));
      if (!oka) ra[u] = make_double2(0.0, 0.0);
      if (!okb) rb[u] = make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < GL; ++u) {
      const int e = tid + u * NT;
      const int rr = e / (GC / 2), cc = (e % (GC / 2)) * 2;
      As[buf][rr * GP + cc] = ra[u].x;
      As[buf][rr * GP + cc + 1] = ra[u].y;
      Bs[buf][rr * GP + cc] = rb[u].x;
      Bs[buf][rr * GP + cc + 1] = rb[u].y;
    }
  };

  dbl4 acc[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[s][t] = dbl4{0.0, 0.0, 0.0, 0.0};

  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) load(ch + 1);
#pragma unroll
    for (int k4 = 0; k4 < GC; k4 += 4) {
      const int c = k4 + lk;
      double av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) av[s] = As[buf][(wr * 64 + s * 16 + l16) * GP + c];
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[t] = Bs[buf][(wc * 64 + t * 16 + l16) * GP + (c ^ 1)];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[s][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[t], acc[s][t], 0, 0, 0);
    }
    if (ch + 1 < nch) store(buf ^ 1);
    __syncthreads();
  }

  // S += acc, one row sub-tile at a time (16 entries per lane), loads unconditional.
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double old[4][4];
    bool on[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t a = r0 + wr * 64 + s * 16 + v * 4 + lk;
        const int64_t b = c0 + wc * 64 + t * 16 + l16;
        on[t][v] = a < nrows && b < g.ncols;
        const double x = sget<PREC>(g.S, on[t][v] ? a * g.S.ld + b : 0);
        old[t][v] = x;
      }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (!on[t][v]) continue;
        const int64_t a = r0 + wr * 64 + s * 16 + v * 4 + lk;
        const int64_t b = c0 + wc * 64 + t * 16 + l16;
        sput<PREC>(g.S, a * g.S.ld + b, old[t][v] + acc[s][t][v]);
      }
  }
}

__global__ __launch_bounds__(256) void lowrank_ref_kernel(LowRankArgs g) {
  const int64_t nrows = g.nrows_dev ? *g.nrows_dev : g.nrows;
  const int64_t t = blockIdx.x;
  if (t >= nrows) return;
  const int64_t b = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (b >= g.ncols) return;
  const bool packed = g.out == nullptr && g.Ahat != nullptr && g.rows != nullptr;
  const int64_t a = g.rows ? ((int64_t)g.rows[t] >> (packed ? 2 : 0)) : t;
  if (g.out == nullptr && g.Ahat) {
    if (!pair_in(g.Ahat, g.Bhat, bit_get(g.Ahat, a), bit_get(g.Bhat, a), b)) return;
  }
  double d = 0.0;
  for (int c = 0; c < g.r; ++c) d += g.P[a * g.pld + c] * g.P[b * g.pld + (c ^ 1)];
  if (g.out) {
    g.out[t * g.ld_out + b] = (float)d;
  } else {
    const int64_t off = a * g.S.ld + b;
    s_put(g.S, off, s_get(g.S, off) + d);
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
                                                           int r, IdList I, int32_t j,
                                                           double* __restrict__ wts) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= r) return;
  double w = 0.0;
  for (int t = 0; t < I.count; ++t) w += P[(int64_t)I.id[t] * pld + (col ^ 1)];
  wts[col] = w;
  wts[r + col] = j >= 0 ? P[(int64_t)j * pld + (col ^ 1)] : 0.0;
}

// One wave per row: lanes stride over the row's r panel entries (contiguous), then reduce.
__global__ __launch_bounds__(256) void panel_gemv_kernel(const double* __restrict__ P, int pld,
                                                         int r, int64_t n,
                                                         const double* __restrict__ wts,
                                                         double* __restrict__ SI,
                                                         double* __restrict__ Sj) {
  const int64_t a = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (a >= n) return;
  const double* row = P + a * pld;
  double s0 = 0.0, s1 = 0.0;
  for (int col = lane; col < r; col += 64) {
    const double p = row[col];
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

}  // namespace

hipError_t launch_panel_correct(const double* P, int pld, int r, int64_t n, const IdList& I,
                                int32_t j, double* wts, double* SI, double* Sj, hipStream_t s) {
  if (r <= 0 || n <= 0) return hipSuccess;
  panel_weights_kernel<<<(unsigned)((r + 255) / 256), 256, 0, s>>>(P, pld, r, I, j, wts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  panel_gemv_kernel<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(P, pld, r, n, wts,
                                                            I.count ? SI : nullptr,
                                                            j >= 0 ? Sj : nullptr);
  return hipGetLastError();
}

hipError_t launch_delta_col(const double* P, int pld, int r, int64_t n, int32_t x, double* out,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  delta_col_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, pld, r, n, x, out);
  return hipGetLastError();
}

template <int PREC, bool MASK, bool COLOUT>
static void strip_launch(const LowRankArgs& a, dim3 grid, hipStream_t s) {
  if (a.rows)
    lowrank_strip_kernel<PREC, MASK, COLOUT, true><<<grid, NT, 0, s>>>(a);
  else
    lowrank_strip_kernel<PREC, MASK, COLOUT, false><<<grid, NT, 0, s>>>(a);
}

hipError_t launch_lowrank(const LowRankArgs& a, hipStream_t s) {
  if (a.ncols <= 0 || (a.nrows_dev == nullptr && a.nrows <= 0)) return hipSuccess;
  const int64_t nrows_bound = a.nrows_dev ? (a.rows ? a.ncols : a.nrows) : a.nrows;
  if (a.r > RC && (a.rows != nullptr || a.nrows_dev != nullptr || a.Ahat != nullptr)) {
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
  if (a.r <= RC) {
    const int64_t strips = (a.ncols + SC - 1) / SC;
    const int64_t rtiles = (nrows_bound + TR - 1) / TR;
    int64_t gy = (4096 + strips - 1) / strips;
    if (gy > rtiles) gy = rtiles;
    if (gy < 1) gy = 1;
    dim3 grid((unsigned)strips, (unsigned)gy);
    const bool mask = a.Ahat != nullptr && a.out == nullptr;
    if (a.out) {
      strip_launch<PREC_FP64, false, true>(a, grid, s);
    } else if (a.S.prec == PREC_FP64) {
      mask ? strip_launch<PREC_FP64, true, false>(a, grid, s)
           : strip_launch<PREC_FP64, false, false>(a, grid, s);
    } else if (a.S.prec == PREC_HILO) {
      mask ? strip_launch<PREC_HILO, true, false>(a, grid, s)
           : strip_launch<PREC_HILO, false, false>(a, grid, s);
    } else {
      mask ? strip_launch<PREC_FP32, true, false>(a, grid, s)
           : strip_launch<PREC_FP32, false, false>(a, grid, s);
    }
    return hipGetLastError();
  }
  // Several blocks: the fused GEMM (all rows and columns; rows list and mask not used).
  if (a.rows != nullptr || a.nrows_dev != nullptr || a.Ahat != nullptr || a.out != nullptr)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((a.ncols + GT - 1) / GT), (unsigned)((a.nrows + GT - 1) / GT));
  if (a.S.prec == PREC_FP64) {
    lowrank_gemm_kernel<PREC_FP64><<<grid, NT, 0, s>>>(a);
  } else if (a.S.prec == PREC_HILO) {
    lowrank_gemm_kernel<PREC_HILO><<<grid, NT, 0, s>>>(a);
  } else {
    lowrank_gemm_kernel<PREC_FP32><<<grid, NT, 0, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_lowrank_ref(const LowRankArgs& a, hipStream_t s) {
  const int64_t nrows = a.nrows_dev ? a.ncols : a.nrows;  // upper bound; kernel checks
  if (a.ncols <= 0 || nrows <= 0) return hipSuccess;
  dim3 grid((unsigned)nrows, (unsigned)((a.ncols + 255) / 256));
  lowrank_ref_kernel<<<grid, 256, 0, s>>>(a);
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

}  // namespace sr
