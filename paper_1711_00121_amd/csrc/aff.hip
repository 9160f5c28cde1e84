// Affected areas of Theorem 4 (eqs (39)-(41)) as bitmaps, and their bit-exact compaction.
//
// Level 0 is built on the old graph: A_0 = {j}, B_0 = F1 | F2 | {j}, F1 = out_old(supp S[i, :])
// (union over the block's sources; computed in pull form by the Q S[:, I] traversal), F2 =
// supp S[j, :] when row j of Q is nonempty before an insertion or after a deletion. Later
// levels use the new graph and the product-of-projections reading
// A_{k+1} = out_new(A_0 | .. | A_k), evaluated in pull form by the series-step traversal.
// Since A_1 c A_2 c ... for k >= 1, the union A_0 | .. | A_k equals A_0 | A_k, and
// A_hat = A_0 | A_K. The same holds for B.
#include "kernels.h"

namespace sr {

namespace {

constexpr int kB = 256;

__global__ __launch_bounds__(kB) void aff_level0_kernel(AffArgs a,
                                                        const uint32_t* __restrict__ suppJ,
                                                        int f2, int32_t j) {
  const int64_t w = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (w < a.W && f2) a.B[w] |= suppJ[w];
  if (w == (j >> 5)) {
    a.A[w] |= 1u << (j & 31);
    a.B[w] |= 1u << (j & 31);
  }
}

__global__ __launch_bounds__(kB) void bits_or_kernel(const uint32_t* __restrict__ x,
                                                     const uint32_t* __restrict__ y,
                                                     uint32_t* __restrict__ d, int W) {
  const int w = blockIdx.x * kB + threadIdx.x;
  if (w < W) d[w] = x[w] | y[w];
}

constexpr int kC = 1024;

// Exclusive scan of one value per thread over a 1024-thread block (wave scans + one pass over
// the 16 wave totals). Returns the exclusive prefix; *total receives the sum.
__device__ int64_t block_exscan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[kC / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int w = 0; w < kC / 64; ++w) {
      const int64_t t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    *total = run;
  }
  __syncthreads();
  return wsum[wid] + x - v;
}

__device__ __forceinline__ void emit_bits(uint32_t word, int64_t base, int32_t* out,
                                          int64_t& pos) {
  while (word) {
    const int b = __builtin_ctz(word);
    out[pos++] = (int32_t)(base + b);
    word &= word - 1;
  }
}

// Row-list entries of the S update: (node << 2) | (in A_hat << 1) | (in B_hat), for the nodes
// of sel (a subset of x | y).
__device__ __forceinline__ void emit_rows(uint32_t x, uint32_t y, uint32_t sel, int64_t base,
                                          int32_t* out, int64_t& pos) {
  uint32_t word = sel;
  while (word) {
    const int b = __builtin_ctz(word);
    out[pos++] = (int32_t)(((base + b) << 2) | (((x >> b) & 1u) << 1) | ((y >> b) & 1u));
    word &= word - 1;
  }
}

// The pairs to update are A_hat x B_hat u B_hat x A_hat. Let X be the smaller of the two
// sets and Y the other. The streaming update gives each listed row its pairs with every
// column; a row y of Y \ X pairs only with the columns of X, so when X is small (at most
// n / 16 nodes) those rows are left out of the list and filled afterwards by copying the
// transposed entries S[y][x] = S[x][y] (launch_aff_mirror): |X| |Y \ X| entries instead of
// |Y \ X| whole rows. cnt[3] = listed rows, cnt[6] = |Y \ X| when mirrored (else 0).
__global__ __launch_bounds__(kC) void aff_compact_kernel(AffArgs a, uint32_t* __restrict__ Ahat,
                                                         uint32_t* __restrict__ Bhat,
                                                         int32_t* __restrict__ rows,
                                                         int32_t* __restrict__ mrows,
                                                         int64_t* __restrict__ cnt) {
  __shared__ int64_t tot;
  __shared__ int64_t red[3][kC / 64];
  __shared__ int mode;  // 0: rows A_hat | B_hat; 1: rows A_hat, mirror B_hat \ A_hat; 2: swapped
  const int W = a.W;
  const int chunk = (W + kC - 1) / kC;
  const int w0 = threadIdx.x * chunk;
  const int w1 = min(W, w0 + chunk);
  const uint32_t* A0 = a.A;
  const uint32_t* AK = a.A + (int64_t)a.K * W;
  const uint32_t* B0 = a.B;
  const uint32_t* BK = a.B + (int64_t)a.K * W;
  int64_t cA = 0, cB = 0, cAB = 0;
  for (int w = w0; w < w1; ++w) {
    const uint32_t x = A0[w] | AK[w];
    const uint32_t y = B0[w] | BK[w];
    Ahat[w] = x;
    Bhat[w] = y;
    cA += __popc(x);
    cB += __popc(y);
    cAB += __popc(x & y);
  }
  // counts first: the orientation depends on them
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    cA += __shfl_xor(cA, o, 64);
    cB += __shfl_xor(cB, o, 64);
    cAB += __shfl_xor(cAB, o, 64);
  }
  if (lane == 0) {
    red[0][wid] = cA;
    red[1][wid] = cB;
    red[2][wid] = cAB;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s0 = 0, s1 = 0, s2 = 0;
    for (int w = 0; w < kC / 64; ++w) {
      s0 += red[0][w];
      s1 += red[1][w];
      s2 += red[2][w];
    }
    cnt[0] = s0;
    cnt[1] = s1;
    cnt[2] = s2;
    const int64_t small = s0 <= s1 ? s0 : s1;
    const int64_t rest = (s0 <= s1 ? s1 : s0) - s2;  // |Y \ X|
    mode = (rest > 0 && 16 * small <= a.n) ? (s0 <= s1 ? 1 : 2) : 0;
  }
  __syncthreads();
  const int md = mode;
  int64_t cR = 0, cM = 0;
  for (int w = w0; w < w1; ++w) {
    const uint32_t x = Ahat[w], y = Bhat[w];
    cR += __popc(md == 0 ? (x | y) : (md == 1 ? x : y));
    cM += __popc(md == 0 ? 0u : (md == 1 ? (y & ~x) : (x & ~y)));
  }
  int64_t pos = block_exscan(cR, &tot);
  for (int w = w0; w < w1; ++w) {
    const uint32_t x = Ahat[w], y = Bhat[w];
    emit_rows(x, y, md == 0 ? (x | y) : (md == 1 ? x : y), (int64_t)w * 32, rows, pos);
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[3] = tot;
  __syncthreads();
  int64_t mpos = block_exscan(cM, &tot);
  if (md != 0)
    for (int w = w0; w < w1; ++w) {
      const uint32_t x = Ahat[w], y = Bhat[w];
      emit_bits(md == 1 ? (y & ~x) : (x & ~y), (int64_t)w * 32, mrows, mpos);
    }
  if (threadIdx.x == 0) cnt[6] = md == 0 ? 0 : tot;
}

// S[y][x] = S[x][y] for x in the listed rows (packed entries, cnt[3] of them) and y in the
// mirror list (cnt[6] entries): the stored element is copied as it is (value and
// compensation), so those pairs hold exactly their transposes' updated values.
template <typename E>
__global__ __launch_bounds__(kB) void aff_mirror_kernel(E* __restrict__ S, int64_t ld,
                                                        const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ mrows,
                                                        const int64_t* __restrict__ cnt) {
  const int64_t ny = cnt[6];
  if (ny == 0) return;
  const int64_t total = cnt[3] * ny;
  for (int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kB) {
    const int64_t x = (int64_t)(rows[t / ny] >> 2);
    const int64_t y = mrows[t % ny];
    S[y * ld + x] = S[x * ld + y];
  }
}

__global__ __launch_bounds__(kC) void bits_to_list_kernel(const uint32_t* __restrict__ bm,
                                                          int W, int32_t* __restrict__ out,
                                                          int64_t* __restrict__ cnt) {
  __shared__ int64_t tot;
  const int chunk = (W + kC - 1) / kC;
  const int w0 = threadIdx.x * chunk;
  const int w1 = min(W, w0 + chunk);
  int64_t c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bm[w]);
  int64_t pos = block_exscan(c, &tot);
  if (out)
    for (int w = w0; w < w1; ++w) emit_bits(bm[w], (int64_t)w * 32, out, pos);
  if (threadIdx.x == 0) *cnt = tot;
}

}  // namespace

hipError_t launch_aff_level0(const AffArgs& a, const uint32_t* suppJ, int f2, int32_t j,
                             hipStream_t s) {
  aff_level0_kernel<<<(unsigned)((a.W + kB - 1) / kB), kB, 0, s>>>(a, suppJ, f2, j);
  return hipGetLastError();
}

hipError_t launch_aff_compact(const AffArgs& a, uint32_t* Ahat, uint32_t* Bhat, int32_t* rows,
                              int32_t* mrows, int64_t* cnt, hipStream_t s) {
  aff_compact_kernel<<<1, kC, 0, s>>>(a, Ahat, Bhat, rows, mrows, cnt);
  return hipGetLastError();
}

hipError_t launch_aff_mirror(SView S, const int32_t* rows, const int32_t* mrows,
                             const int64_t* cnt, hipStream_t s) {
  constexpr unsigned grid = 2048;
  if (S.prec == PREC_FP64)
    aff_mirror_kernel<double><<<grid, kB, 0, s>>>(S.d, S.ld, rows, mrows, cnt);
  else if (S.prec == PREC_HILO)
    aff_mirror_kernel<float2><<<grid, kB, 0, s>>>(S.hl, S.ld, rows, mrows, cnt);
  else
    aff_mirror_kernel<float><<<grid, kB, 0, s>>>(S.hi, S.ld, rows, mrows, cnt);
  return hipGetLastError();
}

hipError_t launch_bits_to_list(const uint32_t* bm, int64_t n, int32_t W, int32_t* out,
                               int64_t* cnt, hipStream_t s) {
  (void)n;
  bits_to_list_kernel<<<1, kC, 0, s>>>(bm, W, out, cnt);
  return hipGetLastError();
}

hipError_t launch_bits_or(const uint32_t* a, const uint32_t* b, uint32_t* dst, int32_t W,
                          hipStream_t s) {
  bits_or_kernel<<<(unsigned)((W + kB - 1) / kB), kB, 0, s>>>(a, b, dst, W);
  return hipGetLastError();
}

}  // namespace sr
