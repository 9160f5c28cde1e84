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

// Row-list entries of the S update: (node << 2) | (in A_hat << 1) | (in B_hat).
__device__ __forceinline__ void emit_rows(uint32_t x, uint32_t y, int64_t base, int32_t* out,
                                          int64_t& pos) {
  uint32_t word = x | y;
  while (word) {
    const int b = __builtin_ctz(word);
    out[pos++] = (int32_t)(((base + b) << 2) | (((x >> b) & 1u) << 1) | ((y >> b) & 1u));
    word &= word - 1;
  }
}

__global__ __launch_bounds__(kC) void aff_compact_kernel(AffArgs a, uint32_t* __restrict__ Ahat,
                                                         uint32_t* __restrict__ Bhat,
                                                         int32_t* __restrict__ rows,
                                                         int64_t* __restrict__ cnt) {
  __shared__ int64_t tot;
  __shared__ int64_t red[4][kC / 64];
  const int W = a.W;
  const int chunk = (W + kC - 1) / kC;
  const int w0 = threadIdx.x * chunk;
  const int w1 = min(W, w0 + chunk);
  const uint32_t* A0 = a.A;
  const uint32_t* AK = a.A + (int64_t)a.K * W;
  const uint32_t* B0 = a.B;
  const uint32_t* BK = a.B + (int64_t)a.K * W;
  int64_t cA = 0, cB = 0, cAB = 0, cR = 0;
  for (int w = w0; w < w1; ++w) {
    const uint32_t x = A0[w] | AK[w];
    const uint32_t y = B0[w] | BK[w];
    Ahat[w] = x;
    Bhat[w] = y;
    cA += __popc(x);
    cB += __popc(y);
    cAB += __popc(x & y);
    cR += __popc(x | y);
  }
  int64_t pos = block_exscan(cR, &tot);
  for (int w = w0; w < w1; ++w) emit_rows(Ahat[w], Bhat[w], (int64_t)w * 32, rows, pos);
  // counts
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
    cnt[3] = tot;
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
                              int64_t* cnt, hipStream_t s) {
  aff_compact_kernel<<<1, kC, 0, s>>>(a, Ahat, Bhat, rows, cnt);
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
