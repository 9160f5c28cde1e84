// Block store of S (Example 1.1): reads of S through the pairs of partition blocks, the
// flags that tell which pairs a fused pass reaches, and the placement of a block's S_Gi.
// The fused pass itself is lowrank_gemm_kernel's block mode (update.hip).
#include "kernels.h"

namespace sr {

namespace {

constexpr int kB = 256;

inline unsigned g1(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// S[a][b] from the store: pair (part[a], part[b]) when part[a] <= part[b], else the transposed
// entry of pair (part[b], part[a]); zero when that pair holds nothing.
__device__ __forceinline__ double bs_get(const BlockStore& B, int64_t a, int64_t b) {
  const int32_t p = B.part[a], q = B.part[b];
  const bool up = p <= q;
  const SView v = B.pairs[up ? (int64_t)p * B.np + q : (int64_t)q * B.np + p];
  if (v.d == nullptr) return 0.0;
  const int64_t la = B.loc[a], lb = B.loc[b];
  return s_get(v, up ? la * v.ld + lb : lb * v.ld + la);
}

__global__ __launch_bounds__(kB) void bs_gather_rows_kernel(BlockStore B, int64_t n, IdList I,
                                                            int32_t j, double* __restrict__ SI,
                                                            double* __restrict__ Sj,
                                                            const double* __restrict__ cI,
                                                            const double* __restrict__ cJ) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  double s = 0.0;
  for (int t = 0; t < I.count; ++t) s += bs_get(B, I.at(t), a);
  SI[a] = cI ? s + cI[a] : s;
  if (j >= 0) {
    const double v = bs_get(B, j, a);
    Sj[a] = cJ ? v + cJ[a] : v;
  }
}

__global__ __launch_bounds__(kB) void bs_rows_kernel(BlockStore B, int64_t n,
                                                     const int32_t* __restrict__ rows,
                                                     double* __restrict__ out,
                                                     float* __restrict__ out32, int64_t ld,
                                                     int64_t nrows) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  for (int64_t t = blockIdx.y; t < nrows; t += gridDim.y) {
    const double v = bs_get(B, rows[t], a);
    if (out32)
      out32[t * ld + a] = (float)v;
    else
      out[t * ld + a] = v;
  }
}

__global__ __launch_bounds__(kB) void bs_pairs_kernel(BlockStore B, int64_t cnt,
                                                      const int32_t* __restrict__ pa,
                                                      const int32_t* __restrict__ pb,
                                                      double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (t < cnt) out[t] = bs_get(B, pa[t], pb[t]);
}

// One thread per (node, deferred block): a nonzero xi_k (eta_k) entry in the node's panel row
// marks the node's partition block for that deferred block and term k. Stores of the value 1
// from many threads to one flag need no atomics.
__global__ __launch_bounds__(kB) void bs_touch_kernel(const double* __restrict__ P, int pld,
                                                      int64_t gstride, int nk, int64_t n,
                                                      const int32_t* __restrict__ part,
                                                      int32_t np, uint32_t* __restrict__ flags) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int d = blockIdx.y;
  if (a >= n) return;
  const double* row = P + (int64_t)d * gstride + a * pld;
  uint32_t* f = flags + ((int64_t)d * np + part[a]) * nk * 2;
  for (int k = 0; k < nk; ++k) {
    const double2 v = *reinterpret_cast<const double2*>(row + 2 * k);
    if (v.x != 0.0) f[2 * k] = 1u;
    if (v.y != 0.0) f[2 * k + 1] = 1u;
  }
}

__global__ __launch_bounds__(kB) void bs_place_kernel(SView dst, const double* __restrict__ Sb,
                                                      int64_t ldb, int64_t nb) {
  const int64_t c = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (c >= nb) return;
  for (int64_t r = blockIdx.y; r < nb; r += gridDim.y)
    s_put(dst, r * dst.ld + c, Sb[r * ldb + c]);
}

}  // namespace

hipError_t launch_bs_gather_rows(const BlockStore& B, int64_t n, const IdList& I, int32_t j,
                                 double* SI, double* Sj, const double* cI, const double* cJ,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  bs_gather_rows_kernel<<<g1(n), kB, 0, s>>>(B, n, I, j, SI, Sj, cI, cJ);
  return hipGetLastError();
}

hipError_t launch_bs_rows(const BlockStore& B, int64_t n, const int32_t* rows, int64_t nrows,
                          double* out, float* out32, int64_t ld_out, hipStream_t s) {
  if (n <= 0 || nrows <= 0) return hipSuccess;
  if (ld_out < n) return hipErrorInvalidValue;
  const unsigned gy = (unsigned)(nrows < 4096 ? nrows : 4096);
  bs_rows_kernel<<<dim3(g1(n), gy), kB, 0, s>>>(B, n, rows, out, out32, ld_out, nrows);
  return hipGetLastError();
}

hipError_t launch_bs_pairs(const BlockStore& B, int64_t cnt, const int32_t* a,
                           const int32_t* b, double* out, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  bs_pairs_kernel<<<g1(cnt), kB, 0, s>>>(B, cnt, a, b, out);
  return hipGetLastError();
}

hipError_t launch_bs_touch(const double* P, int pld, int64_t gstride, int q, int nk, int64_t n,
                           const int32_t* part, int32_t np, uint32_t* flags, hipStream_t s) {
  if (n <= 0 || q <= 0) return hipSuccess;
  if (q > 65535 || 2 * nk > pld || pld % 2 != 0) return hipErrorInvalidValue;
  bs_touch_kernel<<<dim3(g1(n), (unsigned)q), kB, 0, s>>>(P, pld, gstride, nk, n, part, np,
                                                          flags);
  return hipGetLastError();
}

hipError_t launch_bs_place(SView dst, const double* Sb, int64_t ldb, int64_t nb,
                           hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const unsigned gy = (unsigned)(nb < 4096 ? nb : 4096);
  bs_place_kernel<<<dim3(g1(nb), gy), kB, 0, s>>>(dst, Sb, ldb, nb);
  return hipGetLastError();
}

}  // namespace sr
