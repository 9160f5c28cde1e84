// Sparse traversals of the graph: products with the backward transition matrix Q and its
// transpose, the series step of eq (16a) fused with the affected-area level of Theorem 4, and
// in-place patches of the slotted CSR.
//
// Q[a][x] = 1/indeg(a) for an edge x -> a (section 3.1). Rows are in-lists by sink, so
// (Q x)[a] gathers over a's in-neighbours and (Q^T x)[b] over b's out-neighbours.
//
// Power-law rows: a row of at most kLight entries is handled by a group of 8 lanes that
// combine with shuffles. Longer rows ("heavy", listed by the host) are cut into chunks of
// kChunk entries, one 256-thread workgroup per chunk; each chunk writes a partial sum and the
// last chunk to finish (device-scope counter, no waiting) adds the partials in chunk order,
// so results do not depend on scheduling.
#include "kernels.h"

namespace sr {

namespace {

constexpr int kB = 256;
constexpr int kG = 8;                   // lanes per light row
constexpr int kRowsPerBlock = kB / kG;  // 32

__global__ __launch_bounds__(64) void patch_kernel(AdjPtrs t, Patch p) {
  int i = threadIdx.x;
  if (i < p.count) t.p[p.array[i]][p.index[i]] = p.value[i];
}

// What one traversal computes. Values per entry: NV = 1 (x) or 2 (xi, eta pair).
struct Op {
  int kind;             // 0: y = post*(base + scale*Q x); 1: series step; 2: y = scale*Q^T x
  const double* x;      // kind 0/2 input vector
  double* y;            // kind 0/2 output vector
  double scale, post;
  const double* base;
  double* P;            // kind 1 panel
  int pld, k;           // kind 1: columns 2k, 2k+1 -> 2k+2, 2k+3
  double sx, sy;
  // optional bitmaps (pull form of Theorem 4): out bit b = OR_{x in row b} (in0 | in1)(x)
  const uint32_t* a0;
  const uint32_t* a1;
  uint32_t* aout;
  const uint32_t* b0;
  const uint32_t* b1;
  uint32_t* bout;
};

__device__ __forceinline__ bool member(const uint32_t* s0, const uint32_t* s1, int64_t x) {
  return (s0 && bit_get(s0, x)) || (s1 && bit_get(s1, x));
}

// Accumulates the entries [p0, p1) of row `row` (list L) with stride `step` from lane `lane`.
__device__ __forceinline__ void accumulate(const Op& o, const DevQ& q, const DevAdj& L, int st,
                                           int p0, int p1, int lane, int step, double& v0,
                                           double& v1, bool& fa, bool& fb) {
  for (int p = p0 + lane; p < p1; p += step) {
    const int64_t x = L.idx[st + p];
    if (o.kind == 1) {
      const double2 v = *reinterpret_cast<const double2*>(o.P + x * o.pld + 2 * o.k);
      const double w = L.w ? L.w[st + p] : 1.0;
      v0 += w * v.x;
      v1 += w * v.y;
    } else if (o.kind == 0) {
      const double w = L.w ? L.w[st + p] : 1.0;
      v0 += w * o.x[x];
    } else {
      const double qa = q.W ? L.w[st + p] / q.W[x] : 1.0 / (double)q.in.len[x];
      v0 += qa * o.x[x];
    }
    if (o.aout && !fa) fa = member(o.a0, o.a1, x);
    if (o.bout && !fb) fb = member(o.b0, o.b1, x);
  }
}

__device__ __forceinline__ void finish(const Op& o, const DevQ& q, int64_t row, int len,
                                       double v0, double v1, bool fa, bool fb) {
  if (o.kind == 1) {
    double2 out = make_double2(0.0, 0.0);
    if (len > 0) {
      const double inv = q.W ? 1.0 / q.W[row] : 1.0 / (double)len;
      out.x = o.sx * (v0 * inv);
      out.y = o.sy * (v1 * inv);
    }
    *reinterpret_cast<double2*>(o.P + row * o.pld + 2 * (o.k + 1)) = out;
  } else if (o.kind == 0) {
    double v = 0.0;
    if (len > 0) v = q.W ? v0 / q.W[row] : v0 / (double)len;
    v *= o.scale;
    if (o.base) v += o.base[row];
    o.y[row] = o.post * v;
  } else {
    o.y[row] = o.scale * v0;
  }
  if (fa) bit_set_atomic(o.aout, row);
  if (fb) bit_set_atomic(o.bout, row);
}

__global__ __launch_bounds__(kB) void traverse_kernel(Op o, DevQ q, DevAdj L, int64_t n,
                                                      int64_t n_light_blocks, HeavyArgs h) {
  __shared__ double red0[kB / 64], red1[kB / 64];
  __shared__ int redf[kB / 64];
  __shared__ int is_last;
  if ((int64_t)blockIdx.x < n_light_blocks) {
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kG;
    const int lane = threadIdx.x % kG;
    double v0 = 0.0, v1 = 0.0;
    bool fa = false, fb = false;
    int len = 0;
    bool mine = false;
    if (row < n) {
      len = L.len[row];
      mine = len <= kLight;
      if (mine) accumulate(o, q, L, L.start[row], 0, len, lane, kG, v0, v1, fa, fb);
    }
    v0 = wave_sum(v0, kG);
    v1 = wave_sum(v1, kG);
    for (int s = kG >> 1; s > 0; s >>= 1) {
      fa |= (bool)__shfl_xor((int)fa, s, kG);
      fb |= (bool)__shfl_xor((int)fb, s, kG);
    }
    if (mine && lane == 0) finish(o, q, row, len, v0, v1, fa, fb);
    return;
  }
  // heavy chunk
  const int64_t hc = (int64_t)blockIdx.x - n_light_blocks;
  const int hi = (int)(hc / h.maxc);
  const int c = (int)(hc % h.maxc);
  if (hi >= h.nh) return;
  const int64_t row = h.rows[hi];
  const int len = L.len[row];
  const int nch = (len + kChunk - 1) / kChunk;
  if (c >= nch) return;
  double v0 = 0.0, v1 = 0.0;
  bool fa = false, fb = false;
  const int p0 = c * kChunk;
  const int p1 = min(len, p0 + kChunk);
  accumulate(o, q, L, L.start[row], p0, p1, threadIdx.x, kB, v0, v1, fa, fb);
  v0 = wave_sum(v0, 64);
  v1 = wave_sum(v1, 64);
  int fw = (fa ? 1 : 0) | (fb ? 2 : 0);
  for (int sh = 32; sh > 0; sh >>= 1) fw |= __shfl_xor(fw, sh, 64);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red0[wid] = v0;
    red1[wid] = v1;
    redf[wid] = fw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    int ff = 0;
    for (int w = 0; w < kB / 64; ++w) {
      s0 += red0[w];
      s1 += red1[w];
      ff |= redf[w];
    }
    double* part = h.partial + 2 * ((int64_t)hi * h.maxc + c);
    part[0] = s0;
    part[1] = s1;
    if ((ff & 1) && o.aout) bit_set_atomic(o.aout, row);
    if ((ff & 2) && o.bout) bit_set_atomic(o.bout, row);
    __threadfence();
    const unsigned prev = atomicAdd(h.counter + hi, 1u);
    is_last = (prev == (unsigned)(nch - 1));
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    __threadfence();
    double s0 = 0.0, s1 = 0.0;
    for (int cc = 0; cc < nch; ++cc) {
      const double* part = h.partial + 2 * ((int64_t)hi * h.maxc + cc);
      s0 += __hip_atomic_load(part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s1 += __hip_atomic_load(part + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    finish(o, q, row, len, s0, s1, false, false);
    h.counter[hi] = 0u;
  }
}

hipError_t run(const Op& o, const DevQ& q, const DevAdj& L, int64_t n, const HeavyArgs& h,
               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nlb = (n + kRowsPerBlock - 1) / kRowsPerBlock;
  const int64_t grid = nlb + (int64_t)h.nh * h.maxc;
  traverse_kernel<<<(unsigned)grid, kB, 0, s>>>(o, q, L, n, nlb, h);
  return hipGetLastError();
}

Op blank() {
  Op o{};
  o.scale = 1.0;
  o.post = 1.0;
  o.sx = 1.0;
  o.sy = 1.0;
  return o;
}

}  // namespace

hipError_t launch_patch(const AdjPtrs& t, const Patch& p, hipStream_t s) {
  if (p.count <= 0) return hipSuccess;
  patch_kernel<<<1, 64, 0, s>>>(t, p);
  return hipGetLastError();
}

hipError_t launch_spmv_q(const DevQ& q, const HeavyArgs& h, int64_t n, const double* x,
                         double* y, double scale, hipStream_t s, const double* base,
                         double post, const uint32_t* fin, uint32_t* fout) {
  Op o = blank();
  o.kind = 0;
  o.x = x;
  o.y = y;
  o.scale = scale;
  o.base = base;
  o.post = post;
  o.b0 = fin;
  o.bout = fout;
  return run(o, q, q.in, n, h, s);
}

hipError_t launch_spmv_qt(const DevQ& q, const DevAdj& out, const HeavyArgs& h, int64_t n,
                          const double* x, double* y, double scale, hipStream_t s) {
  Op o = blank();
  o.kind = 2;
  o.x = x;
  o.y = y;
  o.scale = scale;
  return run(o, q, out, n, h, s);
}

hipError_t launch_series_step(const DevQ& q, const HeavyArgs& h, int64_t n, double* P, int pld,
                              int k, double sx, double sy, const AffLevel* aff, hipStream_t s) {
  Op o = blank();
  o.kind = 1;
  o.P = P;
  o.pld = pld;
  o.k = k;
  o.sx = sx;
  o.sy = sy;
  if (aff) {
    o.a0 = aff->a0;
    o.a1 = aff->a1;
    o.aout = aff->aout;
    o.b0 = aff->b0;
    o.b1 = aff->b1;
    o.bout = aff->bout;
  }
  return run(o, q, q.in, n, h, s);
}

}  // namespace sr
