// Edge-weight gradient of a loss on S (not in the paper; it follows from eq (03a)).
//
// With G = dL/dS at the loss pairs, Lam = G + C Q^T Lam Q is the adjoint of eq (03a) and
// dL/dQ = C (Lam + Lam^T) Q S for symmetric S. Sig = Lam + Lam^T solves
// Sig = (G + G^T) + C Q^T Sig Q, so only the symmetric Sig is iterated. Row normalisation
// Q[x][y] = w(y -> x) / W_x gives dL/dw(y -> x) = (dL/dQ[x][y] - sum_y' Q[x][y'] dL/dQ[x][y'])/W_x.
#include "kernels.h"

namespace sr {

namespace {

constexpr int kB = 256;

inline int64_t ldi_of(int64_t n) { return (n + 63) / 64 * 64; }

__global__ __launch_bounds__(kB) void scatter_sym_kernel(double* G, int64_t ldi, int64_t np,
                                                         const int32_t* __restrict__ pa,
                                                         const int32_t* __restrict__ pb,
                                                         const double* __restrict__ g) {
  const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (p >= np) return;
  const int64_t a = pa[p], b = pb[p];
  atomicAdd(G + a * ldi + b, g[p]);
  atomicAdd(G + b * ldi + a, g[p]);
}

constexpr int kRowT = 128;  // threads of a row-gather workgroup (2 columns each)

__global__ __launch_bounds__(kRowT) void spmm_qt_rows_kernel(DevQ q, DevAdj out, int64_t n,
                                                          int64_t ldi,
                                                          const double* __restrict__ X,
                                                          double* __restrict__ Y, double scale,
                                                          const double* __restrict__ Gadd,
                                                          const double* __restrict__ prev,
                                                          unsigned long long* maxdiff) {
  __shared__ double red[kRowT / 64];
  const int64_t b = blockIdx.x;
  const int64_t c = ((int64_t)blockIdx.y * kRowT + threadIdx.x) * 2;
  const int len = out.len[b];
  const int st = out.start[b];
  // Out-neighbours are taken 8 at a time: the 8 row loads of X are issued together, so a
  // long row (a hub) costs one memory latency per 8 neighbours instead of one per neighbour.
  // Columns past n read the zero padding of the leading dimension (c < ldi always).
  constexpr int U = 8;
  double2 acc = make_double2(0.0, 0.0);
  const int64_t cc = c < ldi ? c : 0;
  for (int p0 = 0; p0 < len; p0 += U) {
    int64_t a[U];
    double qa[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u < len ? p0 + u : p0;
      a[u] = out.idx[st + p];
      qa[u] = p0 + u < len ? (q.W ? out.w[st + p] / q.W[a[u]] : 1.0 / (double)q.in.len[a[u]])
                           : 0.0;
    }
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = *reinterpret_cast<const double2*>(X + a[u] * ldi + cc);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc.x += qa[u] * v[u].x;
      acc.y += qa[u] * v[u].y;
    }
  }
  double diff = 0.0;
  if (c < n) {
    double2 o = make_double2(scale * acc.x, scale * acc.y);
    if (Gadd) {
      const double2 gv = load_stream(Gadd + b * ldi + c);
      o.x += gv.x;
      o.y += gv.y;
    }
    if (c + 1 >= n) o.y = 0.0;
    store_stream(Y + b * ldi + c, o);
    if (prev) {
      const double2 pv = load_stream(prev + b * ldi + c);
      diff = fmax(fabs(o.x - pv.x), (c + 1 < n) ? fabs(o.y - pv.y) : 0.0);
    }
  }
  if (maxdiff) {
    for (int o = 32; o > 0; o >>= 1) diff = fmax(diff, __shfl_xor(diff, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = diff;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = red[0];
      for (int w = 1; w < kRowT / 64; ++w) m = fmax(m, red[w]);
      // the maximum only grows during a launch: skip the atomic when it is already larger
      const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
      if (__hip_atomic_load(maxdiff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < mb)
        atomicMax(maxdiff, mb);
    }
  }
}

// One workgroup of 1024 threads per sink x. Each wave takes one in-edge slot at a time and
// forms dq = C <Sig[x, :], T[y, :]> with a wave-level reduction (no workgroup barrier per
// edge); then the row term sum_p Q[x][y_p] dq[p] is reduced in slot order and every edge gets
// its gradient.
constexpr int kEB = 1024;
__global__ __launch_bounds__(kEB) void edge_grad_kernel(DevQ q, int64_t n, int64_t ldi,
                                                        const double* __restrict__ Sig,
                                                        const double* __restrict__ T, double C,
                                                        const int32_t* __restrict__ slot_edge,
                                                        double* __restrict__ dq,
                                                        double* __restrict__ dw) {
  __shared__ double red[kEB / 64];
  const int64_t x = blockIdx.x;
  const int len = q.in.len[x];
  if (len == 0) return;
  const int st = q.in.start[x];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double* sx = Sig + x * ldi;
  for (int p = wid; p < len; p += kEB / 64) {
    const int64_t y = q.in.idx[st + p];
    const double* ty = T + y * ldi;
    double part = 0.0;
    for (int64_t c = lane; c < n; c += 64) part += sx[c] * ty[c];
    part = wave_sum(part, 64);
    if (lane == 0) dq[st + p] = C * part;
  }
  __syncthreads();
  // row term, in slot order per thread, then a fixed tree over the waves
  double rt = 0.0;
  for (int p = threadIdx.x; p < len; p += kEB) {
    const double qxy = q.W ? q.in.w[st + p] / q.W[x] : 1.0 / (double)len;
    rt += qxy * dq[st + p];
  }
  rt = wave_sum(rt, 64);
  if (lane == 0) red[wid] = rt;
  __syncthreads();
  double rowterm = 0.0;
  for (int w = 0; w < kEB / 64; ++w) rowterm += red[w];
  const double Wx = q.W ? q.W[x] : (double)len;
  for (int p = threadIdx.x; p < len; p += kEB) {
    const int32_t e = slot_edge[st + p];
    if (e >= 0) dw[e] = (dq[st + p] - rowterm) / Wx;
  }
}

}  // namespace

hipError_t launch_scatter_pairs_sym(double* G, int64_t n, int64_t np, const int32_t* a,
                                    const int32_t* b, const double* g, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  scatter_sym_kernel<<<(unsigned)((np + kB - 1) / kB), kB, 0, s>>>(G, ldi_of(n), np, a, b, g);
  return hipGetLastError();
}

hipError_t launch_spmm_qt_rows(const DevQ& q, const DevAdj& out, int64_t n, const double* X,
                               double* Y, double scale, const double* Gadd, const double* prev,
                               unsigned long long* maxdiff, hipStream_t s) {
  dim3 grid((unsigned)n, (unsigned)((n + 2 * kRowT - 1) / (2 * kRowT)));
  spmm_qt_rows_kernel<<<grid, kRowT, 0, s>>>(q, out, n, ldi_of(n), X, Y, scale, Gadd, prev,
                                          maxdiff);
  return hipGetLastError();
}

hipError_t launch_edge_grad(const DevQ& q, int64_t n, const double* Sig, const double* T,
                            double C, const int32_t* slot_edge, double* dq, double* dw,
                            hipStream_t s) {
  edge_grad_kernel<<<(unsigned)n, kEB, 0, s>>>(q, n, ldi_of(n), Sig, T, C, slot_edge, dq,
                                               dw);
  return hipGetLastError();
}

}  // namespace sr
