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

// Y[b][:] = scale (Q^T X)[b][:] = scale sum_{a in out(b)} Q[a][b] X[a][:] (+ Gadd[b][:]),
// one workgroup per row b and 256 columns; with prev, maxdiff = max |Y - prev|. The weights
// Q[a][b] of the out-list slots are precomputed (qv, one per slot), so a gathered neighbour
// row costs one uniform index load, one uniform value load and one vector load per lane, 8
// neighbours' row loads issued together. Columns past n read the zero padding of the
// leading dimension (c < ldi always).
//
// Measured at n = 20k, m = 200k (adjoint workload): 5.8 ms per launch, with the gathers
// fetching about 25 GB from the data fabric per launch (the rows of a 256-column chunk of X
// take 40 MB, over an XCD's 4 MB L2). Forming Q[a][b] at every use instead took 7.0 ms;
// 16 neighbours in flight 6.1 ms; two rows per workgroup 6.7 ms; column tiles small enough
// for an XCD's L2 (16, 32, 64 columns, each XCD taking whole tiles) 13.8, 9.6 and 7.1 ms,
// since every lane then loads its own indices and values.
template <int U, int RW>
__global__ __launch_bounds__(kRowT) void spmm_qt_rows_kernel(DevAdj out, const double* qv,
                                                           int64_t n, int64_t ldi,
                                                           const double* __restrict__ X,
                                                           double* __restrict__ Y, double scale,
                                                           const double* __restrict__ Gadd,
                                                           const double* __restrict__ prev,
                                                           unsigned long long* maxdiff) {
  __shared__ double red[kRowT / 64];
  const int64_t c = ((int64_t)blockIdx.y * kRowT + threadIdx.x) * 2;
  const int64_t cc = c < ldi ? c : 0;
  double diff = 0.0;
  // RW rows per workgroup, their neighbour batches interleaved (more gathers in flight)
  int64_t bb[RW];
  int len[RW], st[RW], lmax = 0;
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    bb[r] = (int64_t)blockIdx.x * RW + r;
    const bool ok = bb[r] < n;
    len[r] = ok ? out.len[bb[r]] : 0;
    st[r] = ok ? out.start[bb[r]] : 0;
    lmax = len[r] > lmax ? len[r] : lmax;
  }
  double2 acc[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int p0 = 0; p0 < lmax; p0 += U) {
    int64_t a[RW][U];
    double qa[RW][U];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = p0 + u < len[r];
        const int p = in ? p0 + u : 0;
        a[r][u] = len[r] ? out.idx[st[r] + p] : 0;
        qa[r][u] = in ? qv[st[r] + p] : 0.0;
      }
    double2 v[RW][U];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u)
        v[r][u] = *reinterpret_cast<const double2*>(X + a[r][u] * ldi + cc);
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc[r].x += qa[r][u] * v[r][u].x;
        acc[r].y += qa[r][u] * v[r][u].y;
      }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const int64_t b = bb[r];
    if (b >= n || c >= n) continue;
    double2 o = make_double2(scale * acc[r].x, scale * acc[r].y);
    if (Gadd) {
      const double2 gv = load_stream(Gadd + b * ldi + c);
      o.x += gv.x;
      o.y += gv.y;
    }
    if (c + 1 >= n) o.y = 0.0;
    store_stream(Y + b * ldi + c, o);
    if (prev) {
      const double2 pv = load_stream(prev + b * ldi + c);
      diff = fmax(diff, fmax(fabs(o.x - pv.x), (c + 1 < n) ? fabs(o.y - pv.y) : 0.0));
    }
  }
  if (maxdiff) {
    for (int o = 32; o > 0; o >>= 1) diff = fmax(diff, __shfl_xor(diff, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = diff;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = red[0];
      for (int k = 1; k < kRowT / 64; ++k) m = fmax(m, red[k]);
      const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
      if (__hip_atomic_load(maxdiff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < mb)
        atomicMax(maxdiff, mb);
    }
  }
}

// qv[p] = Q[a][b] for out-list slot p of row b (a = out.idx[p]), over the slots of rows < n.
__global__ __launch_bounds__(kB) void qt_values_kernel(DevQ q, DevAdj out, int64_t n,
                                                       double* qv) {
  const int64_t b = (int64_t)blockIdx.x * (kB / 64) + (threadIdx.x >> 6);
  if (b >= n) return;
  const int len = out.len[b];
  const int st = out.start[b];
  for (int p = threadIdx.x & 63; p < len; p += 64) {
    const int64_t a = out.idx[st + p];
    qv[st + p] = q.W ? out.w[st + p] / q.W[a] : 1.0 / (double)q.in.len[a];
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

hipError_t launch_qt_values(const DevQ& q, const DevAdj& out, int64_t n, double* qv,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  qt_values_kernel<<<(unsigned)((n + kB / 64 - 1) / (kB / 64)), kB, 0, s>>>(q, out, n, qv);
  return hipGetLastError();
}

hipError_t launch_spmm_qt_rows(const DevAdj& out, const double* qv, int64_t n, const double* X,
                               double* Y, double scale, const double* Gadd, const double* prev,
                               unsigned long long* maxdiff, hipStream_t s) {
  dim3 grid((unsigned)n, (unsigned)((n + 2 * kRowT - 1) / (2 * kRowT)));
  spmm_qt_rows_kernel<8, 1><<<grid, kRowT, 0, s>>>(out, qv, n, ldi_of(n), X, Y, scale, Gadd,
                                                   prev, maxdiff);
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
