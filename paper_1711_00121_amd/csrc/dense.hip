// Dense-S kernels: row gathers and the gamma vector of the rank-one Sylvester equation
// (Theorems 2, 3, 7, 9 and Table 2), new-node writes (Theorem 8, Algorithm 5), the initial S
// by the fixed point of eq (03a), and queries.
#include <algorithm>

#include "kernels.h"

namespace sr {

namespace {

constexpr int kB = 256;

__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* dst) {
  // v >= 0: the IEEE bit patterns of nonnegative doubles order like unsigned integers.
  __shared__ double red[kB / 64];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    // The maximum only grows during a launch, so a block whose value does not exceed the one
    // already there skips the atomic: with one address and ~10^6 blocks, unconditional
    // atomics serialise and dominate the launch.
    const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
    if (__hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < mb)
      atomicMax(dst, mb);
  }
}

__global__ __launch_bounds__(kB) void gather_rows_kernel(SView S, int64_t n, IdList I, int acc,
                                                         int32_t j, double* __restrict__ SI,
                                                         double* __restrict__ Sj,
                                                         uint32_t* __restrict__ suppI,
                                                         uint32_t* __restrict__ suppJ,
                                                         const double* __restrict__ cI,
                                                         const double* __restrict__ cJ) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  const bool in = a < n;
  double s = (in && acc) ? SI[a] : 0.0;
  bool sup = false;
  if (in) {
    for (int t = 0; t < I.count; ++t) {
      const double v = s_get(S, (int64_t)I.at(t) * S.ld + a);
      s += v;
      sup |= (v != 0.0);
    }
    SI[a] = cI ? s + cI[a] : s;
  }
  const uint64_t bI = __ballot(sup);
  const int lane = threadIdx.x & 63;
  const int64_t word = a >> 5;
  if (lane == 0 || lane == 32) {
    const uint32_t bits = (uint32_t)(lane == 0 ? bI : (bI >> 32));
    if (a < n) suppI[word] = acc ? (suppI[word] | bits) : bits;
  }
  if (j >= 0) {
    bool supj = false;
    if (in) {
      const double v = s_get(S, (int64_t)j * S.ld + a);
      Sj[a] = cJ ? v + cJ[a] : v;
      supj = v != 0.0;
    }
    const uint64_t bJ = __ballot(supj);
    if ((lane == 0 || lane == 32) && a < n)
      suppJ[word] = (uint32_t)(lane == 0 ? bJ : (bJ >> 32));
  }
}

__global__ __launch_bounds__(kB) void gather_inrows_kernel(SView S, int64_t n, DevQ q, int32_t j,
                                                           double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  const int len = q.in.len[j];
  const int st = q.in.start[j];
  double s = 0.0;
  for (int p = 0; p < len; ++p) s += s_get(S, (int64_t)q.in.idx[st + p] * S.ld + a);
  out[a] = s;
}

__device__ __forceinline__ double sum_at(const double* v, const IdList& I) {
  double s = 0.0;
  for (int t = 0; t < I.count; ++t) s += v[I.at(t)];
  return s;
}

// One wave: out[0] = sum over the list of v[I.at(t)], lane-strided partial sums combined in a
// fixed order.
__global__ __launch_bounds__(64) void sum_at_kernel(const double* __restrict__ v, IdList I,
                                                    double* __restrict__ out) {
  double s = 0.0;
  for (int t = threadIdx.x; t < I.count; t += 64) s += v[I.at(t)];
  s = wave_sum(s, 64);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(kB) void direct_z_kernel(GammaArgs g, int64_t n,
                                                      const double* __restrict__ SI,
                                                      const double* __restrict__ zsum,
                                                      double* __restrict__ z) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  const double d = (double)g.delta;
  const double si = SI[a] / d;
  double v;
  if (g.op > 0) {
    v = (g.dj == 0) ? si : si - zsum[a] / (double)g.dj;
  } else {
    v = (g.dj == g.delta) ? -si : zsum[a] / (double)g.dj - si;
  }
  z[a] = v;
}

__global__ __launch_bounds__(kB) void gamma_kernel(GammaArgs g, int64_t n,
                                                   const double* __restrict__ SI,
                                                   const double* __restrict__ Sj,
                                                   const double* __restrict__ QSI,
                                                   const double* __restrict__ z,
                                                   const double* __restrict__ Qz,
                                                   double* __restrict__ P, int pld,
                                                   unsigned long long* maxabs) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  const double C = g.C;
  const double d = (double)g.delta;
  const double dj = (double)g.dj;
  const bool isj = (a == g.j);
  double gam = 0.0;
  if (a < n) {
    if (g.kind == 0) {
      // Theorem 3 (eqs (29aa), (29bb), (29b)), Theorem 9, Table 2 rows (C0).
      const double SII = g.sumI ? *g.sumI : sum_at(SI, g.I);
      const double lam = SII / (d * d) + Sj[g.j] / C - (2.0 / d) * QSI[g.j] - 1.0 / C + 1.0;
      if (g.op > 0) {
        if (g.dj == 0) {
          gam = QSI[a] / d + (isj ? SII / (2.0 * d * d) : 0.0);
        } else {
          const double f = d / (dj + d);
          gam = f * (QSI[a] / d - Sj[a] / C +
                     (isj ? lam * d / (2.0 * (dj + d)) + 1.0 / C - 1.0 : 0.0));
        }
      } else {
        if (g.dj == g.delta) {
          gam = -QSI[a] / d + (isj ? SII / (2.0 * d * d) : 0.0);
        } else {
          const double f = d / (dj - d);
          gam = f * (Sj[a] / C - QSI[a] / d +
                     (isj ? lam * d / (2.0 * (dj - d)) - 1.0 / C + 1.0 : 0.0));
        }
      }
    } else if (g.kind == 1) {
      // Theorem 2, eq (20): w = Q z + (v^T z / 2) u with z = S v; gamma = u_j w.
      const double zI = (g.sumI ? *g.sumI : sum_at(z, g.I)) / d;
      double vz, uj;
      if (g.op > 0) {
        vz = (g.dj == 0) ? zI : zI - Qz[g.j];
        uj = (g.dj == 0) ? 1.0 : d / (dj + d);
      } else {
        vz = (g.dj == g.delta) ? -zI : Qz[g.j] - zI;
        uj = (g.dj == g.delta) ? 1.0 : d / (dj - d);
      }
      gam = uj * (Qz[a] + (isj ? 0.5 * vz * uj : 0.0));
    } else if (g.kind == 2) {
      // Eq (60) and Table 2 row (C2): the z vector is eta_0. A weighted new source of weight
      // w takes a = w / (W_j + w) in place of 1 / (d_j + 1) (delta = 1).
      const double sjj = Sj[g.j];
      const double diag = g.alpha > 0.0
                              ? g.alpha * (sjj - (1.0 - C) * (1.0 - C)) / (2.0 * C)
                              : (d * sjj - (d - C) * (1.0 - C)) / (2.0 * C * (dj + d));
      gam = (isj ? diag + (1.0 - C) / C : 0.0) - Sj[a] / C;
    } else {
      // A weighted edge change i -> j by dw, Delta Q = e_j a (e_i - Q[j, :])^T with
      // a = dw / (W_j + dw): Theorem 3's closed form with a in place of 1 / (d_j + 1)
      // (it rests only on the fixed-point identity of eq (33)),
      //   gamma = a (Q S e_i - S e_j / C) + (a (1 - C) / C + a^2 lambda / 2) e_j.
      const double al = g.alpha;
      const double Sii = sum_at(SI, g.I);
      const double lam = Sii + Sj[g.j] / C - 2.0 * QSI[g.j] - 1.0 / C + 1.0;
      gam = al * (QSI[a] - Sj[a] / C) +
            (isj ? al * (1.0 - C) / C + 0.5 * al * al * lam : 0.0);
    }
    *reinterpret_cast<double2*>(P + a * pld) = make_double2(isj ? g.xi0 : 0.0, gam);
  }
  if (maxabs) block_max_atomic(a < n ? fabs(gam) : 0.0, maxabs);
}

__global__ __launch_bounds__(kB) void c1_border_kernel(SView S, int64_t n_old, int32_t j,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ SI, IdList I,
                                                       double C, const double* sumI) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a < n_old && a != j) {
    const double v = y[a];
    s_put(S, (int64_t)j * S.ld + a, v);
    s_put(S, a * S.ld + j, v);
  }
  if (a == 0) {
    const double d = (double)I.count;
    const double SII = sumI ? *sumI : sum_at(SI, I);
    s_put(S, (int64_t)j * S.ld + j, C / (d * d) * SII + 1.0 - C);
  }
}

__global__ void set_diag_kernel(SView S, DiagList dl) {
  const int t = threadIdx.x;
  if (t < dl.count) s_put(S, (int64_t)dl.id[t] * S.ld + dl.id[t], dl.val[t]);
}

// Y[a][c] = scale * (1/d_a) sum_{x in in(a)} X[x][c] (+ add_diag at c == a). X and Y use the
// leading dimension ldi (a multiple of 64), rows and columns < n.
constexpr int kRowT = 128;  // threads of a row-gather workgroup (2 columns each)

__global__ __launch_bounds__(kRowT) void spmm_rows_kernel(DevQ q, int64_t n, int64_t ldi,
                                                       const double* __restrict__ X,
                                                       double* __restrict__ Y, double scale,
                                                       double add_diag,
                                                       const double* __restrict__ prev,
                                                       unsigned long long* maxdiff) {
  const int64_t a = blockIdx.x;
  const int64_t c = ((int64_t)blockIdx.y * kRowT + threadIdx.x) * 2;
  const int len = q.in.len[a];
  const int st = q.in.start[a];
  // In-neighbours are taken 8 at a time with their row loads issued together (one memory
  // latency per 8 neighbours). Columns past n read the padding of the leading dimension.
  constexpr int U = 8;
  double2 acc = make_double2(0.0, 0.0);
  const int64_t cc = c < ldi ? c : 0;
  for (int p0 = 0; p0 < len; p0 += U) {
    int64_t x[U];
    double w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u < len ? p0 + u : p0;
      x[u] = q.in.idx[st + p];
      w[u] = p0 + u < len ? (q.in.w ? q.in.w[st + p] : 1.0) : 0.0;
    }
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = *reinterpret_cast<const double2*>(X + x[u] * ldi + cc);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc.x += w[u] * v[u].x;
      acc.y += w[u] * v[u].y;
    }
  }
  double diff = 0.0;
  if (c < n) {
    double inv = 0.0;
    if (len > 0) inv = q.W ? 1.0 / q.W[a] : 1.0 / (double)len;
    double2 o = make_double2(scale * (acc.x * inv), scale * (acc.y * inv));
    if (c == a) o.x += add_diag;
    if (c + 1 == a) o.y += add_diag;
    if (c + 1 >= n) o.y = 0.0;
    store_stream(Y + a * ldi + c, o);
    if (prev) {
      const double2 pv = load_stream(prev + a * ldi + c);
      diff = fmax(fabs(o.x - pv.x), (c + 1 < n) ? fabs(o.y - pv.y) : 0.0);
    }
  }
  if (maxdiff) block_max_atomic(diff, maxdiff);
}

__global__ __launch_bounds__(1024) void transpose_kernel(int64_t n, int64_t ldi,
                                                         const double* __restrict__ X,
                                                         double* __restrict__ Y) {
  __shared__ double tile[32][33];
  const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  if (by + ty < n && bx + tx < n) tile[ty][tx] = X[(by + ty) * ldi + bx + tx];
  __syncthreads();
  if (bx + ty < n && by + tx < n) Y[(bx + ty) * ldi + by + tx] = tile[tx][ty];
}

__global__ __launch_bounds__(kB) void to_store_kernel(SView dst, int64_t n, int64_t ldi,
                                                      const double* __restrict__ src,
                                                      const double* __restrict__ srcT) {
  const int64_t a = blockIdx.x;
  const int64_t c = (int64_t)blockIdx.y * kB + threadIdx.x;
  if (c >= n) return;
  // with the transpose: (x + y) / 2 rounds the same for (a, c) and (c, a)
  const double v = srcT ? 0.5 * (src[a * ldi + c] + srcT[a * ldi + c]) : src[a * ldi + c];
  s_put(dst, a * dst.ld + c, v);
}

__global__ __launch_bounds__(kB) void from_store_kernel(SView src, int64_t n,
                                                        double* __restrict__ dst,
                                                        int64_t ld_dst) {
  const int64_t a = blockIdx.x;
  const int64_t c = (int64_t)blockIdx.y * kB + threadIdx.x;
  if (c < n) dst[a * ld_dst + c] = s_get(src, a * src.ld + c);
}

__global__ __launch_bounds__(kB) void copy_row_kernel(SView S, int64_t n, int32_t x,
                                                      double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a < n) out[a] = s_get(S, (int64_t)x * S.ld + a);
}

__global__ __launch_bounds__(kB) void gather_pairs_kernel(SView S, int64_t np,
                                                          const int32_t* __restrict__ pa,
                                                          const int32_t* __restrict__ pb,
                                                          double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (p < np) out[p] = s_get(S, (int64_t)pa[p] * S.ld + pb[p]);
}

__global__ __launch_bounds__(kB) void rows_to_f32_kernel(SView S, int64_t n,
                                                         const int32_t* __restrict__ rows,
                                                         float* __restrict__ out,
                                                         int64_t ld_out) {
  const int64_t t = blockIdx.x;
  const int64_t a = (int64_t)blockIdx.y * kB + threadIdx.x;
  if (a < n) out[t * ld_out + a] = (float)s_get(S, (int64_t)rows[t] * S.ld + a);
}

// x = indicator of the ids (sum of e_i); with xd, also xd[a] = x[a] / d[a] (0 where d[a] = 0)
__global__ __launch_bounds__(kB) void indicator_kernel(double* x, int64_t n, IdList ids, DevQ dq,
                                                       double* xd) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  double v = 0.0;
  for (int t = 0; t < ids.count; ++t) v = (ids.at(t) == a) ? 1.0 : v;
  x[a] = v;
  if (xd) {
    double r = 0.0;
    if (v != 0.0) {
      const double d = dq.W ? dq.W[a] : (double)dq.in.len[a];
      r = d > 0.0 ? v / d : 0.0;
    }
    xd[a] = r;
  }
}

__global__ __launch_bounds__(kB) void indicator2_kernel(double* x2, int64_t n, IdList ia,
                                                        IdList ib, DevQ dq, double* xd2) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  double u = 0.0, v = 0.0;
  for (int t = 0; t < ia.count; ++t) u = (ia.at(t) == a) ? 1.0 : u;
  for (int t = 0; t < ib.count; ++t) v = (ib.at(t) == a) ? 1.0 : v;
  *reinterpret_cast<double2*>(x2 + 2 * a) = make_double2(u, v);
  const double d = dq.W ? dq.W[a] : (double)dq.in.len[a];
  const double r = d > 0.0 ? 1.0 / d : 0.0;
  *reinterpret_cast<double2*>(xd2 + 2 * a) = make_double2(u * r, v * r);
}

// mm[0] = min and mm[1] = max over the np pairs' ids a[p], b[p] (mm preset by the launcher's
// first kernel to INT32_MAX, INT32_MIN).
__global__ void ids_range_init_kernel(int32_t* mm) {
  mm[0] = 2147483647;
  mm[1] = -2147483647 - 1;
}

__global__ __launch_bounds__(kB) void ids_range_kernel(const int32_t* __restrict__ a,
                                                       const int32_t* __restrict__ b, int64_t np,
                                                       int32_t* mm) {
  int lo = 2147483647, hi = -2147483647 - 1;
  for (int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x; p < np;
       p += (int64_t)gridDim.x * kB) {
    const int x = a[p], y = b[p];
    lo = min(lo, min(x, y));
    hi = max(hi, max(x, y));
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(mm, lo);
    atomicMax(mm + 1, hi);
  }
}

// Delta S columns of a node insertion without a low-rank part (column method, Algorithm 7 with
// Theorem 8 / Table 2 rows C1 and C3). Column x = rows[t] (or x when rows is null), nodes
// a < n:
//   kind 1 (C1, new sink j): y holds the new column of j (y[j] its diagonal), so
//          value = x == j ? y[a] : (a == j ? y[x] : 0)
//   kind 3 (C3, new nodes i and j): value = a == x ? (x == i ? vi : (x == j ? vj : 0)) : 0
// written as float32 (out32, row t at out32 + t ld) or float64 (out64).
__global__ __launch_bounds__(kB) void node_cols_kernel(const int32_t* __restrict__ rows,
                                                       int32_t x0, int64_t nrows, int64_t n,
                                                       int kind,
                                                       int32_t i, int32_t j,
                                                       const double* __restrict__ y, double vi,
                                                       double vj, float* out32, double* out64,
                                                       int64_t ld) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a >= n) return;
  for (int64_t t = blockIdx.y; t < nrows; t += gridDim.y) {
    const int32_t x = rows ? rows[t] : x0;
    double v = 0.0;
    if (kind == 1) {
      v = (x == j) ? y[a] : (a == j ? y[x] : 0.0);
    } else if (a == x) {
      v = x == i ? vi : (x == j ? vj : 0.0);
    }
    if (out32)
      out32[t * ld + a] = (float)v;
    else
      out64[t * ld + a] = v;
  }
}

// Case C2 after the panel product: the new source i is isolated apart from its out-edge, so
// its own column is vi e_i, which the panel (zero at row i) leaves out.
__global__ void node_fix_kernel(const int32_t* __restrict__ rows, int32_t x0, int32_t nrows,
                                int32_t i, double vi, float* out32, double* out64, int64_t ld) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const int32_t x = rows ? rows[t] : x0;
  if (x != i) return;
  if (out32)
    out32[(int64_t)t * ld + i] = (float)vi;
  else
    out64[(int64_t)t * ld + i] = vi;
}

// y[j] = C / delta^2 S_II + 1 - C: the new sink's diagonal (Theorem 8, Table 2 row C1).
__global__ void c1_corner_kernel(double* y, int32_t j, const double* __restrict__ SI, IdList I,
                                 double C, const double* sumI) {
  const double d = (double)I.count;
  y[j] = C / (d * d) * (sumI ? *sumI : sum_at(SI, I)) + 1.0 - C;
}

// Long id lists: after a zero fill, one thread per listed id sets its entry (the ids of a
// list are distinct). x has stride `stride` doubles per node and offset `half`; xd (optional)
// receives the entry divided by the node's row weight of Q (0 where that is 0).
__global__ __launch_bounds__(kB) void indicator_scatter_kernel(double* x, IdList ids, int stride,
                                                               int half, DevQ dq, double* xd) {
  const int t = blockIdx.x * kB + threadIdx.x;
  if (t >= ids.count) return;
  const int64_t a = ids.at(t);
  x[stride * a + half] = 1.0;
  if (xd) {
    const double d = dq.W ? dq.W[a] : (double)dq.in.len[a];
    xd[stride * a + half] = d > 0.0 ? 1.0 / d : 0.0;
  }
}

// S of a spanning forest (Example 1.2): row a of the tile, columns c0 + t, t < kTreeCols.
// Nodes at different depths score 0; at one depth H they climb to their lowest common
// ancestor (lambda steps) and score C^lambda (1 - C^(H - lambda + 1)), or 0 if they reach
// different roots. Every entry of the n x n block is written.
constexpr int kTreeT = 256;
constexpr int kTreeCols = 1024;

__global__ __launch_bounds__(kTreeT) void tree_init_kernel(SView S, int64_t n, int64_t ncb,
                                                           const int32_t* parent,
                                                           const int32_t* depth, double C) {
  const int64_t a = (int64_t)blockIdx.x / ncb;
  const int64_t c0 = ((int64_t)blockIdx.x % ncb) * kTreeCols;
  const int ha = depth[a];
  for (int t = threadIdx.x; t < kTreeCols; t += kTreeT) {
    const int64_t b = c0 + t;
    if (b >= n) break;
    double v = 0.0;
    if (depth[b] == ha) {
      // a and b are at one depth, so they reach their roots together: at most ha steps
      int32_t x = (int32_t)a, y = (int32_t)b;
      int lam = 0;
      bool meet = true;
      while (x != y) {
        const int32_t px = parent[x], py = parent[y];
        if (px < 0 || py < 0) {
          meet = false;
          break;
        }
        x = px;
        y = py;
        ++lam;
      }
      if (meet) {
        double cl = 1.0, ch = 1.0;
        for (int k = 0; k < lam; ++k) cl *= C;
        for (int k = 0; k < ha - lam + 1; ++k) ch *= C;
        v = cl * (1.0 - ch);
      }
    }
    s_put(S, a * S.ld + b, v);
  }
}

// Places a block's float64 S (nb x nb, leading dimension ldb) at the rows and columns of its
// nodes: S[gid[a]][gid[b]] = Sb[a][b].
__global__ __launch_bounds__(kB) void place_block_kernel(SView S, const int32_t* gid, int64_t nb,
                                                         const double* Sb, int64_t ldb) {
  const int64_t a = blockIdx.x;
  const int64_t row = (int64_t)gid[a] * S.ld;
  for (int64_t b = (int64_t)blockIdx.y * kB + threadIdx.x; b < nb; b += (int64_t)gridDim.y * kB)
    s_put(S, row + gid[b], Sb[a * ldb + b]);
}

__global__ __launch_bounds__(kB) void fill_diag_kernel(double* A, int64_t n, int64_t ld,
                                                       double v) {
  const int64_t a = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a < n) A[a * ld + a] = v;
}

__global__ __launch_bounds__(kB) void diag_range_kernel(SView S, int64_t lo, int64_t hi,
                                                        double v) {
  const int64_t a = lo + (int64_t)blockIdx.x * kB + threadIdx.x;
  if (a < hi) s_put(S, a * S.ld + a, v);
}

inline unsigned g1(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

}  // namespace

// A list held in device memory is written by a zero fill and a scatter (no thread loops over
// a long list).
static IdList empty_list() {
  IdList e;
  e.count = 0;
  e.dev = nullptr;
  return e;
}

hipError_t launch_indicator(double* x, int64_t n, const IdList& ids, hipStream_t s,
                            const DevQ* dq, double* xd) {
  if (n <= 0) return hipSuccess;
  const DevQ q = dq ? *dq : DevQ{};
  double* xo = dq ? xd : nullptr;
  indicator_kernel<<<g1(n), kB, 0, s>>>(x, n, ids.dev ? empty_list() : ids, q, xo);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && ids.dev && ids.count > 0) {
    indicator_scatter_kernel<<<g1(ids.count), kB, 0, s>>>(x, ids, 1, 0, q, xo);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_indicator2(double* x2, int64_t n, const IdList& a, const IdList& b,
                             hipStream_t s, const DevQ& dq, double* xd2) {
  if (n <= 0) return hipSuccess;
  indicator2_kernel<<<g1(n), kB, 0, s>>>(x2, n, a.dev ? empty_list() : a,
                                         b.dev ? empty_list() : b, dq, xd2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && a.dev && a.count > 0) {
    indicator_scatter_kernel<<<g1(a.count), kB, 0, s>>>(x2, a, 2, 0, dq, xd2);
    e = hipGetLastError();
  }
  if (e == hipSuccess && b.dev && b.count > 0) {
    indicator_scatter_kernel<<<g1(b.count), kB, 0, s>>>(x2, b, 2, 1, dq, xd2);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_ids_range(const int32_t* a, const int32_t* b, int64_t np, int32_t* mm,
                            hipStream_t s) {
  ids_range_init_kernel<<<1, 1, 0, s>>>(mm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || np <= 0) return e;
  const int64_t blocks = std::min<int64_t>((np + kB - 1) / kB, 1024);
  ids_range_kernel<<<(unsigned)blocks, kB, 0, s>>>(a, b, np, mm);
  return hipGetLastError();
}

hipError_t launch_node_cols(const int32_t* rows, int32_t x, int32_t nrows, int64_t n, int kind,
                            int32_t i, int32_t j, const double* y, double vi, double vj,
                            float* out32, double* out64, int64_t ld, hipStream_t s) {
  if (nrows <= 0 || n <= 0) return hipSuccess;
  if (kind == 2) {
    node_fix_kernel<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(rows, x, nrows, i, vi, out32,
                                                                    out64, ld);
  } else {
    const unsigned gy = (unsigned)std::min<int64_t>(nrows, 65535);
    node_cols_kernel<<<dim3(g1(n), gy), kB, 0, s>>>(rows, x, nrows, n, kind, i, j, y, vi, vj,
                                                    out32, out64, ld);
  }
  return hipGetLastError();
}

hipError_t launch_c1_corner(double* y, int32_t j, const double* SI, const IdList& I, double C,
                            hipStream_t s, const double* sumI) {
  c1_corner_kernel<<<1, 1, 0, s>>>(y, j, SI, I, C, sumI);
  return hipGetLastError();
}

hipError_t launch_sum_at(const double* v, const IdList& I, double* out, hipStream_t s) {
  sum_at_kernel<<<1, 64, 0, s>>>(v, I, out);
  return hipGetLastError();
}

hipError_t launch_tree_init(SView S, int64_t n, const int32_t* parent, const int32_t* depth,
                            double C, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t ncb = (n + kTreeCols - 1) / kTreeCols;
  const int64_t grid = n * ncb;
  if (grid >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  tree_init_kernel<<<(unsigned)grid, kTreeT, 0, s>>>(S, n, ncb, parent, depth, C);
  return hipGetLastError();
}

hipError_t launch_place_block(SView S, const int32_t* gid, int64_t nb, const double* Sb,
                              int64_t ldb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const unsigned gy = (unsigned)std::min<int64_t>((nb + kB - 1) / kB, 64);
  place_block_kernel<<<dim3((unsigned)nb, gy), kB, 0, s>>>(S, gid, nb, Sb, ldb);
  return hipGetLastError();
}

hipError_t launch_fill_diag(double* A, int64_t n, int64_t ld, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_diag_kernel<<<g1(n), kB, 0, s>>>(A, n, ld, v);
  return hipGetLastError();
}

hipError_t launch_diag_range(SView S, int64_t lo, int64_t hi, double v, hipStream_t s) {
  if (hi <= lo) return hipSuccess;
  diag_range_kernel<<<g1(hi - lo), kB, 0, s>>>(S, lo, hi, v);
  return hipGetLastError();
}

hipError_t launch_gather_rows(SView S, int64_t n, const IdList& I, int acc, int32_t j,
                              double* SI, double* Sj, uint32_t* suppI, uint32_t* suppJ,
                              hipStream_t s, const double* cI, const double* cJ) {
  gather_rows_kernel<<<g1(n), kB, 0, s>>>(S, n, I, acc, j, SI, Sj, suppI, suppJ, cI, cJ);
  return hipGetLastError();
}

hipError_t launch_gather_inrows(SView S, int64_t n, const DevQ& q, int32_t j, double* out,
                                hipStream_t s) {
  gather_inrows_kernel<<<g1(n), kB, 0, s>>>(S, n, q, j, out);
  return hipGetLastError();
}

hipError_t launch_direct_z(const GammaArgs& g, int64_t n, const double* SI, const double* zsum,
                           double* zbuf, hipStream_t s) {
  direct_z_kernel<<<g1(n), kB, 0, s>>>(g, n, SI, zsum, zbuf);
  return hipGetLastError();
}

hipError_t launch_gamma(const GammaArgs& g, int64_t n, const double* SI, const double* Sj,
                        const double* QSI, const double* zbuf, const double* Qz, double* P,
                        int pld, unsigned long long* maxabs, hipStream_t s) {
  gamma_kernel<<<g1(n), kB, 0, s>>>(g, n, SI, Sj, QSI, zbuf, Qz, P, pld, maxabs);
  return hipGetLastError();
}

hipError_t launch_c1_border(SView S, int64_t n_old, int32_t j, const double* y,
                            const double* SI, const IdList& I, double C, hipStream_t s,
                            const double* sumI) {
  c1_border_kernel<<<g1(n_old > 0 ? n_old : 1), kB, 0, s>>>(S, n_old, j, y, SI, I, C, sumI);
  return hipGetLastError();
}

hipError_t launch_set_diag(SView S, const DiagList& d, hipStream_t s) {
  if (d.count <= 0) return hipSuccess;
  set_diag_kernel<<<1, 64, 0, s>>>(S, d);
  return hipGetLastError();
}

static int64_t init_ld(int64_t n) { return (n + 63) / 64 * 64; }

hipError_t launch_spmm_rows(const DevQ& q, int64_t n, const double* X, double* Y, double scale,
                            double add_diag, const double* prev, unsigned long long* maxdiff,
                            hipStream_t s) {
  const int64_t ldi = init_ld(n);
  dim3 grid((unsigned)n, (unsigned)((n + 2 * kRowT - 1) / (2 * kRowT)));
  spmm_rows_kernel<<<grid, kRowT, 0, s>>>(q, n, ldi, X, Y, scale, add_diag, prev, maxdiff);
  return hipGetLastError();
}

hipError_t launch_transpose(int64_t n, const double* X, double* Y, hipStream_t s) {
  const int64_t ldi = init_ld(n);
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
  transpose_kernel<<<grid, dim3(32, 32), 0, s>>>(n, ldi, X, Y);
  return hipGetLastError();
}

hipError_t launch_to_store(SView dst, int64_t n, const double* src, hipStream_t s,
                           const double* srcT) {
  dim3 grid((unsigned)n, g1(n));
  to_store_kernel<<<grid, kB, 0, s>>>(dst, n, init_ld(n), src, srcT);
  return hipGetLastError();
}

hipError_t launch_from_store(SView src, int64_t n, double* dst, int64_t ld_dst, hipStream_t s) {
  dim3 grid((unsigned)n, g1(n));
  from_store_kernel<<<grid, kB, 0, s>>>(src, n, dst, ld_dst);
  return hipGetLastError();
}

hipError_t launch_copy_row(SView S, int64_t n, int32_t x, double* out, hipStream_t s) {
  copy_row_kernel<<<g1(n), kB, 0, s>>>(S, n, x, out);
  return hipGetLastError();
}

hipError_t launch_gather_pairs(SView S, int64_t np, const int32_t* a, const int32_t* b,
                               double* out, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  gather_pairs_kernel<<<g1(np), kB, 0, s>>>(S, np, a, b, out);
  return hipGetLastError();
}

hipError_t launch_rows_to_f32(SView S, int64_t n, const int32_t* rows, int32_t nrows,
                              float* out, int64_t ld_out, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  dim3 grid((unsigned)nrows, g1(n));
  rows_to_f32_kernel<<<grid, kB, 0, s>>>(S, n, rows, out, ld_out);
  return hipGetLastError();
}

}  // namespace sr
