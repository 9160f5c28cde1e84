// Sparse traversals of the graph: products with the backward transition matrix Q and its
// transpose, the series step of eq (16a) fused with the affected-area level of Theorem 4, and
// in-place patches of the slotted CSR.
//
// Q[a][x] = 1/indeg(a) for an edge x -> a (section 3.1). Rows are in-lists by sink, so
// (Q x)[a] gathers over a's in-neighbours and (Q^T x)[b] over b's out-neighbours.
//
// Power-law rows, four tiers, all in 512-thread workgroups of one launch: a row of at most
// kLight entries is handled by a group of 8 lanes, a medium row (at most kMedium entries,
// listed by the host) by one wave, a heavy row (up to the split threshold) by a whole
// workgroup, and a huge row is cut into chunks of kChunk entries, one workgroup each, whose
// partial sums a second small launch adds in chunk order. Workgroups are ordered longest work first (chunks,
// heavy, medium, light) so that the long rows do not trail the launch. Each lane takes its
// entries 8 or 16 at a time with all loads issued together, since the traversal is bound by
// memory latency; every sum is reduced in a fixed order, with no cross-workgroup combine
// inside a launch (whose device-scope fences write back the L2 of an XCD), so the results do
// not depend on scheduling.
#include "kernels.h"

namespace sr {

namespace {

constexpr int kB = 512;
constexpr int kG = 8;                   // lanes per light row
constexpr int kRowsPerBlock = kB / kG;  // 128
constexpr int kWaves = kB / 64;         // 16: medium rows per workgroup

__global__ __launch_bounds__(64) void patch_kernel(AdjPtrs t, Patch p) {
  int i = threadIdx.x;
  if (i < p.count) t.p[p.array[i]][p.index[i]] = p.value[i];
}

__global__ __launch_bounds__(64) void patch_w_kernel(WPtrs t, WPatch p) {
  int i = threadIdx.x;
  if (i < p.count) t.p[p.array[i]][p.index[i]] = p.value[i];
}

// What one traversal computes. Values per entry: NV = 1 (x) or 2 (xi, eta pair).
struct Op {
  int kind;             // 0: y = post*(base + scale*Q x); 1: series step; 2: y = scale*Q^T x;
                        // 3, 4: kinds 0 and 2 on two vectors at once (pairs of double)
  const double* x;      // kind 0/2 input vector (kind 2: divided by the row weight of Q)
  double* y;            // kind 0/2 output vector
  double* yd;           // kind 2: optional output divided by the row weight of Q
  double scale, post;
  const double* base;
  double* P;            // kind 1 panel
  int pld, k;           // kind 1: columns 2k, 2k+1 -> 2k+2, 2k+3
  const double* src;    // kind 1: the (xi_k, eta_k) pair of row x at src + x * sld
  int sld;
  double* cdst;         // kind 1: optional compact copy of the new pair (row a at 2 a)
  double sx, sy;
  // kinds 3 and 4: the input pairs are read through src / sld (sld = 2); y, yd and base hold
  // pairs (row a at 2 a); kind 3 writes the two halves to ya and yb instead when ya is set
  double* ya;
  double* yb;
  // optional bitmaps (pull form of Theorem 4): out bit b = OR_{x in row b} (in0 | in1)(x)
  const uint32_t* a0;
  const uint32_t* a1;
  uint32_t* aout;
  const uint32_t* b0;
  const uint32_t* b1;
  uint32_t* bout;
  int64_t nwords;       // bitmap words, ceil(n / 32)
};

// Bitmaps are staged in LDS when the (a0 | a1, b0 | b1) words of all nodes fit in this many
// bytes; a gather then reads LDS instead of four scattered global words.
constexpr int64_t kLdsBitmapBytes = 48 * 1024;

// Compile-time shape of one traversal: KIND (0: y = post (base + scale Q x); 1: series step;
// 2: y = scale Q^T x; 3, 4: kinds 0 and 2 on pairs), WT (weighted graph), AFF (0: no bitmaps; 1: bout only, from b0 | b1;
// 2: aout and bout), LDSB (bitmaps staged in LDS). Every instantiation is straight-line: no load sits under a branch, so
// no load waits for another that it does not depend on.
template <int KIND, bool WT, int AFF>
struct Shape {};

// Accumulates the entries [p0, p1) of the row starting at slot st of list L, lane `lane` of
// `step` lanes. Entries are taken U at a time: the U index loads, then the U dependent
// gathers (and bitmap words), are issued together; positions past p1 read entry p0 and are
// masked out. A lane thus waits for two memory latencies per U entries instead of two per
// entry. With PIPE (rows of several passes) the index loads of the next pass are issued
// right after the gathers of the current one, so a pass costs about one latency.
template <int U, int KIND, bool WT, int AFF, bool LDSB, bool PIPE = false>
__device__ __forceinline__ void accumulate(const Op& o, const DevQ& q, const DevAdj& L,
                                           const uint32_t* lbits, int64_t st, int p0, int p1,
                                           int lane, int step, double& v0, double& v1,
                                           uint32_t& fa, uint32_t& fb) {
  // entries base, base + step, ..: positions at or past p1 read entry p0 (p0 < p1 wherever
  // this runs)
  auto load_idx = [&](int base, int32_t (&xx)[U], double (&ww)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = base + u * step;
      const int64_t pc = st + (p < p1 ? p : p0);
      xx[u] = L.idx[pc];
      ww[u] = WT ? L.w[pc] : 1.0;
    }
  };
  int32_t xn[U];
  double wn[U];
  int base = p0 + lane;
  if (PIPE && base < p1) load_idx(base, xn, wn);
  for (; base < p1; base += U * step) {
    int32_t x[U];
    double w[U];
    bool ok[U];
    if constexpr (PIPE) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        x[u] = xn[u];
        w[u] = wn[u];
      }
    } else {
      load_idx(base, x, w);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) ok[u] = base + u * step < p1;
    // next pass's indices (clamped, so the loads are unconditional)
    if constexpr (PIPE) load_idx(base + U * step, xn, wn);
    if constexpr (KIND == 1 || KIND >= 3) {
      // a pair per node: both vectors of a gather share one cache line
      double2 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        v[u] = *reinterpret_cast<const double2*>(o.src + (int64_t)x[u] * o.sld);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v0 += ok[u] ? w[u] * v[u].x : 0.0;
        v1 += ok[u] ? w[u] * v[u].y : 0.0;
      }
    } else if constexpr (KIND == 0) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = o.x[x[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) v0 += ok[u] ? w[u] * v[u] : 0.0;
    } else {
      // (Q^T x)[b] = sum over out-neighbours a of Q[a][b] x[a], Q[a][b] = w / W_a or 1 / indeg(a);
      // the input holds x[a] / W_a (or x[a] / indeg(a)) already
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = o.x[x[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) v0 += ok[u] ? w[u] * v[u] : 0.0;
    }
    if constexpr (AFF == 2) {
      // staged words: lbits[2 w] = (a0 | a1)[w], lbits[2 w + 1] = (b0 | b1)[w]
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint32_t wa, wb;
        if constexpr (LDSB) {
          const uint2 ab = reinterpret_cast<const uint2*>(lbits)[x[u] >> 5];
          wa = ab.x;
          wb = ab.y;
        } else {
          wa = o.a0[x[u] >> 5] | o.a1[x[u] >> 5];
          wb = o.b0[x[u] >> 5] | o.b1[x[u] >> 5];
        }
        fa |= ok[u] ? (wa >> (x[u] & 31)) & 1u : 0u;
        fb |= ok[u] ? (wb >> (x[u] & 31)) & 1u : 0u;
      }
    } else if constexpr (AFF == 1) {
      // staged words: lbits[w] = (b0 | b1)[w]
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t wb = LDSB ? lbits[x[u] >> 5] : (o.b0[x[u] >> 5] | o.b1[x[u] >> 5]);
        fb |= ok[u] ? (wb >> (x[u] & 31)) & 1u : 0u;
      }
    }
  }
}

template <int KIND, bool WT>
__device__ __forceinline__ void finish(const Op& o, const DevQ& q, int64_t row, int len,
                                       double v0, double v1) {
  if constexpr (KIND == 1) {
    double2 out = make_double2(0.0, 0.0);
    if (len > 0) {
      const double inv = WT ? 1.0 / q.W[row] : 1.0 / (double)len;
      out.x = o.sx * (v0 * inv);
      out.y = o.sy * (v1 * inv);
    }
    *reinterpret_cast<double2*>(o.P + row * o.pld + 2 * (o.k + 1)) = out;
    if (o.cdst) *reinterpret_cast<double2*>(o.cdst + 2 * row) = out;
  } else if constexpr (KIND == 0) {
    double v = 0.0;
    if (len > 0) v = WT ? v0 / q.W[row] : v0 / (double)len;
    v *= o.scale;
    if (o.base) v += o.base[row];
    o.y[row] = o.post * v;
  } else if constexpr (KIND == 2) {
    const double v = o.scale * v0;
    o.y[row] = v;
    if (o.yd) {
      const double d = WT ? q.W[row] : (double)q.in.len[row];
      o.yd[row] = d > 0.0 ? v / d : 0.0;
    }
  } else if constexpr (KIND == 3) {
    double2 v = make_double2(0.0, 0.0);
    if (len > 0) {
      const double inv = WT ? 1.0 / q.W[row] : 1.0 / (double)len;
      v.x = v0 * inv;
      v.y = v1 * inv;
    }
    v.x *= o.scale;
    v.y *= o.scale;
    if (o.base) {
      const double2 b = *reinterpret_cast<const double2*>(o.base + 2 * row);
      v.x += b.x;
      v.y += b.y;
    }
    v.x *= o.post;
    v.y *= o.post;
    if (o.ya) {
      o.ya[row] = v.x;
      o.yb[row] = v.y;
    } else {
      *reinterpret_cast<double2*>(o.y + 2 * row) = v;
    }
  } else {
    const double2 v = make_double2(o.scale * v0, o.scale * v1);
    *reinterpret_cast<double2*>(o.y + 2 * row) = v;
    if (o.yd) {
      const double d = WT ? q.W[row] : (double)q.in.len[row];
      const double r = d > 0.0 ? 1.0 / d : 0.0;
      *reinterpret_cast<double2*>(o.yd + 2 * row) = make_double2(v.x * r, v.y * r);
    }
  }
}

// Sums of a whole workgroup in a fixed order (shuffles, then the wave sums in wave order);
// the result is valid in thread 0.
__device__ __forceinline__ void block_reduce(double& v0, double& v1, int& fw, double* red0,
                                             double* red1, int* redf) {
  const int lane64 = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  v0 = wave_sum(v0, 64);
  v1 = wave_sum(v1, 64);
  for (int sh = 32; sh > 0; sh >>= 1) fw |= __shfl_xor(fw, sh, 64);
  if (lane64 == 0) {
    red0[wid] = v0;
    red1[wid] = v1;
    redf[wid] = fw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    int ff = 0;
    for (int w = 0; w < kWaves; ++w) {
      s0 += red0[w];
      s1 += red1[w];
      ff |= redf[w];
    }
    v0 = s0;
    v1 = s1;
    fw = ff;
  }
}

// Workgroup roles by block index, longest work first: [0, nchunk) chunks of huge rows,
// then one workgroup per heavy row, then medium blocks (kWaves rows each), then light blocks
// (kRowsPerBlock consecutive rows each; rows of other tiers are skipped there).
//
// Affected-area bits: with LDSB every workgroup first copies the OR-ed source bitmaps of all
// nodes into LDS (coalesced), so a gather reads one LDS word (pair) instead of two (four)
// scattered global words. A light wave sets the bits of its 8 rows with one atomic per
// bitmap; medium, heavy and huge rows set theirs one atomic per row.
template <int KIND, bool WT, int AFF, bool LDSB>
__global__ __launch_bounds__(kB) void traverse_kernel(Op o, DevQ q, DevAdj L, int64_t n,
                                                      int64_t n_med_blocks, HeavyArgs h) {
  __shared__ double red0[kWaves], red1[kWaves];
  __shared__ int redf[kWaves];
  extern __shared__ uint32_t lbits[];
  int64_t bid = blockIdx.x;
  const int lane64 = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  double v0 = 0.0, v1 = 0.0;
  uint32_t fa = 0, fb = 0;
  if constexpr (LDSB && AFF > 0) {
    for (int64_t w = threadIdx.x; w < o.nwords; w += kB) {
      if constexpr (AFF == 2) {
        lbits[2 * w] = o.a0[w] | o.a1[w];
        lbits[2 * w + 1] = o.b0[w] | o.b1[w];
      } else {
        lbits[w] = o.b0[w] | o.b1[w];
      }
    }
    __syncthreads();
  }
  if (bid < h.nchunk) {
    // one chunk of a huge row: kChunk entries, 8 per thread, partial sums to the scratch
    const int2 c = h.chunk[bid];
    const int len = L.len[c.x];
    const int p1 = min(len, c.y + kChunk);
    accumulate<kChunk / kB, KIND, WT, AFF, LDSB>(o, q, L, lbits, L.start[c.x], c.y, p1,
                                                 threadIdx.x, kB, v0, v1, fa, fb);
    int fw = (fa ? 1 : 0) | (fb ? 2 : 0);
    block_reduce(v0, v1, fw, red0, red1, redf);
    if (threadIdx.x == 0) {
      h.part[bid] = make_double2(v0, v1);
      h.pflag[bid] = (uint32_t)fw;
    }
    return;
  }
  bid -= h.nchunk;
  if (bid < h.nheavy) {
    // heavy row (kMedium < len <= split threshold): the whole workgroup, 8 entries per thread
    // per pass
    const int64_t row = h.heavy[bid];
    const int len = L.len[row];
    if (len > 8 * kB)  // several passes: pipelined index loads
      accumulate<8, KIND, WT, AFF, LDSB, true>(o, q, L, lbits, L.start[row], 0, len,
                                               threadIdx.x, kB, v0, v1, fa, fb);
    else
      accumulate<8, KIND, WT, AFF, LDSB>(o, q, L, lbits, L.start[row], 0, len, threadIdx.x,
                                         kB, v0, v1, fa, fb);
    int fw = (fa ? 1 : 0) | (fb ? 2 : 0);
    block_reduce(v0, v1, fw, red0, red1, redf);
    if (threadIdx.x == 0) {
      finish<KIND, WT>(o, q, row, len, v0, v1);
      if (AFF == 2 && (fw & 1)) bit_set_atomic(o.aout, row);
      if (AFF >= 1 && (fw & 2)) bit_set_atomic(o.bout, row);
    }
    return;
  }
  bid -= h.nheavy;
  if (bid < n_med_blocks) {
    // medium rows (kLight < len <= kMedium): one wave per row, 16 entries per lane per pass
    // for Q x; 8 for the pair kinds, Q^T x, both bitmaps or weights: fewer registers let more
    // waves share a CU (the pair products at n = 1M ran 15% faster with 8 and 512-thread
    // workgroups than with 16 and 1024-thread ones)
    const int64_t mi = bid * kWaves + wid;
    if (mi >= h.nmed) return;
    const int64_t row = h.med[mi];
    const int len = L.len[row];
    constexpr int UM = (AFF == 2 || WT || KIND != 0) ? 8 : 16;
    if (len > UM * 64)  // several passes: pipelined index loads
      accumulate<UM, KIND, WT, AFF, LDSB, true>(o, q, L, lbits, L.start[row], 0, len, lane64,
                                                64, v0, v1, fa, fb);
    else
      accumulate<UM, KIND, WT, AFF, LDSB>(o, q, L, lbits, L.start[row], 0, len, lane64, 64,
                                          v0, v1, fa, fb);
    v0 = wave_sum(v0, 64);
    v1 = wave_sum(v1, 64);
    if constexpr (AFF > 0) {
      for (int s = 32; s > 0; s >>= 1) {
        fa |= (uint32_t)__shfl_xor((int)fa, s, 64);
        fb |= (uint32_t)__shfl_xor((int)fb, s, 64);
      }
    }
    if (lane64 == 0) {
      finish<KIND, WT>(o, q, row, len, v0, v1);
      if (AFF == 2 && fa) bit_set_atomic(o.aout, row);
      if (AFF >= 1 && fb) bit_set_atomic(o.bout, row);
    }
    return;
  }
  bid -= n_med_blocks;
  // light rows (<= kLight entries): 8 lanes per row, one pass of 8 entries per lane
  const int64_t row = bid * kRowsPerBlock + threadIdx.x / kG;
  const int lane = threadIdx.x % kG;
  int len = 0;
  bool mine = false;
  if (row < n) {
    len = L.len[row];
    mine = len <= kLight;
    if (mine)
      accumulate<kLight / kG, KIND, WT, AFF, LDSB>(o, q, L, lbits, L.start[row], 0, len, lane,
                                                   kG, v0, v1, fa, fb);
  }
  v0 = wave_sum(v0, kG);
  v1 = wave_sum(v1, kG);
  if constexpr (AFF > 0) {
    for (int s = kG >> 1; s > 0; s >>= 1) {
      fa |= (uint32_t)__shfl_xor((int)fa, s, kG);
      fb |= (uint32_t)__shfl_xor((int)fb, s, kG);
    }
  }
  if (mine && lane == 0) finish<KIND, WT>(o, q, row, len, v0, v1);
  if constexpr (AFF > 0) {
    // the wave's 8 rows start at a multiple of 8, so their bits share one word: gather the
    // group leaders' flags (lanes 0, 8, .., 56) and set them with one atomic per bitmap
    const uint64_t ma = __ballot(mine && lane == 0 && fa != 0);
    const uint64_t mb = __ballot(mine && lane == 0 && fb != 0);
    if (lane64 == 0) {
      uint32_t ba = 0, bb = 0;
#pragma unroll
      for (int g = 0; g < 64 / kG; ++g) {
        ba |= (uint32_t)((ma >> (kG * g)) & 1u) << g;
        bb |= (uint32_t)((mb >> (kG * g)) & 1u) << g;
      }
      const int64_t r0 = bid * kRowsPerBlock + wid * (64 / kG);
      if (AFF == 2 && ba) atomicOr(o.aout + (r0 >> 5), ba << (r0 & 31));
      if (bb) atomicOr(o.bout + (r0 >> 5), bb << (r0 & 31));
    }
  }
}

// Second launch for huge rows: one thread per row adds its chunks' partial sums in chunk
// order and finishes the row as the traversal does.
template <int KIND, bool WT, int AFF>
__global__ __launch_bounds__(64) void traverse_combine_kernel(Op o, DevQ q, DevAdj L,
                                                              HeavyArgs h) {
  const int hi = blockIdx.x * 64 + threadIdx.x;
  if (hi >= h.nhuge) return;
  double s0 = 0.0, s1 = 0.0;
  uint32_t ff = 0;
  for (int c = h.hfirst[hi]; c < h.hfirst[hi + 1]; ++c) {
    const double2 p = h.part[c];
    s0 += p.x;
    s1 += p.y;
    ff |= h.pflag[c];
  }
  const int64_t row = h.huge[hi];
  finish<KIND, WT>(o, q, row, L.len[row], s0, s1);
  if (AFF == 2 && (ff & 1)) bit_set_atomic(o.aout, row);
  if (AFF >= 1 && (ff & 2)) bit_set_atomic(o.bout, row);
}

template <int KIND, bool WT, int AFF>
hipError_t run_shape(const Op& o, const DevQ& q, const DevAdj& L, int64_t n,
                     const HeavyArgs& h, hipStream_t s) {
  const int64_t nlb = (n + kRowsPerBlock - 1) / kRowsPerBlock;
  const int64_t nmb = ((int64_t)h.nmed + kWaves - 1) / kWaves;
  const int64_t grid = (int64_t)h.nchunk + h.nheavy + nmb + nlb;
  const int64_t lds = AFF == 0 ? 0 : o.nwords * 4 * (AFF == 2 ? 2 : 1);
  if (AFF > 0 && lds <= kLdsBitmapBytes)
    traverse_kernel<KIND, WT, AFF, true><<<(unsigned)grid, kB, (size_t)lds, s>>>(o, q, L, n, nmb,
                                                                                  h);
  else
    traverse_kernel<KIND, WT, AFF, false><<<(unsigned)grid, kB, 0, s>>>(o, q, L, n, nmb, h);
  if (h.nhuge > 0)
    traverse_combine_kernel<KIND, WT, AFF><<<(unsigned)((h.nhuge + 63) / 64), 64, 0, s>>>(
        o, q, L, h);
  return hipGetLastError();
}

hipError_t run(const Op& o, const DevQ& q, const DevAdj& L, int64_t n, const HeavyArgs& h,
               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool wt = q.W != nullptr;
  // bitmaps: every set used is non-null (an absent second set is passed as the first)
  if (o.kind == 0) {
    if (o.bout)
      return wt ? run_shape<0, true, 1>(o, q, L, n, h, s) : run_shape<0, false, 1>(o, q, L, n, h, s);
    return wt ? run_shape<0, true, 0>(o, q, L, n, h, s) : run_shape<0, false, 0>(o, q, L, n, h, s);
  }
  if (o.kind == 1) {
    if (o.aout)
      return wt ? run_shape<1, true, 2>(o, q, L, n, h, s) : run_shape<1, false, 2>(o, q, L, n, h, s);
    return wt ? run_shape<1, true, 0>(o, q, L, n, h, s) : run_shape<1, false, 0>(o, q, L, n, h, s);
  }
  if (o.kind == 3)
    return wt ? run_shape<3, true, 0>(o, q, L, n, h, s) : run_shape<3, false, 0>(o, q, L, n, h, s);
  if (o.kind == 4)
    return wt ? run_shape<4, true, 0>(o, q, L, n, h, s) : run_shape<4, false, 0>(o, q, L, n, h, s);
  return wt ? run_shape<2, true, 0>(o, q, L, n, h, s) : run_shape<2, false, 0>(o, q, L, n, h, s);
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

hipError_t launch_patch_w(const WPtrs& t, const WPatch& p, hipStream_t s) {
  if (p.count <= 0) return hipSuccess;
  patch_w_kernel<<<1, 64, 0, s>>>(t, p);
  return hipGetLastError();
}

hipError_t launch_spmv_q(const DevQ& q, const HeavyArgs& h, int64_t n, const double* x,
                         double* y, double scale, hipStream_t s, const double* base,
                         double post, const uint32_t* fin, uint32_t* fout, int64_t nwords) {
  if (fout && nwords < (n + 31) / 32) return hipErrorInvalidValue;
  Op o = blank();
  o.kind = 0;
  o.x = x;
  o.y = y;
  o.scale = scale;
  o.base = base;
  o.post = post;
  o.b0 = fin;
  o.b1 = fin;
  o.bout = fout;
  o.nwords = nwords;
  return run(o, q, q.in, n, h, s);
}

hipError_t launch_spmv_qt(const DevQ& q, const DevAdj& out, const HeavyArgs& h, int64_t n,
                          const double* xd, double* y, double* yd, double scale,
                          hipStream_t s) {
  Op o = blank();
  o.kind = 2;
  o.x = xd;
  o.y = y;
  o.yd = yd;
  o.scale = scale;
  return run(o, q, out, n, h, s);
}

hipError_t launch_spmv_q2(const DevQ& q, const HeavyArgs& h, int64_t n, const double* x2,
                          double* y2, double scale, hipStream_t s, const double* base2,
                          double post, double* ya, double* yb) {
  if ((ya == nullptr) != (yb == nullptr) || (ya == nullptr && y2 == nullptr))
    return hipErrorInvalidValue;
  Op o = blank();
  o.kind = 3;
  o.src = x2;
  o.sld = 2;
  o.y = y2;
  o.ya = ya;
  o.yb = yb;
  o.scale = scale;
  o.base = base2;
  o.post = post;
  return run(o, q, q.in, n, h, s);
}

hipError_t launch_spmv_qt2(const DevQ& q, const DevAdj& out, const HeavyArgs& h, int64_t n,
                           const double* xd2, double* y2, double* yd2, double scale,
                           hipStream_t s) {
  Op o = blank();
  o.kind = 4;
  o.src = xd2;
  o.sld = 2;
  o.y = y2;
  o.yd = yd2;
  o.scale = scale;
  return run(o, q, out, n, h, s);
}

hipError_t launch_series_step_to(const DevQ& q, const HeavyArgs& h, int64_t n, double* wbase,
                                 int wld, const double* src, int sld, double* cdst, double sx,
                                 double sy, hipStream_t s) {
  Op o = blank();
  o.kind = 1;
  o.P = wbase;  // with k = -1 the new pair of row a goes to wbase + a * wld
  o.pld = wld;
  o.k = -1;
  o.src = src;
  o.sld = sld;
  o.cdst = cdst;
  o.sx = sx;
  o.sy = sy;
  return run(o, q, q.in, n, h, s);
}

hipError_t launch_series_step(const DevQ& q, const HeavyArgs& h, int64_t n, double* P, int pld,
                              int k, double sx, double sy, const AffLevel* aff, hipStream_t s,
                              double* pairs, int64_t pairs_cap) {
  Op o = blank();
  o.kind = 1;
  o.P = P;
  o.pld = pld;
  o.k = k;
  // The gathers of a step read the previous pair of every in-neighbour. From a compact
  // double-buffered copy (16 B per node, resident in L2) they are cheaper than from the panel
  // (256-byte rows); step 0 reads the panel's first pair.
  if (pairs && k > 0) {
    o.src = pairs + ((k - 1) % 2) * 2 * pairs_cap;
    o.sld = 2;
  } else {
    o.src = P + 2 * k;
    o.sld = pld;
  }
  o.cdst = pairs ? pairs + (k % 2) * 2 * pairs_cap : nullptr;
  o.sx = sx;
  o.sy = sy;
  if (aff) {
    if (aff->nwords < (n + 31) / 32) return hipErrorInvalidValue;
    o.nwords = aff->nwords;
    o.a0 = aff->a0;
    o.a1 = aff->a1 ? aff->a1 : aff->a0;
    o.aout = aff->aout;
    o.b0 = aff->b0;
    o.b1 = aff->b1 ? aff->b1 : aff->b0;
    o.bout = aff->bout;
  }
  return run(o, q, q.in, n, h, s);
}

}  // namespace sr
