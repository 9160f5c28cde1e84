// Top-k single-source similarity search: for each query node x, the k nodes b with the
// largest S[x][b] (ties to the smaller id), optionally leaving x itself out. S is symmetric,
// so the row of x is its column and is read contiguously.
//
// One 1024-thread workgroup per query makes one pass over the row in id order, 1024 entries
// at a time. Entries above the current threshold are appended to an LDS buffer (wave ballots
// and a workgroup scan give their slots, in id order); when the next chunk might not fit, the
// buffer is sorted (bitonic, by value descending then id ascending), cut to k entries, and the
// threshold becomes the k-th value. A later entry equal to the threshold has a larger id than
// every kept one, so the strict comparison also keeps the tie rule. The row is read once.
// For k <= 1024 one wave per query does the same without workgroup barriers.
#include <type_traits>

#include "kernels.h"

namespace sr {

namespace {

constexpr int kT = 1024;
constexpr int kCap = 4096;  // candidate buffer; k <= kCap - kT = kTopkMax
constexpr int kG = 4;       // chunks whose values are loaded together

// Orders doubles as unsigned integers (larger value, larger key), negatives included; -0 is
// taken as +0 so that equal values tie.
__device__ __forceinline__ uint64_t order_key(double v) {
  v = v == 0.0 ? 0.0 : v;
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double key_value(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

// a before b: larger key first, then smaller id
__device__ __forceinline__ bool before(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

// Sorts the first kCap entries (the tail past `cnt` already padded to sort last).
__device__ void bitonic(uint64_t* key, int32_t* id) {
  for (int size = 2; size <= kCap; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int p = threadIdx.x; p < kCap / 2; p += kT) {
        const int lo = 2 * p - (p & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;  // this run sorts in "before" order
        const uint64_t ka = key[lo], kb = key[hi];
        const int32_t ia = id[lo], ib = id[hi];
        if (before(kb, ib, ka, ia) == up) {
          key[lo] = kb;
          key[hi] = ka;
          id[lo] = ib;
          id[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
}

// The row of one query in the store's layout (PREC_FP64 also serves a plain vector). The
// pointer is fixed before the loads, so no load sits under a branch (which would make each
// wait for the one before).
// load() returns the stored form, value() converts it, so that a group's loads can stay in
// flight until their values are used.
template <int PREC>
struct Row {
  using raw_t = typename std::conditional<
      PREC == PREC_FP64, double, typename std::conditional<PREC == PREC_HILO, float2,
                                                           float>::type>::type;
  const void* p;
  __device__ __forceinline__ raw_t load(int64_t b) const {
    return static_cast<const raw_t*>(p)[b];
  }
  static __device__ __forceinline__ double value(raw_t r) {
    if constexpr (PREC == PREC_FP64) {
      return r;
    } else if constexpr (PREC == PREC_HILO) {
      return (double)r.x + (double)r.y;
    } else {
      return (double)r;
    }
  }
  __device__ __forceinline__ double operator[](int64_t b) const { return value(load(b)); }
};

template <int PREC>
__device__ __forceinline__ Row<PREC> row_of(const SView& S, const double* vec, int64_t x) {
  if (vec) return Row<PREC>{vec};
  if constexpr (PREC == PREC_FP64) return Row<PREC>{S.d + x * S.ld};
  if constexpr (PREC == PREC_HILO) return Row<PREC>{S.hl + x * S.ld};
  return Row<PREC>{S.hi + x * S.ld};
}

template <int PREC>
__global__ __launch_bounds__(kT) void topk_kernel(SView S, const double* vecs, int64_t ldv,
                                                 const int32_t* q, int64_t n, int k,
                                                 int exclude_self, int32_t* out_idx,
                                                 double* out_val) {
  __shared__ uint64_t key[kCap];
  __shared__ int32_t id[kCap];
  __shared__ int wtot[kT / 64];
  __shared__ int cnt_s;
  __shared__ uint64_t thr_s;
  const int t = blockIdx.x;
  const int64_t x = q[t];
  const Row<PREC> row = row_of<PREC>(S, vecs ? vecs + (int64_t)t * ldv : nullptr, x);
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    cnt_s = 0;
    thr_s = 0;
  }
  __syncthreads();
  bool have_thr = false;
  auto sort_cut = [&](int cnt) {
    for (int p = cnt + threadIdx.x; p < kCap; p += kT) {
      key[p] = 0;
      id[p] = 0x7fffffff;
    }
    __syncthreads();
    bitonic(key, id);
  };
  // Values of kG chunks are loaded together, and the next kG chunks' loads are issued before
  // this group is processed, so a memory latency is paid about once per kG chunks.
  auto load_group = [&](int64_t base, double (&v)[kG]) {
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const int64_t b = base + (int64_t)u * kT + threadIdx.x;
      v[u] = row[b < n ? b : 0];
    }
  };
  double cur[kG], nxt[kG];
  load_group(0, nxt);
  for (int64_t gbase = 0; gbase < n; gbase += (int64_t)kG * kT) {
#pragma unroll
    for (int u = 0; u < kG; ++u) cur[u] = nxt[u];
    load_group(gbase + (int64_t)kG * kT, nxt);  // clamped: past the row it rereads entry 0
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const int64_t base = gbase + (int64_t)u * kT;
      if (base >= n) break;  // uniform across the workgroup
      const int64_t b = base + threadIdx.x;
      const bool valid = b < n && !(exclude_self && b == x);
      const uint64_t kv = valid ? order_key(cur[u]) : 0;
      const uint64_t thr = thr_s;
      const bool take = valid && (!have_thr || kv > thr);
      const uint64_t m = __ballot(take);
      const int pre = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wtot[wid] = __popcll(m);
      __syncthreads();
      int off = 0, tot = 0;
      for (int w = 0; w < kT / 64; ++w) {
        const int c = wtot[w];
        off += w < wid ? c : 0;
        tot += c;
      }
      const int cnt = cnt_s;
      if (take) {
        key[cnt + off + pre] = kv;
        id[cnt + off + pre] = (int32_t)b;
      }
      __syncthreads();
      const int ncnt = cnt + tot;
      if (ncnt > kCap - kT) {
        // the next chunk might not fit: keep the best k, raise the threshold to the k-th
        sort_cut(ncnt);
        if (threadIdx.x == 0) {
          cnt_s = k;
          thr_s = key[k - 1];
        }
        have_thr = true;
      } else if (threadIdx.x == 0) {
        cnt_s = ncnt;
      }
      __syncthreads();
    }
  }
  const int cnt = cnt_s;
  sort_cut(cnt);
  for (int r = threadIdx.x; r < k; r += kT) {
    const bool ok = r < cnt;
    out_idx[(int64_t)t * k + r] = ok ? id[r] : -1;
    out_val[(int64_t)t * k + r] = ok ? key_value(key[r]) : 0.0;
  }
}

// The same selection by one wave per query, for k <= kWaveK: no workgroup barriers, 8
// entries per lane per group of loads (512 per group, two groups in flight; 16 per lane took
// 35% longer at k = 100, with twice the registers and half the waves, and four groups in
// flight 0.81 ms against 0.58-0.68 ms per 4,096 queries at n = 52k: the loads in flight are
// not what bounds it). The buffer is
// cut back to k whenever it reaches about 2k entries, so it never holds more than
// 2 * kWaveK entries and each sort is small. Two buffer sizes: k <= 256 in 512 entries (6 KB
// of LDS, so registers rather than LDS bound the waves per CU) and k <= 1024 in 2,048.
constexpr int kWaveK = 1024;
constexpr int kWaveKSmall = 256;
constexpr int kWCap = 2 * kWaveK;
constexpr int kWU = 8;

// Sorts the first N entries (N a power of two, 64 <= N <= the buffer size). Each lane takes up to four
// pairs of a step at once: all their reads, then the compare-exchanges and writes (the pairs of
// one step are disjoint).
__device__ __noinline__ void bitonic_wave(uint64_t* key, int32_t* id, int N) {
  const int lane = threadIdx.x;
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int p0 = 0; p0 < N / 2; p0 += 256) {
        uint64_t ka[4], kb[4];
        int32_t ia[4], ib[4];
        int lo[4];
        bool act[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = p0 + j * 64 + lane;
          act[j] = p < N / 2;
          const int pc = act[j] ? p : 0;
          lo[j] = 2 * pc - (pc & (stride - 1));
          ka[j] = key[lo[j]];
          kb[j] = key[lo[j] + stride];
          ia[j] = id[lo[j]];
          ib[j] = id[lo[j] + stride];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool up = (lo[j] & size) == 0;
          if (act[j] && before(kb[j], ib[j], ka[j], ia[j]) == up) {
            key[lo[j]] = kb[j];
            key[lo[j] + stride] = ka[j];
            id[lo[j]] = ib[j];
            id[lo[j] + stride] = ia[j];
          }
        }
      }
      __syncthreads();  // one wave: orders the LDS accesses of consecutive steps
    }
  }
}

template <int PREC, int CAP>
__global__ __launch_bounds__(64) void topk_wave_kernel(SView S, const double* vecs, int64_t ldv,
                                                       const int32_t* q, int64_t n, int k,
                                                       int exclude_self, int32_t* out_idx,
                                                       double* out_val) {
  static_assert(CAP <= kWCap, "wave buffer");
  __shared__ uint64_t key[CAP];
  __shared__ int32_t id[CAP];
  const int t = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t x = q[t];
  const Row<PREC> row = row_of<PREC>(S, vecs ? vecs + (int64_t)t * ldv : nullptr, x);
  int cnt = 0;
  uint64_t thr = 0;
  bool have_thr = false;
  // sorts the cnt buffered entries (padded to a power of two, at least 64)
  auto sort_cut = [&]() {
    int N = 64;
    while (N < cnt) N <<= 1;
    for (int p = cnt + lane; p < N; p += 64) {
      key[p] = 0;
      id[p] = 0x7fffffff;
    }
    __syncthreads();
    bitonic_wave(key, id, N);
  };
  using raw_t = typename Row<PREC>::raw_t;
  auto load_group = [&](int64_t base, raw_t (&v)[kWU]) {
#pragma unroll
    for (int u = 0; u < kWU; ++u) {
      const int64_t b = base + (int64_t)u * 64 + lane;
      v[u] = row.load(b < n ? b : 0);
    }
  };
  // The buffer is cut back to k whenever it reaches cut_at (about twice k): each sort is
  // small, and the threshold rises early, so few later entries are appended at all.
  int kp = 64;
  while (kp < k) kp <<= 1;
  const int cut_at = 2 * kp - 64;
  auto process = [&](const raw_t (&v)[kWU], int64_t gbase) {
#pragma unroll
    for (int u = 0; u < kWU; ++u) {
      const int64_t b = gbase + (int64_t)u * 64 + lane;
      const bool valid = b < n && !(exclude_self && b == x);
      const uint64_t kv = valid ? order_key(Row<PREC>::value(v[u])) : 0;
      const bool take = valid && (!have_thr || kv > thr);
      const uint64_t m = __ballot(take);
      const int pos = cnt + __popcll(m & ((1ull << lane) - 1ull));
      if (take) {
        key[pos] = kv;
        id[pos] = (int32_t)b;
      }
      cnt += __popcll(m);
      if (cnt >= cut_at && cnt >= k) {
        __syncthreads();
        sort_cut();
        cnt = k;
        thr = key[k - 1];
        have_thr = true;
        __syncthreads();
      }
    }
  };
  // two groups in flight: while one is processed the other's loads are outstanding
  constexpr int64_t G = 64 * kWU;
  raw_t va[kWU], vb[kWU];
  load_group(0, va);
  load_group(G, vb);
  for (int64_t gbase = 0; gbase < n; gbase += 2 * G) {
    process(va, gbase);
    load_group(gbase + 2 * G, va);  // clamped: past the row it rereads entry 0
    if (gbase + G < n) process(vb, gbase + G);
    load_group(gbase + 3 * G, vb);
  }
  __syncthreads();
  sort_cut();
  for (int r = lane; r < k; r += 64) {
    const bool ok = r < cnt;
    out_idx[(int64_t)t * k + r] = ok ? id[r] : -1;
    out_val[(int64_t)t * k + r] = ok ? key_value(key[r]) : 0.0;
  }
}

}  // namespace

hipError_t launch_topk(const SView& S, const double* vecs, int64_t ldv, const int32_t* q,
                       int nq, int64_t n, int k, int exclude_self, int32_t* out_idx,
                       double* out_val, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  static_assert(kTopkMax == kCap - kT, "top-k bound");
  if (k < 1 || k > kTopkMax || n <= 0) return hipErrorInvalidValue;
  if (k <= kWaveK) {
    auto wave = [&](auto cap) {
      constexpr int CAP = decltype(cap)::value;
      if (vecs || S.prec == PREC_FP64)
        topk_wave_kernel<PREC_FP64, CAP><<<nq, 64, 0, s>>>(S, vecs, ldv, q, n, k, exclude_self,
                                                           out_idx, out_val);
      else if (S.prec == PREC_HILO)
        topk_wave_kernel<PREC_HILO, CAP><<<nq, 64, 0, s>>>(S, nullptr, 0, q, n, k,
                                                           exclude_self, out_idx, out_val);
      else
        topk_wave_kernel<PREC_FP32, CAP><<<nq, 64, 0, s>>>(S, nullptr, 0, q, n, k,
                                                           exclude_self, out_idx, out_val);
    };
    if (k <= kWaveKSmall)
      wave(std::integral_constant<int, 2 * kWaveKSmall>{});
    else
      wave(std::integral_constant<int, 2 * kWaveK>{});
    return hipGetLastError();
  }
  if (vecs) {
    topk_kernel<PREC_FP64><<<nq, kT, 0, s>>>(S, vecs, ldv, q, n, k, exclude_self, out_idx,
                                             out_val);
  } else if (S.prec == PREC_FP64) {
    topk_kernel<PREC_FP64><<<nq, kT, 0, s>>>(S, nullptr, 0, q, n, k, exclude_self, out_idx,
                                             out_val);
  } else if (S.prec == PREC_HILO) {
    topk_kernel<PREC_HILO><<<nq, kT, 0, s>>>(S, nullptr, 0, q, n, k, exclude_self, out_idx,
                                             out_val);
  } else {
    topk_kernel<PREC_FP32><<<nq, kT, 0, s>>>(S, nullptr, 0, q, n, k, exclude_self, out_idx,
                                             out_val);
  }
  return hipGetLastError();
}

}  // namespace sr
