// Device-side definitions shared by the kernels of libsimrank (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

// Storage kinds of the dense S (values of sr_config::s_prec).
enum { PREC_FP64 = 0, PREC_HILO = 1, PREC_FP32 = 2 };

// A view of the dense S: row-major with leading dimension ld.
//  FP64:  value = d[a*ld + b]
//  HILO:  value = (double)hl[a*ld + b].x + (double)hl[a*ld + b].y; .y holds the rounding
//         error of .x, so the pair carries about 48 significant bits. The two floats of an
//         entry are adjacent, so an update reads and writes one 8-byte stream.
//  FP32:  value = hi[a*ld + b]
struct SView {
  int prec;
  double* d;
  float2* hl;
  float* hi;
  int64_t ld;
};

__device__ __forceinline__ double s_get(const SView& s, int64_t off) {
  if (s.prec == PREC_FP64) return s.d[off];
  if (s.prec == PREC_HILO) {
    const float2 v = s.hl[off];
    return (double)v.x + (double)v.y;
  }
  return (double)s.hi[off];
}

// Stores the float64 value t: HILO splits it into the nearest float and the float nearest to
// the remainder.
__device__ __forceinline__ void s_put(const SView& s, int64_t off, double t) {
  if (s.prec == PREC_FP64) {
    s.d[off] = t;
  } else if (s.prec == PREC_HILO) {
    const float h = (float)t;
    s.hl[off] = make_float2(h, (float)(t - (double)h));
  } else {
    s.hi[off] = (float)t;
  }
}

// Slotted CSR on the device. Row r of a list occupies idx[start[r] .. start[r] + len[r]);
// rows keep spare slots so single-edge insertions patch in place.
struct DevAdj {
  const int32_t* start;
  const int32_t* len;
  const int32_t* idx;
  const double* w;  // per-slot weight, or null (unweighted)
};

// Q of the current graph: in-lists by sink. Q[a][x] = 1/len[a] (unweighted) or w/W[a].
struct DevQ {
  DevAdj in;
  const double* W;  // row weight sums (weighted), or null
};

// Streaming (non-temporal) access to dense rows that are touched once per launch, so that
// they do not displace gathered data from the caches.
typedef double stream_dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 load_stream(const double* p) {
  const stream_dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const stream_dbl2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void store_stream(double* p, double2 v) {
  const stream_dbl2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<stream_dbl2*>(p));
}

__device__ __forceinline__ double wave_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

__device__ __forceinline__ bool bit_get(const uint32_t* bm, int64_t v) {
  return (bm[v >> 5] >> (v & 31)) & 1u;
}

__device__ __forceinline__ void bit_set_atomic(uint32_t* bm, int64_t v) {
  atomicOr(bm + (v >> 5), 1u << (v & 31));
}

}  // namespace sr
