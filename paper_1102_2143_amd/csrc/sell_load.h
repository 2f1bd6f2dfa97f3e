// Loads of the sliced ELLPACK layout (see Sell in msc_internal.h), shared by the
// single-system and the batched kernels.
#pragma once

#include <type_traits>

#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

// MSC_SELL_NT: stream the matrix with non-temporal loads (1) or ordinary loads (0; measured
// faster on MI355X at 16^4 and for the FP64 kernels at 32^3x64).
#ifndef MSC_SELL_NT
#define MSC_SELL_NT 0
#endif

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

template <class T> __device__ __forceinline__ T stream_load(const T* p) {
  if (MSC_SELL_NT) return __builtin_nontemporal_load(p);
  return *p;
}

// Entries 2q and 2q+1 of one lane (pair index q counts kSlice pairs per slice column).
__device__ __forceinline__ void load_pair(const float2* __restrict__ v, int64_t q, float2& e0,
                                          float2& e1) {
  const f32x4 w = stream_load(reinterpret_cast<const f32x4*>(v) + q);
  e0 = float2{w.x, w.y};
  e1 = float2{w.z, w.w};
}
__device__ __forceinline__ void load_pair(const double2* __restrict__ v, int64_t q, double2& e0,
                                          double2& e1) {
  const f64x2 a = stream_load(reinterpret_cast<const f64x2*>(v) + 2 * q);
  const f64x2 b = stream_load(reinterpret_cast<const f64x2*>(v) + 2 * q + 1);
  e0 = double2{a.x, a.y};
  e1 = double2{b.x, b.y};
}
__device__ __forceinline__ int2 load_cols(const int32_t* __restrict__ col, int64_t q) {
  const i32x2 c = stream_load(reinterpret_cast<const i32x2*>(col) + q);
  return int2{c.x, c.y};
}

// Slice offsets and column bases are read through the scalar cache: the address is
// wavefront-uniform and the arrays are never written while a solve runs.
__device__ __forceinline__ int32_t load_uniform(const int32_t* p, int64_t i) {
  using cptr_t = const __attribute__((address_space(4))) int32_t*;
  return ((cptr_t)p)[i];
}

// Columns of pair q = c kSlice + lane (c wavefront-uniform): 32-bit, or (NARROW) the two
// 16-bit offsets added to the pair column's bases.
template <bool NARROW, class V>
__device__ __forceinline__ int2 sell_cols(const Sell<V>& m, int32_t c, int64_t q) {
  if (NARROW) {
    const uint32_t w = stream_load(m.col16 + q);
    return int2{load_uniform(m.cbase, 2 * int64_t(c)) + int32_t(w & 0xffffu),
                load_uniform(m.cbase, 2 * int64_t(c) + 1) + int32_t(w >> 16)};
  }
  return load_cols(m.col, q);
}

// Column and value loads of KP pairs starting at pair column c (np < KP: only the first
// np pairs exist; the rest read as zero).
template <class R, int KP, bool FULL, bool NARROW>
__device__ __forceinline__ void sell_load(const Sell<cplx<R>>& m, int32_t c, int np, int lane,
                                          int2 (&cc)[KP], cplx<R> (&v)[2 * KP]) {
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    if (FULL || u < np) {
      const int64_t q = int64_t(c + u) * kSlice + lane;
      cc[u] = sell_cols<NARROW>(m, c + u, q);
      load_pair(m.val, q, v[2 * u], v[2 * u + 1]);
    } else {
      cc[u] = int2{0, 0};
      v[2 * u] = v[2 * u + 1] = czero<R>();
    }
  }
}

// ---- several right-hand sides interleaved, v[i RR + q] ----------------------------------

// The RR interleaved values of column c, loaded 16 bytes at a time.
template <class R, int RR>
__device__ __forceinline__ void load_rhs(const cplx<R>* __restrict__ x, int64_t c, cplx<R> (&o)[RR]) {
  if constexpr (std::is_same<R, float>::value && RR % 2 == 0) {
    const f32x4* v = reinterpret_cast<const f32x4*>(x + c * RR);
#pragma unroll
    for (int h = 0; h < RR / 2; ++h) {
      const f32x4 w = v[h];
      o[2 * h] = float2{w.x, w.y};
      o[2 * h + 1] = float2{w.z, w.w};
    }
  } else {
#pragma unroll
    for (int q = 0; q < RR; ++q) o[q] = x[c * RR + q];
  }
}

template <class R, int RR, int KP, bool FULL>
__device__ __forceinline__ void gather_rhs_fma(const cplx<R>* __restrict__ x, int np,
                                               const int2 (&cc)[KP], const cplx<R> (&v)[2 * KP],
                                               cplx<R> (&acc)[RR]) {
  cplx<R> xs[2 * KP][RR];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    if (FULL || u < np) {
      load_rhs<R, RR>(x, cc[u].x, xs[2 * u]);
      load_rhs<R, RR>(x, cc[u].y, xs[2 * u + 1]);
    } else {
#pragma unroll
      for (int q = 0; q < RR; ++q) xs[2 * u][q] = xs[2 * u + 1][q] = czero<R>();
    }
  }
#pragma unroll
  for (int u = 0; u < 2 * KP; ++u) {
#pragma unroll
    for (int q = 0; q < RR; ++q) cfma<R>(acc[q], v[u], xs[u][q]);
  }
}

// Off-diagonal part of one sliced ELLPACK row per lane times the RR interleaved vectors
// of x (slice `sl` wavefront-uniform); one read of the matrix row serves every rhs.
template <class R, int RR, int KP, bool NARROW>
__device__ __forceinline__ void sell_row_rhs_cols(const Sell<cplx<R>>& m,
                                                  const cplx<R>* __restrict__ x, int64_t sl,
                                                  int lane, cplx<R> (&acc)[RR]) {
#pragma unroll
  for (int q = 0; q < RR; ++q) acc[q] = czero<R>();
  int32_t c, c1;
  if (m.wp > 0) {
    c = int32_t(sl) * m.wp;
    c1 = c + m.wp;
  } else {
    c = load_uniform(m.cptr, sl);
    c1 = load_uniform(m.cptr, sl + 1);
  }
  int2 cc[KP];
  cplx<R> v[2 * KP];
  for (; c + KP <= c1; c += KP) {
    sell_load<R, KP, true, NARROW>(m, c, KP, lane, cc, v);
    gather_rhs_fma<R, RR, KP, true>(x, KP, cc, v, acc);
  }
  if (c < c1) {
    const int np = c1 - c;
    sell_load<R, KP, false, NARROW>(m, c, np, lane, cc, v);
    gather_rhs_fma<R, RR, KP, false>(x, np, cc, v, acc);
  }
}
template <class R, int RR, int KP>
__device__ __forceinline__ void sell_row_rhs(const Sell<cplx<R>>& m, const cplx<R>* __restrict__ x,
                                             int64_t sl, int lane, cplx<R> (&acc)[RR]) {
  if (m.col16)
    sell_row_rhs_cols<R, RR, KP, true>(m, x, sl, lane, acc);
  else
    sell_row_rhs_cols<R, RR, KP, false>(m, x, sl, lane, acc);
}

// ---- several separate vectors: x_q = xs[q], q < kc <= KC --------------------------------

template <class R, int KC, int KP, bool NARROW>
__device__ __forceinline__ void sell_row_multi_cols(const Sell<cplx<R>>& m,
                                                    const cplx<R>* const (&xs)[KC], int kc,
                                                    int64_t sl, int lane, cplx<R> (&acc)[KC]) {
  int32_t c, c1;
  if (m.wp > 0) {
    c = int32_t(sl) * m.wp;
    c1 = c + m.wp;
  } else {
    c = load_uniform(m.cptr, sl);
    c1 = load_uniform(m.cptr, sl + 1);
  }
  int2 cc[KP];
  cplx<R> v[2 * KP];
  for (; c < c1; c += KP) {
    const int np = c1 - c;
    sell_load<R, KP, false, NARROW>(m, c, np, lane, cc, v);
    cplx<R> g[2 * KP][KC];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        if (u < np && q < kc) {
          g[2 * u][q] = xs[q][cc[u].x];
          g[2 * u + 1][q] = xs[q][cc[u].y];
        } else {
          g[2 * u][q] = g[2 * u + 1][q] = czero<R>();
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2 * KP; ++u) {
#pragma unroll
      for (int q = 0; q < KC; ++q) cfma<R>(acc[q], v[u], g[u][q]);
    }
  }
}

// Off-diagonal part of one sliced ELLPACK row per lane times each of kc separate vectors
// (slice `sl` wavefront-uniform; vectors q >= kc give zero).
template <class R, int KC, int KP>
__device__ __forceinline__ void sell_row_multi(const Sell<cplx<R>>& m,
                                               const cplx<R>* const (&xs)[KC], int kc,
                                               int64_t sl, int lane, cplx<R> (&acc)[KC]) {
#pragma unroll
  for (int q = 0; q < KC; ++q) acc[q] = czero<R>();
  if (m.col16)
    sell_row_multi_cols<R, KC, KP, true>(m, xs, kc, sl, lane, acc);
  else
    sell_row_multi_cols<R, KC, KP, false>(m, xs, kc, sl, lane, acc);
}

}  // namespace msc
