// Multishift CG for a real symmetric positive-definite A (the paper's own benchmark
// matrix, the 2-D 5-point Poisson operator of Section 4 / Table 1, is real): the same
// shifted recurrences as the complex solve (Section 2, Algorithm 1 with the re-derived
// constants), on real vectors and a real copy of the sliced ELLPACK matrix, so every
// matrix value and vector element moves half the bytes of the complex path.  T = double
// (FP64) or float (single-precision storage and arithmetic with FP64 reductions and FP64
// shift scalars, the paper's "single" column).
//
// One iteration is three kernels; each reduction is finished by the last workgroup to
// arrive, which also derives the scalars:
//   RK1  t = A p (sliced ELLPACK, one row per lane), P = p.t + sigma0 p.p
//        -> a = R / P; per shift zeta', a_k
//   RK2  r <- r - a (t + sigma0 p), R' = r.r
//        -> b' = R'/R, b_k = b' (zeta'/zeta)^2, freezing, halting
//   RK3  x_0 += a p; x_k += a_k p_k, p_k <- zeta'_k r + b_k p_k (live shifts); p <- r + b' p
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

namespace {

template <class T> __device__ __forceinline__ SellReal<T> rmat(const RealArgs& a);
template <> __device__ __forceinline__ SellReal<double> rmat<double>(const RealArgs& a) { return a.m64; }
template <> __device__ __forceinline__ SellReal<float> rmat<float>(const RealArgs& a) { return a.m32; }

__device__ __forceinline__ int32_t ld_uniform(const int32_t* p, int64_t i) {
  using cptr_t = const __attribute__((address_space(4))) int32_t*;
  return ((cptr_t)p)[i];
}

// Columns of pair q = c kSlice + lane of pair column c (32-bit or narrow 16-bit offsets).
template <class T>
__device__ __forceinline__ int2 r_cols(const SellReal<T>& m, int32_t c, int64_t q) {
  if (m.col16) {
    const uint32_t w = m.col16[q];
    return int2{ld_uniform(m.cbase, 2 * int64_t(c)) + int32_t(w & 0xffffu),
                ld_uniform(m.cbase, 2 * int64_t(c) + 1) + int32_t(w >> 16)};
  }
  return int2{m.col[2 * q], m.col[2 * q + 1]};
}

// One sliced ELLPACK row per lane times x (off-diagonal part plus the diagonal); four
// pairs per round trip, all their loads issued before the first multiply-add.
template <class T>
__device__ __forceinline__ T r_row(const SellReal<T>& m, const T* __restrict__ x, int64_t sl,
                                   int lane, int64_t row) {
  int32_t c, c1;
  if (m.wp > 0) {
    c = int32_t(sl) * m.wp;
    c1 = c + m.wp;
  } else {
    c = ld_uniform(m.cptr, sl);
    c1 = ld_uniform(m.cptr, sl + 1);
  }
  T acc = m.diag[row] * x[row];
  constexpr int KP = 4;
  for (; c < c1; c += KP) {
    int2 cc[KP];
    T v0[KP], v1[KP], g0[KP], g1[KP];
#pragma unroll
    for (int u = 0; u < KP; ++u) {
      if (c + u < c1) {
        const int64_t q = int64_t(c + u) * kSlice + lane;
        cc[u] = r_cols(m, c + u, q);
        v0[u] = m.val[2 * q];
        v1[u] = m.val[2 * q + 1];
      } else {
        cc[u] = int2{int32_t(row), int32_t(row)};
        v0[u] = v1[u] = T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < KP; ++u) {
      g0[u] = x[cc[u].x];
      g1[u] = x[cc[u].y];
    }
#pragma unroll
    for (int u = 0; u < KP; ++u) acc = fma(v1[u], g1[u], fma(v0[u], g0[u], acc));
  }
  return acc;
}

__device__ double r_sum(const double* partial, int count, int stride, int k) {
  constexpr int kPer = kMaxGrid / kBlock;
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kBlock;
    v[u] = i < count ? load_agent(&partial[i * stride + k]) : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) s += v[u];
  return block_sum<kBlock>(s);
}

// Store this workgroup's partial; true in the last workgroup, with the grid sum in *tot.
__device__ bool r_reduce(const RealArgs& a, double v, double* tot) {
  const double bs = block_sum<kBlock>(v);
  if (threadIdx.x == 0) store_agent(&a.partial[blockIdx.x], bs);
  if (!arrive_last(a.tickets)) return false;
  __shared__ double sh;
  const double t = r_sum(a.partial, gridDim.x, 1, 0);
  if (threadIdx.x == 0) sh = t;
  __syncthreads();
  *tot = sh;
  return true;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_r_init(RealArgs a) {
  RealState* st = a.st;
  T* __restrict__ r = static_cast<T*>(a.r);
  T* __restrict__ p = static_cast<T*>(a.p);
  T* __restrict__ pk = static_cast<T*>(a.pk);
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double bv = a.b[i];
    const T bt = T(bv);
    r[i] = bt;
    p[i] = bt;
    for (int j = 1; j < a.ns; ++j) pk[int64_t(j - 1) * a.n + i] = bt;
    for (int j = 0; j < a.ns; ++j) a.x[int64_t(st->orig[j]) * a.n + i] = 0.0;
    acc = fma(bv, bv, acc);
  }
  double tot;
  if (!r_reduce(a, acc, &tot)) return;
  if (threadIdx.x == 0) {
    st->bnorm2 = tot;
    st->R = tot;
    st->eps2 = st->eps2 * tot;  // the host stored tol^2
    if (!(tot > 0.0) || !isfinite(tot)) {
      st->halt = 1;
      st->status = isfinite(tot) ? 0 : 1;
    }
  }
}

// ---- RK1: t = A p, P = p.t + sigma0 p.p; a, zeta', a_k --------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void k_r_k1(RealArgs a) {
  RealState* st = a.st;
  if (st->halt) return;
  const SellReal<T> m = rmat<T>(a);
  const T* __restrict__ p = static_cast<const T*>(a.p);
  T* __restrict__ t = static_cast<T*>(a.t);
  const double sigma0 = st->sigma0;
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  int64_t beg, end;
  block_range(a.nslices, SPB, beg, end);
  double acc = 0.0;
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < a.n ? row : a.n - 1;
    const T v = r_row<T>(m, p, sl, lane, rr);
    if (row < a.n) {
      t[row] = v;
      const double pr = double(p[row]);
      acc += pr * double(v) + sigma0 * pr * pr;
    }
  }
  double P;
  if (!r_reduce(a, acc, &P)) return;
  const int j = threadIdx.x;
  // rotate the previous iteration's shift state, then this iteration's constants
  if (j < a.ns && st->rotate) {
    if (st->active[j]) {
      st->zeta_prev[j] = st->zeta[j];
      st->zeta[j] = st->zeta_new[j];
    }
    st->active[j] = st->active_next[j];
  }
  __syncthreads();
  const bool ok = P > 0.0 && isfinite(P);
  const double step = ok ? st->R / P : 0.0;
  if (ok && j < a.ns && j >= 1 && st->active[j]) {
    const double z = st->zeta[j], zp = st->zeta_prev[j], sj = st->s[j];
    const double ap = st->a_prev, b = st->b;
    const double zn = z * zp * ap / (step * b * (zp - z) + zp * ap * (1.0 + sj * step));
    st->zeta_new[j] = zn;
    st->ak[j] = step * zn / z;
  }
  if (j == 0) {
    st->rotate = 0;
    if (!ok) {
      st->halt = 1;
      st->status = 1;
    } else {
      st->a = step;
      st->P = P;
    }
  }
}

// ---- RK2: r <- r - a (t + sigma0 p), R' = r.r; b', b_k, freezing, halting -------------
template <class T>
__global__ __launch_bounds__(kBlock) void k_r_k2(RealArgs a, int launch) {
  RealState* st = a.st;
  if (st->halt) return;
  T* __restrict__ r = static_cast<T*>(a.r);
  const T* __restrict__ p = static_cast<const T*>(a.p);
  const T* __restrict__ t = static_cast<const T*>(a.t);
  const double step = st->a, sigma0 = st->sigma0;
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double nr = double(r[i]) - step * (double(t[i]) + sigma0 * double(p[i]));
    const T st_r = T(nr);
    r[i] = st_r;
    acc += double(st_r) * double(st_r);
  }
  double Rn;
  if (!r_reduce(a, acc, &Rn)) return;
  const int j = threadIdx.x;
  const double bn = Rn / st->R;
  if (j < a.ns) {
    int nxt = st->active[j];
    if (j >= 1 && nxt) {
      const double ratio = st->zeta_new[j] / st->zeta[j];
      st->bk[j] = bn * ratio * ratio;
      if (st->freeze && st->zeta_new[j] * st->zeta_new[j] * Rn <= st->eps2) {
        nxt = 0;
        st->freeze_iter[j] = st->iter + 1;
      }
    }
    st->active_next[j] = nxt;
  }
  __syncthreads();
  if (j == 0) {
    st->b_new = bn;
    st->a_prev = step;
    st->b = bn;
    st->R = Rn;
    st->iter += 1;
    st->rotate = 1;
    st->upd_launch = launch;
    if (!isfinite(Rn)) {
      st->halt = 1;
      st->status = 1;
    } else if (Rn <= st->eps2 || st->iter >= st->max_iter) {
      st->halt = 1;
    }
  }
}

// ---- RK3: the step of x_0, of every live shift, and the new direction -----------------
template <class T>
__global__ __launch_bounds__(kBlock) void k_r_k3(RealArgs a, int launch) {
  RealState* st = a.st;
  if (st->upd_launch != launch) return;
  __shared__ double ak[kMaxShifts], zn[kMaxShifts], bk[kMaxShifts];
  __shared__ int64_t xo[kMaxShifts], po[kMaxShifts];
  __shared__ int nlive;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int j = 1; j < a.ns; ++j) {
      if (st->active[j]) {
        ak[c] = st->ak[j];
        zn[c] = st->zeta_new[j];
        bk[c] = st->active_next[j] ? st->bk[j] : 0.0;
        xo[c] = int64_t(st->orig[j]) * a.n;
        po[c] = int64_t(j - 1) * a.n;
        ++c;
      }
    }
    nlive = c;
  }
  __syncthreads();
  const double step = st->a, bn = st->b_new;
  const int live = nlive;
  T* __restrict__ p = static_cast<T*>(a.p);
  T* __restrict__ pk = static_cast<T*>(a.pk);
  const T* __restrict__ r = static_cast<const T*>(a.r);
  double* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double rv = double(r[i]), pv = double(p[i]);
    x0[i] = fma(step, pv, x0[i]);
    for (int c = 0; c < live; ++c) {
      const double pj = double(pk[po[c] + i]);
      a.x[xo[c] + i] = fma(ak[c], pj, a.x[xo[c] + i]);
      pk[po[c] + i] = T(fma(zn[c], rv, bk[c] * pj));
    }
    p[i] = T(fma(bn, pv, rv));
  }
}

// ---- FP64 true residual |b - (A + sigma) x|^2 of one shift ---------------------------
__global__ __launch_bounds__(kBlock) void k_r_verify(RealArgs a, const double* __restrict__ x,
                                                     double sigma, double* out) {
  const SellReal<double> m = rmat<double>(a);
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  int64_t beg, end;
  block_range(a.nslices, SPB, beg, end);
  double acc = 0.0;
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < a.n ? row : a.n - 1;
    const double v = r_row<double>(m, x, sl, lane, rr);
    if (row < a.n) {
      const double d = a.b[row] - v - sigma * x[row];
      acc = fma(d, d, acc);
    }
  }
  double tot;
  if (!r_reduce(a, acc, &tot)) return;
  if (threadIdx.x == 0) *out = tot;
}

// Real parts of the complex sliced copy (values and diagonal) and the largest imaginary
// part seen (atomic max on its bits: non-negative doubles order like their bit patterns).
__global__ void k_r_extract(const double2* __restrict__ v64, double* __restrict__ r64,
                            float* __restrict__ r32, int64_t count,
                            unsigned long long* __restrict__ imax) {
  unsigned long long local = 0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double2 v = v64[i];
    r64[i] = v.x;
    r32[i] = float(v.x);
    const double ai = fabs(v.y);
    const unsigned long long bits = __double_as_longlong(ai);
    local = bits > local ? bits : local;
  }
  if (local) atomicMax(imax, local);
}

int r_grid(int64_t n, int rows_per_pass) {
  int64_t g = (n + rows_per_pass - 1) / rows_per_pass;
  if (g > kMaxGrid) g = kMaxGrid;
  if (g < kXcds) g = kXcds;
  g = (g + kXcds - 1) / kXcds * kXcds;
  if (g > kMaxGrid) g = kMaxGrid;
  return int(g);
}

}  // namespace

hipError_t launch_real_extract(const double2* v64, double* r64, float* r32, int64_t count,
                               unsigned long long* imax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  k_r_extract<<<unsigned(g), 256, 0, s>>>(v64, r64, r32, count, imax);
  return hipGetLastError();
}

hipError_t launch_real_init(int prec, const RealArgs& a, hipStream_t s) {
  const int g = r_grid(a.n, kBlock);
  if (prec == MSC_PREC_MIXED)
    k_r_init<float><<<g, kBlock, 0, s>>>(a);
  else
    k_r_init<double><<<g, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_real_iteration(int prec, const RealArgs& a, int launch, hipStream_t s) {
  const int gs = r_grid(a.nslices, kBlock / kSlice);
  const int g3 = r_grid(a.n, kBlock);
  if (prec == MSC_PREC_MIXED) {
    k_r_k1<float><<<gs, kBlock, 0, s>>>(a);
    k_r_k2<float><<<g3, kBlock, 0, s>>>(a, launch);
    k_r_k3<float><<<g3, kBlock, 0, s>>>(a, launch);
  } else {
    k_r_k1<double><<<gs, kBlock, 0, s>>>(a);
    k_r_k2<double><<<g3, kBlock, 0, s>>>(a, launch);
    k_r_k3<double><<<g3, kBlock, 0, s>>>(a, launch);
  }
  return hipGetLastError();
}

hipError_t launch_real_verify(const RealArgs& a, const double* x, double sigma, double* out,
                              hipStream_t s) {
  const int gs = r_grid(a.nslices, kBlock / kSlice);
  k_r_verify<<<gs, kBlock, 0, s>>>(a, x, sigma, out);
  return hipGetLastError();
}

}  // namespace msc
