// Batched single-shift CG: m <= 16 systems (A + sigma_j) e_j = f_j that share one
// operator, advanced together so every iteration reads the matrix once for all of them.
//
// Used for the per-shift refinement after a mixed-precision multishift sequence (each
// shift's FP64 true residual becomes the right-hand side of a correction solve) and for
// adjoint solves with unrelated right-hand sides.  Vectors of the batch are interleaved,
// v[i * MP + j] (MP = padded batch width), so a gather of row i's neighbour c reads the
// MP values of all systems from one contiguous segment; lane j of a row group owns
// system j, so no cross-lane reduction is needed inside a row.
//
// An outer defect-correction cycle recomputes f_j - (A + sigma_j) x_j in FP64 (the
// multi-vector kernels below), the inner CG runs in the working precision from e = 0,
// and x_j += e_j is accumulated in FP64.
#include <type_traits>

#include "dev_common.h"
#include "msc_internal.h"
#include "sell_load.h"

namespace msc {

namespace {

template <class R> __device__ __forceinline__ Csr<cplx<R>> pick_a(const BssArgs& a, bool second);
template <> __device__ __forceinline__ Csr<float2> pick_a<float>(const BssArgs& a, bool second) {
  return second ? a.mh32 : a.m32;
}
template <> __device__ __forceinline__ Csr<double2> pick_a<double>(const BssArgs& a, bool second) {
  return second ? a.mh64 : a.m64;
}

// Reduce one double per thread to per-system sums (system = lane % MP) and store the
// workgroup's MP partials.
template <int MP>
__device__ __forceinline__ void store_system_partials(double v, double* partial) {
  __shared__ double part[kBlock / kWave][kBssMax];
#pragma unroll
  for (int off = MP; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane < MP) part[w][lane] = v;
  __syncthreads();
  if (threadIdx.x < MP) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; ++q) s += part[q][threadIdx.x];
    store_agent(&partial[blockIdx.x * kBssMax + threadIdx.x], s);
  }
}

// In the last workgroup: per-system totals of all workgroups' partials into out[0..15].
__device__ __forceinline__ void sum_system_partials(const double* partial, int count, double* out) {
  // thread -> (system j = tid / 16, sub-lane s = tid % 16)
  const int j = threadIdx.x / 16, s = threadIdx.x % 16;
  double acc = 0.0;
  for (int b = s; b < count; b += 16) acc += load_agent(&partial[b * kBssMax + j]);
  acc = group_sum<16>(acc);
  if (s == 0) out[j] = acc;
  __syncthreads();
}

// After the partials of IK1 are stored: the last workgroup forms a_j = R_j / P_j.
__device__ void ik1_finish(const BssArgs& a) {
  BssState* st = a.st;
  if (!arrive_last(a.tickets + 8 * kTicketSite)) return;
  __shared__ double tot[kBssMax];
  sum_system_partials(a.partial, gridDim.x, tot);
  const int q = threadIdx.x;
  if (q < st->m && st->active[q]) {
    const double P = tot[q];
    if (P > 0.0 && isfinite(P)) {
      st->a[q] = st->R[q] / P;
    } else {
      st->a[q] = 0.0;
      st->active[q] = 0;
      st->bad[q] = 1;
    }
  }
}

// After the partials of IK2 are stored: the last workgroup forms b_j and R_j, retires
// converged systems and decides whether the batch halts.
__device__ void ik2_finish(const BssArgs& a) {
  BssState* st = a.st;
  if (!arrive_last(a.tickets + 9 * kTicketSite)) return;
  __shared__ double tot[kBssMax];
  sum_system_partials(a.partial, gridDim.x, tot);
  if (threadIdx.x < kWave) {
    const int qq = threadIdx.x;
    bool upd = false, act = false;
    if (qq < st->m && st->active[qq]) {
      const double Rn = tot[qq];
      upd = true;
      if (!isfinite(Rn)) {
        st->bad[qq] = 1;
        st->active[qq] = 0;
        upd = false;
      } else {
        st->b[qq] = Rn / st->R[qq];
        st->R[qq] = Rn;
        st->iters[qq] += 1;
        if (Rn <= st->target2[qq]) st->active[qq] = 0;
        act = st->active[qq] != 0;
      }
    }
    if (qq < kBssMax) st->upd[qq] = upd ? 1 : 0;
    const uint64_t am = __ballot(act);
    if (qq == 0) {
      st->iter += 1;
      st->nact = __popcll(am);
      if (st->nact == 0 || st->iter >= st->max_iter) {
        st->halt = 1;
        store_host_flag(a.hflag, 1);
      }
      st->k3_enable = 1;
    }
  }
}

// ---- IK1: t_j = A1 p_j and P_j = p_j^H (A + sigma_j) p_j ----------------------------
template <class R, int MP, bool MHM>
__global__ __launch_bounds__(kBlock) void ik1(BssArgs a) {
  BssState* st = a.st;
  if (st->halt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->k3_enable = 0;
    return;
  }
  const Csr<cplx<R>> m = pick_a<R>(a, false);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.p);
  cplx<R>* __restrict__ t = static_cast<cplx<R>*>(a.t);
  constexpr int GPB = kBlock / MP;
  const int j = threadIdx.x % MP, grp = threadIdx.x / MP;
  const double sig = st->sigma[j];
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double acc = 0.0;
  for (int64_t row = beg + grp; row < end; row += GPB) {
    cplx<R> sum = czero<R>();
    const int32_t e0 = m.rowptr[row], e1 = m.rowptr[row + 1];
    int32_t e = e0;
    for (; e + 3 < e1; e += 4) {
      const int32_t c0 = m.col[e], c1 = m.col[e + 1], c2 = m.col[e + 2], c3 = m.col[e + 3];
      const cplx<R> v0 = m.val[e], v1 = m.val[e + 1], v2 = m.val[e + 2], v3 = m.val[e + 3];
      const cplx<R> x0 = p[int64_t(c0) * MP + j], x1 = p[int64_t(c1) * MP + j];
      const cplx<R> x2 = p[int64_t(c2) * MP + j], x3 = p[int64_t(c3) * MP + j];
      cfma<R>(sum, v0, x0);
      cfma<R>(sum, v1, x1);
      cfma<R>(sum, v2, x2);
      cfma<R>(sum, v3, x3);
    }
    for (; e < e1; ++e) cfma<R>(sum, m.val[e], p[int64_t(m.col[e]) * MP + j]);
    t[row * MP + j] = sum;
    const cplx<R> pr = p[row * MP + j];
    if (MHM)
      acc += norm2d<R>(sum) + sig * norm2d<R>(pr);
    else
      acc += double(pr.x) * double(sum.x) + double(pr.y) * double(sum.y) + sig * norm2d<R>(pr);
  }
  store_system_partials<MP>(acc, a.partial);
  ik1_finish(a);
}

// ---- IK2: r_j <- r_j - a_j (A2 t_j + sigma_j p_j), R_j = |r_j|^2 ----------------------
template <class R, int MP, bool MHM>
__global__ __launch_bounds__(kBlock) void ik2(BssArgs a) {
  BssState* st = a.st;
  if (st->halt) return;
  const cplx<R>* __restrict__ t = static_cast<const cplx<R>*>(a.t);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.p);
  cplx<R>* __restrict__ r = static_cast<cplx<R>*>(a.r);
  constexpr int GPB = kBlock / MP;
  const int j = threadIdx.x % MP, grp = threadIdx.x / MP;
  const double sig = st->sigma[j];
  const double step = st->active[j] ? st->a[j] : 0.0;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double acc = 0.0;
  for (int64_t row = beg + grp; row < end; row += GPB) {
    double2 q;
    if (MHM) {
      const Csr<cplx<R>> mh = pick_a<R>(a, true);
      cplx<R> sum = czero<R>();
      const int32_t e0 = mh.rowptr[row], e1 = mh.rowptr[row + 1];
      int32_t e = e0;
      for (; e + 3 < e1; e += 4) {
        const int32_t c0 = mh.col[e], c1 = mh.col[e + 1], c2 = mh.col[e + 2], c3 = mh.col[e + 3];
        const cplx<R> v0 = mh.val[e], v1 = mh.val[e + 1], v2 = mh.val[e + 2], v3 = mh.val[e + 3];
        const cplx<R> x0 = t[int64_t(c0) * MP + j], x1 = t[int64_t(c1) * MP + j];
        const cplx<R> x2 = t[int64_t(c2) * MP + j], x3 = t[int64_t(c3) * MP + j];
        cfma<R>(sum, v0, x0);
        cfma<R>(sum, v1, x1);
        cfma<R>(sum, v2, x2);
        cfma<R>(sum, v3, x3);
      }
      for (; e < e1; ++e) cfma<R>(sum, mh.val[e], t[int64_t(mh.col[e]) * MP + j]);
      q = to_d(sum);
    } else {
      q = to_d(t[row * MP + j]);
    }
    const double2 pr = to_d(p[row * MP + j]);
    const double2 rr = to_d(r[row * MP + j]);
    double2 nr;
    nr.x = rr.x - step * (q.x + sig * pr.x);
    nr.y = rr.y - step * (q.y + sig * pr.y);
    const cplx<R> sr = from_d<R>(nr);
    r[row * MP + j] = sr;
    acc += norm2d<R>(sr);
  }
  store_system_partials<MP>(acc, a.partial);
  ik2_finish(a);
}

// ---- IK1 and IK2 on the sliced ELLPACK copies: one row per lane, every system of the
// batch per lane (one read of the matrix row serves all of them) ----------------------
// Pairs per round trip: the MP gathered values of 2 KP entries stay within the budget.
template <class R, int MP> constexpr int kp_bss() {
  return std::is_same<R, float>::value ? (MP <= 4 ? 4 : (MP == 8 ? 2 : 1))
                                       : (MP <= 4 ? 2 : 1);
}
template <class R> __device__ __forceinline__ Sell<cplx<R>> pick_s(const BssArgs& a, bool second);
template <> __device__ __forceinline__ Sell<float2> pick_s<float>(const BssArgs& a, bool second) {
  return second ? a.sh32 : a.s32;
}
template <> __device__ __forceinline__ Sell<double2> pick_s<double>(const BssArgs& a, bool second) {
  return second ? a.sh64 : a.s64;
}

// Per-system workgroup sums of MP doubles per thread, stored as the workgroup's partials.
template <int MP>
__device__ __forceinline__ void store_rr_partials(double (&v)[MP], double* partial) {
  block_sum_k<kBlock, MP>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < MP; ++q) store_agent(&partial[blockIdx.x * kBssMax + q], v[q]);
  }
}

template <class R, int MP, bool MHM>
__global__ __launch_bounds__(kBlock) void ik1s(BssArgs a) {
  BssState* st = a.st;
  if (st->halt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->k3_enable = 0;
    return;
  }
  const Sell<cplx<R>> m = pick_s<R>(a, false);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.p);
  cplx<R>* __restrict__ t = static_cast<cplx<R>*>(a.t);
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  double sig[MP], acc[MP];
#pragma unroll
  for (int q = 0; q < MP; ++q) {
    sig[q] = st->sigma[q];
    acc[q] = 0.0;
  }
  int64_t beg, end;
  block_range(a.nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const bool live = row < a.n;
    const int64_t rr = live ? row : a.n - 1;  // lanes past n read a valid row, unused
    cplx<R> v[MP], pr[MP];
    sell_row_rhs<R, MP, kp_bss<R, MP>()>(m, p, sl, lane, v);
    load_rhs<R, MP>(p, rr, pr);
    const cplx<R> d = m.diag[rr];
    if (live) {
#pragma unroll
      for (int q = 0; q < MP; ++q) {
        cfma<R>(v[q], d, pr[q]);
        t[row * MP + q] = v[q];
        if (MHM)
          acc[q] += norm2d<R>(v[q]) + sig[q] * norm2d<R>(pr[q]);
        else
          acc[q] += double(pr[q].x) * double(v[q].x) + double(pr[q].y) * double(v[q].y) +
                    sig[q] * norm2d<R>(pr[q]);
      }
    }
  }
  store_rr_partials<MP>(acc, a.partial);
  ik1_finish(a);
}

template <class R, int MP, bool MHM>
__global__ __launch_bounds__(kBlock) void ik2s(BssArgs a) {
  BssState* st = a.st;
  if (st->halt) return;
  const cplx<R>* __restrict__ t = static_cast<const cplx<R>*>(a.t);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.p);
  cplx<R>* __restrict__ r = static_cast<cplx<R>*>(a.r);
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  double sig[MP], step[MP], acc[MP];
#pragma unroll
  for (int q = 0; q < MP; ++q) {
    sig[q] = st->sigma[q];
    step[q] = st->active[q] ? st->a[q] : 0.0;
    acc[q] = 0.0;
  }
  int64_t beg, end;
  block_range(a.nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const bool live = row < a.n;
    const int64_t rr = live ? row : a.n - 1;
    cplx<R> v[MP], pr[MP], rv[MP];
    if (MHM) {
      const Sell<cplx<R>> mh = pick_s<R>(a, true);
      cplx<R> tr[MP];
      sell_row_rhs<R, MP, kp_bss<R, MP>()>(mh, t, sl, lane, v);
      load_rhs<R, MP>(t, rr, tr);
      const cplx<R> d = mh.diag[rr];
#pragma unroll
      for (int q = 0; q < MP; ++q) cfma<R>(v[q], d, tr[q]);
    } else {
      load_rhs<R, MP>(t, rr, v);
    }
    load_rhs<R, MP>(p, rr, pr);
    load_rhs<R, MP>(r, rr, rv);
    if (live) {
#pragma unroll
      for (int q = 0; q < MP; ++q) {
        const double2 qd = to_d(v[q]), pd = to_d(pr[q]), rd = to_d(rv[q]);
        double2 nr;
        nr.x = rd.x - step[q] * (qd.x + sig[q] * pd.x);
        nr.y = rd.y - step[q] * (qd.y + sig[q] * pd.y);
        const cplx<R> sr = from_d<R>(nr);
        r[row * MP + q] = sr;
        acc[q] += norm2d<R>(sr);
      }
    }
  }
  store_rr_partials<MP>(acc, a.partial);
  ik2_finish(a);
}

// ---- IK3: e_j += a_j p_j; p_j <- r_j + b_j p_j (elementwise over the batch) --------------
template <class R, int MP>
__global__ __launch_bounds__(kBlock) void ik3(BssArgs a) {
  const BssState* st = a.st;
  if (!st->k3_enable) return;
  const cplx<R>* __restrict__ r = static_cast<const cplx<R>*>(a.r);
  cplx<R>* __restrict__ p = static_cast<cplx<R>*>(a.p);
  cplx<R>* __restrict__ ev = static_cast<cplx<R>*>(a.e);
  const int64_t total = a.n * MP;
  int64_t beg, end;
  block_range(total, kBlock, beg, end);
  for (int64_t idx = beg + threadIdx.x; idx < end; idx += kBlock) {
    const int j = int(idx % MP);
    if (!st->upd[j]) continue;
    const double2 pd = to_d(p[idx]);
    double2 ed = to_d(ev[idx]);
    const double aj = st->a[j];
    ed.x = fma(aj, pd.x, ed.x);
    ed.y = fma(aj, pd.y, ed.y);
    ev[idx] = from_d<R>(ed);
    if (st->active[j]) {
      const double2 rd = to_d(r[idx]);
      const double bj = st->b[j];
      p[idx] = from_d<R>(double2{fma(bj, pd.x, rd.x), fma(bj, pd.y, rd.y)});
    }
  }
}

// ---- FP64 residual of up to 8 systems: r_j = f_j - (A + sigma_j) x_j ---------------------
template <int L>
__device__ __forceinline__ void row_dot_ptrs(const Csr<double2>& m, const double2* const* xs, int kc,
                                             int64_t row, int lane, double2 (&acc)[kResChunk]) {
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) acc[q] = double2{0.0, 0.0};
  const int32_t beg = m.rowptr[row], end = m.rowptr[row + 1];
  for (int32_t e = beg + lane; e < end; e += L) {
    const int32_t c = m.col[e];
    const double2 v = m.val[e];
#pragma unroll
    for (int q = 0; q < kResChunk; ++q)
      if (q < kc) cfma<double>(acc[q], v, xs[q][c]);
  }
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) acc[q] = group_sum_c<L, double>(acc[q]);
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_res_first(ResArgs v) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(v.n, GPB, beg, end);
  double2 acc[kResChunk];
  for (int64_t row = beg + grp; row < end; row += GPB) {
    row_dot_ptrs<L>(v.m1, v.x, v.kc, row, lane, acc);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kResChunk; ++q)
        if (q < v.kc) v.u[int64_t(q) * v.n + row] = acc[q];
    }
  }
}

// Per-system norms: workgroup partials, then the last workgroup's totals in out[0..kc).
__device__ void res_finish(const ResArgs& v, double (&nrm)[kResChunk]) {
  block_sum_k<kBlock, kResChunk>(nrm);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kResChunk; ++q) store_agent(&v.partial[blockIdx.x * kResChunk + q], nrm[q]);
  }
  if (!arrive_last(v.ticket)) return;
  for (int q = 0; q < v.kc; ++q) {
    double s = 0.0;
    for (int i = threadIdx.x; i < int(gridDim.x); i += kBlock) s += load_agent(&v.partial[i * kResChunk + q]);
    s = block_sum<kBlock>(s);
    if (threadIdx.x == 0) v.out[q] = s;
  }
}

// Row `row`'s residuals from the products acc_q = (A x_q)[row]: norms, and the
// interleaved r = p = residual, e = 0 when r is set.
template <class R>
__device__ __forceinline__ void res_row(const ResArgs& v, int64_t row, const double2 (&acc)[kResChunk],
                                        double (&nrm)[kResChunk]) {
  cplx<R>* __restrict__ r = static_cast<cplx<R>*>(v.r);
  cplx<R>* __restrict__ p = static_cast<cplx<R>*>(v.p);
  cplx<R>* __restrict__ e = static_cast<cplx<R>*>(v.e);
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) {
    if (q < v.kc) {
      const double2 fv = v.f[q][row], xv = v.x[q][row];
      double2 rt;
      rt.x = fv.x - acc[q].x - v.sig[q] * xv.x;
      rt.y = fv.y - acc[q].y - v.sig[q] * xv.y;
      nrm[q] += fma(rt.x, rt.x, rt.y * rt.y);
      if (r) {
        const int64_t idx = row * v.mp + v.j0 + q;
        const cplx<R> rc = from_d<R>(rt);
        r[idx] = rc;
        p[idx] = rc;
        e[idx] = czero<R>();
      }
    }
  }
}

template <class R, int L>
__global__ __launch_bounds__(kBlock) void k_res_second(ResArgs v) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(v.n, GPB, beg, end);
  double2 acc[kResChunk];
  double nrm[kResChunk];
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) nrm[q] = 0.0;
  const double2* in[kResChunk];
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) in[q] = v.mhm ? v.u + int64_t(q) * v.n : v.x[q];
  for (int64_t row = beg + grp; row < end; row += GPB) {
    row_dot_ptrs<L>(v.m2, in, v.kc, row, lane, acc);
    if (lane == 0) res_row<R>(v, row, acc, nrm);
  }
  res_finish(v, nrm);
}

// The same two steps on the sliced ELLPACK copies: one row per lane.
__global__ __launch_bounds__(kBlock) void k_res_first_s(ResArgs v) {
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  const double2* xs[kResChunk];
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) xs[q] = v.x[q < v.kc ? q : 0];
  int64_t beg, end;
  block_range(v.nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < v.n ? row : v.n - 1;
    double2 acc[kResChunk];
    sell_row_multi<double, kResChunk, 1>(v.s1, xs, v.kc, sl, lane, acc);
    const double2 d = v.s1.diag[rr];
#pragma unroll
    for (int q = 0; q < kResChunk; ++q) {
      if (q < v.kc) {
        cfma<double>(acc[q], d, xs[q][rr]);
        if (row < v.n) v.u[int64_t(q) * v.n + row] = acc[q];
      }
    }
  }
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_res_second_s(ResArgs v) {
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  const double2* in[kResChunk];
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) {
    const int qq = q < v.kc ? q : 0;
    in[q] = v.mhm ? v.u + int64_t(qq) * v.n : v.x[qq];
  }
  double nrm[kResChunk];
#pragma unroll
  for (int q = 0; q < kResChunk; ++q) nrm[q] = 0.0;
  int64_t beg, end;
  block_range(v.nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < v.n ? row : v.n - 1;
    double2 acc[kResChunk];
    sell_row_multi<double, kResChunk, 1>(v.s2, in, v.kc, sl, lane, acc);
    const double2 d = v.s2.diag[rr];
#pragma unroll
    for (int q = 0; q < kResChunk; ++q)
      if (q < v.kc) cfma<double>(acc[q], d, in[q][rr]);
    if (row < v.n) res_row<R>(v, row, acc, nrm);
  }
  res_finish(v, nrm);
}

// x_j += e_j (FP64 accumulation of the correction)
template <class R, int MP>
__global__ __launch_bounds__(kBlock) void k_accum(BssArgs a, XPtrs xp) {
  const cplx<R>* __restrict__ ev = static_cast<const cplx<R>*>(a.e);
  const int m = a.st->m;
  for (int j = 0; j < m; ++j) {
    double2* __restrict__ x = xp.x[j];
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * kBlock) {
      const double2 d = to_d(ev[i * MP + j]);
      double2 v = x[i];
      v.x += d.x;
      v.y += d.y;
      x[i] = v;
    }
  }
}

int grid_for(int64_t items, int per_pass) {
  int64_t g = (items + per_pass - 1) / per_pass;
  if (g > kMaxGrid) g = kMaxGrid;
  if (g < kXcds) g = kXcds;
  return int((g + kXcds - 1) / kXcds * kXcds);
}

#define MSC_MP_SWITCH(MPV, CALL)                         \
  switch (MPV) {                                         \
    case 4: { constexpr int MPP = 4; CALL; } break;      \
    case 8: { constexpr int MPP = 8; CALL; } break;      \
    case 16: { constexpr int MPP = 16; CALL; } break;    \
    default: return hipErrorInvalidValue;                \
  }

#define MSC_L_SWITCH(LANES, CALL)                        \
  switch (LANES) {                                       \
    case 4: { constexpr int LL = 4; CALL; } break;       \
    case 8: { constexpr int LL = 8; CALL; } break;       \
    case 16: { constexpr int LL = 16; CALL; } break;     \
    case 32: { constexpr int LL = 32; CALL; } break;     \
    default: return hipErrorInvalidValue;                \
  }

template <class R>
hipError_t bss_iteration_impl(const BssArgs& a, hipStream_t s) {
  const int g1 = grid_for(a.n, kBlock / a.mp);
  const int g3 = grid_for(a.n * a.mp, kBlock);
  if (a.sell) {
    const int gs = grid_for(a.nslices, kBlock / kSlice);
    if (a.kind == MSC_A_MHM) {
      MSC_MP_SWITCH(a.mp, (ik1s<R, MPP, true><<<gs, kBlock, 0, s>>>(a)));
      MSC_MP_SWITCH(a.mp, (ik2s<R, MPP, true><<<gs, kBlock, 0, s>>>(a)));
    } else {
      MSC_MP_SWITCH(a.mp, (ik1s<R, MPP, false><<<gs, kBlock, 0, s>>>(a)));
      MSC_MP_SWITCH(a.mp, (ik2s<R, MPP, false><<<gs, kBlock, 0, s>>>(a)));
    }
  } else if (a.kind == MSC_A_MHM) {
    MSC_MP_SWITCH(a.mp, (ik1<R, MPP, true><<<g1, kBlock, 0, s>>>(a)));
    MSC_MP_SWITCH(a.mp, (ik2<R, MPP, true><<<g1, kBlock, 0, s>>>(a)));
  } else {
    MSC_MP_SWITCH(a.mp, (ik1<R, MPP, false><<<g1, kBlock, 0, s>>>(a)));
    MSC_MP_SWITCH(a.mp, (ik2<R, MPP, false><<<g1, kBlock, 0, s>>>(a)));
  }
  MSC_MP_SWITCH(a.mp, (ik3<R, MPP><<<g3, kBlock, 0, s>>>(a)));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bss_iteration(int prec, const BssArgs& a, hipStream_t s) {
  return prec == MSC_PREC_MIXED ? bss_iteration_impl<float>(a, s) : bss_iteration_impl<double>(a, s);
}

hipError_t launch_residual(int prec, int lanes, const ResArgs& v, hipStream_t s) {
  if (v.kc < 1 || v.kc > kResChunk) return hipErrorInvalidValue;
  if (v.sell) {
    const int gs = grid_for(v.nslices, kBlock / kSlice);
    if (v.mhm) k_res_first_s<<<gs, kBlock, 0, s>>>(v);
    if (prec == MSC_PREC_MIXED)
      k_res_second_s<float><<<gs, kBlock, 0, s>>>(v);
    else
      k_res_second_s<double><<<gs, kBlock, 0, s>>>(v);
    return hipGetLastError();
  }
  const int g1 = grid_for(v.n, kBlock / lanes);
  if (v.mhm) MSC_L_SWITCH(lanes, (k_res_first<LL><<<g1, kBlock, 0, s>>>(v)));
  if (prec == MSC_PREC_MIXED) {
    MSC_L_SWITCH(lanes, (k_res_second<float, LL><<<g1, kBlock, 0, s>>>(v)));
  } else {
    MSC_L_SWITCH(lanes, (k_res_second<double, LL><<<g1, kBlock, 0, s>>>(v)));
  }
  return hipGetLastError();
}

hipError_t launch_accum(int prec, const BssArgs& a, const XPtrs& xp, hipStream_t s) {
  const int g = grid_for(a.n, kBlock);
  if (prec == MSC_PREC_MIXED) {
    MSC_MP_SWITCH(a.mp, (k_accum<float, MPP><<<g, kBlock, 0, s>>>(a, xp)));
  } else {
    MSC_MP_SWITCH(a.mp, (k_accum<double, MPP><<<g, kBlock, 0, s>>>(a, xp)));
  }
  return hipGetLastError();
}

}  // namespace msc
