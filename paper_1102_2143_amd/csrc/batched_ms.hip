// Batched multishift solves: many independent systems of uneven size, each with up to
// four right-hand sides and up to sixteen shifts, advanced together -- one launch of
// each iteration kernel covers every row of every unfinished system.
//
// Work is split into chunks of rows (each chunk belongs to one system); the kernels are
// persistent (a bounded grid loops over the chunk list).  The right-hand sides of a
// system are interleaved, v[i * R + q], so one read of a matrix row serves all of them.
// Every system has its own scalar state; the last chunk of a system to finish a kernel
// finalises that system's reductions and recurrences (one lane per (rhs, shift) pair).
// Each system runs its multishift sequence in FP64 until all its right-hand sides reach
// switch_tol, then in complex64 with FP64 reliable updates (same scheme as the single
// solve).
#include <type_traits>

#include "dev_common.h"
#include "msc_internal.h"
#include "sell_load.h"

namespace msc {

namespace {

constexpr int kQK = kBatchMaxRhs * kBatchMaxShifts;  // 64 lanes of the finalising wave

template <class R> __device__ __forceinline__ cplx<R>* vec_r(const BatchSys& S);
template <> __device__ __forceinline__ double2* vec_r<double>(const BatchSys& S) { return S.r64; }
template <> __device__ __forceinline__ float2* vec_r<float>(const BatchSys& S) { return S.r32; }
template <class R> __device__ __forceinline__ cplx<R>* vec_p(const BatchSys& S);
template <> __device__ __forceinline__ double2* vec_p<double>(const BatchSys& S) { return S.p64; }
template <> __device__ __forceinline__ float2* vec_p<float>(const BatchSys& S) { return S.p32; }
template <class R> __device__ __forceinline__ cplx<R>* vec_t(const BatchSys& S);
template <> __device__ __forceinline__ double2* vec_t<double>(const BatchSys& S) { return S.t64; }
template <> __device__ __forceinline__ float2* vec_t<float>(const BatchSys& S) { return S.t32; }
template <class R> __device__ __forceinline__ cplx<R>* vec_pk(const BatchSys& S);
template <> __device__ __forceinline__ double2* vec_pk<double>(const BatchSys& S) { return S.pk64; }
template <> __device__ __forceinline__ float2* vec_pk<float>(const BatchSys& S) { return S.pk32; }
template <class R> __device__ __forceinline__ Csr<cplx<R>> mat1(const BatchSys& S);
template <> __device__ __forceinline__ Csr<double2> mat1<double>(const BatchSys& S) { return S.m64; }
template <> __device__ __forceinline__ Csr<float2> mat1<float>(const BatchSys& S) { return S.m32; }
template <class R> __device__ __forceinline__ Csr<cplx<R>> mat2(const BatchSys& S);
template <> __device__ __forceinline__ Csr<double2> mat2<double>(const BatchSys& S) { return S.mh64; }
template <> __device__ __forceinline__ Csr<float2> mat2<float>(const BatchSys& S) { return S.mh32; }

// Row i of a CSR times the RHS-interleaved vector x (RR right-hand sides), L lanes per
// row; sums returned in every lane of the row group.
template <class R, int L, int RR>
__device__ __forceinline__ void row_dot_rhs(const Csr<cplx<R>>& m, const cplx<R>* __restrict__ x,
                                            int64_t row, int lane, cplx<R> (&acc)[RR]) {
#pragma unroll
  for (int q = 0; q < RR; ++q) acc[q] = czero<R>();
  const int32_t beg = m.rowptr[row], end = m.rowptr[row + 1];
  for (int32_t base = beg; base < end; base += 4 * L) {
    int32_t c[4];
    cplx<R> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t j = base + lane + u * L;
      const bool ok = j < end;
      c[u] = ok ? m.col[j] : 0;
      v[u] = ok ? m.val[j] : czero<R>();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int q = 0; q < RR; ++q) cfma<R>(acc[q], v[u], x[int64_t(c[u]) * RR + q]);
    }
  }
#pragma unroll
  for (int q = 0; q < RR; ++q) acc[q] = group_sum_c<L, R>(acc[q]);
}

template <class R> __device__ __forceinline__ Sell<cplx<R>> sell1(const BatchSys& S);
template <> __device__ __forceinline__ Sell<double2> sell1<double>(const BatchSys& S) { return S.s64; }
template <> __device__ __forceinline__ Sell<float2> sell1<float>(const BatchSys& S) { return S.s32; }
template <class R> __device__ __forceinline__ Sell<cplx<R>> sell2(const BatchSys& S);
template <> __device__ __forceinline__ Sell<double2> sell2<double>(const BatchSys& S) { return S.sh64; }
template <> __device__ __forceinline__ Sell<float2> sell2<float>(const BatchSys& S) { return S.sh32; }

// Pairs per round trip of the RR-rhs product (MSC_BATCH_KP32 / MSC_BATCH_KP64 at four
// right-hand sides, twice that for fewer).
#ifndef MSC_BATCH_KP32
#define MSC_BATCH_KP32 4
#endif
#ifndef MSC_BATCH_KP64
#define MSC_BATCH_KP64 2
#endif
template <class R, int RR> constexpr int kp_rhs() {
  return std::is_same<R, float>::value ? (RR >= 4 ? MSC_BATCH_KP32 : 2 * MSC_BATCH_KP32)
                                       : (RR >= 4 ? MSC_BATCH_KP64 : 2 * MSC_BATCH_KP64);
}

// Per-rhs workgroup partials of a chunk: store, take the system's ticket; true in the
// last chunk of the system, which then holds the per-rhs totals in tot[].
__device__ __forceinline__ bool chunk_reduce(double (&v)[kBatchMaxRhs], const BatchSys& S, int cidx,
                                             int ticket, double* tot) {
  block_sum_k<kBlock, kBatchMaxRhs>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kBatchMaxRhs; ++q) store_agent(&S.partial[cidx * kBatchMaxRhs + q], v[q]);
  }
  if (!arrive_last(S.tickets + ticket * kTicketSite, unsigned(S.nchunks), unsigned(cidx))) return false;
  // thread -> (rhs q = tid / 64, sub-lane) : all loads of a rhs in flight together
  const int q = threadIdx.x / kWave, s = threadIdx.x % kWave;
  double acc = 0.0;
  for (int c = s; c < S.nchunks; c += kWave) acc += load_agent(&S.partial[c * kBatchMaxRhs + q]);
  acc = group_sum<kWave>(acc);
  if (s == 0) tot[q] = acc;
  __syncthreads();
  return true;
}

// ---- BK1: t = A1 p for every rhs; per rhs P = |t|^2 + s0|p|^2 (or Re p^H t + s0|p|^2) ----
template <class R, int L, int RR>
__device__ void bk1_chunk(const BatchSys& S, BatchState* st, const int4& ch) {
  const Csr<cplx<R>> m = mat1<R>(S);
  const cplx<R>* __restrict__ p = vec_p<R>(S);
  cplx<R>* __restrict__ t = vec_t<R>(S);
  const double s0 = st->sigma0;
  const bool mhm = S.kind == MSC_A_MHM;
  double acc[kBatchMaxRhs] = {0.0, 0.0, 0.0, 0.0};
  auto epilogue = [&](int64_t row, const cplx<R> (&v)[RR], const cplx<R> (&pr)[RR]) {
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      t[row * RR + q] = v[q];
      acc[q] += (mhm ? norm2d<R>(v[q])
                     : double(pr[q].x) * double(v[q].x) + double(pr[q].y) * double(v[q].y)) +
                s0 * norm2d<R>(pr[q]);
    }
  };
  if (S.sell) {
    // one row per lane: the chunk's four slices, one per wave
    const Sell<cplx<R>> ms = sell1<R>(S);
    const int lane = threadIdx.x % kSlice;
    const int64_t sl = ch.y / kSlice + __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
    if (sl * kSlice < ch.z) {
      const int64_t row = sl * kSlice + lane;
      const int64_t rr = row < ch.z ? row : ch.z - 1;
      cplx<R> pr[RR], v[RR];
      load_rhs<R, RR>(p, rr, pr);
      const cplx<R> d = ms.diag[rr];
      sell_row_rhs<R, RR, kp_rhs<R, RR>()>(ms, p, sl, lane, v);
#pragma unroll
      for (int q = 0; q < RR; ++q) cfma<R>(v[q], d, pr[q]);
      if (row < ch.z) epilogue(row, v, pr);
    }
  } else {
    constexpr int GPB = kBlock / L;
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    for (int64_t row = ch.y + grp; row < ch.z; row += GPB) {
      cplx<R> v[RR];
      row_dot_rhs<R, L, RR>(m, p, row, lane, v);
      if (lane == 0) {
        cplx<R> pr[RR];
#pragma unroll
        for (int q = 0; q < RR; ++q) pr[q] = p[row * RR + q];
        epilogue(row, v, pr);
      }
    }
  }
  __shared__ double tot[kBatchMaxRhs];
  if (!chunk_reduce(acc, S, ch.w, 0, tot)) return;
  // finalise: lane = q * 16 + k
  const int lk = threadIdx.x;
  if (lk >= kQK) return;
  if (lk == 0 && st->switch_pending) {
    // this launch read the complex64 buffers written by the switching update
    st->switch_pending = 0;
    st->phase32 = 1;
  }
  const int q = lk / kBatchMaxShifts, k = lk % kBatchMaxShifts;
  if (q >= st->nrhs || st->halt[q]) return;
  const double P = tot[q];
  if (!(P > 0.0 && isfinite(P))) {
    if (k == 0) {
      st->status[q] = 1;
      st->halt[q] = 1;
    }
    return;
  }
  const double a = st->R[q] / P;
  if (k >= 1 && k < st->ns && st->active[lk]) {
    const double z = st->zeta[lk], zp = st->zeta_prev[lk], ap = st->a_prev[q], b = st->b[q];
    const double zn = z * zp * ap / (a * b * (zp - z) + zp * ap * (1.0 + st->s[k] * a));
    st->zk[lk] = zn;
    st->ak[lk] = a * zn / z;
  }
  if (k == 0) st->a[q] = a;
}

// ---- BK2: r <- r - a (A2 t + s0 p), R' = |r|^2; recurrences, freezing, halting ------------
template <class R, int L, int RR>
__device__ void bk2_chunk(const BatchSys& S, BatchState* st, const int4& ch, int* active_systems,
                          int defer_ok, int steps) {
  const cplx<R>* __restrict__ t = vec_t<R>(S);
  const cplx<R>* __restrict__ p = vec_p<R>(S);
  cplx<R>* __restrict__ r = vec_r<R>(S);
  const double s0 = st->sigma0;
  const bool mhm = S.kind == MSC_A_MHM;
  double step[RR];
#pragma unroll
  for (int q = 0; q < RR; ++q) step[q] = (q < st->nrhs && !st->halt[q]) ? st->a[q] : 0.0;
  double acc[kBatchMaxRhs] = {0.0, 0.0, 0.0, 0.0};
  auto epilogue = [&](int64_t row, const cplx<R> (&qv)[RR]) {
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      const double2 pr = to_d(p[row * RR + q]), rr = to_d(r[row * RR + q]), qd = to_d(qv[q]);
      const double2 nr{rr.x - step[q] * (qd.x + s0 * pr.x), rr.y - step[q] * (qd.y + s0 * pr.y)};
      const cplx<R> sr = from_d<R>(nr);
      r[row * RR + q] = sr;
      acc[q] += norm2d<R>(sr);
    }
  };
  if (S.sell && mhm) {
    // one row per lane: the chunk's four slices, one per wave
    const Sell<cplx<R>> ms = sell2<R>(S);
    const int lane = threadIdx.x % kSlice;
    const int64_t sl = ch.y / kSlice + __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
    if (sl * kSlice < ch.z) {
      const int64_t row = sl * kSlice + lane;
      const int64_t rr = row < ch.z ? row : ch.z - 1;
      cplx<R> tr[RR], qv[RR];
      load_rhs<R, RR>(t, rr, tr);
      const cplx<R> d = ms.diag[rr];
      sell_row_rhs<R, RR, kp_rhs<R, RR>()>(ms, t, sl, lane, qv);
#pragma unroll
      for (int q = 0; q < RR; ++q) cfma<R>(qv[q], d, tr[q]);
      if (row < ch.z) epilogue(row, qv);
    }
  } else {
    constexpr int GPB = kBlock / L;
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    for (int64_t row = ch.y + grp; row < ch.z; row += GPB) {
      cplx<R> qv[RR];
      if (mhm) {
        row_dot_rhs<R, L, RR>(mat2<R>(S), t, row, lane, qv);
      } else {
#pragma unroll
        for (int q = 0; q < RR; ++q) qv[q] = t[row * RR + q];
      }
      if (lane == 0) epilogue(row, qv);
    }
  }
  __shared__ double tot[kBatchMaxRhs];
  if (!chunk_reduce(acc, S, ch.w, 1, tot)) return;
  // one wave finalises: lane = q * 16 + k; every lane reads the state before any lane
  // writes it, and system-wide decisions travel by ballot, not through memory
  const int lk = threadIdx.x;
  if (lk >= kWave) return;
  const int q = lk / kBatchMaxShifts, k = lk % kBatchMaxShifts;
  const int nrhs = st->nrhs, ns = st->ns;
  const bool live = q < nrhs && !st->halt[q];
  const double Rq = live ? st->R[q] : 1.0;
  const double aq = live ? st->a[q] : 0.0;
  const int itq = live ? st->iter[q] : 0;
  const double eps2q = q < nrhs ? st->eps2[q] : 0.0;
  const double sw2q = q < nrhs ? st->sw_eps2[q] : 0.0;
  const int max_iter = st->max_iter;
  const int phase32 = st->phase32;
  // lane k = 0 of each rhs composes x_0's steps like a shift with zeta = 1 (step a_q,
  // direction coefficient b): x_0 then takes them in the BK3 that applies
  const bool drv = k == 0;
  const bool act = live && (drv || (k >= 1 && k < ns && st->active[lk]));
  const double z = (act && !drv) ? st->zeta[lk] : 1.0, zn = (act && !drv) ? st->zk[lk] : 1.0;
  const double akq = act ? (drv ? aq : st->ak[lk]) : 0.0;
  // steps this rhs deferred in previous BK3s, composed (read before any lane writes the
  // state): x_k gained cx[0] p_k + sum_i cx[i+1] r_i, p_k now is cp[0] p_k + sum_i cp[i+1] r_i
  const int md = q < nrhs ? st->ndef[q] : 0;
  double cx[kBatchMaxSteps + 1], cp[kBatchMaxSteps + 1];
#pragma unroll
  for (int i = 0; i <= kBatchMaxSteps; ++i) cx[i] = cp[i] = 0.0;
  cp[0] = 1.0;
  bool dact = false, dupd = false;
  if (md > 0 && k < ns) {
#pragma unroll
    for (int i = 0; i < kBatchMaxSteps; ++i) {
      if (i <= md) {
        cx[i] = st->dcx[i][lk];
        cp[i] = st->dcp[i][lk];
      }
    }
    dact = st->dact[lk] != 0;
    dupd = st->dupd[lk] != 0;
  }
  const double Rn = live ? tot[q] : 0.0;
  const double bn = Rn / Rq;
  bool keep_p = false;
  double bkq = 0.0;
  if (act && drv) {
    bkq = bn;
    keep_p = true;
  } else if (act) {
    const double ratio = zn / z;
    bkq = bn * ratio * ratio;
    st->bk[lk] = bkq;
    st->zeta_prev[lk] = z;
    st->zeta[lk] = zn;
    keep_p = true;
    if (zn * zn * Rn <= eps2q) {
      st->active[lk] = 0;
      st->freeze_iter[lk] = itq + 1;
      keep_p = false;
    }
  }
  // per right-hand side (lanes k == 0)
  const bool halt_q = live && (!isfinite(Rn) || Rn <= eps2q || itq + 1 >= max_iter);
  bool halted_after = true, below = true;
  if (k == 0 && q < nrhs) {
    st->x0_upd[q] = live ? 1 : 0;
    if (live) {
      st->b_new[q] = bn;
      st->a_prev[q] = aq;
      st->b[q] = bn;
      st->R[q] = Rn;
      st->iter[q] = itq + 1;
      if (!isfinite(Rn)) {
        st->status[q] = 1;
        st->halt[q] = 1;
      } else if (Rn <= eps2q || itq + 1 >= max_iter) {
        st->halt[q] = 1;
      } else {
        halted_after = false;
        below = Rn <= sw2q;
      }
    }
  }
  const bool all_halted = __ballot(!halted_after) == 0;
  const bool all_below = __ballot(!halted_after && !below) == 0;
  const bool switching = !all_halted && !phase32 && all_below;
  // fold this step into the composition (x_k += a_k p_k; p_k <- zeta_k' r + b_k p_k unless
  // k freezes now); then BK3 either defers it (this rhs continues, the vectors keep their
  // precision, fewer than `steps` - 1 steps pending) or applies every pending step
  if (act) {
#pragma unroll
    for (int i = 0; i < kBatchMaxSteps; ++i)
      if (i <= md) cx[i] = fma(akq, cp[i], cx[i]);
  }
  if (act && keep_p) {
#pragma unroll
    for (int i = 0; i < kBatchMaxSteps; ++i)
      if (i <= md) cp[i] *= bkq;
#pragma unroll
    for (int i = 1; i <= kBatchMaxSteps; ++i)
      if (i == md + 1) cp[i] = zn;
  }
  dact = dact || act;
  dupd = dupd || (act && keep_p);
  const bool defer = live && !halt_q && !switching && defer_ok && md + 1 < steps;
  const bool listed = !defer && dact && !drv;
  st->upd_x[lk] = listed ? 1 : 0;
  st->upd_p[lk] = (listed && dupd) ? 1 : 0;
#pragma unroll
  for (int i = 0; i < kBatchMaxSteps; ++i) st->cx[i][lk] = i <= md ? cx[i] : 0.0;
#pragma unroll
  for (int i = 0; i <= kBatchMaxSteps; ++i) st->cp[i][lk] = i <= md + 1 ? cp[i] : 0.0;
  if (defer) {
#pragma unroll
    for (int i = 0; i < kBatchMaxSteps; ++i) {
      st->dcx[i][lk] = i <= md ? cx[i] : 0.0;
      st->dcp[i][lk] = i <= md + 1 ? cp[i] : 0.0;
    }
    st->dact[lk] = dact ? 1 : 0;
    st->dupd[lk] = dupd ? 1 : 0;
  }
  const uint64_t lm = __ballot(listed);
  if (k == 0 && q < nrhs) {
    st->ndef[q] = defer ? md + 1 : 0;
    st->m[q] = defer ? 0 : md;
    st->keep[q] = defer ? md : -1;
    if (live) {
      const int ph = phase32 ? 1 : 0;
      st->n_upd[q][ph] += __popcll((lm >> (q * kBatchMaxShifts)) & 0xffffull);
      st->n_kept[q][ph] += defer ? 1 : md;
      st->n_x0[q][ph] += defer ? 0 : 1;
      st->n_k0[q][ph] += (defer && md == 0) ? 1 : 0;
    }
  }
  if (lk == 0) {
    st->k3_enable = 1;
    if (all_halted) {
      st->done = 1;
      atomicSub(active_systems, 1);
    } else if (switching) {
      st->switch_pending = 1;
      st->iters_fp64 = itq + 1;
    }
  }
}

// ---- BK3: x_q += a_q p_q, shifted updates, p_q <- r_q + b_q p_q --------------------------
// The update's per-(rhs, shift) coefficients, staged in LDS once per chunk so the loop
// over shifts issues its vector loads without first waiting on the scalar state.
struct K3Coef {
  double cx[kBatchMaxSteps][kQK], cp[kBatchMaxSteps + 1][kQK];
  int upd_x[kQK], upd_p[kQK];
  int orig[kBatchMaxShifts];
  double bnew[kBatchMaxRhs];
  int x0_upd[kBatchMaxRhs], m[kBatchMaxRhs], keep[kBatchMaxRhs];
  int nrhs, ns;
};

template <class R, class W, int RR>
__device__ void bk3_chunk(const BatchSys& S, const BatchState* st, const int4& ch) {
  __shared__ K3Coef cf;
  const int tid = threadIdx.x;
  __syncthreads();  // the previous chunk of this workgroup is done with cf
  if (tid < kQK) {
#pragma unroll
    for (int i = 0; i < kBatchMaxSteps; ++i) cf.cx[i][tid] = st->cx[i][tid];
#pragma unroll
    for (int i = 0; i <= kBatchMaxSteps; ++i) cf.cp[i][tid] = st->cp[i][tid];
    cf.upd_x[tid] = st->upd_x[tid];
    cf.upd_p[tid] = st->upd_p[tid];
  }
  if (tid < kBatchMaxShifts) cf.orig[tid] = st->orig[tid];
  if (tid < kBatchMaxRhs) {
    cf.bnew[tid] = st->b_new[tid];
    cf.x0_upd[tid] = st->x0_upd[tid];
    cf.m[tid] = st->m[tid];
    cf.keep[tid] = st->keep[tid];
  }
  if (tid == 0) {
    cf.nrhs = st->nrhs;
    cf.ns = st->ns;
  }
  __syncthreads();
  const cplx<R>* __restrict__ r = vec_r<R>(S);
  cplx<R>* __restrict__ p = vec_p<R>(S);
  cplx<R>* __restrict__ pk = vec_pk<R>(S);
  // outputs go to the W buffers: W == R except on the switching iteration (FP64 -> FP32)
  cplx<W>* __restrict__ pw = vec_p<W>(S);
  cplx<W>* __restrict__ rw = vec_r<W>(S);
  cplx<W>* __restrict__ pkw = vec_pk<W>(S);
  const int64_t n = S.n;
  const int ns = cf.ns;
  const int64_t rows = ch.z - ch.y;
  for (int64_t e = tid; e < rows * RR; e += kBlock) {
    const int64_t i = ch.y + e / RR;
    const int q = int(e % RR);
    const int64_t idx = i * RR + q;
    const double2 rd = to_d(r[idx]);
    const double2 pd = to_d(p[idx]);
    if (q < cf.nrhs && cf.x0_upd[q]) {
      // a deferring BK3 keeps r (the first of a cycle p too); the one that applies reads
      // the m kept residuals and updates x_0 and the shifts (with m = 0 the multiply-adds
      // round exactly as one step)
      const int mq = cf.m[q], kq = cf.keep[q];
      cplx<R>* __restrict__ pkeep0 = static_cast<cplx<R>*>(S.pkeep0);
      if (kq >= 0) static_cast<cplx<R>*>(S.rkeep[kq])[idx] = r[idx];
      if (kq == 0) pkeep0[idx] = p[idx];
      double2 rk[kBatchMaxSteps - 1];
#pragma unroll
      for (int kk = 0; kk < kBatchMaxSteps - 1; ++kk)
        rk[kk] = kk < mq ? to_d(static_cast<const cplx<R>*>(S.rkeep[kk])[idx]) : double2{0.0, 0.0};
      if (kq < 0) {
        double2* x0 = S.x + (int64_t(q) * ns + cf.orig[0]) * n + i;
        const int l0 = q * kBatchMaxShifts;
        const double2 p1 = mq > 0 ? to_d(pkeep0[idx]) : pd;
        double2 xv = *x0;
#pragma unroll
        for (int kk = kBatchMaxSteps - 2; kk >= 0; --kk) {
          if (kk < mq) {
            xv.x = fma(cf.cx[kk + 1][l0], rk[kk].x, xv.x);
            xv.y = fma(cf.cx[kk + 1][l0], rk[kk].y, xv.y);
          }
        }
        xv.x = fma(cf.cx[0][l0], p1.x, xv.x);
        xv.y = fma(cf.cx[0][l0], p1.y, xv.y);
        *x0 = xv;
      }
      constexpr bool same = std::is_same<R, W>::value;
      // two shifts at a time, their loads issued before either store (x_k and p_k of
      // different shifts share one array each, so the compiler cannot reorder); frozen
      // shifts are skipped except on the switching iteration, which copies them
      for (int k0 = 1; k0 < ns; k0 += 2) {
        double2 pj[2], xk[2];
        bool ux[2], ld[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int k = k0 + u;
          const int lk = q * kBatchMaxShifts + k;
          ux[u] = k < ns && cf.upd_x[lk];
          ld[u] = k < ns && (ux[u] || !same);
          if (ld[u]) pj[u] = to_d(pk[int64_t(k - 1) * n * RR + idx]);
          if (ux[u]) xk[u] = S.x[(int64_t(q) * ns + cf.orig[k]) * n + i];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int k = k0 + u;
          if (!ld[u]) continue;
          const int lk = q * kBatchMaxShifts + k;
          const int64_t pidx = int64_t(k - 1) * n * RR + idx;
          if (ux[u]) {
            double2 xv = xk[u];
#pragma unroll
            for (int kk = kBatchMaxSteps - 2; kk >= 0; --kk) {
              if (kk < mq) {
                xv.x = fma(cf.cx[kk + 1][lk], rk[kk].x, xv.x);
                xv.y = fma(cf.cx[kk + 1][lk], rk[kk].y, xv.y);
              }
            }
            xv.x = fma(cf.cx[0][lk], pj[u].x, xv.x);
            xv.y = fma(cf.cx[0][lk], pj[u].y, xv.y);
            S.x[(int64_t(q) * ns + cf.orig[k]) * n + i] = xv;
          }
          if (cf.upd_p[lk]) {
            const double c0 = cf.cp[0][lk];
            double2 np{c0 * pj[u].x, c0 * pj[u].y};
#pragma unroll
            for (int kk = 0; kk < kBatchMaxSteps - 1; ++kk) {
              if (kk < mq) {
                np.x = fma(cf.cp[kk + 1][lk], rk[kk].x, np.x);
                np.y = fma(cf.cp[kk + 1][lk], rk[kk].y, np.y);
              }
            }
            const double cr = cf.cp[mq + 1][lk];
            np.x = fma(cr, rd.x, np.x);
            np.y = fma(cr, rd.y, np.y);
            pkw[pidx] = from_d<W>(np);
          } else if (!same) {
            pkw[pidx] = from_d<W>(pj[u]);
          }
        }
      }
      const double bq = cf.bnew[q];
      pw[idx] = from_d<W>(double2{fma(bq, pd.x, rd.x), fma(bq, pd.y, rd.y)});
    } else if (!std::is_same<R, W>::value) {
      pw[idx] = from_d<W>(pd);
      for (int k = 1; k < ns; ++k) {
        const int64_t pidx = int64_t(k - 1) * n * RR + idx;
        pkw[pidx] = from_d<W>(to_d(pk[pidx]));
      }
    }
    if (!std::is_same<R, W>::value) rw[idx] = from_d<W>(rd);
  }
}

// ---- init: r = p = p_k = b_q, x = 0, |b_q|^2 ----------------------------------------------
template <int RR>
__device__ void binit_chunk(const BatchSys& S, BatchState* st, const int4& ch) {
  const int64_t n = S.n;
  const int ns = st->ns;
  const int64_t rows = ch.z - ch.y;
  double acc[kBatchMaxRhs] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t e = threadIdx.x; e < rows * RR; e += kBlock) {
    const int64_t i = ch.y + e / RR;
    const int q = int(e % RR);
    const int64_t idx = i * RR + q;
    const double2 bv = q < st->nrhs ? S.b[int64_t(q) * n + i] : double2{0.0, 0.0};
    S.r64[idx] = bv;
    S.p64[idx] = bv;
    for (int k = 1; k < ns; ++k) S.pk64[int64_t(k - 1) * n * RR + idx] = bv;
    if (q < st->nrhs)
      for (int k = 0; k < ns; ++k) S.x[(int64_t(q) * ns + k) * n + i] = double2{0.0, 0.0};
#pragma unroll
    for (int qq = 0; qq < kBatchMaxRhs; ++qq)
      if (qq == q) acc[qq] += fma(bv.x, bv.x, bv.y * bv.y);
  }
  __shared__ double tot[kBatchMaxRhs];
  if (!chunk_reduce(acc, S, ch.w, 2, tot)) return;
  if (threadIdx.x < st->nrhs) {
    const int q = threadIdx.x;
    const double B2 = tot[q];
    st->bnorm2[q] = B2;
    st->R[q] = B2;
    st->eps2[q] *= B2;
    st->sw_eps2[q] *= B2;
    if (!(B2 > 0.0) || !isfinite(B2)) {
      st->halt[q] = 1;
      if (!isfinite(B2)) st->status[q] = 1;
    }
  }
}

// ---- reliable update of a system in its complex64 phase: r_q = b_q - (A + s0) x_q0 -------
template <int L, int RR>
__device__ void bru1_chunk(const BatchSys& S, const BatchState* st, const int4& ch) {
  // u = M x_q0 (FP64), stored interleaved in S.u64
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  const int64_t n = S.n;
  for (int64_t row = ch.y + grp; row < ch.z; row += GPB) {
    const int32_t beg = S.m64.rowptr[row], end = S.m64.rowptr[row + 1];
    double2 acc[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) acc[q] = double2{0.0, 0.0};
    for (int32_t j = beg + lane; j < end; j += L) {
      const int32_t c = S.m64.col[j];
      const double2 v = S.m64.val[j];
#pragma unroll
      for (int q = 0; q < RR; ++q)
        if (q < st->nrhs) cfma<double>(acc[q], v, S.x[(int64_t(q) * st->ns + st->orig[0]) * n + c]);
    }
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      acc[q] = group_sum_c<L, double>(acc[q]);
      if (lane == 0) S.u64[row * RR + q] = acc[q];
    }
  }
}

template <int L, int RR>
__device__ void bru2_chunk(const BatchSys& S, BatchState* st, const int4& ch) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  const int64_t n = S.n;
  const bool mhm = S.kind == MSC_A_MHM;
  const double s0 = st->sigma0;
  double acc[kBatchMaxRhs] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t row = ch.y + grp; row < ch.z; row += GPB) {
    const Csr<double2> m2 = mhm ? S.mh64 : S.m64;
    const int32_t beg = m2.rowptr[row], end = m2.rowptr[row + 1];
    double2 qv[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) qv[q] = double2{0.0, 0.0};
    for (int32_t j = beg + lane; j < end; j += L) {
      const int32_t c = m2.col[j];
      const double2 v = m2.val[j];
#pragma unroll
      for (int q = 0; q < RR; ++q) {
        if (q < st->nrhs) {
          const double2 in = mhm ? S.u64[int64_t(c) * RR + q] : S.x[(int64_t(q) * st->ns + st->orig[0]) * n + c];
          cfma<double>(qv[q], v, in);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RR; ++q) {
      qv[q] = group_sum_c<L, double>(qv[q]);
      if (lane == 0 && q < st->nrhs) {
        const double2 bv = S.b[int64_t(q) * n + row];
        const double2 xv = S.x[(int64_t(q) * st->ns + st->orig[0]) * n + row];
        const double2 rt{bv.x - qv[q].x - s0 * xv.x, bv.y - qv[q].y - s0 * xv.y};
        S.r32[row * RR + q] = from_d<float>(rt);
        acc[q] += fma(rt.x, rt.x, rt.y * rt.y);
      }
    }
  }
  __shared__ double tot[kBatchMaxRhs];
  if (!chunk_reduce(acc, S, ch.w, 3, tot)) return;
  if (threadIdx.x < st->nrhs) {
    const int q = threadIdx.x;
    if (!st->halt[q]) {
      st->R[q] = tot[q];
      if (!isfinite(tot[q])) {
        st->status[q] = 1;
        st->halt[q] = 1;
      } else if (tot[q] <= st->eps2[q]) {
        st->halt[q] = 1;
      }
    }
    if (q == 0) st->n_reliable += 1;
  }
}

// ---- persistent drivers over the chunk list ---------------------------------------------
template <int L, int RR>
__global__ __launch_bounds__(kBlock) void bk1(BatchArgs a) {
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    const BatchSys& S = a.sys[ch.x];
    BatchState* st = S.st;
    if (st->done) continue;
    if (st->phase32 || st->switch_pending)
      bk1_chunk<float, L, RR>(S, st, ch);
    else
      bk1_chunk<double, L, RR>(S, st, ch);
  }
}

template <int L, int RR>
__global__ __launch_bounds__(kBlock) void bk2(BatchArgs a) {
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    const BatchSys& S = a.sys[ch.x];
    BatchState* st = S.st;
    if (st->done) continue;
    if (st->phase32)
      bk2_chunk<float, L, RR>(S, st, ch, a.active_systems, a.defer_ok, a.steps);
    else
      bk2_chunk<double, L, RR>(S, st, ch, a.active_systems, a.defer_ok, a.steps);
  }
}

template <int RR>
__global__ __launch_bounds__(kBlock, 4) void bk3(BatchArgs a) {
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    const BatchSys& S = a.sys[ch.x];
    const BatchState* st = S.st;
    if (!st->k3_enable) continue;
    if (st->phase32)
      bk3_chunk<float, float, RR>(S, st, ch);
    else if (st->switch_pending)
      bk3_chunk<double, float, RR>(S, st, ch);
    else
      bk3_chunk<double, double, RR>(S, st, ch);
  }
}

// k3_enable is consumed by bk3 and cleared for finished systems before the next bk1.
__global__ void bk_clear(BatchArgs a) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < a.nsys; s += gridDim.x * blockDim.x) {
    BatchState* st = a.sys[s].st;
    if (st->done) st->k3_enable = 0;
  }
}

template <int RR>
__global__ __launch_bounds__(kBlock) void binit(BatchArgs a) {
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    binit_chunk<RR>(a.sys[ch.x], a.sys[ch.x].st, ch);
  }
}

template <int L, int RR>
__global__ __launch_bounds__(kBlock) void bru1(BatchArgs a) {
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    const BatchSys& S = a.sys[ch.x];
    if (S.st->done || !S.st->phase32) continue;
    bru1_chunk<L, RR>(S, S.st, ch);
  }
}

template <int L, int RR>
__global__ __launch_bounds__(kBlock) void bru2(BatchArgs a) {
  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const int4 ch = a.chunks[c];
    const BatchSys& S = a.sys[ch.x];
    if (S.st->done || !S.st->phase32) continue;
    bru2_chunk<L, RR>(S, S.st, ch);
  }
}

template <int RP>
hipError_t iteration_rr(const BatchArgs& a, hipStream_t s) {
  switch (a.lanes) {
    case 4: bk1<4, RP><<<a.grid, kBlock, 0, s>>>(a); bk2<4, RP><<<a.grid, kBlock, 0, s>>>(a); break;
    case 8: bk1<8, RP><<<a.grid, kBlock, 0, s>>>(a); bk2<8, RP><<<a.grid, kBlock, 0, s>>>(a); break;
    case 16: bk1<16, RP><<<a.grid, kBlock, 0, s>>>(a); bk2<16, RP><<<a.grid, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  bk3<RP><<<a.grid, kBlock, 0, s>>>(a);
  bk_clear<<<1, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

template <int RP>
hipError_t reliable_rr(const BatchArgs& a, hipStream_t s) {
  switch (a.lanes) {
    case 4: bru1<4, RP><<<a.grid, kBlock, 0, s>>>(a); bru2<4, RP><<<a.grid, kBlock, 0, s>>>(a); break;
    case 8: bru1<8, RP><<<a.grid, kBlock, 0, s>>>(a); bru2<8, RP><<<a.grid, kBlock, 0, s>>>(a); break;
    case 16: bru1<16, RP><<<a.grid, kBlock, 0, s>>>(a); bru2<16, RP><<<a.grid, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_init(const BatchArgs& a, hipStream_t s) {
  switch (a.rr) {
    case 1: binit<1><<<a.grid, kBlock, 0, s>>>(a); break;
    case 2: binit<2><<<a.grid, kBlock, 0, s>>>(a); break;
    case 4: binit<4><<<a.grid, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_iteration(const BatchArgs& a, hipStream_t s) {
  switch (a.rr) {
    case 1: return iteration_rr<1>(a, s);
    case 2: return iteration_rr<2>(a, s);
    case 4: return iteration_rr<4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_reliable(const BatchArgs& a, hipStream_t s) {
  switch (a.rr) {
    case 1: return reliable_rr<1>(a, s);
    case 2: return reliable_rr<2>(a, s);
    case 4: return reliable_rr<4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace msc
