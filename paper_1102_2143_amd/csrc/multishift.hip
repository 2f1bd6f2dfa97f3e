// The multishift CG iteration (paper: Section 2, Algorithm 1; Section 3 design rules):
//
//   K1  t = M p                and  P = |t|^2 + sigma0 |p|^2   (A = M^H M)
//       t = A p                and  P = Re(p^H t) + sigma0 |p|^2 (A given)
//   K2  a = R/P and, per shift, zeta^(n+1) and a_j (one lane per shift);
//       r <- r - a (M^H t + sigma0 p)  and  R' = |r|^2
//   K3  b = R'/R, b_j, rotation of zeta, freezing, halting;  x_0 += a p;  for every
//       active shift j: x_j += a_j p_j, p_j <- zeta_j r + b_j p_j;  p <- r + b p  -- one
//       pass over r and p serves all shifts (Section 3: the shifted updates are the next
//       most expensive step; register reuse of r and p).
//
// On the sliced ELLPACK path an iteration is two kernels: the head (K3 of the previous
// iteration, then K1 on the new direction, formed at each gathered column) and K2.
// A head may defer the shifted part of K3; a later one applies up to four composed steps
// in one pass over x_j and p_j.
//
// The shift recurrences are the values forced by the collinearity r_j = zeta_j r:
//   zeta' = zeta zeta_prev a_prev / (a b (zeta_prev - zeta) + zeta_prev a_prev (1 + s a)),
//   a_j = a zeta'/zeta,  b_j = b' (zeta'/zeta)^2,  with s = sigma_j - sigma0 >= 0.
// All scalar work stays on the device in FP64 (Section 3: the iteration constants are
// computed on the GPU to avoid host round trips).  Reductions are deterministic: each
// workgroup writes one partial, and every workgroup of the consuming kernel sums them in
// one fixed order (set-up, reliable update and verification: the last workgroup to
// arrive does).
#include <hip/hip_ext.h>

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "dev_common.h"
#include "msc_internal.h"
#include "sell_load.h"
#include "stencil.h"

namespace msc {

namespace {

template <class R> __device__ __forceinline__ Csr<cplx<R>> pick_m(const MsArgs& a);
template <> __device__ __forceinline__ Csr<float2> pick_m<float>(const MsArgs& a) { return a.m32; }
template <> __device__ __forceinline__ Csr<double2> pick_m<double>(const MsArgs& a) { return a.m64; }
template <class R> __device__ __forceinline__ Csr<cplx<R>> pick_mh(const MsArgs& a);
template <> __device__ __forceinline__ Csr<float2> pick_mh<float>(const MsArgs& a) { return a.mh32; }
template <> __device__ __forceinline__ Csr<double2> pick_mh<double>(const MsArgs& a) { return a.mh64; }

template <class R> __device__ __forceinline__ Sell<cplx<R>> pick_sm(const MsArgs& a);
template <> __device__ __forceinline__ Sell<float2> pick_sm<float>(const MsArgs& a) { return a.s32; }
template <> __device__ __forceinline__ Sell<double2> pick_sm<double>(const MsArgs& a) { return a.s64; }
template <class R> __device__ __forceinline__ Stencil<cplx<R>> pick_w(const MsArgs& a);
template <> __device__ __forceinline__ Stencil<float2> pick_w<float>(const MsArgs& a) { return a.w32; }
template <> __device__ __forceinline__ Stencil<double2> pick_w<double>(const MsArgs& a) { return a.w64; }
template <class R> __device__ __forceinline__ Sell<cplx<R>> pick_shm(const MsArgs& a);
template <> __device__ __forceinline__ Sell<float2> pick_shm<float>(const MsArgs& a) { return a.sh32; }
template <> __device__ __forceinline__ Sell<double2> pick_shm<double>(const MsArgs& a) { return a.sh64; }

// Tuning knobs of the sliced ELLPACK SpMV (defaults measured best on MI355X):
//   MSC_SELL_KP32 / MSC_SELL_KP64: pairs per round trip for complex64 / complex128.
#ifndef MSC_SELL_KP32
#define MSC_SELL_KP32 12
#endif
#ifndef MSC_SELL_KP64
#define MSC_SELL_KP64 6
#endif

// Pairs per round trip of the sliced ELLPACK row product (register budget: complex64
// keeps a 24-entry staggered row in flight at once, complex128 half of it).
// Slot k of the residual ring (slot 0: a.r, slot k >= 1: a.rkeep[k - 1]); k is uniform.
template <class R>
__device__ __forceinline__ cplx<R>* rslot(const MsArgs& a, int k) {
  void* q = a.r;
#pragma unroll
  for (int j = 1; j < kMaxSteps; ++j)
    if (k == j) q = a.rkeep[j - 1];
  return static_cast<cplx<R>*>(q);
}

template <class R> constexpr int sell_kp();
template <> constexpr int sell_kp<float>() { return MSC_SELL_KP32; }
template <> constexpr int sell_kp<double>() { return MSC_SELL_KP64; }

template <class R, int KP, bool FULL>
__device__ __forceinline__ void sell_gather_fma(const cplx<R>* __restrict__ x, int np,
                                                const int2 (&cc)[KP], const cplx<R> (&v)[2 * KP],
                                                cplx<R>& acc) {
  cplx<R> xv[2 * KP];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    if (FULL || u < np) {
      xv[2 * u] = x[cc[u].x];
      xv[2 * u + 1] = x[cc[u].y];
    } else {
      xv[2 * u] = xv[2 * u + 1] = czero<R>();
    }
  }
#pragma unroll
  for (int u = 0; u < 2 * KP; ++u) cfma<R>(acc, v[u], xv[u]);
}

// Off-diagonal part of the product of one sliced ELLPACK row per lane with x; slice `sl`
// is wavefront-uniform.  Pairs go KP at a time: a chunk's column and value loads, then
// its gathers, are all issued before its first multiply-add.
template <class R, bool NARROW>
__device__ __forceinline__ cplx<R> sell_row_cols(const Sell<cplx<R>>& m,
                                                 const cplx<R>* __restrict__ x, int64_t sl,
                                                 int lane) {
  constexpr int KP = sell_kp<R>();
  int32_t c, c1;
  if (m.wp > 0) {
    c = int32_t(sl) * m.wp;
    c1 = c + m.wp;
  } else {
    c = load_uniform(m.cptr, sl);
    c1 = load_uniform(m.cptr, sl + 1);
  }
  cplx<R> acc = czero<R>();
  int2 cc[KP];
  cplx<R> v[2 * KP];
  for (; c + KP <= c1; c += KP) {
    sell_load<R, KP, true, NARROW>(m, c, KP, lane, cc, v);
    sell_gather_fma<R, KP, true>(x, KP, cc, v, acc);
  }
  if (c < c1) {
    const int np = c1 - c;
    sell_load<R, KP, false, NARROW>(m, c, np, lane, cc, v);
    sell_gather_fma<R, KP, false>(x, np, cc, v, acc);
  }
  return acc;
}
template <class R>
__device__ __forceinline__ cplx<R> sell_row(const Sell<cplx<R>>& m, const cplx<R>* __restrict__ x,
                                            int64_t sl, int lane) {
  return m.col16 ? sell_row_cols<R, true>(m, x, sl, lane) : sell_row_cols<R, false>(m, x, sl, lane);
}

// The next direction r + b p, formed in FP64 and rounded once; a lane that gathers p'
// at a neighbouring row forms the same bits as the row's owner stores.
template <class R>
__device__ __forceinline__ cplx<R> next_dir(double b, const cplx<R>& r, const cplx<R>& p) {
  const double2 rd = to_d(r), pd = to_d(p);
  double2 v;
  v.x = fma(b, pd.x, rd.x);
  v.y = fma(b, pd.y, rd.y);
  return from_d<R>(v);
}

// Minimum waves per SIMD asked of the compiler for the matrix-free head and K2 (1: no
// constraint).  The FP64 heads need the bound and a scheduling barrier between their
// update and stencil parts (MSC_SITE_SB): without them the compiler interleaves the two
// into 256 VGPRs, one wave per SIMD.
#ifndef MSC_SITE_HEAD_WPE
#define MSC_SITE_HEAD_WPE 2
#endif
#ifndef MSC_SITE_K2_WPE
#define MSC_SITE_K2_WPE 1
#endif
#ifndef MSC_SITE_SB
#define MSC_SITE_SB 1
#endif
// Dynamic LDS of the complex64 site K2 (bytes per workgroup, within the 64 KB a
// workgroup may hold): three workgroups fit a CU's 160 KB, four do not.
constexpr size_t kC64K2Lds = size_t(48) << 10;
// most t-slices per column of K2's march along t
#ifndef MSC_K2_MARCH
#define MSC_K2_MARCH 16
#endif
constexpr int kK2March = MSC_K2_MARCH;
#ifndef MSC_HEAD_MARCH
#define MSC_HEAD_MARCH 1
#endif
constexpr bool kHeadMarch = MSC_HEAD_MARCH != 0;
// waves per SIMD the marching K2 is compiled for (FP64, complex64)
#ifndef MSC_K2_MARCH_WPE64
#define MSC_K2_MARCH_WPE64 2
#endif
#ifndef MSC_K2_MARCH_WPE32
#define MSC_K2_MARCH_WPE32 2
#endif

// Pairs per round trip when each entry gathers two vectors (MSC_SELL_KPN32 / 64).
#ifndef MSC_SELL_KPN32
#define MSC_SELL_KPN32 4
#endif
#ifndef MSC_SELL_KPN64
#define MSC_SELL_KPN64 2
#endif
template <class R> constexpr int sell_kp_next();
template <> constexpr int sell_kp_next<float>() { return MSC_SELL_KPN32; }
template <> constexpr int sell_kp_next<double>() { return MSC_SELL_KPN64; }

template <class R, int KP, bool FULL>
__device__ __forceinline__ void sell_gather2_fma(const cplx<R>* __restrict__ r,
                                                 const cplx<R>* __restrict__ p, double b, int np,
                                                 const int2 (&cc)[KP], const cplx<R> (&v)[2 * KP],
                                                 cplx<R>& acc) {
  cplx<R> xr[2 * KP], xp[2 * KP];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    if (FULL || u < np) {
      xr[2 * u] = r[cc[u].x];
      xp[2 * u] = p[cc[u].x];
      xr[2 * u + 1] = r[cc[u].y];
      xp[2 * u + 1] = p[cc[u].y];
    } else {
      xr[2 * u] = xr[2 * u + 1] = xp[2 * u] = xp[2 * u + 1] = czero<R>();
    }
  }
#pragma unroll
  for (int u = 0; u < 2 * KP; ++u) cfma<R>(acc, v[u], next_dir<R>(b, xr[u], xp[u]));
}

// Off-diagonal part of one sliced ELLPACK row per lane times p' = r + b p, with p' formed
// at each gathered column.
template <class R, bool NARROW>
__device__ __forceinline__ cplx<R> sell_row_next_cols(const Sell<cplx<R>>& m,
                                                      const cplx<R>* __restrict__ r,
                                                      const cplx<R>* __restrict__ p, double b,
                                                      int64_t sl, int lane) {
  constexpr int KP = sell_kp_next<R>();
  int32_t c, c1;
  if (m.wp > 0) {
    c = int32_t(sl) * m.wp;
    c1 = c + m.wp;
  } else {
    c = load_uniform(m.cptr, sl);
    c1 = load_uniform(m.cptr, sl + 1);
  }
  cplx<R> acc = czero<R>();
  int2 cc[KP];
  cplx<R> v[2 * KP];
  for (; c + KP <= c1; c += KP) {
    sell_load<R, KP, true, NARROW>(m, c, KP, lane, cc, v);
    sell_gather2_fma<R, KP, true>(r, p, b, KP, cc, v, acc);
  }
  if (c < c1) {
    const int np = c1 - c;
    sell_load<R, KP, false, NARROW>(m, c, np, lane, cc, v);
    sell_gather2_fma<R, KP, false>(r, p, b, np, cc, v, acc);
  }
  return acc;
}
template <class R>
__device__ __forceinline__ cplx<R> sell_row_next(const Sell<cplx<R>>& m,
                                                 const cplx<R>* __restrict__ r,
                                                 const cplx<R>* __restrict__ p, double b,
                                                 int64_t sl, int lane) {
  return m.col16 ? sell_row_next_cols<R, true>(m, r, p, b, sl, lane)
                 : sell_row_next_cols<R, false>(m, r, p, b, sl, lane);
}

// One CSR row times a vector, L lanes per row; the sum is returned in every lane.
// Entries of one row handled by a lane per chunk: the column and value loads of a chunk,
// then its gathers, are all issued before the first multiply-add, so a row of up to
// kChunk * L entries costs one round trip for the matrix and one for the gather.
constexpr int kChunk = 4;

template <class R, int L>
__device__ __forceinline__ cplx<R> row_dot(const Csr<cplx<R>>& m, const cplx<R>* __restrict__ x,
                                           int64_t row, int lane) {
  const int32_t beg = m.rowptr[row], end = m.rowptr[row + 1];
  cplx<R> acc = czero<R>();
  for (int32_t base = beg; base < end; base += kChunk * L) {
    int32_t c[kChunk];
    cplx<R> v[kChunk], xv[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int32_t j = base + lane + u * L;
      const bool ok = j < end;
      c[u] = ok ? m.col[j] : 0;
      v[u] = ok ? m.val[j] : czero<R>();
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) cfma<R>(acc, v[u], xv[u]);
  }
  return group_sum_c<L, R>(acc);
}

// Two rows per row group at a time: both rows' loads share one round trip.  An empty
// second row (beg1 == end1) contributes zero.
template <class R, int L>
__device__ __forceinline__ void row_dot2(const Csr<cplx<R>>& m, const cplx<R>* __restrict__ x,
                                         int64_t row0, int64_t row1, bool has1, int lane,
                                         cplx<R>& out0, cplx<R>& out1) {
  const int32_t b0 = m.rowptr[row0], e0 = m.rowptr[row0 + 1];
  const int32_t b1 = has1 ? m.rowptr[row1] : 0, e1 = has1 ? m.rowptr[row1 + 1] : 0;
  const int32_t len = (e0 - b0) > (e1 - b1) ? (e0 - b0) : (e1 - b1);
  cplx<R> a0 = czero<R>(), a1 = czero<R>();
  for (int32_t base = 0; base < len; base += kChunk * L) {
    int32_t c0[kChunk], c1[kChunk];
    cplx<R> v0[kChunk], v1[kChunk], x0[kChunk], x1[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int32_t j0 = b0 + base + lane + u * L, j1 = b1 + base + lane + u * L;
      const bool ok0 = j0 < e0, ok1 = j1 < e1;
      c0[u] = ok0 ? m.col[j0] : 0;
      v0[u] = ok0 ? m.val[j0] : czero<R>();
      c1[u] = ok1 ? m.col[j1] : 0;
      v1[u] = ok1 ? m.val[j1] : czero<R>();
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      x0[u] = x[c0[u]];
      x1[u] = x[c1[u]];
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      cfma<R>(a0, v0[u], x0[u]);
      cfma<R>(a1, v1[u], x1[u]);
    }
  }
  out0 = group_sum_c<L, R>(a0);
  out1 = group_sum_c<L, R>(a1);
}

// The last workgroup sums `count` (<= kMaxGrid) partials (stride `stride`, offset `k`)
// in a fixed order; all loads are in flight together.  The result is valid in thread 0.
__device__ __forceinline__ double sum_partials(const double* partial, int count, int stride, int k) {
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

// ---- the iteration's reductions ------------------------------------------------------
// K1 stores one partial of P per workgroup in region 0, K2 one partial of R' in region 1;
// the workgroups of the next kernel each add all of them up in the same order.
__device__ __forceinline__ double* region(const MsArgs& a, int k) {
  return a.sc.partial + k * kMaxGrid;
}

__device__ __forceinline__ void store_partial(double* reg, double acc) {
  const double tot = block_sum<kBlock>(acc);
  if (threadIdx.x == 0) store_agent(&reg[blockIdx.x], tot);
}

// Partials are loaded early (four per thread, covering grids of up to 1024 workgroups)
// so their round trip overlaps the caller's own first loads; the sum is identical in
// every thread of every workgroup that forms it.
constexpr int kEarly = 4;
struct Early {
  double v[kEarly];
};

__device__ __forceinline__ void load_early(const double* reg, int count, Early& e) {
#pragma unroll
  for (int u = 0; u < kEarly; ++u) {
    const int i = threadIdx.x + u * kBlock;
    e.v[u] = i < count ? load_agent(&reg[i]) : 0.0;
  }
}

__device__ __forceinline__ double all_sum(const double* reg, int count, const Early& e) {
  __shared__ double total;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kEarly; ++u) s += e.v[u];
  for (int i = threadIdx.x + kEarly * kBlock; i < count; i += kBlock) s += load_agent(&reg[i]);
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) total = s;
  __syncthreads();
  return total;
}

// K2 prologue: a = R / P.  Workgroup 0 also stores a, P and, for every active shift j
// (wave 0, lane j), zeta_j^(n+1) = zeta zeta_- a_- / (a b (zeta_- - zeta) + zeta_- a_-
// (1 + s_j a)) and a_j = a zeta_j^(n+1) / zeta_j for the next head, and marks the update
// pending; a breakdown (P <= 0 or not finite) is flagged instead.  Returns false on
// breakdown.  The iteration's state is the one its head wrote, rot[par ^ 1].
__device__ bool k2_step(const MsArgs& a, const Early& e, double& step) {
  SolveState* st = a.st;
  RotState& rs = st->rot[a.par ^ 1];
  const int j = threadIdx.x;
  const bool lead = blockIdx.x == 0 && j < kWave;
  // workgroup 0, lane j: shift j's state, loaded before the partial sum
  double z = 1.0, zp = 1.0, sj = 0.0;
  int act = 0;
  if (lead && j >= 1 && j < st->ns) {
    act = rs.active[j];
    z = rs.zeta[j];
    zp = st->zeta_prev[j];
    sj = st->s[j];
  }
  const double ap = st->a_prev, b = st->b, R = rs.R;
  const double P = all_sum(region(a, 0), a.gk1, e);
  const bool ok = (P > 0.0) && isfinite(P);
  step = ok ? R / P : 0.0;
  if (lead) {
    if (j == 0) rs.pending = 1;
    if (!ok) {
      if (j == 0) {
        st->P = P;
        st->kstatus = 1;
      }
    } else {
      if (act) {
        const double zn = z * zp * ap / (step * b * (zp - z) + zp * ap * (1.0 + sj * step));
        st->zk[j] = zn;
        st->ak[j] = step * zn / z;
      }
      if (j == 0) {
        st->P = P;
        st->a = step;
      }
    }
  }
  return ok;
}

// Head prologue, shared through LDS.  When the previous K2 left its update pending:
// R' (from K2's partials) and b = R'/R, and per shift j the coefficients of its update,
// whether it freezes now (zeta_j^(n+1)^2 R' <= eps2), and the list of shifts to update.
// Workgroup 0 writes the state the rest of the iteration and the next head start from.
// Shifts whose x_j and p_j loads the head's update issues together (MSC_UPD_GROUP).
#ifndef MSC_UPD_GROUP
#define MSC_UPD_GROUP 4
#endif
constexpr int kUpdGroup = MSC_UPD_GROUP;

struct Plan {
  double bn;                 // b of p <- r + b p (0: p is current, nothing pending)
  // the shifts this head updates, in list order, with the element offsets of x_j (the
  // caller's order) and of p_j:  x_j += cx[0] p_j + sum_{k<m} cx[k+1] r_k  and, where pw,
  // p_j <- cp[0] p_j + sum_{k<m} cp[k+1] r_k + cp[m+1] r  (r_k: the residuals kept by the
  // m heads that deferred; r: the current one; unused coefficients are 0)
  double cx[kMaxSteps][kMaxShifts];
  double cp[kMaxSteps + 1][kMaxShifts];
  int64_t xo[kMaxShifts];
  int64_t po[kMaxShifts];
  int pw[kMaxShifts];
  // the driving system in the same form (zeta = 1): x_0 += x0c[0] p_1 + sum_{k<m}
  // x0c[k+1] r_k, p_1 the direction at the first pending step (the current p when m = 0,
  // else the one the first deferring head kept)
  double x0c[kMaxSteps];
  int keep0;                 // 1: this deferring head keeps p for x_0 (first of a cycle)
  int nact;
  int mode;                  // 0: apply (the current step and m deferred ones); 1: defer
  int m;                     // kept residuals read (mode 0)
  int pending;               // the update runs in this head
  int ok;                    // 0: breakdown, the head stops
  int spmv;                  // 1: this head also computes t = M p
};

// Consecutive steps of shift j compose: with p_j = cp[0] p + sum_k cp[k+1] r_k after the
// deferred ones, the next step adds a_j p_j to x_j and turns p_j into
// zeta_j' r + b_j p_j (r: that step's residual), unless j freezes there (p_j stays); a
// frozen shift takes no further step.  The driving system (lane 0) composes the same way
// with zeta = 1, a_0 = a and b_0 = b: its x is x_0, its direction p.  A head defers (its r
// stays in its ring slot; it touches no x_j, p_j and not x_0) while fewer than `steps` - 1
// steps are pending,
// its iteration continues and no reliable update (which reads x_0) runs after it;
// otherwise it applies all of them in one pass.
template <class T>
__device__ void head_plan(const MsArgs& a, const Early& e, Plan& pl) {
  constexpr int ph = sizeof(T) == 4 ? 1 : 0;  // phase: 0 FP64, 1 complex64
  SolveState* st = a.st;
  const RotState& rs = st->rot[a.par];
  RotState& nx = st->rot[a.par ^ 1];
  const int j = threadIdx.x;
  const int pending = rs.pending;
  const int m = rs.ndef;
  // wave 0, lane j: shift j's state, loaded before the partial sum
  int act0 = 0, origj = 0, dact = 0, dupd = 0;
  double z = 1.0, zn = 0.0, akj = 0.0;
  double cx[kMaxSteps + 1], cp[kMaxSteps + 1];
#pragma unroll
  for (int i = 0; i <= kMaxSteps; ++i) cx[i] = cp[i] = 0.0;
  cp[0] = 1.0;
  const bool drv = j == 0;  // lane 0: the driving system
  if (j < kWave && j < st->ns) {
    if (pending) {
      act0 = drv ? 1 : rs.active[j];
      z = drv ? 1.0 : rs.zeta[j];
      zn = drv ? 1.0 : st->zk[j];
      akj = drv ? st->a : st->ak[j];
    }
    if (!drv && (pending || m > 0)) origj = st->orig[j];
    if (m > 0) {
      const DeferState& d = st->dfs[a.par];
#pragma unroll
      for (int i = 0; i < kMaxSteps; ++i) {
        if (i <= m) {
          cx[i] = d.cx[i][j];
          cp[i] = d.cp[i][j];
        }
      }
      dact = d.act[j];
      dupd = d.upd[j];
    }
  }
  const double R = rs.R, eps2 = st->eps2;
  const int kst = st->kstatus, frz = st->freeze;
  const double Rn = pending ? all_sum(region(a, 1), a.gk2, e) : R;
  if (j < kWave) {
    const bool ok = !pending || (isfinite(Rn) && kst == 0);
    const double bn = pending ? Rn / R : 0.0;
    const bool act = pending && ok && act0;
    const bool freeze_now = act && !drv && frz && zn * zn * Rn <= eps2;
    const double ratio = act ? zn / z : 0.0;
    const double bk = bn * ratio * ratio;
    const int it = pending ? rs.iter + 1 : rs.iter;
    const bool done = pending && (Rn <= eps2 || it >= st->max_iter);
    // the FP64 phase of a mixed solve ends here: the update still runs, then the host
    // converts the Krylov vectors to complex64 and continues
    const bool sw = pending && !done && Rn <= st->sw_eps2;
    const bool cont = ok && !done && !sw;
    // fold the current step into the composition
    if (act) {
#pragma unroll
      for (int i = 0; i < kMaxSteps; ++i)
        if (i <= m) cx[i] = fma(akj, cp[i], cx[i]);
    }
    if (act && !freeze_now) {
#pragma unroll
      for (int i = 0; i < kMaxSteps; ++i)
        if (i <= m) cp[i] *= bk;
#pragma unroll
      for (int i = 1; i <= kMaxSteps; ++i)
        if (i == m + 1) cp[i] = zn;
    }
    dact = dact || act;
    dupd = dupd || (act && !freeze_now);
    // a reliable update after this head reads x_0: the same test as ru_due on the R this
    // head writes
    const bool ru_now = a.ru_check && (a.ru_force || Rn < kRuDelta2 * st->R_ru);
    const int mode = (pending && cont && a.defer_ok && m + 1 < a.steps && !ru_now) ? 1 : 0;
    const bool listed = mode == 0 && dact && !drv;
    const uint64_t mask = __ballot(listed);
    if (listed) {
      const int pos = __popcll(mask & ((uint64_t(1) << j) - 1));
#pragma unroll
      for (int i = 0; i < kMaxSteps; ++i) pl.cx[i][pos] = i <= m ? cx[i] : 0.0;
#pragma unroll
      for (int i = 0; i <= kMaxSteps; ++i) pl.cp[i][pos] = i <= m + 1 ? cp[i] : 0.0;
      pl.xo[pos] = int64_t(origj) * a.n;
      pl.po[pos] = int64_t(j - 1) * a.n;
      pl.pw[pos] = dupd ? 1 : 0;
    }
    const int nlist = __popcll(mask);
    if (drv) {
#pragma unroll
      for (int i = 0; i < kMaxSteps; ++i) pl.x0c[i] = (mode == 0 && i <= m) ? cx[i] : 0.0;
      pl.keep0 = (mode == 1 && m == 0) ? 1 : 0;
      pl.bn = bn;
      pl.nact = nlist;
      pl.mode = mode;
      pl.m = mode == 0 ? m : 0;
      pl.pending = pending;
      pl.ok = ok ? 1 : 0;
      pl.spmv = cont ? 1 : 0;
    }
    if (blockIdx.x == 0) {
      if (j < st->ns) {
        if (!drv) {
          nx.zeta[j] = act ? zn : rs.zeta[j];
          nx.active[j] = act ? (freeze_now ? 0 : 1) : rs.active[j];
        } else {
          nx.zeta[0] = rs.zeta[0];
          nx.active[0] = rs.active[0];
        }
        if (mode == 1) {
          DeferState& d = st->dfs[a.par ^ 1];
#pragma unroll
          for (int i = 0; i < kMaxSteps; ++i) {
            d.cx[i][j] = i <= m ? cx[i] : 0.0;
            d.cp[i][j] = i <= m + 1 ? cp[i] : 0.0;
          }
          d.act[j] = dact ? 1 : 0;
          d.upd[j] = dupd ? 1 : 0;
        }
      }
      if (act && !drv) {
        st->zeta_prev[j] = z;
        if (freeze_now) st->freeze_iter[j] = it;
      }
      if (drv) {
        nx.pending = 0;
        nx.ndef = (ok && mode == 1) ? m + 1 : 0;
        if (a.sample >= 0 && a.sample < kMaxSamples) {
          st->smp_mode[a.sample] = mode;
          st->smp_nact[a.sample] = nlist;
          st->smp_m[a.sample] = m;
        }
        if (pending && ok) {
          st->n_shift_upd[ph] += nlist;
          st->n_defer[ph] += mode == 1 ? 1 : 0;
          st->n_two[ph] += mode == 0 ? m : 0;
          st->n_apply[ph] += mode == 0 ? 1 : 0;
          st->n_keep0[ph] += (mode == 1 && m == 0) ? 1 : 0;
        }
        if (!ok) {
          nx.R = R;
          nx.iter = rs.iter;
          nx.halt = 1;
          nx.switch_req = 0;
          nx.status = 1;
          nx.pcur = rs.pcur;
          store_host_flag(a.hflag, 1);
        } else {
          nx.R = Rn;
          nx.iter = it;
          nx.status = 0;
          nx.halt = (done || sw) ? 1 : 0;
          if (done || sw) st->rslot = m;  // no K2 follows: r stays in this head's slot
          nx.switch_req = sw ? 1 : 0;
          nx.pcur = pending ? rs.pcur ^ 1 : rs.pcur;
          store_host_flag(a.hflag, ((done || sw) ? 1 : 0) | (sw ? 2 : 0));
          if (pending) {
            st->b = bn;
            st->a_prev = st->a;
          }
        }
      }
    }
  }
  __syncthreads();
}

// A halted iteration carries its state over to the next one (head, workgroup 0).
__device__ void carry_state(const MsArgs& a) {
  if (blockIdx.x != 0) return;
  SolveState* st = a.st;
  const RotState& rs = st->rot[a.par];
  RotState& nx = st->rot[a.par ^ 1];
  const int j = threadIdx.x;
  if (j < kMaxShifts) {
    nx.zeta[j] = rs.zeta[j];
    nx.active[j] = rs.active[j];
  }
  if (j == 0) {
    nx.R = rs.R;
    nx.iter = rs.iter;
    nx.halt = 1;
    nx.switch_req = rs.switch_req;
    nx.status = rs.status;
    nx.pending = rs.pending;
    nx.pcur = rs.pcur;
    nx.ndef = rs.ndef;
    store_host_flag(a.hflag, 1 | (rs.switch_req ? 2 : 0));
  }
}

// The pending update of row i: the listed shifts' x_j and p_j and x_0 as the plan
// composes them (the current step and the m deferred ones, reading the residuals of the
// m deferring heads from ring slots 0..m-1; a deferring head touches neither x_0 nor any
// shift, and the first of a cycle keeps p), then the new direction r + b p, which is
// stored in the other direction buffer and returned.  rr, pp: the row's r and p (already
// loaded).
template <class R>
__device__ __forceinline__ cplx<R> update_row(const MsArgs& a, const Plan& pl, int64_t i,
                                              const cplx<R>& rr, const cplx<R>& pp,
                                              double2* __restrict__ x0,
                                              cplx<R>* __restrict__ pnew) {
  cplx<R>* __restrict__ pk = static_cast<cplx<R>*>(a.pk);
  cplx<R>* __restrict__ pkeep0 = static_cast<cplx<R>*>(a.pkeep0);
  double2* __restrict__ x = a.x;
  const double2 rd = to_d(rr), pd = to_d(pp);
  if (pl.keep0) st_stream(&pkeep0[i], pp);
  // the residuals of the m heads that deferred, in ring slots 0..m-1 (zero beyond m,
  // where the coefficients are zero too)
  double2 rk[kMaxSteps - 1];
#pragma unroll
  for (int k = 0; k < kMaxSteps - 1; ++k)
    rk[k] = k < pl.m ? to_d(ld_stream(&rslot<R>(a, k)[i])) : double2{0.0, 0.0};
  const int m = pl.m;
  if (pl.mode == 0) {
    // x_0: with one step (m = 0) the fused multiply-add rounds exactly as x_0 += a p
    double2 xv = ld_stream(&x0[i]);
    const double2 p1 = m > 0 ? to_d(ld_stream(&pkeep0[i])) : pd;
#pragma unroll
    for (int k = kMaxSteps - 2; k >= 0; --k) {
      if (k < m) {
        xv.x = fma(pl.x0c[k + 1], rk[k].x, xv.x);
        xv.y = fma(pl.x0c[k + 1], rk[k].y, xv.y);
      }
    }
    xv.x = fma(pl.x0c[0], p1.x, xv.x);
    xv.y = fma(pl.x0c[0], p1.y, xv.y);
    st_stream(&x0[i], xv);
  }
  // shifts in groups of MSC_UPD_GROUP: a group's loads are all issued before its first
  // store; a last, partial group is masked.  With one step (m = 0) the fused
  // multiply-adds round exactly as x += a p and p <- zeta r + b p.
  const int nact = pl.nact;
  auto group = [&](int q, int cnt, auto full) {
    cplx<R> pj[kUpdGroup];
    double2 xj[kUpdGroup];
#pragma unroll
    for (int u = 0; u < kUpdGroup; ++u) {
      if (decltype(full)::value || u < cnt) {
        pj[u] = ld_stream(&pk[pl.po[q + u] + i]);
        xj[u] = ld_stream(&x[pl.xo[q + u] + i]);
      }
    }
#pragma unroll
    for (int u = 0; u < kUpdGroup; ++u) {
      if (decltype(full)::value || u < cnt) {
        const int c = q + u;
        const double2 pjd = to_d(pj[u]);
        double2 xv = xj[u];
#pragma unroll
        for (int k = kMaxSteps - 2; k >= 0; --k) {
          if (k < m) {
            xv.x = fma(pl.cx[k + 1][c], rk[k].x, xv.x);
            xv.y = fma(pl.cx[k + 1][c], rk[k].y, xv.y);
          }
        }
        xv.x = fma(pl.cx[0][c], pjd.x, xv.x);
        xv.y = fma(pl.cx[0][c], pjd.y, xv.y);
        st_stream(&x[pl.xo[c] + i], xv);
        if (pl.pw[c]) {
          const double c0 = pl.cp[0][c];
          double2 np{c0 * pjd.x, c0 * pjd.y};
#pragma unroll
          for (int k = 0; k < kMaxSteps - 1; ++k) {
            if (k < m) {
              np.x = fma(pl.cp[k + 1][c], rk[k].x, np.x);
              np.y = fma(pl.cp[k + 1][c], rk[k].y, np.y);
            }
          }
          const double cr = pl.cp[m + 1][c];
          np.x = fma(cr, rd.x, np.x);
          np.y = fma(cr, rd.y, np.y);
          st_stream(&pk[pl.po[c] + i], from_d<R>(np));
        }
      }
    }
  };
  int q = 0;
  for (; q + kUpdGroup <= nact; q += kUpdGroup) group(q, kUpdGroup, std::true_type{});
  if (q < nact) group(q, nact - q, std::false_type{});
  const cplx<R> np = next_dir<R>(pl.bn, rr, pp);
  st_stream(&pnew[i], np);
  return np;
}

// ---- head on the CSR path: the pending update only (K1 follows as its own kernel) -----
template <class R>
__global__ __launch_bounds__(kBlock) void k_update(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& rs = st->rot[a.par];
  if (rs.halt) {
    carry_state(a);
    return;
  }
  Early e;
  if (rs.pending) load_early(region(a, 1), a.gk2, e);
  const int pc = rs.pcur;
  const int64_t n = a.n;
  const cplx<R>* __restrict__ rv = rslot<R>(a, rs.ndef);
  const cplx<R>* __restrict__ pv = static_cast<const cplx<R>*>(a.pb[pc]);
  cplx<R>* __restrict__ pnew = static_cast<cplx<R>*>(a.pb[pc ^ 1]);
  double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * n;
  int64_t beg, end;
  block_range(n, kBlock, beg, end);
  // this thread's first row is read while R' is being summed
  const int64_t i0 = beg + threadIdx.x;
  const int64_t ic = i0 < end ? i0 : n - 1;
  const cplx<R> r_first = rv[ic], p_first = pv[ic];
  __shared__ Plan pl;
  head_plan<R>(a, e, pl);
  if (!pl.ok || !pl.pending) return;
  for (int64_t i = i0; i < end; i += kBlock) {
    const bool first = i == i0;
    update_row<R>(a, pl, i, first ? r_first : rv[i], first ? p_first : pv[i], x0, pnew);
  }
}

// ---- head on the sliced ELLPACK path: pending update fused with K1 -------------------
// One row per lane, one slice per wave.  With an update pending, the lane first updates
// its own row (x, p_j, and p' = r + b p stored in the other buffer), then t = M p' takes
// p' at the gathered columns from r and the old p, rounded exactly as the owning lane
// rounds it; P = |t|^2 + sigma0 |p'|^2 (A = M^H M) or Re p'^H t + sigma0 |p'|^2.
template <class R, bool MHM>
__global__ __launch_bounds__(kBlock) void k1_fused(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& rs = st->rot[a.par];
  if (rs.halt) {
    carry_state(a);
    return;
  }
  const int pending = rs.pending;
  Early e;
  if (pending) load_early(region(a, 1), a.gk2, e);
  const int pc = rs.pcur;
  const Sell<cplx<R>> m = pick_sm<R>(a);
  const cplx<R>* __restrict__ rv = rslot<R>(a, rs.ndef);
  const cplx<R>* __restrict__ pv = static_cast<const cplx<R>*>(a.pb[pc]);
  cplx<R>* __restrict__ pnew = static_cast<cplx<R>*>(a.pb[pc ^ 1]);
  cplx<R>* __restrict__ t = static_cast<cplx<R>*>(a.t);
  double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  const double sigma0 = st->sigma0;
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  Sweep sw = make_sweep(a.nslices, a.ord, SPB);
  // the first slice's own row is read while R' is being summed
  const bool has0 = sw.more();
  const int64_t sl0 = has0 ? sw.slice() : 0;
  const int64_t row0 = sl0 * kSlice + lane;
  const int64_t rc = (has0 && row0 < a.n) ? row0 : a.n - 1;
  const cplx<R> r_first = rv[rc], p_first = pv[rc];
  __shared__ Plan pl;
  head_plan<R>(a, e, pl);
  if (!pl.ok) return;
  const bool upd = pl.pending != 0;
  const double bn = pl.bn;
  double acc = 0.0;
  for (bool first = true; sw.more(); sw.next(), first = false) {
    const int64_t sl = first ? sl0 : sw.slice();
    const int64_t row = sl * kSlice + lane;
    const bool live = row < a.n;
    const int64_t rr = live ? row : a.n - 1;  // lanes past n read a valid row, unused
    const cplx<R> r_i = first ? r_first : rv[rr];
    const cplx<R> p_i = first ? p_first : pv[rr];
    cplx<R> p_row = p_i;
    if (upd) {
      if (live)
        p_row = update_row<R>(a, pl, row, r_i, p_i, x0, pnew);
      else
        p_row = next_dir<R>(bn, r_i, p_i);
    }
    if (!pl.spmv) continue;
    // without a pending update p' = p: the same product with r := p and b = 0 (exact)
    const cplx<R> d = m.diag[rr];
    cplx<R> v = sell_row_next<R>(m, upd ? rv : pv, pv, bn, sl, lane);
    cfma<R>(v, d, p_row);
    if (live) {
      st_stream(&t[row], v);
      if (MHM)
        acc += norm2d<R>(v) + sigma0 * norm2d<R>(p_row);
      else
        acc += double(p_row.x) * double(v.x) + double(p_row.y) * double(v.y) +
               sigma0 * norm2d<R>(p_row);
    }
  }
  if (pl.spmv) store_partial(region(a, 0), acc);
}

// ---- K1 -------------------------------------------------------------------------------
template <class R, int L, bool MHM>
__global__ __launch_bounds__(kBlock) void k1_apply(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& ns = st->rot[a.par ^ 1];  // written by this iteration's head
  if (ns.halt) return;
  const Csr<cplx<R>> m = pick_m<R>(a);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.pb[ns.pcur]);
  cplx<R>* __restrict__ t = static_cast<cplx<R>*>(a.t);
  const double sigma0 = st->sigma0;
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double acc = 0.0;
  auto epilogue = [&](int64_t row, const cplx<R>& v) {
    t[row] = v;
    const cplx<R> pr = p[row];
    if (MHM)
      acc += norm2d<R>(v) + sigma0 * norm2d<R>(pr);
    else
      acc += double(pr.x) * double(v.x) + double(pr.y) * double(v.y) + sigma0 * norm2d<R>(pr);
  };
  for (int64_t row = beg + grp; row < end; row += 2 * GPB) {
    const int64_t row1 = row + GPB;
    const bool has1 = row1 < end;
    cplx<R> v0, v1;
    row_dot2<R, L>(m, p, row, row1, has1, lane, v0, v1);
    if (lane == 0) {
      epilogue(row, v0);
      if (has1) epilogue(row1, v1);
    }
  }
  store_partial(region(a, 0), acc);
}

// ---- K2 (A = M^H M): r <- r - a (M^H t + sigma0 p), R' = |r|^2 ------------------------
template <class R, int L>
__global__ __launch_bounds__(kBlock) void k2_mhm(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& ns = st->rot[a.par ^ 1];  // written by this iteration's head
  if (ns.halt) return;
  Early e;
  load_early(region(a, 0), a.gk1, e);
  double step;
  if (!k2_step(a, e, step)) return;  // breakdown: every workgroup sees the same P
  const Csr<cplx<R>> mh = pick_mh<R>(a);
  const cplx<R>* __restrict__ t = static_cast<const cplx<R>*>(a.t);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.pb[ns.pcur]);
  // the residual moves from this head's ring slot to the next one's (in place when equal)
  const cplx<R>* rin = rslot<R>(a, st->rot[a.par].ndef);
  cplx<R>* r = rslot<R>(a, ns.ndef);
  const double sigma0 = st->sigma0;
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double acc = 0.0;
  auto epilogue = [&](int64_t row, const cplx<R>& q) {
    const double2 pr = to_d(p[row]);
    const double2 rr = to_d(rin[row]);
    const double2 qd = to_d(q);
    double2 nr;
    nr.x = rr.x - step * (qd.x + sigma0 * pr.x);
    nr.y = rr.y - step * (qd.y + sigma0 * pr.y);
    const cplx<R> st_r = from_d<R>(nr);
    r[row] = st_r;
    acc += norm2d<R>(st_r);
  };
  for (int64_t row = beg + grp; row < end; row += 2 * GPB) {
    const int64_t row1 = row + GPB;
    const bool has1 = row1 < end;
    cplx<R> q0, q1;
    row_dot2<R, L>(mh, t, row, row1, has1, lane, q0, q1);
    if (lane == 0) {
      epilogue(row, q0);
      if (has1) epilogue(row1, q1);
    }
  }
  store_partial(region(a, 1), acc);
}

// ---- K2 on the sliced ELLPACK copy of M^H: one row per lane, one slice per wave ------
template <class R>
__global__ __launch_bounds__(kBlock) void k2_sell(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& ns = st->rot[a.par ^ 1];  // written by this iteration's head
  if (ns.halt) return;
  Early e;
  load_early(region(a, 0), a.gk1, e);
  const Sell<cplx<R>> mh = pick_shm<R>(a);
  const cplx<R>* __restrict__ t = static_cast<const cplx<R>*>(a.t);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.pb[ns.pcur]);
  // the residual moves from this head's ring slot to the next one's (in place when equal)
  const cplx<R>* rin = rslot<R>(a, st->rot[a.par].ndef);
  cplx<R>* r = rslot<R>(a, ns.ndef);
  const double sigma0 = st->sigma0;
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  Sweep sw = make_sweep(a.nslices, a.ord, SPB);
  double acc = 0.0;
  double step = 0.0;
  // q = M^H t for one slice, with the row operands of the epilogue
  struct Row {
    cplx<R> q, p, r;
  };
  auto product = [&](int64_t sl) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < a.n ? row : a.n - 1;  // lanes past n read a valid row, unused
    const cplx<R> tr = t[rr];
    Row o;
    o.p = ld_stream(&p[rr]);
    o.r = ld_stream(&rin[rr]);
    const cplx<R> d = mh.diag[rr];
    o.q = sell_row<R>(mh, t, sl, lane);
    cfma<R>(o.q, d, tr);
    return o;
  };
  auto epilogue = [&](int64_t sl, const Row& o) {
    const int64_t row = sl * kSlice + lane;
    if (row >= a.n) return;
    const double2 pr = to_d(o.p);
    const double2 rr = to_d(o.r);
    const double2 qd = to_d(o.q);
    double2 nr;
    nr.x = rr.x - step * (qd.x + sigma0 * pr.x);
    nr.y = rr.y - step * (qd.y + sigma0 * pr.y);
    const cplx<R> st_r = from_d<R>(nr);
    st_stream(&r[row], st_r);
    acc += norm2d<R>(st_r);
  };
  // the first slice's product runs while P's partials are on their way
  const bool has0 = sw.more();
  const int64_t sl0 = has0 ? sw.slice() : 0;
  Row first{};
  if (has0) first = product(sl0);
  if (!k2_step(a, e, step)) return;  // breakdown: every workgroup sees the same P
  if (has0) epilogue(sl0, first);
  for (sw.next(); sw.more(); sw.next()) {
    const int64_t sl = sw.slice();
    epilogue(sl, product(sl));
  }
  store_partial(region(a, 1), acc);
}

// The march positions [beg, end) of this wave: its XCD's share of [0, n) (workgroups are
// dealt to the XCDs in turn), split evenly and contiguously over the XCD's waves.
__device__ __forceinline__ void march_range(int64_t n, int wpb, int64_t& beg, int64_t& end) {
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kWave));
  const int g = gridDim.x;
  int64_t lo = 0, hi = n, nw = int64_t(g) * wpb, w = int64_t(blockIdx.x) * wpb + wv;
  if (g % kXcds == 0) {
    const int x = int(blockIdx.x % kXcds);
    lo = n * x / kXcds;
    hi = n * (x + 1) / kXcds;
    nw = int64_t(g / kXcds) * wpb;
    w = int64_t(blockIdx.x / kXcds) * wpb + wv;
  }
  beg = lo + (hi - lo) * w / nw;
  end = lo + (hi - lo) * (w + 1) / nw;
}

// ---- matrix-free head and K2: one lattice site (three rows) per lane ------------------
// The waves sweep blocks of 64 sites (192 rows).  The head first applies the pending
// update to the block's rows, one row per lane in three passes (the same update_row as on
// the sliced path), then computes t' = M p' for the block's sites, one site per lane,
// forming p' = r + b p at its own and at every gathered neighbour's rows with next_dir,
// so that all of them round exactly as the row's owner does; P = |t'|^2 + sigma0 |p'|^2.
// LR: rows stored per link (3, or 2 for SU(3) links).
// TR (FP64): t' = M r + b t instead of M (r + b p), the old t being M p from the previous
// head: one gathered vector instead of two.  The recurrence's rounding stays at the FP64
// level over the launches between two direct products (the host interleaves a direct
// one every kTrEvery launches).
// A lane's own rows (48 or 24 contiguous bytes, read or written by three instructions
// whose lanes lie 48 or 24 bytes apart) take ordinary loads and stores: with streaming
// hints a line could leave the cache between the three.
constexpr int kSiteBlock = kWave;  // sites per wave pass

// MARCH (two-row links; a.head_march = tc >= 2): K2's column order along t, with the t
// link and the gathered values (p', or r with TR) at the site and at its forward t
// neighbour carried from one site of a column to the next (TCarry).
template <class R, int LR, bool TR, bool MARCH = false>
__global__ __launch_bounds__(kBlock, MSC_SITE_HEAD_WPE) void k1_site(MsArgs a) {
  static_assert(!MARCH || LR == 2, "the head marches on two-row links");
  const SolveState* st = a.st;
  const RotState& rs = st->rot[a.par];
  if (rs.halt) {
    carry_state(a);
    return;
  }
  const int pending = rs.pending;
  Early e;
  if (pending) load_early(region(a, 1), a.gk2, e);
  const int pc = rs.pcur;
  const cplx<R>* __restrict__ rv = rslot<R>(a, rs.ndef);
  const cplx<R>* __restrict__ pv = static_cast<const cplx<R>*>(a.pb[pc]);
  cplx<R>* __restrict__ pnew = static_cast<cplx<R>*>(a.pb[pc ^ 1]);
  cplx<R>* __restrict__ t = static_cast<cplx<R>*>(a.t);
  double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  const Stencil<cplx<R>> w = pick_w<R>(a);
  const uint32_t vol = uint32_t(w.vol);
  const int64_t nblk = (int64_t(vol) + kSiteBlock - 1) / kSiteBlock;
  const double sigma0 = st->sigma0;
  constexpr int WPB = kBlock / kWave;
  const int lane = threadIdx.x % kWave;
  Sweep sw = make_sweep(nblk, a.ord, WPB);
  __shared__ Plan pl;
  head_plan<R>(a, e, pl);
  if (!pl.ok) return;
  const bool upd = pl.pending != 0;
  const double bn = pl.bn;
  double acc = 0.0;
  if constexpr (MARCH) {
    const uint32_t tc = uint32_t(a.head_march);
    const uint32_t vol3 = vol / uint32_t(w.L[3]);  // sites per t-slice
    const uint32_t bs = vol3 / uint32_t(kSiteBlock);
    constexpr int K = 3 * LR;
    const cplx<R>* __restrict__ rg = upd ? rv : pv;
    // the gathered vector at row i: r with TR (p without a pending update), else p'
    // (without a pending update bn = 0 and p' = p exactly)
    auto gv = [&](int64_t i) {
      if constexpr (TR)
        return rg[i];
      else
        return next_dir<R>(bn, rg[i], pv[i]);
    };
    TCarry<R, LR> car;
    int64_t qb, qe;
    march_range(nblk, WPB, qb, qe);
    for (uint32_t q = uint32_t(qb); q < uint32_t(qe); ++q) {
      const uint32_t col = q / tc, chunk = col / bs;
      const int64_t blk = int64_t((chunk * tc + (q - col * tc)) * bs + (col - chunk * bs));
      if (upd) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int64_t row = (3 * blk + k) * kWave + lane;
          update_row<R>(a, pl, row, rv[row], pv[row], x0, pnew);  // below n
        }
      }
#if MSC_SITE_SB
      __builtin_amdgcn_sched_barrier(0);
#endif
      if (!pl.spmv) continue;
      const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);  // below vol
      if (q == uint32_t(qb) || q % tc == 0) {
        // a run's first site or a column's: the carry from memory
        const uint32_t sb = site >= vol3 ? site - vol3 : site + (vol - vol3);  // periodic
        const cplx<R>* __restrict__ wt = w.w + int64_t(3) * K * vol;
#pragma unroll
        for (int k = 0; k < K; ++k) car.u[k] = wt[int64_t(k) * vol + sb];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          car.own[c] = gv(3 * int64_t(sb) + c);
          car.fw[c] = gv(3 * int64_t(site) + c);
        }
      }
      const int64_t r0 = 3 * int64_t(site);
      cplx<R> own[3], pr[3], v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        own[c] = car.fw[c];
        // p' at the site: with TR own is r (p without a pending update), else p' itself
        pr[c] = (TR && upd) ? next_dir<R>(bn, own[c], pv[r0 + c]) : own[c];
      }
      stencil_site_c<R, LR, true>(w, site, own, 1, gv, v, &car);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        car.own[c] = own[c];
        if constexpr (TR) {
          const cplx<R> told = t[r0 + c];
          v[c].x = fma(bn, told.x, v[c].x);
          v[c].y = fma(bn, told.y, v[c].y);
        }
        t[r0 + c] = v[c];
        acc += norm2d<R>(v[c]) + sigma0 * norm2d<R>(pr[c]);
      }
    }
    if (pl.spmv) store_partial(region(a, 0), acc);
    return;
  }
  for (; sw.more(); sw.next()) {
    const int64_t blk = sw.slice();
    if (upd) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int64_t row = (3 * blk + k) * kWave + lane;
        if (row < a.n) update_row<R>(a, pl, row, rv[row], pv[row], x0, pnew);
      }
    }
#if MSC_SITE_SB
    __builtin_amdgcn_sched_barrier(0);
#endif
    if (!pl.spmv) continue;
    const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);
    const bool live = site < vol;
    const uint32_t ss = live ? site : vol - 1;  // lanes past the volume compute a valid site, unused
    const int64_t r0 = 3 * int64_t(ss);
    cplx<R> pr[3], own[3], v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx<R> ri = rv[r0 + c], pi = pv[r0 + c];
      pr[c] = upd ? next_dir<R>(bn, ri, pi) : pi;
      own[c] = TR ? (upd ? ri : pi) : pr[c];
    }
    const cplx<R>* __restrict__ rg = upd ? rv : pv;
    if constexpr (TR) {
      // without a pending update bn = 0 and the product is M p
      stencil_site<R, LR>(w, ss, own, 1, [&](int64_t c) { return rg[c]; }, v);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cplx<R> told = t[r0 + c];
        v[c].x = fma(bn, told.x, v[c].x);
        v[c].y = fma(bn, told.y, v[c].y);
      }
    } else {
      // without a pending update p' = p: the same product with r := p and b = 0 (exact)
      stencil_site<R, LR>(w, ss, own, 1, [&](int64_t c) { return next_dir<R>(bn, rg[c], pv[c]); },
                          v);
    }
    if (live) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        t[r0 + c] = v[c];
        acc += norm2d<R>(v[c]) + sigma0 * norm2d<R>(pr[c]);
      }
    }
  }
  if (pl.spmv) store_partial(region(a, 0), acc);
}

// K2: q = M^H t = m t - D t for the block's sites, then r <- r - a (q + sigma0 p) and
// R' = |r|^2 on their rows.
// MARCH (a.k2_march = tc >= 2; the host checks that a t-slice holds whole blocks of 64
// sites and that tc divides L_t): the blocks are taken in columns of tc consecutive
// t-slices (march position q: column q / tc, slice q % tc of it; the columns of one
// chunk of tc slices first), each wave a contiguous run of positions, so that within a
// column a lane's next site is its last one moved one slice along t: its t link and its
// values stay in registers (TCarry), and the XCD's waves work through the same few
// slices together, where the other neighbours lie.
template <class R, int LR, bool MARCH>
__global__ __launch_bounds__(kBlock, MARCH ? (sizeof(R) == 8 ? MSC_K2_MARCH_WPE64
                                                               : MSC_K2_MARCH_WPE32)
                                            : MSC_SITE_K2_WPE) void k2_site(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& ns = st->rot[a.par ^ 1];  // written by this iteration's head
  if (ns.halt) return;
  Early e;
  load_early(region(a, 0), a.gk1, e);
  const cplx<R>* __restrict__ t = static_cast<const cplx<R>*>(a.t);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.pb[ns.pcur]);
  // the residual moves from this head's ring slot to the next one's (in place when equal)
  const cplx<R>* rin = rslot<R>(a, st->rot[a.par].ndef);
  cplx<R>* r = rslot<R>(a, ns.ndef);
  const Stencil<cplx<R>> w = pick_w<R>(a);
  const uint32_t vol = uint32_t(w.vol);
  const int64_t nblk = (int64_t(vol) + kSiteBlock - 1) / kSiteBlock;
  const double sigma0 = st->sigma0;
  constexpr int WPB = kBlock / kWave;
  const int lane = threadIdx.x % kWave;
  Sweep sw = make_sweep(nblk, a.ord, WPB);
  double acc = 0.0;
  double step = 0.0;
  struct Site {
    cplx<R> q[3];
  };
  auto product = [&](int64_t blk) {
    const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);
    const uint32_t ss = site < vol ? site : vol - 1;  // lanes past the volume: unused
    const int64_t r0 = 3 * int64_t(ss);
    cplx<R> own[3];
    Site o;
#pragma unroll
    for (int c = 0; c < 3; ++c) own[c] = t[r0 + c];
    stencil_site<R, LR>(w, ss, own, -1, [&](int64_t c) { return t[c]; }, o.q);
    return o;
  };
  auto epilogue = [&](int64_t blk, const Site& o) {
    const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);
    if (site >= vol) return;
    const int64_t r0 = 3 * int64_t(site);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 pr = to_d(p[r0 + c]);
      const double2 rr = to_d(rin[r0 + c]);
      const double2 qd = to_d(o.q[c]);
      double2 nr;
      nr.x = rr.x - step * (qd.x + sigma0 * pr.x);
      nr.y = rr.y - step * (qd.y + sigma0 * pr.y);
      const cplx<R> st_r = from_d<R>(nr);
      r[r0 + c] = st_r;
      acc += norm2d<R>(st_r);
    }
  };
  if constexpr (MARCH) {
    // positions and blocks in 32 bits (the volume is below 2^31)
    const uint32_t tc = uint32_t(a.k2_march);
    const uint32_t bs = vol / uint32_t(w.L[3]) / uint32_t(kSiteBlock);  // blocks per t-slice
    auto block_at = [&](uint32_t q) {
      const uint32_t col = q / tc, chunk = col / bs;
      return int64_t((chunk * tc + (q - col * tc)) * bs + (col - chunk * bs));
    };
    TCarry<R, LR> car;
    const uint32_t vol3 = vol / uint32_t(w.L[3]);  // sites per t-slice
    constexpr int K = 3 * LR;
    // the carry for a block whose previous site along t this wave did not just take: the
    // backward t link and the values at the backward t neighbour and at the site
    auto preload = [&](int64_t blk) {
      const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);
      const uint32_t sb = site >= vol3 ? site - vol3 : site + (vol - vol3);  // periodic
      const cplx<R>* __restrict__ wt = w.w + int64_t(3) * K * vol;
#pragma unroll
      for (int k = 0; k < K; ++k) car.u[k] = wt[int64_t(k) * vol + sb];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        car.own[c] = t[3 * int64_t(sb) + c];
        car.fw[c] = t[3 * int64_t(site) + c];
      }
    };
    auto product_c = [&](int64_t blk) {
      const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);  // below vol
      cplx<R> own[3];
      Site o;
#pragma unroll
      for (int c = 0; c < 3; ++c) own[c] = car.fw[c];
      stencil_site_c<R, LR, true>(w, site, own, -1, [&](int64_t c) { return t[c]; }, o.q, &car);
#pragma unroll
      for (int c = 0; c < 3; ++c) car.own[c] = own[c];
      return o;
    };
    int64_t qb, qe;
    march_range(nblk, WPB, qb, qe);
    uint32_t q = uint32_t(qb);
    const uint32_t qend = uint32_t(qe);
    const bool has0 = q < qend;
    const int64_t b0 = has0 ? block_at(q) : 0;
    Site first{};
    if (has0) {
      preload(b0);
      first = product_c(b0);
    }
    if (!k2_step(a, e, step)) return;  // breakdown: every workgroup sees the same P
    if (has0) {
      epilogue(b0, first);
      // within a column the carry moves on; a new column starts from memory
#pragma nounroll
      for (++q; q < qend; ++q) {
        const int64_t blk = block_at(q);
        if (q % tc == 0) preload(blk);
        epilogue(blk, product_c(blk));
      }
    }
    store_partial(region(a, 1), acc);
    return;
  }
  // the first block's product runs while P's partials are on their way
  const bool has0 = sw.more();
  const int64_t b0 = has0 ? sw.slice() : 0;
  Site first{};
  if (has0) first = product(b0);
  if (!k2_step(a, e, step)) return;  // breakdown: every workgroup sees the same P
  if (has0) epilogue(b0, first);
  for (sw.next(); sw.more(); sw.next()) {
    const int64_t blk = sw.slice();
    epilogue(blk, product(blk));
  }
  store_partial(region(a, 1), acc);
}

// ---- K2 (A given): elementwise r <- r - a (t + sigma0 p) -------------------------------
template <class R>
__global__ __launch_bounds__(kBlock) void k2_herm(MsArgs a) {
  const SolveState* st = a.st;
  const RotState& ns = st->rot[a.par ^ 1];  // written by this iteration's head
  if (ns.halt) return;
  Early e;
  load_early(region(a, 0), a.gk1, e);
  double step;
  if (!k2_step(a, e, step)) return;  // breakdown: every workgroup sees the same P
  const cplx<R>* __restrict__ t = static_cast<const cplx<R>*>(a.t);
  const cplx<R>* __restrict__ p = static_cast<const cplx<R>*>(a.pb[ns.pcur]);
  // the residual moves from this head's ring slot to the next one's (in place when equal)
  const cplx<R>* rin = rslot<R>(a, st->rot[a.par].ndef);
  cplx<R>* r = rslot<R>(a, ns.ndef);
  const double sigma0 = st->sigma0;
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 pr = to_d(p[i]), rr = to_d(rin[i]), td = to_d(t[i]);
    double2 nr;
    nr.x = rr.x - step * (td.x + sigma0 * pr.x);
    nr.y = rr.y - step * (td.y + sigma0 * pr.y);
    const cplx<R> st_r = from_d<R>(nr);
    r[i] = st_r;
    acc += norm2d<R>(st_r);
  }
  store_partial(region(a, 1), acc);
}

// ---- initialisation: r = p = p_j = b, x = 0, |b|^2 ------------------------------------
template <class R>
__global__ __launch_bounds__(kBlock) void k_init(MsArgs a) {
  SolveState* st = a.st;
  const int64_t n = a.n;
  const int ns = st->ns;
  cplx<R>* __restrict__ r = static_cast<cplx<R>*>(a.r);
  cplx<R>* __restrict__ p = static_cast<cplx<R>*>(a.pb[0]);  // rot[par].pcur = 0
  cplx<R>* __restrict__ pk = static_cast<cplx<R>*>(a.pk);
  int64_t beg, end;
  block_range(n, kBlock, beg, end);
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 bv = a.b[i];
    const cplx<R> br = from_d<R>(bv);
    r[i] = br;
    p[i] = br;
    for (int j = 1; j < ns; ++j) pk[int64_t(j - 1) * n + i] = br;
    for (int k = 0; k < ns; ++k) a.x[int64_t(k) * n + i] = double2{0.0, 0.0};
    acc += fma(bv.x, bv.x, bv.y * bv.y);
  }
  const double tot = block_sum<kBlock>(acc);
  if (threadIdx.x == 0) store_agent(&a.sc.partial[blockIdx.x], tot);
  if (!arrive_last(a.sc.tickets + 3 * kTicketSite)) return;
  const double B2 = sum_partials(a.sc.partial, gridDim.x, 1, 0);
  if (threadIdx.x == 0) {
    RotState& r0 = st->rot[a.par];
    st->bnorm2 = B2;
    r0.R = B2;
    st->eps2 = st->eps2 * B2;        // host stored tol^2 here
    st->sw_eps2 = st->sw_eps2 * B2;  // and switch_tol^2 (0 when there is no switch)
    if (!(B2 > 0.0) || !isfinite(B2)) {
      r0.halt = 1;
      if (!isfinite(B2)) r0.status = 1;
    }
  }
}

// ---- end of the FP64 phase of a mixed solve: Krylov vectors to complex64 -------------
__global__ __launch_bounds__(kBlock) void k_switch(MsArgs a64, MsArgs a32, int ns) {
  const int64_t n = a64.n;
  const int pc = a64.st->rot[a64.par].pcur;  // the direction buffer in use carries over
  // r stays in the ring slot the halting (switching) head read; slot 0 of complex64
  const double2* __restrict__ r = rslot<double>(a64, a64.st->rslot);
  const double2* __restrict__ p = static_cast<const double2*>(a64.pb[pc]);
  const double2* __restrict__ pk = static_cast<const double2*>(a64.pk);
  float2* __restrict__ r32 = static_cast<float2*>(a32.r);
  float2* __restrict__ p32 = static_cast<float2*>(a32.pb[pc]);
  float2* __restrict__ pk32 = static_cast<float2*>(a32.pk);
  const int64_t total = int64_t(ns) * n;  // r, p, then ns-1 shift directions
  for (int64_t idx = blockIdx.x * int64_t(kBlock) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * kBlock) {
    if (idx < n) {
      r32[idx] = from_d<float>(r[idx]);
      p32[idx] = from_d<float>(p[idx]);
    } else {
      pk32[idx - n] = from_d<float>(pk[idx - n]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SolveState* st = a64.st;
    RotState& rs = st->rot[a64.par];
    if (rs.status == 0 && rs.switch_req) {
      rs.halt = 0;
      rs.switch_req = 0;
      st->sw_eps2 = 0.0;
      st->R_ru = rs.R;
    }
  }
}

// ---- reliable update: r = b - (A + sigma0) x_0 in FP64, between the head and K2 ----------
// Launched at check points; runs (in every workgroup alike) when forced by the period or
// when the recursive residual has dropped by kRuDelta2 in |r|^2 since the last one.
__device__ __forceinline__ bool ru_due(const MsArgs& a) {
  const SolveState* st = a.st;
  const RotState& ns = st->rot[a.par ^ 1];  // written by this iteration's head
  if (ns.halt) return false;
  return a.ru_force || ns.R < kRuDelta2 * st->R_ru;
}

// After each workgroup's share of |r|^2 (acc per thread): the last workgroup replaces R.
// The update never halts the sequence (K2 decides on the replaced residual), so heads
// before it may defer their all-shift update; a non-finite residual is a breakdown.
__device__ void ru_finish(const MsArgs& a, double acc) {
  SolveState* st = a.st;
  // region 2: the head's partials in region 0 still wait for K2
  double* reg = region(a, 2);
  const double tot = block_sum<kBlock>(acc);
  if (threadIdx.x == 0) store_agent(&reg[blockIdx.x], tot);
  if (!arrive_last(a.sc.tickets + 2 * kTicketSite)) return;
  const double Rt = sum_partials(reg, gridDim.x, 1, 0);
  if (threadIdx.x == 0) {
    RotState& rs = st->rot[a.par ^ 1];
    rs.R = Rt;
    st->R_ru = Rt;
    st->n_reliable += 1;
    if (!isfinite(Rt)) {
      rs.status = 1;
      rs.halt = 1;
      store_host_flag(a.hflag, 1);
    }
  }
}

template <int L, bool MHM>
__global__ __launch_bounds__(kBlock) void k_ru_first(MsArgs a) {
  // t64 = M x_0 (A = M^H M) -- first half of the FP64 operator
  const SolveState* st = a.st;
  if (!ru_due(a)) return;
  const double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  for (int64_t row = beg + grp; row < end; row += GPB) {
    const double2 v = row_dot<double, L>(a.m64, x0, row, lane);
    if (lane == 0) a.t64[row] = v;
  }
}

template <class R, int L, bool MHM>
__global__ __launch_bounds__(kBlock) void k_ru_second(MsArgs a) {
  SolveState* st = a.st;
  if (!ru_due(a)) return;
  const double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  cplx<R>* __restrict__ r = rslot<R>(a, st->rot[a.par].ndef);  // r_i's ring slot
  const double sigma0 = st->sigma0;
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double acc = 0.0;
  for (int64_t row = beg + grp; row < end; row += GPB) {
    const double2 q = MHM ? row_dot<double, L>(a.mh64, a.t64, row, lane)
                          : row_dot<double, L>(a.m64, x0, row, lane);
    if (lane == 0) {
      const double2 bv = a.b[row], xv = x0[row];
      double2 rt;
      rt.x = bv.x - q.x - sigma0 * xv.x;
      rt.y = bv.y - q.y - sigma0 * xv.y;
      r[row] = from_d<R>(rt);
      acc += fma(rt.x, rt.x, rt.y * rt.y);
    }
  }
  ru_finish(a, acc);
}

// The same on the sliced ELLPACK copies: one row per lane, one slice per wavefront.
__global__ __launch_bounds__(kBlock) void k_ru_first_s(MsArgs a) {
  const SolveState* st = a.st;
  if (!ru_due(a)) return;
  const double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  int64_t beg, end;
  block_range(a.nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < a.n ? row : a.n - 1;
    double2 v = sell_row<double>(a.s64, x0, sl, lane);
    cfma<double>(v, a.s64.diag[rr], x0[rr]);
    if (row < a.n) a.t64[row] = v;
  }
}

template <class R, bool MHM>
__global__ __launch_bounds__(kBlock) void k_ru_second_s(MsArgs a) {
  SolveState* st = a.st;
  if (!ru_due(a)) return;
  const double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  cplx<R>* __restrict__ r = rslot<R>(a, st->rot[a.par].ndef);  // r_i's ring slot
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
    const Sell<double2> m = MHM ? a.sh64 : a.s64;
    const double2* __restrict__ in = MHM ? a.t64 : x0;
    double2 q = sell_row<double>(m, in, sl, lane);
    cfma<double>(q, m.diag[rr], in[rr]);
    if (row < a.n) {
      const double2 bv = a.b[row], xv = x0[row];
      double2 rt;
      rt.x = bv.x - q.x - sigma0 * xv.x;
      rt.y = bv.y - q.y - sigma0 * xv.y;
      r[row] = from_d<R>(rt);
      acc += fma(rt.x, rt.x, rt.y * rt.y);
    }
  }
  ru_finish(a, acc);
}

// The same on the links (matrix-free staggered operator, LR rows per link), one site per
// lane: t64 = M x_0, then r = b - M^H t64 - sigma0 x_0.
template <int LR>
__global__ __launch_bounds__(kBlock) void k_ru_first_site(MsArgs a) {
  const SolveState* st = a.st;
  if (!ru_due(a)) return;
  const double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  const Stencil<double2> w = a.w64;
  const uint32_t vol = uint32_t(w.vol);
  constexpr int WPB = kBlock / kWave;
  const int lane = threadIdx.x % kWave;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kWave));
  int64_t beg, end;
  block_range((int64_t(vol) + kSiteBlock - 1) / kSiteBlock, WPB, beg, end);
  for (int64_t blk = beg + wv; blk < end; blk += WPB) {
    const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);
    const uint32_t ss = site < vol ? site : vol - 1;  // lanes past the volume: unused
    const int64_t r0 = 3 * int64_t(ss);
    double2 own[3], v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) own[c] = x0[r0 + c];
    stencil_site<double, LR>(w, ss, own, 1, [&](int64_t c) { return x0[c]; }, v);
    if (site < vol) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.t64[r0 + c] = v[c];
    }
  }
}

template <class R, int LR>
__global__ __launch_bounds__(kBlock) void k_ru_second_site(MsArgs a) {
  SolveState* st = a.st;
  if (!ru_due(a)) return;
  const double2* __restrict__ x0 = a.x + int64_t(st->orig[0]) * a.n;
  const double2* __restrict__ u = a.t64;
  cplx<R>* __restrict__ r = rslot<R>(a, st->rot[a.par].ndef);  // r_i's ring slot
  const double sigma0 = st->sigma0;
  const Stencil<double2> w = a.w64;
  const uint32_t vol = uint32_t(w.vol);
  constexpr int WPB = kBlock / kWave;
  const int lane = threadIdx.x % kWave;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kWave));
  int64_t beg, end;
  block_range((int64_t(vol) + kSiteBlock - 1) / kSiteBlock, WPB, beg, end);
  double acc = 0.0;
  for (int64_t blk = beg + wv; blk < end; blk += WPB) {
    const uint32_t site = uint32_t(blk * kSiteBlock) + uint32_t(lane);
    const uint32_t ss = site < vol ? site : vol - 1;  // lanes past the volume: unused
    const int64_t r0 = 3 * int64_t(ss);
    double2 own[3], q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) own[c] = u[r0 + c];
    stencil_site<double, LR>(w, ss, own, -1, [&](int64_t c) { return u[c]; }, q);
    if (site < vol) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double2 bv = a.b[r0 + c], xv = x0[r0 + c];
        double2 rt;
        rt.x = bv.x - q[c].x - sigma0 * xv.x;
        rt.y = bv.y - q[c].y - sigma0 * xv.y;
        r[r0 + c] = from_d<R>(rt);
        acc += fma(rt.x, rt.x, rt.y * rt.y);
      }
    }
  }
  ru_finish(a, acc);
}

// ---- verification: FP64 true residual norms of up to 8 solutions ---------------------
constexpr int kVerifyChunk = 8;

template <int L>
__device__ __forceinline__ void row_dot_multi(const Csr<double2>& m, const double2* __restrict__ x,
                                              int64_t n, int kc, int64_t row, int lane,
                                              double2 (&acc)[kVerifyChunk]) {
#pragma unroll
  for (int q = 0; q < kVerifyChunk; ++q) acc[q] = double2{0.0, 0.0};
  const int32_t beg = m.rowptr[row], end = m.rowptr[row + 1];
  for (int32_t j = beg + lane; j < end; j += L) {
    const int32_t c = m.col[j];
    const double2 v = m.val[j];
#pragma unroll
    for (int q = 0; q < kVerifyChunk; ++q)
      if (q < kc) cfma<double>(acc[q], v, x[int64_t(q) * n + c]);
  }
#pragma unroll
  for (int q = 0; q < kVerifyChunk; ++q) acc[q] = group_sum_c<L, double>(acc[q]);
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_verify_first(Csr<double2> m, const double2* x, int64_t n,
                                                         int kc, double2* u) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(n, GPB, beg, end);
  double2 acc[kVerifyChunk];
  for (int64_t row = beg + grp; row < end; row += GPB) {
    row_dot_multi<L>(m, x, n, kc, row, lane, acc);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kVerifyChunk; ++q)
        if (q < kc) u[int64_t(q) * n + row] = acc[q];
    }
  }
}

struct VerifyArgs {
  Csr<double2> m;        // M^H (MHM) or A (HERM)
  Sell<double2> s;       // its sliced ELLPACK copy (the SELL kernels)
  int64_t nslices;
  const double2* in;     // U = M X (MHM) or X (HERM), chunk of kc vectors
  const double2* x;      // X, chunk of kc vectors
  const double2* b;
  double sig[kVerifyChunk];
  int64_t n;
  int kc;
  double* partial;
  unsigned* ticket;
  double* out;           // res2 of the chunk
};

// Per-chunk norms: workgroup partials, then the last workgroup's totals in out[0..kc).
__device__ void verify_finish(const VerifyArgs& v, double (&nrm)[kVerifyChunk]) {
  block_sum_k<kBlock, kVerifyChunk>(nrm);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kVerifyChunk; ++q) store_agent(&v.partial[blockIdx.x * kVerifyChunk + q], nrm[q]);
  }
  if (!arrive_last(v.ticket)) return;
  for (int q = 0; q < v.kc; ++q) {
    const double s = sum_partials(v.partial, gridDim.x, kVerifyChunk, q);
    if (threadIdx.x == 0) v.out[q] = s;
  }
}

template <int L>
__global__ __launch_bounds__(kBlock) void k_verify_second(VerifyArgs v) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(v.n, GPB, beg, end);
  double2 acc[kVerifyChunk];
  double nrm[kVerifyChunk];
#pragma unroll
  for (int q = 0; q < kVerifyChunk; ++q) nrm[q] = 0.0;
  for (int64_t row = beg + grp; row < end; row += GPB) {
    row_dot_multi<L>(v.m, v.in, v.n, v.kc, row, lane, acc);
    if (lane == 0) {
      const double2 bv = v.b[row];
#pragma unroll
      for (int q = 0; q < kVerifyChunk; ++q) {
        if (q < v.kc) {
          const double2 xv = v.x[int64_t(q) * v.n + row];
          const double rx = bv.x - acc[q].x - v.sig[q] * xv.x;
          const double ry = bv.y - acc[q].y - v.sig[q] * xv.y;
          nrm[q] += fma(rx, rx, ry * ry);
        }
      }
    }
  }
  verify_finish(v, nrm);
}

// One row per lane on the sliced ELLPACK copies: u_q = M x_q, then the residual norms.
__global__ __launch_bounds__(kBlock) void k_verify_first_s(Sell<double2> m, const double2* x,
                                                           int64_t n, int64_t nslices, int kc,
                                                           double2* u) {
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  const double2* xs[kVerifyChunk];
#pragma unroll
  for (int q = 0; q < kVerifyChunk; ++q) xs[q] = x + int64_t(q < kc ? q : 0) * n;
  int64_t beg, end;
  block_range(nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < n ? row : n - 1;
    double2 acc[kVerifyChunk];
    sell_row_multi<double, kVerifyChunk, 1>(m, xs, kc, sl, lane, acc);
    const double2 d = m.diag[rr];
#pragma unroll
    for (int q = 0; q < kVerifyChunk; ++q) {
      if (q < kc) {
        cfma<double>(acc[q], d, xs[q][rr]);
        if (row < n) u[int64_t(q) * n + row] = acc[q];
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_verify_second_s(VerifyArgs v) {
  constexpr int SPB = kBlock / kSlice;
  const int lane = threadIdx.x % kSlice;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kSlice));
  const double2* ins[kVerifyChunk];
#pragma unroll
  for (int q = 0; q < kVerifyChunk; ++q) ins[q] = v.in + int64_t(q < v.kc ? q : 0) * v.n;
  double nrm[kVerifyChunk];
#pragma unroll
  for (int q = 0; q < kVerifyChunk; ++q) nrm[q] = 0.0;
  int64_t beg, end;
  block_range(v.nslices, SPB, beg, end);
  for (int64_t sl = beg + wv; sl < end; sl += SPB) {
    const int64_t row = sl * kSlice + lane;
    const int64_t rr = row < v.n ? row : v.n - 1;
    double2 acc[kVerifyChunk];
    sell_row_multi<double, kVerifyChunk, 1>(v.s, ins, v.kc, sl, lane, acc);
    const double2 d = v.s.diag[rr];
    if (row < v.n) {
      const double2 bv = v.b[row];
#pragma unroll
      for (int q = 0; q < kVerifyChunk; ++q) {
        if (q < v.kc) {
          cfma<double>(acc[q], d, ins[q][row]);
          const double2 xv = v.x[int64_t(q) * v.n + row];
          const double rx = bv.x - acc[q].x - v.sig[q] * xv.x;
          const double ry = bv.y - acc[q].y - v.sig[q] * xv.y;
          nrm[q] += fma(rx, rx, ry * ry);
        }
      }
    }
  }
  verify_finish(v, nrm);
}

// ---- plain SpMV with optional shift epilogue (operator application) -------------------
template <class R, int L>
__global__ __launch_bounds__(kBlock) void k_spmv(Csr<cplx<R>> m, const cplx<R>* x, cplx<R>* y,
                                                 int64_t n) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(n, GPB, beg, end);
  for (int64_t row = beg + grp; row < end; row += GPB) {
    const cplx<R> v = row_dot<R, L>(m, x, row, lane);
    if (lane == 0) y[row] = v;
  }
}

template <class R>
__global__ void k_shift_out(const cplx<R>* q, const double2* in, double2* out, double shift, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double2 qd = to_d(q[i]), xv = in[i];
    out[i] = double2{qd.x + shift * xv.x, qd.y + shift * xv.y};
  }
}

__global__ void k_to32(const double2* in, float2* out, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = float2{float(in[i].x), float(in[i].y)};
}

// Workgroups for `n` items processed `rows_per_pass` at a time: one pass each when that
// fits under the cap (kMaxGrid, or a smaller tuning value), a multiple of the XCD count.
int grid_rows(int64_t n, int rows_per_pass, int cap = kMaxGrid) {
  if (cap <= 0 || cap > kMaxGrid) cap = kMaxGrid;
  int64_t g = (n + rows_per_pass - 1) / rows_per_pass;
  if (g > cap) g = cap;
  if (g < kXcds) g = kXcds;
  g = (g + kXcds - 1) / kXcds * kXcds;
  if (g > kMaxGrid) g = kMaxGrid;
  return int(g);
}

// Workgroups of kernel `kern` (kBlock threads) that the device holds resident at once,
// rounded down to a multiple of the XCD count: the grid of a launch whose waves sweep a
// lattice order in step (a larger grid would leave the later workgroups' positions to a
// second round).  Cached per device and kernel.
int resident_grid(const void* kern, int cap, size_t lds = 0) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return cap;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, kern);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int per_cu = 0, cus = 0;
    int g = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      g = per_cu * cus / kXcds * kXcds;
    it = cache.emplace(key, g).first;
  }
  const int g = it->second;
  return g >= kXcds && g < cap ? g : cap;
}

// Dispatch on lanes per row.
#define MSC_LANES_SWITCH(LANES, CALL) \
  switch (LANES) {                    \
    case 4: { constexpr int LL = 4; CALL; } break;   \
    case 8: { constexpr int LL = 8; CALL; } break;   \
    case 16: { constexpr int LL = 16; CALL; } break;  \
    case 32: { constexpr int LL = 32; CALL; } break;  \
    default: return hipErrorInvalidValue;            \
  }

// Launch one kernel of an iteration.  With `ev`, the start/stop events of pair `k` are
// attached to the dispatch itself (their timestamps are the kernel's own begin and
// end), so the elapsed time excludes the queue gap between kernels.
template <class K>
void launch_timed(K kern, int grid, hipStream_t s, hipEvent_t* ev, int k, const MsArgs& a,
                  size_t lds = 0) {
  if (ev)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, ev[2 * k], ev[2 * k + 1], 0, a);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, a);
}

template <class R>
hipError_t reliable_impl(const MsArgs& a, hipStream_t s) {
  if (a.sell && a.kind == MSC_A_MHM && a.stencil != 0) {
    // the links: the same FP64 operator as the stored copies, a third of their bytes
    const int gs = grid_rows((a.w64.vol + kSiteBlock - 1) / kSiteBlock, kBlock / kWave);
    if (a.stencil == 2) {
      k_ru_first_site<2><<<gs, kBlock, 0, s>>>(a);
      k_ru_second_site<R, 2><<<gs, kBlock, 0, s>>>(a);
    } else {
      k_ru_first_site<3><<<gs, kBlock, 0, s>>>(a);
      k_ru_second_site<R, 3><<<gs, kBlock, 0, s>>>(a);
    }
    return hipGetLastError();
  }
  if (a.sell) {
    const int gs = grid_rows(a.nslices, kBlock / kSlice);
    if (a.kind == MSC_A_MHM) {
      k_ru_first_s<<<gs, kBlock, 0, s>>>(a);
      k_ru_second_s<R, true><<<gs, kBlock, 0, s>>>(a);
    } else {
      k_ru_second_s<R, false><<<gs, kBlock, 0, s>>>(a);
    }
    return hipGetLastError();
  }
  const int g1 = grid_rows(a.n, kBlock / a.lanes);
  if (a.kind == MSC_A_MHM) {
    MSC_LANES_SWITCH(a.lanes, (k_ru_first<LL, true><<<g1, kBlock, 0, s>>>(a)));
    MSC_LANES_SWITCH(a.lanes, (k_ru_second<R, LL, true><<<g1, kBlock, 0, s>>>(a)));
  } else {
    MSC_LANES_SWITCH(a.lanes, (k_ru_second<R, LL, false><<<g1, kBlock, 0, s>>>(a)));
  }
  return hipGetLastError();
}

// One iteration: the head (pending update fused with K1 on the sliced ELLPACK path; a
// separate update kernel followed by the CSR K1 otherwise), the optional reliable
// update, then K2.
template <class R>
hipError_t iteration_impl(const MsArgs& args, hipStream_t s, hipEvent_t* ev, bool reliable) {
  const int g1 = grid_rows(args.n, kBlock / args.lanes, args.grid);
  const int g3 = grid_rows(args.n, kBlock, args.grid);
  MsArgs a = args;
  const int lr = (a.sell && a.kind == MSC_A_MHM) ? a.stencil : 0;  // links: rows per link
  // the head and K2 on the sliced path, and their grids: with a lattice order, the
  // resident workgroups only (their waves sweep the order in step)
  const bool tr = a.t_rec && std::is_same<R, double>::value;
  auto head = lr == 3 ? (tr ? k1_site<R, 3, true> : k1_site<R, 3, false>)
              : lr == 2 ? (tr ? k1_site<R, 2, true> : k1_site<R, 2, false>)
                        : (a.kind == MSC_A_MHM ? k1_fused<R, true> : k1_fused<R, false>);
  // K2 on two-row links marches along t (k2_site<.., true>) when it runs on the resident
  // grid, a t-slice holds whole blocks of 64 sites, some tc >= 2 (at most kK2March)
  // divides L_t and every wave gets a run of at least 4 blocks
  const int64_t lt = a.w64.L[3], vol = a.w64.vol;
  int tc = 1;
  if (lr == 2 && a.ord.on && lt > 0 && (vol / lt) % kSiteBlock == 0)
    for (int c = kK2March; c >= 2 && tc == 1; c /= 2)
      if (lt % c == 0) tc = c;
  const int tc_lattice = tc;
  auto k2s = lr == 3   ? k2_site<R, 3, false>
             : lr == 2 ? (tc > 1 ? k2_site<R, 2, true> : k2_site<R, 2, false>)
                       : k2_sell<R>;
  // the links' kernels take one block of 64 sites per wave pass
  const int gsite = lr ? grid_rows((vol + kSiteBlock - 1) / kSiteBlock, kBlock / kWave, a.grid)
                       : g3;
  int gh = lr ? gsite : g3, gk = gh;
  // the complex64 K2 on the links takes unused dynamic LDS that leaves room for three of
  // its workgroups per CU (three waves per SIMD instead of the four its registers allow):
  // fewer waves in flight keep more of the neighbours in L2
  const size_t k2lds = (lr && std::is_same<R, float>::value) ? kC64K2Lds : 0;
  if (a.sell && a.ord.on) {
    gh = resident_grid(reinterpret_cast<const void*>(head), gh);
    if (a.kind == MSC_A_MHM) gk = resident_grid(reinterpret_cast<const void*>(k2s), gk, k2lds);
  }
  if (tc > 1 && (vol / kSiteBlock) < int64_t(gk) * (kBlock / kWave) * 4) {
    // runs too short to carry much: the plain order
    tc = 1;
    k2s = k2_site<R, 2, false>;
    gk = resident_grid(reinterpret_cast<const void*>(k2s), gsite, k2lds);
  }
  a.k2_march = tc;
  // the heads on two-row links march with K2's columns (FP64: the recurrence's heads; the
  // direct products keep the sweep order) when every resident wave gets a run of at
  // least 4 blocks
  a.head_march = 1;
  if (kHeadMarch && lr == 2 && tc_lattice > 1) {
    decltype(head) hm = nullptr;
    if constexpr (std::is_same<R, float>::value)
      hm = k1_site<R, 2, false, true>;
    else if (tr)
      hm = k1_site<R, 2, true, true>;
    if (hm) {
      const int gm = resident_grid(reinterpret_cast<const void*>(hm), gsite);
      if (vol / kSiteBlock >= int64_t(gm) * (kBlock / kWave) * 4) {
        head = hm;
        gh = gm;
        a.head_march = tc_lattice;
      }
    }
  }
  // workgroups of K1 and K2, whose partials K2 and the next head add up
  if (a.sell) {
    a.gk1 = gh;
    a.gk2 = gk;
  } else {
    a.gk1 = g1;
    a.gk2 = a.kind == MSC_A_MHM ? g1 : g3;
  }
  if (a.sell) {
    launch_timed(head, gh, s, ev, 0, a);
  } else {
    launch_timed(k_update<R>, g3, s, ev, 2, a);
    if (a.kind == MSC_A_MHM) {
      MSC_LANES_SWITCH(a.lanes, (launch_timed(k1_apply<R, LL, true>, g1, s, ev, 0, a)));
    } else {
      MSC_LANES_SWITCH(a.lanes, (launch_timed(k1_apply<R, LL, false>, g1, s, ev, 0, a)));
    }
  }
  if (reliable) {
    const hipError_t e = reliable_impl<R>(a, s);
    if (e != hipSuccess) return e;
  }
  if (a.kind == MSC_A_MHM) {
    if (a.sell) {
      launch_timed(k2s, gk, s, ev, 1, a, k2lds);
    } else {
      MSC_LANES_SWITCH(a.lanes, (launch_timed(k2_mhm<R, LL>, g1, s, ev, 1, a)));
    }
  } else {
    launch_timed(k2_herm<R>, g3, s, ev, 1, a);
  }
  return hipGetLastError();
}

}  // namespace

int default_grid(int64_t n, int lanes) { return grid_rows(n, kBlock / lanes); }

hipError_t launch_init(int prec, const MsArgs& a, hipStream_t s) {
  const int g3 = grid_rows(a.n, kBlock);
  if (prec == MSC_PREC_MIXED)
    k_init<float><<<g3, kBlock, 0, s>>>(a);
  else
    k_init<double><<<g3, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_iteration(int prec, const MsArgs& a, hipStream_t s, hipEvent_t* ev,
                            bool reliable) {
  return prec == MSC_PREC_MIXED ? iteration_impl<float>(a, s, ev, reliable)
                                : iteration_impl<double>(a, s, ev, reliable);
}

hipError_t launch_switch_to_mixed(const MsArgs& a64, const MsArgs& a32, int ns, hipStream_t s) {
  const int g = grid_rows(int64_t(ns) * a64.n, kBlock);
  k_switch<<<g, kBlock, 0, s>>>(a64, a32, ns);
  return hipGetLastError();
}

hipError_t launch_verify(const MsArgs& a, const double* sigma_by_caller_index, int k0, int kc,
                         double2* u64, hipStream_t s) {
  if (kc < 1 || kc > kVerifyChunk) return hipErrorInvalidValue;
  const int g1 = grid_rows(a.n, kBlock / a.lanes);
  const double2* xc = a.x + int64_t(k0) * a.n;
  VerifyArgs v;
  v.in = xc;
  v.x = xc;
  v.b = a.b;
  for (int q = 0; q < kVerifyChunk; ++q) v.sig[q] = q < kc ? sigma_by_caller_index[k0 + q] : 0.0;
  v.n = a.n;
  v.kc = kc;
  v.partial = a.sc.partial;
  v.ticket = a.sc.tickets + 4 * kTicketSite;
  v.out = a.sc.res2 + k0;
  if (a.sell) {
    const int gs = grid_rows(a.nslices, kBlock / kSlice);
    v.nslices = a.nslices;
    if (a.kind == MSC_A_MHM) {
      k_verify_first_s<<<gs, kBlock, 0, s>>>(a.s64, xc, a.n, a.nslices, kc, u64);
      v.s = a.sh64;
      v.in = u64;
    } else {
      v.s = a.s64;
    }
    k_verify_second_s<<<gs, kBlock, 0, s>>>(v);
    return hipGetLastError();
  }
  if (a.kind == MSC_A_MHM) {
    MSC_LANES_SWITCH(a.lanes, (k_verify_first<LL><<<g1, kBlock, 0, s>>>(a.m64, xc, a.n, kc, u64)));
    v.m = a.mh64;
    v.in = u64;
  } else {
    v.m = a.m64;
  }
  MSC_LANES_SWITCH(a.lanes, (k_verify_second<LL><<<g1, kBlock, 0, s>>>(v)));
  return hipGetLastError();
}

hipError_t launch_apply(int kind, int prec, int lanes, int64_t n, const Csr<double2>& m64,
                        const Csr<double2>& mh64, const Csr<float2>& m32,
                        const Csr<float2>& mh32, const double2* in, double2* out,
                        double shift, void* tmp_a, void* tmp_b, hipStream_t s) {
  const int g1 = grid_rows(n, kBlock / lanes);
  const int g3 = grid_rows(n, kBlock);
  if (prec == MSC_PREC_MIXED) {
    float2* a32 = static_cast<float2*>(tmp_a);
    float2* b32 = static_cast<float2*>(tmp_b);
    k_to32<<<g3, kBlock, 0, s>>>(in, a32, n);
    MSC_LANES_SWITCH(lanes, (k_spmv<float, LL><<<g1, kBlock, 0, s>>>(m32, a32, b32, n)));
    if (kind == MSC_A_MHM) {
      MSC_LANES_SWITCH(lanes, (k_spmv<float, LL><<<g1, kBlock, 0, s>>>(mh32, b32, a32, n)));
      k_shift_out<float><<<g3, kBlock, 0, s>>>(a32, in, out, shift, n);
    } else {
      k_shift_out<float><<<g3, kBlock, 0, s>>>(b32, in, out, shift, n);
    }
  } else {
    double2* a64 = static_cast<double2*>(tmp_a);
    MSC_LANES_SWITCH(lanes, (k_spmv<double, LL><<<g1, kBlock, 0, s>>>(m64, in, a64, n)));
    if (kind == MSC_A_MHM) {
      double2* b64 = static_cast<double2*>(tmp_b);
      MSC_LANES_SWITCH(lanes, (k_spmv<double, LL><<<g1, kBlock, 0, s>>>(mh64, a64, b64, n)));
      k_shift_out<double><<<g3, kBlock, 0, s>>>(b64, in, out, shift, n);
    } else {
      k_shift_out<double><<<g3, kBlock, 0, s>>>(a64, in, out, shift, n);
    }
  }
  return hipGetLastError();
}

// ---- operator application without allocation ------------------------------------------
// The two temporaries of the no-allocation apply live in a file-scope device array: each
// GPU the library runs on holds its own copy, until the process ends.  In host code the
// name `scratch` is only a host-side stand-in, so it is never passed to a kernel: the
// array's address on each device comes from hipGetSymbolAddress, looked up once per
// device with that device current, and kept in scratch_addr.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void* scratch_addr[kMaxDevices] = {};
}  // namespace

size_t apply_scratch_bytes(int kind, int prec, int64_t n) {
  // mixed: the complex64 input and one complex64 product (both kinds);
  // FP64: one complex128 product, two for A = M^H M; each temporary 256-byte aligned
  const size_t elem = prec == MSC_PREC_MIXED ? sizeof(float2) : sizeof(double2);
  const int count = (prec == MSC_PREC_MIXED || kind == MSC_A_MHM) ? 2 : 1;
  const size_t one = (elem * size_t(n) + 255) / 256 * 256;
  return one * count;
}

hipError_t noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[device] = p;
  }
  *ptr = scratch_addr[device];
  return hipSuccess;
}

hipError_t launch_apply_noalloc(int kind, int prec, int lanes, int64_t n,
                                const Csr<double2>& m64, const Csr<double2>& mh64,
                                const Csr<float2>& m32, const Csr<float2>& mh32,
                                const double2* in, double2* out, double shift, void* base,
                                hipStream_t s) {
  const size_t need = apply_scratch_bytes(kind, prec, n);
  if (need > kNoAllocScratchBytes) return hipErrorInvalidValue;
  const size_t elem = prec == MSC_PREC_MIXED ? sizeof(float2) : sizeof(double2);
  const size_t one = (elem * size_t(n) + 255) / 256 * 256;
  unsigned char* b = static_cast<unsigned char*>(base);
  return launch_apply(kind, prec, lanes, n, m64, mh64, m32, mh32, in, out, shift, b,
                      b + one, s);
}

}  // namespace msc
