// Multishift BiCGStab (BiCGStab-M) for a general, non-Hermitian sparse A: the family
// (A + sigma_k I) x_k = b (paper: Section 2, eq. linprob) from one BiCGStab sequence of
// the driving matrix B = A + sigma0 I (the paper's second shifted solver, Sections 1
// and 3).  The shifted constants follow from the BiCG polynomials: the shifted BiCG
// residuals are multiples of the driving one (the zeta recurrence of CG-M), and the
// shifted stabilising steps om / (1 + s om) keep the whole shifted residual a multiple
// of the driving one, r_n(s) = (z_n / tau_n) r_n, so every shift is advanced from r_n,
// s_n and r_{n+1} with no extra operator product.
//
// One iteration is four kernels; each reduction is finished by the last workgroup to
// arrive (deterministic fixed-order sum), which also derives the scalars:
//   BV   v = B p,  w^H v          -> al = rho / w^H v; per shift z_{n+1}, al(s)
//   BT   t = B s with s = r - al v formed at each gathered column (and stored for the
//        own row),  t^H s, t^H t  -> om; per shift om(s), tau_{n+1}
//   BR   r' = s - om t,  w^H r', |r'|^2 -> rho', be; per shift be(s), the update
//        coefficients, freezing; halt once every shift has converged
//   BU   every live shift: x(s) += al(s) p(s) + om(s) (z'/tau) s,
//        p(s) <- (z'/tau') r' + be(s) [p(s) - (om(s)/al(s)) ((z/tau) r - (z'/tau) s)];
//        the driving direction p <- r' + be (p - om v)
// Complex scalars are FP64 throughout; the shadow vector is b.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's scaling keeps the quotient finite for any finite non-zero b
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return double2{(a.x + a.y * r) / d, (a.y - a.x * r) / d};
  }
  const double r = b.x / b.y, d = b.x * r + b.y;
  return double2{(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return double2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return double2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }
// acc += conj(a) b
__device__ __forceinline__ void cdot_acc(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
// c += a b
__device__ __forceinline__ void cmad(double2& c, double2 a, double2 b) {
  c.x = fma(a.x, b.x, c.x);
  c.x = fma(-a.y, b.y, c.x);
  c.y = fma(a.x, b.y, c.y);
  c.y = fma(a.y, b.x, c.y);
}

// s = r - al v, written so that the owner of a row and every lane that gathers it form
// the same bits.
__device__ __forceinline__ double2 s_of(double2 r, double2 v, double2 al) {
  double2 s;
  s.x = fma(-al.x, v.x, fma(al.y, v.y, r.x));
  s.y = fma(-al.x, v.y, fma(-al.y, v.x, r.y));
  return s;
}

// One CSR row of A times a vector read through gather(col); L lanes per row, the sum in
// every lane.  All loads of a chunk are issued before its first multiply-add.
constexpr int kBcgChunk = 4;
template <int L, class G>
__device__ __forceinline__ double2 row_f(const Csr<double2>& m, int64_t row, int lane, G gather) {
  const int32_t beg = m.rowptr[row], end = m.rowptr[row + 1];
  double2 acc{0.0, 0.0};
  for (int32_t base = beg; base < end; base += kBcgChunk * L) {
    int32_t c[kBcgChunk];
    double2 v[kBcgChunk], xv[kBcgChunk];
#pragma unroll
    for (int u = 0; u < kBcgChunk; ++u) {
      const int32_t j = base + lane + u * L;
      const bool ok = j < end;
      c[u] = ok ? m.col[j] : 0;
      v[u] = ok ? m.val[j] : double2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kBcgChunk; ++u) xv[u] = gather(c[u]);
#pragma unroll
    for (int u = 0; u < kBcgChunk; ++u) cmad(acc, v[u], xv[u]);
  }
  return group_sum_c<L, double>(acc);
}

// The last workgroup's fixed-order sum of `count` partials (component k of `stride`).
__device__ __forceinline__ double bcg_sum(const double* partial, int count, int stride, int k) {
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

// Store this workgroup's four partial components; returns true in the last workgroup,
// where tot[0..3] then hold the grid sums (valid in thread 0, broadcast through LDS).
__device__ bool bcg_reduce(const BcgArgs& a, double c0, double c1, double c2, double c3,
                           double (&tot)[4]) {
  const double v[4] = {c0, c1, c2, c3};
  double bs[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) bs[k] = block_sum<kBlock>(v[k]);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) store_agent(&a.partial[blockIdx.x * 4 + k], bs[k]);
  }
  if (!arrive_last(a.tickets)) return false;
  __shared__ double sh[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double t = bcg_sum(a.partial, gridDim.x, 4, k);
    if (threadIdx.x == 0) sh[k] = t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) tot[k] = sh[k];
  return true;
}

__device__ __forceinline__ void bcg_halt(BcgState* st, int status) {
  st->status = status;
  st->halt = 1;
}

// ---- initialisation: r = p = b, p(s) = b, x(s) = 0, rho = |b|^2 ------------------------
__global__ __launch_bounds__(kBlock) void k_bcg_init(BcgArgs a) {
  BcgState* st = a.st;
  const int ns = a.ns;
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 bv = a.b[i];
    a.r[0][i] = bv;
    a.p[i] = bv;
    for (int j = 0; j < ns; ++j) {
      a.pk[int64_t(j) * a.n + i] = bv;
      a.x[int64_t(st->orig[j]) * a.n + i] = double2{0.0, 0.0};
    }
    acc += cabs2(bv);
  }
  double tot[4];
  if (!bcg_reduce(a, acc, 0.0, 0.0, 0.0, tot)) return;
  if (threadIdx.x == 0) {
    st->bnorm2 = tot[0];
    st->rho = double2{tot[0], 0.0};
    st->eps2 = st->eps2 * tot[0];  // the host stored tol^2
    if (!(tot[0] > 0.0) || !isfinite(tot[0])) bcg_halt(st, isfinite(tot[0]) ? 0 : 1);
  }
}

// ---- BV: v = B p and w^H v; al and the shifted BiCG constants --------------------------
template <int L>
__global__ __launch_bounds__(kBlock) void k_bcg_v(BcgArgs a) {
  BcgState* st = a.st;
  if (st->halt) return;
  const double sigma0 = st->sigma0;
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double2 acc{0.0, 0.0};
  const double2* __restrict__ p = a.p;
  for (int64_t row = beg + grp; row < end; row += GPB) {
    double2 q = row_f<L>(a.m, row, lane, [&](int32_t c) { return p[c]; });
    const double2 pr = p[row];
    q.x = fma(sigma0, pr.x, q.x);
    q.y = fma(sigma0, pr.y, q.y);
    if (lane == 0) {
      a.v[row] = q;
      cdot_acc(acc, a.b[row], q);
    }
  }
  double tot[4];
  if (!bcg_reduce(a, acc.x, acc.y, 0.0, 0.0, tot)) return;
  const int j = threadIdx.x;
  // rotate the shifted state of the previous iteration, then z_{n+1} and al(s)
  if (j < a.ns) {
    if (st->rotate && st->active[j]) {
      st->z_old[j] = st->z[j];
      st->z[j] = st->z_new[j];
      st->tau[j] = st->tau_new[j];
    }
    if (st->rotate) st->active[j] = st->active_next[j];
  }
  __syncthreads();
  const double2 wv{tot[0], tot[1]};
  const bool ok = cfinite(wv) && (wv.x != 0.0 || wv.y != 0.0);
  const double2 al = ok ? cdiv(st->rho, wv) : double2{0.0, 0.0};
  if (ok && j < a.ns && st->active[j]) {
    const double2 z = st->z[j], zo = st->z_old[j];
    const double2 alp = st->al_prev, bep = st->be_prev;
    const double s = st->s[j];
    // z' = z zo alp / (al bep (zo - z) + zo alp (1 + s al))
    const double2 one_sal{1.0 + s * al.x, s * al.y};
    const double2 den = cadd(cmul(cmul(al, bep), csub(zo, z)), cmul(cmul(zo, alp), one_sal));
    const double2 zn = cdiv(cmul(cmul(z, zo), alp), den);
    st->z_new[j] = zn;
    st->al_s[j] = cdiv(cmul(al, zn), z);
  }
  if (j == 0) {
    st->rotate = 0;
    if (!ok) {
      bcg_halt(st, 1);
    } else {
      st->alpha = al;
    }
  }
}

// ---- BT: t = B s with s = r - al v formed at each gathered column; t^H s, t^H t -------
template <int L>
__global__ __launch_bounds__(kBlock) void k_bcg_t(BcgArgs a) {
  BcgState* st = a.st;
  if (st->halt) return;
  const double sigma0 = st->sigma0;
  const double2 al = st->alpha;
  const double2* __restrict__ r = a.r[a.par];
  const double2* __restrict__ v = a.v;
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(a.n, GPB, beg, end);
  double2 ts{0.0, 0.0};
  double tt = 0.0;
  for (int64_t row = beg + grp; row < end; row += GPB) {
    double2 q = row_f<L>(a.m, row, lane, [&](int32_t c) { return s_of(r[c], v[c], al); });
    const double2 sr = s_of(r[row], v[row], al);
    q.x = fma(sigma0, sr.x, q.x);
    q.y = fma(sigma0, sr.y, q.y);
    if (lane == 0) {
      a.s[row] = sr;
      a.t[row] = q;
      cdot_acc(ts, q, sr);
      tt += cabs2(q);
    }
  }
  double tot[4];
  if (!bcg_reduce(a, ts.x, ts.y, tt, 0.0, tot)) return;
  const int j = threadIdx.x;
  const double2 tsum{tot[0], tot[1]};
  const bool ok = tot[2] > 0.0 && isfinite(tot[2]) && cfinite(tsum);
  const double2 om = ok ? double2{tsum.x / tot[2], tsum.y / tot[2]} : double2{0.0, 0.0};
  bool bad = !ok;
  if (ok && j < a.ns && st->active[j]) {
    const double s = st->s[j];
    const double2 g{1.0 + s * om.x, s * om.y};
    if (g.x == 0.0 && g.y == 0.0) {
      bad = true;
    } else {
      st->om_s[j] = cdiv(om, g);
      st->tau_new[j] = cmul(st->tau[j], g);
    }
  }
  __shared__ int any_bad;
  if (j == 0) any_bad = 0;
  __syncthreads();
  if (bad) atomicOr(&any_bad, 1);
  __syncthreads();
  if (j == 0) {
    if (any_bad)
      bcg_halt(st, 1);
    else
      st->omega = om;
  }
}

// ---- BR: r' = s - om t; w^H r', |r'|^2; be, per-shift coefficients, freezing ---------
__global__ __launch_bounds__(kBlock) void k_bcg_r(BcgArgs a, int launch) {
  BcgState* st = a.st;
  if (st->halt) return;
  const double2 om = st->omega;
  double2* __restrict__ rn = a.r[a.par ^ 1];
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  double2 wr{0.0, 0.0};
  double rr = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 sv = a.s[i], tv = a.t[i];
    double2 nv;
    nv.x = fma(-om.x, tv.x, fma(om.y, tv.y, sv.x));
    nv.y = fma(-om.x, tv.y, fma(-om.y, tv.x, sv.y));
    rn[i] = nv;
    cdot_acc(wr, a.b[i], nv);
    rr += cabs2(nv);
  }
  double tot[4];
  if (!bcg_reduce(a, wr.x, wr.y, rr, 0.0, tot)) return;
  const int j = threadIdx.x;
  const double2 rho_new{tot[0], tot[1]};
  const double R = tot[2];
  const double2 al = st->alpha;
  const bool rho_ok = rho_new.x != 0.0 || rho_new.y != 0.0;
  const bool om_ok = om.x != 0.0 || om.y != 0.0;
  // be = (rho' / rho)(al / om); a vanishing rho' or om ends the sequence after this step
  const double2 be = (rho_ok && om_ok) ? cmul(cdiv(rho_new, st->rho), cdiv(al, om))
                                       : double2{0.0, 0.0};
  int still = 0;
  if (j < a.ns) {
    const int act = st->active[j];
    int nxt = act;
    if (act) {
      const double2 z = st->z[j], zn = st->z_new[j], tau = st->tau[j], taun = st->tau_new[j];
      const double2 als = st->al_s[j], oms = st->om_s[j];
      const double2 c1 = cdiv(zn, tau);              // s_n(s) = c1 s_n
      const double2 c2 = cdiv(zn, taun);             // r_{n+1}(s) = c2 r_{n+1}
      const double2 c3 = cdiv(z, tau);               // r_n(s) = c3 r_n
      const double2 ratio = cdiv(zn, z);
      const double2 bes = cmul(be, cmul(ratio, ratio));
      const double2 q = cmul(bes, cdiv(oms, als));
      BcgCoef& cf = st->cf[j];
      cf.xp = als;                 // x(s) += xp p(s) + xs s
      cf.xs = cmul(oms, c1);
      cf.pr = c2;                  // p(s) <- pr r' + pp p(s) + po r + ps s
      cf.pp = bes;
      cf.po = double2{-(q.x * c3.x - q.y * c3.y), -(q.x * c3.y + q.y * c3.x)};
      cf.ps = cmul(q, c1);
      // this shift's residual after the step: |c2|^2 |r'|^2
      const double res2 = cabs2(c2) * R;
      if (res2 <= st->eps2) {
        nxt = 0;
        st->freeze_iter[j] = st->iter + 1;
      }
      if (!(isfinite(res2))) nxt = 0;
    }
    st->active_next[j] = nxt;
    still = nxt;
  }
  const bool any_live = __syncthreads_or(still);
  if (j == 0) {
    const bool finite = isfinite(R) && cfinite(rho_new);
    st->beta = be;
    st->al_prev = al;
    st->be_prev = be;
    st->rho = rho_new;
    st->R = R;
    st->iter += 1;
    st->rotate = 1;
    st->upd_launch = launch;  // BU of this launch applies the step
    if (!finite) {
      bcg_halt(st, 1);
    } else if (!any_live || !rho_ok || !om_ok || st->iter >= st->max_iter) {
      st->halt = 1;
    }
  }
}

// ---- BU: the step of every live shift and the driving direction ----------------------
__global__ __launch_bounds__(kBlock) void k_bcg_u(BcgArgs a, int launch) {
  BcgState* st = a.st;
  if (st->upd_launch != launch) return;
  __shared__ BcgCoef cf[kMaxShifts];
  __shared__ int64_t xo[kMaxShifts];
  __shared__ int64_t po[kMaxShifts];
  __shared__ int nlive;
  if (threadIdx.x == 0) {
    int c = 0;
    for (int j = 0; j < a.ns; ++j) {
      if (st->active[j]) {
        cf[c] = st->cf[j];
        xo[c] = int64_t(st->orig[j]) * a.n;
        po[c] = int64_t(j) * a.n;
        ++c;
      }
    }
    nlive = c;
  }
  __syncthreads();
  const double2 be = st->beta, om = st->omega;
  const double2* __restrict__ r0 = a.r[a.par];
  const double2* __restrict__ r1 = a.r[a.par ^ 1];
  const int live = nlive;
  int64_t beg, end;
  block_range(a.n, kBlock, beg, end);
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 rv = r0[i], sv = a.s[i], rnv = r1[i];
    for (int c = 0; c < live; ++c) {
      double2* __restrict__ xj = a.x + xo[c];
      double2* __restrict__ pj = a.pk + po[c];
      const double2 pv = pj[i];
      double2 xv = xj[i];
      cmad(xv, cf[c].xp, pv);
      cmad(xv, cf[c].xs, sv);
      xj[i] = xv;
      double2 np{0.0, 0.0};
      cmad(np, cf[c].pr, rnv);
      cmad(np, cf[c].pp, pv);
      cmad(np, cf[c].po, rv);
      cmad(np, cf[c].ps, sv);
      pj[i] = np;
    }
    // driving direction p <- r' + be (p - om v)
    const double2 pv = a.p[i], vv = a.v[i];
    double2 d = pv;
    d.x = fma(-om.x, vv.x, fma(om.y, vv.y, d.x));
    d.y = fma(-om.x, vv.y, fma(-om.y, vv.x, d.y));
    double2 np = rnv;
    cmad(np, be, d);
    a.p[i] = np;
  }
}

// Workgroups for n items, rows_per_pass at a time: one pass each up to kMaxGrid, a
// multiple of the XCD count.
int bcg_grid(int64_t n, int rows_per_pass) {
  int64_t g = (n + rows_per_pass - 1) / rows_per_pass;
  if (g > kMaxGrid) g = kMaxGrid;
  if (g < kXcds) g = kXcds;
  g = (g + kXcds - 1) / kXcds * kXcds;
  if (g > kMaxGrid) g = kMaxGrid;
  return int(g);
}

}  // namespace

hipError_t launch_bcg_init(const BcgArgs& a, hipStream_t s) {
  const int g = bcg_grid(a.n, kBlock);
  k_bcg_init<<<g, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_bcg_iteration(const BcgArgs& args, int launch, hipStream_t s) {
  BcgArgs a = args;
  const int g1 = bcg_grid(a.n, kBlock / a.lanes);
  const int g3 = bcg_grid(a.n, kBlock);
  a.par = launch & 1;
  switch (a.lanes) {
    case 4: k_bcg_v<4><<<g1, kBlock, 0, s>>>(a); k_bcg_t<4><<<g1, kBlock, 0, s>>>(a); break;
    case 8: k_bcg_v<8><<<g1, kBlock, 0, s>>>(a); k_bcg_t<8><<<g1, kBlock, 0, s>>>(a); break;
    case 16: k_bcg_v<16><<<g1, kBlock, 0, s>>>(a); k_bcg_t<16><<<g1, kBlock, 0, s>>>(a); break;
    case 32: k_bcg_v<32><<<g1, kBlock, 0, s>>>(a); k_bcg_t<32><<<g1, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  k_bcg_r<<<g3, kBlock, 0, s>>>(a, launch);
  k_bcg_u<<<g3, kBlock, 0, s>>>(a, launch);
  return hipGetLastError();
}

}  // namespace msc
