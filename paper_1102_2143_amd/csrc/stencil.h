// Matrix-free staggered operator: the rows of M = m + D and M^H = m - D computed from the
// link field (Stencil in msc_internal.h) instead of a stored matrix, one row per lane.
//
// D v at row 3 s + c reads row c of the four forward links W_mu(s) and column c of the
// four backward links W_mu(s - mu): per row 12 + 12 link values and 24 gathered values,
// like the 24 off-diagonal entries of a sliced ELLPACK row but with no column indices,
// and each link is shared by the three rows of its site and by the neighbour that reads
// it backwards (paper: Section 3, where the library leaves room for a custom linear
// operator kernel in place of the stored matrix when an application warrants one).
#pragma once

#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

// acc += conj(a) * b
template <class R>
__device__ __forceinline__ void cfma_conj(cplx<R>& acc, const cplx<R>& a, const cplx<R>& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// conj(a b - c d)
template <class R>
__device__ __forceinline__ cplx<R> conj_diff(const cplx<R>& a, const cplx<R>& b, const cplx<R>& c,
                                             const cplx<R>& d) {
  const R re = fma(a.x, b.x, fma(-a.y, b.y, fma(-c.x, d.x, c.y * d.y)));
  const R im = fma(a.x, b.y, fma(a.y, b.x, fma(-c.x, d.y, -c.y * d.x)));
  return cplx<R>{re, -im};
}

// Hopping part (D v) of row `row`, with v read through gather(col); the four directions
// are taken DPR at a time, each group's link and vector loads issued before its first
// multiply-add (DPR = 1 where the gather itself reads two vectors).
// LR = 3: every link holds its 9 values.  LR = 2: it holds rows 0 and 1 of W = (eta/2) U
// with U in SU(3), whose third row is conj(u0 x u1); for W that is conj(w0 x w1) / (eta/2)
// = 2 eta conj(w0 x w1), eta = eta_mu(x) the link's sign (equal for the site and its
// backward neighbour in direction mu, since eta_mu does not depend on x_mu).
template <class R, int DPR, int LR, class G>
__device__ __forceinline__ cplx<R> stencil_hop(const Stencil<cplx<R>>& op, int64_t row, G gather) {
  static_assert(DPR == 1 || DPR == 2 || DPR == 4, "directions per round trip");
  static_assert(LR == 2 || LR == 3, "link rows");
  const uint32_t s = uint32_t(row / 3);
  const int c = int(row - 3 * int64_t(s));
  uint32_t rem = s;
  int64_t fwd[4], bwd[4];
  R two_eta[4];
  uint32_t par = 0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const uint32_t L = uint32_t(op.L[mu]);
    const uint32_t q = rem / L;
    const uint32_t xm = rem - q * L;
    rem = q;
    two_eta[mu] = (par & 1u) ? R(-2) : R(2);
    par += xm;
    const int64_t st = op.stride[mu];
    fwd[mu] = xm == L - 1 ? int64_t(s) - int64_t(L - 1) * st : int64_t(s) + st;
    bwd[mu] = xm == 0 ? int64_t(s) + int64_t(L - 1) * st : int64_t(s) - st;
  }
  cplx<R> fw = czero<R>(), bw = czero<R>();
  if constexpr (LR == 2) {
    // per lane: the six link values it needs, at lane-dependent offsets.  Forward, row c
    // of W_mu(x): rows 0 and 1 for c = 2 (whose row is rebuilt), row c twice otherwise.
    // Backward, column c of W_mu(x - mu): (0, c), (1, c) and the four entries of rows 0
    // and 1 in columns c + 1 and c + 2 that give (2, c).
    const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
    const int f0 = c < 2 ? 3 * c : 0, f1 = c < 2 ? 3 * c : 3;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const cplx<R>* __restrict__ wf = op.w + (int64_t(mu) * op.vol + s) * 6;
      const cplx<R>* __restrict__ wb = op.w + (int64_t(mu) * op.vol + bwd[mu]) * 6;
      cplx<R> F[6], gf[3], gb[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        F[j] = wf[f0 + j];
        F[3 + j] = wf[f1 + j];
      }
      const cplx<R> a0 = wb[c], a1 = wb[3 + c];
      const cplx<R> b0 = wb[c1], b1 = wb[3 + c2], d0 = wb[c2], d1 = wb[3 + c1];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        gf[j] = gather(3 * fwd[mu] + j);
        gb[j] = gather(3 * bwd[mu] + j);
      }
      const R te = two_eta[mu];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        cplx<R> r2 = conj_diff<R>(F[j1], F[3 + j2], F[j2], F[3 + j1]);
        r2.x *= te;
        r2.y *= te;
        cfma<R>(fw, c < 2 ? F[j] : r2, gf[j]);
      }
      cplx<R> e2 = conj_diff<R>(b0, b1, d0, d1);
      e2.x *= te;
      e2.y *= te;
      cfma_conj<R>(bw, a0, gb[0]);
      cfma_conj<R>(bw, a1, gb[1]);
      cfma_conj<R>(bw, e2, gb[2]);
    }
  } else {
#pragma unroll
    for (int h = 0; h < 4; h += DPR) {
      cplx<R> uf[DPR][3], ub[DPR][3], gf[DPR][3], gb[DPR][3];
#pragma unroll
      for (int d = 0; d < DPR; ++d) {
        const int mu = h + d;
        const cplx<R>* __restrict__ wf = op.w + (int64_t(mu) * op.vol + s) * 9 + 3 * c;
        const cplx<R>* __restrict__ wb = op.w + (int64_t(mu) * op.vol + bwd[mu]) * 9 + c;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          uf[d][j] = wf[j];
          ub[d][j] = wb[3 * j];
          gf[d][j] = gather(3 * fwd[mu] + j);
          gb[d][j] = gather(3 * bwd[mu] + j);
        }
      }
#pragma unroll
      for (int d = 0; d < DPR; ++d) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          cfma<R>(fw, uf[d][j], gf[d][j]);
          cfma_conj<R>(bw, ub[d][j], gb[d][j]);
        }
      }
    }
  }
  return cplx<R>{fw.x - bw.x, fw.y - bw.y};
}

// Row `row` of M v (sign = +1) or M^H v (sign = -1): m v_row + sign (D v)_row.
template <class R, int DPR, int LR, class G>
__device__ __forceinline__ cplx<R> stencil_row(const Stencil<cplx<R>>& op, int64_t row,
                                               const cplx<R>& v_row, int sign, G gather) {
  const cplx<R> h = stencil_hop<R, DPR, LR>(op, row, gather);
  const R m = R(op.mass);
  cplx<R> o;
  o.x = sign > 0 ? fma(m, v_row.x, h.x) : fma(m, v_row.x, -h.x);
  o.y = sign > 0 ? fma(m, v_row.y, h.y) : fma(m, v_row.y, -h.y);
  return o;
}

}  // namespace msc
