// Matrix-free staggered operator: M = m + D and M^H = m - D computed from the link field
// (Stencil in msc_internal.h) instead of a stored matrix, one lattice site per lane.
//
// D v at site s, colour c, reads row c of the four forward links W_mu(s) and column c of
// the four backward links W_mu(s - mu), and the three colours of the eight neighbours.  A
// lane computes all three colours of its site, so it reads each of its eight links once,
// whole, and each neighbour's three values once (paper: Section 3, where the library
// leaves room for a custom linear operator kernel in place of the stored matrix when an
// application warrants one).
//
// The links are stored value-major: entry k (row-major within the 3 x 3 matrix) of W_mu
// at site s is w[(mu K + k) vol + s], K = 9, or K = 6 when only rows 0 and 1 are kept.
// The 64 lanes of a wave hold 64 consecutive sites, so each of their link loads reads
// one contiguous run of 64 values.
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

// Row 2 of an SU(3) link W = (eta/2) U from its rows 0 and 1 (u[0..2], u[3..5]): the third
// row of U is conj(u0 x u1), so that of W is conj(w0 x w1) / (eta/2) = 2 eta conj(w0 x w1).
// te = 2 eta, equal for a site and its backward neighbour in direction mu (eta_mu does
// not depend on x_mu).
template <class R>
__device__ __forceinline__ void third_row(cplx<R> (&u)[9], R te) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    cplx<R> r2 = conj_diff<R>(u[j1], u[3 + j2], u[j2], u[3 + j1]);
    r2.x *= te;
    r2.y *= te;
    u[6 + j] = r2;
  }
}

// What a wave marching along t (one site per lane, the next site one t-slice further on)
// keeps from one site to the next: the stored entries of the site's t link, which are
// the next site's backward t link, and the values at the site and at its forward t
// neighbour, which are the next site's backward t neighbour and its own values.
template <class R, int LR> struct TCarry {
  cplx<R> u[3 * LR];
  cplx<R> own[3];
  cplx<R> fw[3];
};

// out[c] = m own[c] + sign (D v)_(3 s + c), c = 0, 1, 2, with v read through gather(row)
// and own[c] = v at the site's own rows.  LR: link rows stored (3, or 2 for SU(3) links).
// The sums run over mu = 0..3 and, within a direction, over the neighbour's colours j,
// forward and backward terms apart, in that order.
// CAR: car->u and car->own stand in for the backward t link and the backward t
// neighbour's values, and must hold exactly those (the previous site's t link and values
// when the site lies one t-slice past it, else loaded for the site); on return car->u
// holds this site's t link and car->fw the forward t neighbour's values (car->own is the
// caller's to set).  The arithmetic is the same either way.
template <class R, int LR, bool CAR, class G>
__device__ __forceinline__ void stencil_site_c(const Stencil<cplx<R>>& op, uint32_t s,
                                               const cplx<R> (&own)[3], int sign, G gather,
                                               cplx<R> (&out)[3], TCarry<R, LR>* car) {
  static_assert(LR == 2 || LR == 3, "link rows");
  constexpr int K = 3 * LR;
  // neighbours and the sign mask in 32 bits (the volume is below 2^31, checked at
  // creation)
  const uint32_t vol = uint32_t(op.vol);
  uint32_t rem = s;
  uint32_t fwd[4], bwd[4];
  uint32_t neg = 0;  // bit mu: eta_mu(x) = -1
  uint32_t par = 0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const uint32_t L = uint32_t(op.L[mu]);
    const uint32_t q = rem / L;
    const uint32_t xm = rem - q * L;
    rem = q;
    neg |= (par & 1u) << mu;
    par += xm;
    const uint32_t st = uint32_t(op.stride[mu]);
    fwd[mu] = xm == L - 1 ? s - (L - 1) * st : s + st;
    bwd[mu] = xm == 0 ? s + (L - 1) * st : s - st;
  }
  cplx<R> fw[3], bw[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) fw[c] = bw[c] = czero<R>();
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const cplx<R>* __restrict__ wm = op.w + int64_t(mu) * K * vol;
    cplx<R> U[9], B[9], gf[3], gb[3];
    const bool kept = CAR && mu == 3;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      U[k] = wm[int64_t(k) * vol + s];
      if (kept)
        B[k] = car->u[k];
      else
        B[k] = wm[int64_t(k) * vol + bwd[mu]];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gf[j] = gather(3 * int64_t(fwd[mu]) + j);
      if (kept)
        gb[j] = car->own[j];
      else
        gb[j] = gather(3 * int64_t(bwd[mu]) + j);
    }
    if constexpr (CAR) {
      if (mu == 3) {
#pragma unroll
        for (int k = 0; k < K; ++k) car->u[k] = U[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) car->fw[j] = gf[j];
      }
    }
    if constexpr (LR == 2) {
      const R te = ((neg >> mu) & 1u) ? R(-2) : R(2);
      third_row<R>(U, te);
      third_row<R>(B, te);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        cfma<R>(fw[c], U[3 * c + j], gf[j]);
        cfma_conj<R>(bw[c], B[3 * j + c], gb[j]);
      }
    }
  }
  const R m = R(op.mass);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<R> h{fw[c].x - bw[c].x, fw[c].y - bw[c].y};
    out[c].x = sign > 0 ? fma(m, own[c].x, h.x) : fma(m, own[c].x, -h.x);
    out[c].y = sign > 0 ? fma(m, own[c].y, h.y) : fma(m, own[c].y, -h.y);
  }
}

template <class R, int LR, class G>
__device__ __forceinline__ void stencil_site(const Stencil<cplx<R>>& op, uint32_t s,
                                             const cplx<R> (&own)[3], int sign, G gather,
                                             cplx<R> (&out)[3]) {
  stencil_site_c<R, LR, false>(op, s, own, sign, gather, out,
                               static_cast<TCarry<R, LR>*>(nullptr));
}

}  // namespace msc
