// Adjoint support kernels: the collinearity test of the loss gradients g_k, scaling and
// summing of shift solutions, and the gradient with respect to the stored values of M
// (or A).  For L(x_0..x_{ns-1}) with dL/dx_k = g_k and y_k = (A + sigma_k)^{-1} g_k:
//   A = M^H M : dL/dM_e = -sum_k [ (M y_k)_i conj(x_k)_j + (M x_k)_i conj(y_k)_j ]
//   A given  : dL/dA_e = -sum_k (y_k)_i conj(x_k)_j
// for the entry e = (i, j), in torch's convention grad = dL/dRe + i dL/dIm.  The sum
// over shifts is the force shape of the rational hybrid Monte Carlo use of the shifted
// family (Section 2).
#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

namespace {

constexpr int kGramMax = 16;

// For q < kc: re/im of <g_ref, g_q> and |g_q|^2 (three sums per vector).
__global__ __launch_bounds__(kBlock) void k_gram(const double2* gref, const double2* g, int64_t n,
                                                 int kc, double* partial, unsigned* ticket,
                                                 double* out) {
  double acc[3 * kGramMax];
#pragma unroll
  for (int q = 0; q < 3 * kGramMax; ++q) acc[q] = 0.0;
  int64_t beg, end;
  block_range(n, kBlock, beg, end);
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 r = gref[i];
#pragma unroll
    for (int q = 0; q < kGramMax; ++q) {
      if (q < kc) {
        const double2 v = g[int64_t(q) * n + i];
        acc[3 * q] += r.x * v.x + r.y * v.y;       // Re(conj(r) v)
        acc[3 * q + 1] += r.x * v.y - r.y * v.x;   // Im(conj(r) v)
        acc[3 * q + 2] += v.x * v.x + v.y * v.y;
      }
    }
  }
  block_sum_k<kBlock, 3 * kGramMax>(acc);
  if (threadIdx.x == 0) {
    for (int q = 0; q < 3 * kc; ++q) store_agent(&partial[blockIdx.x * 3 * kGramMax + q], acc[q]);
  }
  if (!arrive_last(ticket)) return;
  for (int q = 0; q < 3 * kc; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < int(gridDim.x); b += kBlock) s += load_agent(&partial[b * 3 * kGramMax + q]);
    s = block_sum<kBlock>(s);
    if (threadIdx.x == 0) out[q] = s;
  }
}

// |g_q - c_q gref|^2 for q < kc
__global__ __launch_bounds__(kBlock) void k_diffnorm(const double2* gref, const double2* g,
                                                     const double* c, int64_t n, int kc,
                                                     double* partial, unsigned* ticket, double* out) {
  double acc[kGramMax];
#pragma unroll
  for (int q = 0; q < kGramMax; ++q) acc[q] = 0.0;
  int64_t beg, end;
  block_range(n, kBlock, beg, end);
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 r = gref[i];
#pragma unroll
    for (int q = 0; q < kGramMax; ++q) {
      if (q < kc) {
        const double2 v = g[int64_t(q) * n + i];
        const double dx = v.x - c[q] * r.x, dy = v.y - c[q] * r.y;
        acc[q] += dx * dx + dy * dy;
      }
    }
  }
  block_sum_k<kBlock, kGramMax>(acc);
  if (threadIdx.x == 0) {
    for (int q = 0; q < kc; ++q) store_agent(&partial[blockIdx.x * kGramMax + q], acc[q]);
  }
  if (!arrive_last(ticket)) return;
  for (int q = 0; q < kc; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < int(gridDim.x); b += kBlock) s += load_agent(&partial[b * kGramMax + q]);
    s = block_sum<kBlock>(s);
    if (threadIdx.x == 0) out[q] = s;
  }
}

// y_k <- c_k y_k for every shift (shift-major)
__global__ void k_scale(double2* y, const double* c, int ns, int64_t n) {
  const int64_t total = int64_t(ns) * n;
  for (int64_t idx = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const double ck = c[idx / n];
    y[idx] = double2{ck * y[idx].x, ck * y[idx].y};
  }
}

// out = sum_k y_k
__global__ void k_sum_shifts(const double2* y, int ns, int64_t n, double2* out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    double2 s{0.0, 0.0};
    for (int k = 0; k < ns; ++k) {
      const double2 v = y[int64_t(k) * n + i];
      s.x += v.x;
      s.y += v.y;
    }
    out[i] = s;
  }
}

constexpr int kGradChunk = 4;

// U_q = M x_q and W_q = M y_q for q < kc (FP64), rows split over L lanes.
template <int L>
__global__ __launch_bounds__(kBlock) void k_grad_mv(Csr<double2> m, const double2* x, const double2* y,
                                                    int64_t n, int kc, double2* u, double2* w) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(n, GPB, beg, end);
  for (int64_t row = beg + grp; row < end; row += GPB) {
    double2 au[kGradChunk], aw[kGradChunk];
#pragma unroll
    for (int q = 0; q < kGradChunk; ++q) au[q] = aw[q] = double2{0.0, 0.0};
    for (int32_t e = m.rowptr[row] + lane; e < m.rowptr[row + 1]; e += L) {
      const int32_t c = m.col[e];
      const double2 v = m.val[e];
#pragma unroll
      for (int q = 0; q < kGradChunk; ++q) {
        if (q < kc) {
          cfma<double>(au[q], v, x[int64_t(q) * n + c]);
          cfma<double>(aw[q], v, y[int64_t(q) * n + c]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kGradChunk; ++q) {
      au[q] = group_sum_c<L, double>(au[q]);
      aw[q] = group_sum_c<L, double>(aw[q]);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kGradChunk; ++q) {
        if (q < kc) {
          u[int64_t(q) * n + row] = au[q];
          w[int64_t(q) * n + row] = aw[q];
        }
      }
    }
  }
}

// grad[e] (+)= -sum_q [ W_q[i] conj(x_q[j]) + U_q[i] conj(y_q[j]) ]   (A = M^H M)
// grad[e] (+)= -sum_q  y_q[i] conj(x_q[j])                           (A given)
template <int L, bool MHM>
__global__ __launch_bounds__(kBlock) void k_grad_vals(Csr<double2> m, const double2* x, const double2* y,
                                                      const double2* u, const double2* w, int64_t n,
                                                      int kc, int accumulate, double2* grad) {
  constexpr int GPB = kBlock / L;
  const int lane = threadIdx.x % L, grp = threadIdx.x / L;
  int64_t beg, end;
  block_range(n, GPB, beg, end);
  for (int64_t row = beg + grp; row < end; row += GPB) {
    double2 wi[kGradChunk], ui[kGradChunk];
#pragma unroll
    for (int q = 0; q < kGradChunk; ++q) {
      if (q < kc) {
        wi[q] = MHM ? w[int64_t(q) * n + row] : y[int64_t(q) * n + row];
        ui[q] = MHM ? u[int64_t(q) * n + row] : double2{0.0, 0.0};
      } else {
        wi[q] = ui[q] = double2{0.0, 0.0};
      }
    }
    for (int32_t e = m.rowptr[row] + lane; e < m.rowptr[row + 1]; e += L) {
      const int32_t c = m.col[e];
      double2 g = accumulate ? grad[e] : double2{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kGradChunk; ++q) {
        if (q < kc) {
          const double2 xj = x[int64_t(q) * n + c];
          // - W conj(x)
          g.x -= wi[q].x * xj.x + wi[q].y * xj.y;
          g.y -= wi[q].y * xj.x - wi[q].x * xj.y;
          if (MHM) {
            const double2 yj = y[int64_t(q) * n + c];
            g.x -= ui[q].x * yj.x + ui[q].y * yj.y;
            g.y -= ui[q].y * yj.x - ui[q].x * yj.y;
          }
        }
      }
      grad[e] = g;
    }
  }
}

int grid_g(int64_t items, int per_pass) {
  int64_t g = (items + per_pass - 1) / per_pass;
  if (g > kMaxGrid) g = kMaxGrid;
  if (g < kXcds) g = kXcds;
  return int((g + kXcds - 1) / kXcds * kXcds);
}

#define MSC_GL_SWITCH(LANES, CALL)                       \
  switch (LANES) {                                       \
    case 4: { constexpr int LL = 4; CALL; } break;       \
    case 8: { constexpr int LL = 8; CALL; } break;       \
    case 16: { constexpr int LL = 16; CALL; } break;     \
    case 32: { constexpr int LL = 32; CALL; } break;     \
    default: return hipErrorInvalidValue;                \
  }

}  // namespace

hipError_t launch_gram(const double2* gref, const double2* g, int64_t n, int kc, double* partial,
                       unsigned* ticket, double* out, hipStream_t s) {
  if (kc < 1 || kc > kGramMax) return hipErrorInvalidValue;
  k_gram<<<grid_g(n, kBlock), kBlock, 0, s>>>(gref, g, n, kc, partial, ticket, out);
  return hipGetLastError();
}

hipError_t launch_diffnorm(const double2* gref, const double2* g, const double* d_c, int64_t n,
                           int kc, double* partial, unsigned* ticket, double* out, hipStream_t s) {
  if (kc < 1 || kc > kGramMax) return hipErrorInvalidValue;
  k_diffnorm<<<grid_g(n, kBlock), kBlock, 0, s>>>(gref, g, d_c, n, kc, partial, ticket, out);
  return hipGetLastError();
}

hipError_t launch_scale_shifts(double2* y, const double* d_c, int ns, int64_t n, hipStream_t s) {
  k_scale<<<grid_g(int64_t(ns) * n, kBlock), kBlock, 0, s>>>(y, d_c, ns, n);
  return hipGetLastError();
}

hipError_t launch_sum_shifts(const double2* y, int ns, int64_t n, double2* out, hipStream_t s) {
  k_sum_shifts<<<grid_g(n, kBlock), kBlock, 0, s>>>(y, ns, n, out);
  return hipGetLastError();
}

hipError_t launch_grad_vals(int kind, int lanes, const Csr<double2>& m, const double2* x,
                            const double2* y, int64_t n, int ns, double2* u, double2* w,
                            double2* grad, hipStream_t s) {
  const int g1 = grid_g(n, kBlock / lanes);
  for (int q0 = 0; q0 < ns; q0 += kGradChunk) {
    const int kc = ns - q0 < kGradChunk ? ns - q0 : kGradChunk;
    const double2* xc = x + int64_t(q0) * n;
    const double2* yc = y + int64_t(q0) * n;
    if (kind == MSC_A_MHM) {
      MSC_GL_SWITCH(lanes, (k_grad_mv<LL><<<g1, kBlock, 0, s>>>(m, xc, yc, n, kc, u, w)));
      MSC_GL_SWITCH(lanes, (k_grad_vals<LL, true><<<g1, kBlock, 0, s>>>(m, xc, yc, u, w, n, kc, q0 > 0, grad)));
    } else {
      MSC_GL_SWITCH(lanes, (k_grad_vals<LL, false><<<g1, kBlock, 0, s>>>(m, xc, yc, u, w, n, kc, q0 > 0, grad)));
    }
  }
  return hipGetLastError();
}

}  // namespace msc
