// A different right-hand side per shift (paper: Section 5, eq. linprobgen): initial
// guesses x0_k that leave every shifted system the same residual r0, so that one
// multishift solve of (A + sigma_k) d_k = r0 finishes the family, x_k = x0_k + d_k.
//
// The guesses come from the Newton interpolant of the right-hand sides over the shifts
// (ascending s_0 < ... < s_{m-1}): with the divided differences D_j = b[s_0..s_j] and
// x(s) = sum_j Y_j w_j(s), w_j(s) = prod_{l<j} (s - s_l), the choice
//   Y_{m-2} = D_{m-1},   Y_{j-1} = D_j - (A + s_j) Y_j   (j = m-2 .. 1)
// leaves b(s) - (A + s) x(s) = D_0 - (A + s_0) Y_0 = r0 for every s; x0_k = x(s_k).
// The products with A use the operator's FP64 kernels (launch_apply); the kernels here
// are the elementwise steps.  All FP64.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

namespace {

int osb_grid(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 4 * kMaxGrid) g = 4 * kMaxGrid;
  if (g < 1) g = 1;
  return int(g);
}

// W[j] = b_{orig[j]} for the sorted shifts, then the divided differences in place:
// for each level, W[k] <- (W[k] - W[k-1]) inv[k * m + level], k = m-1 .. level.
__global__ __launch_bounds__(kBlock) void k_osb_divdiff(const double2* __restrict__ B,
                                                        const int* __restrict__ orig,
                                                        const double* __restrict__ inv,
                                                        double2* __restrict__ W, int m, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    for (int j = 0; j < m; ++j) W[int64_t(j) * n + i] = B[int64_t(orig[j]) * n + i];
    // descending k: W[k - 1] still holds the previous level when W[k] is formed
    for (int level = 1; level < m; ++level) {
      for (int k = m - 1; k >= level; --k) {
        const double2 cur = W[int64_t(k) * n + i];
        const double2 prev = W[int64_t(k - 1) * n + i];
        const double c = inv[k * m + level];
        W[int64_t(k) * n + i] = double2{(cur.x - prev.x) * c, (cur.y - prev.y) * c};
      }
    }
  }
}

// y <- y - t
__global__ __launch_bounds__(kBlock) void k_osb_sub(double2* __restrict__ y,
                                                    const double2* __restrict__ t, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const double2 a = y[i], b = t[i];
    y[i] = double2{a.x - b.x, a.y - b.y};
  }
}

// x_{orig[k]} = sum_{j <= min(k, m-2)} w[k * m + j] W[j + 1]   (W[j + 1] holds Y_j)
__global__ __launch_bounds__(kBlock) void k_osb_combine(const double2* __restrict__ W,
                                                        const double* __restrict__ w,
                                                        const int* __restrict__ orig,
                                                        double2* __restrict__ x, int m, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    for (int k = 0; k < m; ++k) {
      double2 acc{0.0, 0.0};
      const int top = k < m - 2 ? k : m - 2;
      for (int j = 0; j <= top; ++j) {
        const double c = w[k * m + j];
        const double2 y = W[int64_t(j + 1) * n + i];
        acc.x = fma(c, y.x, acc.x);
        acc.y = fma(c, y.y, acc.y);
      }
      x[int64_t(orig[k]) * n + i] = acc;
    }
  }
}

// x <- x + d over `count` elements
__global__ __launch_bounds__(kBlock) void k_osb_add(double2* __restrict__ x,
                                                    const double2* __restrict__ d, int64_t count) {
  for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * kBlock) {
    const double2 a = x[i], b = d[i];
    x[i] = double2{a.x + b.x, a.y + b.y};
  }
}

// |v_q|^2 for q < count contiguous vectors of length n: one workgroup per (vector,
// slice); the last workgroup of each vector's slices sums them in a fixed order.
__global__ __launch_bounds__(kBlock) void k_osb_norms(const double2* __restrict__ v, int count,
                                                      int64_t n, int slices, double* partial,
                                                      unsigned* tickets, double* out) {
  const int q = blockIdx.x / slices, sl = blockIdx.x % slices;
  const int64_t per = (n + slices - 1) / slices;
  const int64_t beg = int64_t(sl) * per;
  const int64_t end = beg + per < n ? beg + per : n;
  double acc = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const double2 a = v[int64_t(q) * n + i];
    acc = fma(a.x, a.x, fma(a.y, a.y, acc));
  }
  const double tot = block_sum<kBlock>(acc);
  if (threadIdx.x == 0) store_agent(&partial[blockIdx.x], tot);
  if (!arrive_last(tickets + q * kTicketSite, unsigned(slices), unsigned(sl))) return;
  double s = 0.0;
  for (int k = threadIdx.x; k < slices; k += kBlock) s += load_agent(&partial[q * slices + k]);
  s = block_sum<kBlock>(s);
  if (threadIdx.x == 0) out[q] = s;
  (void)count;
}

}  // namespace

hipError_t launch_osb_divdiff(const double2* B, const int* orig, const double* inv, double2* W,
                              int m, int64_t n, hipStream_t s) {
  k_osb_divdiff<<<osb_grid(n), kBlock, 0, s>>>(B, orig, inv, W, m, n);
  return hipGetLastError();
}

hipError_t launch_osb_sub(double2* y, const double2* t, int64_t n, hipStream_t s) {
  k_osb_sub<<<osb_grid(n), kBlock, 0, s>>>(y, t, n);
  return hipGetLastError();
}

hipError_t launch_osb_combine(const double2* W, const double* w, const int* orig, double2* x,
                              int m, int64_t n, hipStream_t s) {
  k_osb_combine<<<osb_grid(n), kBlock, 0, s>>>(W, w, orig, x, m, n);
  return hipGetLastError();
}

hipError_t launch_osb_add(double2* x, const double2* d, int64_t count, hipStream_t s) {
  k_osb_add<<<osb_grid(count), kBlock, 0, s>>>(x, d, count);
  return hipGetLastError();
}

hipError_t launch_osb_norms(const double2* v, int count, int64_t n, double* partial,
                            unsigned* tickets, double* out, hipStream_t s) {
  // slices per vector: enough workgroups to fill the chip; partial holds count *
  // kOsbSlices doubles and tickets count ticket sites
  int slices = int((n + 4 * kBlock - 1) / (4 * kBlock));
  if (slices > kOsbSlices) slices = kOsbSlices;
  if (slices < 1) slices = 1;
  k_osb_norms<<<count * slices, kBlock, 0, s>>>(v, count, n, slices, partial, tickets, out);
  return hipGetLastError();
}

}  // namespace msc
