// Operator set-up on the device: CSR validation, index and value conversions, and the
// conjugate transpose M^H (counting sort by column, then a per-row sort so the result
// is deterministic), and the sliced ELLPACK copies the iteration SpMVs read.  Runs once
// per operator (the values again after an update); not on the iteration path.
#include <algorithm>
#include <vector>

#include "dev_common.h"
#include "msc_internal.h"

namespace msc {

namespace {

constexpr int kSetupBlock = 256;

inline int blocks_for(int64_t items, int per_block = kSetupBlock, int cap = 65535 * 8) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return int(b);
}

// err bits: 1 rowptr[0] != 0, 2 rowptr decreasing, 4 rowptr[n] != nnz, 8 col out of range
__global__ void k_validate_rowptr(const int64_t* __restrict__ rowptr, int64_t n, int64_t nnz,
                                  int* __restrict__ err) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t a = rowptr[i], b = rowptr[i + 1];
    if (b < a) atomicOr(err, 2);
    if (i == 0 && a != 0) atomicOr(err, 1);
    if (i == n - 1 && b != nnz) atomicOr(err, 4);
  }
}

__global__ void k_validate_col(const int32_t* __restrict__ col, int64_t n, int64_t nnz,
                               int* __restrict__ err) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nnz;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int32_t c = col[e];
    if (c < 0 || int64_t(c) >= n) atomicOr(err, 8);
  }
}

// Row lengths of a CSR matrix in 8 buckets (0, 1, 2-3, 4-7, ..., 32-63, >= 64 entries):
// one LDS histogram per workgroup, added to hist[8].
__global__ void k_row_hist(const int32_t* __restrict__ rowptr, int64_t n,
                           unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[8];
  if (threadIdx.x < 8) h[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int len = rowptr[i + 1] - rowptr[i];
    const int bkt = len <= 0 ? 0 : min(7, 32 - __clz(len));
    atomicAdd(&h[bkt], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 8 && h[threadIdx.x] != 0u)
    atomicAdd(&hist[threadIdx.x], static_cast<unsigned long long>(h[threadIdx.x]));
}

__global__ void k_rowptr_to32(const int64_t* __restrict__ in, int32_t* __restrict__ out,
                              int64_t count) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = int32_t(in[i]);
}

__global__ void k_cast_vals(const double2* __restrict__ in, float2* __restrict__ out,
                            int64_t count) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    out[i] = float2{float(in[i].x), float(in[i].y)};
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_count_cols(const int32_t* __restrict__ col, int64_t nnz,
                             int32_t* __restrict__ counts) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nnz;
       e += int64_t(gridDim.x) * blockDim.x)
    atomicAdd(&counts[col[e]], 1);
}

// Exclusive scan in three passes: per-block scan of 1024 items, a single-block scan of
// the block totals, then the add-back.
constexpr int kScanItems = 4;
constexpr int kScanTile = kSetupBlock * kScanItems;

__global__ void k_scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                             int64_t count, int32_t* __restrict__ tile_sums) {
  __shared__ int32_t sh[kSetupBlock];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int32_t v[kScanItems];
  int32_t local = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = (base + q < count) ? in[base + q] : 0;
    local += v[q];
  }
  sh[threadIdx.x] = local;
  __syncthreads();
  for (int off = 1; off < kSetupBlock; off <<= 1) {
    const int32_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - local;  // exclusive prefix of this thread
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < count) out[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == kSetupBlock - 1) tile_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void k_scan_tile_sums(int32_t* __restrict__ sums, int64_t ntiles) {
  __shared__ int32_t sh[kSetupBlock];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < ntiles; base += kSetupBlock) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = i < ntiles ? sums[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kSetupBlock; off <<= 1) {
      const int32_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < ntiles) sums[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kSetupBlock - 1) carry += sh[threadIdx.x];
    __syncthreads();
  }
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t count,
                           const int32_t* __restrict__ tile_sums) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  const int32_t add = tile_sums[blockIdx.x];
  for (int q = threadIdx.x; q < kScanTile; q += kSetupBlock)
    if (base + q < count) out[base + q] += add;
}

__global__ void k_scatter_adjoint(const int32_t* __restrict__ rowptr,
                                  const int32_t* __restrict__ col, int64_t n,
                                  int32_t* __restrict__ cursor, int32_t* __restrict__ col_h,
                                  int32_t* __restrict__ perm_h) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int32_t pos = atomicAdd(&cursor[col[e]], 1);
      col_h[pos] = int32_t(i);
      perm_h[pos] = e;
    }
  }
}

// Insertion sort of each row of M^H by (column, source entry): rows are short.
__global__ void k_sort_rows(const int32_t* __restrict__ rowptr_h, int64_t n,
                            int32_t* __restrict__ col_h, int32_t* __restrict__ perm_h) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t beg = rowptr_h[i], end = rowptr_h[i + 1];
    for (int32_t a = beg + 1; a < end; ++a) {
      const int32_t c = col_h[a], pe = perm_h[a];
      int32_t b = a - 1;
      while (b >= beg && (col_h[b] > c || (col_h[b] == c && perm_h[b] > pe))) {
        col_h[b + 1] = col_h[b];
        perm_h[b + 1] = perm_h[b];
        --b;
      }
      col_h[b + 1] = c;
      perm_h[b + 1] = pe;
    }
  }
}

__global__ void k_adjoint_vals(const int32_t* __restrict__ perm_h, const double2* __restrict__ v,
                               double2* __restrict__ vh64, float2* __restrict__ vh32,
                               int64_t nnz) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nnz;
       e += int64_t(gridDim.x) * blockDim.x) {
    const double2 a = v[perm_h[e]];
    vh64[e] = double2{a.x, -a.y};
    vh32[e] = float2{float(a.x), float(-a.y)};
  }
}

// ---- sliced ELLPACK copy ------------------------------------------------------------
// One thread per row slot of a slice (slots past n belong to the last, partial slice).
// Pairs of off-diagonal entries each slice needs: the wavefront maximum of its rows.
__global__ void k_sell_pairs(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             int64_t n, int64_t nslices, int32_t* __restrict__ pairs) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  int cnt = 0;
  if (i < n)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) cnt += col[e] != int32_t(i);
#pragma unroll
  for (int off = kSlice / 2; off > 0; off >>= 1) {
    const int o = __shfl_xor(cnt, off, kSlice);
    cnt = o > cnt ? o : cnt;
  }
  const int64_t sl = i / kSlice;
  if ((i % kSlice) == 0 && sl < nslices) pairs[sl] = (cnt + 1) / 2;
}

// Scatter each row into its slice: off-diagonal entries in CSR order, padding with the
// row's own column and value 0, diagonal entries summed into diag.
__global__ void k_sell_fill(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double2* __restrict__ val, int64_t n, int64_t nslices,
                            const int32_t* __restrict__ cptr, int32_t* __restrict__ scol,
                            double2* __restrict__ sv64, float2* __restrict__ sv32,
                            double2* __restrict__ d64, float2* __restrict__ d32) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t sl = i / kSlice;
  if (sl >= nslices) return;
  const int lane = int(i % kSlice);
  const int64_t base = int64_t(cptr[sl]) * (2 * kSlice) + 2 * lane;
  const int width = 2 * (cptr[sl + 1] - cptr[sl]);
  int k = 0;
  if (i < n) {
    double2 d{0.0, 0.0};
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int32_t c = col[e];
      const double2 v = val[e];
      if (c == int32_t(i)) {
        d.x += v.x;
        d.y += v.y;
        continue;
      }
      const int64_t at = base + int64_t(k >> 1) * (2 * kSlice) + (k & 1);
      scol[at] = c;
      sv64[at] = v;
      sv32[at] = float2{float(v.x), float(v.y)};
      ++k;
    }
    d64[i] = d;
    d32[i] = float2{float(d.x), float(d.y)};
  }
  // padding points at the row itself (slots past n: at the last row), so that it stays
  // inside the column span of its neighbours
  const int32_t pad = int32_t(i < n ? i : n - 1);
  for (; k < width; ++k) {
    const int64_t at = base + int64_t(k >> 1) * (2 * kSlice) + (k & 1);
    scol[at] = pad;
    sv64[at] = double2{0.0, 0.0};
    sv32[at] = float2{0.f, 0.f};
  }
}

// Narrow columns of a built copy: one wavefront per slice.  For each pair column and
// entry position the wavefront minimum is the base and each lane keeps its 16-bit offset;
// *wide is set when some span reaches 2^16 (the narrow copy is then unusable).
__global__ void __launch_bounds__(kSlice) k_sell_narrow(const int32_t* __restrict__ cptr,
                                                      const int32_t* __restrict__ scol,
                                                      uint32_t* __restrict__ col16,
                                                      int32_t* __restrict__ cbase,
                                                      int* __restrict__ wide) {
  const int64_t sl = blockIdx.x;
  const int lane = int(threadIdx.x);
  const int32_t c1 = cptr[sl + 1];
  for (int32_t c = cptr[sl]; c < c1; ++c) {
    const int64_t q = int64_t(c) * kSlice + lane;
    const int32_t e0 = scol[2 * q], e1 = scol[2 * q + 1];
    int32_t lo0 = e0, hi0 = e0, lo1 = e1, hi1 = e1;
#pragma unroll
    for (int off = kSlice / 2; off > 0; off >>= 1) {
      lo0 = min(lo0, __shfl_xor(lo0, off, kSlice));
      hi0 = max(hi0, __shfl_xor(hi0, off, kSlice));
      lo1 = min(lo1, __shfl_xor(lo1, off, kSlice));
      hi1 = max(hi1, __shfl_xor(hi1, off, kSlice));
    }
    if (lane == 0 && (hi0 - lo0 > 0xffff || hi1 - lo1 > 0xffff)) *wide = 1;
    col16[q] = uint32_t(e0 - lo0) | (uint32_t(e1 - lo1) << 16);
    if (lane == 0) {
      cbase[2 * int64_t(c)] = lo0;
      cbase[2 * int64_t(c) + 1] = lo1;
    }
  }
}

}  // namespace

hipError_t launch_validate_csr(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                               int* d_err, hipStream_t s) {
  k_validate_rowptr<<<blocks_for(n), kSetupBlock, 0, s>>>(rowptr, n, nnz, d_err);
  if (nnz > 0) k_validate_col<<<blocks_for(nnz), kSetupBlock, 0, s>>>(col, n, nnz, d_err);
  return hipGetLastError();
}

hipError_t launch_row_hist(const int32_t* rowptr, int64_t n, unsigned long long* hist, hipStream_t s) {
  hipError_t e = hipMemsetAsync(hist, 0, 8 * sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  k_row_hist<<<blocks_for(n), kSetupBlock, 0, s>>>(rowptr, n, hist);
  return hipGetLastError();
}

hipError_t launch_rowptr_to32(const int64_t* in, int32_t* out, int64_t n, hipStream_t s) {
  k_rowptr_to32<<<blocks_for(n + 1), kSetupBlock, 0, s>>>(in, out, n + 1);
  return hipGetLastError();
}

hipError_t launch_cast_vals(const double2* in, float2* out, int64_t nnz, hipStream_t s) {
  if (nnz > 0) k_cast_vals<<<blocks_for(nnz), kSetupBlock, 0, s>>>(in, out, nnz);
  return hipGetLastError();
}

hipError_t build_adjoint(const int32_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                         int32_t* rowptr_h, int32_t* col_h, int32_t* perm_h, hipStream_t s) {
  const int64_t count = n + 1;
  const int64_t ntiles = (count + kScanTile - 1) / kScanTile;
  int32_t* counts = nullptr;
  int32_t* tile_sums = nullptr;
  hipError_t e = hipMalloc(&counts, sizeof(int32_t) * (count + n));
  if (e != hipSuccess) return e;
  e = hipMalloc(&tile_sums, sizeof(int32_t) * ntiles);
  if (e != hipSuccess) {
    (void)hipFree(counts);
    return e;
  }
  int32_t* cursor = counts + count;
  k_fill_i32<<<blocks_for(count), kSetupBlock, 0, s>>>(counts, count, 0);
  if (nnz > 0) k_count_cols<<<blocks_for(nnz), kSetupBlock, 0, s>>>(col, nnz, counts);
  k_scan_tiles<<<int(ntiles), kSetupBlock, 0, s>>>(counts, rowptr_h, count, tile_sums);
  k_scan_tile_sums<<<1, kSetupBlock, 0, s>>>(tile_sums, ntiles);
  k_scan_add<<<int(ntiles), kSetupBlock, 0, s>>>(rowptr_h, count, tile_sums);
  e = hipMemcpyAsync(cursor, rowptr_h, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) {
    k_scatter_adjoint<<<blocks_for(n), kSetupBlock, 0, s>>>(rowptr, col, n, cursor, col_h, perm_h);
    k_sort_rows<<<blocks_for(n), kSetupBlock, 0, s>>>(rowptr_h, n, col_h, perm_h);
    e = hipGetLastError();
  }
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(counts);
  (void)hipFree(tile_sums);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_adjoint_vals(const int32_t* perm_h, const double2* val64, double2* val64_h,
                               float2* val32_h, int64_t nnz, hipStream_t s) {
  if (nnz > 0)
    k_adjoint_vals<<<blocks_for(nnz), kSetupBlock, 0, s>>>(perm_h, val64, val64_h, val32_h, nnz);
  return hipGetLastError();
}

void free_sell(SellStore& m) {
  for (void* q : {static_cast<void*>(m.cptr), static_cast<void*>(m.col), static_cast<void*>(m.val64),
                  static_cast<void*>(m.val32), static_cast<void*>(m.diag64),
                  static_cast<void*>(m.diag32), static_cast<void*>(m.col16),
                  static_cast<void*>(m.cbase)})
    if (q) (void)hipFree(q);
  m = SellStore{};
}

hipError_t refill_sell(const int32_t* rowptr, const int32_t* col, const double2* val64, int64_t n,
                       const SellStore& m, hipStream_t s) {
  const int64_t slots = m.nslices * kSlice;
  k_sell_fill<<<dim3(unsigned((slots + kSetupBlock - 1) / kSetupBlock)), kSetupBlock, 0, s>>>(
      rowptr, col, val64, n, m.nslices, m.cptr, m.col, m.val64, m.val32, m.diag64, m.diag32);
  return hipGetLastError();
}

hipError_t build_sell(const int32_t* rowptr, const int32_t* col, const double2* val64, int64_t n,
                      int64_t nnz, SellStore& m, bool* built, hipStream_t s) {
  *built = false;
  free_sell(m);
  const int64_t nslices = (n + kSlice - 1) / kSlice;
  const int64_t slots = nslices * kSlice;
  const unsigned blocks = unsigned((slots + kSetupBlock - 1) / kSetupBlock);
  int32_t* pairs = nullptr;
  hipError_t e = hipMalloc(&pairs, sizeof(int32_t) * nslices);
  if (e != hipSuccess) return e;
  k_sell_pairs<<<dim3(blocks), kSetupBlock, 0, s>>>(rowptr, col, n, nslices, pairs);
  std::vector<int32_t> h(size_t(nslices) + 1, 0);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data() + 1, pairs, sizeof(int32_t) * nslices,
                                          hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(pairs);
  if (e != hipSuccess) return e;
  int64_t total = 0;
  bool uniform = true;
  for (int64_t q = 1; q <= nslices; ++q) {
    uniform = uniform && h[q] == h[1];
    total += h[q];
    if (total >= (int64_t(1) << 31)) return hipSuccess;  // offsets would not fit: keep CSR
    h[q] = int32_t(total);
  }
  const double sell_slots = double(total) * 2.0 * kSlice;
  if (sell_slots > 1.5 * double(nnz) + 2.0 * kSlice * double(nslices)) return hipSuccess;
  m.nslices = nslices;
  m.pairs = total;
  m.wp = uniform ? h[1] : 0;
  const size_t cells = size_t(total) * 2 * kSlice;
  if ((e = hipMalloc(&m.cptr, sizeof(int32_t) * (nslices + 1))) != hipSuccess ||
      (e = hipMalloc(&m.col, sizeof(int32_t) * (cells ? cells : 1))) != hipSuccess ||
      (e = hipMalloc(&m.val64, sizeof(double2) * (cells ? cells : 1))) != hipSuccess ||
      (e = hipMalloc(&m.val32, sizeof(float2) * (cells ? cells : 1))) != hipSuccess ||
      (e = hipMalloc(&m.diag64, sizeof(double2) * n)) != hipSuccess ||
      (e = hipMalloc(&m.diag32, sizeof(float2) * n)) != hipSuccess) {
    free_sell(m);
    return e;
  }
  e = hipMemcpyAsync(m.cptr, h.data(), sizeof(int32_t) * (nslices + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = refill_sell(rowptr, col, val64, n, m, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_sell(m);
    return e;
  }
  *built = true;
  if (total == 0) return hipSuccess;
  // narrow columns: kept only when every span fits
  int* wide = nullptr;
  if ((e = hipMalloc(&m.col16, sizeof(uint32_t) * total * kSlice)) != hipSuccess ||
      (e = hipMalloc(&m.cbase, sizeof(int32_t) * 2 * total)) != hipSuccess ||
      (e = hipMalloc(&wide, sizeof(int))) != hipSuccess) {
    if (wide) (void)hipFree(wide);
    free_sell(m);
    *built = false;
    return e;
  }
  int h_wide = 0;
  e = hipMemsetAsync(wide, 0, sizeof(int), s);
  if (e == hipSuccess) {
    k_sell_narrow<<<dim3(unsigned(nslices)), kSlice, 0, s>>>(m.cptr, m.col, m.col16, m.cbase, wide);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h_wide, wide, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(wide);
  if (e != hipSuccess) {
    free_sell(m);
    *built = false;
    return e;
  }
  if (h_wide) {
    (void)hipFree(m.col16);
    (void)hipFree(m.cbase);
    m.col16 = nullptr;
    m.cbase = nullptr;
  }
  return hipSuccess;
}

// ---- matrix-free staggered operator --------------------------------------------------
namespace {

// w = eta_mu(x)/2 U_mu(x) (complex128 and complex64), stored value-major: entry k of the
// link at (mu, s), links[(mu vol + s) 9 + k], goes to w[(mu 9 + k) vol + s].  One thread
// per stored value.
__global__ void k_stencil_links(const double2* __restrict__ links, Stencil<double2> geo,
                                double2* __restrict__ w64, float2* __restrict__ w32) {
  const int64_t vol = geo.vol, total = 4 * vol * 9;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t mk = i / vol;  // mu 9 + k
    const int64_t site = i - mk * vol;
    const int mu = int(mk / 9), k = int(mk - 9 * mu);
    // eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1})
    int64_t rem = site;
    int parity = 0;
    for (int nu = 0; nu < mu; ++nu) {
      parity += int(rem % geo.L[nu]);
      rem /= geo.L[nu];
    }
    const double h = (parity & 1) ? -0.5 : 0.5;
    const double2 u = links[(int64_t(mu) * vol + site) * 9 + k];
    const double2 v{h * u.x, h * u.y};
    w64[i] = v;
    w32[i] = float2{float(v.x), float(v.y)};
  }
}

// max over the links of |U U^H - I| and |det U - 1| (entrywise moduli), one link per
// thread; non-negative doubles order like their bit patterns, so one atomicMax on the
// bits keeps the largest.
__global__ void k_su3_deviation(const double2* __restrict__ links, int64_t nlinks,
                                unsigned long long* __restrict__ dev) {
  double worst = 0.0;
  for (int64_t l = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; l < nlinks;
       l += int64_t(gridDim.x) * blockDim.x) {
    double2 u[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) u[i][j] = links[l * 9 + 3 * i + j];
    // U U^H - I
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        double re = (i == k) ? -1.0 : 0.0, im = 0.0;
        for (int j = 0; j < 3; ++j) {  // u[i][j] conj(u[k][j])
          re += u[i][j].x * u[k][j].x + u[i][j].y * u[k][j].y;
          im += u[i][j].y * u[k][j].x - u[i][j].x * u[k][j].y;
        }
        worst = fmax(worst, sqrt(re * re + im * im));
      }
    // det U = u0 . (u1 x u2)
    double dre = 0.0, dim = 0.0;
    for (int j = 0; j < 3; ++j) {
      const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      const double cre = u[1][j1].x * u[2][j2].x - u[1][j1].y * u[2][j2].y -
                         (u[1][j2].x * u[2][j1].x - u[1][j2].y * u[2][j1].y);
      const double cim = u[1][j1].x * u[2][j2].y + u[1][j1].y * u[2][j2].x -
                         (u[1][j2].x * u[2][j1].y + u[1][j2].y * u[2][j1].x);
      dre += u[0][j].x * cre - u[0][j].y * cim;
      dim += u[0][j].x * cim + u[0][j].y * cre;
    }
    const double dd = sqrt((dre - 1.0) * (dre - 1.0) + dim * dim);
    worst = fmax(worst, isfinite(dd) ? dd : 1e300);
  }
  if (!(worst >= 0.0)) worst = 1e300;  // NaN entries
  atomicMax(dev, static_cast<unsigned long long>(__double_as_longlong(worst)));
}

// Rows 0 and 1 of every link (entries k < 6), value-major like w: wc[(mu 6 + k) vol + s].
__global__ void k_two_rows(const double2* __restrict__ w64, int64_t vol,
                           double2* __restrict__ wc64, float2* __restrict__ wc32) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < 4 * vol * 6;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t mu = i / (6 * vol);
    const double2 v = w64[i + 3 * vol * mu];  // (mu 9 + k) vol + s = i + 3 vol mu
    wc64[i] = v;
    wc32[i] = float2{float(v.x), float(v.y)};
  }
}

// The scalar CSR of M = m + D from w, one thread per row: the row's own site (the mass
// on the diagonal) and its eight neighbours (three columns each), in ascending site order,
// so the columns come out sorted.
__global__ void k_stencil_csr(Stencil<double2> op, int64_t* __restrict__ rowptr,
                              int32_t* __restrict__ col, double2* __restrict__ vals) {
  const int64_t n = 3 * op.vol;
  for (int64_t row = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; row <= n;
       row += int64_t(gridDim.x) * blockDim.x) {
    rowptr[row] = 25 * row;
    if (row == n) continue;
    const int64_t s = row / 3;
    const int c = int(row - 3 * s);
    // site and kind of each of the nine blocks: -1 the diagonal, 2 mu forward, 2 mu + 1
    // backward
    int64_t site[9];
    int kind[9];
    site[0] = s;
    kind[0] = -1;
    int64_t rem = s;
    for (int mu = 0; mu < 4; ++mu) {
      const int64_t L = op.L[mu];
      const int64_t xm = rem % L;
      rem /= L;
      const int64_t st = op.stride[mu];
      site[1 + 2 * mu] = xm == L - 1 ? s - (L - 1) * st : s + st;
      kind[1 + 2 * mu] = 2 * mu;
      site[2 + 2 * mu] = xm == 0 ? s + (L - 1) * st : s - st;
      kind[2 + 2 * mu] = 2 * mu + 1;
    }
    // insertion sort of the nine distinct sites (every extent >= 3)
    for (int i = 1; i < 9; ++i) {
      const int64_t ks = site[i];
      const int kk = kind[i];
      int j = i - 1;
      while (j >= 0 && site[j] > ks) {
        site[j + 1] = site[j];
        kind[j + 1] = kind[j];
        --j;
      }
      site[j + 1] = ks;
      kind[j + 1] = kk;
    }
    int64_t e = 25 * row;
    for (int i = 0; i < 9; ++i) {
      const int64_t y = site[i];
      if (kind[i] < 0) {
        col[e] = int32_t(3 * y + c);
        vals[e] = double2{op.mass, 0.0};
        ++e;
        continue;
      }
      const int mu = kind[i] >> 1;
      const bool forward = (kind[i] & 1) == 0;
      for (int j = 0; j < 3; ++j) {
        double2 v;
        if (forward) {
          v = op.w[(int64_t(mu) * 9 + 3 * c + j) * op.vol + s];  // W_mu(s)[c][j]
        } else {
          const double2 u = op.w[(int64_t(mu) * 9 + 3 * j + c) * op.vol + y];
          v = double2{-u.x, u.y};                                  // -conj(W_mu(s-mu)[j][c])
        }
        col[e] = int32_t(3 * y + j);
        vals[e] = v;
        ++e;
      }
    }
  }
}

}  // namespace

hipError_t launch_stencil_links(const double2* links, const Stencil<double2>& geo,
                                double2* w64, float2* w32, hipStream_t s) {
  const int64_t total = 4 * geo.vol * 9;
  const int64_t g = std::min<int64_t>((total + 255) / 256, 8192);
  k_stencil_links<<<dim3(unsigned(g)), 256, 0, s>>>(links, geo, w64, w32);
  return hipGetLastError();
}

hipError_t launch_su3_deviation(const double2* links, int64_t nlinks, unsigned long long* dev,
                                hipStream_t s) {
  const int64_t g = std::min<int64_t>((nlinks + 255) / 256, 8192);
  k_su3_deviation<<<dim3(unsigned(std::max<int64_t>(g, 1))), 256, 0, s>>>(links, nlinks, dev);
  return hipGetLastError();
}

hipError_t launch_two_rows(const double2* w64, int64_t nlinks, double2* wc64, float2* wc32,
                           hipStream_t s) {
  const int64_t g = std::min<int64_t>((6 * nlinks + 255) / 256, 8192);
  k_two_rows<<<dim3(unsigned(std::max<int64_t>(g, 1))), 256, 0, s>>>(w64, nlinks / 4, wc64, wc32);
  return hipGetLastError();
}

hipError_t launch_stencil_csr(const Stencil<double2>& op, int64_t* rowptr, int32_t* col,
                              double2* vals, hipStream_t s) {
  const int64_t rows = 3 * op.vol + 1;
  const int64_t g = std::min<int64_t>((rows + 255) / 256, 8192);
  k_stencil_csr<<<dim3(unsigned(g)), 256, 0, s>>>(op, rowptr, col, vals);
  return hipGetLastError();
}

}  // namespace msc
