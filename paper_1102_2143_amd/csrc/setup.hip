// Operator set-up on the device: CSR validation, index and value conversions, and the
// conjugate transpose M^H (counting sort by column, then a per-row sort so the result
// is deterministic).  Runs once per operator; not on the iteration path.
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

}  // namespace

hipError_t launch_validate_csr(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                               int* d_err, hipStream_t s) {
  k_validate_rowptr<<<blocks_for(n), kSetupBlock, 0, s>>>(rowptr, n, nnz, d_err);
  if (nnz > 0) k_validate_col<<<blocks_for(nnz), kSetupBlock, 0, s>>>(col, n, nnz, d_err);
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

}  // namespace msc
