// Device-side helpers shared by the HIP kernels: complex arithmetic on float2/double2,
// wavefront and workgroup reductions in FP64, the "last workgroup finalises" ticket and
// the XCD-aware mapping of workgroups to contiguous row ranges.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msc_internal.h"

namespace msc {

constexpr int kWave = 64;   // CDNA wavefront width
constexpr int kXcds = 8;    // MI355X: 8 accelerator complex dies, one L2 each

template <class R> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <class R> using cplx = typename vec2<R>::type;

template <class R> __device__ __forceinline__ cplx<R> czero() { return cplx<R>{R(0), R(0)}; }

// acc += a * b (complex)
template <class R>
__device__ __forceinline__ void cfma(cplx<R>& acc, const cplx<R>& a, const cplx<R>& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

template <class R> __device__ __forceinline__ double norm2d(const cplx<R>& v) {
  const double x = double(v.x), y = double(v.y);
  return fma(x, x, y * y);
}

__device__ __forceinline__ double2 to_d(const float2 v) { return double2{double(v.x), double(v.y)}; }
__device__ __forceinline__ double2 to_d(const double2 v) { return v; }
template <class R> __device__ __forceinline__ cplx<R> from_d(const double2 v);
template <> __device__ __forceinline__ float2 from_d<float>(const double2 v) {
  return float2{float(v.x), float(v.y)};
}
template <> __device__ __forceinline__ double2 from_d<double>(const double2 v) { return v; }

// Sum over the L consecutive lanes of a row group (L a power of two <= 64).
template <int L, class T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
  return v;
}

template <int L, class R> __device__ __forceinline__ cplx<R> group_sum_c(cplx<R> v) {
  v.x = group_sum<L>(v.x);
  v.y = group_sum<L>(v.y);
  return v;
}

// Workgroup sum of one double per thread; the result is valid in thread 0.
template <int BS> __device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[BS / kWave];
  v = group_sum<kWave>(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / kWave; ++i) s += part[i];
  }
  __syncthreads();
  return s;
}

// Workgroup sums of K doubles per thread (K small); results valid in thread 0.
template <int BS, int K> __device__ __forceinline__ void block_sum_k(double (&v)[K]) {
  __shared__ double part[K][BS / kWave];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = group_sum<kWave>(v[k]);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) part[k][w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < BS / kWave; ++i) s += part[k][i];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Agent-scope stores/loads for values exchanged between workgroups of one launch
// (the eight XCD L2 caches are not coherent with each other for plain accesses).
__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A word in host-coherent memory that the host polls after an event: one vector store at
// system scope (no cache maintenance; the host reads it once the kernel has completed).
__device__ __forceinline__ void store_host_flag(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Every workgroup calls this once, after its partial(s) are stored with store_agent by
// wave 0.  Returns true (in all threads) in the workgroup that arrives last; that
// workgroup then sees every partial through load_agent.  The counters are reset by the
// last arrivals, so the same site serves the next launch.
//
// Why no acquire/release fence is needed.  Only the partials cross workgroups inside a
// launch, and every access to them is an agent-scope atomic: store_agent compiles to a
// store with the agent-coherence bit (written through the XCD's L2 to the coherence
// point shared by all XCDs) and load_agent to a load with the same bit (served from
// that point, never from a stale L1/L2 line).  Before taking a ticket, the wave that
// stored the partials waits for its memory counter to drain (s_waitcnt 0): a store
// completes only once the coherence point has acknowledged it, so every partial is
// there before the increment that reports it.  The last arrival issues its loads only
// after its increment has returned the final count, i.e. after every other increment,
// hence after every partial store completed.  This is the ordering an agent-scope
// release/acquire pair would give; the pair would add an L2 write-back in every
// workgroup and an L2 invalidate in the last ones (what the compiler emits for
// non-coherent data), which the partials do not need, and which evict the gathered
// vectors the kernels rely on (measured: the 64-system batch ran 296 ms per solve with
// them against 182 ms without).  Compiler barriers keep the stores, the wait, the
// increment and the loads in program order.
//
// Arrivals on one counter serialise at the memory side, so the ticket is two-level:
// arrival `idx` (0 <= idx < arrivals) first takes a ticket in group idx % 8 (eight
// counters on separate 128-byte lines), and only the last arrival of each group takes
// the final ticket.  A ticket site is kTicketSite unsigned words (msc_internal.h).

__device__ __forceinline__ bool arrive_last(unsigned* site, unsigned arrivals, unsigned idx) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // vmcnt = expcnt = lgkmcnt = 0: partial stores done
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const unsigned g = idx & 7u;
    const unsigned in_group = (arrivals - g + 7u) / 8u;  // arrivals whose index is g mod 8
    const unsigned groups = arrivals < 8u ? arrivals : 8u;
    unsigned* gc = site + g * kTicketStride;
    const unsigned t = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int is_last = 0;
    if (t == in_group - 1) {
      __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned* fc = site + 8 * kTicketStride;
      const unsigned f = __hip_atomic_fetch_add(fc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (f == groups - 1) {
        __hip_atomic_store(fc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = 1;
      }
    }
    last = is_last;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  __syncthreads();
  return last != 0;
}

// Grid-wide form: every workgroup of the launch arrives once.
__device__ __forceinline__ bool arrive_last(unsigned* site) {
  return arrive_last(site, gridDim.x, blockIdx.x);
}

// Workgroups are dispatched round-robin over the XCDs.  Renumber them so that the
// workgroups of one XCD own one contiguous block of rows (its L2 then serves the
// neighbouring-row gathers of that block).  Requires gridDim.x % 8 == 0 to permute.
__device__ __forceinline__ int logical_block() {
  const int g = gridDim.x, b = blockIdx.x;
  if ((g & (kXcds - 1)) != 0) return b;
  return (b & (kXcds - 1)) * (g / kXcds) + b / kXcds;
}

// Contiguous [beg, end) slice of `n` items for this workgroup, in units of `step`.
__device__ __forceinline__ void block_range(int64_t n, int step, int64_t& beg, int64_t& end) {
  const int64_t g = gridDim.x;
  const int64_t units = (n + step - 1) / step;
  const int64_t per = (units + g - 1) / g;
  beg = int64_t(logical_block()) * per * step;
  end = beg + per * step;
  if (end > n) end = n;
  if (beg > n) beg = n;
}

}  // namespace msc
