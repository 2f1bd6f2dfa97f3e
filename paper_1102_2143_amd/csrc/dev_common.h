// Device-side helpers shared by the HIP kernels: complex arithmetic on float2/double2,
// wavefront and workgroup reductions in FP64, the "last workgroup finalises" ticket and
// the XCD-aware mapping of workgroups to contiguous row ranges.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msc_internal.h"

namespace msc {

constexpr int kWave = 64;   // CDNA wavefront width

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
// Streaming accesses: data a launch touches once (the shifted solutions and directions,
// kept residuals, rows no other wave of the launch gathers, outputs the next kernel reads
// back) carry the non-temporal hint, so that they do not evict from L2 what the launch
// gathers again (neighbouring rows, the links).
typedef double vd2_t __attribute__((ext_vector_type(2)));
typedef float vf2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const vd2_t v = __builtin_nontemporal_load(reinterpret_cast<const vd2_t*>(p));
  return double2{v.x, v.y};
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const vf2_t v = __builtin_nontemporal_load(reinterpret_cast<const vf2_t*>(p));
  return float2{v.x, v.y};
}
__device__ __forceinline__ void st_stream(double2* p, const double2& v) {
  const vd2_t w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<vd2_t*>(p));
}
__device__ __forceinline__ void st_stream(float2* p, const float2& v) {
  const vf2_t w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<vf2_t*>(p));
}

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
// release/acquire pair would give (the release's wait on the memory counter, without
// its L2 write-back, which only dirty lines written by plain stores need; the
// acquire's L2 invalidate is for plain loads); the pair would add that write-back in
// every workgroup and the invalidate in the last ones, which evict the gathered
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

// The slices one wave of an iteration kernel visits, in order.  With a lattice order
// (SweepOrder::on), XCD x (workgroups b with b % 8 == x under the round-robin dispatch)
// owns slices [x N / 8, (x + 1) N / 8) of the N slices, and its U waves visit positions
// j = u, u + U, u + 2U, ... of a permutation of that range (u: the wave's index among
// them), so the slices in flight on an XCD at any moment are consecutive positions.  The
// permutation walks the range's whole slabs tile by tile: position
// j = ((cb nb + b) na + a) cs + cc names slice a s2 + b s1 + cb cs + cc (slab a of na,
// plane b of nb, tile cb, slice cc), so the same tile of neighbouring slabs lies cs
// positions away and that of neighbouring planes cs na positions away, within what the
// XCD has in flight: its L2 then serves the neighbours' gathers and shared operands.
// Without an order, workgroup b sweeps one contiguous range (block_range) with its waves
// interleaved.  The position arithmetic is wave-uniform (scalar unit).
struct Sweep {
  int64_t lo;      // first slice of the range
  uint32_t len;    // slices in the range
  uint32_t j, step;
  uint32_t na, nb, s1, s2, cs;  // na = 0: identity permutation
  __device__ __forceinline__ bool more() const { return j < len; }
  __device__ __forceinline__ void next() { j += step; }
  __device__ __forceinline__ int64_t slice() const {
    uint32_t k = j;
    if (na > 0 && j < na * s2) {
      const uint32_t cc = j % cs, r1 = j / cs;
      const uint32_t sa = r1 % na, r2 = r1 / na;
      const uint32_t pb = r2 % nb, cb = r2 / nb;
      k = sa * s2 + pb * s1 + cb * cs + cc;
    }
    return lo + int64_t(k);
  }
};

// wpb: waves per workgroup, each taking one slice at a time.
__device__ __forceinline__ Sweep make_sweep(int64_t nslices, const SweepOrder& o, int wpb) {
  Sweep w{};
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / kWave));
  const int g = gridDim.x;
  if (o.on && (g % kXcds) == 0) {
    const int x = int(blockIdx.x % kXcds);
    const int64_t lo = nslices * x / kXcds, hi = nslices * (x + 1) / kXcds;
    w.lo = lo;
    w.len = uint32_t(hi - lo);
    w.j = uint32_t(int(blockIdx.x / kXcds) * wpb + wv);
    w.step = uint32_t((g / kXcds) * wpb);
    if (o.s1 > 0 && o.s2 > 0 && o.cs > 0) {
      w.na = w.len / uint32_t(o.s2);
      w.nb = uint32_t(o.s2 / o.s1);
      w.s1 = uint32_t(o.s1);
      w.s2 = uint32_t(o.s2);
      w.cs = uint32_t(o.cs);
    }
  } else {
    int64_t beg, end;
    block_range(nslices, wpb, beg, end);
    w.lo = beg;
    w.len = uint32_t(end - beg);
    w.j = uint32_t(wv);
    w.step = uint32_t(wpb);
  }
  return w;
}

}  // namespace msc
