// Host driver and C ABI: operator creation (device-side M^H and complex64 copies), the
// iteration loop with device-resident convergence state, verification, and error
// reporting.  No exception crosses the ABI; every failure sets a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <string>
#include <vector>

#include "msc.h"
#include "msc_internal.h"

using namespace msc;

namespace {

thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return e_ == hipErrorOutOfMemory ? MSC_ENOMEM : MSC_EHIP;                    \
    }                                                                              \
  } while (0)

template <class T> hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count);
}

template <class T> void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_workspace(Workspace& w) {
  for (void* q : {w.r, w.p[0], w.p[1], w.t, w.pk, w.r32, w.p32[0], w.p32[1], w.t32, w.pk32,
                  w.pkeep0})
    if (q) (void)hipFree(q);
  for (void*& q : w.rkeep) {
    if (q) (void)hipFree(q);
    q = nullptr;
  }
  dfree(w.t64);
  dfree(w.u64);
  dfree(w.st);
  if (w.h_halt) (void)hipHostFree(w.h_halt);
  for (auto& e : w.ev)
    if (e) (void)hipEventDestroy(e);
  w = Workspace{};
}

// Buffers are cleared on the stream that first uses them: a hipMemset would run on the
// null stream, which does not order itself with the library's non-blocking streams (the
// batched solve's internal stream), so the clearing could land after the first kernels
// had already written the buffers.
msc_status ensure_scratch(msc_op op, hipStream_t s) {
  Scratch& sc = op->scratch;
  if (sc.partial) return MSC_OK;
  HIP_TRY(dalloc(&sc.partial, size_t(kMaxGrid) * kMaxShifts));
  HIP_TRY(dalloc(&sc.tickets, 16 * kTicketSite));
  HIP_TRY(dalloc(&sc.res2, kMaxShifts));
  HIP_TRY(hipMemsetAsync(sc.tickets, 0, sizeof(unsigned) * 16 * kTicketSite, s));
  return MSC_OK;
}

// Krylov buffers: complex128 always (the FP64 solve and the first phase of a mixed
// solve), complex64 copies when a mixed solve needs its second phase.
msc_status ensure_workspace(msc_op op, int prec, int ns) {
  Workspace& w = op->ws;
  const size_t n = size_t(op->n);
  const size_t nk = size_t(std::max(ns - 1, 1));
  if (!(w.st && w.ns >= ns && w.n == n)) {
    free_workspace(w);
    HIP_TRY(hipMalloc(&w.r, sizeof(double2) * n));
    HIP_TRY(hipMalloc(&w.p[0], sizeof(double2) * n));
    HIP_TRY(hipMalloc(&w.p[1], sizeof(double2) * n));
    HIP_TRY(hipMalloc(&w.t, sizeof(double2) * n));
    HIP_TRY(hipMalloc(&w.pk, sizeof(double2) * n * nk));
    HIP_TRY(dalloc(&w.t64, n));
    HIP_TRY(dalloc(&w.u64, n * 8));
    for (auto& q : w.rkeep) HIP_TRY(hipMalloc(&q, sizeof(double2) * n));
    HIP_TRY(hipMalloc(&w.pkeep0, sizeof(double2) * n));
    HIP_TRY(dalloc(&w.st, 1));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_halt), 4 * sizeof(int),
                          hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.d_halt), w.h_halt, 0));
    HIP_TRY(hipEventCreateWithFlags(&w.ev[0], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&w.ev[1], hipEventDisableTiming));
    w.n = n;
    w.ns = ns;
    w.prec = MSC_PREC_FP64;
  }
  if (prec == MSC_PREC_MIXED && !w.r32) {
    const size_t wn = std::max<size_t>(size_t(w.ns) - 1, 1);
    HIP_TRY(hipMalloc(&w.r32, sizeof(float2) * n));
    HIP_TRY(hipMalloc(&w.p32[0], sizeof(float2) * n));
    HIP_TRY(hipMalloc(&w.p32[1], sizeof(float2) * n));
    HIP_TRY(hipMalloc(&w.t32, sizeof(float2) * n));
    HIP_TRY(hipMalloc(&w.pk32, sizeof(float2) * n * wn));
    w.prec = MSC_PREC_MIXED;
  }
  return MSC_OK;
}

int choose_lanes(msc_op op, const msc_params& prm) {
  if (prm.lanes == 4 || prm.lanes == 8 || prm.lanes == 16 || prm.lanes == 32) return prm.lanes;
  const double avg = op->n > 0 ? double(op->nnz) / double(op->n) : 1.0;
  if (avg <= 6.0) return 4;
  if (avg <= 40.0) return 8;
  if (avg <= 80.0) return 16;
  return 32;
}

// View of a sliced ELLPACK copy with one value precision; narrow columns when the copy
// has them and `narrow` asks for them.
template <class V>
Sell<V> sell_view(const SellStore& m, const V* val, const V* diag, bool narrow) {
  Sell<V> v{m.cptr, m.col, val, diag, m.wp};
  if (narrow && m.col16) {
    v.col16 = m.col16;
    v.cbase = m.cbase;
  }
  return v;
}

// Bytes per column index of the matrix copy an SpMV reads (CSR and 32-bit sliced
// ELLPACK: 4, narrow sliced ELLPACK: 2, the per-column bases being negligible).
template <class V> double index_bytes(bool sell, const Sell<V>& m) {
  return sell && m.col16 ? 2.0 : 4.0;
}

// Sweep order of a lattice whose neighbouring planes lie s1 slices and neighbouring slabs
// s2 slices apart (s2 a multiple of s1): planes are cut into tiles of cs slices, the
// largest divisor of s1 that keeps neighbouring planes (cs * slabs-per-XCD positions
// apart in the sweep) within kTileSpan positions.  Zeros when the structure does not fit.
#ifndef MSC_TILE_SPAN
#define MSC_TILE_SPAN 48
#endif
// The links' kernels sweep blocks of 64 sites (192 rows), with their own spans: the
// complex64 ones, and the FP64 ones (twice the bytes per site in flight).
#ifndef MSC_TILE_SPAN_SITES
#define MSC_TILE_SPAN_SITES 16
#endif
#ifndef MSC_TILE_SPAN_SITES64
#define MSC_TILE_SPAN_SITES64 32
#endif
#ifndef MSC_C64_TWO_ROWS
#define MSC_C64_TWO_ROWS 1
#endif
constexpr int64_t kTileSpan = MSC_TILE_SPAN;
constexpr int64_t kTileSpanSites = MSC_TILE_SPAN_SITES;
constexpr int64_t kTileSpanSites64 = MSC_TILE_SPAN_SITES64;
constexpr bool kC64TwoRows = MSC_C64_TWO_ROWS != 0;
SweepOrder lattice_order(int64_t nslices, int64_t s1, int64_t s2, int64_t span = kTileSpan) {
  SweepOrder o{0, 0, 0, 0};
  if (s1 < 1 || s2 <= s1 || s2 % s1 != 0 || s2 > nslices / kXcds) return o;
  const int64_t na = std::max<int64_t>(1, nslices / kXcds / s2);
  int64_t cs = 1;
  for (int64_t c = 1; c <= s1; ++c)
    if (s1 % c == 0 && c * na <= span) cs = c;
  o.s1 = int32_t(s1);
  o.s2 = int32_t(s2);
  o.cs = int32_t(cs);
  return o;
}

// Lattice structure of a stored matrix, read from its columns: in blocks of rows spread
// over the matrix (at scattered offsets, so that they do not all sit on one lattice
// boundary), the row-to-column distances (periodic: min(d, n - d)) that are whole slices
// and occur in at least 3/4 of the sampled rows (a boundary row reaches one neighbour
// the long way round); the two largest give the plane and slab distances.  A matrix
// without such a structure gets zeros (contiguous sweeps).
SweepOrder detect_order(const int64_t* d_rowptr, const int32_t* d_col, int64_t n, int64_t nnz,
                        int64_t nslices, hipStream_t s) {
  const SweepOrder none{0, 0, 0, 0};
  constexpr int kBlocks = 8, kRows = 16, kMaxEntries = 64 * kRows;
  if (nslices < 2 * kXcds || nnz == 0) return none;
  std::map<int64_t, int> seen;  // distance in slices -> sampled rows having it
  for (int bk = 0; bk < kBlocks; ++bk) {
    const int64_t r0 = (n * (2 * bk + 1) / (2 * kBlocks) + 1009 * int64_t(bk * bk + 3 * bk + 1)) %
                       std::max<int64_t>(1, n - kRows);
    if (r0 + kRows > n) return none;
    int64_t rp[kRows + 1];
    if (hipMemcpyAsync(rp, d_rowptr + r0, sizeof rp, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return none;
    const int64_t cnt = rp[kRows] - rp[0];
    if (cnt <= 0 || cnt > kMaxEntries) return none;
    std::vector<int32_t> cols(size_t(cnt), 0);
    if (hipMemcpyAsync(cols.data(), d_col + rp[0], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return none;
    for (int i = 0; i < kRows; ++i) {
      std::vector<int64_t> ds;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        int64_t d = std::llabs(int64_t(cols[size_t(e - rp[0])]) - (r0 + i));
        d = std::min(d, n - d);
        if (d >= kSlice && d % kSlice == 0) ds.push_back(d / kSlice);
      }
      std::sort(ds.begin(), ds.end());
      ds.erase(std::unique(ds.begin(), ds.end()), ds.end());
      for (int64_t d : ds) ++seen[d];
    }
  }
  std::vector<int64_t> common;
  for (const auto& kv : seen)
    if (4 * kv.second >= 3 * kBlocks * kRows) common.push_back(kv.first);
  if (common.size() < 2) return none;
  return lattice_order(nslices, common[common.size() - 2], common.back());
}

MsArgs make_args(msc_op op, int lanes, const double* d_b, double* d_x) {
  MsArgs a{};
  a.kind = op->kind;
  a.n = op->n;
  a.lanes = lanes;
  // cap on workgroups per iteration kernel (overridden by max_grid): 1024 measured best
  // at 16^4 (fewer final reductions than 2048, enough rows in flight)
  a.grid = 1024;
  a.m64 = Csr<double2>{op->rowptr, op->col, op->val64};
  a.m32 = Csr<float2>{op->rowptr, op->col, op->val32};
  if (op->kind == MSC_A_MHM) {
    a.mh64 = Csr<double2>{op->rowptr_h, op->col_h, op->val64_h};
    a.mh32 = Csr<float2>{op->rowptr_h, op->col_h, op->val32_h};
  }
  a.sell = op->sell ? 1 : 0;
  if (op->sell) {
    const SellStore& sm = op->sell_m;
    a.nslices = sm.nslices;
    a.s64 = sell_view(sm, sm.val64, sm.diag64, true);
    a.s32 = sell_view(sm, sm.val32, sm.diag32, true);
    if (op->kind == MSC_A_MHM) {
      const SellStore& sh = op->sell_mh;
      a.sh64 = sell_view(sh, sh.val64, sh.diag64, true);
      a.sh32 = sell_view(sh, sh.val32, sh.diag32, true);
    }
  }
  a.stencil = 0;
  a.w64 = op->w64;
  a.w32 = op->w32;
  a.b = reinterpret_cast<const double2*>(d_b);
  a.x = reinterpret_cast<double2*>(d_x);
  a.r = op->ws.r;
  a.pb[0] = op->ws.p[0];
  a.pb[1] = op->ws.p[1];
  a.t = op->ws.t;
  a.pk = op->ws.pk;
  for (int k = 0; k < kMaxSteps - 1; ++k) a.rkeep[k] = op->ws.rkeep[k];  // complex64 in phase 2
  a.pkeep0 = op->ws.pkeep0;
  a.hflag = op->ws.d_halt;
  a.steps = 1;
  a.defer_ok = 0;
  a.sample = -1;
  a.t64 = op->ws.t64;
  a.st = op->ws.st;
  a.sc = op->scratch;
  return a;
}

// Which FP64 heads on the links form their product by the recurrence: all but the first
// launch and the launches kTrEvery / 2 mod kTrEvery (off the timing samples' positions,
// which start at multiples of 128); and how many of the first n launches do.
bool tr_launch(bool eligible, int launch) {
  return eligible && launch != 0 && launch % kTrEvery != kTrEvery / 2;
}
int tr_launches(int n) {
  return n <= 1 ? 0 : n - 1 - (n + kTrEvery / 2 - 1) / kTrEvery;
}

// Algorithmic HBM bytes of one multishift iteration (each array touched once, gathers
// counted once), per row: see the byte model in the design notes of the repository.
// Algorithmic bytes of one launch: K1 (t = M p), K2 (r <- r - a (M^H t + sigma0 p)), the
// all-shift update with `act` active shifts, and the head that fuses the update with K1
// (the old p is read once for both).
struct KernelBytes {
  double k1, k2, upd, head;
};
// launch with `act` active shifts; ib / ibh: bytes per column index of the copies of the
// operator's matrix and of M^H that the SpMVs read.
// `kept`: residual vectors the head's update writes (a deferring head keeps r) or reads
// back (an applying head after deferred steps).
// Matrix bytes of one application of M (or A) and of M^H in precision `prec`: the stored
// copy (value + index per entry, 4-byte row pointers), or for the matrix-free staggered
// operator the links, each read once: 4 links x 9 values per site = 12 values per row.
struct MatBytes {
  double m, mh;
};
MatBytes mat_bytes(int kind, int prec, double n, double nnz, double nnz_h, double ib, double ibh,
                   int stencil) {
  const double w = prec == MSC_PREC_MIXED ? 8.0 : 16.0;
  // links: each read once per site and direction, 3 or 2 rows of 3 values: 12 or 8
  // values per row of the operator
  if (stencil) return MatBytes{4.0 * stencil * w * n, 4.0 * stencil * w * n};
  return MatBytes{nnz * (w + ib) + 4.0 * (n + 1),
                  kind == MSC_A_MHM ? nnz_h * (w + ibh) + 4.0 * (n + 1) : 0.0};
}

// x0b: bytes per row of x_0 and of its kept direction that the update moves (an applying
// head reads and writes x_0, 32, and reads the kept direction after deferred steps; the
// first deferring head of a cycle writes it).
KernelBytes kernel_bytes(int kind, int prec, double n, const MatBytes& mb, double act,
                         bool pending, int kept, double x0b) {
  const double w = prec == MSC_PREC_MIXED ? 8.0 : 16.0;
  KernelBytes b{};
  b.k1 = mb.m + 2.0 * n * w;
  b.k2 = (kind == MSC_A_MHM ? mb.mh + n * w : n * w) + 3.0 * n * w;
  b.upd = pending ? n * (3.0 * w + x0b) + act * n * (32.0 + 2.0 * w) + kept * n * w : 0.0;
  b.head = b.k1 + (pending ? b.upd - n * w : 0.0);
  return b;
}

// act_sum: x_j/p_j row-vector updates performed (shifts listed, summed over the heads);
// kept: heads that kept r for a deferred step or read it back.
// x0_total: bytes per row of x_0 and its kept direction summed over the heads (negative:
// x_0 read and written in every iteration, 32 bytes per row each).
double iter_bytes(int kind, int prec, double n, const MatBytes& mb, double act_sum,
                  double iters, double kept, double x0_total = -1.0) {
  const double w = prec == MSC_PREC_MIXED ? 8.0 : 16.0;   // Krylov vector element
  const double mat = mb.m + mb.mh;
  double vec;
  if (kind == MSC_A_MHM)
    vec = n * (w + w) + n * (w + w + 2 * w);  // K1: p gather, t write; K2: t gather, p, r r/w
  else
    vec = n * (w + w) + n * (w + w + 2 * w);  // K1: p, t; K2: t, p, r r/w
  vec += n * (w + 2 * w);                      // K3: r, p r/w
  const double x0 = x0_total < 0.0 ? 32.0 * n * iters : x0_total * n;
  const double per_shift = n * (32.0 + 2 * w); // x_j r/w (complex128) + p_j r/w
  return iters * (mat + vec) + x0 + act_sum * per_shift + kept * n * w;
}

// Events for sampled per-kernel timing; destroyed with the pool.
struct EventPool {
  std::vector<std::array<hipEvent_t, 6>> groups;
  hipEvent_t* next() {
    std::array<hipEvent_t, 6> g{};
    for (auto& e : g)
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
    groups.push_back(g);
    return groups.back().data();
  }
  ~EventPool() {
    for (auto& g : groups)
      for (auto e : g)
        if (e) (void)hipEventDestroy(e);
  }
};

// The kernel timing fields of a report, cleared (calls that sample nothing leave them 0).
void clear_timing(msc_info& I) {
  for (int k = 0; k < 3; ++k)
    I.kernel_ms[k] = I.kernel_bytes[k] = I.fp64_kernel_ms[k] = I.fp64_kernel_bytes[k] = 0.0;
  I.kernel_samples = I.fp64_kernel_samples = 0;
  I.reserved = 0;
}

msc_status run_multishift(msc_op op, const double* d_b, double* d_x, const msc_params& prm,
                          msc_info* info, hipStream_t s, double tol_stop, int prec,
                          std::vector<double>* rel_out, int* iters_out, int* status_out,
                          double* bytes_out, double* bnorm_out) {
  const int ns = int(op->sigma.size());
  msc_status rc = ensure_scratch(op, s);
  if (rc != MSC_OK) return rc;
  rc = ensure_workspace(op, prec, ns);
  if (rc != MSC_OK) return rc;
  const int lanes = choose_lanes(op, prm);
  if (prm.format < MSC_FORMAT_AUTO || prm.format > MSC_FORMAT_STENCIL ||
      ((prm.format == MSC_FORMAT_SELL || prm.format == MSC_FORMAT_SELL32) && !op->sell)) {
    set_error("msc_solve: format %d unavailable (sliced ELLPACK copy %s)", prm.format,
              op->sell ? "built" : "not built: padding too large");
    return MSC_EINVAL;
  }
  if (prm.format == MSC_FORMAT_STENCIL && !(op->stencil && op->sell)) {
    set_error("msc_solve: format stencil needs an operator made by msc_op_create_staggered");
    return MSC_EINVAL;
  }
  MsArgs a64 = make_args(op, lanes, d_b, d_x);
  if (prm.max_grid > 0) a64.grid = std::min(prm.max_grid, kMaxGrid);
  if (prm.format == MSC_FORMAT_CSR) a64.sell = 0;
  // the iteration's two operator halves from the links: the default for staggered
  // operators (verification and refinement keep the stored copies)
  a64.stencil = op->stencil && a64.sell &&
                (prm.format == MSC_FORMAT_AUTO || prm.format == MSC_FORMAT_STENCIL)
                    ? (op->two_rows ? 2 : 3) : 0;
  if (a64.stencil == 2) a64.w64 = op->wc64;
  a64.ord = a64.stencil ? op->order_sites64 : op->order;
  a64.ord.on = (prm.sweep == 0 && a64.ord.s1 > 0) ? 1 : 0;
  if (prm.format == MSC_FORMAT_SELL32 && op->sell) {
    const SellStore &sm = op->sell_m, &sh = op->sell_mh;
    a64.s64 = sell_view(sm, sm.val64, sm.diag64, false);
    a64.s32 = sell_view(sm, sm.val32, sm.diag32, false);
    if (op->kind == MSC_A_MHM) {
      a64.sh64 = sell_view(sh, sh.val64, sh.diag64, false);
      a64.sh32 = sell_view(sh, sh.val32, sh.diag32, false);
    }
  }
  const double ib = index_bytes(a64.sell, a64.s64), ibh = index_bytes(a64.sell, a64.sh64);
  MsArgs a32 = a64;
  if (a32.stencil != 0) {  // the complex64 kernels' tile span
    a32.ord = op->order_sites;
    a32.ord.on = a64.ord.on;
  }
  // the complex64 phase reads two rows per SU(3) link too, unless told otherwise
  if (a32.stencil == 2) {
    if (kC64TwoRows)
      a32.w32 = op->wc32;
    else
      a32.stencil = 3;
  }
  const bool mixed = prec == MSC_PREC_MIXED;
  if (mixed) {
    a32.r = op->ws.r32;
    a32.pb[0] = op->ws.p32[0];
    a32.pb[1] = op->ws.p32[1];
    a32.t = op->ws.t32;
    a32.pk = op->ws.pk32;
  }

  std::vector<int> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int i, int j) { return op->sigma[i] < op->sigma[j]; });
  SolveState h{};
  h.sigma0 = op->sigma[order[0]];
  h.eps2 = tol_stop * tol_stop;  // scaled by |b|^2 in the init kernel
  // a mixed solve runs in FP64 until |r| <= switch_tol |b|, then in complex64
  const double sw = mixed ? std::max(prm.switch_tol, tol_stop) : 0.0;
  h.sw_eps2 = sw * sw;
  h.a_prev = 1.0;
  h.b = 0.0;
  h.max_iter = prm.max_iter;
  h.ns = ns;
  h.freeze = prm.freeze ? 1 : 0;
  for (int j = 0; j < ns; ++j) {
    h.s[j] = op->sigma[order[j]] - h.sigma0;
    h.rot[0].zeta[j] = 1.0;
    h.zeta_prev[j] = 1.0;
    h.rot[0].active[j] = 1;
    h.freeze_iter[j] = -1;
    h.orig[j] = order[j];
  }
  HIP_TRY(hipMemcpyAsync(op->ws.st, &h, sizeof h, hipMemcpyHostToDevice, s));
  __atomic_store_n(op->ws.h_halt, 0, __ATOMIC_RELEASE);  // no kernel of this op is in flight
  a64.par = a32.par = 0;
  HIP_TRY(launch_init(MSC_PREC_FP64, a64, s));

  const int G = std::max(1, prm.poll_every);
  int phase = MSC_PREC_FP64;
  MsArgs* cur = &a64;
  int launched = 0, chunk = 0, launched_at_switch = -1, iter_at_switch = -1;
  bool done = prm.max_iter <= 0;
  EventPool pool;
  std::vector<int> sample_launch;
  while (!done) {
    for (int g = 0; g < G; ++g) {
      hipEvent_t* ev = nullptr;
      cur->sample = -1;
      // consecutive launches are sampled in runs as long as a folding cycle (heads that
      // defer and the one that applies the folded steps), in both phases of a mixed solve;
      // the FP64 phase of a mixed solve takes at most half of the records
      const int cap = mixed && phase == MSC_PREC_FP64 ? kMaxSamples / 2 : kMaxSamples;
      if (prm.timing > 0 && launched % prm.timing < std::max(2, prm.update_steps) &&
          int(sample_launch.size()) < cap) {
        ev = pool.next();
        if (!ev) {
          set_error("msc_solve: event creation failed");
          return MSC_EHIP;
        }
        cur->sample = int(sample_launch.size());
        sample_launch.push_back(launched);
      }
      // iteration `launched` starts from the state rot[launched & 1]; in the complex64
      // phase the reliable update (r recomputed in FP64 after the head has brought x_0 up
      // to date) is launched every kRuCheck-th iteration and on its period: it runs on
      // the period, or at a check when the recursive residual has fallen fast
      cur->par = launched & 1;
      const int since = launched - launched_at_switch;
      const bool ru_period = phase == MSC_PREC_MIXED && prm.reliable_every > 0 && since > 0 &&
                             since % prm.reliable_every == 0;
      const bool ru = ru_period || (phase == MSC_PREC_MIXED && prm.reliable_every > 0 &&
                                    since > 0 && since % kRuCheck == 0);
      cur->ru_force = ru_period ? 1 : 0;
      cur->ru_check = ru ? 1 : 0;
      // links, FP64: the head's product by the recurrence t' = M r + b t; a direct one in
      // the first launch (no old t yet) and every kTrEvery launches
      cur->t_rec = tr_launch(phase == MSC_PREC_FP64 && cur->stencil != 0, launched) ? 1 : 0;
      cur->defer_ok = 1;
      cur->steps = prm.update_steps;
      HIP_TRY(launch_iteration(phase, *cur, s, ev, ru));
      ++launched;
    }
    const int slot = chunk & 1;
    HIP_TRY(hipEventRecord(op->ws.ev[slot], s));
    ++chunk;
    if (chunk >= 2) {
      HIP_TRY(hipEventSynchronize(op->ws.ev[slot ^ 1]));
      // halt | switch_req << 1 of the newest state a head has written: at least as recent
      // as the end of that chunk (within a phase the halt only ever gets set)
      const int f = __atomic_load_n(op->ws.h_halt, __ATOMIC_ACQUIRE);
      if (f & 1) {
        if ((f & 2) && phase == MSC_PREC_FP64 && mixed) {
          // end of the FP64 phase: drain, convert the Krylov vectors, continue in complex64
          HIP_TRY(hipStreamSynchronize(s));
          __atomic_store_n(op->ws.h_halt, 0, __ATOMIC_RELEASE);
          HIP_TRY(hipMemcpy(&iter_at_switch, &op->ws.st->rot[launched & 1].iter, sizeof(int),
                            hipMemcpyDeviceToHost));
          a64.par = a32.par = launched & 1;
          HIP_TRY(launch_switch_to_mixed(a64, a32, ns, s));
          phase = MSC_PREC_MIXED;
          cur = &a32;
          launched_at_switch = launched;
          chunk = 0;
        } else {
          done = true;
        }
      }
    }
    if (launched >= prm.max_iter + 4 * G) done = true;
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(&h, op->ws.st, sizeof h, hipMemcpyDeviceToHost));
  const RotState& fin = h.rot[launched & 1];  // state after the last launched iteration
  const int iters_fp64 = iter_at_switch >= 0 ? iter_at_switch : fin.iter;
  if (info) {
    clear_timing(*info);
    // only iterations that did work are counted (the loop runs a little past the halt)
    const int first = launched_at_switch >= 0 ? launched_at_switch : 0;
    const int useful_launches = first + (fin.iter - (iter_at_switch >= 0 ? iter_at_switch : 0));
    // slot 2 (the separate update kernel) exists on the CSR path only
    const int slots = a64.sell ? 2 : 3;
    const double nn = double(op->n), nz = double(op->nnz), nzh = double(op->nnz_h);
    for (size_t q = 0; q < pool.groups.size(); ++q) {
      const int L = sample_launch[q];
      if (L >= useful_launches) continue;
      // FP64-phase launches between the switch request and the host's switch did no work
      if (launched_at_switch >= 0 && L < launched_at_switch && L >= iter_at_switch) continue;
      // the FP64 phase of a mixed solve is reported apart from its complex64 phase
      const bool ph32 = launched_at_switch >= 0 && L >= launched_at_switch;
      const bool apart = mixed && !ph32;
      double* kms = apart ? info->fp64_kernel_ms : info->kernel_ms;
      double* kby = apart ? info->fp64_kernel_bytes : info->kernel_bytes;
      for (int k = 0; k < slots; ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pool.groups[q][2 * k], pool.groups[q][2 * k + 1]));
        kms[k] += ms;
      }
      // the head's update mode and the shifts it listed, as recorded by the head itself
      const bool pending = !(L == 0 || (ph32 && L == launched_at_switch));
      const int act = h.smp_nact[q];
      // an applying head reads the m kept residuals (the deferring ones leave theirs in
      // the ring)
      const int kept = h.smp_mode[q] == 1 ? 0 : h.smp_m[q];
      const int phq = ph32 ? MSC_PREC_MIXED : MSC_PREC_FP64;
      const double wq = ph32 ? 8.0 : 16.0;
      const double x0b = h.smp_mode[q] == 0 ? 32.0 + (h.smp_m[q] > 0 ? wq : 0.0)
                                            : (h.smp_m[q] == 0 ? wq : 0.0);
      const KernelBytes kb =
          kernel_bytes(op->kind, phq, nn, mat_bytes(op->kind, phq, nn, nz, nzh, ib, ibh,
                                                   phq == MSC_PREC_FP64 ? a64.stencil : a32.stencil),
                       double(act), pending, kept, x0b);
      // a recurrence head also reads the old t (its own row)
      const bool trq = tr_launch(phq == MSC_PREC_FP64 && a64.stencil != 0, L);
      kby[0] += (a64.sell ? kb.head : kb.k1) + (trq ? 16.0 * nn : 0.0);
      kby[1] += kb.k2;
      if (!a64.sell) kby[2] += kb.upd;
      (apart ? info->fp64_kernel_samples : info->kernel_samples) += 1;
    }
  }

  // per-shift freeze iterations in the caller's order
  if (info && info->freeze_iter) {
    for (int j = 0; j < ns; ++j) {
      int fi = h.freeze_iter[j];
      if (j == 0 || (fi < 0 && h.s[j] == 0.0)) fi = (fin.R <= h.eps2) ? fin.iter : -1;
      info->freeze_iter[order[j]] = fi;
    }
  }
  *iters_out = fin.iter;
  *status_out = fin.status;
  if (info) info->n_reliable = h.n_reliable;

  // shift-vector updates and kept-r passes counted by the heads, per phase
  const double act64 = h.n_shift_upd[0], act32 = h.n_shift_upd[1];
  const double kept64 = h.n_two[0], kept32 = h.n_two[1];
  const double nn = double(op->n), nz = double(op->nnz), nzh = double(op->nnz_h);
  // x_0 (and its kept direction) per phase: applying heads read and write x_0, and each
  // cycle with deferred steps writes and reads the kept direction once
  const double x064 = 32.0 * h.n_apply[0] + 2.0 * 16.0 * h.n_keep0[0];
  const double x032 = 32.0 * h.n_apply[1] + 2.0 * 8.0 * h.n_keep0[1];
  *bytes_out = iter_bytes(op->kind, MSC_PREC_FP64, nn,
                          mat_bytes(op->kind, MSC_PREC_FP64, nn, nz, nzh, ib, ibh, a64.stencil), act64,
                          double(iters_fp64), kept64, x064) +
               iter_bytes(op->kind, MSC_PREC_MIXED, nn,
                          mat_bytes(op->kind, MSC_PREC_MIXED, nn, nz, nzh, ib, ibh, a32.stencil), act32,
                          double(fin.iter - iters_fp64), kept32, x032) +
               (a64.stencil != 0 ? 16.0 * nn * double(tr_launches(iters_fp64)) : 0.0) +
               double(h.n_reliable) *
                   ((a32.stencil != 0
                         ? [&] {
                             // the reliable update reads the FP64 links
                             const MatBytes rb = mat_bytes(op->kind, MSC_PREC_FP64, nn, nz, nzh, ib,
                                                           ibh, a32.stencil);
                             return rb.m + rb.mh;
                           }()
                         : nz * (16.0 + ib) + nzh * (16.0 + ibh) +
                               4.0 * (nn + 1) * (op->kind == MSC_A_MHM ? 2.0 : 1.0)) +
                    nn * (16.0 * 3 + 8.0));
  // the fused head reads the old direction once for the update and the product
  if (a64.sell) *bytes_out -= nn * (16.0 * iters_fp64 + 8.0 * (fin.iter - iters_fp64));
  if (info) info->iters_fp64 = iters_fp64;

  rel_out->assign(ns, 0.0);
  *bnorm_out = std::sqrt(h.bnorm2);
  if (prm.verify && fin.status == 0) {
    const double bn = std::sqrt(h.bnorm2);
    for (int k0 = 0; k0 < ns; k0 += 8) {
      const int kc = std::min(8, ns - k0);
      HIP_TRY(launch_verify(a64, op->sigma.data(), k0, kc, op->ws.u64, s));
    }
    std::vector<double> r2(ns);
    HIP_TRY(hipMemcpyAsync(r2.data(), op->scratch.res2, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < ns; ++k) (*rel_out)[k] = bn > 0 ? std::sqrt(r2[k]) / bn : 0.0;
    const double nvec = op->kind == MSC_A_MHM ? 2.0 : 1.0;
    *bytes_out += (nz * (16.0 + ib) + nzh * (16.0 + ibh) + nvec * 4.0 * (nn + 1)) * std::ceil(ns / 8.0) +
                  double(op->n) * 16.0 * ns * (op->kind == MSC_A_MHM ? 4.0 : 2.0) + 16.0 * op->n;
  }
  return MSC_OK;
}

void free_bss(BssWorkspace& w) {
  for (void* q : {w.p, w.t, w.r, w.e})
    if (q) (void)hipFree(q);
  dfree(w.st);
  if (w.h_halt) (void)hipHostFree(w.h_halt);
  for (auto& e : w.ev)
    if (e) (void)hipEventDestroy(e);
  w = BssWorkspace{};
}

msc_status ensure_bss(msc_op op, int prec, int mp, hipStream_t s) {
  BssWorkspace& w = op->bws;
  const size_t n = size_t(op->n);
  if (w.st && w.prec == prec && w.mp == mp && w.n == n) return MSC_OK;
  free_bss(w);
  const size_t bytes = (prec == MSC_PREC_MIXED ? sizeof(float2) : sizeof(double2)) * n * mp;
  for (void** q : {&w.p, &w.t, &w.r, &w.e}) {
    HIP_TRY(hipMalloc(q, bytes));
    HIP_TRY(hipMemsetAsync(*q, 0, bytes, s));
  }
  HIP_TRY(dalloc(&w.st, 1));
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.h_halt), 2 * sizeof(int),
                        hipHostMallocMapped | hipHostMallocCoherent));
  HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&w.d_halt), w.h_halt, 0));
  HIP_TRY(hipEventCreateWithFlags(&w.ev[0], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&w.ev[1], hipEventDisableTiming));
  w.n = n;
  w.mp = mp;
  w.prec = prec;
  return MSC_OK;
}

// FP64 residual norms (and, when write_vectors, the interleaved r = p = residual, e = 0)
// of systems j in [0, m): r_j = f_j - (A + sig_j) x_j.  res2 receives |r_j|^2.
msc_status batch_residual(msc_op op, int prec, int lanes, int m, int mp, const double* sig,
                          const double2* const* f, double2* const* x, bool write_vectors,
                          std::vector<double>& res2, hipStream_t s, double* bytes,
                          const msc_params& prm) {
  res2.assign(m, 0.0);
  for (int q0 = 0; q0 < m; q0 += kResChunk) {
    ResArgs v{};
    v.m1 = Csr<double2>{op->rowptr, op->col, op->val64};
    v.mhm = op->kind == MSC_A_MHM;
    v.m2 = v.mhm ? Csr<double2>{op->rowptr_h, op->col_h, op->val64_h} : v.m1;
    v.sell = op->sell && prm.format != MSC_FORMAT_CSR ? 1 : 0;
    if (v.sell) {
      const bool narrow = prm.format != MSC_FORMAT_SELL32;
      const SellStore &sm = op->sell_m, &sh = op->sell_mh;
      v.nslices = sm.nslices;
      v.s1 = sell_view(sm, sm.val64, sm.diag64, narrow);
      v.s2 = v.mhm ? sell_view(sh, sh.val64, sh.diag64, narrow) : v.s1;
    }
    v.n = op->n;
    v.kc = std::min(kResChunk, m - q0);
    v.mp = mp;
    v.j0 = q0;
    for (int q = 0; q < v.kc; ++q) {
      v.x[q] = x[q0 + q];
      v.f[q] = f[q0 + q];
      v.sig[q] = sig[q0 + q];
    }
    v.u = op->ws.u64;
    if (write_vectors) {
      v.r = op->bws.r;
      v.p = op->bws.p;
      v.e = op->bws.e;
    }
    v.partial = op->scratch.partial;
    v.ticket = op->scratch.tickets + 10 * kTicketSite;
    v.out = op->scratch.res2 + q0;
    HIP_TRY(launch_residual(prec, lanes, v, s));
    const double ib = index_bytes(v.sell, v.s1), ibh = v.mhm ? index_bytes(v.sell, v.s2) : 0.0;
    *bytes += double(op->nnz) * (16.0 + ib) + (v.mhm ? double(op->nnz) * (16.0 + ibh) : 0.0) +
              (v.mhm ? 2.0 : 1.0) * 4.0 * (op->n + 1) +
              double(op->n) * v.kc * 16.0 * (v.mhm ? 5.0 : 3.0);
  }
  HIP_TRY(hipMemcpyAsync(res2.data(), op->scratch.res2, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MSC_OK;
}

// Defect correction over m <= kBssMax systems sharing the operator:
//   repeat: r_j = f_j - (A + sig_j) x_j in FP64; stop when |r_j| <= tol_abs_j;
//           CG on (A + sig_j) e_j = r_j in the working precision from e = 0 until
//           |r_in| <= max(delta |r_j|, tol_abs_j / 2); x_j += e_j in FP64.
// On return res_abs[j] = |f_j - (A + sig_j) x_j| of the final iterates.
// The inner CG of a refinement cycle stops at this fraction of the outer tolerance (the
// next FP64 residual decides whether another cycle runs).
#ifndef MSC_REFINE_TARGET
#define MSC_REFINE_TARGET 0.7
#endif
constexpr double kRefineTarget = MSC_REFINE_TARGET;
msc_status run_batched_cg(msc_op op, int prec, int m, const double* sig, const double2* const* f,
                          double2* const* x, const double* tol_abs, double delta,
                          const msc_params& prm, hipStream_t s, std::vector<double>& res_abs,
                          int* inner_total, double* bytes, bool* breakdown) {
  *inner_total = 0;
  *breakdown = false;
  if (m < 1 || m > kBssMax) {
    set_error("batched CG: 1 <= m <= %d systems", kBssMax);
    return MSC_EINVAL;
  }
  const int mp = m <= 4 ? 4 : (m <= 8 ? 8 : 16);
  msc_status rc = ensure_scratch(op, s);
  if (rc != MSC_OK) return rc;
  rc = ensure_workspace(op, op->ws.prec >= 0 ? op->ws.prec : prec, std::max<int>(1, int(op->sigma.size())));
  if (rc != MSC_OK) return rc;
  rc = ensure_bss(op, prec, mp, s);
  if (rc != MSC_OK) return rc;
  const int lanes = choose_lanes(op, prm);
  BssArgs a{};
  a.kind = op->kind;
  a.mp = mp;
  a.n = op->n;
  a.m64 = Csr<double2>{op->rowptr, op->col, op->val64};
  a.m32 = Csr<float2>{op->rowptr, op->col, op->val32};
  if (op->kind == MSC_A_MHM) {
    a.mh64 = Csr<double2>{op->rowptr_h, op->col_h, op->val64_h};
    a.mh32 = Csr<float2>{op->rowptr_h, op->col_h, op->val32_h};
  }
  // the SpMVs read the sliced ELLPACK copies where they exist (as the multishift does),
  // up to 8 systems (16 gathered FP64 values per entry exceed the register budget)
  a.sell = op->sell && prm.format != MSC_FORMAT_CSR && mp <= 8 ? 1 : 0;
  if (a.sell) {
    const bool narrow = prm.format != MSC_FORMAT_SELL32;
    const SellStore &sm = op->sell_m, &sh = op->sell_mh;
    a.nslices = sm.nslices;
    a.s64 = sell_view(sm, sm.val64, sm.diag64, narrow);
    a.s32 = sell_view(sm, sm.val32, sm.diag32, narrow);
    if (op->kind == MSC_A_MHM) {
      a.sh64 = sell_view(sh, sh.val64, sh.diag64, narrow);
      a.sh32 = sell_view(sh, sh.val32, sh.diag32, narrow);
    }
  }
  a.p = op->bws.p;
  a.t = op->bws.t;
  a.r = op->bws.r;
  a.e = op->bws.e;
  a.st = op->bws.st;
  a.partial = op->scratch.partial;
  a.tickets = op->scratch.tickets;
  a.hflag = op->bws.d_halt;
  XPtrs xp{};
  for (int j = 0; j < m; ++j) xp.x[j] = x[j];

  const double w = prec == MSC_PREC_MIXED ? 8.0 : 16.0;
  const double mat = double(op->nnz) * (w + index_bytes(a.sell, a.s64)) +
                     double(op->nnz_h) * (w + index_bytes(a.sell, a.sh64)) +
                     4.0 * (op->n + 1) * (op->kind == MSC_A_MHM ? 2.0 : 1.0);
  const int max_cycles = 12;
  std::vector<double> res2;
  for (int cycle = 0;; ++cycle) {
    rc = batch_residual(op, prec, lanes, m, mp, sig, f, x, true, res2, s, bytes, prm);
    if (rc != MSC_OK) return rc;
    bool all_done = true;
    BssState h{};
    h.m = m;
    h.mp = mp;
    h.max_iter = prm.refine_max_iter;
    for (int j = 0; j < kBssMax; ++j) h.R[j] = 1.0;
    for (int j = 0; j < m; ++j) {
      const double rn = std::sqrt(res2[j]);
      h.sigma[j] = sig[j];
      h.R[j] = res2[j];
      const bool done = !(rn > tol_abs[j]);
      if (!std::isfinite(rn)) *breakdown = true;
      h.active[j] = (done || !std::isfinite(rn)) ? 0 : 1;
      const double tgt = std::max(delta * rn, kRefineTarget * tol_abs[j]);
      h.target2[j] = tgt * tgt;
      if (h.active[j]) all_done = false;
    }
    res_abs.assign(m, 0.0);
    for (int j = 0; j < m; ++j) res_abs[j] = std::sqrt(res2[j]);
    if (all_done || cycle >= max_cycles || *breakdown) break;
    HIP_TRY(hipMemcpyAsync(op->bws.st, &h, sizeof h, hipMemcpyHostToDevice, s));
    __atomic_store_n(op->bws.h_halt, 0, __ATOMIC_RELEASE);  // the previous cycle has drained
    // chunks of 2, 4, 8, ... iterations up to poll_every: a correction solve often needs
    // only a few iterations, and the halt flag of a chunk is read after the next one is
    // queued
    const int G = std::max(1, prm.poll_every);
    int launched = 0, chunk = 0;
    bool done = false;
    while (!done) {
      const int cg = std::min(G, 2 << std::min(chunk, 20));
      for (int g = 0; g < cg; ++g) {
        HIP_TRY(launch_bss_iteration(prec, a, s));
        ++launched;
      }
      const int slot = chunk & 1;
      HIP_TRY(hipEventRecord(op->bws.ev[slot], s));
      if (chunk >= 1) {
        HIP_TRY(hipEventSynchronize(op->bws.ev[slot ^ 1]));
        // set by the last IK2 once every system is done (it only ever gets set)
        if (__atomic_load_n(op->bws.h_halt, __ATOMIC_ACQUIRE)) done = true;
      }
      if (launched >= prm.refine_max_iter + 2 * G) done = true;
      ++chunk;
    }
    HIP_TRY(launch_accum(prec, a, xp, s));
    HIP_TRY(hipMemcpyAsync(&h, op->bws.st, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j < m; ++j)
      if (h.bad[j]) *breakdown = true;
    *inner_total += h.iter;
    *bytes += double(h.iter) * (mat + double(op->n) * mp * w * 11.0) +
              double(op->n) * m * (16.0 * 2.0 + w);
    if (*breakdown) break;
  }
  return MSC_OK;
}

// Inner precision of the per-shift refinement (defect correction: FP64 residuals outside,
// batched CG inside).  Shifts that miss tol by a small factor (the usual case after a
// mixed solve: well under one digit to gain) are refined in FP64 in one inner solve; when
// some shift is more than kRefineMixedGap x tol away, the inner CG runs in complex64, each
// cycle reducing its residual kRefineDelta times before the next FP64 residual.
constexpr double kRefineMixedGap = 1e3;
constexpr double kRefineDelta = 1e-4;
int refine_precision(const std::vector<double>& rel, const std::vector<int>& todo,
                     const msc_params& prm) {
  if (prm.prec != MSC_PREC_MIXED) return MSC_PREC_FP64;
  double worst = 0.0;
  for (int k : todo) worst = std::max(worst, std::isfinite(rel[k]) ? rel[k] : HUGE_VAL);
  return worst > kRefineMixedGap * prm.tol ? MSC_PREC_MIXED : MSC_PREC_FP64;
}

// The full solve: multishift sequence, FP64 verification of every shift, and batched
// refinement of the shifts whose true residual is above tol.  With the mixed path and
// refinement on, shifts that the complex64 phase left slightly above tol are refined in
// FP64.
msc_status solve_impl(msc_op op, const double* d_b, double* d_x, const msc_params& prm,
                      msc_info* info, hipStream_t s) {
  const int ns = int(op->sigma.size());
  std::vector<double> rel;
  int iters = 0, status = 0;
  double bytes = 0.0;
  double bnorm = 0.0;
  const bool refine = prm.refine && prm.verify;
  const double tol_stop = prm.prec == MSC_PREC_MIXED ? prm.tol * prm.mixed_margin : prm.tol;
  msc_status rc = run_multishift(op, d_b, d_x, prm, info, s, tol_stop, prm.prec, &rel, &iters,
                                 &status, &bytes, &bnorm);
  if (rc != MSC_OK) return rc;
  int refine_iters = 0, n_refined = 0;
  msc_status result = MSC_OK;
  if (status != 0) {
    set_error("msc_solve: breakdown (p^H (A+sigma_min) p <= 0 or not finite) at iteration %d", iters);
    result = MSC_EBREAKDOWN;
  } else if (prm.verify) {
    std::vector<int> todo;
    for (int k = 0; k < ns; ++k)
      if (!(rel[k] <= prm.tol)) todo.push_back(k);
    if (refine && !todo.empty() && bnorm > 0.0) {
      n_refined = int(todo.size());
      const int rprec = refine_precision(rel, todo, prm);
      const double delta = rprec == MSC_PREC_MIXED ? kRefineDelta : 0.0;
      for (size_t g0 = 0; g0 < todo.size(); g0 += kBssMax) {
        const int m = int(std::min<size_t>(kBssMax, todo.size() - g0));
        std::vector<double> sig(m), tol_abs(m), res;
        std::vector<const double2*> f(m);
        std::vector<double2*> x(m);
        for (int j = 0; j < m; ++j) {
          const int k = todo[g0 + j];
          sig[j] = op->sigma[k];
          tol_abs[j] = prm.tol * bnorm;
          f[j] = reinterpret_cast<const double2*>(d_b);
          x[j] = reinterpret_cast<double2*>(d_x) + int64_t(k) * op->n;
        }
        int inner = 0;
        bool bd = false;
        rc = run_batched_cg(op, rprec, m, sig.data(), f.data(), x.data(), tol_abs.data(), delta,
                            prm, s, res, &inner, &bytes, &bd);
        if (rc != MSC_OK) return rc;
        refine_iters += inner;
        for (int j = 0; j < m; ++j) rel[todo[g0 + j]] = res[j] / bnorm;
        if (bd) status = 1;
      }
    }
    if (status != 0) {
      set_error("msc_solve: breakdown during refinement");
      result = MSC_EBREAKDOWN;
    } else {
      for (int k = 0; k < ns; ++k)
        if (!(rel[k] <= prm.tol)) result = MSC_ENOTCONV;
      if (result == MSC_ENOTCONV) set_error("msc_solve: some shift did not reach tol");
    }
  }
  if (info) {
    info->iters = iters;
    info->refine_iters = refine_iters;
    info->n_refined = n_refined;
    if (info->true_rel_res)
      for (int k = 0; k < ns; ++k) info->true_rel_res[k] = rel[k];
    info->alg_bytes = bytes;
  }
  return result;
}

// ---- batched solves --------------------------------------------------------------------

// Batch launch choices, measured once per batch shape and kept in process; with the
// environment variable MSC_TUNE_CACHE naming a file, also on disk (read at the first
// batched solve, one line appended per new shape: "<key> = <sell> <lanes> <grid>").
// The key: systems, right-hand sides per system, total rows and entries, the requested
// format and lanes, and the total row-length histogram (rows with 0, 1, 2-3, ..., >= 64
// entries) of the batch.
struct TuneChoice {
  int sell, lanes, grid;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;
bool g_tune_loaded = false;

void tune_cache_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("MSC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char* eq = std::strchr(line, '=');
    if (!eq) continue;
    TuneChoice c{};
    if (std::sscanf(eq + 1, "%d %d %d", &c.sell, &c.lanes, &c.grid) != 3) continue;
    if ((c.lanes != 4 && c.lanes != 8 && c.lanes != 16) || c.grid < 8 || c.grid > kMaxGrid ||
        (c.sell != 0 && c.sell != 1))
      continue;
    std::string key(line, size_t(eq - line));
    while (!key.empty() && key.back() == ' ') key.pop_back();
    g_tune_cache[key] = c;
  }
  std::fclose(f);
}

void tune_cache_store_locked(const std::string& key, const TuneChoice& c) {
  g_tune_cache[key] = c;
  const char* path = std::getenv("MSC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s = %d %d %d\n", key.c_str(), c.sell, c.lanes, c.grid);
  std::fclose(f);
}

struct BatchRun {
  int nsys = 0, rr = 1, nchunks = 0, lanes = 8, grid = 8;
  const msc_op* ops = nullptr;
  const int32_t* nrhs = nullptr;
  const double* const* d_b = nullptr;
  double* const* d_x = nullptr;
  std::vector<BatchSys> sys;
  std::vector<int4> chunks;
  std::vector<BatchState> hst;
  void* pool = nullptr;
  BatchSys* d_sys = nullptr;
  int4* d_chunks = nullptr;
  BatchState* d_st = nullptr;
  unsigned* d_tickets = nullptr;
  int* d_active = nullptr;
  int* h_poll = nullptr;
  hipStream_t sint = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t ev_sync = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int replays = 0, n_reliable_launches = 0;

  ~BatchRun() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (sint) (void)hipStreamSynchronize(sint);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
    if (ev_sync) (void)hipEventDestroy(ev_sync);
    if (sint) (void)hipStreamDestroy(sint);
    if (h_poll) (void)hipHostFree(h_poll);
    if (pool) (void)hipFree(pool);
  }

  msc_status setup(int nsys_, const msc_op* ops_, const int32_t* nrhs_, const double* const* b_,
                   double* const* x_, int rr_, const msc_params& prm) {
    nsys = nsys_;
    ops = ops_;
    nrhs = nrhs_;
    d_b = b_;
    d_x = x_;
    rr = rr_;
    // sizes of the pool
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t bytes = 0;
    std::vector<size_t> off(nsys);
    for (int s = 0; s < nsys; ++s) {
      const size_t n = size_t(ops[s]->n), nk = std::max<size_t>(ops[s]->sigma.size() - 1, 1);
      const size_t nch = (n + kBatchChunkRows - 1) / kBatchChunkRows;
      off[s] = bytes;
      bytes += (5 + kBatchMaxSteps - 1) * align(sizeof(double2) * n * rr) +
               align(sizeof(double2) * n * rr * nk) +
               3 * align(sizeof(float2) * n * rr) + align(sizeof(float2) * n * rr * nk) +
               align(sizeof(double) * nch * kBatchMaxRhs);
      for (size_t c = 0; c < nch; ++c) {
        const int64_t r0 = int64_t(c) * kBatchChunkRows;
        const int64_t r1 = std::min<int64_t>(r0 + kBatchChunkRows, int64_t(n));
        chunks.push_back(int4{s, int(r0), int(r1), int(c)});
      }
    }
    nchunks = int(chunks.size());
    const size_t off_sys = bytes;
    bytes += align(sizeof(BatchSys) * nsys);
    const size_t off_ch = bytes;
    bytes += align(sizeof(int4) * nchunks);
    const size_t off_st = bytes;
    bytes += align(sizeof(BatchState) * nsys);
    const size_t off_tk = bytes;
    bytes += align(sizeof(unsigned) * 4 * kTicketSite * nsys);
    const size_t off_act = bytes;
    bytes += 256;
    HIP_TRY(hipMalloc(&pool, bytes));
    char* base = static_cast<char*>(pool);
    d_sys = reinterpret_cast<BatchSys*>(base + off_sys);
    d_chunks = reinterpret_cast<int4*>(base + off_ch);
    d_st = reinterpret_cast<BatchState*>(base + off_st);
    d_tickets = reinterpret_cast<unsigned*>(base + off_tk);
    d_active = reinterpret_cast<int*>(base + off_act);
    sys.resize(nsys);
    hst.assign(nsys, BatchState{});
    const double sw = prm.prec == MSC_PREC_MIXED ? std::max(prm.switch_tol, prm.tol) : 0.0;
    for (int s = 0; s < nsys; ++s) {
      const msc_op op = ops[s];
      const size_t n = size_t(op->n), nk = std::max<size_t>(op->sigma.size() - 1, 1);
      char* p = base + off[s];
      auto take = [&](size_t b) {
        char* q = p;
        p += align(b);
        return q;
      };
      BatchSys& S = sys[s];
      S.kind = op->kind;
      S.n = op->n;
      S.nchunks = int((n + kBatchChunkRows - 1) / kBatchChunkRows);
      S.m64 = Csr<double2>{op->rowptr, op->col, op->val64};
      S.m32 = Csr<float2>{op->rowptr, op->col, op->val32};
      if (op->kind == MSC_A_MHM) {
        S.mh64 = Csr<double2>{op->rowptr_h, op->col_h, op->val64_h};
        S.mh32 = Csr<float2>{op->rowptr_h, op->col_h, op->val32_h};
      }
      S.sell = 0;  // chosen by tune()
      if (op->sell) {
        const SellStore& sm = op->sell_m;
        const bool narrow = prm.format != MSC_FORMAT_SELL32;
        S.s64 = sell_view(sm, sm.val64, sm.diag64, narrow);
        S.s32 = sell_view(sm, sm.val32, sm.diag32, narrow);
        if (op->kind == MSC_A_MHM) {
          const SellStore& sh = op->sell_mh;
          S.sh64 = sell_view(sh, sh.val64, sh.diag64, narrow);
          S.sh32 = sell_view(sh, sh.val32, sh.diag32, narrow);
        }
      }
      S.b = reinterpret_cast<const double2*>(d_b[s]);
      S.x = reinterpret_cast<double2*>(d_x[s]);
      S.r64 = reinterpret_cast<double2*>(take(sizeof(double2) * n * rr));
      S.p64 = reinterpret_cast<double2*>(take(sizeof(double2) * n * rr));
      S.t64 = reinterpret_cast<double2*>(take(sizeof(double2) * n * rr));
      S.u64 = reinterpret_cast<double2*>(take(sizeof(double2) * n * rr));
      for (auto& q : S.rkeep) q = take(sizeof(double2) * n * rr);
      S.pkeep0 = take(sizeof(double2) * n * rr);
      S.pk64 = reinterpret_cast<double2*>(take(sizeof(double2) * n * rr * nk));
      S.r32 = reinterpret_cast<float2*>(take(sizeof(float2) * n * rr));
      S.p32 = reinterpret_cast<float2*>(take(sizeof(float2) * n * rr));
      S.t32 = reinterpret_cast<float2*>(take(sizeof(float2) * n * rr));
      S.pk32 = reinterpret_cast<float2*>(take(sizeof(float2) * n * rr * nk));
      S.partial = reinterpret_cast<double*>(take(sizeof(double) * S.nchunks * kBatchMaxRhs));
      S.tickets = d_tickets + 4 * kTicketSite * s;
      S.st = d_st + s;
      // scalar state: shifts sorted ascending, the smallest drives
      const int ns = int(op->sigma.size());
      std::vector<int> order(ns);
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(),
                       [&](int i, int j) { return op->sigma[i] < op->sigma[j]; });
      BatchState& h = hst[s];
      h.sigma0 = op->sigma[order[0]];
      h.ns = ns;
      h.nrhs = nrhs[s];
      h.max_iter = prm.max_iter;
      h.iters_fp64 = -1;
      for (int k = 0; k < ns; ++k) {
        h.s[k] = op->sigma[order[k]] - h.sigma0;
        h.orig[k] = order[k];
      }
      for (int q = 0; q < kBatchMaxRhs; ++q) {
        const double ts = prm.prec == MSC_PREC_MIXED ? prm.tol * prm.mixed_margin : prm.tol;
        h.eps2[q] = ts * ts;
        h.sw_eps2[q] = sw * sw;
        h.a_prev[q] = 1.0;
        h.b[q] = 0.0;
        h.R[q] = 1.0;
        for (int k = 0; k < kBatchMaxShifts; ++k) {
          const int lk = q * kBatchMaxShifts + k;
          h.zeta[lk] = h.zeta_prev[lk] = 1.0;
          h.active[lk] = (q < nrhs[s] && k >= 1 && k < ns) ? 1 : 0;
          h.freeze_iter[lk] = -1;
        }
      }
    }
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h_poll), 4 * sizeof(int), hipHostMallocDefault));
    HIP_TRY(hipStreamCreateWithFlags(&sint, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ev_sync, hipEventDisableTiming));
    return MSC_OK;
  }

  BatchArgs args() const {
    BatchArgs a{};
    a.sys = d_sys;
    a.chunks = d_chunks;
    a.nchunks = nchunks;
    a.nsys = nsys;
    a.grid = grid;
    a.lanes = lanes;
    a.rr = rr;
    a.active_systems = d_active;
    return a;
  }

  // upload the descriptors and the initial state, then r = p = p_k = b, x = 0
  msc_status reset(hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(d_sys, sys.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_chunks, chunks.data(), sizeof(int4) * nchunks, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_st, hst.data(), sizeof(BatchState) * nsys, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(d_tickets, 0, sizeof(unsigned) * 4 * kTicketSite * nsys, s));
    HIP_TRY(hipMemcpyAsync(d_active, &nsys, sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_batch_init(args(), s));
    return MSC_OK;
  }

  // Launch choices of the batch, measured on this batch over a few iterations of each
  // candidate and cached per shape: the SpMV layout -- the sliced ELLPACK copies (one row
  // per lane, 64 rows per wavefront; systems without a copy use CSR) or CSR throughout
  // with 4, 8 or 16 lanes per row (16, 8 or 4 rows per wavefront) -- times the grid of
  // the persistent kernels (all chunks' worth up to kMaxGrid, or half of it).
  // msc_params.format / lanes / max_grid narrow the candidates.
  msc_status tune(const msc_params& prm) {
    const bool fixed_lanes = prm.lanes == 4 || prm.lanes == 8 || prm.lanes == 16;
    bool any_sell = false;
    for (int s = 0; s < nsys; ++s) any_sell = any_sell || ops[s]->sell;
    std::vector<std::pair<bool, int>> layouts;  // (sliced ELLPACK where built, lanes)
    if (any_sell && prm.format != MSC_FORMAT_CSR) layouts.push_back({true, fixed_lanes ? prm.lanes : 8});
    if ((prm.format != MSC_FORMAT_SELL && prm.format != MSC_FORMAT_SELL32) || !any_sell) {
      if (fixed_lanes)
        layouts.push_back({false, prm.lanes});
      else
        for (int l : {4, 8, 16}) layouts.push_back({false, l});
    }
    const int full = grid;
    std::vector<int> grids{full};
    const int half = std::max(8, full / 2 / kXcds * kXcds);
    if (prm.max_grid <= 0 && half < full) grids.push_back(half);
    std::vector<TuneChoice> cands;
    for (const auto& l : layouts)
      for (int g : grids) cands.push_back(TuneChoice{l.first ? 1 : 0, l.second, g});
    auto apply = [&](const TuneChoice& c) {
      lanes = c.lanes;
      grid = c.grid;
      for (int s = 0; s < nsys; ++s) sys[s].sell = (c.sell && ops[s]->sell) ? 1 : 0;
    };
    if (cands.size() == 1) {
      apply(cands[0]);
      return MSC_OK;
    }
    int64_t rows = 0, nnz = 0, hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < nsys; ++s) {
      rows += ops[s]->n;
      nnz += ops[s]->nnz;
      for (int k = 0; k < 8; ++k) hist[k] += ops[s]->rowhist[k];
    }
    char kb[320];
    std::snprintf(kb, sizeof kb, "batch sys %d rhs %d rows %lld nnz %lld format %d lanes %d grid %d hist",
                  nsys, rr, (long long)rows, (long long)nnz, prm.format, prm.lanes, full);
    std::string key(kb);
    for (int k = 0; k < 8; ++k) key += " " + std::to_string(hist[k]);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_cache_load_locked();
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        TuneChoice c = it->second;
        // a cached layout is used only where it is still a candidate (the copies exist)
        bool ok = false;
        for (const auto& d : cands) ok = ok || (d.sell == c.sell && d.lanes == c.lanes && d.grid == c.grid);
        if (ok) {
          apply(c);
          return MSC_OK;
        }
      }
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    TuneChoice best_c = cands[0];
    for (const auto& c : cands) {
      apply(c);
      msc_status rc = reset(sint);
      if (rc != MSC_OK) return rc;
      HIP_TRY(launch_batch_iteration(args(), sint));  // warm-up
      HIP_TRY(hipEventRecord(e0, sint));
      for (int i = 0; i < 4; ++i) HIP_TRY(launch_batch_iteration(args(), sint));
      HIP_TRY(hipEventRecord(e1, sint));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_c = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    apply(best_c);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_store_locked(key, best_c);
    return MSC_OK;
  }

  msc_status solve(const msc_params& prm, hipStream_t user) {
    grid = std::max(8, std::min(nchunks, kMaxGrid));
    if (prm.max_grid > 0) grid = std::max(8, std::min(grid, prm.max_grid));
    // order the internal stream after the caller's prior work
    HIP_TRY(hipEventRecord(ev_sync, user));
    HIP_TRY(hipStreamWaitEvent(sint, ev_sync, 0));
    msc_status rc = tune(prm);
    if (rc != MSC_OK) return rc;
    rc = reset(sint);
    if (rc != MSC_OK) return rc;
    // G iterations captured once, replayed until every system has finished
    const int G = std::max(1, prm.poll_every);
    HIP_TRY(hipStreamBeginCapture(sint, hipStreamCaptureModeThreadLocal));
    for (int g = 0; g < G; ++g) {
      // BK3 may defer its shifted update except in the graph's last iteration (a reliable
      // update or the end of the solve may follow it)
      BatchArgs ga = args();
      const int steps = std::min(prm.update_steps, kBatchMaxSteps);
      ga.defer_ok = (steps > 1 && g < G - 1) ? 1 : 0;
      ga.steps = steps;
      hipError_t e = launch_batch_iteration(ga, sint);
      if (e != hipSuccess) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(sint, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        set_error("batched iteration capture failed: %s", hipGetErrorString(e));
        return MSC_EHIP;
      }
    }
    HIP_TRY(hipStreamEndCapture(sint, &graph));
    HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    const int ru_every = (prm.prec == MSC_PREC_MIXED && prm.reliable_every > 0)
                             ? std::max(1, prm.reliable_every / G) : 0;
    const int max_replays = (prm.max_iter + G - 1) / G + 4;
    int chunk = 0;
    bool done = false;
    while (!done) {
      HIP_TRY(hipGraphLaunch(gexec, sint));
      ++replays;
      if (ru_every > 0 && replays % ru_every == 0) {
        HIP_TRY(launch_batch_reliable(args(), sint));
        ++n_reliable_launches;
      }
      const int slot = chunk & 1;
      HIP_TRY(hipMemcpyAsync(&h_poll[slot], d_active, sizeof(int), hipMemcpyDeviceToHost, sint));
      HIP_TRY(hipEventRecord(ev[slot], sint));
      ++chunk;
      if (chunk >= 2) {
        HIP_TRY(hipEventSynchronize(ev[slot ^ 1]));
        if (h_poll[slot ^ 1] <= 0) done = true;
      }
      if (replays >= max_replays) done = true;
    }
    HIP_TRY(hipStreamSynchronize(sint));
    HIP_TRY(hipMemcpy(hst.data(), d_st, sizeof(BatchState) * nsys, hipMemcpyDeviceToHost));
    return MSC_OK;
  }

  msc_status finish(const msc_params& prm, msc_info* info, hipStream_t user,
                    std::chrono::steady_clock::time_point t0) {
    msc_status result = MSC_OK;
    // every (system, rhs) verification is queued first, each writing its own slot, and
    // read back with one copy
    int total = 0;
    for (int s = 0; s < nsys; ++s) total += nrhs[s];
    double* d_res2 = nullptr;
    std::vector<double> r2all(size_t(total) * kMaxShifts, 0.0);
    struct Res2Guard {
      double*& p;
      ~Res2Guard() { dfree(p); }
    } res2_guard{d_res2};
    if (prm.verify) {
      HIP_TRY(dalloc(&d_res2, size_t(total) * kMaxShifts));
      int t = 0;
      for (int s = 0; s < nsys; ++s) {
        const msc_op op = ops[s];
        const int ns = int(op->sigma.size());
        const int64_t n = op->n;
        msc_status rc = ensure_scratch(op, sint);
        if (rc != MSC_OK) return rc;
        rc = ensure_workspace(op, MSC_PREC_FP64, ns);
        if (rc != MSC_OK) return rc;
        for (int q = 0; q < nrhs[s]; ++q, ++t) {
          if (hst[s].status[q] != 0) continue;
          MsArgs a = make_args(op, choose_lanes(op, prm), d_b[s] + 2 * int64_t(q) * n,
                               d_x[s] + 2 * int64_t(q) * ns * n);
          a.sc.res2 = d_res2 + size_t(t) * kMaxShifts;
          for (int k0 = 0; k0 < ns; k0 += 8)
            HIP_TRY(launch_verify(a, op->sigma.data(), k0, std::min(8, ns - k0), op->ws.u64, sint));
        }
      }
      HIP_TRY(hipMemcpyAsync(r2all.data(), d_res2, sizeof(double) * r2all.size(),
                             hipMemcpyDeviceToHost, sint));
      HIP_TRY(hipStreamSynchronize(sint));
    }
    int t = 0;
    for (int s = 0; s < nsys; ++s) {
      const msc_op op = ops[s];
      const int ns = int(op->sigma.size());
      const int64_t n = op->n;
      const BatchState& h = hst[s];
      for (int q = 0; q < nrhs[s]; ++q, ++t) {
        const double* bq = d_b[s] + 2 * int64_t(q) * n;
        double* xq = d_x[s] + 2 * int64_t(q) * ns * n;
        std::vector<double> rel(ns, 0.0);
        const double bn = std::sqrt(h.bnorm2[q]);
        int refine_iters = 0, n_refined = 0;
        bool bd = h.status[q] != 0;
        const bool bd_seq = bd;
        if (!bd && prm.verify) {
          const double* r2 = r2all.data() + size_t(t) * kMaxShifts;
          std::vector<int> todo;
          for (int k = 0; k < ns; ++k) {
            rel[k] = bn > 0 ? std::sqrt(r2[k]) / bn : 0.0;
            if (!(rel[k] <= prm.tol)) todo.push_back(k);
          }
          if (prm.refine && !todo.empty() && bn > 0) {
            n_refined = int(todo.size());
            std::vector<double> sig(todo.size()), tol_abs(todo.size()), res;
            std::vector<const double2*> f(todo.size());
            std::vector<double2*> xs(todo.size());
            for (size_t j = 0; j < todo.size(); ++j) {
              sig[j] = op->sigma[todo[j]];
              tol_abs[j] = prm.tol * bn;
              f[j] = reinterpret_cast<const double2*>(bq);
              xs[j] = reinterpret_cast<double2*>(xq) + int64_t(todo[j]) * n;
            }
            double bytes = 0.0;
            bool b1 = false;
            const int rprec = refine_precision(rel, todo, prm);
            const msc_status rc = run_batched_cg(op, rprec, int(todo.size()), sig.data(), f.data(), xs.data(),
                                tol_abs.data(), rprec == MSC_PREC_MIXED ? kRefineDelta : 0.0, prm,
                                sint, res, &refine_iters, &bytes, &b1);
            if (rc != MSC_OK) return rc;
            bd = bd || b1;
            for (size_t j = 0; j < todo.size(); ++j) rel[todo[j]] = res[j] / bn;
          }
        }
        if (bd) {
          result = MSC_EBREAKDOWN;
          set_error("msc_solve_batched: breakdown in system %d rhs %d (%s, iteration %d)", s, q,
                    bd_seq ? "multishift sequence" : "refinement", h.iter[q]);
        } else if (prm.verify) {
          for (int k = 0; k < ns; ++k)
            if (!(rel[k] <= prm.tol) && result == MSC_OK) {
              result = MSC_ENOTCONV;
              set_error("msc_solve_batched: system %d rhs %d did not reach tol", s, q);
            }
        }
        if (info) {
          msc_info& I = info[t];
          I.iters = h.iter[q];
          I.refine_iters = refine_iters;
          I.n_refined = n_refined;
          I.n_reliable = h.n_reliable;
          I.iters_fp64 = h.iters_fp64 >= 0 ? h.iters_fp64 : h.iter[q];
          if (I.true_rel_res)
            for (int k = 0; k < ns; ++k) I.true_rel_res[k] = rel[k];
          if (I.freeze_iter)
            for (int k = 0; k < ns; ++k) {
              const int fi = h.freeze_iter[q * kBatchMaxShifts + k];
              I.freeze_iter[h.orig[k]] = (k == 0 || fi < 0) ? h.iter[q] : fi;
            }
          clear_timing(I);
          // algorithmic bytes: this system's share, matrix read once for all its rhs; the
          // shift-vector updates and kept-r passes as counted by BK2 per phase
          const int it = h.iter[q], i64 = std::min(I.iters_fp64, it);
          const double act64 = h.n_upd[q][0], act32 = h.n_upd[q][1];
          const double kept64 = h.n_kept[q][0], kept32 = h.n_kept[q][1];
          // x_0 read and written by the BK3s that applied, p kept and read back once per
          // cycle of deferred steps
          const double x064 = 32.0 * h.n_x0[q][0] + 2.0 * 16.0 * h.n_k0[q][0];
          const double x032 = 32.0 * h.n_x0[q][1] + 2.0 * 8.0 * h.n_k0[q][1];
          const double nn = double(n), nz = double(op->nnz), nzh = double(op->nnz_h);
          const double ib = index_bytes(sys[s].sell, sys[s].s64);
          const double ibh = index_bytes(sys[s].sell, sys[s].sh64);
          I.alg_bytes = iter_bytes(op->kind, MSC_PREC_FP64, nn,
                                   mat_bytes(op->kind, MSC_PREC_FP64, nn, nz, nzh, ib, ibh, false),
                                   act64, i64, kept64, x064) +
                        iter_bytes(op->kind, MSC_PREC_MIXED, nn,
                                   mat_bytes(op->kind, MSC_PREC_MIXED, nn, nz, nzh, ib, ibh, false),
                                   act32, it - i64, kept32, x032) -
                        (double(nrhs[s]) - 1.0) / double(nrhs[s]) *
                            ((nz * (16.0 + ib) + nzh * (16.0 + ibh)) * i64 +
                             (nz * (8.0 + ib) + nzh * (8.0 + ibh)) * (it - i64));
          I.seconds = 0.0;
        }
      }
    }
    HIP_TRY(hipEventRecord(ev_sync, sint));
    HIP_TRY(hipStreamWaitEvent(user, ev_sync, 0));
    HIP_TRY(hipStreamSynchronize(sint));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
      for (int i = 0; i < t; ++i) info[i].seconds = secs;
    return result;
  }
};

msc_status check_op(msc_op op) {
  if (!op) {
    set_error("null operator");
    return MSC_EINVAL;
  }
  return MSC_OK;
}

}  // namespace

// New values of the stored matrix (same pattern): copies, casts, M^H and sliced copies.
msc_status update_values_impl(msc_op op, const double* d_vals, hipStream_t s);

// Links of a staggered operator in SU(3) (to 1e-12) are also kept as their first two
// rows, which the iteration reads (it rebuilds the third); otherwise that copy is off.
constexpr double kSu3Tol = 1e-12;
msc_status refresh_two_rows(msc_op op, const double2* d_links, hipStream_t s) {
  const int64_t nlinks = 4 * op->w64.vol;
  unsigned long long* d_dev = nullptr;
  HIP_TRY(dalloc(&d_dev, 1));
  unsigned long long bits = 0;
  hipError_t e = hipMemsetAsync(d_dev, 0, sizeof(unsigned long long), s);
  if (e == hipSuccess) e = launch_su3_deviation(d_links, nlinks, d_dev, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&bits, d_dev, sizeof bits, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_dev);
  if (e != hipSuccess) {
    set_error("SU(3) check of the links: %s", hipGetErrorString(e));
    return MSC_EHIP;
  }
  double dev = 0.0;
  std::memcpy(&dev, &bits, sizeof dev);
  op->two_rows = false;
  if (!(dev <= kSu3Tol)) return MSC_OK;
  if (!op->wc64.w) {
    double2* w64 = nullptr;
    float2* w32 = nullptr;
    HIP_TRY(dalloc(&w64, size_t(6) * size_t(nlinks)));
    e = dalloc(&w32, size_t(6) * size_t(nlinks));
    if (e != hipSuccess) {
      dfree(w64);
      set_error("two-row links: %s", hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? MSC_ENOMEM : MSC_EHIP;
    }
    op->wc64 = op->w64;
    op->wc64.w = w64;
    op->wc64.rows = 2;
    op->wc32 = op->w32;
    op->wc32.w = w32;
    op->wc32.rows = 2;
  }
  HIP_TRY(launch_two_rows(op->w64.w, nlinks, const_cast<double2*>(op->wc64.w),
                          const_cast<float2*>(op->wc32.w), s));
  op->two_rows = true;
  return MSC_OK;
}

struct MultiRhsOut {
  int iters = 0, refine_iters = 0, n_refined = 0;
  bool breakdown = false;
  std::vector<double> rel;  // per shift, caller's order
};
msc_status multi_rhs_impl(msc_op op, const double2* B, double2* X, const msc_params& prm,
                          hipStream_t s, MultiRhsOut& out);

extern "C" {

void msc_params_default(msc_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->tol = 1e-10;
  p->max_iter = 10000;
  p->prec = MSC_PREC_FP64;
  p->reliable_every = 50;
  p->freeze = 1;
  p->refine = 1;
  p->poll_every = 16;
  p->switch_tol = 3e-5;
  p->refine_max_iter = 10000;
  p->lanes = 0;
  p->verify = 1;
  p->mixed_margin = 0.7;
  p->update_steps = kMaxSteps;
}

const char* msc_version(void) { return "msc 0.1 (gfx950)"; }

const char* msc_last_error(void) { return g_last_error.c_str(); }

msc_status msc_op_create_csr(msc_op* out, int32_t kind, int64_t n, int64_t nnz,
                             const int64_t* d_rowptr, const int32_t* d_col, const double* d_vals,
                             msc_stream stream) {
  if (!out) {
    set_error("msc_op_create_csr: out is NULL");
    return MSC_EINVAL;
  }
  *out = nullptr;
  if (kind != MSC_A_MHM && kind != MSC_A_HERM && kind != MSC_A_GENERAL) {
    set_error("msc_op_create_csr: unknown kind %d", kind);
    return MSC_EINVAL;
  }
  if (n < 1 || nnz < 0 || nnz >= (int64_t(1) << 31) || n >= (int64_t(1) << 31)) {
    set_error("msc_op_create_csr: need 1 <= n < 2^31 and 0 <= nnz < 2^31 (n=%lld nnz=%lld)",
              (long long)n, (long long)nnz);
    return MSC_EINVAL;
  }
  if (!d_rowptr || (nnz > 0 && (!d_col || !d_vals))) {
    set_error("msc_op_create_csr: null array");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  msc_op op = new (std::nothrow) msc_op_s();
  if (!op) {
    set_error("msc_op_create_csr: host allocation failed");
    return MSC_ENOMEM;
  }
  auto fail = [&](msc_status st) {
    msc_op_destroy(op);
    return st;
  };
  op->kind = kind;
  op->n = n;
  op->nnz = nnz;
  op->nnz_h = kind == MSC_A_MHM ? nnz : 0;
  if (hipGetDevice(&op->device) != hipSuccess) {
    set_error("msc_op_create_csr: no HIP device");
    return fail(MSC_EHIP);
  }
  int* d_err = nullptr;
#define CREATE_TRY(expr)                                                          \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                   \
      if (d_err) (void)hipFree(d_err);                                            \
      return fail(e_ == hipErrorOutOfMemory ? MSC_ENOMEM : MSC_EHIP);             \
    }                                                                             \
  } while (0)
  CREATE_TRY(dalloc(&d_err, 1));
  CREATE_TRY(hipMemsetAsync(d_err, 0, sizeof(int), s));
  CREATE_TRY(launch_validate_csr(d_rowptr, d_col, n, nnz, d_err, s));
  int h_err = 0;
  CREATE_TRY(hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  CREATE_TRY(hipStreamSynchronize(s));
  (void)hipFree(d_err);
  d_err = nullptr;
  if (h_err) {
    set_error("msc_op_create_csr: invalid CSR (%s%s%s%s)", (h_err & 1) ? "rowptr[0]!=0 " : "",
              (h_err & 2) ? "rowptr decreasing " : "", (h_err & 4) ? "rowptr[n]!=nnz " : "",
              (h_err & 8) ? "column out of range" : "");
    return fail(MSC_EINVAL);
  }
  CREATE_TRY(dalloc(&op->rowptr, size_t(n) + 1));
  CREATE_TRY(dalloc(&op->col, size_t(nnz)));
  CREATE_TRY(dalloc(&op->val64, size_t(nnz)));
  CREATE_TRY(dalloc(&op->val32, size_t(nnz)));
  CREATE_TRY(launch_rowptr_to32(d_rowptr, op->rowptr, n, s));
  if (nnz > 0) {
    CREATE_TRY(hipMemcpyAsync(op->col, d_col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
    CREATE_TRY(hipMemcpyAsync(op->val64, d_vals, sizeof(double2) * nnz, hipMemcpyDeviceToDevice, s));
  }
  CREATE_TRY(launch_cast_vals(op->val64, op->val32, nnz, s));
  {
    unsigned long long* d_hist = nullptr;
    unsigned long long h_hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    CREATE_TRY(dalloc(&d_hist, 8));
    hipError_t e = launch_row_hist(op->rowptr, n, d_hist, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_hist, d_hist, sizeof h_hist, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_hist);
    CREATE_TRY(e);
    for (int k = 0; k < 8; ++k) op->rowhist[k] = int64_t(h_hist[k]);
  }
  if (kind == MSC_A_MHM) {
    CREATE_TRY(dalloc(&op->rowptr_h, size_t(n) + 1));
    CREATE_TRY(dalloc(&op->col_h, size_t(nnz)));
    CREATE_TRY(dalloc(&op->perm_h, size_t(nnz)));
    CREATE_TRY(dalloc(&op->val64_h, size_t(nnz)));
    CREATE_TRY(dalloc(&op->val32_h, size_t(nnz)));
    CREATE_TRY(build_adjoint(op->rowptr, op->col, n, nnz, op->rowptr_h, op->col_h, op->perm_h, s));
    CREATE_TRY(launch_adjoint_vals(op->perm_h, op->val64, op->val64_h, op->val32_h, nnz, s));
  }
  // sliced ELLPACK copies for the iteration SpMVs, when their padding is small
  bool built_m = false, built_mh = kind != MSC_A_MHM;
  CREATE_TRY(build_sell(op->rowptr, op->col, op->val64, n, nnz, op->sell_m, &built_m, s));
  if (built_m && kind == MSC_A_MHM)
    CREATE_TRY(build_sell(op->rowptr_h, op->col_h, op->val64_h, n, nnz, op->sell_mh, &built_mh, s));
  op->sell = built_m && built_mh;
  if (!op->sell) {
    free_sell(op->sell_m);
    free_sell(op->sell_mh);
  }
  CREATE_TRY(hipStreamSynchronize(s));
  if (op->sell) op->order = detect_order(d_rowptr, d_col, n, nnz, op->sell_m.nslices, s);
#undef CREATE_TRY
  *out = op;
  return MSC_OK;
}

msc_status msc_op_update_values(msc_op op, const double* d_vals, msc_stream stream) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (op->nnz > 0 && !d_vals) {
    set_error("msc_op_update_values: null values");
    return MSC_EINVAL;
  }
  if (op->stencil) {
    set_error("msc_op_update_values: a staggered operator takes new links "
              "(msc_op_update_links), not new matrix values");
    return MSC_EINVAL;
  }
  return update_values_impl(op, d_vals, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// A different right-hand side per shift (Section 5, eq. linprobgen): B and X are ns x n
// complex128 (caller's shift order).  Common-residual initial guesses, one multishift
// solve of the common residual, then every shift checked against its own b_k in FP64
// and completed by the batched CG; the guesses are dropped when the stop they need
// falls below 1e-14 or the shifts repeat.
msc_status multi_rhs_impl(msc_op op, const double2* B, double2* X, const msc_params& prm,
                          hipStream_t s, MultiRhsOut& out) {
  const int ns = int(op->sigma.size());
  const int64_t n = op->n;
  msc_status rc = ensure_scratch(op, s);
  if (rc != MSC_OK) return rc;
  rc = ensure_workspace(op, prm.prec, ns);
  if (rc != MSC_OK) return rc;
  // buffers: W (ns n), r0 (n), d (ns n), product (n); tables; norms, partials, tickets
  auto align = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t vec = sizeof(double2) * size_t(n);
  const size_t tab = align(sizeof(double) * ns * ns);
  const size_t need = align(vec * ns) + align(vec) + align(vec * ns) + align(vec) + 2 * tab +
                      align(sizeof(int) * ns) + align(sizeof(double) * (ns + 1)) +
                      align(sizeof(double) * (ns + 1) * kOsbSlices) +
                      align(sizeof(unsigned) * (ns + 1) * kTicketSite);
  if (op->osb_bytes < need) {
    if (op->osb) (void)hipFree(op->osb);
    op->osb = nullptr;
    op->osb_bytes = 0;
    HIP_TRY(hipMalloc(&op->osb, need));
    op->osb_bytes = need;
  }
  unsigned char* cur = static_cast<unsigned char*>(op->osb);
  auto carve = [&](size_t b) {
    unsigned char* p = cur;
    cur += align(b);
    return p;
  };
  double2* W = reinterpret_cast<double2*>(carve(vec * ns));
  double2* r0 = reinterpret_cast<double2*>(carve(vec));
  double2* dl = reinterpret_cast<double2*>(carve(vec * ns));
  double2* prod = reinterpret_cast<double2*>(carve(vec));
  double* d_inv = reinterpret_cast<double*>(carve(sizeof(double) * ns * ns));
  double* d_w = reinterpret_cast<double*>(carve(sizeof(double) * ns * ns));
  int* d_orig = reinterpret_cast<int*>(carve(sizeof(int) * ns));
  double* d_norm = reinterpret_cast<double*>(carve(sizeof(double) * (ns + 1)));
  double* d_part = reinterpret_cast<double*>(carve(sizeof(double) * (ns + 1) * kOsbSlices));
  unsigned* d_tick = reinterpret_cast<unsigned*>(carve(sizeof(unsigned) * (ns + 1) * kTicketSite));
  HIP_TRY(hipMemsetAsync(d_tick, 0, sizeof(unsigned) * (ns + 1) * kTicketSite, s));

  // sorted shifts, the divided-difference and Newton-weight tables
  std::vector<int> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int i, int j) { return op->sigma[i] < op->sigma[j]; });
  std::vector<double> sv(ns), inv(size_t(ns) * ns, 0.0), w(size_t(ns) * ns, 0.0);
  bool distinct = true;
  for (int j = 0; j < ns; ++j) sv[j] = op->sigma[order[j]];
  for (int j = 1; j < ns; ++j)
    if (!(sv[j] > sv[j - 1])) distinct = false;
  for (int k = 0; k < ns; ++k) {
    for (int level = 1; level <= k; ++level) inv[size_t(k) * ns + level] = 1.0 / (sv[k] - sv[k - level]);
    double wk = 1.0;
    for (int j = 0; j <= std::min(k, ns - 2); ++j) {
      w[size_t(k) * ns + j] = wk;
      wk *= sv[k] - sv[j];
    }
  }
  HIP_TRY(hipMemcpy(d_inv, inv.data(), sizeof(double) * ns * ns, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_w, w.data(), sizeof(double) * ns * ns, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_orig, order.data(), sizeof(int) * ns, hipMemcpyHostToDevice));

  const int lanes = choose_lanes(op, prm);
  auto apply = [&](const double2* in, double2* out, double shift) {
    return launch_apply(op->kind, MSC_PREC_FP64, lanes, n,
                        Csr<double2>{op->rowptr, op->col, op->val64},
                        Csr<double2>{op->rowptr_h, op->col_h, op->val64_h},
                        Csr<float2>{op->rowptr, op->col, op->val32},
                        Csr<float2>{op->rowptr_h, op->col_h, op->val32_h}, in, out, shift,
                        op->ws.t64, op->ws.u64, s);
  };
  // |b_k|^2 in the caller's order
  std::vector<double> bn2(ns + 1, 0.0);
  HIP_TRY(launch_osb_norms(B, ns, n, d_part, d_tick, d_norm, s));
  HIP_TRY(hipMemcpyAsync(bn2.data(), d_norm, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // the smallest nonzero |b_k| sets the stop (a zero b_k gets x_k = 0 below)
  double bmin = HUGE_VAL;
  for (int k = 0; k < ns; ++k)
    if (bn2[k] > 0.0) bmin = std::min(bmin, std::sqrt(bn2[k]));
  if (!(bmin < HUGE_VAL)) bmin = 0.0;

  int& iters = out.iters;
  iters = 0;
  bool used = false;
  if (distinct) {
    // guesses x0 into x, common residual into r0
    HIP_TRY(launch_osb_divdiff(B, d_orig, d_inv, W, ns, n, s));
    for (int m = ns - 2; m >= 1; --m) {
      HIP_TRY(apply(W + int64_t(m + 1) * n, prod, sv[m]));  // (A + s_m) Y_m
      HIP_TRY(launch_osb_sub(W + int64_t(m) * n, prod, n, s));  // W[m] <- Y_{m-1}
    }
    if (ns >= 2) {
      HIP_TRY(apply(W + n, prod, sv[0]));
      HIP_TRY(launch_osb_sub(W, prod, n, s));
    }
    HIP_TRY(hipMemcpyAsync(r0, W, vec, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_osb_combine(W, d_w, d_orig, X, ns, n, s));
    double rr = 0.0;
    HIP_TRY(launch_osb_norms(r0, 1, n, d_part, d_tick + size_t(ns) * kTicketSite, d_norm + ns, s));
    HIP_TRY(hipMemcpyAsync(&rr, d_norm + ns, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double rn = std::sqrt(rr);
    // the multishift stop that gives every shift tol |b_k|; beyond FP64's reach the
    // guesses are dropped and each shift is solved from zero by the batched CG
    const double tol_inner = rn > 0.0 ? prm.tol * bmin / rn : 0.0;
    if (rn == 0.0) {
      used = true;
    } else if (std::isfinite(rn) && tol_inner >= 1e-14) {
      used = true;
      msc_params p2 = prm;
      p2.verify = 0;
      std::vector<double> rel;
      int st = 0;
      double bytes = 0.0, bnorm = 0.0;
      const double tol_stop = tol_inner * (prm.prec == MSC_PREC_MIXED ? prm.mixed_margin : 1.0);
      rc = run_multishift(op, reinterpret_cast<const double*>(r0), reinterpret_cast<double*>(dl),
                          p2, nullptr, s, tol_stop, prm.prec, &rel, &iters, &st, &bytes, &bnorm);
      if (rc != MSC_OK) return rc;
      if (st != 0) {
        set_error("breakdown in the multishift solve of the common residual");
        out.breakdown = true;
        return MSC_EBREAKDOWN;
      }
      HIP_TRY(launch_osb_add(X, dl, int64_t(ns) * n, s));
    }
  }
  if (!used) HIP_TRY(hipMemsetAsync(X, 0, vec * ns, s));
  for (int k = 0; k < ns; ++k)
    if (!(bn2[k] > 0.0)) HIP_TRY(hipMemsetAsync(X + int64_t(k) * n, 0, vec, s));

  // every shift against its own b_k in FP64; those above tol continue with the batched CG
  std::vector<double>& rel = out.rel;
  rel.assign(ns, 0.0);
  int& refine_iters = out.refine_iters;
  int& n_refined = out.n_refined;
  bool& breakdown = out.breakdown;
  refine_iters = n_refined = 0;
  breakdown = false;
  for (int g0 = 0; g0 < ns; g0 += kBssMax) {
    const int m = std::min(kBssMax, ns - g0);
    std::vector<double> sig(m), tol_abs(m), res;
    std::vector<const double2*> f(m);
    std::vector<double2*> x(m);
    for (int j = 0; j < m; ++j) {
      const int k = g0 + j;
      sig[j] = op->sigma[k];
      tol_abs[j] = prm.tol * std::sqrt(bn2[k]);
      f[j] = B + int64_t(k) * n;
      x[j] = X + int64_t(k) * n;
    }
    int inner = 0;
    bool bd = false;
    double bytes = 0.0;
    rc = run_batched_cg(op, MSC_PREC_FP64, m, sig.data(), f.data(), x.data(), tol_abs.data(), 0.0,
                        prm, s, res, &inner, &bytes, &bd);
    if (rc != MSC_OK) return rc;
    refine_iters = std::max(refine_iters, inner);
    for (int j = 0; j < m; ++j) {
      const double bk = std::sqrt(bn2[g0 + j]);
      rel[g0 + j] = bk > 0.0 ? res[j] / bk : 0.0;
    }
    if (inner > 0) n_refined += m;  // the group needed CG iterations
    if (bd) breakdown = true;
  }
  return MSC_OK;
}

msc_status update_values_impl(msc_op op, const double* d_vals, hipStream_t s) {
  if (op->nnz > 0) {
    HIP_TRY(hipMemcpyAsync(op->val64, d_vals, sizeof(double2) * op->nnz, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_cast_vals(op->val64, op->val32, op->nnz, s));
    if (op->kind == MSC_A_MHM)
      HIP_TRY(launch_adjoint_vals(op->perm_h, op->val64, op->val64_h, op->val32_h, op->nnz, s));
    op->real_state = 0;  // the real copies are rebuilt by the next real solve
    dfree(op->rval64);
    dfree(op->rval32);
    dfree(op->rdiag64);
    dfree(op->rdiag32);
    if (op->sell) {
      HIP_TRY(refill_sell(op->rowptr, op->col, op->val64, op->n, op->sell_m, s));
      if (op->kind == MSC_A_MHM)
        HIP_TRY(refill_sell(op->rowptr_h, op->col_h, op->val64_h, op->n, op->sell_mh, s));
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return MSC_OK;
}

namespace {

// Geometry of a staggered operator (links pointer left null), or false with the error set.
bool staggered_geometry(const char* who, const int32_t* dims, double mass, Stencil<double2>& g) {
  if (!dims) {
    set_error("%s: null dims", who);
    return false;
  }
  int64_t vol = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (dims[mu] < 3) {
      set_error("%s: every extent must be >= 3 (dims[%d] = %d)", who, mu, dims[mu]);
      return false;
    }
    g.L[mu] = dims[mu];
    g.stride[mu] = vol;
    vol *= dims[mu];
    if (vol > (int64_t(1) << 31)) break;
  }
  if (vol * 3 * 25 >= (int64_t(1) << 31)) {
    set_error("%s: 25 * 3 * volume must stay below 2^31", who);
    return false;
  }
  if (!std::isfinite(mass)) {
    set_error("%s: mass is not finite", who);
    return false;
  }
  g.vol = vol;
  g.mass = mass;
  return true;
}

// The op's links from the caller's U (w64, w32) and the CSR of M built from them
// (device temporaries owned by the caller of this function).
msc_status staggered_csr(const Stencil<double2>& w, int64_t** rowptr, int32_t** col,
                         double2** vals, hipStream_t s) {
  const int64_t n = 3 * w.vol;
  HIP_TRY(dalloc(rowptr, size_t(n) + 1));
  HIP_TRY(dalloc(col, size_t(25 * n)));
  HIP_TRY(dalloc(vals, size_t(25 * n)));
  HIP_TRY(launch_stencil_csr(w, *rowptr, *col, *vals, s));
  return MSC_OK;
}

}  // namespace

extern "C" {

msc_status msc_op_create_staggered(msc_op* out, const int32_t* dims, double mass,
                                   const double* d_links, msc_stream stream) {
  if (!out) {
    set_error("msc_op_create_staggered: out is NULL");
    return MSC_EINVAL;
  }
  *out = nullptr;
  Stencil<double2> geo;
  if (!staggered_geometry("msc_op_create_staggered", dims, mass, geo)) return MSC_EINVAL;
  if (!d_links) {
    set_error("msc_op_create_staggered: null links");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nw = size_t(4 * 9) * size_t(geo.vol);
  double2* w64 = nullptr;
  float2* w32 = nullptr;
  int64_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double2* vals = nullptr;
  auto cleanup = [&](bool keep_links) {
    if (rowptr) (void)hipFree(rowptr);
    if (col) (void)hipFree(col);
    if (vals) (void)hipFree(vals);
    if (!keep_links) {
      dfree(w64);
      dfree(w32);
    }
  };
  hipError_t e = dalloc(&w64, nw);
  if (e == hipSuccess) e = dalloc(&w32, nw);
  if (e == hipSuccess) e = launch_stencil_links(reinterpret_cast<const double2*>(d_links), geo, w64, w32, s);
  if (e != hipSuccess) {
    set_error("msc_op_create_staggered: %s", hipGetErrorString(e));
    cleanup(false);
    return e == hipErrorOutOfMemory ? MSC_ENOMEM : MSC_EHIP;
  }
  Stencil<double2> w = geo;
  w.w = w64;
  msc_status rc = staggered_csr(w, &rowptr, &col, &vals, s);
  const int64_t n = 3 * geo.vol;
  msc_op op = nullptr;
  if (rc == MSC_OK)
    rc = msc_op_create_csr(&op, MSC_A_MHM, n, 25 * n, rowptr, col,
                           reinterpret_cast<const double*>(vals), stream);
  if (rc != MSC_OK) {
    cleanup(false);
    return rc;
  }
  cleanup(true);
  op->stencil = true;
  op->w64 = w;
  op->w32 = Stencil<float2>{};
  op->w32.w = w32;
  for (int mu = 0; mu < 4; ++mu) {
    op->w32.L[mu] = geo.L[mu];
    op->w32.stride[mu] = geo.stride[mu];
  }
  op->w32.vol = geo.vol;
  op->w32.mass = geo.mass;
  // the lattice's planes (fixed x2, x3) and slabs (fixed x3), when they are whole slices
  const int64_t plane = 3 * int64_t(geo.L[0]) * geo.L[1], slab = plane * geo.L[2];
  op->order = (op->sell && plane % kSlice == 0)
                  ? lattice_order(op->sell_m.nslices, plane / kSlice, slab / kSlice)
                  : SweepOrder{0, 0, 0, 0};
  // the same structure in blocks of 64 sites, for the kernels that read the links
  const int64_t splane = int64_t(geo.L[0]) * geo.L[1], sslab = splane * geo.L[2];
  op->order_sites = splane % 64 == 0
                        ? lattice_order((geo.vol + 63) / 64, splane / 64, sslab / 64, kTileSpanSites)
                        : SweepOrder{0, 0, 0, 0};
  op->order_sites64 = splane % 64 == 0
                          ? lattice_order((geo.vol + 63) / 64, splane / 64, sslab / 64,
                                          kTileSpanSites64)
                          : SweepOrder{0, 0, 0, 0};
  rc = refresh_two_rows(op, reinterpret_cast<const double2*>(d_links), s);
  if (rc != MSC_OK) {
    msc_op_destroy(op);
    return rc;
  }
  *out = op;
  return MSC_OK;
}

msc_status msc_op_update_links(msc_op op, const double* d_links, msc_stream stream) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!op->stencil) {
    set_error("msc_op_update_links: the operator was not made by msc_op_create_staggered");
    return MSC_EINVAL;
  }
  if (!d_links) {
    set_error("msc_op_update_links: null links");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_stencil_links(reinterpret_cast<const double2*>(d_links), op->w64,
                               const_cast<double2*>(op->w64.w), const_cast<float2*>(op->w32.w), s));
  int64_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double2* vals = nullptr;
  msc_status rc = staggered_csr(op->w64, &rowptr, &col, &vals, s);
  if (rc == MSC_OK) rc = update_values_impl(op, reinterpret_cast<const double*>(vals), s);
  if (rowptr) (void)hipFree(rowptr);
  if (col) (void)hipFree(col);
  if (vals) (void)hipFree(vals);
  if (rc == MSC_OK) rc = refresh_two_rows(op, reinterpret_cast<const double2*>(d_links), s);
  return rc;
}

msc_status msc_op_set_shifts(msc_op op, const double* h_sigma, int32_t ns) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!h_sigma || ns < 1 || ns > kMaxShifts) {
    set_error("msc_op_set_shifts: need 1 <= ns <= %d and a host array", kMaxShifts);
    return MSC_EINVAL;
  }
  for (int k = 0; k < ns; ++k)
    if (!std::isfinite(h_sigma[k])) {
      set_error("msc_op_set_shifts: sigma[%d] is not finite", k);
      return MSC_EINVAL;
    }
  op->sigma.assign(h_sigma, h_sigma + ns);
  return MSC_OK;
}

msc_status msc_op_query(msc_op op, int64_t* n, int64_t* nnz, int32_t* ns, int32_t* kind) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (n) *n = op->n;
  if (nnz) *nnz = op->nnz;
  if (ns) *ns = int32_t(op->sigma.size());
  if (kind) *kind = op->kind;
  return MSC_OK;
}

msc_status msc_op_storage(msc_op op, int32_t* sell, int32_t* narrow) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (sell) *sell = op->sell ? 1 : 0;
  if (narrow)
    *narrow = (op->sell && op->sell_m.col16 ? 1 : 0) |
              (op->sell && op->kind == MSC_A_MHM && op->sell_mh.col16 ? 2 : 0) |
              (op->stencil && op->two_rows ? 4 : 0);
  return MSC_OK;
}

msc_status msc_op_apply(msc_op op, int32_t prec, const double* d_in, double* d_out, double shift,
                        msc_stream stream) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_in || !d_out || (prec != MSC_PREC_FP64 && prec != MSC_PREC_MIXED)) {
    set_error("msc_op_apply: null vector or unknown precision");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  msc_params prm;
  msc_params_default(&prm);
  const int ns = std::max<int>(1, int(op->sigma.size()));
  msc_status rc = ensure_workspace(op, prec, ns);
  if (rc != MSC_OK) return rc;
  // the FP64 path needs two complex128 temporaries: t64 and the first slice of u64
  void* ta = prec == MSC_PREC_MIXED ? op->ws.r : static_cast<void*>(op->ws.t64);
  void* tb = prec == MSC_PREC_MIXED ? op->ws.t : static_cast<void*>(op->ws.u64);
  HIP_TRY(launch_apply(op->kind, prec, choose_lanes(op, prm), op->n,
                       Csr<double2>{op->rowptr, op->col, op->val64},
                       Csr<double2>{op->rowptr_h, op->col_h, op->val64_h},
                       Csr<float2>{op->rowptr, op->col, op->val32},
                       Csr<float2>{op->rowptr_h, op->col_h, op->val32_h},
                       reinterpret_cast<const double2*>(d_in), reinterpret_cast<double2*>(d_out),
                       shift, ta, tb, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MSC_OK;
}

msc_status msc_op_apply_noalloc(msc_op op, int32_t prec, const double* d_in, double* d_out,
                                double shift, msc_stream stream) {
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_in || !d_out || (prec != MSC_PREC_FP64 && prec != MSC_PREC_MIXED)) {
    set_error("msc_op_apply_noalloc: null vector or unknown precision");
    return MSC_EINVAL;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != op->device) {
    set_error("msc_op_apply_noalloc: device %d is current, the operator lives on device %d",
              dev, op->device);
    return MSC_EINVAL;
  }
  const size_t need = apply_scratch_bytes(op->kind, prec, op->n);
  if (need > kNoAllocScratchBytes) {
    set_error("msc_op_apply_noalloc: n = %lld needs %zu bytes of scratch, above the "
              "%zu-byte limit (use msc_op_apply)",
              (long long)op->n, need, kNoAllocScratchBytes);
    return MSC_EINVAL;
  }
  void* base = nullptr;
  HIP_TRY(noalloc_scratch(dev, &base));
  msc_params prm;
  msc_params_default(&prm);
  HIP_TRY(launch_apply_noalloc(op->kind, prec, choose_lanes(op, prm), op->n,
                               Csr<double2>{op->rowptr, op->col, op->val64},
                               Csr<double2>{op->rowptr_h, op->col_h, op->val64_h},
                               Csr<float2>{op->rowptr, op->col, op->val32},
                               Csr<float2>{op->rowptr_h, op->col_h, op->val32_h},
                               reinterpret_cast<const double2*>(d_in),
                               reinterpret_cast<double2*>(d_out), shift, base,
                               static_cast<hipStream_t>(stream)));
  return MSC_OK;
}

msc_status msc_solve(msc_op op, const double* d_b, double* d_x, const msc_params* params,
                     msc_info* info, msc_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_b || !d_x) {
    set_error("msc_solve: null b or x");
    return MSC_EINVAL;
  }
  if (op->sigma.empty()) {
    set_error("msc_solve: no shifts set");
    return MSC_EINVAL;
  }
  if (op->kind == MSC_A_GENERAL) {
    set_error("msc_solve: CG-M needs a Hermitian positive-definite A; a general operator "
              "takes msc_solve_bicgstab");
    return MSC_EINVAL;
  }
  msc_params prm;
  if (params)
    prm = *params;
  else
    msc_params_default(&prm);
  if (!(prm.tol >= 0.0) || (prm.prec != MSC_PREC_FP64 && prm.prec != MSC_PREC_MIXED) ||
      !(prm.mixed_margin > 0.0 && prm.mixed_margin <= 1.0) ||
      prm.update_steps < 1 || prm.update_steps > kMaxSteps || (prm.sweep != 0 && prm.sweep != 1)) {
    set_error("msc_solve: invalid tol, precision, mixed_margin, update_steps or sweep");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  msc_status result = solve_impl(op, d_b, d_x, prm, info, s);
  if (info)
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return result;
}

msc_status msc_solve_adjoint(msc_op op, const double* d_g, const double* d_x, double* d_grad_b,
                             double* d_grad_vals, const msc_params* params, msc_info* info,
                             msc_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_g || !d_x) {
    set_error("msc_solve_adjoint: null g or x");
    return MSC_EINVAL;
  }
  if (op->sigma.empty()) {
    set_error("msc_solve_adjoint: no shifts set");
    return MSC_EINVAL;
  }
  if (op->kind == MSC_A_GENERAL) {
    set_error("msc_solve_adjoint: not available for a general operator");
    return MSC_EINVAL;
  }
  msc_params prm;
  if (params)
    prm = *params;
  else
    msc_params_default(&prm);
  if (!(prm.tol >= 0.0) || (prm.prec != MSC_PREC_FP64 && prm.prec != MSC_PREC_MIXED) ||
      !(prm.mixed_margin > 0.0 && prm.mixed_margin <= 1.0) ||
      prm.update_steps < 1 || prm.update_steps > kMaxSteps || (prm.sweep != 0 && prm.sweep != 1)) {
    set_error("msc_solve_adjoint: invalid tol, precision, mixed_margin, update_steps or sweep");
    return MSC_EINVAL;
  }
  prm.verify = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = int(op->sigma.size());
  const int64_t n = op->n;
  msc_status rc = ensure_scratch(op, s);
  if (rc != MSC_OK) return rc;
  rc = ensure_workspace(op, prm.prec, ns);
  if (rc != MSC_OK) return rc;
  if (op->yadj_count < size_t(ns) * size_t(n)) {
    dfree(op->yadj);
    HIP_TRY(dalloc(&op->yadj, size_t(ns) * size_t(n)));
    op->yadj_count = size_t(ns) * size_t(n);
  }
  if (!op->adj_small) HIP_TRY(dalloc(&op->adj_small, 256));
  const double2* g = reinterpret_cast<const double2*>(d_g);
  const double2* x = reinterpret_cast<const double2*>(d_x);
  double2* y = op->yadj;

  // 1. norms |g_k|^2, then the largest as reference and the real factors c_k
  std::vector<double> gram(3 * ns), gn2(ns);
  for (int q0 = 0; q0 < ns; q0 += 16) {
    const int kc = std::min(16, ns - q0);
    HIP_TRY(launch_gram(g, g + int64_t(q0) * n, n, kc, op->scratch.partial, op->scratch.tickets + 11 * kTicketSite,
                        op->adj_small + 3 * q0, s));
  }
  HIP_TRY(hipMemcpyAsync(gram.data(), op->adj_small, sizeof(double) * 3 * ns, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < ns; ++k) gn2[k] = gram[3 * k + 2];
  const int ref = int(std::max_element(gn2.begin(), gn2.end()) - gn2.begin());
  bool collinear = gn2[ref] > 0.0 && std::isfinite(gn2[ref]);
  std::vector<double> c(ns, 0.0);
  if (collinear) {
    const double2* gref = g + int64_t(ref) * n;
    for (int q0 = 0; q0 < ns; q0 += 16) {
      const int kc = std::min(16, ns - q0);
      HIP_TRY(launch_gram(gref, g + int64_t(q0) * n, n, kc, op->scratch.partial,
                          op->scratch.tickets + 11 * kTicketSite, op->adj_small + 3 * q0, s));
    }
    HIP_TRY(hipMemcpyAsync(gram.data(), op->adj_small, sizeof(double) * 3 * ns, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < ns; ++k) c[k] = gram[3 * k] / gn2[ref];
    HIP_TRY(hipMemcpyAsync(op->adj_small + 192, c.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
    std::vector<double> dn(ns);
    for (int q0 = 0; q0 < ns; q0 += 16) {
      const int kc = std::min(16, ns - q0);
      HIP_TRY(launch_diffnorm(gref, g + int64_t(q0) * n, op->adj_small + 192 + q0, n, kc,
                              op->scratch.partial, op->scratch.tickets + 11 * kTicketSite, op->adj_small + q0, s));
    }
    HIP_TRY(hipMemcpyAsync(dn.data(), op->adj_small, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < ns; ++k)
      if (!(dn[k] <= 1e-26 * gn2[k])) collinear = false;
    if (collinear) HIP_TRY(hipMemcpyAsync(op->adj_small + 192, c.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
  }

  // 2. y_k = (A + sigma_k)^{-1} g_k
  msc_status result = MSC_OK;
  int iters = 0, refine_iters = 0, n_refined = 0;
  std::vector<double> rel(ns, 0.0);
  double bytes = 0.0;
  if (collinear) {
    msc_info sub{};
    std::vector<double> sub_rel(ns);
    sub.true_rel_res = sub_rel.data();
    const double2* gref = g + int64_t(ref) * n;
    result = solve_impl(op, reinterpret_cast<const double*>(gref), reinterpret_cast<double*>(y), prm,
                        &sub, s);
    if (result < 0) return result;
    HIP_TRY(launch_scale_shifts(y, op->adj_small + 192, ns, n, s));
    iters = sub.iters;
    refine_iters = sub.refine_iters;
    n_refined = sub.n_refined;
    bytes = sub.alg_bytes;
    rel = sub_rel;
  } else {
    // a different g_k per shift: the common-residual guesses and one multishift solve
    // where the shifts allow it, every shift completed by the batched CG (Section 5)
    MultiRhsOut out;
    rc = multi_rhs_impl(op, g, y, prm, s, out);
    if (rc != MSC_OK && rc != MSC_EBREAKDOWN) return rc;
    iters = out.iters;
    refine_iters = out.refine_iters;
    n_refined = out.n_refined;
    rel = out.rel;
    if (rc == MSC_EBREAKDOWN || out.breakdown) {
      set_error("msc_solve_adjoint: breakdown in an adjoint solve");
      result = MSC_EBREAKDOWN;
    } else {
      for (int k = 0; k < ns; ++k)
        if (!(rel[k] <= prm.tol)) result = MSC_ENOTCONV;
    }
  }

  // 3. gradients
  if (d_grad_b) HIP_TRY(launch_sum_shifts(y, ns, n, reinterpret_cast<double2*>(d_grad_b), s));
  if (d_grad_vals && op->nnz > 0) {
    HIP_TRY(launch_grad_vals(op->kind, choose_lanes(op, prm), Csr<double2>{op->rowptr, op->col, op->val64},
                             x, y, n, ns, op->ws.u64, op->ws.u64 + 4 * n,
                             reinterpret_cast<double2*>(d_grad_vals), s));
    bytes += double(ns) / 4.0 * (double(op->nnz) * 20.0) + double(op->nnz) * 32.0;
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (info) {
    info->iters = iters;
    info->refine_iters = refine_iters;
    info->n_refined = n_refined;
    info->n_reliable = 0;
    if (info->true_rel_res)
      for (int k = 0; k < ns; ++k) info->true_rel_res[k] = rel[k];
    if (info->freeze_iter)
      for (int k = 0; k < ns; ++k) info->freeze_iter[k] = -1;
    clear_timing(*info);
    info->alg_bytes = bytes;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return result;
}

msc_status msc_solve_bicgstab(msc_op op, const double* d_b, double* d_x,
                              const msc_params* params, msc_info* info, msc_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_b || !d_x) {
    set_error("msc_solve_bicgstab: null b or x");
    return MSC_EINVAL;
  }
  if (op->sigma.empty()) {
    set_error("msc_solve_bicgstab: no shifts set");
    return MSC_EINVAL;
  }
  if (op->kind == MSC_A_MHM) {
    set_error("msc_solve_bicgstab: A = M^H M is Hermitian positive definite: use msc_solve "
              "(or create the operator of M itself with kind MSC_A_GENERAL)");
    return MSC_EINVAL;
  }
  msc_params prm;
  if (params)
    prm = *params;
  else
    msc_params_default(&prm);
  if (!(prm.tol >= 0.0) || prm.prec != MSC_PREC_FP64 || (prm.sweep != 0 && prm.sweep != 1)) {
    set_error("msc_solve_bicgstab: invalid tol, precision (FP64 only) or sweep");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = int(op->sigma.size());
  const int64_t n = op->n;
  msc_status rc = ensure_scratch(op, s);
  if (rc != MSC_OK) return rc;
  // buffers: r[2], p, v, s, t (n each), ns directions, the state
  const size_t vec = sizeof(double2) * size_t(n);
  const size_t need = vec * (6 + size_t(ns)) + sizeof(BcgState) + 256;
  if (op->bcg_bytes < need) {
    if (op->bcg) (void)hipFree(op->bcg);
    op->bcg = nullptr;
    op->bcg_bytes = 0;
    HIP_TRY(hipMalloc(&op->bcg, need));
    op->bcg_bytes = need;
  }
  unsigned char* base = static_cast<unsigned char*>(op->bcg);
  BcgArgs a{};
  a.n = n;
  a.ns = ns;
  a.lanes = choose_lanes(op, prm);
  a.m = Csr<double2>{op->rowptr, op->col, op->val64};
  a.b = reinterpret_cast<const double2*>(d_b);
  a.x = reinterpret_cast<double2*>(d_x);
  double2* vbase = reinterpret_cast<double2*>(base);
  a.r[0] = vbase;
  a.r[1] = vbase + n;
  a.p = vbase + 2 * n;
  a.v = vbase + 3 * n;
  a.s = vbase + 4 * n;
  a.t = vbase + 5 * n;
  a.pk = vbase + 6 * n;
  a.st = reinterpret_cast<BcgState*>(base + vec * (6 + size_t(ns)));
  a.partial = op->scratch.partial;
  a.tickets = op->scratch.tickets + 12 * kTicketSite;

  std::vector<int> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int i, int j) { return op->sigma[i] < op->sigma[j]; });
  BcgState h{};
  h.sigma0 = op->sigma[order[0]];
  h.eps2 = prm.tol * prm.tol;  // scaled by |b|^2 in the init kernel
  h.al_prev = double2{1.0, 0.0};
  h.be_prev = double2{0.0, 0.0};
  h.max_iter = prm.max_iter;
  h.ns = ns;
  h.upd_launch = -1;
  for (int j = 0; j < ns; ++j) {
    h.s[j] = op->sigma[order[j]] - h.sigma0;
    h.z[j] = h.z_old[j] = h.tau[j] = double2{1.0, 0.0};
    h.active[j] = 1;
    h.freeze_iter[j] = -1;
    h.orig[j] = order[j];
  }
  HIP_TRY(hipMemcpyAsync(a.st, &h, sizeof h, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_bcg_init(a, s));
  const int G = std::max(1, prm.poll_every);
  int launched = 0;
  bool done = prm.max_iter <= 0;
  while (!done) {
    for (int g = 0; g < G; ++g) {
      HIP_TRY(launch_bcg_iteration(a, launched, s));
      ++launched;
    }
    int halt = 0;
    HIP_TRY(hipMemcpyAsync(&halt, &a.st->halt, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (halt || launched >= prm.max_iter + G) done = true;
  }
  HIP_TRY(hipMemcpyAsync(&h, a.st, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<double> rel(ns, 0.0);
  const double bn = std::sqrt(h.bnorm2);
  if (prm.verify && h.status == 0 && bn > 0.0) {
    MsArgs va = make_args(op, a.lanes, d_b, d_x);
    for (int k0 = 0; k0 < ns; k0 += 8) {
      const int kc = std::min(8, ns - k0);
      HIP_TRY(launch_verify(va, op->sigma.data(), k0, kc, nullptr, s));
    }
    std::vector<double> r2(ns);
    HIP_TRY(hipMemcpyAsync(r2.data(), op->scratch.res2, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < ns; ++k) rel[k] = std::sqrt(r2[k]) / bn;
  }
  bool all_ok = true;
  for (int j = 0; j < ns; ++j)
    if (h.iter > 0 && h.active_next[j]) all_ok = false;  // still advanced at the end
  if (prm.verify)
    for (int k = 0; k < ns; ++k)
      if (!(rel[k] <= prm.tol)) all_ok = false;
  if (info) {
    clear_timing(*info);
    info->iters = h.iter;
    info->refine_iters = 0;
    info->n_reliable = 0;
    info->n_refined = 0;
    info->iters_fp64 = h.iter;
    info->alg_bytes = 0.0;
    if (info->true_rel_res)
      for (int k = 0; k < ns; ++k) info->true_rel_res[k] = rel[k];
    if (info->freeze_iter)
      for (int j = 0; j < ns; ++j) info->freeze_iter[order[j]] = h.freeze_iter[j];
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (h.status != 0) {
    set_error("msc_solve_bicgstab: breakdown (w^H v, t^H t or rho vanished, 1 + s om = 0, "
              "or a non-finite value) at iteration %d", h.iter);
    return MSC_EBREAKDOWN;
  }
  return all_ok ? MSC_OK : MSC_ENOTCONV;
}

msc_status msc_solve_multi_rhs(msc_op op, const double* d_B, double* d_x,
                               const msc_params* params, msc_info* info, msc_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_B || !d_x) {
    set_error("msc_solve_multi_rhs: null B or x");
    return MSC_EINVAL;
  }
  if (op->sigma.empty()) {
    set_error("msc_solve_multi_rhs: no shifts set");
    return MSC_EINVAL;
  }
  if (op->kind == MSC_A_GENERAL) {
    set_error("msc_solve_multi_rhs: needs a Hermitian positive-definite A");
    return MSC_EINVAL;
  }
  msc_params prm;
  if (params)
    prm = *params;
  else
    msc_params_default(&prm);
  if (!(prm.tol >= 0.0) || (prm.prec != MSC_PREC_FP64 && prm.prec != MSC_PREC_MIXED) ||
      !(prm.mixed_margin > 0.0 && prm.mixed_margin <= 1.0) ||
      prm.update_steps < 1 || prm.update_steps > kMaxSteps || (prm.sweep != 0 && prm.sweep != 1)) {
    set_error("msc_solve_multi_rhs: invalid tol, precision, mixed_margin, update_steps or sweep");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = int(op->sigma.size());
  MultiRhsOut out;
  msc_status rc = multi_rhs_impl(op, reinterpret_cast<const double2*>(d_B),
                                 reinterpret_cast<double2*>(d_x), prm, s, out);
  if (rc == MSC_EBREAKDOWN) {
    const std::string why = msc_last_error();
    set_error("msc_solve_multi_rhs: %s", why.c_str());
    return rc;
  }
  if (rc != MSC_OK) return rc;
  const int iters = out.iters, refine_iters = out.refine_iters, n_refined = out.n_refined;
  const bool breakdown = out.breakdown;
  const std::vector<double>& rel = out.rel;
  if (info) {
    clear_timing(*info);
    info->iters = iters;
    info->refine_iters = refine_iters;
    info->n_reliable = 0;
    info->n_refined = n_refined;
    info->iters_fp64 = iters;
    info->alg_bytes = 0.0;
    if (info->true_rel_res)
      for (int k = 0; k < ns; ++k) info->true_rel_res[k] = rel[k];
    if (info->freeze_iter)
      for (int k = 0; k < ns; ++k) info->freeze_iter[k] = -1;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (breakdown) {
    set_error("msc_solve_multi_rhs: breakdown in the per-shift CG");
    return MSC_EBREAKDOWN;
  }
  for (int k = 0; k < ns; ++k)
    if (!(rel[k] <= prm.tol)) {
      set_error("msc_solve_multi_rhs: some shift did not reach tol");
      return MSC_ENOTCONV;
    }
  return MSC_OK;
}

msc_status msc_solve_real(msc_op op, const double* d_b, double* d_x, const msc_params* params,
                          msc_info* info, msc_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (check_op(op) != MSC_OK) return MSC_EINVAL;
  if (!d_b || !d_x) {
    set_error("msc_solve_real: null b or x");
    return MSC_EINVAL;
  }
  if (op->sigma.empty()) {
    set_error("msc_solve_real: no shifts set");
    return MSC_EINVAL;
  }
  if (op->kind != MSC_A_HERM || !op->sell) {
    set_error("msc_solve_real: needs an operator of kind MSC_A_HERM with its sliced ELLPACK "
              "copy built");
    return MSC_EINVAL;
  }
  msc_params prm;
  if (params)
    prm = *params;
  else
    msc_params_default(&prm);
  if (!(prm.tol >= 0.0) || (prm.prec != MSC_PREC_FP64 && prm.prec != MSC_PREC_MIXED) ||
      (prm.sweep != 0 && prm.sweep != 1)) {
    set_error("msc_solve_real: invalid tol, precision or sweep");
    return MSC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = int(op->sigma.size());
  const int64_t n = op->n;
  msc_status rc = ensure_scratch(op, s);
  if (rc != MSC_OK) return rc;
  const SellStore& sm = op->sell_m;
  const int64_t cells = sm.pairs * 2 * kSlice;
  // real copies of the sliced values and diagonal, after checking every imaginary part is 0
  if (op->real_state == 0) {
    unsigned long long* d_imax = nullptr;
    HIP_TRY(dalloc(&op->rval64, size_t(cells)));
    HIP_TRY(dalloc(&op->rval32, size_t(cells)));
    HIP_TRY(dalloc(&op->rdiag64, size_t(n)));
    HIP_TRY(dalloc(&op->rdiag32, size_t(n)));
    HIP_TRY(dalloc(&d_imax, 1));
    HIP_TRY(hipMemsetAsync(d_imax, 0, sizeof(unsigned long long), s));
    HIP_TRY(launch_real_extract(sm.val64, op->rval64, op->rval32, cells, d_imax, s));
    HIP_TRY(launch_real_extract(sm.diag64, op->rdiag64, op->rdiag32, n, d_imax, s));
    unsigned long long h_imax = 0;
    HIP_TRY(hipMemcpyAsync(&h_imax, d_imax, sizeof(h_imax), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(d_imax);
    op->real_state = h_imax == 0 ? 1 : -1;
  }
  if (op->real_state != 1) {
    set_error("msc_solve_real: the operator has non-zero imaginary parts");
    return MSC_EINVAL;
  }
  const int prec = prm.prec;
  const size_t el = prec == MSC_PREC_MIXED ? sizeof(float) : sizeof(double);
  auto align = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t vec = align(el * size_t(n));
  const size_t need = 3 * vec + align(el * size_t(n) * size_t(std::max(ns - 1, 1))) +
                      align(sizeof(RealState)) + align(sizeof(double) * ns);
  if (op->rws_bytes < need) {
    if (op->rws) (void)hipFree(op->rws);
    op->rws = nullptr;
    op->rws_bytes = 0;
    HIP_TRY(hipMalloc(&op->rws, need));
    op->rws_bytes = need;
  }
  unsigned char* cur = static_cast<unsigned char*>(op->rws);
  RealArgs a{};
  a.n = n;
  a.nslices = sm.nslices;
  a.ns = ns;
  a.m64 = SellReal<double>{sm.cptr, sm.col, sm.col16, sm.cbase, sm.wp, op->rval64, op->rdiag64};
  a.m32 = SellReal<float>{sm.cptr, sm.col, sm.col16, sm.cbase, sm.wp, op->rval32, op->rdiag32};
  a.b = d_b;
  a.x = d_x;
  a.r = cur;
  cur += vec;
  a.p = cur;
  cur += vec;
  a.t = cur;
  cur += vec;
  a.pk = cur;
  cur += align(el * size_t(n) * size_t(std::max(ns - 1, 1)));
  a.st = reinterpret_cast<RealState*>(cur);
  cur += align(sizeof(RealState));
  double* d_res2 = reinterpret_cast<double*>(cur);
  a.partial = op->scratch.partial;
  a.tickets = op->scratch.tickets + 13 * kTicketSite;

  std::vector<int> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int i, int j) { return op->sigma[i] < op->sigma[j]; });
  RealState h{};
  h.sigma0 = op->sigma[order[0]];
  h.eps2 = prm.tol * prm.tol;
  h.a_prev = 1.0;
  h.b = 0.0;
  h.max_iter = prm.max_iter;
  h.ns = ns;
  h.freeze = prm.freeze ? 1 : 0;
  h.upd_launch = -1;
  for (int j = 0; j < ns; ++j) {
    h.s[j] = op->sigma[order[j]] - h.sigma0;
    h.zeta[j] = h.zeta_prev[j] = 1.0;
    h.active[j] = 1;
    h.freeze_iter[j] = -1;
    h.orig[j] = order[j];
  }
  HIP_TRY(hipMemcpyAsync(a.st, &h, sizeof h, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_real_init(prec, a, s));
  const int G = std::max(1, prm.poll_every);
  int launched = 0;
  bool done = prm.max_iter <= 0;
  while (!done) {
    for (int g = 0; g < G; ++g) {
      HIP_TRY(launch_real_iteration(prec, a, launched, s));
      ++launched;
    }
    int halt = 0;
    HIP_TRY(hipMemcpyAsync(&halt, &a.st->halt, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (halt || launched >= prm.max_iter + G) done = true;
  }
  HIP_TRY(hipMemcpyAsync(&h, a.st, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::vector<double> rel(ns, 0.0);
  const double bn = std::sqrt(h.bnorm2);
  if (prm.verify && h.status == 0 && bn > 0.0) {
    for (int k = 0; k < ns; ++k)
      HIP_TRY(launch_real_verify(a, d_x + int64_t(k) * n, op->sigma[k], d_res2 + k, s));
    std::vector<double> r2(ns);
    HIP_TRY(hipMemcpyAsync(r2.data(), d_res2, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < ns; ++k) rel[k] = std::sqrt(r2[k]) / bn;
  }
  if (info) {
    clear_timing(*info);
    info->iters = h.iter;
    info->refine_iters = 0;
    info->n_reliable = 0;
    info->n_refined = 0;
    info->iters_fp64 = prec == MSC_PREC_FP64 ? h.iter : 0;
    const double w = double(el), nn = double(n);
    // per iteration: matrix (value + index per stored entry, diagonal), p gather and t
    // write (RK1); r r/w, t, p (RK2); r, p r/w, x_0 r/w (RK3); per live shift x_k r/w
    // (FP64) and p_k r/w
    const double ib = sm.col16 ? 2.0 : 4.0;
    const double mat = double(op->nnz) * (w + ib) + 4.0 * (nn + 1);
    double upd = 0.0;
    for (int j = 1; j < ns; ++j) {
      const int fi = h.freeze_iter[j] < 0 ? h.iter : h.freeze_iter[j];
      upd += double(fi) * nn * (16.0 + 2 * w);
    }
    info->alg_bytes =
        double(h.iter) * (mat + nn * (2 * w) + nn * (4 * w) + nn * (3 * w + 16.0)) + upd;
    if (info->true_rel_res)
      for (int k = 0; k < ns; ++k) info->true_rel_res[k] = rel[k];
    if (info->freeze_iter)
      for (int j = 0; j < ns; ++j) {
        int fi = h.freeze_iter[j];
        if (j == 0 || fi < 0) fi = h.R <= h.eps2 ? h.iter : -1;
        info->freeze_iter[order[j]] = fi;
      }
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (h.status != 0) {
    set_error("msc_solve_real: breakdown (p.(A + sigma_min) p <= 0 or not finite) at iteration %d",
              h.iter);
    return MSC_EBREAKDOWN;
  }
  if (!(h.R <= h.eps2)) {
    set_error("msc_solve_real: the iteration limit was reached");
    return MSC_ENOTCONV;
  }
  if (prm.verify)
    for (int k = 0; k < ns; ++k)
      if (!(rel[k] <= prm.tol)) {
        set_error("msc_solve_real: shift %d misses tol in FP64 (%.3e)", k, rel[k]);
        return MSC_ENOTCONV;
      }
  return MSC_OK;
}

msc_status msc_solve_batched(int32_t nsys, const msc_op* ops, const int32_t* nrhs,
                             const double* const* d_b, double* const* d_x,
                             const msc_params* params, msc_info* info, msc_stream stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (nsys < 1 || !ops || !nrhs || !d_b || !d_x) {
    set_error("msc_solve_batched: need nsys >= 1 and non-null host arrays");
    return MSC_EINVAL;
  }
  msc_params prm;
  if (params)
    prm = *params;
  else
    msc_params_default(&prm);
  if (!(prm.tol >= 0.0) || (prm.prec != MSC_PREC_FP64 && prm.prec != MSC_PREC_MIXED) ||
      !(prm.mixed_margin > 0.0 && prm.mixed_margin <= 1.0) ||
      prm.format < MSC_FORMAT_AUTO || prm.format > MSC_FORMAT_SELL32 ||
      prm.update_steps < 1 || prm.update_steps > kMaxSteps || (prm.sweep != 0 && prm.sweep != 1)) {
    set_error("msc_solve_batched: invalid tol, precision, mixed_margin, format, update_steps "
              "or sweep");
    return MSC_EINVAL;
  }
  int rr = 1, max_nrhs = 0;
  for (int s = 0; s < nsys; ++s) {
    const msc_op op = ops[s];
    if (!op || op->kind == MSC_A_GENERAL || op->sigma.empty() ||
        int(op->sigma.size()) > kBatchMaxShifts || nrhs[s] < 1 ||
        nrhs[s] > kBatchMaxRhs || !d_b[s] || !d_x[s]) {
      set_error("msc_solve_batched: system %d: need a Hermitian operator with 1..%d shifts, "
                "1..%d right-hand sides and non-null b and x", s, kBatchMaxShifts, kBatchMaxRhs);
      return MSC_EINVAL;
    }
    max_nrhs = std::max(max_nrhs, int(nrhs[s]));
  }
  while (rr < max_nrhs) rr *= 2;
  hipStream_t user = static_cast<hipStream_t>(stream);
  BatchRun run;
  msc_status rc = run.setup(nsys, ops, nrhs, d_b, d_x, rr, prm);
  if (rc != MSC_OK) return rc;
  rc = run.solve(prm, user);
  if (rc != MSC_OK) return rc;
  return run.finish(prm, info, user, t0);
}

void msc_op_destroy(msc_op op) {
  if (!op) return;
  free_workspace(op->ws);
  free_bss(op->bws);
  dfree(op->yadj);
  dfree(op->adj_small);
  dfree(op->scratch.partial);
  dfree(op->scratch.tickets);
  dfree(op->scratch.res2);
  dfree(op->rowptr);
  dfree(op->col);
  dfree(op->val64);
  dfree(op->val32);
  dfree(op->rowptr_h);
  dfree(op->col_h);
  dfree(op->perm_h);
  dfree(op->val64_h);
  dfree(op->val32_h);
  free_sell(op->sell_m);
  free_sell(op->sell_mh);
  if (op->bcg) (void)hipFree(op->bcg);
  if (op->osb) (void)hipFree(op->osb);
  if (op->rws) (void)hipFree(op->rws);
  dfree(op->rval64);
  dfree(op->rval32);
  dfree(op->rdiag64);
  dfree(op->rdiag32);
  if (op->w64.w) (void)hipFree(const_cast<double2*>(op->w64.w));
  if (op->w32.w) (void)hipFree(const_cast<float2*>(op->w32.w));
  if (op->wc64.w) (void)hipFree(const_cast<double2*>(op->wc64.w));
  if (op->wc32.w) (void)hipFree(const_cast<float2*>(op->wc32.w));
  delete op;
}

}  // extern "C"
