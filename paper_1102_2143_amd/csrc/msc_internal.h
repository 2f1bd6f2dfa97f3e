// Internal declarations shared by the host driver and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "msc.h"

namespace msc {

constexpr int kMaxShifts = 64;
constexpr int kBlock = 256;          // threads per workgroup for every solver kernel
constexpr int kMaxGrid = 2048;       // 256 CUs x 8 resident workgroups
constexpr int kXcds = 8;             // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kTrEvery = 64;         // launches between two direct products t = M p
// A "last workgroup" ticket site: eight group counters 128 bytes apart and a final one.
constexpr int kTicketStride = 32;
constexpr int kTicketSite = 9 * kTicketStride;

// Scalar state of one multishift solve, resident in device memory.  Shift index j runs
// over the shifts sorted ascending; j = 0 is the driving shift sigma0.
//
// An iteration is a head kernel, which first applies the previous iteration's update
// (x, p_j, p) and then computes t = M p (K1), followed by K2.  No kernel waits for its
// own reduction: each workgroup stores a partial sum and the workgroups of the next
// kernel add the partials up themselves, in one fixed order, so they all obtain the same
// value.  Workgroup 0 of K2 stores the step constants for the next head; workgroup 0 of
// the head stores the state the rest of the iteration and the next head start from.
// What every head workgroup reads while its workgroup 0 writes the successor values is
// kept twice (RotState): the head of an iteration of parity par reads rot[par] and
// writes rot[par ^ 1], which K2 and the reliable update then use.
struct RotState {
  double R;                    // |r|^2 of the driving recursive residual
  int iter;                    // iterations completed
  int halt;                    // 1: the kernels of this iteration do no work
  int switch_req;              // 1: halted because the FP64 phase of a mixed solve ended
  int status;                  // 0 running/ok, 1 breakdown
  int pending;                 // 1: the previous K2's r awaits its update of x, p_j and p
  int pcur;                    // which of the two direction buffers holds p
  int ndef;                    // steps of the all-shift update deferred so far (their
                               // residuals kept; SolveState::dfs)
  double zeta[kMaxShifts];     // zeta_j^(n)
  int active[kMaxShifts];      // shift j still updated
};

// Reliable updates of the complex64 phase: the host launches the update kernels every
// kRuCheck iterations; they run when the period (msc_params::reliable_every) is due, or
// when the recursive |r|^2 has dropped below kRuDelta2 times its value at the last update
// (a residual that falls fast would otherwise run far below what the complex64 operator
// can certify before the next replacement).
constexpr int kRuCheck = 10;
constexpr double kRuDelta2 = 1e-2;

// Head launches whose update mode is recorded for the byte model of sampled timings.
constexpr int kMaxSamples = 256;

// Steps of the all-shift update one pass over x_j and p_j may fold together: up to 8 in
// the single solve, up to 4 in the batched one (whose update kernel holds the kept
// residuals of four right-hand sides).
constexpr int kMaxSteps = 8;
constexpr int kBatchMaxSteps = 4;

// Deferred steps of shift j composed against the direction p_j at the first of them and
// the residuals r_0..r_{m-1} the deferring heads kept: so far
//   x_j gained cx[0] p_j + sum_k cx[k+1] r_k,  and p_j now is cp[0] p_j + sum_k cp[k+1] r_k.
struct DeferState {
  double cx[kMaxSteps][kMaxShifts];
  double cp[kMaxSteps][kMaxShifts];
  int act[kMaxShifts];          // shift j took part in a deferred step
  int upd[kMaxShifts];          // a deferred step changed p_j
};

struct SolveState {
  double a;          // a_n = R / (p^H (A + sigma0) p)      (K2, workgroup 0)
  double a_prev;     // a_{n-1} (1 before the first iteration)
  double b;          // b_{n-1}, last direction coefficient (0 at start)
  double P;          // p^H (A + sigma0) p                  (K2, workgroup 0)
  double sigma0;
  double bnorm2;
  double eps2;       // (mixed_margin) tol^2 |b|^2
  double sw_eps2;    // switch_tol^2 |b|^2: end of the FP64 phase of a mixed solve (0: none)
  int max_iter;
  int ns;
  int freeze;
  int n_reliable;
  int kstatus;       // 1: a K2 found p^H (A + sigma0) p <= 0
  int rslot;         // residual slot a halting head read (where r stays: no K2 follows it)
  double R_ru;       // |r|^2 right after the last reliable update (or the precision switch)
  double s[kMaxShifts];         // sigma_j - sigma0
  double zeta_prev[kMaxShifts]; // zeta_j^(n-1)
  double zk[kMaxShifts];        // zeta_j^(n+1) of the current iteration (K2 -> head)
  double ak[kMaxShifts];        // a_j^(n) = a_n zeta^(n+1)/zeta^(n)       (K2 -> head)
  int freeze_iter[kMaxShifts];
  int orig[kMaxShifts];         // caller's index of sorted shift j
  RotState rot[2];              // rot[par]: state at the start of an iteration of parity par
  // the deferred steps of the all-shift update, composed (DeferState), indexed by the
  // parity of the head that writes them
  DeferState dfs[2];
  // per sampled head launch (MsArgs::sample): its update mode (Plan), shifts listed and
  // kept residuals read
  int smp_mode[kMaxSamples];
  int smp_nact[kMaxSamples];
  int smp_m[kMaxSamples];
  // per phase (0: FP64, 1: complex64): x_j/p_j row updates performed (in units of n
  // rows), heads that deferred their update, passes over kept residuals (an applying head
  // reads the ones pending from the ring), heads that applied the
  // update (x_0 read and written), and heads that kept the direction for x_0's deferred
  // steps (the applying head of that cycle reads it back)
  int n_shift_upd[2];
  int n_defer[2];
  int n_two[2];
  int n_apply[2];
  int n_keep0[2];
  int pad2_[2];
};

// Per-kernel partial-sum scratch, sized for kMaxGrid workgroups x kMaxShifts values.
struct Scratch {
  double* partial = nullptr;    // kMaxGrid * kMaxShifts doubles
  unsigned* tickets = nullptr;  // 16 counters, zero between launches
  double* res2 = nullptr;       // kMaxShifts doubles (verification output)
};

// CSR in device memory with int32 row pointers.
template <class V> struct Csr {
  const int32_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const V* val = nullptr;
};

// Sliced ELLPACK copy of a CSR matrix for the iteration SpMVs: slices of kSlice rows
// (one wavefront, one row per lane), the diagonal held apart in `diag`, the off-diagonal
// entries of a slice stored by pairs.  Entry k of lane l of slice s sits at
//   (cptr[s] + k / 2) * 2 kSlice + 2 l + (k % 2),
// so a lane reads two entries with one load and a wavefront reads whole cache lines;
// cptr[s + 1] - cptr[s] is the slice's width in pairs.  Padding entries hold 0 and a
// valid column.
constexpr int kSlice = 64;
template <class V> struct Sell {
  const int32_t* cptr = nullptr;  // nslices + 1
  const int32_t* col = nullptr;
  const V* val = nullptr;
  const V* diag = nullptr;        // n
  int32_t wp = 0;                 // > 0: every slice is wp pairs wide (cptr[s] = s wp)
  // Narrow columns (both set, or both null: then col is read).  Entry position e of pair
  // column c (e = 0, 1; c counts pair columns over all slices) has base cbase[2c + e];
  // the pair of lane l holds the two 16-bit offsets from those bases, entry 0 in the low
  // half, at col16[c kSlice + l].
  const uint32_t* col16 = nullptr;
  const int32_t* cbase = nullptr;
};

// Matrix-free staggered operator M = m + D on a periodic 4-D lattice (every extent >= 3):
// w holds W_mu(x) = eta_mu(x)/2 U_mu(x) value-major as [4][K][V] (direction, entry of the
// row-major 3x3 matrix, site with x0 fastest; K = 9, or 6 with rows = 2), so that
//   (D v)(x) = sum_mu [ W_mu(x) v(x + mu) - W_mu(x - mu)^H v(x - mu) ]
// (eta_mu does not depend on x_mu).  Row 3 s + c of M is colour c of site s.
template <class V> struct Stencil {
  const V* w = nullptr;
  int32_t rows = 3;  // rows of each link stored: 3, or 2 (SU(3): the third is rebuilt)
  int32_t L[4] = {0, 0, 0, 0};
  int64_t stride[4] = {0, 0, 0, 0};  // 1, L0, L0 L1, L0 L1 L2
  int64_t vol = 0;
  double mass = 0.0;
};

// Order in which the waves of the iteration kernels (head and K2 on the sliced path) visit
// the slices of 64 rows, for operators with a lattice structure: rows s1 slices apart are
// neighbours in one direction (a plane), rows s2 slices apart in the slowest one (a slab),
// and a plane is cut into tiles of cs slices.  on = 0: every workgroup sweeps one
// contiguous range of slices.
struct SweepOrder {
  int32_t s1, s2, cs, on;
};

// Device buffers of one sliced ELLPACK matrix (both value precisions share the columns).
struct SellStore {
  int64_t nslices = 0;
  int64_t pairs = 0;              // total pairs of all slices
  int32_t wp = 0;                 // common width in pairs when all slices agree, else 0
  int32_t* cptr = nullptr;
  int32_t* col = nullptr;
  double2* val64 = nullptr;
  float2* val32 = nullptr;
  double2* diag64 = nullptr;
  float2* diag32 = nullptr;
  uint32_t* col16 = nullptr;      // narrow columns, when every slice column's entries span
  int32_t* cbase = nullptr;       // less than 2^16 (else both null)
};

struct Workspace {
  size_t n = 0;
  int ns = 0;
  int prec = -1;
  void* r = nullptr;    // n complex128
  void* p[2] = {nullptr, nullptr};    // two n complex128 direction buffers
  void* t = nullptr;    // n complex128
  void* pk = nullptr;   // (ns-1) * n complex128
  void* r32 = nullptr;  // complex64 copies for the second phase of a mixed solve
  void* p32[2] = {nullptr, nullptr};
  void* t32 = nullptr;
  void* pk32 = nullptr;
  double2* t64 = nullptr;   // n complex128 (reliable updates, verification)
  void* pkeep0 = nullptr;           // n complex128 (complex64 in phase 2): x_0's first deferred direction
  void* rkeep[kMaxSteps - 1] = {};  // n complex128 each (complex64
                            // in the second phase): residuals kept by deferring heads
  double2* u64 = nullptr;   // 8 * n complex128 (verification SpMM chunk)
  SolveState* st = nullptr;
  int* h_halt = nullptr;    // host-coherent word the heads write: halt | switch_req << 1
  int* d_halt = nullptr;    // its device address
  hipEvent_t ev[2] = {nullptr, nullptr};
};

struct BssState;

// Buffers of the batched single-shift CG (interleaved n x mp vectors).
struct BssWorkspace {
  size_t n = 0;
  int mp = 0;
  int prec = -1;
  void* p = nullptr;
  void* t = nullptr;
  void* r = nullptr;
  void* e = nullptr;
  BssState* st = nullptr;
  int* h_halt = nullptr;    // host-coherent copy of st->halt, written by the last IK2
  int* d_halt = nullptr;    // its device address
  hipEvent_t ev[2] = {nullptr, nullptr};
};

}  // namespace msc

struct msc_op_s {
  int kind = 0;
  int64_t n = 0, nnz = 0, nnz_h = 0;
  int device = 0;
  int32_t* rowptr = nullptr;     // M (or A): int32[n+1]
  int32_t* col = nullptr;
  double2* val64 = nullptr;
  float2* val32 = nullptr;
  int32_t* rowptr_h = nullptr;   // M^H (kind MHM only)
  int32_t* col_h = nullptr;
  int32_t* perm_h = nullptr;     // entry of M^H -> entry of M
  double2* val64_h = nullptr;
  float2* val32_h = nullptr;
  std::vector<double> sigma;
  msc::Workspace ws;
  msc::BssWorkspace bws;
  msc::Scratch scratch;
  void* bcg = nullptr;           // BiCGStab-M buffers (one allocation)
  size_t bcg_bytes = 0;
  void* osb = nullptr;           // per-shift right-hand sides: guesses and tables
  size_t osb_bytes = 0;
  // real copies of the sliced matrix (built on the first real solve of a real operator)
  double* rval64 = nullptr;
  float* rval32 = nullptr;
  double* rdiag64 = nullptr;
  float* rdiag32 = nullptr;
  int real_state = 0;            // 0 not checked, 1 real (copies built), -1 not real
  void* rws = nullptr;           // real solve buffers
  size_t rws_bytes = 0;
  double2* yadj = nullptr;       // adjoint solutions, ns * n complex128
  size_t yadj_count = 0;
  double* adj_small = nullptr;   // 256 doubles: Gram sums and shift factors
  int lanes64 = 0, lanes32 = 0;  // chosen lanes per row (0 = not yet tuned)
  msc::SweepOrder order{0, 0, 0, 0};  // lattice structure of the rows (zeros: none found)
  msc::SweepOrder order_sites{0, 0, 0, 0};    // the same in blocks of 64 sites (links'
  msc::SweepOrder order_sites64{0, 0, 0, 0};  // kernels; complex64 and FP64 tile spans)
  int64_t rowhist[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // rows by length: 0, 1, 2-3, ..., >= 64
  bool stencil = false;          // matrix-free staggered operator (links kept below)
  msc::Stencil<double2> w64;     // W_mu(x) = eta_mu(x)/2 U_mu(x), complex128 and
  msc::Stencil<float2> w32;      // complex64 copies (device memory owned by the op)
  bool two_rows = false;         // every link is in SU(3): the iteration reads wc64 / wc32,
  msc::Stencil<double2> wc64;    // the first two rows of each W_mu(x) (6 values), and
  msc::Stencil<float2> wc32;     // rebuilds the third from them
  bool sell = false;             // sliced ELLPACK copies built (M, and M^H for kind MHM)
  msc::SellStore sell_m, sell_mh;
};

namespace msc {

// ---- launchers implemented in the kernel translation units -------------------------
// All launchers enqueue on `s` and return hipGetLastError() of the launch.

// setup.hip
hipError_t launch_validate_csr(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                               int* d_err, hipStream_t s);
hipError_t launch_rowptr_to32(const int64_t* in, int32_t* out, int64_t n, hipStream_t s);
// Row-length histogram (8 power-of-two buckets: 0, 1, 2-3, ..., >= 64) into hist[8].
hipError_t launch_row_hist(const int32_t* rowptr, int64_t n, unsigned long long* hist, hipStream_t s);
hipError_t launch_cast_vals(const double2* in, float2* out, int64_t nnz, hipStream_t s);
hipError_t build_adjoint(const int32_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                         int32_t* rowptr_h, int32_t* col_h, int32_t* perm_h, hipStream_t s);
hipError_t launch_adjoint_vals(const int32_t* perm_h, const double2* val64, double2* val64_h,
                               float2* val32_h, int64_t nnz, hipStream_t s);
// Build the sliced ELLPACK copy of a CSR matrix into `out` when its padding stays small
// (slots <= 1.5 nnz + 2 kSlice per slice); *built tells whether it was.  The narrow
// columns are added when every slice column's entries span less than 2^16.  Synchronises `s`.
hipError_t build_sell(const int32_t* rowptr, const int32_t* col, const double2* val64, int64_t n,
                      int64_t nnz, SellStore& out, bool* built, hipStream_t s);
// Rewrite the values (and diagonal) of a built copy from the CSR values.
hipError_t refill_sell(const int32_t* rowptr, const int32_t* col, const double2* val64, int64_t n,
                       const SellStore& out, hipStream_t s);
void free_sell(SellStore& out);
// Matrix-free staggered operator set-up: w64 = eta/2 U from the caller's complex128
// links [4][V][3][3], stored [4][9][V], w32 = complex64 copy; and the scalar CSR of M = m + D built from
// w64 (25 entries per row, columns sorted): rowptr int64[n+1], col int32[25n],
// vals complex128[25n].
hipError_t launch_stencil_links(const double2* links, const Stencil<double2>& geo,
                                double2* w64, float2* w32, hipStream_t s);
hipError_t launch_stencil_csr(const Stencil<double2>& op, int64_t* rowptr, int32_t* col,
                              double2* vals, hipStream_t s);
// Largest deviation of the caller's links [4][V][3][3] from SU(3) over all links,
// max(|U U^H - I|, |det U - 1|) entrywise, into *dev (as the bits of a double; the
// caller zeroes it first).
hipError_t launch_su3_deviation(const double2* links, int64_t nlinks, unsigned long long* dev,
                                hipStream_t s);
// The first two rows of every W_mu(x) of the full copy w64 [4][9][V] into wc64 / wc32
// [4][6][V].
hipError_t launch_two_rows(const double2* w64, int64_t nlinks, double2* wc64, float2* wc32,
                           hipStream_t s);

// multishift.hip
struct MsArgs {
  int kind;
  int64_t n;
  int lanes;
  int grid;
  Csr<double2> m64, mh64;
  Csr<float2> m32, mh32;
  int par;               // parity of the iteration: its state is st->rot[par]
  int gk1, gk2;          // workgroups of this iteration's K1 and K2 (partials to sum)
  int sell;              // K1/K2 read the sliced ELLPACK copies below
  int64_t nslices;
  Sell<double2> s64, sh64;
  Sell<float2> s32, sh32;
  const double2* b;
  double2* x;            // caller's x, shift-major, caller order
  void* r; void* t; void* pk;
  void* pb[2];           // the two direction buffers (p of consecutive iterations)
  // the residual lives in a ring of kMaxSteps slots: slot 0 is r, slot k >= 1 is
  // rkeep[k - 1]; a head with m steps deferred reads r from slot m, so the m residuals of
  // the heads that deferred stay in slots 0..m-1 without a copy, and K2 writes the next
  // residual into the slot of the next head (0 after a head that applied)
  void* rkeep[kMaxSteps - 1];
  void* pkeep0;          // the direction p at the first deferred step (x_0's deferred update)
  int* hflag;            // host-coherent word: halt | switch_req << 1 of the next state
  int steps;             // steps of the all-shift update folded into one pass (1..kMaxSteps)
  int defer_ok;          // 1: this launch's head may defer its all-shift update
  int ru_force;          // reliable-update launch: 1 runs it whatever the residual
  int ru_check;          // 1: the reliable-update kernels follow this head (x_0 must be
                         // current when they run)
  int stencil;           // the head and K2 apply M and M^H from links (kind MHM, sell = 1):
                         // 0 no, 3 full links, 2 two rows per link (w64 / w32 in that form)
  SweepOrder ord;        // slice order of the head and K2 on the sliced path
  int k2_march;          // links: t-slices per column of K2's march (set per launch; 1: none)
  int head_march;        // links: the same for the head (1: the sweep order)
  int t_rec;             // links, FP64: this head forms t' = M r + b t (the old t = M p)
  Stencil<double2> w64;
  Stencil<float2> w32;
  int sample;            // slot of SolveState::smp_* for this head, -1: not sampled
  double2* t64;
  SolveState* st;
  Scratch sc;
};
hipError_t launch_init(int prec, const MsArgs& a, hipStream_t s);
// One iteration of parity a.par; with `reliable`, the FP64 reliable update runs between
// the head and K2.  ev (optional, 6 events): start/stop pairs attached to the K1 (head),
// K2 and, on the CSR path, the separate update kernel.
hipError_t launch_iteration(int prec, const MsArgs& a, hipStream_t s, hipEvent_t* ev = nullptr,
                            bool reliable = false);
// Second phase of a mixed solve: copy r, p, p_j of a64 (complex128) into a32's complex64
// buffers and re-arm the state (halt = switch_req = 0, no further switch).
hipError_t launch_switch_to_mixed(const MsArgs& a64, const MsArgs& a32, int ns, hipStream_t s);
// FP64 true residual norms^2 of shifts [k0, k0+kc) (kc <= 8) of x into sc.res2[k0..].
hipError_t launch_verify(const MsArgs& a, const double* sigma_by_caller_index, int k0, int kc,
                         double2* u64, hipStream_t s);
hipError_t launch_apply(int kind, int prec, int lanes, int64_t n, const Csr<double2>& m64,
                        const Csr<double2>& mh64, const Csr<float2>& m32,
                        const Csr<float2>& mh32, const double2* in, double2* out,
                        double shift, void* tmp_a, void* tmp_b, hipStream_t s);

// No-allocation apply: temporaries in a file-scope device array of this many bytes per GPU
// (FP64: n <= 2^21 rows for A = M^H M, 2^22 for A given; complex64: n <= 2^22).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Bytes of that array one apply of n rows needs.
size_t apply_scratch_bytes(int kind, int prec, int64_t n);
// The array's address on `device`, which must be the current device; looked up with
// hipGetSymbolAddress on the first call per device and kept.
hipError_t noalloc_scratch(int device, void** ptr);
// launch_apply with its temporaries carved from `base` (the address noalloc_scratch
// returned); hipErrorInvalidValue when n exceeds the array.
hipError_t launch_apply_noalloc(int kind, int prec, int lanes, int64_t n,
                                const Csr<double2>& m64, const Csr<double2>& mh64,
                                const Csr<float2>& m32, const Csr<float2>& mh32,
                                const double2* in, double2* out, double shift, void* base,
                                hipStream_t s);

int default_grid(int64_t n, int lanes);

// bicgstab.hip -- multishift BiCGStab for a general A (complex FP64 scalars)
struct BcgCoef {
  double2 xp, xs;          // x(s) += xp p(s) + xs s
  double2 pr, pp, po, ps;  // p(s) <- pr r' + pp p(s) + po r + ps s
};
struct BcgState {
  double sigma0, bnorm2, eps2, R;
  double2 rho, alpha, omega, beta, al_prev, be_prev;
  int iter, max_iter, halt, status, rotate, upd_launch, ns, pad_;
  double s[kMaxShifts];              // sigma_j - sigma0, shifts sorted ascending
  double2 z[kMaxShifts], z_old[kMaxShifts], z_new[kMaxShifts];
  double2 tau[kMaxShifts], tau_new[kMaxShifts];
  double2 al_s[kMaxShifts], om_s[kMaxShifts];
  BcgCoef cf[kMaxShifts];
  int active[kMaxShifts], active_next[kMaxShifts], freeze_iter[kMaxShifts], orig[kMaxShifts];
};
struct BcgArgs {
  int64_t n;
  int ns, lanes, par;
  Csr<double2> m;
  const double2* b;       // right-hand side, also the shadow vector
  double2* x;             // caller's x, shift-major, caller order
  double2* r[2];          // r_n and r_{n+1} alternate
  double2 *p, *v, *s, *t;
  double2* pk;            // ns directions, sorted order
  BcgState* st;
  double* partial;        // >= 4 kMaxGrid doubles
  unsigned* tickets;      // one ticket site
};
hipError_t launch_bcg_init(const BcgArgs& a, hipStream_t s);
hipError_t launch_bcg_iteration(const BcgArgs& a, int launch, hipStream_t s);

// real_ms.hip -- multishift CG for a real symmetric positive-definite A
template <class T> struct SellReal {
  const int32_t* cptr = nullptr;
  const int32_t* col = nullptr;
  const uint32_t* col16 = nullptr;  // narrow columns (with cbase), or null: col is read
  const int32_t* cbase = nullptr;
  int32_t wp = 0;
  const T* val = nullptr;           // real parts of the sliced copy's values
  const T* diag = nullptr;
};
struct RealState {
  double a, a_prev, b, b_new, P, R, sigma0, bnorm2, eps2;
  int iter, max_iter, ns, halt, status, rotate, upd_launch, freeze;
  double s[kMaxShifts], zeta[kMaxShifts], zeta_prev[kMaxShifts], zeta_new[kMaxShifts];
  double ak[kMaxShifts], bk[kMaxShifts];
  int active[kMaxShifts], active_next[kMaxShifts], freeze_iter[kMaxShifts], orig[kMaxShifts];
};
struct RealArgs {
  int64_t n, nslices;
  int ns;
  SellReal<double> m64;
  SellReal<float> m32;
  const double* b;
  double* x;               // caller's x, shift-major, caller order (FP64 always)
  void *r, *p, *t, *pk;    // double or float by precision
  RealState* st;
  double* partial;
  unsigned* tickets;       // one ticket site
};
hipError_t launch_real_extract(const double2* v64, double* r64, float* r32, int64_t count,
                               unsigned long long* imax, hipStream_t s);
hipError_t launch_real_init(int prec, const RealArgs& a, hipStream_t s);
hipError_t launch_real_iteration(int prec, const RealArgs& a, int launch, hipStream_t s);
hipError_t launch_real_verify(const RealArgs& a, const double* x, double sigma, double* out,
                              hipStream_t s);

// osborn.hip -- a right-hand side per shift through common-residual initial guesses
constexpr int kOsbSlices = 256;  // workgroups per vector of the norm reduction
hipError_t launch_osb_divdiff(const double2* B, const int* orig, const double* inv, double2* W,
                              int m, int64_t n, hipStream_t s);
hipError_t launch_osb_sub(double2* y, const double2* t, int64_t n, hipStream_t s);
hipError_t launch_osb_combine(const double2* W, const double* w, const int* orig, double2* x,
                              int m, int64_t n, hipStream_t s);
hipError_t launch_osb_add(double2* x, const double2* d, int64_t count, hipStream_t s);
hipError_t launch_osb_norms(const double2* v, int count, int64_t n, double* partial,
                            unsigned* tickets, double* out, hipStream_t s);

// batched_cg.hip -- m <= kBssMax single-shift systems sharing one operator
constexpr int kBssMax = 16;
constexpr int kResChunk = 8;

struct BssState {
  double R[kBssMax];        // |r_j|^2 (recursive, inner)
  double a[kBssMax];        // step of system j this iteration
  double b[kBssMax];        // direction coefficient of system j
  double target2[kBssMax];  // inner stop: R_j <= target2_j
  double sigma[kBssMax];
  int active[kBssMax];
  int upd[kBssMax];         // system j was updated this iteration (e_j += a_j p_j)
  int iters[kBssMax];
  int bad[kBssMax];         // breakdown of system j
  int m, mp, iter, max_iter, halt, nact, k3_enable, pad_;
};

struct BssArgs {
  int kind;
  int mp;
  int64_t n;
  Csr<double2> m64, mh64;
  Csr<float2> m32, mh32;
  int sell;                             // 1: the SpMVs read the sliced ELLPACK copies
  int64_t nslices;
  Sell<double2> s64, sh64;
  Sell<float2> s32, sh32;
  void* p; void* t; void* r; void* e;   // interleaved n x mp vectors of the working precision
  BssState* st;
  double* partial;                      // kMaxGrid * kBssMax
  unsigned* tickets;
  int* hflag;                           // host-coherent copy of st->halt
};

struct XPtrs {
  double2* x[kBssMax];
};

// FP64 residual r_q = f_q - (A + sig_q) x_q for q < kc (<= kResChunk) systems; writes
// |r_q|^2 to out[q] and, when r != nullptr, r (cast) into column j0 + q of the
// interleaved r and p and zero into e.
struct ResArgs {
  Csr<double2> m1;          // M (MHM) -- first half
  Csr<double2> m2;          // M^H (MHM) or A (HERM)
  int sell;                 // 1: read the sliced ELLPACK copies s1, s2 instead
  int64_t nslices;
  Sell<double2> s1, s2;
  int mhm;
  int64_t n;
  int kc;
  int mp, j0;
  const double2* x[kResChunk];
  const double2* f[kResChunk];
  double sig[kResChunk];
  double2* u;               // kResChunk * n scratch (MHM)
  void* r; void* p; void* e;
  double* partial;
  unsigned* ticket;
  double* out;
};

// batched_ms.hip -- many independent multishift solves per launch
constexpr int kBatchMaxRhs = 4;
constexpr int kBatchMaxShifts = 16;
constexpr int kBatchChunkRows = 256;

struct BatchState {
  // per right-hand side q
  double R[kBatchMaxRhs], a[kBatchMaxRhs], a_prev[kBatchMaxRhs], b[kBatchMaxRhs];
  double b_new[kBatchMaxRhs], bnorm2[kBatchMaxRhs], eps2[kBatchMaxRhs], sw_eps2[kBatchMaxRhs];
  int iter[kBatchMaxRhs], halt[kBatchMaxRhs], status[kBatchMaxRhs], x0_upd[kBatchMaxRhs];
  // per (q, sorted shift k), index q * 16 + k
  double zeta[kBatchMaxRhs * kBatchMaxShifts], zeta_prev[kBatchMaxRhs * kBatchMaxShifts];
  double zk[kBatchMaxRhs * kBatchMaxShifts], ak[kBatchMaxRhs * kBatchMaxShifts];
  double bk[kBatchMaxRhs * kBatchMaxShifts];
  int active[kBatchMaxRhs * kBatchMaxShifts], freeze_iter[kBatchMaxRhs * kBatchMaxShifts];
  int upd_p[kBatchMaxRhs * kBatchMaxShifts], upd_x[kBatchMaxRhs * kBatchMaxShifts];
  // BK3's update of (q, k) (upd_x, upd_p): x += cx[0] p_k + sum_{i<m} cx[i+1] r_i and
  // p_k <- cp[0] p_k + sum_{i<m} cp[i+1] r_i + cp[m+1] r, the r_i being the residuals
  // kept by the m BK3s that deferred (one step: m = 0)
  double cx[kBatchMaxSteps][kBatchMaxRhs * kBatchMaxShifts];
  double cp[kBatchMaxSteps + 1][kBatchMaxRhs * kBatchMaxShifts];
  // the deferred steps of (q, k) composed as in DeferState
  double dcx[kBatchMaxSteps][kBatchMaxRhs * kBatchMaxShifts];
  double dcp[kBatchMaxSteps][kBatchMaxRhs * kBatchMaxShifts];
  int dact[kBatchMaxRhs * kBatchMaxShifts], dupd[kBatchMaxRhs * kBatchMaxShifts];
  // per right-hand side: steps deferred so far, BK3's kept residuals to read (m) and the
  // slot it keeps r in (-1: none; slot 0 also keeps p, the direction x_0's deferred steps
  // start from), and per phase (FP64, complex64) the shift-vector updates, kept-r
  // passes, BK3s that updated x_0 and BK3s that kept p
  int ndef[kBatchMaxRhs], m[kBatchMaxRhs], keep[kBatchMaxRhs];
  int n_upd[kBatchMaxRhs][2], n_kept[kBatchMaxRhs][2];
  int n_x0[kBatchMaxRhs][2], n_k0[kBatchMaxRhs][2];
  // per system
  double s[kBatchMaxShifts];
  int orig[kBatchMaxShifts];
  double sigma0;
  int ns, nrhs, phase32, switch_pending, done, k3_enable, max_iter, n_reliable, iters_fp64, pad_;
};

struct BatchSys {
  int kind;
  int nchunks;            // chunks of this system (its partial array has 4 slots each)
  int64_t n;
  Csr<double2> m64, mh64;
  Csr<float2> m32, mh32;
  int sell;               // the SpMVs read the system's sliced ELLPACK copies below
  Sell<double2> s64, sh64;
  Sell<float2> s32, sh32;
  const double2* b;       // nrhs * n (rhs-major)
  double2* x;             // nrhs * ns * n (rhs-major, shift-major, caller order)
  double2 *r64, *p64, *t64, *pk64, *u64;   // rhs-interleaved n x RR; pk: (ns-1) blocks
  float2 *r32, *p32, *t32, *pk32;
  void* rkeep[kBatchMaxSteps - 1];  // n x RR each: residuals kept by deferring BK3s
                               // (complex128, or complex64 in the second phase)
  void* pkeep0;           // n x RR: p at the first deferred step (x_0's composition)
  BatchState* st;
  double* partial;
  unsigned* tickets;      // 8 counters
};

struct BatchArgs {
  const BatchSys* sys;
  const int4* chunks;     // (system, row0, row1, chunk index within the system)
  int nchunks;
  int nsys;
  int grid;
  int lanes;
  int rr;                 // right-hand sides per system, padded (1, 2 or 4)
  int* active_systems;
  int defer_ok;           // 1: this iteration's BK3 may defer the shifted update
  int steps;              // steps of the shifted update folded into one pass (1..kBatchMaxSteps)
};

hipError_t launch_batch_init(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_iteration(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_reliable(const BatchArgs& a, hipStream_t s);

// grad.hip
// out[3q..3q+2] = Re<gref, g_q>, Im<gref, g_q>, |g_q|^2 for q < kc (<= 16); g shift-major.
hipError_t launch_gram(const double2* gref, const double2* g, int64_t n, int kc, double* partial,
                       unsigned* ticket, double* out, hipStream_t s);
hipError_t launch_scale_shifts(double2* y, const double* d_c, int ns, int64_t n, hipStream_t s);
// out[q] = |g_q - c_q gref|^2 for q < kc (<= 16)
hipError_t launch_diffnorm(const double2* gref, const double2* g, const double* d_c, int64_t n,
                           int kc, double* partial, unsigned* ticket, double* out, hipStream_t s);
hipError_t launch_sum_shifts(const double2* y, int ns, int64_t n, double2* out, hipStream_t s);
// grad (nnz complex128, creation order) of sum_k Re(g_k^H x_k) given x and y (shift-major);
// u, w: scratch of 4 n complex128 each (A = M^H M only).
hipError_t launch_grad_vals(int kind, int lanes, const Csr<double2>& m, const double2* x,
                            const double2* y, int64_t n, int ns, double2* u, double2* w,
                            double2* grad, hipStream_t s);

hipError_t launch_bss_iteration(int prec, const BssArgs& a, hipStream_t s);
hipError_t launch_residual(int prec, int lanes, const ResArgs& v, hipStream_t s);
hipError_t launch_accum(int prec, const BssArgs& a, const XPtrs& xp, hipStream_t s);

}  // namespace msc
