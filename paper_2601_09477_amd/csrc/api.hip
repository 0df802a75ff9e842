// C-ABI entry points of libcmm: argument checks on the host, then launches.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "cmm_internal.h"

namespace cmm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

cmm_status invalid(const std::string& msg) {
  set_error(msg);
  return CMM_EINVAL;
}

cmm_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return CMM_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return CMM_EHIP;
}

// ------------------------------------------------------------ kernel timing
namespace {
std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_prof;
std::string g_prof_only;  // guarded by g_prof_mu; empty: every kernel is bracketed

// the names ProfScope is constructed with
const char* const kProfNames[] = {
    "hash",        "transpose",       "plan",          "compress",    "reduce",
    "fwht",        "extract",         "sketch",        "accumulate",  "wscatter",
    "adjoint",     "adjoint_reduce",  "extract_entries", "extract_heavy",
    "extract_reps", "extract_topk", "correctness", "fft",        "pairs"};

void prof_clear_locked() {
  for (auto& kv : g_prof)
    for (auto& ev : kv.second) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  g_prof.clear();
}
}  // namespace

// Set on the calling thread while an entry point that must not create any
// runtime object (cmm_estimate_static) runs: its kernels are not timed.
thread_local bool t_prof_suppressed = false;

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), stream_(s) {
  // a host range per launch step, named as its timing category (seen by
  // tracing tools such as rocprofv3 --marker-trace; a few tens of ns when
  // no tool is attached)
  roctxRangePushA(name_);
  if (t_prof_suppressed || !g_prof_on.load(std::memory_order_relaxed)) return;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_only.empty() && g_prof_only != name_) return;
  }
  if (hipEventCreate(&start_) != hipSuccess) { start_ = nullptr; return; }
  if (hipEventRecord(start_, stream_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    start_ = nullptr;
  }
}

ProfScope::~ProfScope() {
  roctxRangePop();
  if (!start_) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess) { (void)hipEventDestroy(start_); return; }
  if (hipEventRecord(stop, stream_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    (void)hipEventDestroy(stop);
    return;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof[name_].emplace_back(start_, stop);
}

namespace {

// Compute units of the current device (256 when it cannot be queried).
int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return 256;
  return cus;
}

// k-ranges per work unit of a fused kernel that runs one work-group per
// CU: its units * g work-groups take ceil(units g / CUs) rounds of
// ceil(n_inner / g) values of k each.  The g that minimises that product
// (the fewest work-groups on ties), among those with units * g a multiple
// of 8 for the XCD-aware order, within eight times the count that gives
// 2048 work-groups and with at least 32 values of k per work-group (each
// work-group first builds its gather offsets and collision descriptors).
int64_t pick_groups(int64_t units, int64_t n_inner) {
  if (n_inner <= 1 || units < 1) return 1;
  const int64_t cus = device_cus();
  int64_t hi = 8 * ((2048 + units - 1) / units);
  if (hi > n_inner / 32) hi = n_inner / 32;
  if (hi < 1) hi = 1;
  int64_t best = 0, best_cost = 0;
  for (int64_t g = 1; g <= hi; ++g) {
    if (((units * g) & 7) != 0 && g != n_inner) continue;
    const int64_t cost = ((units * g + cus - 1) / cus) * ((n_inner + g - 1) / g);
    if (best == 0 || cost < best_cost) {
      best = g;
      best_cost = cost;
    }
  }
  return best > 0 ? best : 1;
}

constexpr int kMaxLog2b = 30;
constexpr int kMaxFftLog2 = 24;       // two LDS-tile passes of at most 2^12 points
// Every buffer the kernels address holds fewer than 2^31 elements: their
// index arithmetic is not audited beyond that.
constexpr int64_t kMaxElems = (int64_t)1 << 31;
// top-K: k plus the last bin's candidates are counted in 32-bit integers
constexpr int64_t kMaxTopK = ((int64_t)1 << 31) - ((int64_t)1 << 15);

// a * b (* c) < 2^31 for non-negative factors (exact: 128-bit product)
bool fits_elems(int64_t a, int64_t b, int64_t c = 1) {
  if (a <= 0 || b <= 0 || c <= 0) return true;
  return (unsigned __int128)a * (unsigned __int128)b * (unsigned __int128)c <
         (unsigned __int128)kMaxElems;
}

cmm_status too_large(const std::string& fn, const char* what) {
  set_error(fn + ": " + what + " would hold 2^31 or more elements, beyond the kernels' "
            "index range");
  return CMM_EUNSUPPORTED;
}
constexpr size_t kLdsBytes = 160 * 1024;
constexpr int64_t kMaxHashDomain = (int64_t)1 << 32;

bool is_f64_or_f32(cmm_dtype t) { return t == CMM_F64 || t == CMM_F32; }

cmm_status check_log2b(int log2b, const char* fn) {
  if (log2b < 1 || log2b > kMaxLog2b)
    return invalid(std::string(fn) + ": log2b must be in [1, 30]");
  return CMM_OK;
}

cmm_status check_d(int d, const char* fn) {
  if (d < 1 || d > 65535) return invalid(std::string(fn) + ": d must be in [1, 65535]");
  return CMM_OK;
}

// ------------------------------------------------------------ estimate plan
// Everything cmm_estimate needs besides the caller's buffers, laid out in
// the workspace in this order.
struct EstimatePlan {
  bool fused = false;
  bool mfma = false;   // precision form (bf16 / fp16 on the matrix cores)
  int lb = 0;          // log2 b_lo of the fused kernel
  int groups = 1;      // k-ranges of the fused kernel
  int64_t kc = 0;      // k-chunk of the composed path
  cmm_dtype cdt = CMM_F64;
  size_t off_at = 0, off_bc = 0, off_planA = 0, off_planB = 0, off_part = 0, off_p = 0;
  size_t off_x = 0, off_y = 0;
  // fused forms with fold bits: tables rotated to the chosen transform window
  bool window = false;
  size_t off_rtab1 = 0, off_rtab2 = 0, off_rot = 0;
  // precision form: merged two-row chains (lists, counts, sums) per operand
  int pair_cap[2] = {0, 0};
  size_t off_plist[2] = {0, 0}, off_pcount[2] = {0, 0}, off_pvals[2] = {0, 0};
  size_t bytes = 0;
};

}  // namespace

cmm_status validate_problem(const cmm_problem* pr, const char* fn) {
  if (!pr) return invalid(std::string(fn) + ": null problem");
  if (pr->n_rows < 0 || pr->n_inner < 0 || pr->n_cols < 0)
    return invalid(std::string(fn) + ": negative dimension");
  if (pr->n_rows > kMaxHashDomain || pr->n_cols > kMaxHashDomain)
    return invalid(std::string(fn) + ": n_rows and n_cols must be <= 2^32 (hash domain)");
  cmm_status s = check_log2b(pr->log2b, fn);
  if (s != CMM_OK) return s;
  if ((s = check_d(pr->d, fn)) != CMM_OK) return s;
  if (pr->estimator != CMM_MEDIAN && pr->estimator != CMM_MEAN)
    return invalid(std::string(fn) + ": unknown estimator");
  if (pr->estimator == CMM_MEDIAN && (pr->d % 2) == 0)
    return invalid(std::string(fn) + ": the median estimator needs an odd d");
  if (!is_f64_or_f32(pr->in_dtype))
    return invalid(std::string(fn) + ": in_dtype must be CMM_F64 or CMM_F32");
  if (pr->compute == CMM_F64 && pr->in_dtype != CMM_F64)
    return invalid(std::string(fn) + ": compute CMM_F64 needs in_dtype CMM_F64");
  if (pr->compute != CMM_F64 && pr->compute != CMM_F32 && pr->compute != CMM_BF16 &&
      pr->compute != CMM_F16)
    return invalid(std::string(fn) + ": unknown compute type");
  // leading dimensions matter only for matrices that hold elements
  if ((pr->n_rows > 0 && pr->lda < pr->n_inner) || (pr->n_inner > 0 && pr->ldb < pr->n_cols))
    return invalid(std::string(fn) + ": leading dimension smaller than the row length");
  if (pr->n_rows > 0 && pr->n_inner > 0 && !pr->A) return invalid(std::string(fn) + ": A is null");
  if (pr->n_inner > 0 && pr->n_cols > 0 && !pr->B) return invalid(std::string(fn) + ": B is null");
  if ((pr->n_rows > 0 && !pr->tab1) || (pr->n_cols > 0 && !pr->tab2))
    return invalid(std::string(fn) + ": tab1 / tab2 must be given (outputs when keys != NULL)");
  if (pr->compute == CMM_BF16 || pr->compute == CMM_F16) {
    if (pr->log2b < 14) {
      set_error(std::string(fn) + ": the bf16/f16 precision form needs log2b >= 14");
      return CMM_EUNSUPPORTED;
    }
    if (pr->n_rows > 16383 || pr->n_cols > 16383 ||
        (2 * 16384 + (pr->n_rows + 72) / 8 * 8 + (pr->n_cols + 72) / 8 * 8) * 2 > 160 * 1024 - 256 ||
        plan_lds_bytes(pr->n_rows, 14) > 160 * 1024 || plan_lds_bytes(pr->n_cols, 14) > 160 * 1024) {
      set_error(std::string(fn) + ": the bf16/f16 precision form needs n_rows, n_cols <= 16383");
      return CMM_EUNSUPPORTED;
    }
  }
  if (pr->C_hat) {
    if (!is_f64_or_f32(pr->out_dtype))
      return invalid(std::string(fn) + ": out_dtype must be CMM_F64 or CMM_F32");
    if (pr->n_rows > 0 && pr->ldc < pr->n_cols) return invalid(std::string(fn) + ": ldc < n_cols");
    if (!fits_elems(pr->n_rows, pr->ldc)) return too_large(fn, "C_hat (n_rows x ldc)");
  }
  if (!fits_elems(pr->n_rows, pr->lda) || !fits_elems(pr->n_rows, pr->n_inner))
    return too_large(fn, "A (n_rows x lda)");
  if (!fits_elems(pr->n_inner, pr->ldb) || !fits_elems(pr->n_inner, pr->n_cols))
    return too_large(fn, "B (n_inner x ldb)");
  if (!fits_elems(pr->d, (int64_t)1 << pr->log2b)) return too_large(fn, "p (d x 2^log2b)");
  if (!fits_elems(pr->d, pr->n_rows) || !fits_elems(pr->d, pr->n_cols))
    return too_large(fn, "a hash table (d x n)");
  return CMM_OK;
}

namespace {

// Rotated tables and window choices for the fused forms when b > b_lo.
size_t add_window(EstimatePlan& P, const cmm_problem* pr, size_t off) {
  P.window = pr->log2b > P.lb;
  if (!P.window) return off;
  const int d = pr->d;
  P.off_rtab1 = off; off = align_up(off + sizeof(uint32_t) * (size_t)d * pr->n_rows, 256);
  P.off_rtab2 = off; off = align_up(off + sizeof(uint32_t) * (size_t)d * pr->n_cols, 256);
  P.off_rot = off; off = align_up(off + sizeof(int32_t) * (size_t)d, 256);
  return off;
}

EstimatePlan make_plan(const cmm_problem* pr) {
  EstimatePlan P;
  P.cdt = pr->compute == CMM_F64 ? CMM_F64 : CMM_F32;
  const size_t es = dtype_size(P.cdt);
  const int64_t b = (int64_t)1 << pr->log2b;
  const int d = pr->d;
  if (pr->compute == CMM_BF16 || pr->compute == CMM_F16) {
    // precision form: b_lo = 2^14, low-precision operand copies in the workspace
    P.mfma = true;
    P.fused = true;
    P.lb = 14;
    const int64_t units = (int64_t)d << (pr->log2b - 14);
    P.groups = (int)pick_groups(units, pr->n_inner);
    size_t off = 0;
    P.off_at = off; off = align_up(off + 2 * (size_t)pr->n_rows * pr->n_inner, 256);
    P.off_bc = off; off = align_up(off + 2 * (size_t)pr->n_inner * pr->n_cols, 256);
    P.off_planA = off; off = align_up(off + plan_bytes(d, pr->n_rows, 14), 256);
    P.off_planB = off; off = align_up(off + plan_bytes(d, pr->n_cols, 14), 256);
    off = add_window(P, pr, off);
    P.off_part = off; off = align_up(off + sizeof(double) * (size_t)P.groups * d * b, 256);
    P.off_p = off; off = align_up(off + sizeof(double) * (size_t)d * b, 256);
    for (int op = 0; op < 2; ++op) {
      const int64_t n = op ? pr->n_cols : pr->n_rows;
      P.pair_cap[op] = pr->n_inner > 0 ? mfma_pair_cap(pr->n_rows, pr->n_cols, op) : 0;
      if (P.pair_cap[op] == 0) continue;
      P.off_plist[op] = off; off = align_up(off + sizeof(uint2) * (size_t)d * (n / 2 + 1), 256);
      P.off_pcount[op] = off; off = align_up(off + sizeof(int32_t) * (size_t)d, 256);
      P.off_pvals[op] = off;
      off = align_up(off + 2 * (size_t)d * pr->n_inner * 2 * P.pair_cap[op], 256);
    }
    P.bytes = off;
    return P;
  }
  // fused path: b_lo = 2^lb with 11 <= lb <= log2b; LDS holds the transpose
  // buffer and one staged row of each operand.
  // b_lo = 2^13 for both types: the 16-element layout (512 threads) for
  // b >= 2^13, the 32-element one below
  const int lb_max = 13;
  int lb = pr->log2b < lb_max ? pr->log2b : lb_max;
  auto fits = [&](int l) {
    const size_t v = 16 / es;
    const size_t ra = ((size_t)pr->n_rows + v) / v * v, rb = ((size_t)pr->n_cols + v) / v * v;
    // the b_lo = 2^13 kernel can also time-share one row buffer
    const size_t rows = (l == 13) ? (ra > rb ? ra : rb) : ra + rb;
    const size_t xb = ((size_t)1 << l) + ((size_t)1 << (l - 6)) + 16;
    return (xb + rows) * es <= kLdsBytes && plan_lds_bytes(pr->n_rows, l) <= kLdsBytes &&
           plan_lds_bytes(pr->n_cols, l) <= kLdsBytes;
  };
  while (lb >= 11 && !fits(lb)) --lb;
  P.fused = lb >= 11 && pr->n_rows <= 65534 && pr->n_cols <= 65534 && pr->n_rows > 0 &&
            pr->n_cols > 0 && pr->n_inner > 0;
  size_t off = 0;
  if (P.fused) {
    P.lb = lb;
    const int64_t units = (int64_t)d << (pr->log2b - lb);
    P.groups = (int)pick_groups(units, pr->n_inner);
    P.off_at = off; off = align_up(off + es * (size_t)pr->n_rows * pr->n_inner, 256);
    if (P.cdt != pr->in_dtype) {
      P.off_bc = off; off = align_up(off + es * (size_t)pr->n_inner * pr->n_cols, 256);
    }
    P.off_planA = off; off = align_up(off + plan_bytes(d, pr->n_rows, lb), 256);
    P.off_planB = off; off = align_up(off + plan_bytes(d, pr->n_cols, lb), 256);
    off = add_window(P, pr, off);
    P.off_part = off; off = align_up(off + sizeof(double) * (size_t)P.groups * d * b, 256);
  } else {
    // composed path: standalone sketch / transform / accumulate over k-chunks
    const size_t budget = (size_t)1 << 29;   // 512 MB for the two chunk buffers
    int64_t kc = (int64_t)(budget / (2 * es * (size_t)d * b));
    if (kc < 1) kc = 1;
    if (kc > pr->n_inner) kc = pr->n_inner;
    P.kc = kc < 1 ? 1 : kc;
    if (P.cdt != pr->in_dtype) {
      P.off_at = off; off = align_up(off + es * (size_t)pr->n_rows * pr->n_inner, 256);
      P.off_bc = off; off = align_up(off + es * (size_t)pr->n_inner * pr->n_cols, 256);
    }
    P.off_x = off; off = align_up(off + es * (size_t)d * P.kc * b, 256);
    P.off_y = off; off = align_up(off + es * (size_t)d * P.kc * b, 256);
    P.off_part = off; off = align_up(off + sizeof(double) * (size_t)d * b, 256);
  }
  P.off_p = off; off = align_up(off + sizeof(double) * (size_t)d * b, 256);
  P.bytes = off;
  return P;
}

// Choose each repetition's transform window and point the compress at the
// rotated tables (natural tables and no rotation when b = b_lo); the reduce
// of the partials restores the natural order.
cmm_status apply_window(const EstimatePlan& P, const cmm_problem* pr, char* ws, CompressArgs& a,
                        hipStream_t s) {
  if (!P.window) return CMM_OK;
  uint32_t* r1 = reinterpret_cast<uint32_t*>(ws + P.off_rtab1);
  uint32_t* r2 = reinterpret_cast<uint32_t*>(ws + P.off_rtab2);
  int32_t* rot = reinterpret_cast<int32_t*>(ws + P.off_rot);
  cmm_status st = launch_window(pr->tab1, pr->tab2, pr->d, pr->n_rows, pr->n_cols, pr->log2b,
                                P.lb, r1, r2, rot, s);
  if (st != CMM_OK) return st;
  a.tab1 = r1;
  a.tab2 = r2;
  return CMM_OK;
}

cmm_status run_estimate(const cmm_problem* pr, char* ws, hipStream_t s) {
  const EstimatePlan P = make_plan(pr);
  const int d = pr->d;
  const int64_t b = (int64_t)1 << pr->log2b;
  cmm_status st;
  if (pr->keys) {
    st = launch_hash(pr->keys, d, pr->n_rows, pr->n_cols, pr->log2b, pr->tab1, pr->tab2, s);
    if (st != CMM_OK) return st;
  }
  double* p = pr->p ? pr->p : reinterpret_cast<double*>(ws + P.off_p);
  if (pr->n_inner == 0 || pr->n_rows == 0 || pr->n_cols == 0) {
    if ((st = launch_zero(p, (size_t)d * b, s)) != CMM_OK) return st;
  } else if (P.mfma) {
    void* At = ws + P.off_at;
    void* Bc = ws + P.off_bc;
    st = launch_lp_copy(pr->A, pr->in_dtype, pr->n_rows, pr->n_inner, pr->lda, At, pr->compute,
                        true, s);
    if (st != CMM_OK) return st;
    st = launch_lp_copy(pr->B, pr->in_dtype, pr->n_inner, pr->n_cols, pr->ldb, Bc, pr->compute,
                        false, s);
    if (st != CMM_OK) return st;
    CompressArgs a;
    a.At = At;
    a.B = Bc;
    a.ldb = pr->n_cols;
    a.n_rows = pr->n_rows;
    a.n_cols = pr->n_cols;
    a.n_inner = pr->n_inner;
    a.tab1 = pr->tab1;
    a.tab2 = pr->tab2;
    a.planA = carve_plan(ws + P.off_planA, d, pr->n_rows, P.lb);
    a.planB = carve_plan(ws + P.off_planB, d, pr->n_cols, P.lb);
    a.d = d;
    a.log2b = pr->log2b;
    a.groups = P.groups;
    a.partial = reinterpret_cast<double*>(ws + P.off_part);
    a.ex_cap = 0;
    a.dma = 0;
    a.variant = 0;
    if ((st = apply_window(P, pr, ws, a, s)) != CMM_OK) return st;
    if ((st = launch_plan(a.tab1, d, pr->n_rows, P.lb, a.planA, s)) != CMM_OK) return st;
    if ((st = launch_plan(a.tab2, d, pr->n_cols, P.lb, a.planB, s)) != CMM_OK) return st;
    // the two-row chains merged ahead of the kernel, from the low-precision rows
    for (int op = 0; op < 2; ++op) {
      if (P.pair_cap[op] == 0) continue;
      const int64_t n = op ? pr->n_cols : pr->n_rows;
      uint2* list = reinterpret_cast<uint2*>(ws + P.off_plist[op]);
      int32_t* count = reinterpret_cast<int32_t*>(ws + P.off_pcount[op]);
      void* vals = ws + P.off_pvals[op];
      if ((st = launch_pair_list(op ? a.planB : a.planA, d, n, list, count, s)) != CMM_OK) return st;
      if ((st = launch_pair_sums(op ? Bc : At, n, pr->compute, d, pr->n_inner, n, list, count,
                                 P.pair_cap[op], vals, s)) != CMM_OK)
        return st;
      if (op) { a.pair_listB = list; a.pair_countB = count; a.pair_valsB = vals; a.pair_capB = P.pair_cap[1]; }
      else { a.pair_listA = list; a.pair_countA = count; a.pair_valsA = vals; a.pair_capA = P.pair_cap[0]; }
    }
    if ((st = launch_compress_mfma(a, pr->compute, s)) != CMM_OK) return st;
    st = launch_reduce_window(a.partial, P.groups, d, pr->log2b,
                              P.window ? reinterpret_cast<const int32_t*>(ws + P.off_rot) : nullptr,
                              p, s);
    if (st != CMM_OK) return st;
  } else if (P.fused) {
    void* At = ws + P.off_at;
    st = launch_transpose(pr->A, pr->in_dtype, pr->n_rows, pr->n_inner, pr->lda, At, P.cdt, s);
    if (st != CMM_OK) return st;
    const void* Bc = pr->B;
    int64_t ldb = pr->ldb;
    if (P.cdt != pr->in_dtype) {
      Bc = ws + P.off_bc;
      ldb = pr->n_cols;
      st = launch_convert(pr->B, pr->in_dtype, pr->n_inner, pr->n_cols, pr->ldb,
                          const_cast<void*>(Bc), P.cdt, s);
      if (st != CMM_OK) return st;
    }
    CompressArgs a;
    a.At = At;
    a.B = Bc;
    a.ldb = ldb;
    a.n_rows = pr->n_rows;
    a.n_cols = pr->n_cols;
    a.n_inner = pr->n_inner;
    a.tab1 = pr->tab1;
    a.tab2 = pr->tab2;
    a.planA = carve_plan(ws + P.off_planA, d, pr->n_rows, P.lb);
    a.planB = carve_plan(ws + P.off_planB, d, pr->n_cols, P.lb);
    a.d = d;
    a.log2b = pr->log2b;
    a.groups = P.groups;
    a.partial = reinterpret_cast<double*>(ws + P.off_part);
    a.ex_cap = 0;
    a.dma = 0;
    a.variant = 0;
    if ((st = apply_window(P, pr, ws, a, s)) != CMM_OK) return st;
    if ((st = launch_plan(a.tab1, d, pr->n_rows, P.lb, a.planA, s)) != CMM_OK) return st;
    if ((st = launch_plan(a.tab2, d, pr->n_cols, P.lb, a.planB, s)) != CMM_OK) return st;
    if ((st = launch_compress(a, P.cdt, P.lb, s)) != CMM_OK) return st;
    st = launch_reduce_window(a.partial, P.groups, d, pr->log2b,
                              P.window ? reinterpret_cast<const int32_t*>(ws + P.off_rot) : nullptr,
                              p, s);
    if (st != CMM_OK) return st;
  } else {
    const void* A = pr->A;
    const void* B = pr->B;
    int64_t lda = pr->lda, ldb = pr->ldb;
    if (P.cdt != pr->in_dtype) {
      void* Ac = ws + P.off_at;
      void* Bc = ws + P.off_bc;
      st = launch_convert(pr->A, pr->in_dtype, pr->n_rows, pr->n_inner, pr->lda, Ac, P.cdt, s);
      if (st != CMM_OK) return st;
      st = launch_convert(pr->B, pr->in_dtype, pr->n_inner, pr->n_cols, pr->ldb, Bc, P.cdt, s);
      if (st != CMM_OK) return st;
      A = Ac; B = Bc; lda = pr->n_inner; ldb = pr->n_cols;
    }
    double* p_hat = reinterpret_cast<double*>(ws + P.off_part);
    void* X = ws + P.off_x;
    void* Y = ws + P.off_y;
    if ((st = launch_zero(p_hat, (size_t)d * b, s)) != CMM_OK) return st;
    for (int64_t k0 = 0; k0 < pr->n_inner; k0 += P.kc) {
      const int64_t kc = (pr->n_inner - k0) < P.kc ? (pr->n_inner - k0) : P.kc;
      if ((st = launch_sketch(0, A, P.cdt, pr->n_rows, pr->n_inner, lda, pr->tab1, d,
                              pr->log2b, k0, kc, X, P.cdt, s)) != CMM_OK) return st;
      if ((st = launch_sketch(1, B, P.cdt, pr->n_inner, pr->n_cols, ldb, pr->tab2, d,
                              pr->log2b, k0, kc, Y, P.cdt, s)) != CMM_OK) return st;
      if ((st = launch_fwht(X, P.cdt, (int64_t)d * kc, pr->log2b, 1.0, s)) != CMM_OK) return st;
      if ((st = launch_fwht(Y, P.cdt, (int64_t)d * kc, pr->log2b, 1.0, s)) != CMM_OK) return st;
      if ((st = launch_accumulate(X, Y, P.cdt, d, kc, pr->log2b, p_hat, s)) != CMM_OK) return st;
    }
    if ((st = launch_reduce_partials(p_hat, 1, (size_t)d * b, p, s)) != CMM_OK) return st;
  }
  if (pr->n_inner > 0 && pr->n_rows > 0 && pr->n_cols > 0) {
    st = launch_fwht(p, CMM_F64, d, pr->log2b, std::ldexp(1.0, -pr->log2b), s);
    if (st != CMM_OK) return st;
  }
  if (pr->C_hat && pr->n_rows > 0 && pr->n_cols > 0)
    return launch_extract(p, pr->tab1, pr->tab2, d, pr->n_rows, pr->n_cols, pr->log2b,
                          pr->estimator, pr->C_hat, pr->out_dtype, pr->ldc, s);
  return CMM_OK;
}


// ------------------------------------------------------- backward plan
// The adjoint of the mean-over-d estimator (see k_adjoint): W scatter into
// q partials, their sum q, r = 2^-log2b H q, then per k-chunk the fused
// adjoint kernel's per-(t, u_hi) partials and their reduction into dA, dB.
struct BackwardPlan {
  cmm_dtype cdt = CMM_F64;
  int lb = 0;
  int groups = 1;
  int64_t kc = 0;        // k-chunk of the adjoint partials
  ScatterShape sh{};
  size_t off_at = 0, off_bc = 0, off_planA = 0, off_planB = 0, off_qpart = 0, off_r = 0,
         off_pa = 0, off_pb = 0;
  size_t bytes = 0;
  bool ok = false;       // a b_lo fits the LDS
};

cmm_status validate_backward(const cmm_problem* pr, const char* fn) {
  cmm_status s = validate_problem(pr, fn);
  if (s != CMM_OK) return s;
  if (pr->estimator != CMM_MEAN) {
    set_error(std::string(fn) + ": the differentiation form is the mean-over-d estimator "
              "(estimator must be CMM_MEAN)");
    return CMM_EUNSUPPORTED;
  }
  if (pr->compute != CMM_F64 && pr->compute != CMM_F32) {
    set_error(std::string(fn) + ": the adjoint computes in CMM_F64 or CMM_F32");
    return CMM_EUNSUPPORTED;
  }
  if (pr->log2b < 11) {
    set_error(std::string(fn) + ": the adjoint needs log2b >= 11");
    return CMM_EUNSUPPORTED;
  }
  if (pr->n_rows > 65534 || pr->n_cols > 65534) {
    set_error(std::string(fn) + ": the adjoint needs n_rows, n_cols <= 65534");
    return CMM_EUNSUPPORTED;
  }
  return CMM_OK;
}

BackwardPlan make_backward_plan(const cmm_problem* pr) {
  BackwardPlan P;
  P.cdt = pr->compute == CMM_F64 ? CMM_F64 : CMM_F32;
  const size_t es = dtype_size(P.cdt);
  const int d = pr->d;
  const int64_t b = (int64_t)1 << pr->log2b;
  // b_lo = 2^13 for both types (the float32 2^14 variant runs out of registers)
  const int lb_max = 13;
  int lb = pr->log2b < lb_max ? pr->log2b : lb_max;
  while (lb >= 11 && (adjoint_lds_bytes(P.cdt, lb, pr->n_rows, pr->n_cols) > kLdsBytes ||
                      plan_lds_bytes(pr->n_rows, lb) > kLdsBytes ||
                      plan_lds_bytes(pr->n_cols, lb) > kLdsBytes))
    --lb;
  P.ok = lb >= 11;
  P.lb = P.ok ? lb : 11;
  const int64_t units = (int64_t)d << (pr->log2b - P.lb);
  // adjoint partials: at most 512 MB per chunk
  const size_t per_k = es * (size_t)units * (size_t)(pr->n_rows + pr->n_cols);
  int64_t kc = per_k > 0 ? (int64_t)(((size_t)1 << 29) / per_k) : pr->n_inner;
  if (kc > pr->n_inner) kc = pr->n_inner;
  if (kc > 65535) kc = 65535;
  if (kc < 1) kc = 1;
  P.kc = kc;
  P.groups = (int)pick_groups(units, kc);
  // W scatter: LDS windows of 128 KB (2^15 float32 or 2^14 float64 sums),
  // about 512 work-groups
  P.sh.f32 = P.cdt == CMM_F32;
  const int wb_max = P.sh.f32 ? 15 : 14;
  P.sh.wb = pr->log2b < wb_max ? pr->log2b : wb_max;
  const int64_t nwin = (int64_t)1 << (pr->log2b - P.sh.wb);
  int64_t blocks = 512 / ((int64_t)d * nwin);
  if (blocks < 1) blocks = 1;
  if (blocks > pr->n_rows) blocks = pr->n_rows > 0 ? pr->n_rows : 1;
  P.sh.rows_per = pr->n_rows > 0 ? (pr->n_rows + blocks - 1) / blocks : 1;
  P.sh.blocks = pr->n_rows > 0 ? (pr->n_rows + P.sh.rows_per - 1) / P.sh.rows_per : 1;
  size_t off = 0;
  P.off_at = off; off = align_up(off + es * (size_t)pr->n_rows * pr->n_inner, 256);
  if (P.cdt != pr->in_dtype) {
    P.off_bc = off; off = align_up(off + es * (size_t)pr->n_inner * pr->n_cols, 256);
  }
  P.off_planA = off; off = align_up(off + plan_bytes(d, pr->n_rows, P.lb), 256);
  P.off_planB = off; off = align_up(off + plan_bytes(d, pr->n_cols, P.lb), 256);
  P.off_qpart = off; off = align_up(off + sizeof(double) * (size_t)P.sh.blocks * d * b, 256);
  P.off_r = off; off = align_up(off + sizeof(double) * (size_t)d * b, 256);
  P.off_pa = off; off = align_up(off + es * (size_t)units * kc * pr->n_rows, 256);
  P.off_pb = off; off = align_up(off + es * (size_t)units * kc * pr->n_cols, 256);
  P.bytes = off;
  return P;
}

cmm_status run_backward(const cmm_problem* pr, const void* W, int64_t ldw, void* dA,
                        int64_t ldda, void* dB, int64_t lddb, char* ws, hipStream_t s) {
  const BackwardPlan P = make_backward_plan(pr);
  const int d = pr->d;
  const int64_t b = (int64_t)1 << pr->log2b;
  cmm_status st;
  if (pr->keys) {
    st = launch_hash(pr->keys, d, pr->n_rows, pr->n_cols, pr->log2b, pr->tab1, pr->tab2, s);
    if (st != CMM_OK) return st;
  }
  if (pr->n_inner == 0) return CMM_OK;   // dA and dB are empty
  if (pr->n_rows == 0 || pr->n_cols == 0) {
    // C_hat is empty, so L does not depend on A or B
    if (pr->n_rows > 0 &&
        (st = launch_zero_matrix(dA, pr->in_dtype, pr->n_rows, pr->n_inner, ldda, s)) != CMM_OK)
      return st;
    if (pr->n_cols > 0 &&
        (st = launch_zero_matrix(dB, pr->in_dtype, pr->n_inner, pr->n_cols, lddb, s)) != CMM_OK)
      return st;
    return CMM_OK;
  }
  // r = 2^-log2b H q, q = bucket sums of W
  double* qpart = reinterpret_cast<double*>(ws + P.off_qpart);
  double* r = reinterpret_cast<double*>(ws + P.off_r);
  if ((st = launch_wscatter(W, pr->in_dtype, ldw, pr->tab1, pr->tab2, d, pr->n_rows, pr->n_cols,
                            pr->log2b, P.sh, qpart, s)) != CMM_OK) return st;
  if ((st = launch_reduce_partials(qpart, (int)P.sh.blocks, (size_t)d * b, r, s)) != CMM_OK)
    return st;
  if ((st = launch_fwht(r, CMM_F64, d, pr->log2b, std::ldexp(1.0, -pr->log2b), s)) != CMM_OK)
    return st;
  void* At = ws + P.off_at;
  st = launch_transpose(pr->A, pr->in_dtype, pr->n_rows, pr->n_inner, pr->lda, At, P.cdt, s);
  if (st != CMM_OK) return st;
  const void* Bc = pr->B;
  int64_t ldb = pr->ldb;
  if (P.cdt != pr->in_dtype) {
    Bc = ws + P.off_bc;
    ldb = pr->n_cols;
    st = launch_convert(pr->B, pr->in_dtype, pr->n_inner, pr->n_cols, pr->ldb,
                        const_cast<void*>(Bc), P.cdt, s);
    if (st != CMM_OK) return st;
  }
  AdjointArgs aa;
  CompressArgs& a = aa.c;
  a.ldb = ldb;
  a.n_rows = pr->n_rows;
  a.n_cols = pr->n_cols;
  a.tab1 = pr->tab1;
  a.tab2 = pr->tab2;
  a.planA = carve_plan(ws + P.off_planA, d, pr->n_rows, P.lb);
  a.planB = carve_plan(ws + P.off_planB, d, pr->n_cols, P.lb);
  a.d = d;
  a.log2b = pr->log2b;
  a.groups = P.groups;
  a.partial = nullptr;
  a.ex_cap = 0;
  a.dma = 0;
  a.variant = 0;
  aa.r = r;
  aa.scale = 1.0 / d;
  aa.partA = ws + P.off_pa;
  aa.partB = ws + P.off_pb;
  if ((st = launch_plan(pr->tab1, d, pr->n_rows, P.lb, a.planA, s)) != CMM_OK) return st;
  if ((st = launch_plan(pr->tab2, d, pr->n_cols, P.lb, a.planB, s)) != CMM_OK) return st;
  const int units = d << (pr->log2b - P.lb);
  const size_t es = dtype_size(P.cdt);
  for (int64_t kb = 0; kb < pr->n_inner; kb += P.kc) {
    const int64_t kc = (pr->n_inner - kb) < P.kc ? (pr->n_inner - kb) : P.kc;
    a.At = static_cast<const char*>(At) + es * (size_t)kb * pr->n_rows;
    a.B = static_cast<const char*>(Bc) + es * (size_t)kb * ldb;
    a.n_inner = kc;
    int64_t g = P.groups < kc ? P.groups : kc;
    while (g > 1 && (((int64_t)units * g) & 7) != 0 && g < kc) ++g;
    a.groups = (int)g;
    if ((st = launch_adjoint(aa, P.cdt, P.lb, s)) != CMM_OK) return st;
    if ((st = launch_adjoint_reduce(aa.partA, P.cdt, units, kc, pr->n_rows, dA, pr->in_dtype,
                                    ldda, kb, true, s)) != CMM_OK) return st;
    if ((st = launch_adjoint_reduce(aa.partB, P.cdt, units, kc, pr->n_cols, dB, pr->in_dtype,
                                    lddb, kb, false, s)) != CMM_OK) return st;
  }
  return CMM_OK;
}

}  // namespace
}  // namespace cmm

using namespace cmm;

extern "C" {

int cmm_abi_version(void) { return 2; }

void cmm_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  prof_clear_locked();
  g_prof_on.store(on ? 1 : 0);
}

cmm_status cmm_profile_only(const char* kernel) {
  if (kernel) {
    bool known = false;
    for (const char* k : kProfNames) known = known || std::strcmp(k, kernel) == 0;
    if (!known) return invalid(std::string("cmm_profile_only: unknown kernel name ") + kernel);
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  prof_clear_locked();
  g_prof_only = kernel ? kernel : "";
  return CMM_OK;
}

cmm_status cmm_profile_query(const char* kernel, double* total_ms, int* launches) {
  if (!kernel || !total_ms || !launches) return invalid("cmm_profile_query: null pointer");
  std::lock_guard<std::mutex> g(g_prof_mu);
  *total_ms = 0.0;
  *launches = 0;
  auto it = g_prof.find(kernel);
  if (it == g_prof.end()) return CMM_OK;
  for (auto& ev : it->second) {
    cmm_status s = hip_check(hipEventSynchronize(ev.second), "cmm_profile_query");
    if (s != CMM_OK) return s;
    float ms = 0.f;
    if ((s = hip_check(hipEventElapsedTime(&ms, ev.first, ev.second), "cmm_profile_query")) != CMM_OK)
      return s;
    *total_ms += ms;
    *launches += 1;
  }
  return CMM_OK;
}

const char* cmm_status_string(cmm_status s) {
  switch (s) {
    case CMM_OK: return "CMM_OK";
    case CMM_EINVAL: return "CMM_EINVAL";
    case CMM_ENOMEM: return "CMM_ENOMEM";
    case CMM_EHIP: return "CMM_EHIP";
    case CMM_EUNSUPPORTED: return "CMM_EUNSUPPORTED";
  }
  return "unknown status";
}

const char* cmm_last_error(void) { return g_last_error.c_str(); }

cmm_status cmm_hash(const uint64_t* keys, int d, int64_t n_rows, int64_t n_cols, int log2b,
                    uint32_t* tab1, uint32_t* tab2, void* stream) {
  cmm_status s;
  if ((s = check_d(d, "cmm_hash")) != CMM_OK) return s;
  if ((s = check_log2b(log2b, "cmm_hash")) != CMM_OK) return s;
  if (n_rows < 0 || n_cols < 0) return invalid("cmm_hash: negative size");
  if (n_rows > kMaxHashDomain || n_cols > kMaxHashDomain)
    return invalid("cmm_hash: sizes must be <= 2^32 (hash domain)");
  if (n_rows == 0 && n_cols == 0) return CMM_OK;
  if (!keys) return invalid("cmm_hash: keys is null");
  if ((n_rows > 0 && !tab1) || (n_cols > 0 && !tab2)) return invalid("cmm_hash: table is null");
  return launch_hash(keys, d, n_rows, n_cols, log2b, tab1, tab2, as_stream(stream));
}

cmm_status cmm_hash_family(cmm_hash_kind kind, const uint64_t* keys, int d, int64_t n_rows,
                           int64_t n_cols, int log2b, uint32_t* tab1, uint32_t* tab2,
                           void* stream) {
  if (kind != CMM_HASH_MULTIPLY_ADD_SHIFT && kind != CMM_HASH_MULTIPLY_SHIFT &&
      kind != CMM_HASH_TABULATION)
    return invalid("cmm_hash_family: unknown hash family");
  cmm_status s;
  if ((s = check_d(d, "cmm_hash_family")) != CMM_OK) return s;
  if ((s = check_log2b(log2b, "cmm_hash_family")) != CMM_OK) return s;
  if (n_rows < 0 || n_cols < 0) return invalid("cmm_hash_family: negative size");
  if (n_rows > kMaxHashDomain || n_cols > kMaxHashDomain)
    return invalid("cmm_hash_family: sizes must be <= 2^32 (hash domain)");
  if (n_rows == 0 && n_cols == 0) return CMM_OK;
  if (!keys) return invalid("cmm_hash_family: keys is null");
  if ((n_rows > 0 && !tab1) || (n_cols > 0 && !tab2))
    return invalid("cmm_hash_family: table is null");
  return launch_hash_family(kind, keys, d, n_rows, n_cols, log2b, tab1, tab2, as_stream(stream));
}

cmm_status cmm_sketch(int side, const void* M, cmm_dtype dtype, int64_t rows, int64_t cols,
                      int64_t ld, const uint32_t* tab, int d, int log2b, int64_t k0, int64_t kc,
                      void* out, cmm_dtype out_dtype, void* stream) {
  cmm_status s;
  if (side != 0 && side != 1) return invalid("cmm_sketch: side must be 0 (A) or 1 (B)");
  if (!is_f64_or_f32(dtype)) return invalid("cmm_sketch: dtype must be CMM_F64 or CMM_F32");
  if (!is_f64_or_f32(out_dtype))
    return invalid("cmm_sketch: out_dtype must be CMM_F64 or CMM_F32");
  if ((s = check_d(d, "cmm_sketch")) != CMM_OK) return s;
  if ((s = check_log2b(log2b, "cmm_sketch")) != CMM_OK) return s;
  if (rows < 0 || cols < 0 || k0 < 0 || kc < 0) return invalid("cmm_sketch: negative size");
  if (ld < cols) return invalid("cmm_sketch: ld < cols");
  const int64_t n_inner = side == 0 ? cols : rows;
  if (k0 + kc > n_inner) return invalid("cmm_sketch: k0 + kc exceeds the inner dimension");
  if (kc == 0) return CMM_OK;
  if (!fits_elems(rows, ld) || !fits_elems(d, kc, (int64_t)1 << log2b) ||
      !fits_elems(d, side == 0 ? rows : cols))
    return too_large("cmm_sketch", "M, out or the table");
  if (!out || !tab || (rows > 0 && cols > 0 && !M)) return invalid("cmm_sketch: null pointer");
  return launch_sketch(side, M, dtype, rows, cols, ld, tab, d, log2b, k0, kc, out, out_dtype,
                       as_stream(stream));
}

cmm_status cmm_fwht(void* x, cmm_dtype dtype, int64_t batch, int log2b, double scale,
                    void* stream) {
  cmm_status s;
  if (!is_f64_or_f32(dtype)) return invalid("cmm_fwht: dtype must be CMM_F64 or CMM_F32");
  if ((s = check_log2b(log2b, "cmm_fwht")) != CMM_OK) return s;
  if (batch < 0) return invalid("cmm_fwht: negative batch");
  int ex = 0;
  const double m = std::frexp(scale, &ex);
  if (!(scale > 0) || m != 0.5) return invalid("cmm_fwht: scale must be a positive power of two");
  if (batch == 0) return CMM_OK;
  if (!fits_elems(batch, (int64_t)1 << log2b)) return too_large("cmm_fwht", "x (batch x 2^log2b)");
  if (!x) return invalid("cmm_fwht: x is null");
  return launch_fwht(x, dtype, batch, log2b, scale, as_stream(stream));
}

cmm_status cmm_accumulate(const void* X, const void* Y, cmm_dtype dtype, int d, int64_t kc,
                          int log2b, double* p_hat, void* stream) {
  cmm_status s;
  if (!is_f64_or_f32(dtype)) return invalid("cmm_accumulate: dtype must be CMM_F64 or CMM_F32");
  if ((s = check_d(d, "cmm_accumulate")) != CMM_OK) return s;
  if ((s = check_log2b(log2b, "cmm_accumulate")) != CMM_OK) return s;
  if (kc < 0) return invalid("cmm_accumulate: negative kc");
  if (kc == 0) return CMM_OK;
  if (!fits_elems(d, kc, (int64_t)1 << log2b))
    return too_large("cmm_accumulate", "X and Y (d x kc x 2^log2b)");
  if (!X || !Y || !p_hat) return invalid("cmm_accumulate: null pointer");
  return launch_accumulate(X, Y, dtype, d, kc, log2b, p_hat, as_stream(stream));
}

cmm_status cmm_extract(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                       int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                       void* C_hat, cmm_dtype out_dtype, int64_t ldc, void* stream) {
  cmm_status s;
  if ((s = check_d(d, "cmm_extract")) != CMM_OK) return s;
  if ((s = check_log2b(log2b, "cmm_extract")) != CMM_OK) return s;
  if (estimator != CMM_MEDIAN && estimator != CMM_MEAN)
    return invalid("cmm_extract: unknown estimator");
  if (estimator == CMM_MEDIAN && d % 2 == 0)
    return invalid("cmm_extract: the median estimator needs an odd d");
  if (d > 63 && estimator == CMM_MEDIAN) {
    set_error("cmm_extract: median over more than 63 repetitions is not implemented");
    return CMM_EUNSUPPORTED;
  }
  if (!is_f64_or_f32(out_dtype)) return invalid("cmm_extract: out_dtype must be CMM_F64 or CMM_F32");
  if (n_rows < 0 || n_cols < 0) return invalid("cmm_extract: negative size");
  if (n_rows > kMaxHashDomain || n_cols > kMaxHashDomain)
    return invalid("cmm_extract: sizes must be <= 2^32");
  if (ldc < n_cols) return invalid("cmm_extract: ldc < n_cols");
  if (n_rows == 0 || n_cols == 0) return CMM_OK;
  if (!fits_elems(n_rows, ldc)) return too_large("cmm_extract", "C_hat (n_rows x ldc)");
  if (!fits_elems(d, (int64_t)1 << log2b) || !fits_elems(d, n_rows) || !fits_elems(d, n_cols))
    return too_large("cmm_extract", "p or a table");
  if (!p || !tab1 || !tab2 || !C_hat) return invalid("cmm_extract: null pointer");
  return launch_extract(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, C_hat, out_dtype,
                        ldc, as_stream(stream));
}

static cmm_status check_decompress(const double* p, const uint32_t* tab1, const uint32_t* tab2,
                                   int d, int64_t n_rows, int64_t n_cols, int log2b,
                                   cmm_estimator estimator, cmm_dtype out_dtype, const char* fn) {
  cmm_status s;
  if ((s = check_d(d, fn)) != CMM_OK) return s;
  if ((s = check_log2b(log2b, fn)) != CMM_OK) return s;
  if (estimator != CMM_MEDIAN && estimator != CMM_MEAN)
    return invalid(std::string(fn) + ": unknown estimator");
  if (estimator == CMM_MEDIAN && d % 2 == 0)
    return invalid(std::string(fn) + ": the median estimator needs an odd d");
  if (d > 63 && estimator == CMM_MEDIAN) {
    set_error(std::string(fn) + ": median over more than 63 repetitions is not implemented");
    return CMM_EUNSUPPORTED;
  }
  if (!is_f64_or_f32(out_dtype)) return invalid(std::string(fn) + ": out_dtype must be CMM_F64 or CMM_F32");
  if (n_rows < 0 || n_cols < 0) return invalid(std::string(fn) + ": negative size");
  if (n_rows > kMaxHashDomain || n_cols > kMaxHashDomain)
    return invalid(std::string(fn) + ": sizes must be <= 2^32");
  if ((n_rows > 0 && n_cols > 0) && (!p || !tab1 || !tab2))
    return invalid(std::string(fn) + ": null pointer");
  if (!fits_elems(d, (int64_t)1 << log2b) || !fits_elems(d, n_rows) || !fits_elems(d, n_cols))
    return too_large(fn, "p or a table");
  return CMM_OK;
}

cmm_status cmm_extract_entries(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                               int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                               const int64_t* rows, const int64_t* cols, int64_t count, void* out,
                               cmm_dtype out_dtype, void* stream) {
  cmm_status s = check_decompress(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, out_dtype,
                                  "cmm_extract_entries");
  if (s != CMM_OK) return s;
  if (count < 0) return invalid("cmm_extract_entries: negative count");
  if (count == 0) return CMM_OK;
  if (!fits_elems(count, 1)) return too_large("cmm_extract_entries", "the entry list");
  if (!rows || !cols || !out) return invalid("cmm_extract_entries: null pointer");
  return launch_extract_entries(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, rows, cols,
                                count, out, out_dtype, as_stream(stream));
}

cmm_status cmm_extract_heavy(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                             int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                             double threshold, int64_t* out_rows, int64_t* out_cols,
                             void* out_vals, cmm_dtype out_dtype, int64_t capacity,
                             int64_t* count, void* stream) {
  cmm_status s = check_decompress(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, out_dtype,
                                  "cmm_extract_heavy");
  if (s != CMM_OK) return s;
  if (!count) return invalid("cmm_extract_heavy: count is null");
  if (capacity < 0) return invalid("cmm_extract_heavy: negative capacity");
  if (capacity > 0 && (!out_rows || !out_cols || !out_vals))
    return invalid("cmm_extract_heavy: null output list");
  if (!(threshold >= 0.0)) return invalid("cmm_extract_heavy: threshold must be >= 0 (not NaN)");
  if (!fits_elems(capacity, 1) || !fits_elems(n_rows, n_cols))
    return too_large("cmm_extract_heavy", "the output list or the scanned block");
  return launch_extract_heavy(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, threshold,
                              out_rows, out_cols, out_vals, out_dtype, capacity, count,
                              as_stream(stream));
}

cmm_status cmm_topk_workspace_size(int64_t k, size_t* bytes) {
  if (!bytes) return invalid("cmm_topk_workspace_size: bytes is null");
  if (k < 0) return invalid("cmm_topk_workspace_size: negative k");
  if (k > kMaxTopK) {
    set_error("cmm_topk_workspace_size: k above 2^31 - 2^15 is not supported");
    return CMM_EUNSUPPORTED;
  }
  return topk_workspace_bytes(k, bytes);
}

cmm_status cmm_extract_topk(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                            int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                            int64_t k, int64_t* out_rows, int64_t* out_cols, void* out_vals,
                            cmm_dtype out_dtype, void* workspace, size_t workspace_bytes,
                            void* stream) {
  const char* fn = "cmm_extract_topk";
  cmm_status s = check_decompress(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, out_dtype, fn);
  if (s != CMM_OK) return s;
  if (k < 0) return invalid("cmm_extract_topk: negative k");
  if (k == 0) return CMM_OK;
  if (!fits_elems(n_rows, n_cols)) return too_large(fn, "the scanned block (n_rows x n_cols)");
  if (k > n_rows * n_cols) return invalid("cmm_extract_topk: k exceeds n_rows * n_cols");
  if (k > kMaxTopK) {
    set_error("cmm_extract_topk: k above 2^31 - 2^15 is not supported");
    return CMM_EUNSUPPORTED;
  }
  if (!out_rows || !out_cols || !out_vals) return invalid("cmm_extract_topk: null output");
  if (!workspace) return invalid("cmm_extract_topk: workspace is null");
  return launch_extract_topk(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, k, out_rows,
                             out_cols, out_vals, out_dtype, workspace, workspace_bytes,
                             as_stream(stream));
}

cmm_status cmm_extract_reps(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                            int64_t n_rows, int64_t n_cols, int log2b, const int64_t* rows,
                            const int64_t* cols, int64_t count, void* out, cmm_dtype out_dtype,
                            void* stream) {
  // the estimator plays no part: MEAN lets every d through the shared checks
  cmm_status s = check_decompress(p, tab1, tab2, d, n_rows, n_cols, log2b, CMM_MEAN, out_dtype,
                                  "cmm_extract_reps");
  if (s != CMM_OK) return s;
  if (count < 0) return invalid("cmm_extract_reps: negative count");
  if (count == 0) return CMM_OK;
  if (!fits_elems(d, count)) return too_large("cmm_extract_reps", "out (d x count)");
  if (!rows || !cols || !out) return invalid("cmm_extract_reps: null pointer");
  return launch_extract_reps(p, tab1, tab2, d, n_rows, n_cols, log2b, rows, cols, count, out,
                             out_dtype, as_stream(stream));
}

cmm_status cmm_correctness_counts(const void* C_hat, cmm_dtype C_hat_dtype, int64_t ldh,
                                  const double* C, int64_t ldc, int64_t n_rows, int64_t n_cols,
                                  const int64_t* big_rows, const int64_t* big_cols, int64_t n_big,
                                  double threshold, double tolerance, int64_t* counts,
                                  void* stream) {
  const char* fn = "cmm_correctness_counts";
  if (!is_f64_or_f32(C_hat_dtype))
    return invalid(std::string(fn) + ": C_hat_dtype must be CMM_F64 or CMM_F32");
  if (n_rows < 0 || n_cols < 0 || n_big < 0) return invalid(std::string(fn) + ": negative size");
  if (n_rows > 0 && n_cols > 0 && (ldh < n_cols || ldc < n_cols))
    return invalid(std::string(fn) + ": leading dimension < n_cols");
  if (!(threshold >= 0.0) || !(tolerance >= 0.0))
    return invalid(std::string(fn) + ": threshold and tolerance must be >= 0 (not NaN)");
  if (!counts) return invalid(std::string(fn) + ": counts is null");
  if (n_rows > 0 && n_cols > 0 && (!fits_elems(n_rows, ldh) || !fits_elems(n_rows, ldc)))
    return too_large(fn, "C_hat or C (n_rows x leading dimension)");
  if (!fits_elems(n_big, 1)) return too_large(fn, "the big-entry list");
  if (n_rows > 0 && n_cols > 0 && (!C_hat || !C)) return invalid(std::string(fn) + ": null matrix");
  if (n_big > 0 && (!big_rows || !big_cols)) return invalid(std::string(fn) + ": null big list");
  return launch_correctness(C_hat, C_hat_dtype, ldh, C, ldc, n_rows, n_cols, big_rows, big_cols,
                            n_big, threshold, tolerance, counts, as_stream(stream));
}

}  // extern "C"

// ---------------------------------------------------- Pagh's FFT form
namespace cmm {
namespace {

struct FftPlan {
  bool fused = false;
  int groups = 1;     // k-ranges of the fused kernel
  int64_t kc = 1;     // k-chunk of the staged path
  size_t off_x = 0, off_y = 0, off_z = 0, off_z2 = 0, off_P = 0, off_Q = 0, off_p = 0;
  size_t off_at = 0, off_planA = 0, off_planB = 0, off_part = 0;
  size_t bytes = 0;
};

// Fused path: A^T, the bucket plans (b_lo = 2^12), complex partials
// [groups][d][b]; staged path: sketches X, Y (float64 [d][kc][b]), their
// packed complex sequence and its transform ([d][kc][b] complex each), the
// chunk keeping these buffers near 1 GiB.  Both: the transformed
// accumulator P and its inverse ([d][b] complex each), and p when the
// caller passes none.
FftPlan make_fft_plan(const cmm_problem* pr) {
  FftPlan P;
  const size_t d = (size_t)pr->d, b = (size_t)1 << pr->log2b;
  size_t off = 0;
  P.fused = pr->n_inner > 0 && compress_fft_supported(pr->n_rows, pr->n_cols, pr->log2b) &&
            plan_lds_bytes(pr->n_rows, 12) <= 160 * 1024 &&
            plan_lds_bytes(pr->n_cols, 12) <= 160 * 1024;
  if (P.fused) {
    const int64_t units = (int64_t)d * (((int64_t)1 << (pr->log2b - 12)) / 2 + 1);
    P.groups = (int)pick_groups(units, pr->n_inner);
    P.off_at = off; off = align_up(off + 8 * (size_t)pr->n_rows * pr->n_inner, 256);
    P.off_planA = off; off = align_up(off + plan_bytes(pr->d, pr->n_rows, 12), 256);
    P.off_planB = off; off = align_up(off + plan_bytes(pr->d, pr->n_cols, 12), 256);
    P.off_part = off; off = align_up(off + 16 * (size_t)P.groups * d * b, 256);
  } else {
    const size_t per_k = 48 * d * b;
    int64_t kc = (int64_t)((size_t)1 << 30) / (int64_t)per_k;
    if (kc > pr->n_inner) kc = pr->n_inner;
    if (kc < 1) kc = 1;
    P.kc = kc;
    P.off_x = off; off = align_up(off + 8 * d * kc * b, 256);
    P.off_y = off; off = align_up(off + 8 * d * kc * b, 256);
    P.off_z = off; off = align_up(off + 16 * d * kc * b, 256);
    P.off_z2 = off; off = align_up(off + 16 * d * kc * b, 256);
  }
  P.off_P = off; off = align_up(off + 16 * d * b, 256);
  P.off_Q = off; off = align_up(off + 16 * d * b, 256);
  P.off_p = off; off = align_up(off + 8 * d * b, 256);
  P.bytes = off;
  return P;
}

cmm_status validate_fft_problem(const cmm_problem* pr, const char* fn) {
  cmm_status s = validate_problem(pr, fn);
  if (s != CMM_OK) return s;
  if (pr->compute != CMM_F64 || pr->in_dtype != CMM_F64) {
    set_error(std::string(fn) + ": the FFT form runs in float64 only (compute and in_dtype CMM_F64)");
    return CMM_EUNSUPPORTED;
  }
  if (pr->log2b > kMaxFftLog2) {
    set_error(std::string(fn) + ": the FFT form's transform supports log2b <= 24");
    return CMM_EUNSUPPORTED;
  }
  if (pr->d > 63 && pr->estimator == CMM_MEDIAN && pr->C_hat) {
    set_error(std::string(fn) + ": median over more than 63 repetitions is not implemented");
    return CMM_EUNSUPPORTED;
  }
  return CMM_OK;
}

cmm_status run_estimate_fft(const cmm_problem* pr, char* ws, hipStream_t s) {
  const FftPlan P = make_fft_plan(pr);
  const int d = pr->d;
  const int64_t b = (int64_t)1 << pr->log2b;
  cmm_status st;
  if (pr->keys) {
    st = launch_hash(pr->keys, d, pr->n_rows, pr->n_cols, pr->log2b, pr->tab1, pr->tab2, s);
    if (st != CMM_OK) return st;
  }
  double* p = pr->p ? pr->p : reinterpret_cast<double*>(ws + P.off_p);
  if (pr->n_inner == 0 || pr->n_rows == 0 || pr->n_cols == 0) {
    if ((st = launch_zero(p, (size_t)d * b, s)) != CMM_OK) return st;
  } else {
    void* Pacc = ws + P.off_P;
    if (P.fused) {
      void* At = ws + P.off_at;
      st = launch_transpose(pr->A, pr->in_dtype, pr->n_rows, pr->n_inner, pr->lda, At, CMM_F64, s);
      if (st != CMM_OK) return st;
      CompressArgs a;
      a.At = At;
      a.B = pr->B;
      a.ldb = pr->ldb;
      a.n_rows = pr->n_rows;
      a.n_cols = pr->n_cols;
      a.n_inner = pr->n_inner;
      a.tab1 = pr->tab1;
      a.tab2 = pr->tab2;
      a.planA = carve_plan(ws + P.off_planA, d, pr->n_rows, 12);
      a.planB = carve_plan(ws + P.off_planB, d, pr->n_cols, 12);
      a.d = d;
      a.log2b = pr->log2b;
      a.groups = P.groups;
      a.partial = reinterpret_cast<double*>(ws + P.off_part);
      a.ex_cap = 0;
      a.dma = 0;
      a.variant = 0;
      if ((st = launch_plan(pr->tab1, d, pr->n_rows, 12, a.planA, s)) != CMM_OK) return st;
      if ((st = launch_plan(pr->tab2, d, pr->n_cols, 12, a.planB, s)) != CMM_OK) return st;
      if ((st = launch_compress_fft(a, s)) != CMM_OK) return st;
      st = launch_reduce_fft_partials(a.partial, P.groups, d, pr->log2b, Pacc, s);
      if (st != CMM_OK) return st;
    }
    double* X = reinterpret_cast<double*>(ws + P.off_x);
    double* Y = reinterpret_cast<double*>(ws + P.off_y);
    void* Z = ws + P.off_z;
    void* Z2 = ws + P.off_z2;
    if (!P.fused && (st = launch_zero_complex(Pacc, (size_t)d * b, s)) != CMM_OK) return st;
    for (int64_t k0 = 0; !P.fused && k0 < pr->n_inner; k0 += P.kc) {
      const int64_t kc = (pr->n_inner - k0) < P.kc ? (pr->n_inner - k0) : P.kc;
      if ((st = launch_sketch(0, pr->A, CMM_F64, pr->n_rows, pr->n_inner, pr->lda, pr->tab1, d,
                              pr->log2b, k0, kc, X, CMM_F64, s)) != CMM_OK) return st;
      if ((st = launch_sketch(1, pr->B, CMM_F64, pr->n_inner, pr->n_cols, pr->ldb, pr->tab2, d,
                              pr->log2b, k0, kc, Y, CMM_F64, s)) != CMM_OK) return st;
      if ((st = launch_pack(X, Y, Z, (size_t)d * kc * b, s)) != CMM_OK) return st;
      if ((st = launch_fft(Z, Z2, (int64_t)d * kc, pr->log2b, 0, 1.0, s)) != CMM_OK) return st;
      if ((st = launch_accumulate_cyclic(Z2, d, kc, pr->log2b, Pacc, s)) != CMM_OK) return st;
    }
    void* Q = ws + P.off_Q;
    st = launch_fft(Pacc, Q, d, pr->log2b, 1, std::ldexp(1.0, -pr->log2b), s);
    if (st != CMM_OK) return st;
    if ((st = launch_real_part(Q, p, (size_t)d * b, s)) != CMM_OK) return st;
  }
  if (pr->C_hat && pr->n_rows > 0 && pr->n_cols > 0)
    return launch_extract(p, pr->tab1, pr->tab2, d, pr->n_rows, pr->n_cols, pr->log2b,
                          pr->estimator, pr->C_hat, pr->out_dtype, pr->ldc, s, true);
  return CMM_OK;
}

}  // namespace
}  // namespace cmm

extern "C" {

cmm_status cmm_fft(const void* in, void* out, int64_t batch, int log2n, int inverse, double scale,
                   void* stream) {
  if (log2n < 1 || log2n > 24) return invalid("cmm_fft: log2n must be in [1, 24]");
  if (batch < 0) return invalid("cmm_fft: negative batch");
  if (inverse != 0 && inverse != 1) return invalid("cmm_fft: inverse must be 0 or 1");
  if (!std::isfinite(scale)) return invalid("cmm_fft: scale must be finite");
  if (batch == 0) return CMM_OK;
  if (!fits_elems(batch, (int64_t)1 << log2n)) return too_large("cmm_fft", "x (batch x 2^log2n)");
  if (!in || !out) return invalid("cmm_fft: null pointer");
  if (log2n > 12 && in == out) return invalid("cmm_fft: in and out must differ when log2n > 12");
  return launch_fft(in, out, batch, log2n, inverse, scale, as_stream(stream));
}

cmm_status cmm_fft_workspace_size(const cmm_problem* prob, size_t* bytes) {
  cmm_status s = validate_fft_problem(prob, "cmm_fft_workspace_size");
  if (s != CMM_OK) return s;
  if (!bytes) return invalid("cmm_fft_workspace_size: bytes is null");
  *bytes = make_fft_plan(prob).bytes;
  return CMM_OK;
}

cmm_status cmm_estimate_fft(const cmm_problem* prob, void* workspace, size_t workspace_bytes,
                            void* stream) {
  cmm_status s = validate_fft_problem(prob, "cmm_estimate_fft");
  if (s != CMM_OK) return s;
  const FftPlan P = make_fft_plan(prob);
  if (workspace_bytes < P.bytes) {
    set_error("cmm_estimate_fft: workspace of " + std::to_string(workspace_bytes) +
              " bytes, need " + std::to_string(P.bytes));
    return CMM_ENOMEM;
  }
  if (!workspace) return invalid("cmm_estimate_fft: workspace is null");
  return run_estimate_fft(prob, static_cast<char*>(workspace), as_stream(stream));
}

cmm_status cmm_extract_cyclic(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                              int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                              void* C_hat, cmm_dtype out_dtype, int64_t ldc, void* stream) {
  cmm_status s = check_decompress(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, out_dtype,
                                  "cmm_extract_cyclic");
  if (s != CMM_OK) return s;
  if (ldc < n_cols) return invalid("cmm_extract_cyclic: ldc < n_cols");
  if (n_rows == 0 || n_cols == 0) return CMM_OK;
  if (!fits_elems(n_rows, ldc)) return too_large("cmm_extract_cyclic", "C_hat (n_rows x ldc)");
  if (!C_hat) return invalid("cmm_extract_cyclic: C_hat is null");
  return launch_extract(p, tab1, tab2, d, n_rows, n_cols, log2b, estimator, C_hat, out_dtype, ldc,
                        as_stream(stream), true);
}

}  // extern "C"

// ------------------------------------------- estimate without allocation
// Scratch of cmm_estimate_static: a file-scope device array, one copy per
// device, held until the process ends.  In host code its name stands for a
// host-side shadow, not device memory: kernels only ever receive the
// per-device address hipGetSymbolAddress returns (taken once per device,
// with that device current, on the entry point's first call there).
namespace {
static __device__ __align__(256) unsigned char scratch[CMM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

cmm_status static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "cmm_estimate_static: current device");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("cmm_estimate_static: device ordinal out of range");
    return CMM_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "cmm_estimate_static: scratch address");
    if (!ptr) {
      set_error("cmm_estimate_static: no scratch address on this device");
      return CMM_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CMM_OK;
}

// Kernel timing off on this thread for the lifetime of the guard.
struct NoProfiling {
  NoProfiling() { t_prof_suppressed = true; }
  ~NoProfiling() { t_prof_suppressed = false; }
};
}  // namespace

extern "C" {

cmm_status cmm_estimate_static(const cmm_problem* prob, void* stream) {
  cmm_status s = validate_problem(prob, "cmm_estimate_static");
  if (s != CMM_OK) return s;
  if (prob->d > 63 && prob->estimator == CMM_MEDIAN && prob->C_hat) {
    set_error("cmm_estimate_static: median over more than 63 repetitions is not implemented");
    return CMM_EUNSUPPORTED;
  }
  const EstimatePlan P = make_plan(prob);
  if (P.bytes > (size_t)CMM_STATIC_SCRATCH_BYTES) {
    set_error("cmm_estimate_static: the problem needs " + std::to_string(P.bytes) +
              " bytes of scratch, more than the " +
              std::to_string((size_t)CMM_STATIC_SCRATCH_BYTES) +
              " of the static array; use cmm_estimate with a workspace");
    return CMM_EUNSUPPORTED;
  }
  void* ws = nullptr;
  if ((s = static_scratch(&ws)) != CMM_OK) return s;
  NoProfiling guard;
  return run_estimate(prob, static_cast<char*>(ws), as_stream(stream));
}

cmm_status cmm_workspace_size(const cmm_problem* prob, size_t* bytes) {
  cmm_status s = validate_problem(prob, "cmm_workspace_size");
  if (s != CMM_OK) return s;
  if (!bytes) return invalid("cmm_workspace_size: bytes is null");
  *bytes = make_plan(prob).bytes;
  return CMM_OK;
}

cmm_status cmm_estimate(const cmm_problem* prob, void* workspace, size_t workspace_bytes,
                        void* stream) {
  cmm_status s = validate_problem(prob, "cmm_estimate");
  if (s != CMM_OK) return s;
  if (prob->d > 63 && prob->estimator == CMM_MEDIAN && prob->C_hat) {
    set_error("cmm_estimate: median over more than 63 repetitions is not implemented");
    return CMM_EUNSUPPORTED;
  }
  const EstimatePlan P = make_plan(prob);
  if (workspace_bytes < P.bytes) {
    set_error("cmm_estimate: workspace of " + std::to_string(workspace_bytes) +
              " bytes, need " + std::to_string(P.bytes));
    return CMM_ENOMEM;
  }
  if (!workspace && P.bytes > 0) return invalid("cmm_estimate: workspace is null");
  return run_estimate(prob, static_cast<char*>(workspace), as_stream(stream));
}

cmm_status cmm_backward_workspace_size(const cmm_problem* prob, size_t* bytes) {
  cmm_status s = validate_backward(prob, "cmm_backward_workspace_size");
  if (s != CMM_OK) return s;
  if (!bytes) return invalid("cmm_backward_workspace_size: bytes is null");
  const BackwardPlan P = make_backward_plan(prob);
  if (!P.ok) {
    set_error("cmm_backward_workspace_size: the rows do not fit the adjoint kernel's LDS");
    return CMM_EUNSUPPORTED;
  }
  *bytes = P.bytes;
  return CMM_OK;
}

cmm_status cmm_estimate_backward(const cmm_problem* prob, const void* W, int64_t ldw, void* dA,
                                 int64_t ldda, void* dB, int64_t lddb, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  cmm_status s = validate_backward(prob, "cmm_estimate_backward");
  if (s != CMM_OK) return s;
  const cmm_problem* pr = prob;
  if (pr->n_rows > 0 && pr->n_cols > 0 && !W) return invalid("cmm_estimate_backward: W is null");
  if (pr->n_rows > 0 && ldw < pr->n_cols) return invalid("cmm_estimate_backward: ldw < n_cols");
  if (pr->n_rows > 0 && ldda < pr->n_inner)
    return invalid("cmm_estimate_backward: ldda < n_inner");
  if (pr->n_inner > 0 && lddb < pr->n_cols)
    return invalid("cmm_estimate_backward: lddb < n_cols");
  if ((pr->n_rows > 0 && pr->n_inner > 0 && !dA) || (pr->n_inner > 0 && pr->n_cols > 0 && !dB))
    return invalid("cmm_estimate_backward: dA / dB is null");
  if (!fits_elems(pr->n_rows, ldw) || !fits_elems(pr->n_rows, ldda) ||
      !fits_elems(pr->n_inner, lddb))
    return too_large("cmm_estimate_backward", "W, dA or dB");
  const BackwardPlan P = make_backward_plan(pr);
  if (!P.ok) {
    set_error("cmm_estimate_backward: the rows do not fit the adjoint kernel's LDS");
    return CMM_EUNSUPPORTED;
  }
  if (workspace_bytes < P.bytes) {
    set_error("cmm_estimate_backward: workspace of " + std::to_string(workspace_bytes) +
              " bytes, need " + std::to_string(P.bytes));
    return CMM_ENOMEM;
  }
  if (!workspace && P.bytes > 0) return invalid("cmm_estimate_backward: workspace is null");
  return run_backward(pr, W, ldw, dA, ldda, dB, lddb, static_cast<char*>(workspace),
                      as_stream(stream));
}

}  // extern "C"
