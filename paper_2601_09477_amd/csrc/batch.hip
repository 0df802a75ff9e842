// Batched form: many independent compressed products (uneven sizes) with
// their Compress work in one persistent launch, and a project-written
// autotuner that picks the launch's tile (b_lo), k-range per work item,
// work-groups per compute unit and item order by timing candidates.
//
// A batch is planned once (cmm_batch_create).  Every work item -- one
// (problem, repetition t, slice u_hi, k-range) -- has about the same cost
// (a b_lo-point transform per k plus a sketch of the two input rows), so
// a shared queue balances problems of different sizes without a schedule.
// The item table and the per-problem descriptors are built on the host
// once per configuration into pinned memory; each call copies them into
// the workspace with an asynchronous copy, so a captured graph replays the
// same copy.  Workspace buffers are addressed by offset, which keeps the
// table independent of where the workspace lives.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr size_t kLds = 160 * 1024;
constexpr int kKGrains[] = {32, 64, 128, 256};

struct BatchConfig {
  int lb = 13;         // log2 b_lo of the fused kernel
  int kgrain = 64;     // inner indices per work item
  int wg_per_cu = 1;   // LDS share: 160 KB / wg_per_cu per work-group
  int order = 0;       // 0: largest problems first; 1: round robin over problems
  int radix = 16;      // elements per thread: 16 (b_lo = 2^13) or 32
  bool operator<(const BatchConfig& o) const {
    return std::tie(lb, kgrain, wg_per_cu, order, radix) <
           std::tie(o.lb, o.kgrain, o.wg_per_cu, o.order, o.radix);
  }
};

size_t lds_base(cmm_dtype dt, const BatchConfig& c, int64_t n_rows, int64_t n_cols) {
  return c.radix == 16 ? compress16_lds_base(dt, n_rows, n_cols)
                       : compress_lds_base(dt, c.lb, n_rows, n_cols);
}

struct BatchLayout {
  bool ok = false;
  std::vector<BatchPair> pairs;
  std::vector<BatchItem> items;
  std::vector<int64_t> off_p;       // workspace p per problem (-1: the caller's)
  size_t off_desc = 0, off_items = 0, off_queue = 0, desc_bytes = 0;
  size_t lds = 0;
  bool desc = false;                // 16-element layout with descriptor fix-ups
  size_t bytes = 0;
};

bool active(const cmm_problem& p) { return p.n_rows > 0 && p.n_cols > 0 && p.n_inner > 0; }

}  // namespace
}  // namespace cmm

using namespace cmm;

struct cmm_batch {
  std::vector<cmm_problem> probs;
  cmm_dtype cdt = CMM_F32;
  std::vector<int> lbs;             // b_lo candidates valid for every problem
  BatchConfig cfg;
  int tuned = 0;                    // 0 default, 1 autotuned, 2 from the cache, 3 set
  size_t ws_bytes = 0;              // maximum over all candidate configurations
  std::map<BatchConfig, BatchLayout> layouts;
  std::map<BatchConfig, void*> staging;   // pinned copies of the descriptor tables
  ~cmm_batch() {
    for (auto& kv : staging) (void)hipHostFree(kv.second);
  }
};

namespace cmm {
namespace {

BatchLayout make_layout(const cmm_batch& b, const BatchConfig& c) {
  BatchLayout L;
  const size_t es = dtype_size(b.cdt);
  const int V = (int)(16 / es);
  // dynamic LDS per work-group (the kernel's own queue slot takes a few bytes more)
  const size_t lds_cap = (kLds - 256) / (size_t)c.wg_per_cu / 16 * 16;
  const int n = (int)b.probs.size();
  L.pairs.resize(n);
  L.off_p.assign(n, -1);
  // work per item is about equal, so problems are ordered by item count
  std::vector<int64_t> groups(n, 0), units(n, 0);
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    const cmm_problem& p = b.probs[i];
    if (!active(p)) continue;
    if (p.log2b < c.lb || (c.radix == 16 && c.lb != 13)) return L;
    groups[i] = (p.n_inner + c.kgrain - 1) / c.kgrain;
    units[i] = (int64_t)p.d << (p.log2b - c.lb);
    const size_t base = lds_base(b.cdt, c, p.n_rows, p.n_cols);
    if (base > lds_cap) return L;
    const size_t want = base + sizeof(uint2) * (size_t)(p.n_rows + p.n_cols + (p.n_rows + p.n_cols + 8) / 2);
    lds = std::max(lds, std::min(want, lds_cap));
  }
  // descriptor fix-ups (faster than walking the chains) when every
  // problem's rows, spare elements and descriptors fit the LDS share
  if (c.radix == 16) {
    bool desc = true;
    size_t dl = 0;
    for (int i = 0; i < n && desc; ++i) {
      const cmm_problem& p = b.probs[i];
      if (!active(p)) continue;
      const size_t need = compress16_desc_lds(b.cdt, p.n_rows, p.n_cols);
      desc = need <= lds_cap && p.n_rows + 64 < 32768 && p.n_cols + 64 < 32768;
      dl = std::max(dl, need);
    }
    // room for a partial third descriptor slot of up to 512 positions
    if (desc) {
      L.desc = true;
      lds = std::min(lds_cap, dl + sizeof(uint32_t) * 3 * 2 * 512);
    }
  }
  L.lds = lds;
  // items
  std::vector<int> idx;
  for (int i = 0; i < n; ++i)
    if (active(b.probs[i])) idx.push_back(i);
  if (c.order == 0) {
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      return groups[x] * units[x] > groups[y] * units[y];
    });
    for (int i : idx)
      for (int64_t g = 0; g < groups[i]; ++g)
        for (int64_t u = 0; u < units[i]; ++u)
          L.items.push_back(BatchItem{(uint32_t)i, (uint32_t)u, (uint32_t)g});
  } else {
    std::vector<int64_t> next(n, 0);
    bool more = true;
    while (more) {
      more = false;
      for (int i : idx) {
        const int64_t total = groups[i] * units[i];
        if (next[i] < total) {
          const int64_t q = next[i]++;
          L.items.push_back(BatchItem{(uint32_t)i, (uint32_t)(q % units[i]), (uint32_t)(q / units[i])});
          more = true;
        }
      }
    }
  }
  if (L.items.size() > (size_t)0x7FFFFFFF) return L;
  // workspace
  size_t off = 0;
  L.off_desc = off; off = align_up(off + sizeof(BatchPair) * (size_t)n, 256);
  L.off_items = off; off = align_up(off + sizeof(BatchItem) * L.items.size(), 256);
  L.desc_bytes = off;
  L.off_queue = off; off = align_up(off + sizeof(double), 256);
  for (int i = 0; i < n; ++i) {
    const cmm_problem& p = b.probs[i];
    BatchPair& bp = L.pairs[i];
    bp = BatchPair{};
    bp.bc = -1;
    bp.rtab1 = bp.rtab2 = bp.rot = -1;
    bp.d = p.d;
    bp.log2b = p.log2b;
    bp.n_rows = p.n_rows;
    bp.n_cols = p.n_cols;
    bp.n_inner = p.n_inner;
    bp.tab1 = p.tab1;
    bp.tab2 = p.tab2;
    const size_t blen = (size_t)1 << p.log2b;
    if (!p.p) { L.off_p[i] = (int64_t)off; off = align_up(off + sizeof(double) * p.d * blen, 256); }
    if (!active(p)) continue;
    bp.groups = (int)groups[i];
    bp.at = (int64_t)off; off = align_up(off + es * (size_t)p.n_rows * p.n_inner, 256);
    bp.B = p.B;
    bp.ldb = p.ldb;
    if (p.in_dtype != b.cdt) {
      bp.bc = (int64_t)off; off = align_up(off + es * (size_t)p.n_inner * p.n_cols, 256);
      bp.ldb = p.n_cols;
    }
    bp.planA = (int64_t)off; off = align_up(off + plan_bytes(p.d, p.n_rows, c.lb), 256);
    bp.planB = (int64_t)off; off = align_up(off + plan_bytes(p.d, p.n_cols, c.lb), 256);
    if (p.log2b > c.lb) {   // transform windows, as in the single-problem path
      bp.rtab1 = (int64_t)off; off = align_up(off + sizeof(uint32_t) * (size_t)p.d * p.n_rows, 256);
      bp.rtab2 = (int64_t)off; off = align_up(off + sizeof(uint32_t) * (size_t)p.d * p.n_cols, 256);
      bp.rot = (int64_t)off; off = align_up(off + sizeof(int32_t) * (size_t)p.d, 256);
    }
    bp.partial = (int64_t)off; off = align_up(off + sizeof(double) * groups[i] * p.d * blen, 256);
    const size_t base = lds_base(b.cdt, c, p.n_rows, p.n_cols);
    int64_t cap = (int64_t)((lds - std::min(lds, base)) / sizeof(uint2));
    bp.ex_cap = L.desc ? 0 : std::min<int64_t>(cap, p.n_rows + p.n_cols);
    bp.ovf16 = 0;
    if (L.desc) {
      const size_t need = compress16_desc_lds(b.cdt, p.n_rows, p.n_cols);
      const size_t extra = lds > need ? (lds - need) / (sizeof(uint32_t) * 3 * 2) : 0;
      bp.ovf16 = (int)std::min<size_t>(extra, 512);
    }
    // 16-byte row copies: the workspace is 256-byte aligned, the caller's B is checked here
    const bool b_ok = bp.bc >= 0 || ((uintptr_t)p.B % 16 == 0);
    bp.dma = (p.n_rows % V == 0) && (p.n_cols % V == 0) && (bp.ldb % V == 0) && b_ok;
  }
  L.bytes = off;
  L.ok = true;
  return L;
}

const BatchLayout& layout_of(cmm_batch& b, const BatchConfig& c) {
  auto it = b.layouts.find(c);
  if (it != b.layouts.end()) return it->second;
  return b.layouts.emplace(c, make_layout(b, c)).first->second;
}

std::vector<BatchConfig> candidates(const cmm_batch& b) {
  std::vector<BatchConfig> out;
  for (int lb : b.lbs)
    for (int radix : {16, 32})
      if (radix == 32 || lb == 13)
        for (int kg : kKGrains)
          for (int wg = 1; wg <= 2; ++wg)
            for (int ord = 0; ord <= 1; ++ord) out.push_back(BatchConfig{lb, kg, wg, ord, radix});
  return out;
}

cmm_status staging_of(cmm_batch& b, const BatchConfig& c, void** out) {
  auto it = b.staging.find(c);
  if (it != b.staging.end()) { *out = it->second; return CMM_OK; }
  const BatchLayout& L = layout_of(b, c);
  void* h = nullptr;
  cmm_status st = hip_check(hipHostMalloc(&h, std::max<size_t>(L.desc_bytes, 256), hipHostMallocDefault),
                            "batch: pinned descriptor table");
  if (st != CMM_OK) return st;
  char* hc = static_cast<char*>(h);
  std::memcpy(hc + L.off_desc, L.pairs.data(), sizeof(BatchPair) * L.pairs.size());
  std::memcpy(hc + L.off_items, L.items.data(), sizeof(BatchItem) * L.items.size());
  b.staging[c] = h;
  *out = h;
  return CMM_OK;
}

int compute_units() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 256;
  return cus;
}

// Per-problem work before Compress: tables, A^T (and B) in the compute
// type, the bucket plans for b_lo = 2^lb.
cmm_status prepare(const cmm_batch& b, const BatchLayout& L, int lb, char* ws, hipStream_t s,
                   bool plans_only) {
  cmm_status st;
  for (size_t i = 0; i < b.probs.size(); ++i) {
    const cmm_problem& p = b.probs[i];
    const BatchPair& bp = L.pairs[i];
    if (!plans_only && p.keys) {
      st = launch_hash(p.keys, p.d, p.n_rows, p.n_cols, p.log2b, p.tab1, p.tab2, s);
      if (st != CMM_OK) return st;
    }
    if (!active(p)) continue;
    if (!plans_only) {
      st = launch_transpose(p.A, p.in_dtype, p.n_rows, p.n_inner, p.lda, ws + bp.at, b.cdt, s);
      if (st != CMM_OK) return st;
      if (bp.bc >= 0) {
        st = launch_convert(p.B, p.in_dtype, p.n_inner, p.n_cols, p.ldb, ws + bp.bc, b.cdt, s);
        if (st != CMM_OK) return st;
      }
    }
    // each repetition's transform window (it depends on b_lo, so it is
    // chosen again whenever the plans are), then the plans on the rotated
    // tables
    const uint32_t* t1 = p.tab1;
    const uint32_t* t2 = p.tab2;
    if (bp.rot >= 0) {
      uint32_t* r1 = reinterpret_cast<uint32_t*>(ws + bp.rtab1);
      uint32_t* r2 = reinterpret_cast<uint32_t*>(ws + bp.rtab2);
      st = launch_window(p.tab1, p.tab2, p.d, p.n_rows, p.n_cols, p.log2b, lb, r1, r2,
                         reinterpret_cast<int32_t*>(ws + bp.rot), s);
      if (st != CMM_OK) return st;
      t1 = r1;
      t2 = r2;
    }
    if ((st = launch_plan(t1, p.d, p.n_rows, lb, carve_plan(ws + bp.planA, p.d, p.n_rows, lb), s)) != CMM_OK)
      return st;
    if ((st = launch_plan(t2, p.d, p.n_cols, lb, carve_plan(ws + bp.planB, p.d, p.n_cols, lb), s)) != CMM_OK)
      return st;
  }
  return CMM_OK;
}

// The persistent Compress launch: descriptor copy, queue reset, launch.
cmm_status compress_all(cmm_batch& b, const BatchConfig& c, char* ws, hipStream_t s) {
  const BatchLayout& L = layout_of(b, c);
  if (L.items.empty()) return CMM_OK;
  void* h = nullptr;
  cmm_status st = staging_of(b, c, &h);
  if (st != CMM_OK) return st;
  st = hip_check(hipMemcpyAsync(ws + L.off_desc, h, L.desc_bytes, hipMemcpyHostToDevice, s),
                 "batch: descriptor copy");
  if (st != CMM_OK) return st;
  if ((st = launch_zero(reinterpret_cast<double*>(ws + L.off_queue), 1, s)) != CMM_OK) return st;
  const int wgs = (int)std::min<size_t>(L.items.size(), (size_t)compute_units() * c.wg_per_cu);
  return launch_compress_batched(ws, reinterpret_cast<const BatchPair*>(ws + L.off_desc),
                                 reinterpret_cast<const BatchItem*>(ws + L.off_items),
                                 (int)L.items.size(), reinterpret_cast<int*>(ws + L.off_queue),
                                 b.cdt, c.lb, c.radix, L.desc, wgs, L.lds, s);
}

// Per-problem work after Compress: partial sums, inverse transform, extract.
cmm_status finish(const cmm_batch& b, const BatchLayout& L, char* ws, hipStream_t s) {
  cmm_status st;
  for (size_t i = 0; i < b.probs.size(); ++i) {
    const cmm_problem& p = b.probs[i];
    const BatchPair& bp = L.pairs[i];
    const size_t blen = (size_t)1 << p.log2b;
    double* pp = p.p ? p.p : reinterpret_cast<double*>(ws + L.off_p[i]);
    if (active(p)) {
      if (bp.rot >= 0)   // partials in each repetition's rotated frame
        st = launch_reduce_window(reinterpret_cast<const double*>(ws + bp.partial), bp.groups,
                                  p.d, p.log2b, reinterpret_cast<const int32_t*>(ws + bp.rot),
                                  pp, s);
      else
        st = launch_reduce_partials(reinterpret_cast<const double*>(ws + bp.partial), bp.groups,
                                    (size_t)p.d * blen, pp, s);
      if (st != CMM_OK) return st;
      if ((st = launch_fwht(pp, CMM_F64, p.d, p.log2b, std::ldexp(1.0, -p.log2b), s)) != CMM_OK)
        return st;
    } else {
      if ((st = launch_zero(pp, (size_t)p.d * blen, s)) != CMM_OK) return st;
    }
    if (p.C_hat && p.n_rows > 0 && p.n_cols > 0) {
      st = launch_extract(pp, p.tab1, p.tab2, p.d, p.n_rows, p.n_cols, p.log2b, p.estimator,
                          p.C_hat, p.out_dtype, p.ldc, s);
      if (st != CMM_OK) return st;
    }
  }
  return CMM_OK;
}

cmm_status check_workspace(const cmm_batch* b, void* ws, size_t bytes, const char* fn) {
  if (bytes < b->ws_bytes) {
    set_error(std::string(fn) + ": workspace of " + std::to_string(bytes) + " bytes, need " +
              std::to_string(b->ws_bytes));
    return CMM_ENOMEM;
  }
  if (!ws && b->ws_bytes > 0) return invalid(std::string(fn) + ": workspace is null");
  if ((uintptr_t)ws % 256 != 0) return invalid(std::string(fn) + ": workspace must be 256-byte aligned");
  return CMM_OK;
}

// ---------------------------------------------------------- tuning cache
// Keyed by the device (architecture, compute units) and every problem's
// shape and types.  Kept for the process; with CMM_TUNE_CACHE naming a file
// the entries are also read from and appended to that file.
std::mutex g_tune_mu;
std::map<uint64_t, BatchConfig> g_tune;
bool g_tune_file_read = false;

uint64_t signature(const cmm_batch& b) {
  std::ostringstream os;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    os << prop.gcnArchName << '/' << prop.multiProcessorCount;
  os << '|' << (int)b.cdt;
  for (const cmm_problem& p : b.probs)
    os << '|' << p.n_rows << ',' << p.n_inner << ',' << p.n_cols << ',' << p.log2b << ','
       << p.d << ',' << (int)p.in_dtype << ',' << (p.p ? 1 : 0) << ',' << (p.ldb % 4);
  uint64_t h = 1469598103934665603ull;   // FNV-1a
  for (char ch : os.str()) { h ^= (uint8_t)ch; h *= 1099511628211ull; }
  return h;
}

void read_tune_file_locked() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("CMM_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    uint64_t key;
    BatchConfig c;
    if (is >> std::hex >> key >> std::dec >> c.lb >> c.kgrain >> c.wg_per_cu >> c.order >> c.radix)
      g_tune[key] = c;
  }
}

void write_tune_entry_locked(uint64_t key, const BatchConfig& c) {
  g_tune[key] = c;
  const char* path = std::getenv("CMM_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << std::hex << key << std::dec << ' ' << c.lb << ' ' << c.kgrain << ' ' << c.wg_per_cu << ' '
    << c.order << ' ' << c.radix << '\n';
}

cmm_status time_config(cmm_batch& b, const BatchConfig& c, char* ws, hipStream_t s, float* ms) {
  hipEvent_t e0, e1;
  cmm_status st = hip_check(hipEventCreate(&e0), "autotune: event");
  if (st != CMM_OK) return st;
  if ((st = hip_check(hipEventCreate(&e1), "autotune: event")) != CMM_OK) {
    (void)hipEventDestroy(e0);
    return st;
  }
  float best = 1e30f;
  for (int rep = 0; rep < 3 && st == CMM_OK; ++rep) {   // the first run warms up
    st = hip_check(hipEventRecord(e0, s), "autotune: record");
    if (st == CMM_OK) st = compress_all(b, c, ws, s);
    if (st == CMM_OK) st = hip_check(hipEventRecord(e1, s), "autotune: record");
    if (st == CMM_OK) st = hip_check(hipEventSynchronize(e1), "autotune: wait");
    float t = 0.f;
    if (st == CMM_OK) st = hip_check(hipEventElapsedTime(&t, e0, e1), "autotune: elapsed");
    if (rep > 0 && t < best) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return st;
}

}  // namespace
}  // namespace cmm

extern "C" {

cmm_status cmm_batch_create(const cmm_problem* probs, int count, cmm_batch** out) {
  if (!out) return invalid("cmm_batch_create: out is null");
  *out = nullptr;
  if (count < 1) return invalid("cmm_batch_create: count must be >= 1");
  if (!probs) return invalid("cmm_batch_create: probs is null");
  cmm_status s;
  for (int i = 0; i < count; ++i) {
    const std::string fn = "cmm_batch_create (problem " + std::to_string(i) + ")";
    if ((s = validate_problem(&probs[i], fn.c_str())) != CMM_OK) return s;
    if (probs[i].compute != probs[0].compute) return invalid(fn + ": every problem needs the same compute type");
    if (probs[i].compute != CMM_F64 && probs[i].compute != CMM_F32) {
      set_error(fn + ": the batched form computes in CMM_F64 or CMM_F32");
      return CMM_EUNSUPPORTED;
    }
    if (probs[i].d > 63 && probs[i].estimator == CMM_MEDIAN && probs[i].C_hat) {
      set_error(fn + ": median over more than 63 repetitions is not implemented");
      return CMM_EUNSUPPORTED;
    }
    if (probs[i].n_rows > 65534 || probs[i].n_cols > 65534) {
      set_error(fn + ": the batched form needs n_rows, n_cols <= 65534");
      return CMM_EUNSUPPORTED;
    }
  }
  std::unique_ptr<cmm_batch> b(new cmm_batch());
  b->probs.assign(probs, probs + count);
  b->cdt = probs[0].compute == CMM_F64 ? CMM_F64 : CMM_F32;
  for (int lb = 11; lb <= 13; ++lb) {
    bool ok = true;
    for (const cmm_problem& p : b->probs) {
      if (!active(p)) continue;
      ok = ok && p.log2b >= lb && compress_lds_base(b->cdt, lb, p.n_rows, p.n_cols) <= kLds - 256 &&
           plan_lds_bytes(p.n_rows, lb) <= kLds && plan_lds_bytes(p.n_cols, lb) <= kLds;
    }
    if (ok) b->lbs.push_back(lb);
  }
  if (b->lbs.empty()) {
    set_error("cmm_batch_create: some problem has log2b < 11 or rows too long for the LDS");
    return CMM_EUNSUPPORTED;
  }
  size_t mx = 0;
  for (const BatchConfig& c : candidates(*b)) {
    const BatchLayout& L = layout_of(*b, c);
    if (L.ok) mx = std::max(mx, L.bytes);
  }
  b->ws_bytes = mx;
  b->cfg = BatchConfig{b->lbs.back(), 64, 1, 0, b->lbs.back() == 13 ? 16 : 32};
  if (!layout_of(*b, b->cfg).ok) {
    bool found = false;
    for (const BatchConfig& c : candidates(*b))
      if (layout_of(*b, c).ok) { b->cfg = c; found = true; break; }
    if (!found) {
      set_error("cmm_batch_create: no launch configuration fits");
      return CMM_EUNSUPPORTED;
    }
  }
  void* h = nullptr;
  if ((s = staging_of(*b, b->cfg, &h)) != CMM_OK) return s;
  *out = b.release();
  return CMM_OK;
}

cmm_status cmm_batch_destroy(cmm_batch* batch) {
  delete batch;
  return CMM_OK;
}

cmm_status cmm_batch_workspace_size(const cmm_batch* batch, size_t* bytes) {
  if (!batch || !bytes) return invalid("cmm_batch_workspace_size: null pointer");
  *bytes = batch->ws_bytes;
  return CMM_OK;
}

cmm_status cmm_batch_set_config(cmm_batch* batch, int log2_blo, int k_per_item, int wg_per_cu,
                                int order, int radix) {
  if (!batch) return invalid("cmm_batch_set_config: null batch");
  const BatchConfig c{log2_blo, k_per_item, wg_per_cu, order, radix};
  bool known = false;
  for (const BatchConfig& x : candidates(*batch)) known = known || (!(x < c) && !(c < x));
  if (!known) return invalid("cmm_batch_set_config: not a candidate configuration");
  if (!layout_of(*batch, c).ok) {
    set_error("cmm_batch_set_config: the configuration does not fit these problems");
    return CMM_EUNSUPPORTED;
  }
  void* h = nullptr;
  cmm_status st = staging_of(*batch, c, &h);
  if (st != CMM_OK) return st;
  batch->cfg = c;
  batch->tuned = 3;
  return CMM_OK;
}

cmm_status cmm_batch_get_config(const cmm_batch* batch, int* log2_blo, int* k_per_item,
                                int* wg_per_cu, int* order, int* radix, int* source) {
  if (!batch || !log2_blo || !k_per_item || !wg_per_cu || !order || !radix || !source)
    return invalid("cmm_batch_get_config: null pointer");
  *radix = batch->cfg.radix;
  *log2_blo = batch->cfg.lb;
  *k_per_item = batch->cfg.kgrain;
  *wg_per_cu = batch->cfg.wg_per_cu;
  *order = batch->cfg.order;
  *source = batch->tuned;
  return CMM_OK;
}

cmm_status cmm_batch_autotune(cmm_batch* batch, void* workspace, size_t workspace_bytes,
                              void* stream) {
  if (!batch) return invalid("cmm_batch_autotune: null batch");
  cmm_status st = check_workspace(batch, workspace, workspace_bytes, "cmm_batch_autotune");
  if (st != CMM_OK) return st;
  const uint64_t key = signature(*batch);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    read_tune_file_locked();
    auto it = g_tune.find(key);
    void* h = nullptr;
    if (it != g_tune.end() && layout_of(*batch, it->second).ok &&
        staging_of(*batch, it->second, &h) == CMM_OK) {
      batch->cfg = it->second;
      batch->tuned = 2;
      return CMM_OK;
    }
  }
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
  // tables and operand copies once; plans per b_lo
  BatchConfig cur = batch->cfg;
  if ((st = prepare(*batch, layout_of(*batch, cur), cur.lb, ws, s, false)) != CMM_OK) return st;
  float best_ms = 0.f;
  if ((st = time_config(*batch, cur, ws, s, &best_ms)) != CMM_OK) return st;
  auto try_cfg = [&](const BatchConfig& c) -> cmm_status {
    const BatchLayout& L = layout_of(*batch, c);
    if (!L.ok) return CMM_OK;
    cmm_status r;
    if (c.lb != cur.lb || c.kgrain != cur.kgrain)   // plan offsets move with the layout
      if ((r = prepare(*batch, L, c.lb, ws, s, false)) != CMM_OK) return r;
    float ms = 0.f;
    if ((r = time_config(*batch, c, ws, s, &ms)) != CMM_OK) return r;
    if (ms < best_ms) { best_ms = ms; cur = c; }
    else if ((r = prepare(*batch, layout_of(*batch, cur), cur.lb, ws, s, false)) != CMM_OK) return r;
    return CMM_OK;
  };
  // coordinate descent: k-range, LDS share, tile and radix, order
  auto with = [&](int lb, int kg, int wg, int ord, int radix) { return BatchConfig{lb, kg, wg, ord, radix}; };
  for (int kg : kKGrains)
    if (kg != cur.kgrain &&
        (st = try_cfg(with(cur.lb, kg, cur.wg_per_cu, cur.order, cur.radix))) != CMM_OK) return st;
  for (int wg = 1; wg <= 2; ++wg)
    if (wg != cur.wg_per_cu &&
        (st = try_cfg(with(cur.lb, cur.kgrain, wg, cur.order, cur.radix))) != CMM_OK) return st;
  for (int lb : batch->lbs)
    for (int radix : {16, 32})
      if ((lb != cur.lb || radix != cur.radix) && (radix == 32 || lb == 13) &&
          (st = try_cfg(with(lb, cur.kgrain, cur.wg_per_cu, cur.order, radix))) != CMM_OK) return st;
  for (int ord = 0; ord <= 1; ++ord)
    if (ord != cur.order &&
        (st = try_cfg(with(cur.lb, cur.kgrain, cur.wg_per_cu, ord, cur.radix))) != CMM_OK) return st;
  void* h = nullptr;
  if ((st = staging_of(*batch, cur, &h)) != CMM_OK) return st;
  batch->cfg = cur;
  batch->tuned = 1;
  std::lock_guard<std::mutex> g(g_tune_mu);
  write_tune_entry_locked(key, cur);
  return CMM_OK;
}

cmm_status cmm_estimate_batched(cmm_batch* batch, void* workspace, size_t workspace_bytes,
                                void* stream) {
  if (!batch) return invalid("cmm_estimate_batched: null batch");
  cmm_status st = check_workspace(batch, workspace, workspace_bytes, "cmm_estimate_batched");
  if (st != CMM_OK) return st;
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = as_stream(stream);
  const BatchConfig c = batch->cfg;
  const BatchLayout& L = layout_of(*batch, c);
  if ((st = prepare(*batch, L, c.lb, ws, s, false)) != CMM_OK) return st;
  if ((st = compress_all(*batch, c, ws, s)) != CMM_OK) return st;
  return finish(*batch, L, ws, s);
}

}  // extern "C"
