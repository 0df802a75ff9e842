// Top-K Decompress: the K entries of largest magnitude of the estimate
// C_hat[i][j] = Median_t s1_t(i) s2_t(j) p[t][h1_t(i) xor h2_t(j)] (or the
// mean over t), found without writing the dense C_hat (Algorithm 1's
// Decompress evaluated at every entry, the point of the method being the
// large entries of the product, Section 1).
//
// Order.  Entries are ranked by |C_hat| (its float64 bit pattern, which for
// non-negative values orders like an unsigned integer), ties by the
// smaller row-major index i n_cols + j.  The composite key
//   key = |C_hat| bits << 33  |  (2^31 - 1 - index) << 2     (96 bits)
// is unique per entry, so the K largest keys are exactly the answer.
//
// Radix select.  Eight levels of 12-bit digits from the top of the key.  A
// histogram pass evaluates every entry and counts the digit of level l among
// the entries whose higher digits equal the prefix selected so far; a
// one-work-group select step then takes the digit where the count from the
// top reaches K.  Once the selected bin holds at most kBinCap entries (or
// the key is fully resolved) a collect pass gathers every entry at or above
// the prefix: fewer than K above it plus the bin, at most K + kBinCap in all.
// A stable radix sort (by the index part, then by the magnitude) orders them
// and the first K are written.  Passes after the select step has finished
// return at once, so no host synchronisation is needed.
#include <hipcub/hipcub.hpp>

#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr int kBins = 4096;        // 12-bit digits
constexpr int kLevels = 8;         // 96-bit keys
constexpr int64_t kBinCap = 16384; // entries of the last bin taken whole
constexpr int kTcols = 256;        // columns of a tile (one per thread)
constexpr int kTrows = 8;          // rows of a tile
constexpr int kMaxDTopk = 63;

typedef unsigned __int128 u128;

struct TopkState {
  unsigned long long prefix_hi;   // selected digits (the key's top 12 level bits)
  unsigned long long prefix_lo;
  long long above;                // entries whose key is above the selected bin
  long long need;                 // K - above
  unsigned long long count;       // candidates gathered by the collect pass
  int level;                      // digit levels resolved
  int done;                       // the selection has finished
};

__device__ __forceinline__ u128 make_key(double o, int64_t idx) {
  const uint64_t mag = (uint64_t)__double_as_longlong(fabs(o));
  const uint64_t inv = 0x7FFFFFFFull - (uint64_t)idx;
  return ((u128)mag << 33) | ((u128)inv << 2);
}

__device__ __forceinline__ u128 prefix_of(const TopkState& st) {
  return ((u128)st.prefix_hi << 64) | (u128)st.prefix_lo;
}

// Odd-even transposition network leaving v sorted (the median is v[D / 2]).
template <int D>
__device__ __forceinline__ void sort_small(double (&v)[D]) {
#pragma unroll
  for (int round = 0; round < D; ++round) {
#pragma unroll
    for (int i = round & 1; i + 1 < D; i += 2) {
      const double a = v[i], c = v[i + 1];
      v[i] = fmin(a, c);
      v[i + 1] = fmax(a, c);
    }
  }
}

// Estimate at (i, j) over D repetitions (D = 0: the runtime d, up to
// kMaxDTopk for the median, by insertion into a sorted list).  The values
// are those of the dense Decompress, bit for bit: the same gathers, the
// same sign rule, the median as the exact middle value, the mean summed in
// repetition order.
template <int D>
__device__ __forceinline__ double estimate_at(const double* __restrict__ p,
                                              const uint32_t* __restrict__ tab1,
                                              const uint32_t* __restrict__ tab2, int d,
                                              int64_t n_rows, int64_t n_cols, int64_t b,
                                              int64_t i, int64_t j, bool mean) {
  const uint32_t bmask = (uint32_t)(b - 1);
  if constexpr (D > 0) {
    double v[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const uint32_t e = tab1[(size_t)t * n_rows + i] ^ tab2[(size_t)t * n_cols + j];
      const double x = p[(size_t)t * b + (e & bmask)];
      v[t] = (e & kSignBit) ? -x : x;
    }
    if (mean) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < D; ++t) s += v[t];
      return s / D;
    }
    sort_small<D>(v);
    return v[D / 2];
  } else {
    double v[kMaxDTopk];
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
      const uint32_t e = tab1[(size_t)t * n_rows + i] ^ tab2[(size_t)t * n_cols + j];
      const double x = p[(size_t)t * b + (e & bmask)];
      const double y = (e & kSignBit) ? -x : x;
      s += y;
      if (!mean) {
        int q = t;
        while (q > 0 && v[q - 1] > y) { v[q] = v[q - 1]; --q; }
        v[q] = y;
      }
    }
    return mean ? s / d : v[d / 2];
  }
}

struct TopkArgs {
  const double* p;
  const uint32_t* tab1;
  const uint32_t* tab2;
  int d;
  int64_t n_rows, n_cols;
  int log2b;
  int mean;
  TopkState* st;
  unsigned int* hist;      // [kBins]
  // candidates (collect pass)
  uint64_t* c_mag;         // [cap] magnitude bits
  uint32_t* c_inv;         // [cap] 2^31 - 1 - index
  double* c_val;           // [cap] signed estimate
  int64_t cap;
};

// One count per lane that wants it into lh[digit], one LDS atomic per
// distinct digit in the wave (every lane of the wave takes part).
__device__ __forceinline__ void wave_count(unsigned int* lh, uint32_t digit, bool want) {
  unsigned long long active = __ballot(want);
  const uint32_t lane = threadIdx.x & 63;
  while (active) {
    const int leader = __ffsll((long long)active) - 1;
    const uint32_t dl = __shfl(digit, leader);
    const unsigned long long same = __ballot(want && digit == dl);
    if (lane == (uint32_t)leader) atomicAdd(&lh[dl], (unsigned int)__popcll(same));
    active &= ~same;
  }
}

// Histogram pass of digit level `level`: one tile of kTrows x kTcols
// entries per work-group and round, grid-strided over the tiles.
template <int D>
__global__ __launch_bounds__(kTcols) void topk_hist_kernel(TopkArgs a, int level) {
  __shared__ unsigned int lh[kBins];
  __shared__ int s_skip;
  if (threadIdx.x == 0) s_skip = (a.st->done || a.st->level != level) ? 1 : 0;
  for (int q = threadIdx.x; q < kBins; q += kTcols) lh[q] = 0u;
  __syncthreads();
  if (s_skip) return;   // uniform
  const u128 prefix = prefix_of(*a.st);
  const int hi_shift = 96 - 12 * level;      // key bits above this level
  const int dig_shift = 84 - 12 * level;
  const int64_t b = (int64_t)1 << a.log2b;
  const int64_t tiles_r = (a.n_rows + kTrows - 1) / kTrows;
  const int64_t tiles_c = (a.n_cols + kTcols - 1) / kTcols;
  for (int64_t tile = blockIdx.x; tile < tiles_r * tiles_c; tile += gridDim.x) {
    const int64_t tr = tile / tiles_c, tc = tile - tr * tiles_c;
    const int64_t j = tc * kTcols + threadIdx.x;
    const bool jok = j < a.n_cols;
    for (int r = 0; r < kTrows; ++r) {
      const int64_t i = tr * kTrows + r;
      if (i >= a.n_rows) break;   // uniform over the work-group
      bool want = false;
      uint32_t digit = 0;
      if (jok) {
        const double o = estimate_at<D>(a.p, a.tab1, a.tab2, a.d, a.n_rows, a.n_cols, b, i, j,
                                        a.mean != 0);
        const u128 key = make_key(o, i * a.n_cols + j);
        want = level == 0 || (key >> hi_shift) == prefix;
        digit = (uint32_t)(key >> dig_shift) & (kBins - 1);
      }
      wave_count(lh, digit, want);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kBins; q += kTcols)
    if (lh[q]) atomicAdd(&a.hist[q], lh[q]);
}

// Select step (one work-group): the digit of the current level where the
// count of entries from the top reaches `need`; the histogram is cleared for
// the next level.
__global__ __launch_bounds__(256) void topk_select_kernel(TopkState* st, unsigned int* hist) {
  __shared__ unsigned long long s_sum[256];
  __shared__ int s_skip;
  constexpr int per = kBins / 256;
  if (threadIdx.x == 0) s_skip = st->done;
  __syncthreads();
  if (s_skip) return;
  // thread q owns bins [kBins - per (q + 1), kBins - per q): chunks from the top
  const int hi_bin = kBins - per * (int)threadIdx.x - 1;
  unsigned long long mine = 0;
  for (int u = 0; u < per; ++u) mine += hist[hi_bin - u];
  s_sum[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long need = st->need;
    unsigned long long cum = 0;
    int digit = 0;
    unsigned long long bin = 0;
    for (int q = 0; q < 256; ++q) {
      if (cum + s_sum[q] >= (unsigned long long)need) {
        // inside chunk q, from its top bin down
        const int top = kBins - per * q - 1;
        for (int u = 0; u < per; ++u) {
          const unsigned int c = hist[top - u];
          if (cum + c >= (unsigned long long)need) { digit = top - u; bin = c; break; }
          cum += c;
        }
        break;
      }
      cum += s_sum[q];
    }
    st->above += (long long)cum;
    st->need = need - (long long)cum;
    const u128 pre = (prefix_of(*st) << 12) | (u128)(unsigned)digit;
    st->prefix_hi = (unsigned long long)(pre >> 64);
    st->prefix_lo = (unsigned long long)pre;
    st->level += 1;
    st->done = (bin <= (unsigned long long)kBinCap || st->level == kLevels) ? 1 : 0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kBins; q += 256) hist[q] = 0u;
}

// Collect pass: every entry whose key is at or above the selected prefix.
template <int D>
__global__ __launch_bounds__(kTcols) void topk_collect_kernel(TopkArgs a) {
  const TopkState st = *a.st;
  const u128 prefix = prefix_of(st);
  const int shift = 96 - 12 * st.level;
  const int64_t b = (int64_t)1 << a.log2b;
  const uint32_t lane = threadIdx.x & 63;
  const int64_t tiles_r = (a.n_rows + kTrows - 1) / kTrows;
  const int64_t tiles_c = (a.n_cols + kTcols - 1) / kTcols;
  for (int64_t tile = blockIdx.x; tile < tiles_r * tiles_c; tile += gridDim.x) {
    const int64_t tr = tile / tiles_c, tc = tile - tr * tiles_c;
    const int64_t j = tc * kTcols + threadIdx.x;
    const bool jok = j < a.n_cols;
    for (int r = 0; r < kTrows; ++r) {
      const int64_t i = tr * kTrows + r;
      if (i >= a.n_rows) break;   // uniform over the work-group
      double o = 0.0;
      bool hit = false;
      if (jok) {
        o = estimate_at<D>(a.p, a.tab1, a.tab2, a.d, a.n_rows, a.n_cols, b, i, j, a.mean != 0);
        hit = (make_key(o, i * a.n_cols + j) >> shift) >= prefix;
      }
      const unsigned long long mask = __ballot(hit);
      if (mask == 0ull) continue;
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(&a.st->count, (unsigned long long)__popcll(mask));
      base = __shfl(base, 0);
      if (hit) {
        const unsigned long long slot = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (slot < (unsigned long long)a.cap) {   // at most K + kBinCap by construction
          const int64_t idx = i * a.n_cols + j;
          a.c_mag[slot] = (uint64_t)__double_as_longlong(fabs(o));
          a.c_inv[slot] = (uint32_t)(0x7FFFFFFFll - idx);
          a.c_val[slot] = o;
        }
      }
    }
  }
}

// State, histogram and candidate buffers reset (a kernel: stays valid under
// stream capture).  Unused candidates keep magnitude 0 and index part 0,
// which sort after every real entry of equal key (the sort is stable and
// the real entries come first).
__global__ void topk_init_kernel(TopkState* st, unsigned int* hist, uint64_t* c_mag,
                                 uint32_t* c_inv, double* c_val, uint32_t* perm, int64_t cap,
                                 int64_t k) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (gid == 0) {
    st->prefix_hi = 0ull;
    st->prefix_lo = 0ull;
    st->above = 0;
    st->need = k;
    st->count = 0ull;
    st->level = 0;
    st->done = 0;
  }
  for (int64_t q = gid; q < kBins; q += stride) hist[q] = 0u;
  for (int64_t q = gid; q < cap; q += stride) {
    c_mag[q] = 0ull;
    c_inv[q] = 0u;
    c_val[q] = 0.0;
    perm[q] = (uint32_t)q;
  }
}

__global__ void topk_gather_mag_kernel(const uint64_t* __restrict__ c_mag,
                                       const uint32_t* __restrict__ perm, uint64_t* out,
                                       int64_t cap) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < cap) out[q] = c_mag[perm[q]];
}

template <typename OutT>
__global__ void topk_write_kernel(const uint32_t* __restrict__ perm,
                                  const uint32_t* __restrict__ c_inv,
                                  const double* __restrict__ c_val, int64_t k, int64_t n_cols,
                                  int64_t* rows, int64_t* cols, OutT* vals) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= k) return;
  const uint32_t c = perm[q];
  const int64_t idx = 0x7FFFFFFFll - (int64_t)c_inv[c];
  rows[q] = idx / n_cols;
  cols[q] = idx - (idx / n_cols) * n_cols;
  vals[q] = (OutT)c_val[c];
}

// Workspace layout for k entries.
struct TopkLayout {
  int64_t cap = 0;
  size_t off_state = 0, off_hist = 0, off_mag = 0, off_inv = 0, off_val = 0, off_perm_a = 0,
         off_perm_b = 0, off_inv_b = 0, off_mag_a = 0, off_mag_b = 0, off_temp = 0;
  size_t temp_bytes = 0, bytes = 0;
};

cmm_status topk_layout(int64_t k, TopkLayout* L) {
  L->cap = k + kBinCap;
  const size_t cap = (size_t)L->cap;
  size_t temp1 = 0, temp2 = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(
      nullptr, temp1, (const uint32_t*)nullptr, (uint32_t*)nullptr, (const uint32_t*)nullptr,
      (uint32_t*)nullptr, (int)cap);
  if (e != hipSuccess) return hip_check(e, "top-K: sort workspace size");
  e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, temp2, (const uint64_t*)nullptr,
                                                    (uint64_t*)nullptr, (const uint32_t*)nullptr,
                                                    (uint32_t*)nullptr, (int)cap);
  if (e != hipSuccess) return hip_check(e, "top-K: sort workspace size");
  L->temp_bytes = temp1 > temp2 ? temp1 : temp2;
  size_t off = 0;
  L->off_state = off; off = align_up(off + sizeof(TopkState), 256);
  L->off_hist = off; off = align_up(off + sizeof(unsigned int) * kBins, 256);
  L->off_mag = off; off = align_up(off + sizeof(uint64_t) * cap, 256);
  L->off_inv = off; off = align_up(off + sizeof(uint32_t) * cap, 256);
  L->off_val = off; off = align_up(off + sizeof(double) * cap, 256);
  L->off_perm_a = off; off = align_up(off + sizeof(uint32_t) * cap, 256);
  L->off_perm_b = off; off = align_up(off + sizeof(uint32_t) * cap, 256);
  L->off_inv_b = off; off = align_up(off + sizeof(uint32_t) * cap, 256);
  L->off_mag_a = off; off = align_up(off + sizeof(uint64_t) * cap, 256);
  L->off_mag_b = off; off = align_up(off + sizeof(uint64_t) * cap, 256);
  L->off_temp = off; off = align_up(off + L->temp_bytes, 256);
  L->bytes = off;
  return CMM_OK;
}

template <int D>
void launch_passes(const TopkArgs& a, int64_t grid, hipStream_t s) {
  for (int level = 0; level < kLevels; ++level) {
    hipLaunchKernelGGL(topk_hist_kernel<D>, dim3((unsigned)grid), dim3(kTcols), 0, s, a, level);
    hipLaunchKernelGGL(topk_select_kernel, dim3(1), dim3(256), 0, s, a.st, a.hist);
  }
  hipLaunchKernelGGL(topk_collect_kernel<D>, dim3((unsigned)grid), dim3(kTcols), 0, s, a);
}

}  // namespace

cmm_status topk_workspace_bytes(int64_t k, size_t* bytes) {
  TopkLayout L;
  cmm_status st = topk_layout(k, &L);
  if (st == CMM_OK) *bytes = L.bytes;
  return st;
}

cmm_status launch_extract_topk(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                               int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                               int64_t k, int64_t* rows, int64_t* cols, void* vals,
                               cmm_dtype out_dt, void* workspace, size_t ws_bytes, hipStream_t s) {
  ProfScope prof_("extract_topk", s);
  TopkLayout L;
  cmm_status st = topk_layout(k, &L);
  if (st != CMM_OK) return st;
  if (ws_bytes < L.bytes) {
    set_error("cmm_extract_topk: workspace of " + std::to_string(ws_bytes) + " bytes, need " +
              std::to_string(L.bytes));
    return CMM_ENOMEM;
  }
  char* ws = static_cast<char*>(workspace);
  TopkArgs a;
  a.p = p;
  a.tab1 = tab1;
  a.tab2 = tab2;
  a.d = d;
  a.n_rows = n_rows;
  a.n_cols = n_cols;
  a.log2b = log2b;
  a.mean = est == CMM_MEAN;
  a.st = reinterpret_cast<TopkState*>(ws + L.off_state);
  a.hist = reinterpret_cast<unsigned int*>(ws + L.off_hist);
  a.c_mag = reinterpret_cast<uint64_t*>(ws + L.off_mag);
  a.c_inv = reinterpret_cast<uint32_t*>(ws + L.off_inv);
  a.c_val = reinterpret_cast<double*>(ws + L.off_val);
  a.cap = L.cap;
  uint32_t* perm_a = reinterpret_cast<uint32_t*>(ws + L.off_perm_a);
  uint32_t* perm_b = reinterpret_cast<uint32_t*>(ws + L.off_perm_b);
  uint32_t* inv_b = reinterpret_cast<uint32_t*>(ws + L.off_inv_b);
  uint64_t* mag_a = reinterpret_cast<uint64_t*>(ws + L.off_mag_a);
  uint64_t* mag_b = reinterpret_cast<uint64_t*>(ws + L.off_mag_b);
  void* temp = ws + L.off_temp;
  const int64_t init_blocks = (L.cap + 255) / 256 < 4096 ? (L.cap + 255) / 256 : 4096;
  hipLaunchKernelGGL(topk_init_kernel, dim3((unsigned)init_blocks), dim3(256), 0, s, a.st, a.hist,
                     a.c_mag, a.c_inv, a.c_val, perm_a, L.cap, k);
  if ((st = hip_check(hipGetLastError(), "top-K init launch")) != CMM_OK) return st;
  // every pass visits every tile: at most 8192 work-groups, grid-strided
  const int64_t tiles = ((n_rows + kTrows - 1) / kTrows) * ((n_cols + kTcols - 1) / kTcols);
  const int64_t grid = tiles < 8192 ? tiles : 8192;
#define CMM_TOPK_CASE(DV) \
  case DV: launch_passes<DV>(a, grid, s); break;
  switch (d) {
    CMM_TOPK_CASE(1)
    CMM_TOPK_CASE(3)
    CMM_TOPK_CASE(5)
    CMM_TOPK_CASE(7)
    CMM_TOPK_CASE(9)
    CMM_TOPK_CASE(11)
    CMM_TOPK_CASE(13)
    default: launch_passes<0>(a, grid, s);
  }
#undef CMM_TOPK_CASE
  if ((st = hip_check(hipGetLastError(), "top-K pass launch")) != CMM_OK) return st;
  // stable sorts: by the index part, then by the magnitude (both descending)
  const int n = (int)L.cap;
  size_t tb = L.temp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tb, a.c_inv, inv_b, perm_a,
                                                              perm_b, n, 0, 32, s);
  if (e != hipSuccess) return hip_check(e, "top-K sort by index");
  hipLaunchKernelGGL(topk_gather_mag_kernel, dim3((unsigned)((L.cap + 255) / 256)), dim3(256), 0, s,
                     a.c_mag, perm_b, mag_a, L.cap);
  if ((st = hip_check(hipGetLastError(), "top-K gather launch")) != CMM_OK) return st;
  tb = L.temp_bytes;
  e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tb, mag_a, mag_b, perm_b, perm_a, n, 0,
                                                    64, s);
  if (e != hipSuccess) return hip_check(e, "top-K sort by magnitude");
  const unsigned wb = (unsigned)((k + 255) / 256);
  if (out_dt == CMM_F64)
    hipLaunchKernelGGL(topk_write_kernel<double>, dim3(wb), dim3(256), 0, s, perm_a, a.c_inv,
                       a.c_val, k, n_cols, rows, cols, static_cast<double*>(vals));
  else
    hipLaunchKernelGGL(topk_write_kernel<float>, dim3(wb), dim3(256), 0, s, perm_a, a.c_inv,
                       a.c_val, k, n_cols, rows, cols, static_cast<float*>(vals));
  return hip_check(hipGetLastError(), "top-K write launch");
}

}  // namespace cmm
