// Dense Decompress (Algorithm 1): C_hat[i][j] = Median_t s1 s2 p_t[h1 ^ h2].
//
// A work-group owns a tile of kRows rows x 256 columns.  The repetition loop
// is outermost so that, at any moment, the tiles in flight gather from the
// same one or two length-b slices of p (which stay resident in L2); each
// thread keeps its d candidates per output in registers and takes the
// median with a fixed min/max network.  Signs are applied by XOR of the two
// sign bits (exact).
#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr int kCols = 256;
constexpr int kRows = 8;

// Rows of a tile whose d candidates are gathered together (all of them up to
// d = 11; beyond, the tile is taken in two halves to stay within registers).
__host__ __device__ constexpr int rows_per_round(int d) { return d <= 11 ? kRows : kRows / 2; }

// Entry of (i, j) from the two table entries: the bucket in the low bits
// (the caller masks with b - 1), the sign product in bit 31.  The xor form
// (Section 3.2) xors the buckets; Pagh's FFT form (Section 3.1) adds them
// modulo b.
template <bool CYC>
__device__ __forceinline__ uint32_t combine(uint32_t a, uint32_t b) {
  if (CYC) return ((a & 0x7FFFFFFFu) + (b & 0x7FFFFFFFu)) | ((a ^ b) & kSignBit);
  return a ^ b;
}

// Compare-exchange network (odd-even transposition) leaving v sorted.
template <int D>
__device__ __forceinline__ void sort_net(double (&v)[D]) {
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

template <typename OutT, int D, bool CYC = false>
__global__ __launch_bounds__(kCols) void extract_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int64_t n_rows, int64_t n_cols, int log2b, int mean,
    OutT* __restrict__ C, int64_t ldc) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kRows;
  const int64_t b = (int64_t)1 << log2b;
  const uint32_t bmask = (uint32_t)(b - 1);
  const bool jok = j < n_cols;
  constexpr int RG = rows_per_round(D);
#pragma unroll
  for (int g = 0; g < kRows; g += RG) {
    double v[RG][D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const uint32_t e2 = jok ? tab2[(size_t)t * n_cols + j] : 0u;
      const double* pt = p + (size_t)t * b;
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        const int64_t i = i0 + g + r < n_rows ? i0 + g + r : n_rows - 1;
        const uint32_t e = combine<CYC>(tab1[(size_t)t * n_rows + i], e2);
        const double x = pt[e & bmask];
        v[r][t] = (e & kSignBit) ? -x : x;
      }
    }
    if (!jok) return;
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      if (i0 + g + r >= n_rows) return;
      double out;
      if (mean) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < D; ++t) s += v[r][t];
        out = s / D;
      } else {
        sort_net<D>(v[r]);
        out = v[r][D / 2];
      }
      C[(i0 + g + r) * ldc + j] = (OutT)out;
    }
  }
}

// Generic d: the median (d up to kMaxD) keeps the candidates in a local
// array, insertion sorted; the mean only sums them.
constexpr int kMaxD = 63;
template <typename OutT, bool CYC = false>
__global__ __launch_bounds__(kCols) void extract_generic_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int d, int64_t n_rows, int64_t n_cols, int log2b,
    int mean, OutT* __restrict__ C, int64_t ldc) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t b = (int64_t)1 << log2b;
  if (j >= n_cols) return;
  for (int r = 0; r < kRows; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kRows + r;
    if (i >= n_rows) break;
    double v[kMaxD];
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
      const uint32_t e = combine<CYC>(tab1[(size_t)t * n_rows + i], tab2[(size_t)t * n_cols + j]);
      const double x = p[(size_t)t * b + (e & (uint32_t)(b - 1))];
      const double y = (e & kSignBit) ? -x : x;
      s += y;
      if (!mean) {   // the median keeps d <= kMaxD candidates; the mean any d
        int q = t;
        while (q > 0 && v[q - 1] > y) { v[q] = v[q - 1]; --q; }
        v[q] = y;
      }
    }
    C[i * ldc + j] = (OutT)(mean ? s / d : v[d / 2]);
  }
}

// ------------------------------------------------------- sparse queries
// Decompress at a list of entries: one thread per (rows[q], cols[q]).
template <typename OutT>
__global__ __launch_bounds__(256) void extract_entries_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int d, int64_t n_rows, int64_t n_cols, int log2b, int mean,
    const int64_t* __restrict__ rows, const int64_t* __restrict__ cols, int64_t count,
    OutT* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  const int64_t i = rows[q], j = cols[q];
  if (i < 0 || i >= n_rows || j < 0 || j >= n_cols) {
    out[q] = (OutT)__builtin_nan("");
    return;
  }
  const int64_t b = (int64_t)1 << log2b;
  double v[kMaxD];
  double s = 0.0;
  for (int t = 0; t < d; ++t) {
    const uint32_t e = tab1[(size_t)t * n_rows + i] ^ tab2[(size_t)t * n_cols + j];
    const double x = p[(size_t)t * b + (e & (uint32_t)(b - 1))];
    const double y = (e & kSignBit) ? -x : x;
    s += y;
    if (!mean) {
      int r = t;
      while (r > 0 && v[r - 1] > y) { v[r] = v[r - 1]; --r; }
      v[r] = y;
    }
  }
  out[q] = (OutT)(mean ? s / d : v[d / 2]);
}

// Heavy hitters over the dense grid: the tile structure of extract_kernel,
// but an entry is written only when |C_hat| >= thr.  The hits of a wave are
// counted with a ballot and reserved with one atomic add; each hit lane
// writes at the base plus the number of hit lanes below it.
template <typename OutT, int D>
__global__ __launch_bounds__(kCols) void heavy_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int64_t n_rows, int64_t n_cols, int log2b, int mean,
    double thr, int64_t* __restrict__ out_rows, int64_t* __restrict__ out_cols,
    OutT* __restrict__ out_vals, int64_t capacity, unsigned long long* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kRows;
  const int64_t b = (int64_t)1 << log2b;
  const uint32_t bmask = (uint32_t)(b - 1);
  const bool jok = j < n_cols;
  const uint32_t lane = threadIdx.x & 63;
  constexpr int RG = rows_per_round(D);
#pragma unroll
  for (int g = 0; g < kRows; g += RG) {
    double v[RG][D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const uint32_t e2 = jok ? tab2[(size_t)t * n_cols + j] : 0u;
      const double* pt = p + (size_t)t * b;
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        const int64_t i = i0 + g + r < n_rows ? i0 + g + r : n_rows - 1;
        const uint32_t e = tab1[(size_t)t * n_rows + i] ^ e2;
        const double x = pt[e & bmask];
        v[r][t] = (e & kSignBit) ? -x : x;
      }
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      double o;
      if (mean) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < D; ++t) s += v[r][t];
        o = s / D;
      } else {
        sort_net<D>(v[r]);
        o = v[r][D / 2];
      }
      const bool hit = jok && (i0 + g + r < n_rows) && fabs(o) >= thr;
      const unsigned long long mask = __ballot(hit);   // every lane of the wave takes part
      if (mask == 0ull) continue;
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(mask));
      base = __shfl(base, 0);
      if (hit) {
        const unsigned long long slot = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (slot < (unsigned long long)capacity) {
          out_rows[slot] = i0 + g + r;
          out_cols[slot] = j;
          out_vals[slot] = (OutT)o;
        }
      }
    }
  }
}

template <typename OutT>
__global__ __launch_bounds__(kCols) void heavy_generic_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int d, int64_t n_rows, int64_t n_cols, int log2b,
    int mean, double thr, int64_t* __restrict__ out_rows, int64_t* __restrict__ out_cols,
    OutT* __restrict__ out_vals, int64_t capacity, unsigned long long* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t b = (int64_t)1 << log2b;
  const uint32_t lane = threadIdx.x & 63;
  const bool jok = j < n_cols;
  for (int r = 0; r < kRows; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kRows + r;
    double o = 0.0;
    if (jok && i < n_rows) {
      double v[kMaxD];
      double s = 0.0;
      for (int t = 0; t < d; ++t) {
        const uint32_t e = tab1[(size_t)t * n_rows + i] ^ tab2[(size_t)t * n_cols + j];
        const double x = p[(size_t)t * b + (e & (uint32_t)(b - 1))];
        const double y = (e & kSignBit) ? -x : x;
        s += y;
        if (!mean) {
          int q = t;
          while (q > 0 && v[q - 1] > y) { v[q] = v[q - 1]; --q; }
          v[q] = y;
        }
      }
      o = mean ? s / d : v[d / 2];
    }
    const bool hit = jok && i < n_rows && fabs(o) >= thr;
    const unsigned long long mask = __ballot(hit);
    if (mask == 0ull) continue;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0);
    if (hit) {
      const unsigned long long slot = base + __popcll(mask & ((1ull << lane) - 1ull));
      if (slot < (unsigned long long)capacity) {
        out_rows[slot] = i;
        out_cols[slot] = j;
        out_vals[slot] = (OutT)o;
      }
    }
  }
}

// Per-repetition estimates at a list of entries: out[t][q] = s1 s2 p_t[h1 ^ h2]
// for (rows[q], cols[q]); NaN where the index is outside the tables.
// grid.y walks repetitions in slabs of 65535.
template <typename OutT>
__global__ __launch_bounds__(256) void extract_reps_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int d, int64_t n_rows, int64_t n_cols, int log2b,
    const int64_t* __restrict__ rows, const int64_t* __restrict__ cols, int64_t count,
    OutT* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  const int64_t i = rows[q], j = cols[q];
  const bool ok = i >= 0 && i < n_rows && j >= 0 && j < n_cols;
  const int64_t b = (int64_t)1 << log2b;
  for (int t = blockIdx.y; t < d; t += gridDim.y) {
    double y = __builtin_nan("");
    if (ok) {
      const uint32_t e = tab1[(size_t)t * n_rows + i] ^ tab2[(size_t)t * n_cols + j];
      const double x = p[(size_t)t * b + (e & (uint32_t)(b - 1))];
      y = (e & kSignBit) ? -x : x;
    }
    out[(size_t)t * count + q] = (OutT)y;
  }
}

// Correctness counters of the evaluation protocol over the dense grid:
// c[1] += #{|C_hat| <= thr}, c[3] += #{|C_hat - C| <= tol} (every entry;
// the big entries are taken out again by correctness_big_kernel).  A thread
// counts its column over a strided set of rows; the block sums the threads'
// counts and adds them with one atomic per counter (integer adds: the
// totals do not depend on the order).  The grid is a few thousand blocks,
// so the atomics on the two counters stay few.
template <typename InT>
__global__ __launch_bounds__(256) void correctness_dense_kernel(
    const InT* __restrict__ C_hat, int64_t ldh, const double* __restrict__ C, int64_t ldc,
    int64_t n_rows, int64_t n_cols, double thr, double tol, unsigned long long* __restrict__ c) {
  __shared__ unsigned long long part[2][4];
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  uint32_t le = 0, close = 0;
  if (j < n_cols) {
#pragma unroll 4
    for (int64_t i = blockIdx.x; i < n_rows; i += gridDim.x) {
      const double h = (double)C_hat[i * ldh + j];
      le += fabs(h) <= thr ? 1u : 0u;
      close += fabs(h - C[i * ldc + j]) <= tol ? 1u : 0u;
    }
  }
  unsigned long long a = le, bcl = close;
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off);
    bcl += __shfl_xor(bcl, off);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wv] = a;
    part[1][wv] = bcl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long sa = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    const unsigned long long sc = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    if (sa) atomicAdd(c + 1, sa);
    if (sc) atomicAdd(c + 3, sc);
  }
}

// The big entries (distinct): c[0] += #{|C_hat| >= thr}, c[2] += #{|C_hat - C|
// <= tol}, and their share of the dense counts is subtracted from c[1], c[3]
// (two's-complement adds on the unsigned counters).  An entry outside the
// matrix is skipped.
template <typename InT>
__global__ __launch_bounds__(256) void correctness_big_kernel(
    const InT* __restrict__ C_hat, int64_t ldh, const double* __restrict__ C, int64_t ldc,
    int64_t n_rows, int64_t n_cols, const int64_t* __restrict__ rows,
    const int64_t* __restrict__ cols, int64_t n_big, double thr, double tol,
    unsigned long long* __restrict__ c) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool ge = false, le = false, close = false;
  const int64_t i = q < n_big ? rows[q] : -1, j = q < n_big ? cols[q] : -1;
  if (i >= 0 && i < n_rows && j >= 0 && j < n_cols) {
    const double h = (double)C_hat[i * ldh + j];
    ge = fabs(h) >= thr;
    le = fabs(h) <= thr;
    close = fabs(h - C[i * ldc + j]) <= tol;
  }
  const unsigned long long nge = __popcll(__ballot(ge)), nle = __popcll(__ballot(le)),
                           ncl = __popcll(__ballot(close));
  if ((threadIdx.x & 63) == 0) {
    if (nge) atomicAdd(c + 0, nge);
    if (ncl) atomicAdd(c + 2, ncl);
    if (nle) atomicAdd(c + 1, 0ull - nle);
    if (ncl) atomicAdd(c + 3, 0ull - ncl);
  }
}

__global__ void zero_counters_kernel(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

__global__ void zero_counter_kernel(unsigned long long* c) { *c = 0ull; }

template <typename OutT, bool CYC>
cmm_status run(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
               int64_t n_rows, int64_t n_cols, int log2b, int mean, OutT* C, int64_t ldc,
               hipStream_t s) {
  // grid.x walks row tiles (no practical limit), grid.y column tiles
  const int64_t gx = (n_rows + kRows - 1) / kRows;
  const int64_t gy = (n_cols + kCols - 1) / kCols;
  if (gx > 0x7FFFFFFF || gy > 65535) {
    set_error("cmm_extract: n_cols above 65535 * 256 is not supported");
    return CMM_EUNSUPPORTED;
  }
  dim3 grid((unsigned)gx, (unsigned)gy);
#define CMM_EXTRACT_CASE(DV)                                                                  \
  case DV:                                                                                    \
    hipLaunchKernelGGL((extract_kernel<OutT, DV, CYC>), grid, dim3(kCols), 0, s, p, tab1,     \
                       tab2, n_rows, n_cols, log2b, mean, C, ldc);                            \
    break;
  switch (d) {
    CMM_EXTRACT_CASE(1)
    CMM_EXTRACT_CASE(3)
    CMM_EXTRACT_CASE(5)
    CMM_EXTRACT_CASE(7)
    CMM_EXTRACT_CASE(9)
    CMM_EXTRACT_CASE(11)
    CMM_EXTRACT_CASE(13)
    CMM_EXTRACT_CASE(15)
    CMM_EXTRACT_CASE(17)
    CMM_EXTRACT_CASE(19)
    CMM_EXTRACT_CASE(21)
    default:
      hipLaunchKernelGGL((extract_generic_kernel<OutT, CYC>), grid, dim3(kCols), 0, s, p, tab1, tab2, d,
                         n_rows, n_cols, log2b, mean, C, ldc);
  }
#undef CMM_EXTRACT_CASE
  return hip_check(hipGetLastError(), "extract kernel launch");
}

}  // namespace

cmm_status launch_extract(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                          int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                          void* C_hat, cmm_dtype out_dt, int64_t ldc, hipStream_t s, bool cyclic) {
  ProfScope prof_("extract", s);
  const int mean = est == CMM_MEAN;
  if (cyclic) {
    if (out_dt == CMM_F64)
      return run<double, true>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, (double*)C_hat, ldc, s);
    return run<float, true>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, (float*)C_hat, ldc, s);
  }
  if (out_dt == CMM_F64)
    return run<double, false>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, (double*)C_hat, ldc, s);
  return run<float, false>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, (float*)C_hat, ldc, s);
}

cmm_status launch_extract_entries(const double* p, const uint32_t* tab1, const uint32_t* tab2,
                                  int d, int64_t n_rows, int64_t n_cols, int log2b,
                                  cmm_estimator est, const int64_t* rows, const int64_t* cols,
                                  int64_t count, void* out, cmm_dtype out_dt, hipStream_t s) {
  ProfScope prof_("extract_entries", s);
  const int mean = est == CMM_MEAN;
  const int64_t blocks = (count + 255) / 256;
  if (blocks > 0x7FFFFFFF) { set_error("cmm_extract_entries: too many entries"); return CMM_EUNSUPPORTED; }
  if (out_dt == CMM_F64)
    hipLaunchKernelGGL(extract_entries_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, p,
                       tab1, tab2, d, n_rows, n_cols, log2b, mean, rows, cols, count,
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL(extract_entries_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, p,
                       tab1, tab2, d, n_rows, n_cols, log2b, mean, rows, cols, count,
                       static_cast<float*>(out));
  return hip_check(hipGetLastError(), "extract_entries kernel launch");
}

template <typename OutT>
static cmm_status heavy_run(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                            int64_t n_rows, int64_t n_cols, int log2b, int mean, double thr,
                            int64_t* rows, int64_t* cols, OutT* vals, int64_t capacity,
                            unsigned long long* count, hipStream_t s) {
  const int64_t gx = (n_rows + kRows - 1) / kRows;
  const int64_t gy = (n_cols + kCols - 1) / kCols;
  if (gx > 0x7FFFFFFF || gy > 65535) {
    set_error("cmm_extract_heavy: n_cols above 65535 * 256 is not supported");
    return CMM_EUNSUPPORTED;
  }
  const dim3 grid((unsigned)gx, (unsigned)gy);
#define CMM_HEAVY_CASE(DV)                                                                      \
  case DV:                                                                                      \
    hipLaunchKernelGGL((heavy_kernel<OutT, DV>), grid, dim3(kCols), 0, s, p, tab1, tab2, n_rows, \
                       n_cols, log2b, mean, thr, rows, cols, vals, capacity, count);            \
    break;
  switch (d) {
    CMM_HEAVY_CASE(1)
    CMM_HEAVY_CASE(3)
    CMM_HEAVY_CASE(5)
    CMM_HEAVY_CASE(7)
    CMM_HEAVY_CASE(9)
    CMM_HEAVY_CASE(11)
    CMM_HEAVY_CASE(13)
    CMM_HEAVY_CASE(15)
    CMM_HEAVY_CASE(17)
    CMM_HEAVY_CASE(19)
    CMM_HEAVY_CASE(21)
    default:
      hipLaunchKernelGGL(heavy_generic_kernel<OutT>, grid, dim3(kCols), 0, s, p, tab1, tab2, d,
                         n_rows, n_cols, log2b, mean, thr, rows, cols, vals, capacity, count);
  }
#undef CMM_HEAVY_CASE
  return hip_check(hipGetLastError(), "heavy kernel launch");
}

cmm_status launch_extract_heavy(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                                int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                                double threshold, int64_t* rows, int64_t* cols, void* vals,
                                cmm_dtype out_dt, int64_t capacity, int64_t* count,
                                hipStream_t s) {
  ProfScope prof_("extract_heavy", s);
  unsigned long long* c = reinterpret_cast<unsigned long long*>(count);
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, c);
  cmm_status st = hip_check(hipGetLastError(), "heavy counter reset");
  if (st != CMM_OK || n_rows == 0 || n_cols == 0) return st;
  const int mean = est == CMM_MEAN;
  if (out_dt == CMM_F64)
    return heavy_run<double>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, threshold, rows, cols,
                             static_cast<double*>(vals), capacity, c, s);
  return heavy_run<float>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, threshold, rows, cols,
                          static_cast<float*>(vals), capacity, c, s);
}

cmm_status launch_extract_reps(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                               int64_t n_rows, int64_t n_cols, int log2b, const int64_t* rows,
                               const int64_t* cols, int64_t count, void* out, cmm_dtype out_dt,
                               hipStream_t s) {
  ProfScope prof_("extract_reps", s);
  const int64_t blocks = (count + 255) / 256;
  if (blocks > 0x7FFFFFFF) {
    set_error("cmm_extract_reps: count too large");
    return CMM_EUNSUPPORTED;
  }
  dim3 grid((unsigned)blocks, (unsigned)(d < 65535 ? d : 65535));
  if (out_dt == CMM_F64)
    hipLaunchKernelGGL(extract_reps_kernel<double>, grid, dim3(256), 0, s, p, tab1, tab2, d, n_rows,
                       n_cols, log2b, rows, cols, count, static_cast<double*>(out));
  else
    hipLaunchKernelGGL(extract_reps_kernel<float>, grid, dim3(256), 0, s, p, tab1, tab2, d, n_rows,
                       n_cols, log2b, rows, cols, count, static_cast<float*>(out));
  return hip_check(hipGetLastError(), "extract_reps kernel launch");
}

template <typename InT>
static cmm_status correctness_run(const InT* C_hat, int64_t ldh, const double* C, int64_t ldc,
                                  int64_t n_rows, int64_t n_cols, const int64_t* rows,
                                  const int64_t* cols, int64_t n_big, double thr, double tol,
                                  unsigned long long* c, hipStream_t s) {
  const int64_t gy = (n_cols + 255) / 256;
  if (gy > 65535 || (n_big + 255) / 256 > 0x7FFFFFFF) {
    set_error("cmm_correctness_counts: size not supported");
    return CMM_EUNSUPPORTED;
  }
  if (n_rows > 0 && n_cols > 0) {
    // about 4096 blocks in all: each thread then covers n_rows / gx rows
    const int64_t want = (4096 + gy - 1) / gy;
    const int64_t gx = n_rows < want ? n_rows : want;
    hipLaunchKernelGGL(correctness_dense_kernel<InT>, dim3((unsigned)gx, (unsigned)gy), dim3(256),
                       0, s, C_hat, ldh, C, ldc, n_rows, n_cols, thr, tol, c);
    cmm_status st = hip_check(hipGetLastError(), "correctness kernel launch");
    if (st != CMM_OK) return st;
  }
  if (n_big > 0) {
    hipLaunchKernelGGL(correctness_big_kernel<InT>, dim3((unsigned)((n_big + 255) / 256)),
                       dim3(256), 0, s, C_hat, ldh, C, ldc, n_rows, n_cols, rows, cols, n_big, thr,
                       tol, c);
    return hip_check(hipGetLastError(), "correctness kernel launch");
  }
  return CMM_OK;
}

cmm_status launch_correctness(const void* C_hat, cmm_dtype dt, int64_t ldh, const double* C,
                              int64_t ldc, int64_t n_rows, int64_t n_cols, const int64_t* rows,
                              const int64_t* cols, int64_t n_big, double thr, double tol,
                              int64_t* counts, hipStream_t s) {
  ProfScope prof_("correctness", s);
  unsigned long long* c = reinterpret_cast<unsigned long long*>(counts);
  hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, s, c, 4);
  cmm_status st = hip_check(hipGetLastError(), "correctness counter reset");
  if (st != CMM_OK) return st;
  if (dt == CMM_F64)
    return correctness_run<double>(static_cast<const double*>(C_hat), ldh, C, ldc, n_rows, n_cols,
                                   rows, cols, n_big, thr, tol, c, s);
  return correctness_run<float>(static_cast<const float*>(C_hat), ldh, C, ldc, n_rows, n_cols,
                                rows, cols, n_big, thr, tol, c, s);
}

}  // namespace cmm
