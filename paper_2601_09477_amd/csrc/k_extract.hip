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

template <typename OutT, int D>
__global__ __launch_bounds__(kCols) void extract_kernel(
    const double* __restrict__ p, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int64_t n_rows, int64_t n_cols, int log2b, int mean,
    OutT* __restrict__ C, int64_t ldc) {
  const int64_t j = (int64_t)blockIdx.y * kCols + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kRows;
  const int64_t b = (int64_t)1 << log2b;
  const uint32_t bmask = (uint32_t)(b - 1);
  const bool jok = j < n_cols;
  double v[kRows][D];
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const uint32_t e2 = jok ? tab2[(size_t)t * n_cols + j] : 0u;
    const double* pt = p + (size_t)t * b;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int64_t i = i0 + r < n_rows ? i0 + r : n_rows - 1;
      const uint32_t e = tab1[(size_t)t * n_rows + i] ^ e2;
      const double x = pt[e & bmask];
      v[r][t] = (e & kSignBit) ? -x : x;
    }
  }
  if (!jok) return;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    if (i0 + r >= n_rows) break;
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
    C[(i0 + r) * ldc + j] = (OutT)out;
  }
}

// Generic d (up to kMaxD): candidates in a local array, insertion sort.
constexpr int kMaxD = 63;
template <typename OutT>
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
      const uint32_t e = tab1[(size_t)t * n_rows + i] ^ tab2[(size_t)t * n_cols + j];
      const double x = p[(size_t)t * b + (e & (uint32_t)(b - 1))];
      const double y = (e & kSignBit) ? -x : x;
      s += y;
      int q = t;
      while (q > 0 && v[q - 1] > y) { v[q] = v[q - 1]; --q; }
      v[q] = y;
    }
    C[i * ldc + j] = (OutT)(mean ? s / d : v[d / 2]);
  }
}

template <typename OutT>
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
    hipLaunchKernelGGL((extract_kernel<OutT, DV>), grid, dim3(kCols), 0, s, p, tab1, tab2,    \
                       n_rows, n_cols, log2b, mean, C, ldc);                                  \
    break;
  switch (d) {
    CMM_EXTRACT_CASE(1)
    CMM_EXTRACT_CASE(3)
    CMM_EXTRACT_CASE(5)
    CMM_EXTRACT_CASE(7)
    CMM_EXTRACT_CASE(9)
    CMM_EXTRACT_CASE(11)
    default:
      hipLaunchKernelGGL(extract_generic_kernel<OutT>, grid, dim3(kCols), 0, s, p, tab1, tab2, d,
                         n_rows, n_cols, log2b, mean, C, ldc);
  }
#undef CMM_EXTRACT_CASE
  return hip_check(hipGetLastError(), "extract kernel launch");
}

}  // namespace

cmm_status launch_extract(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                          int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                          void* C_hat, cmm_dtype out_dt, int64_t ldc, hipStream_t s) {
  ProfScope prof_("extract", s);
  const int mean = est == CMM_MEAN;
  if (out_dt == CMM_F64)
    return run<double>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, (double*)C_hat, ldc, s);
  return run<float>(p, tab1, tab2, d, n_rows, n_cols, log2b, mean, (float*)C_hat, ldc, s);
}

}  // namespace cmm
