// Hash tables, zero fill, partial reduction and the standalone accumulate.
#include "cmm_internal.h"

namespace cmm {
namespace {

// Section 4.2: v = (a x + c) mod 2^64 (unsigned 64-bit wrap), bucket = the
// log2b top bits of v; the sign hash keeps the single top bit.  With ADD
// false this is multiply-shift: the additive word is dropped and the
// multiplier made odd.
template <bool ADD>
__global__ void hash_kernel(const uint64_t* __restrict__ keys, int64_t n_rows, int64_t n_cols,
                            int log2b, uint32_t* __restrict__ tab1, uint32_t* __restrict__ tab2) {
  const int t = blockIdx.y;
  const uint64_t* k = keys + 8 * (size_t)t;
  const uint64_t odd = ADD ? 0 : 1;
  const uint64_t a1 = k[0] | odd, c1 = ADD ? k[1] : 0, a2 = k[2] | odd, c2 = ADD ? k[3] : 0;
  const uint64_t as1 = k[4] | odd, cs1 = ADD ? k[5] : 0, as2 = k[6] | odd, cs2 = ADD ? k[7] : 0;
  const int shift = 64 - log2b;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n = n_rows > n_cols ? n_rows : n_cols;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    const uint64_t ux = (uint64_t)x;
    if (x < n_rows) {
      const uint32_t h = (uint32_t)((a1 * ux + c1) >> shift);
      const uint32_t s = (uint32_t)((as1 * ux + cs1) >> 63);
      tab1[(size_t)t * n_rows + x] = h | (s << 31);
    }
    if (x < n_cols) {
      const uint32_t h = (uint32_t)((a2 * ux + c2) >> shift);
      const uint32_t s = (uint32_t)((as2 * ux + cs2) >> 63);
      tab2[(size_t)t * n_cols + x] = h | (s << 31);
    }
  }
}

// Simple tabulation (Patrascu and Thorup): the 32-bit index is cut into
// four bytes and the hash is the xor of one random 64-bit word per byte,
// from the byte's own table; bucket = the log2b top bits, sign = the top
// bit of the sign function.  The 16 tables of repetition t (h1, h2, s1, s2
// x 4 bytes x 256 words = 32 KB) are staged in LDS once per block.
__global__ __launch_bounds__(256) void hash_tabulation_kernel(
    const uint64_t* __restrict__ keys, int64_t n_rows, int64_t n_cols, int log2b,
    uint32_t* __restrict__ tab1, uint32_t* __restrict__ tab2) {
  __shared__ uint64_t T[4 * 4 * 256];
  const int t = blockIdx.y;
  const uint64_t* k = keys + (size_t)t * (4 * 4 * 256);
  for (int q = threadIdx.x; q < 4 * 4 * 256; q += blockDim.x) T[q] = k[q];
  __syncthreads();
  auto h = [&](int f, uint32_t x) -> uint64_t {
    const uint64_t* Tf = T + f * 1024;
    return Tf[x & 0xFF] ^ Tf[256 + ((x >> 8) & 0xFF)] ^ Tf[512 + ((x >> 16) & 0xFF)] ^
           Tf[768 + (x >> 24)];
  };
  const int shift = 64 - log2b;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n = n_rows > n_cols ? n_rows : n_cols;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    const uint32_t ux = (uint32_t)x;
    if (x < n_rows)
      tab1[(size_t)t * n_rows + x] = (uint32_t)(h(0, ux) >> shift) | ((uint32_t)(h(2, ux) >> 63) << 31);
    if (x < n_cols)
      tab2[(size_t)t * n_cols + x] = (uint32_t)(h(1, ux) >> shift) | ((uint32_t)(h(3, ux) >> 63) << 31);
  }
}

__global__ void zero_kernel(double* __restrict__ x, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

__global__ void reduce_partials_kernel(const double* __restrict__ parts, int g, size_t len,
                                       double* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    double s = 0.0;
    for (int q = 0; q < g; ++q) s += parts[(size_t)q * len + i];
    out[i] = s;
  }
}

// p_hat[t][u] += sum_kk X[t][kk][u] * Y[t][kk][u], kk ascending.  The
// product is rounded before the add (no contraction), matching a plain
// multiply-then-add.  float32 operands are widened first: the float64
// product of two float32 values is exact.
template <typename T>
__global__ void accumulate_kernel(const T* __restrict__ X, const T* __restrict__ Y, int64_t kc,
                                  int64_t b, double* __restrict__ p_hat) {
#pragma clang fp contract(off)
  const int t = blockIdx.y;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < b; u += stride) {
    double acc = p_hat[(size_t)t * b + u];
    const T* xp = X + (size_t)t * kc * b + u;
    const T* yp = Y + (size_t)t * kc * b + u;
    // the loads of 8 values of kk are issued before their adds, which stay
    // in ascending kk order
    int64_t kk = 0;
    for (; kk + 8 <= kc; kk += 8) {
      T xv[8], yv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        xv[j] = xp[(kk + j) * b];
        yv[j] = yp[(kk + j) * b];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double prod = (double)xv[j] * (double)yv[j];
        acc = acc + prod;
      }
    }
    for (; kk < kc; ++kk) {
      const double prod = (double)xp[kk * b] * (double)yp[kk * b];
      acc = acc + prod;
    }
    p_hat[(size_t)t * b + u] = acc;
  }
}

inline unsigned grid_for(size_t n, unsigned block, unsigned cap = 65535u * 4) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

cmm_status launch_hash(const uint64_t* keys, int d, int64_t n_rows, int64_t n_cols, int log2b,
                       uint32_t* tab1, uint32_t* tab2, hipStream_t s) {
  ProfScope prof_("hash", s);
  const int64_t n = n_rows > n_cols ? n_rows : n_cols;
  dim3 grid(grid_for((size_t)n, 256, 4096), d);
  hipLaunchKernelGGL(hash_kernel<true>, grid, dim3(256), 0, s, keys, n_rows, n_cols, log2b, tab1,
                     tab2);
  return hip_check(hipGetLastError(), "hash kernel launch");
}

cmm_status launch_hash_family(cmm_hash_kind kind, const uint64_t* keys, int d, int64_t n_rows,
                              int64_t n_cols, int log2b, uint32_t* tab1, uint32_t* tab2,
                              hipStream_t s) {
  if (kind == CMM_HASH_MULTIPLY_ADD_SHIFT)
    return launch_hash(keys, d, n_rows, n_cols, log2b, tab1, tab2, s);
  ProfScope prof_("hash", s);
  const int64_t n = n_rows > n_cols ? n_rows : n_cols;
  if (kind == CMM_HASH_MULTIPLY_SHIFT) {
    dim3 grid(grid_for((size_t)n, 256, 4096), d);
    hipLaunchKernelGGL(hash_kernel<false>, grid, dim3(256), 0, s, keys, n_rows, n_cols, log2b,
                       tab1, tab2);
  } else {
    // each block stages 32 KB of tables: give it a few thousand indices
    dim3 grid(grid_for((size_t)n, 256 * 8, 1024), d);
    hipLaunchKernelGGL(hash_tabulation_kernel, grid, dim3(256), 0, s, keys, n_rows, n_cols, log2b,
                       tab1, tab2);
  }
  return hip_check(hipGetLastError(), "hash kernel launch");
}

cmm_status launch_zero(double* x, size_t n, hipStream_t s) {
  if (n == 0) return CMM_OK;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, x, n);
  return hip_check(hipGetLastError(), "zero kernel launch");
}

cmm_status launch_reduce_partials(const double* parts, int g, size_t len, double* out,
                                  hipStream_t s) {
  if (len == 0) return CMM_OK;
  ProfScope prof_("reduce", s);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(grid_for(len, 256, 8192)), dim3(256), 0, s,
                     parts, g, len, out);
  return hip_check(hipGetLastError(), "reduce kernel launch");
}

cmm_status launch_accumulate(const void* X, const void* Y, cmm_dtype dt, int d, int64_t kc,
                             int log2b, double* p_hat, hipStream_t s) {
  ProfScope prof_("accumulate", s);
  const int64_t b = (int64_t)1 << log2b;
  dim3 grid(grid_for((size_t)b, 256, 4096), d);
  if (dt == CMM_F64)
    hipLaunchKernelGGL(accumulate_kernel<double>, grid, dim3(256), 0, s, (const double*)X,
                       (const double*)Y, kc, b, p_hat);
  else
    hipLaunchKernelGGL(accumulate_kernel<float>, grid, dim3(256), 0, s, (const float*)X,
                       (const float*)Y, kc, b, p_hat);
  return hip_check(hipGetLastError(), "accumulate kernel launch");
}

}  // namespace cmm
