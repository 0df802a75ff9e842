// Standalone count sketch (Algorithm 1, the two sketch loops of Compress).
//
// One wavefront owns one output vector (t, kk) and accumulates it in an LDS
// window of kWin buckets, sweeping the bucket range window by window.  Input
// indices are consumed 64 at a time in ascending order; lanes of a group
// that hit the same bucket are applied in lane order (rank rounds), so every
// bucket receives its terms in ascending index order -- the result does not
// depend on scheduling and equals a sequential left-to-right sum.
#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr int kWaves = 4;

template <typename T>
struct SketchWin { static constexpr int value = 4096; };       // 32 KB of f64 per wave
template <>
struct SketchWin<float> { static constexpr int value = 8192; };  // 32 KB of f32 per wave

template <typename T>
__global__ __launch_bounds__(64 * kWaves) void sketch_kernel(
    int side, const T* __restrict__ M, int64_t ld, const uint32_t* __restrict__ tab,
    int64_t n_idx, int log2b, int64_t k0, int64_t kc, int d, T* __restrict__ out) {
  constexpr int W = SketchWin<T>::value;
  __shared__ T win[kWaves][W];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * kWaves + wv;   // t * kc + kk
  if (col >= (int64_t)d * kc) return;                      // whole wave exits together
  const int t = (int)(col / kc);
  const int64_t kk = col - (int64_t)t * kc;
  const int64_t b = (int64_t)1 << log2b;
  const int win_bits = log2b < 12 ? log2b : (sizeof(T) == 8 ? 12 : 13);
  const int64_t wlen = (int64_t)1 << win_bits;
  const uint32_t* tb = tab + (size_t)t * n_idx;
  T* dst = out + (size_t)col * b;
  T* lds = win[wv];

  for (int64_t w0 = 0; w0 < b; w0 += wlen) {
    for (int64_t x = lane; x < wlen; x += 64) lds[x] = T(0);
    for (int64_t g0 = 0; g0 < n_idx; g0 += 64) {
      const int64_t idx = g0 + lane;
      uint32_t key = 0xFFFFFFFFu;   // lanes outside the window never match a bucket
      T v = T(0);
      if (idx < n_idx) {
        const uint32_t e = tb[idx];
        const int64_t x = (int64_t)(e & (uint32_t)(b - 1));
        if (x >= w0 && x < w0 + wlen) {
          key = (uint32_t)(x - w0);
          const T m = side == 0 ? M[idx * ld + (k0 + kk)] : M[(k0 + kk) * ld + idx];
          v = (e & kSignBit) ? -m : m;
        }
      }
      // rank = number of lower lanes with the same key
      int rank = 0;
      int any = 0;
      for (int j = 0; j < 64; ++j) {
        const uint32_t kj = (uint32_t)__builtin_amdgcn_readlane((int)key, j);
        any |= (kj != 0xFFFFFFFFu);
        rank += (j < lane && kj == key) ? 1 : 0;
      }
      if (!any) continue;
      int maxr = rank;
      for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(maxr, off);
        maxr = o > maxr ? o : maxr;
      }
      for (int r = 0; r <= maxr; ++r) {
        // LDS accesses of one wavefront complete in program order, so round
        // r + 1 reads what round r wrote.
        if (key != 0xFFFFFFFFu && rank == r) lds[key] = lds[key] + v;
      }
    }
    for (int64_t x = lane; x < wlen; x += 64) dst[w0 + x] = lds[x];
  }
}

}  // namespace

cmm_status launch_sketch(int side, const void* M, cmm_dtype dt, int64_t rows, int64_t cols,
                         int64_t ld, const uint32_t* tab, int d, int log2b, int64_t k0,
                         int64_t kc, void* out, hipStream_t s) {
  ProfScope prof_("sketch", s);
  const int64_t n_idx = side == 0 ? rows : cols;
  const int64_t ncol = (int64_t)d * kc;
  const int64_t blocks = (ncol + kWaves - 1) / kWaves;
  if (blocks > 0x7FFFFFFF) return invalid("cmm_sketch: d * kc too large");
  if (dt == CMM_F64)
    hipLaunchKernelGGL(sketch_kernel<double>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, s,
                       side, (const double*)M, ld, tab, n_idx, log2b, k0, kc, d, (double*)out);
  else
    hipLaunchKernelGGL(sketch_kernel<float>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, s,
                       side, (const float*)M, ld, tab, n_idx, log2b, k0, kc, d, (float*)out);
  return hip_check(hipGetLastError(), "sketch kernel launch");
}

}  // namespace cmm
