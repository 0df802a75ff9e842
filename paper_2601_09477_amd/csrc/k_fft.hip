// Pagh's FFT form (Section 3.1): a batched complex discrete Fourier
// transform and the pieces of the staged Compress around it.
//
// Transform: float64 complex, natural order in and out, length N = 2^m with
// m <= 24.  X[k] = scale * sum_n x[n] w^(n k), w = exp(-2 pi i / N) forward,
// exp(+2 pi i / N) inverse.  N <= 4096 is one pass in LDS.  Above that N is
// split as N1 N2 (N1 = 2^ceil(m/2)) and done in two passes (the four-step
// decomposition): pass A transforms the N2 strided sequences x[N2 n1 + n2]
// over n1, multiplies by w_N^(n2 k1) and stores y[n2][k1] contiguously;
// pass B transforms y[.][k1] over n2 in place, which leaves X[k1 + N1 k2]
// at its natural position.  Each work-group takes a tile of consecutive
// sequences (4096 points in all), so both passes read and write whole
// 256-byte runs.  Twiddles come from sincospi of exact rational arguments.
#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr int kTile = 4096;     // points per work-group (64 KB of LDS, 32 KB of roots)
constexpr int kFftThreads = 256;

// exp(sgn * 2 pi i * num / N) for 0 <= num, N a power of two
__device__ __forceinline__ double2 unit_root(int64_t num, int64_t N, int sgn) {
  const int64_t r = num & (N - 1);
  double s, c;
  sincospi(2.0 * (double)r / (double)N, &s, &c);
  return make_double2(c, sgn > 0 ? s : -s);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ uint32_t bit_reverse(uint32_t v, int bits) {
  return __brev(v) >> (32 - bits);
}

// Geometry of one pass: sequence g of vector v has its element e at
// v * N + (g % S) * seq_step + e * elem_stride (input and output each).
struct PassGeom {
  int64_t N;          // vector length
  int64_t S;          // sequences per vector
  int64_t in_step, in_stride, out_step, out_stride;
  int64_t tw_N;       // > 0: multiply output k of sequence s by w_twN^(s k)
};

__global__ __launch_bounds__(kFftThreads) void fft_tile_kernel(
    const double2* __restrict__ in, double2* __restrict__ out, PassGeom G, int logL, int ns,
    int sgn, double scale) {
  extern __shared__ double2 fft_lds[];
  const int L = 1 << logL;
  double2* X = fft_lds;            // ns * L points
  double2* tw = fft_lds + ns * L;  // L / 2 roots
  const int64_t v = blockIdx.y;
  const int64_t s0 = (int64_t)blockIdx.x * ns;     // first sequence of the tile
  const int64_t vbase = v * G.N;
  for (int j = threadIdx.x; j < L / 2; j += kFftThreads) tw[j] = unit_root(j, L, sgn);
  // load, consecutive sequences fastest, into bit-reversed position
  for (int q = threadIdx.x; q < ns * L; q += kFftThreads) {
    const int c = q % ns, e = q / ns;
    X[c * L + bit_reverse((uint32_t)e, logL)] =
        in[vbase + (s0 + c) * G.in_step + (int64_t)e * G.in_stride];
  }
  __syncthreads();
  // in-place radix-2 decimation in time
  for (int h = 1; h < L; h <<= 1) {
    const int step = L / (2 * h);
    for (int q = threadIdx.x; q < ns * (L / 2); q += kFftThreads) {
      const int c = q / (L / 2), r = q % (L / 2);
      const int grp = r / h, j = r % h;
      const int i0 = c * L + grp * 2 * h + j, i1 = i0 + h;
      const double2 t = cmul(X[i1], tw[j * step]);
      const double2 a = X[i0];
      X[i0] = make_double2(a.x + t.x, a.y + t.y);
      X[i1] = make_double2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < ns * L; q += kFftThreads) {
    const int c = q % ns, k = q / ns;
    double2 y = X[c * L + k];
    if (G.tw_N > 0) y = cmul(y, unit_root((s0 + c) * (int64_t)k, G.tw_N, sgn));
    out[vbase + (s0 + c) * G.out_step + (int64_t)k * G.out_stride] =
        make_double2(y.x * scale, y.y * scale);
  }
}

cmm_status launch_pass(const double2* in, double2* out, const PassGeom& G, int logL,
                       int64_t batch, int sgn, double scale, hipStream_t s) {
  const int L = 1 << logL;
  int ns = kTile / L;
  if (ns > G.S) ns = (int)G.S;
  if (ns < 1) {
    set_error("cmm_fft: a pass longer than the LDS tile is not supported (log2n <= 24)");
    return CMM_EUNSUPPORTED;
  }
  const int64_t gx = G.S / ns;
  if (gx > 0x7FFFFFFF || batch > 65535) {
    set_error("cmm_fft: batch above 65535 vectors per launch is not supported");
    return CMM_EUNSUPPORTED;
  }
  const size_t lds = ((size_t)ns * L + L / 2) * sizeof(double2);
  hipError_t e = hipFuncSetAttribute((const void*)fft_tile_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_check(e, "fft kernel LDS size");
  hipLaunchKernelGGL(fft_tile_kernel, dim3((unsigned)gx, (unsigned)batch), dim3(kFftThreads), lds,
                     s, in, out, G, logL, ns, sgn, scale);
  return hip_check(hipGetLastError(), "fft kernel launch");
}

// Z[i] = (X[i], Y[i]): two real sketches as one complex sequence
__global__ void pack_kernel(const double* __restrict__ X, const double* __restrict__ Y,
                            double2* __restrict__ Z, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    Z[i] = make_double2(X[i], Y[i]);
}

// With Z = F(x + i y) for real x, y: F(x)[u] = (Z[u] + conj Z[-u]) / 2 and
// F(y)[u] = (Z[u] - conj Z[-u]) / (2 i), so F(x)[u] F(y)[u] =
// (Z[u]^2 - conj(Z[-u])^2) / (4 i).  P[t][u] += that product for kk
// ascending (fixed order).
__global__ void accumulate_cyclic_kernel(const double2* __restrict__ Z, int64_t kc, int64_t b,
                                         double2* __restrict__ P) {
  const int t = blockIdx.y;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < b; u += stride) {
    const int64_t mu = (b - u) & (b - 1);
    double2 acc = P[(size_t)t * b + u];
    for (int64_t kk = 0; kk < kc; ++kk) {
      const double2* z = Z + ((size_t)t * kc + kk) * b;
      const double2 a = z[u];
      const double2 m = make_double2(z[mu].x, -z[mu].y);   // conj Z[-u]
      // (a^2 - m^2) / (4 i) = -i (a^2 - m^2) / 4
      const double re = a.x * a.x - a.y * a.y - (m.x * m.x - m.y * m.y);
      const double im = 2.0 * a.x * a.y - 2.0 * m.x * m.y;
      acc.x += 0.25 * im;
      acc.y -= 0.25 * re;
    }
    P[(size_t)t * b + u] = acc;
  }
}

__global__ void zero_complex_kernel(double2* __restrict__ x, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    x[i] = make_double2(0.0, 0.0);
}

__global__ void real_part_kernel(const double2* __restrict__ Z, double* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = Z[i].x;
}

inline unsigned blocks_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (unsigned)g;
}

}  // namespace

cmm_status launch_fft(const void* in, void* out, int64_t batch, int log2n, int inverse,
                      double scale, hipStream_t s) {
  ProfScope prof_("fft", s);
  const int sgn = inverse ? 1 : -1;
  const int64_t N = (int64_t)1 << log2n;
  const double2* x = static_cast<const double2*>(in);
  double2* y = static_cast<double2*>(out);
  for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
    const int64_t nb = batch - b0 < 65535 ? batch - b0 : 65535;
    const double2* xi = x + b0 * N;
    double2* yo = y + b0 * N;
    cmm_status st;
    if (log2n <= 12) {
      PassGeom G{N, 1, 0, 1, 0, 1, 0};
      st = launch_pass(xi, yo, G, log2n, nb, sgn, scale, s);
    } else {
      const int l1 = (log2n + 1) / 2, l2 = log2n - l1;
      const int64_t N1 = (int64_t)1 << l1, N2 = (int64_t)1 << l2;
      PassGeom A{N, N2, 1, N2, N1, 1, N};
      st = launch_pass(xi, yo, A, l1, nb, sgn, 1.0, s);
      if (st != CMM_OK) return st;
      PassGeom B{N, N1, 1, N1, 1, N1, 0};
      st = launch_pass(yo, yo, B, l2, nb, sgn, scale, s);
    }
    if (st != CMM_OK) return st;
  }
  return CMM_OK;
}

cmm_status launch_pack(const double* X, const double* Y, void* Z, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(n)), dim3(256), 0, s, X, Y,
                     static_cast<double2*>(Z), n);
  return hip_check(hipGetLastError(), "pack kernel launch");
}

cmm_status launch_accumulate_cyclic(const void* Z, int d, int64_t kc, int log2b, void* P,
                                    hipStream_t s) {
  ProfScope prof_("accumulate", s);
  const int64_t b = (int64_t)1 << log2b;
  dim3 grid(blocks_for((size_t)b), d);
  hipLaunchKernelGGL(accumulate_cyclic_kernel, grid, dim3(256), 0, s,
                     static_cast<const double2*>(Z), kc, b, static_cast<double2*>(P));
  return hip_check(hipGetLastError(), "accumulate kernel launch");
}

cmm_status launch_zero_complex(void* x, size_t n, hipStream_t s) {
  if (n == 0) return CMM_OK;
  hipLaunchKernelGGL(zero_complex_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                     static_cast<double2*>(x), n);
  return hip_check(hipGetLastError(), "zero kernel launch");
}

cmm_status launch_real_part(const void* Z, double* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(real_part_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                     static_cast<const double2*>(Z), p, n);
  return hip_check(hipGetLastError(), "real part kernel launch");
}

}  // namespace cmm
