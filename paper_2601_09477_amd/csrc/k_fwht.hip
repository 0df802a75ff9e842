// Standalone in-place Walsh-Hadamard transform of batched vectors in HBM
// (Section 3.2: +-1 butterflies only, natural order, in place).
//
// The log2b index bits are processed in passes through HBM; the final pass
// applies the power-of-two scale.  For b >= 4096:
//  * the low 12 bits in one pass over tiles of 4096 contiguous elements: the
//    top 4 tile bits as radix-16 in registers straight from global memory
//    (coalesced), the middle 4 and the low 4 through LDS, then vector stores;
//  * every further 4 bits (or fewer) in a register-only pass: a thread owns
//    one column of 2^P elements at stride 2^s, and consecutive threads own
//    consecutive columns, so every access is coalesced.
// Shorter vectors take the general pass: a bit range [s, s + P) over tiles of
// 2^P x W elements (W consecutive low indices) moved through LDS, one LDS
// round trip per 4 bits.
#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr int kTileBits = 12;   // 4096 elements per tile (32 KB of f64)
constexpr int kThreads = 256;

__device__ __forceinline__ int pad(int e) { return e + (e >> 4); }

template <typename T, int R>
__device__ __forceinline__ void wht_regs(T (&v)[16]) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if ((i & h) == 0) {
        const T a = v[i], c = v[i + h];
        v[i] = a + c;
        v[i + h] = a - c;
      }
    }
  }
}

// One sub-pass: butterflies on tile-index bits [bs, bs + rb) for all groups.
template <typename T, int R>
__device__ __forceinline__ void subpass(T* lds, int le, int bs) {
  const int groups = (1 << le) / R;
  const int lowmask = (1 << bs) - 1;
  for (int g = threadIdx.x; g < groups; g += kThreads) {
    const int base = (g & lowmask) | ((g >> bs) << (bs + __builtin_ctz(R)));
    T v[16];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = lds[pad(base + (r << bs))];
    wht_regs<T, R>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) lds[pad(base + (r << bs))] = v[r];
  }
}

template <typename T>
__device__ __forceinline__ void subpass_dispatch(T* lds, int le, int bs, int rb) {
  switch (rb) {
    case 1: subpass<T, 2>(lds, le, bs); break;
    case 2: subpass<T, 4>(lds, le, bs); break;
    case 3: subpass<T, 8>(lds, le, bs); break;
    default: subpass<T, 16>(lds, le, bs); break;
  }
}

// Pass over vector-index bits [s, s + P).  Tile element e (le bits):
//  s == 0: e = v_local * 2^P + m (whole consecutive vectors, contiguous);
//  s  > 0: e = m * W + w, global index = hi * 2^(s+P) + m * 2^s + w0 + w.
template <typename T>
__global__ __launch_bounds__(kThreads) void fwht_pass_kernel(T* __restrict__ x, int64_t batch,
                                                             int log2b, int s, int P, int logW,
                                                             T scale, int apply_scale) {
  __shared__ T lds[(1 << kTileBits) + (1 << (kTileBits - 4))];
  const int64_t b = (int64_t)1 << log2b;
  const int le = P + logW;
  const int E = 1 << le;
  const int64_t tile = blockIdx.x;
  // Global offset of tile element e, or -1 when outside the batch.
  auto gidx = [&](int e) -> int64_t {
    if (s == 0) {
      const int64_t g = tile * E + e;                      // logW counts whole vectors
      return g < batch * b ? g : -1;
    }
    const int64_t tiles_per_vec = (int64_t)1 << (log2b - le);
    const int64_t vec = tile / tiles_per_vec;
    const int64_t r = tile - vec * tiles_per_vec;
    const int64_t lows = (int64_t)1 << (s - logW);          // W-blocks of low bits
    const int64_t hi = r / lows, wblk = r - hi * lows;
    const int m = e >> logW, w = e & ((1 << logW) - 1);
    return vec * b + (hi << (s + P)) + ((int64_t)m << s) + (wblk << logW) + w;
  };
  for (int e = threadIdx.x; e < E; e += kThreads) {
    const int64_t g = gidx(e);
    lds[pad(e)] = g >= 0 ? x[g] : T(0);
  }
  __syncthreads();
  // butterfly bits inside the tile index: [logW, logW + P) for s > 0,
  // [0, P) for s == 0 (there logW holds the vector bits above P).
  const int bit0 = s == 0 ? 0 : logW;
  for (int q = 0; q < P; q += 4) {
    const int rb = (P - q) < 4 ? (P - q) : 4;
    subpass_dispatch<T>(lds, le, bit0 + q, rb);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < E; e += kThreads) {
    const int64_t g = gidx(e);
    if (g >= 0) x[g] = apply_scale ? lds[pad(e)] * scale : lds[pad(e)];
  }
}

template <typename T>
__device__ __forceinline__ void radix16(T (&v)[16]) {
#pragma unroll
  for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if ((i & h) == 0) {
        const T a = v[i], c = v[i + h];
        v[i] = a + c;
        v[i + h] = a - c;
      }
    }
  }
}

template <typename T> struct Pair;
template <> struct Pair<double> { typedef double2 type; };
template <> struct Pair<float> { typedef float2 type; };

// Low 12 bits of vectors of length >= 4096: one work-group per tile of 4096
// contiguous elements (element e of the tile at x[tile * 4096 + e]).
// VEC: x is aligned to two elements, so the stores go out in pairs.
template <typename T, bool VEC>
__global__ __launch_bounds__(kThreads) void fwht_low12_kernel(T* __restrict__ x, T scale,
                                                              int apply_scale) {
  __shared__ T lds[(1 << kTileBits) + (1 << (kTileBits - 4))];
  T* xt = x + ((int64_t)blockIdx.x << kTileBits);
  const int tid = threadIdx.x;
  T v[16];
  // bits 8..11: element tid + 256 r
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = xt[tid + (r << 8)];
  radix16(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) lds[pad(tid + (r << 8))] = v[r];
  __syncthreads();
  // bits 4..7: element (tid & 15) | r << 4 | (tid >> 4) << 8
  const int b1 = (tid & 15) | ((tid >> 4) << 8);
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[pad(b1 + (r << 4))];
  radix16(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) lds[pad(b1 + (r << 4))] = v[r];
  __syncthreads();
  // bits 0..3: the 16 consecutive elements 16 tid + r
  const int b2 = tid << 4;
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[pad(b2 + r)];
  radix16(v);
  if (apply_scale) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = v[r] * scale;
  }
  if (VEC) {
    typedef typename Pair<T>::type T2;
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      T2 q;
      q.x = v[r];
      q.y = v[r + 1];
      *reinterpret_cast<T2*>(xt + b2 + r) = q;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) xt[b2 + r] = v[r];
  }
}

// Bits [s, s + P), P <= 4, s >= 12: column c (of batch * b / 2^P) holds the
// elements ((c >> s) << (s + P)) + (c & (2^s - 1)) + m 2^s, m < 2^P.
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void fwht_cols_kernel(T* __restrict__ x, int64_t ncols,
                                                             int s, T scale, int apply_scale) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= ncols) return;
  T* xc = x + (((c >> s) << (s + P)) + (c & (((int64_t)1 << s) - 1)));
  T v[16];
#pragma unroll
  for (int m = 0; m < (1 << P); ++m) v[m] = xc[(int64_t)m << s];
  wht_regs<T, (1 << P)>(v);
#pragma unroll
  for (int m = 0; m < (1 << P); ++m) xc[(int64_t)m << s] = apply_scale ? v[m] * scale : v[m];
}

template <typename T>
cmm_status run(T* x, int64_t batch, int log2b, double scale, hipStream_t st) {
  if (log2b >= kTileBits) {
    if (batch > ((int64_t)0x7FFFFFFF >> (log2b - kTileBits)))
      return invalid("cmm_fwht: batch too large");
    const int64_t tiles = batch << (log2b - kTileBits);
    const bool vec = (reinterpret_cast<uintptr_t>(x) % (2 * sizeof(T))) == 0;
    auto low = vec ? fwht_low12_kernel<T, true> : fwht_low12_kernel<T, false>;
    hipLaunchKernelGGL(low, dim3((unsigned)tiles), dim3(kThreads), 0, st, x, (T)scale,
                       log2b == kTileBits && scale != 1.0);
    cmm_status r = hip_check(hipGetLastError(), "fwht pass launch");
    for (int s = kTileBits; r == CMM_OK && s < log2b;) {
      const int P = log2b - s < 4 ? log2b - s : 4;
      const int64_t ncols = (batch << log2b) >> P;
      const int64_t blocks = (ncols + kThreads - 1) / kThreads;
      if (blocks > 0x7FFFFFFF) return invalid("cmm_fwht: batch too large");
      const int last = s + P >= log2b && scale != 1.0;
      switch (P) {
        case 1: hipLaunchKernelGGL((fwht_cols_kernel<T, 1>), dim3((unsigned)blocks), dim3(kThreads), 0, st, x, ncols, s, (T)scale, last); break;
        case 2: hipLaunchKernelGGL((fwht_cols_kernel<T, 2>), dim3((unsigned)blocks), dim3(kThreads), 0, st, x, ncols, s, (T)scale, last); break;
        case 3: hipLaunchKernelGGL((fwht_cols_kernel<T, 3>), dim3((unsigned)blocks), dim3(kThreads), 0, st, x, ncols, s, (T)scale, last); break;
        default: hipLaunchKernelGGL((fwht_cols_kernel<T, 4>), dim3((unsigned)blocks), dim3(kThreads), 0, st, x, ncols, s, (T)scale, last); break;
      }
      r = hip_check(hipGetLastError(), "fwht pass launch");
      s += P;
    }
    return r;
  }
  int s = 0;
  while (s < log2b) {
    int P, logW;
    if (s == 0) {
      P = log2b < kTileBits ? log2b : kTileBits;
      // pack whole vectors into a tile when they are short
      int vb = kTileBits - P;
      while (vb > 0 && ((int64_t)1 << vb) > batch) --vb;
      logW = vb;
    } else {
      const int rem = log2b - s;
      P = rem < 8 ? rem : 8;
      logW = (kTileBits - P) < s ? (kTileBits - P) : s;
    }
    const int le = P + logW;
    int64_t tiles;
    if (s == 0)
      tiles = (batch * ((int64_t)1 << log2b) + ((int64_t)1 << le) - 1) >> le;
    else
      tiles = batch << (log2b - le);
    if (tiles > 0x7FFFFFFF) return invalid("cmm_fwht: batch too large");
    const int last = (s + P) >= log2b;
    hipLaunchKernelGGL(fwht_pass_kernel<T>, dim3((unsigned)tiles), dim3(kThreads), 0, st, x,
                       batch, log2b, s, P, logW, (T)scale, last && scale != 1.0);
    cmm_status r = hip_check(hipGetLastError(), "fwht pass launch");
    if (r != CMM_OK) return r;
    s += P;
  }
  return CMM_OK;
}

}  // namespace

cmm_status launch_fwht(void* x, cmm_dtype dt, int64_t batch, int log2b, double scale,
                       hipStream_t s) {
  ProfScope prof_("fwht", s);
  if (dt == CMM_F64) return run<double>((double*)x, batch, log2b, scale, s);
  return run<float>((float*)x, batch, log2b, scale, s);
}

}  // namespace cmm
