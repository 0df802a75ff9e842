// Pagh's FFT form (Section 3.1), fused Compress: count sketch, forward
// transforms and the product accumulation over k in one kernel, float64.
//
// The transform is split the way the FWHT kernel splits H_b.  With
// b = b_hi b_lo, b_lo = 4096 and an output frequency u = u_hi + b_hi u_lo,
//   X[u_hi + b_hi u_lo] = DFT_{b_lo}(F_{u_hi})[u_lo],
//   F_{u_hi}[r] = sum over i with h(i) mod b_lo = r of s(i) w_b^(u_hi h(i)) a_i
// (w_b = exp(-2 pi i / b)): a work-group owning the slice u_hi sketches the
// column into b_lo buckets with a complex fold weight per row and runs one
// 4096-point transform per operand and k.  The inputs are real, so
// X[b - u] = conj X[u] and only the slices u_hi <= b_hi / 2 are computed;
// the reduction fills in the others.
//
// Per work unit (t, u_hi, k-range), 512 threads, 8 points per thread:
// * the fold weight of each thread's 8 buckets (their first row's weight)
//   is kept in registers for both operands;
// * a bucket with several rows is merged in place before the gather: the
//   chain's sum relative to its first row, sum of s w_{b_hi}^q a over the
//   rows (a b_hi-th root of unity per row, from a table), is complex; its
//   real part goes to the first row's slot and its imaginary part to the
//   second row's slot, and the gather reads both;
// * the transform is radix-8 decimation in frequency in four stages (8
//   points per thread, exchanges through a padded LDS buffer), leaving the
//   outputs in digit-reversed order, which the pointwise product does not
//   mind; the partial is written to the natural positions;
// * one row buffer: the copy of B's row of k overlaps the transform of X,
//   the copy of A's row of k + 1 the transform of Y.
#include "cmm_internal.h"
#include "wht_regs.h"

namespace cmm {
namespace {

constexpr int kFLB = 12;                     // b_lo = 2^12 complex points
constexpr int kFNT = 512;                    // threads per work-group
constexpr int kXLen = 4096 + 8 * 64;         // padded exchange buffer (complex)

__device__ __forceinline__ int xpad(int idx) { return idx + ((idx >> 6) << 3); }

__device__ __forceinline__ double2 cmulf(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 caddf(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csubf(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// exp(-2 pi i num / N), N a power of two
__device__ __forceinline__ double2 fwd_root(uint64_t num, uint64_t N) {
  double s, c;
  sincospi(2.0 * (double)(num & (N - 1)) / (double)N, &s, &c);
  return make_double2(c, -s);
}

// X[k] = sum_x x[k] w4^(x k), w4 = -i, in place on (v[i0], v[i1], v[i2], v[i3])
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3) {
  const double2 a0 = caddf(x0, x2), a1 = caddf(x1, x3);
  const double2 b0 = csubf(x0, x2);
  const double2 dd = csubf(x1, x3);
  const double2 b1 = make_double2(dd.y, -dd.x);   // (x1 - x3) (-i)
  x0 = caddf(a0, a1);
  x1 = caddf(b0, b1);
  x2 = csubf(a0, a1);
  x3 = csubf(b0, b1);
}

// V[m] = sum_x v[x] w8^(m x), w8 = exp(-2 pi i / 8), in place: pairs (x,
// x + 4) first, the differences turned by w8^x, then two 4-point
// transforms giving the even and the odd outputs.  Every step overwrites
// its inputs, so only the 8 points and two temporaries are live.
__device__ __forceinline__ void dft8(double2 (&v)[8]) {
  constexpr double r = 0.70710678118654752440;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 t = v[k];
    v[k] = caddf(t, v[k + 4]);
    v[k + 4] = csubf(t, v[k + 4]);
  }
  v[5] = make_double2((v[5].x + v[5].y) * r, (v[5].y - v[5].x) * r);     // (1 - i) / sqrt 2
  v[6] = make_double2(v[6].y, -v[6].x);                                  // -i
  v[7] = make_double2((v[7].y - v[7].x) * r, -(v[7].x + v[7].y) * r);    // (-1 - i) / sqrt 2
  dft4(v[0], v[1], v[2], v[3]);   // -> V0, V2, V4, V6
  dft4(v[4], v[5], v[6], v[7]);   // -> V1, V3, V5, V7
  const double2 o1 = v[1], o2 = v[2], o3 = v[3], o4 = v[4], o5 = v[5], o6 = v[6];
  v[1] = o4; v[2] = o1; v[3] = o5; v[4] = o2; v[5] = o6; v[6] = o3;
}

// v[m] *= w^m, m = 1..7, the powers built one at a time
__device__ __forceinline__ void twiddle8(double2 (&v)[8], double2 w) {
  double2 p = w;
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    v[m] = cmulf(v[m], p);
    if (m < 7) p = cmulf(p, w);
  }
}

// 4096-point forward transform; thread tid enters with x[tid + 512 m] in
// v[m] and leaves with X[a + 8 b1 + 64 c2 + 512 m] in v[m], where
// a = tid >> 6, b1 = (tid >> 3) & 7, c2 = tid & 7.  Ends without a barrier:
// the caller separates the last reads from the next use of xb.
__device__ __forceinline__ void fft4096(double2 (&v)[8], double2* __restrict__ xb,
                                        const double2* __restrict__ stw) {
  // Padded positions xpad(i) = i + 8 (i >> 6).  Within each stage the 8
  // points of a thread sit at one base plus fixed steps: m * 512 -> 576,
  // 64 x -> 72, 8 x -> 8, x -> 1 (the low 6 bits never carry).
  const int tid = threadIdx.x;
  const int a = tid >> 6, jp = tid & 63, b1 = (tid >> 3) & 7, jj = tid & 7;
  dft8(v);
  twiddle8(v, stw[tid]);
  double2* p = xb + xpad(tid);
#pragma unroll
  for (int m = 0; m < 8; ++m) p[576 * m] = v[m];
  __syncthreads();
  p = xb + xpad(a * 512 + jp);
#pragma unroll
  for (int x = 0; x < 8; ++x) v[x] = p[72 * x];
  dft8(v);
  twiddle8(v, stw[512 + jp]);
#pragma unroll
  for (int m = 0; m < 8; ++m) p[72 * m] = v[m];
  __syncthreads();
  p = xb + xpad(a * 512 + b1 * 64 + jj);
#pragma unroll
  for (int x = 0; x < 8; ++x) v[x] = p[8 * x];
  dft8(v);
  twiddle8(v, stw[576 + jj]);
  // the last exchange stores point (m, jj) of a 64-point block at 8 m +
  // (jj ^ m): the writes stay contiguous per m, and the reads below (8
  // consecutive points per thread) fall into distinct banks across lanes
  p = xb + xpad(a * 512 + b1 * 64);
#pragma unroll
  for (int m = 0; m < 8; ++m) p[8 * m + (jj ^ m)] = v[m];
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 8; ++x) v[x] = p[8 * jj + (x ^ jj)];
  dft8(v);
}

// One operand's view for a work unit.
struct OpView {
  const uint32_t* tab;   // [n] entries of repetition t
  const int32_t* first;  // [b_lo]
  const int32_t* cs;     // [n + 2] chain starts
  const uint2* pairs;    // [n]
  int64_t n;
  int nch;
};

// Chain records of one operand in LDS: chain c at rec[c + cs[c]]: header
// f | count << 16, then count words i | q << 16 | sign << 31 (row i, root
// index q of its weight relative to f, sign relative to f).  map[r] gets the
// second row of bucket r's chain (the slot of the imaginary part).
__device__ void build_records(const OpView& o, uint32_t uhi, uint32_t bhi_mask,
                              uint32_t* __restrict__ rec, uint32_t* __restrict__ map) {
  for (int c = threadIdx.x; c < o.nch; c += kFNT) {
    const int32_t beg = o.cs[c], end = o.cs[c + 1];
    const uint32_t f = o.pairs[beg].x >> 16;
    const uint32_t ef = o.tab[f];
    const uint32_t hf = (ef & kBucketMask) >> kFLB;
    uint32_t* r = rec + c + beg;
    r[0] = f | ((uint32_t)(end - beg) << 16);
    for (int32_t q = beg; q < end; ++q) {
      const uint32_t i = o.pairs[q].x & 0xFFFFu;
      const uint32_t ei = o.tab[i];
      const uint32_t hi = (ei & kBucketMask) >> kFLB;
      const uint32_t root = (uhi * ((hi - hf) & bhi_mask)) & bhi_mask;
      r[1 + q - beg] = i | (root << 16) | ((ei ^ ef) & kSignBit);
    }
    map[ef & ((1u << kFLB) - 1u)] = o.pairs[beg].x & 0xFFFFu;
  }
}

// Merge this thread's chains [c0, c0 + cnt) in place (records start at s).
__device__ __forceinline__ void merge_chains(double* __restrict__ row,
                                             const uint32_t* __restrict__ rec, int s, int cnt,
                                             const double2* __restrict__ roots) {
  for (int c = 0; c < cnt; ++c) {
    const uint32_t h = rec[s];
    const uint32_t f = h & 0xFFFFu, len = h >> 16;
    double re = row[f], im = 0.0;
    uint32_t m1 = 0;
    for (uint32_t j = 1; j <= len; ++j) {
      const uint32_t w = rec[s + j];
      const uint32_t i = w & 0xFFFFu;
      const double v = flip_sign(row[i], w & kSignBit);
      const double2 rho = roots[(w >> 16) & 0x7FFFu];
      re = fma(rho.x, v, re);
      im = fma(rho.y, v, im);
      if (j == 1) m1 = i;
    }
    row[f] = re;
    row[m1] = im;
    s += 1 + (int)len;
  }
}

// X[e] = w_e (row[re_e] + i row[im_e]) with w_e = cT dT^e s_e roots[q_e]
__device__ __forceinline__ void gather_weighted(double2 (&X)[8], const double* __restrict__ row,
                                                const uint32_t (&off)[8], const uint32_t (&qs)[4],
                                                const double2* __restrict__ roots, double2 cT,
                                                double2 dT) {
  double2 tw = cT;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    uint32_t o = off[e];
    asm volatile("" : "+v"(o));   // decode per use: keeps 8 registers, not 16
    const uint32_t qe = (qs[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    double2 sg = roots[qe & 0x7FFFu];
    if (qe & 0x8000u) sg = make_double2(-sg.x, -sg.y);
    X[e] = cmulf(cmulf(tw, sg), make_double2(row[o & 0xFFFFu], row[o >> 16]));
    if (e < 7) tw = cmulf(tw, dT);
  }
}

__global__ __launch_bounds__(kFNT, 2) void compress_fft_kernel(CompressArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int bhi_bits = a.log2b - kFLB;
  const uint32_t b_hi = 1u << bhi_bits;
  const uint32_t nslices = b_hi / 2 + 1;
  const int64_t nunits = (int64_t)a.d * nslices;
  const int64_t wg = blockIdx.x;
  const int64_t total = nunits * a.groups;
  int64_t lin = wg;
  if ((total & 7) == 0) lin = (wg & 7) * (total >> 3) + (wg >> 3);
  const int g = (int)(lin / nunits);
  const int64_t unit = lin - (int64_t)g * nunits;
  const int t = (int)(unit / nslices);
  const uint32_t uhi = (uint32_t)(unit - (int64_t)t * nslices);
  const int64_t k_per = (a.n_inner + a.groups - 1) / a.groups;
  const int64_t k0 = (int64_t)g * k_per;
  const int64_t k1 = (k0 + k_per) < a.n_inner ? (k0 + k_per) : a.n_inner;
  const int tid = threadIdx.x;
  const uint64_t b = (uint64_t)1 << a.log2b;

  double2* xb = reinterpret_cast<double2*>(smem);
  double* row = reinterpret_cast<double*>(xb + kXLen);
  const int64_t nmax = a.n_rows > a.n_cols ? a.n_rows : a.n_cols;
  uint32_t* recA = reinterpret_cast<uint32_t*>(row + row_pitch<double>(nmax));
  uint32_t* recB = recA + a.n_rows;
  double2* roots = reinterpret_cast<double2*>(recA + ((a.n_rows + a.n_cols + 3) & ~(int64_t)3));
  double2* stw = roots + b_hi;   // w_4096^j (512), w_512^j (64), w_64^j (8)
  uint32_t* mapA = reinterpret_cast<uint32_t*>(xb);   // [b_lo], in the exchange buffer
  uint32_t* mapB = mapA + (1 << kFLB);

  const OpView oA{a.tab1 + (size_t)t * a.n_rows, a.planA.first + (size_t)t * (1 << kFLB),
                  a.planA.cstart + (size_t)t * (a.n_rows + 2), a.planA.pairs + (size_t)t * a.n_rows,
                  a.n_rows, a.planA.nchains[t]};
  const OpView oB{a.tab2 + (size_t)t * a.n_cols, a.planB.first + (size_t)t * (1 << kFLB),
                  a.planB.cstart + (size_t)t * (a.n_cols + 2), a.planB.pairs + (size_t)t * a.n_cols,
                  a.n_cols, a.planB.nchains[t]};

  // roots of unity of order b_hi, bucket maps, chain records
  for (uint32_t q = tid; q < b_hi; q += kFNT) roots[q] = fwd_root(q, b_hi);
  stw[tid] = fwd_root((uint64_t)tid, 4096);
  if (tid < 64) stw[512 + tid] = fwd_root((uint64_t)tid, 512);
  if (tid < 8) stw[576 + tid] = fwd_root((uint64_t)tid, 64);
  for (int r = tid; r < (1 << kFLB); r += kFNT) {
    mapA[r] = (uint32_t)a.n_rows;
    mapB[r] = (uint32_t)a.n_cols;
  }
  __syncthreads();
  build_records(oA, uhi, b_hi - 1, recA, mapA);
  build_records(oB, uhi, b_hi - 1, recB, mapB);
  __syncthreads();
  // gather slots of the thread's buckets r = tid + 512 e, and their fold
  // weights w_b^(u_hi h(f)) s(f) of the first row f, split as
  // w_b^(u_hi r) (= cT dT^e, shared by the operands) times s(f)
  // w_{b_hi}^(u_hi hi(f)) (a root index and a sign, 16 bits per bucket)
  uint32_t offA[8], offB[8], qA[4], qB[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) { qA[e] = 0; qB[e] = 0; }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int r = tid + 512 * e;
    const int32_t fa = oA.first[r], fb = oB.first[r];
    offA[e] = (uint32_t)(fa >= 0 ? fa : a.n_rows) | (mapA[r] << 16);
    offB[e] = (uint32_t)(fb >= 0 ? fb : a.n_cols) | (mapB[r] << 16);
    if (fa >= 0) {
      const uint32_t ef = oA.tab[fa];
      const uint32_t q = (uhi * ((ef & kBucketMask) >> kFLB)) & (b_hi - 1);
      qA[e >> 1] |= (q | ((ef & kSignBit) >> 16)) << (16 * (e & 1));
    }
    if (fb >= 0) {
      const uint32_t ef = oB.tab[fb];
      const uint32_t q = (uhi * ((ef & kBucketMask) >> kFLB)) & (b_hi - 1);
      qB[e >> 1] |= (q | ((ef & kSignBit) >> 16)) << (16 * (e & 1));
    }
  }
  const double2 cT = fwd_root((uint64_t)uhi * (uint64_t)tid, b);
  const double2 dT = fwd_root((uint64_t)uhi * 512u, b);
  // this thread's chains for the in-place merges
  const int cA0 = (int)((int64_t)oA.nch * tid / kFNT), cA1 = (int)((int64_t)oA.nch * (tid + 1) / kFNT);
  const int cB0 = (int)((int64_t)oB.nch * tid / kFNT), cB1 = (int)((int64_t)oB.nch * (tid + 1) / kFNT);
  const int sA = cA0 < cA1 ? cA0 + oA.cs[cA0] : 0;
  const int sB = cB0 < cB1 ? cB0 + oB.cs[cB0] : 0;
  __syncthreads();   // the maps are read; the exchange buffer is free

  const double* At = reinterpret_cast<const double*>(a.At);
  const double* Bm = reinterpret_cast<const double*>(a.B);
  const bool dma = a.dma != 0;
  double2 acc[8], X[8], Y[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) acc[e] = make_double2(0.0, 0.0);
  if (k0 < k1) {
    if (tid == 0) row[a.n_rows] = 0.0;
    stage_row<double, kFNT>(row, At + k0 * a.n_rows, a.n_rows, dma);
  }
  for (int64_t k = k0; k < k1; ++k) {
    if (dma) wait_dma();
    __syncthreads();   // A's row of k has landed
    merge_chains(row, recA, sA, cA1 - cA0, roots);
    __syncthreads();
    gather_weighted(X, row, offA, qA, roots, cT, dT);
    __syncthreads();   // the row buffer is free
    if (tid == 0) row[a.n_cols] = 0.0;
    stage_row<double, kFNT>(row, Bm + k * a.ldb, a.n_cols, dma);
    fft4096(X, xb, stw);
    if (dma) wait_dma();
    __syncthreads();   // B's row has landed; X's last exchange reads are done
    merge_chains(row, recB, sB, cB1 - cB0, roots);
    __syncthreads();
    gather_weighted(Y, row, offB, qB, roots, cT, dT);
    __syncthreads();
    if (k + 1 < k1) {
      if (tid == 0) row[a.n_rows] = 0.0;
      stage_row<double, kFNT>(row, At + (k + 1) * a.n_rows, a.n_rows, dma);
    }
    fft4096(Y, xb, stw);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      acc[e].x = fma(X[e].x, Y[e].x, fma(-X[e].y, Y[e].y, acc[e].x));
      acc[e].y = fma(X[e].x, Y[e].y, fma(X[e].y, Y[e].x, acc[e].y));
    }
  }
  // natural positions: u = u_hi + b_hi u_lo, u_lo = a + 8 b1 + 64 c2 + 512 m
  double2* dst = reinterpret_cast<double2*>(a.partial) + ((size_t)g * a.d + t) * b;
  const uint32_t ulo0 = (uint32_t)((tid >> 6) + 8 * ((tid >> 3) & 7) + 64 * (tid & 7));
#pragma unroll
  for (int e = 0; e < 8; ++e) dst[uhi + (uint64_t)b_hi * (ulo0 + 512u * e)] = acc[e];
}

// P[t][u] = sum over groups of the partials, in group order; the slices
// above b_hi / 2 are the conjugates of P[t][b - u].
__global__ void reduce_fft_partials_kernel(const double2* __restrict__ part, int groups, int d,
                                           int log2b, double2* __restrict__ P) {
  const int t = blockIdx.y;
  const uint64_t b = (uint64_t)1 << log2b;
  const uint32_t bhi_mask = (1u << (log2b - kFLB)) - 1u;
  const uint32_t half = (bhi_mask + 1u) / 2u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < b; u += stride) {
    const bool mirror = (uint32_t)(u & bhi_mask) > half;
    const uint64_t src = mirror ? ((b - u) & (b - 1)) : u;
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < groups; ++q) {
      const double2 v = part[((size_t)q * d + t) * b + src];
      s.x += v.x;
      s.y += v.y;
    }
    P[(size_t)t * b + u] = mirror ? make_double2(s.x, -s.y) : s;
  }
}

}  // namespace

size_t compress_fft_lds(int64_t n_rows, int64_t n_cols, int log2b) {
  const int64_t nmax = n_rows > n_cols ? n_rows : n_cols;
  return sizeof(double2) * kXLen + sizeof(double) * (size_t)row_pitch<double>(nmax) +
         sizeof(uint32_t) * (size_t)((n_rows + n_cols + 3) & ~(int64_t)3) +
         sizeof(double2) * (((size_t)1 << (log2b - kFLB)) + 512 + 64 + 8);
}

bool compress_fft_supported(int64_t n_rows, int64_t n_cols, int log2b) {
  return log2b >= kFLB && log2b <= kFLB + 8 && n_rows >= 1 && n_cols >= 1 && n_rows <= 65534 &&
         n_cols <= 65534 && compress_fft_lds(n_rows, n_cols, log2b) <= 160 * 1024 - 256;
}

cmm_status launch_compress_fft(const CompressArgs& a0, hipStream_t s) {
  ProfScope prof_("compress", s);
  CompressArgs a = a0;
  const int64_t nslices = ((int64_t)1 << (a.log2b - kFLB)) / 2 + 1;
  const int64_t blocks = (int64_t)a.d * nslices * a.groups;
  const size_t lds = compress_fft_lds(a.n_rows, a.n_cols, a.log2b);
  a.dma = (a.n_rows % 2 == 0) && (a.n_cols % 2 == 0) && (a.ldb % 2 == 0) &&
          ((uintptr_t)a.At % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
  hipError_t e = hipFuncSetAttribute((const void*)compress_fft_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress fft: set LDS size");
  hipLaunchKernelGGL(compress_fft_kernel, dim3((unsigned)blocks), dim3(kFNT), lds, s, a);
  return hip_check(hipGetLastError(), "compress fft kernel launch");
}

cmm_status launch_reduce_fft_partials(const void* part, int groups, int d, int log2b, void* P,
                                      hipStream_t s) {
  ProfScope prof_("reduce", s);
  const uint64_t b = (uint64_t)1 << log2b;
  uint64_t gx = (b + 255) / 256;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(reduce_fft_partials_kernel, dim3((unsigned)gx, (unsigned)d), dim3(256), 0, s,
                     static_cast<const double2*>(part), groups, d, log2b, static_cast<double2*>(P));
  return hip_check(hipGetLastError(), "reduce kernel launch");
}

}  // namespace cmm
