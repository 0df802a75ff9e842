// Adjoint of the mean-over-d estimator (the differentiation form).
//
// For fixed hash functions the mean estimate
//   C_hat = (1/d) sum_t L_t(A B),  L_t(C)[i][j] = s1(i) s2(j) p_t[h1(i) xor h2(j)],
// is bilinear in (A, B), and p_t is Algorithm 1's Compress output
//   p_t = 2^-m H z_t,  z_t = sum_k X_{t,k} o Y_{t,k},
//   X_{t,k} = H S1_t A[:, k],  Y_{t,k} = H S2_t B[k, :]
// (S the count-sketch matrices of Section 3.1, H the Walsh-Hadamard
// matrix of Section 3.2).  For L = sum_ij W[i][j] C_hat[i][j] each step is
// run backwards with its transpose:
//   extract^T    q_t[x] = sum over h1(i) xor h2(j) = x of s1(i) s2(j) W[i][j]
//   inverse^T    r_t = 2^-m H q_t              (H is symmetric)
//   product      dX_{t,k} = (r_t / d) o Y_{t,k},  dY_{t,k} = (r_t / d) o X_{t,k}
//   forward^T    H dX_{t,k},  H dY_{t,k}
//   sketch^T     dA[i][k] = sum_t s1(i) (H dX_{t,k})[h1(i)]
//                dB[k][j] = sum_t s2(j) (H dY_{t,k})[h2(j)]
// (a gather: the transposed count sketch).  Per (t, k) this is four
// length-b transforms, twice the forward work.
//
// The fused kernel mirrors the forward one (Kronecker split b = b_hi b_lo,
// one work-group per (t, u_hi, k-range), rows staged in LDS and sketched by
// gather with folded signs).  With V = H_lo (dX slice u_hi),
//   (H dX)[r] = sum over u_hi of (-1)^popcount(u_hi & r_hi) V_{u_hi}[r_lo],
// so a work-group contributes s1(i) (-1)^popcount(u_hi & hi(h1 i)) V[lo(h1 i)]
// to dA[i][k]; these d * b_hi contributions are written as partials and
// summed in a fixed order by a second kernel (deterministic, no atomics).
#include "cmm_internal.h"
#include "wht_regs.h"

namespace cmm {
namespace {

// ---------------------------------------------------------- extract^T
// q partials: one work-group per (row block, window of 2^wb buckets,
// repetition t).  The window lives in LDS (float64, or float32 for the
// float32 form, where a block adds a few terms per bucket) and is summed
// with LDS atomics (the order of the additions inside a window is not
// fixed); the partials are then added in ascending block order in float64.
constexpr int kScatterThreads = 256;

template <typename TW, typename TA>
__global__ __launch_bounds__(kScatterThreads) void wscatter_kernel(
    const TW* __restrict__ W, int64_t ldw, const uint32_t* __restrict__ tab1,
    const uint32_t* __restrict__ tab2, int64_t n_rows, int64_t n_cols, int log2b, int wb,
    int64_t rows_per, int64_t blocks, int cache_tab2, double* __restrict__ part) {
  extern __shared__ __align__(16) unsigned char smem[];
  TA* q = reinterpret_cast<TA*>(smem);
  const uint32_t wlen = 1u << wb;
  uint32_t* t2c = reinterpret_cast<uint32_t*>(q + wlen);
  const int64_t rb = blockIdx.x % blocks;
  const uint32_t win = (uint32_t)(blockIdx.x / blocks);
  const int t = blockIdx.y;
  const int d = gridDim.y;
  const uint32_t bmask = (uint32_t)(((uint64_t)1 << log2b) - 1u);
  for (uint32_t x = threadIdx.x; x < wlen; x += kScatterThreads) q[x] = TA(0);
  const uint32_t* t1 = tab1 + (size_t)t * n_rows;
  const uint32_t* t2 = tab2 + (size_t)t * n_cols;
  if (cache_tab2)
    for (int64_t j = threadIdx.x; j < n_cols; j += kScatterThreads) t2c[j] = t2[j];
  __syncthreads();
  const int64_t i0 = (int64_t)rb * rows_per;
  const int64_t i1 = (i0 + rows_per) < n_rows ? (i0 + rows_per) : n_rows;
  for (int64_t i = i0; i < i1; ++i) {
    const uint32_t e1 = t1[i];
    const TW* wr = W + i * ldw;
    for (int64_t j = threadIdx.x; j < n_cols; j += kScatterThreads) {
      const uint32_t e2 = cache_tab2 ? t2c[j] : t2[j];
      const uint32_t x = (e1 ^ e2) & bmask;
      if ((x >> wb) == win) {
        const TA v = (TA)wr[j];
        atomicAdd(&q[x & (wlen - 1u)], ((e1 ^ e2) & kSignBit) ? -v : v);
      }
    }
  }
  __syncthreads();
  const size_t b = (size_t)1 << log2b;
  double* dst = part + ((size_t)rb * d + t) * b + ((size_t)win << wb);
  for (uint32_t x = threadIdx.x; x < wlen; x += kScatterThreads) dst[x] = (double)q[x];
}

// --------------------------------------------------------- fused adjoint
template <typename T, int LB>
__global__ __launch_bounds__((1 << LB) / 32) void adjoint_kernel(AdjointArgs aa) {
  const CompressArgs& a = aa.c;
  constexpr int E = Cfg<T, LB>::E;
  constexpr int NT = Cfg<T, LB>::NT;
  constexpr int BLO = 1 << LB;
  extern __shared__ __align__(16) unsigned char smem[];
  T* xbuf = reinterpret_cast<T*>(smem);                          // BLO (+ padding)
  T* rowA = xbuf + BLO + BLO / 128;                              // n_rows (16-byte aligned)
  T* rowB = rowA + row_pitch<T>(a.n_rows);                       // n_cols (+ pad)
  uint32_t* gA = reinterpret_cast<uint32_t*>(rowB + row_pitch<T>(a.n_cols));   // [n_rows]
  uint32_t* gB = gA + a.n_rows;                                                 // [n_cols]
  uint2* exl = reinterpret_cast<uint2*>(gA + (a.n_rows + a.n_cols + 1) / 2 * 2);
  if (threadIdx.x == 0) { rowA[a.n_rows] = T(0); rowB[a.n_cols] = T(0); }

  const int b_hi_bits = a.log2b - LB;
  const int64_t nunits = (int64_t)a.d << b_hi_bits;
  const int64_t wg = blockIdx.x;
  const int64_t total = nunits * a.groups;
  int64_t lin = wg;
  if ((total & 7) == 0) lin = (wg & 7) * (total >> 3) + (wg >> 3);
  const int g = (int)(lin / nunits);
  const int64_t unit = lin - (int64_t)g * nunits;
  const int t = (int)(unit >> b_hi_bits);
  const uint32_t uhi = (uint32_t)(unit & (((int64_t)1 << b_hi_bits) - 1));
  const int64_t k_per = (a.n_inner + a.groups - 1) / a.groups;
  const int64_t k0 = (int64_t)g * k_per;
  const int64_t k1 = (k0 + k_per) < a.n_inner ? (k0 + k_per) : a.n_inner;
  if (k0 >= k1) return;   // uniform over the work-group

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t base1 = ((uint32_t)((lane >> 4) & 1) << 5) | ((uint32_t)((lane >> 5) & 1) << 6) |
                         ((uint32_t)(lane & 15) << 7) | ((uint32_t)w << 11);
  const uint32_t* t1 = a.tab1 + (size_t)t * a.n_rows;
  const uint32_t* t2 = a.tab2 + (size_t)t * a.n_cols;
  // forward gather: first rows of the thread's buckets with folded signs
  uint32_t fa[E / 2], fb[E / 2];
  uint32_t nega = 0, negb = 0;
  {
    const int32_t* f1 = a.planA.first + (size_t)t * BLO + base1;
    const int32_t* f2 = a.planB.first + (size_t)t * BLO + base1;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int32_t r1 = f1[e], r2 = f2[e];
      const uint32_t en1 = t1[r1 >= 0 ? r1 : 0], en2 = t2[r2 >= 0 ? r2 : 0];
      const uint32_t s1 = r1 >= 0 ? (en1 >> 31) ^ (__popc(uhi & ((en1 & kBucketMask) >> LB)) & 1u) : 0u;
      const uint32_t s2 = r2 >= 0 ? (en2 >> 31) ^ (__popc(uhi & ((en2 & kBucketMask) >> LB)) & 1u) : 0u;
      nega |= s1 << e;
      negb |= s2 << e;
      const uint32_t ra = r1 >= 0 ? (uint32_t)r1 : (uint32_t)a.n_rows;
      const uint32_t rb = r2 >= 0 ? (uint32_t)r2 : (uint32_t)a.n_cols;
      if (e & 1) { fa[e >> 1] |= ra << 16; fb[e >> 1] |= rb << 16; }
      else { fa[e >> 1] = ra; fb[e >> 1] = rb; }
    }
  }
  // transposed sketch: LDS address of lo(h(i)) in the natural-order buffer
  // and the folded sign s(i) (-1)^popcount(u_hi & hi(h(i))) in bit 31
  for (int64_t i = threadIdx.x; i < a.n_rows; i += NT) {
    const uint32_t e = t1[i];
    const uint32_t neg = (e >> 31) ^ (__popc(uhi & ((e & kBucketMask) >> LB)) & 1u);
    gA[i] = swz(e & (uint32_t)(BLO - 1)) | (neg << 31);
  }
  for (int64_t j = threadIdx.x; j < a.n_cols; j += NT) {
    const uint32_t e = t2[j];
    const uint32_t neg = (e >> 31) ^ (__popc(uhi & ((e & kBucketMask) >> LB)) & 1u);
    gB[j] = swz(e & (uint32_t)(BLO - 1)) | (neg << 31);
  }
  // collision chains, in LDS when they fit
  const int32_t* gcA = a.planA.cstart + (size_t)t * (a.n_rows + 2);
  const int32_t* gcB = a.planB.cstart + (size_t)t * (a.n_cols + 2);
  const int nchA = a.planA.nchains[t], nchB = a.planB.nchains[t];
  const int cntA = gcA[nchA], cntB = gcB[nchB];
  const bool ex_lds = (int64_t)cntA + cntB + (nchA + nchB + 4) / 2 + 1 <= a.ex_cap;
  const uint2* gpA = a.planA.pairs + (size_t)t * a.n_rows;
  const uint2* gpB = a.planB.pairs + (size_t)t * a.n_cols;
  if (ex_lds) {
    for (int q = threadIdx.x; q < cntA; q += NT) exl[q] = gpA[q];
    for (int q = threadIdx.x; q < cntB; q += NT) exl[cntA + q] = gpB[q];
    int32_t* csl = reinterpret_cast<int32_t*>(exl + cntA + cntB);
    for (int q = threadIdx.x; q <= nchA; q += NT) csl[q] = gcA[q];
    for (int q = threadIdx.x; q <= nchB; q += NT) csl[nchA + 1 + q] = gcB[q];
  }
  // LDS views of the lists; each fix-up call below takes either these or the
  // global lists, so the compiler knows every pointer's memory space
  const uint2* lexA = exl;
  const uint2* lexB = exl + cntA;
  const int32_t* lcsA = reinterpret_cast<const int32_t*>(exl + cntA + cntB);
  const int32_t* lcsB = lcsA + nchA + 1;

  const uint32_t w1 = swz(l1p_lane(lane, w));
  const uint32_t r2lane = swz(l2_lane<LB>(lane, w, false));
  const uint32_t nat = swz(base1);   // + e: this thread's 32 consecutive buckets

  // (r_t / d) on this slice, in the layout the forward transform leaves
  T R[E];
  {
    const int64_t b = (int64_t)1 << a.log2b;
    const double* rs = aa.r + (size_t)t * b + ((int64_t)uhi << LB);
    const uint32_t r2after = l2_lane<LB>(lane, w, true);
#pragma unroll
    for (int e = 0; e < E; ++e) R[e] = (T)(rs[r2after | l2_reg<LB>(e, true)] * aa.scale);
  }

  const T* At = reinterpret_cast<const T*>(a.At);
  const T* Bm = reinterpret_cast<const T*>(a.B);
  T* oA = reinterpret_cast<T*>(aa.partA) + (size_t)unit * a.n_inner * a.n_rows;
  T* oB = reinterpret_cast<T*>(aa.partB) + (size_t)unit * a.n_inner * a.n_cols;
  const bool dma = a.dma != 0;
  stage_row<T, NT>(rowA, At + k0 * a.n_rows, a.n_rows, dma);
  stage_row<T, NT>(rowB, Bm + k0 * a.ldb, a.n_cols, dma);

  for (int64_t k = k0; k < k1; ++k) {
    if (dma) wait_dma();
    __syncthreads();
    if (nchA + nchB > 0) {
      { if (ex_lds) fix_chains<T, NT>(rowA, lexA, lcsA, nchA, uhi); else fix_chains<T, NT>(rowA, gpA, gcA, nchA, uhi); }
      { if (ex_lds) fix_chains<T, NT>(rowB, lexB, lcsB, nchB, uhi); else fix_chains<T, NT>(rowB, gpB, gcB, nchB, uhi); }
      __syncthreads();
    }
    T X[E], Y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t ra = (e & 1) ? (fa[e >> 1] >> 16) : (fa[e >> 1] & 0xFFFFu);
      const uint32_t rb = (e & 1) ? (fb[e >> 1] >> 16) : (fb[e >> 1] & 0xFFFFu);
      X[e] = flip_sign(rowA[ra], (nega << (31 - e)) & 0x80000000u);
      Y[e] = flip_sign(rowB[rb], (negb << (31 - e)) & 0x80000000u);
    }
    __syncthreads();   // the row buffers can be refilled
    if (k + 1 < k1) {
      stage_row<T, NT>(rowA, At + (k + 1) * a.n_rows, a.n_rows, dma);
      stage_row<T, NT>(rowB, Bm + (k + 1) * a.ldb, a.n_cols, dma);
    }
    // forward transform of both sketches (as in Compress)
    pass1(X);
    pass1(Y);
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[w1 + l1p_reg(e)] = X[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) X[e] = xbuf[r2lane + swz(l2_reg<LB>(e, false))];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[w1 + l1p_reg(e)] = Y[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) Y[e] = xbuf[r2lane + swz(l2_reg<LB>(e, false))];
    pass2<LB>(X);
    pass2<LB>(Y);
    // dX = (r / d) o Y, dY = (r / d) o X
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const T x = X[e];
      X[e] = R[e] * Y[e];
      Y[e] = R[e] * x;
    }
    // H_lo again, stages in the reverse order: pass 2 on the current layout
    // (it ends in the pre-exchange layout), LDS transpose back, pass 1 (it
    // ends in the gather layout: bucket base1 + e in register e)
    pass2<LB>(X);
    pass2<LB>(Y);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[r2lane + swz(l2_reg<LB>(e, false))] = X[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) X[e] = xbuf[w1 + l1p_reg(e)];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[r2lane + swz(l2_reg<LB>(e, false))] = Y[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) Y[e] = xbuf[w1 + l1p_reg(e)];
    pass1(X);
    pass1(Y);
    // transposed sketch of each operand from the natural-order buffer
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[nat + e] = X[e];
    __syncthreads();
    {
      T* o = oA + (size_t)k * a.n_rows;
      for (int64_t i = threadIdx.x; i < a.n_rows; i += NT) {
        const uint32_t gi = gA[i];
        o[i] = flip_sign(xbuf[gi & kBucketMask], gi & kSignBit);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[nat + e] = Y[e];
    __syncthreads();
    {
      T* o = oB + (size_t)k * a.n_cols;
      for (int64_t j = threadIdx.x; j < a.n_cols; j += NT) {
        const uint32_t gj = gB[j];
        o[j] = flip_sign(xbuf[gj & kBucketMask], gj & kSignBit);
      }
    }
    // xbuf is rewritten next iteration only after the chain barriers
  }
}

// ---------------------------------------------- fused adjoint, 16 elements
// The same steps on the 16-element layout (b_lo = 2^13, 512 threads, two
// waves per SIMD): forward passes 1 and 2 leave layout L2'; pass 2 applied
// again runs the same stages (ending in layout L2), the transpose back
// gives L1', and pass 1 ends in the gather layout, bucket base1 + e in
// register e.
template <typename T>
__global__ __launch_bounds__(512, 2) void adjoint16_kernel(AdjointArgs aa) {
  const CompressArgs& a = aa.c;
  constexpr int LB = 13;
  constexpr int E = 16;
  constexpr int NT = 512;
  constexpr int BLO = 1 << LB;
  constexpr int XLEN = BLO + BLO / 64 + 16;
  extern __shared__ __align__(16) unsigned char smem[];
  T* xbuf = reinterpret_cast<T*>(smem);
  T* rowA = xbuf + XLEN;
  T* rowB = rowA + row_pitch<T>(a.n_rows);
  uint32_t* gA = reinterpret_cast<uint32_t*>(rowB + row_pitch<T>(a.n_cols));   // [n_rows]
  uint32_t* gB = gA + a.n_rows;                                                 // [n_cols]
  uint2* exl = reinterpret_cast<uint2*>(gA + (a.n_rows + a.n_cols + 1) / 2 * 2);
  if (threadIdx.x == 0) { rowA[a.n_rows] = T(0); rowB[a.n_cols] = T(0); }

  const int b_hi_bits = a.log2b - LB;
  const int64_t nunits = (int64_t)a.d << b_hi_bits;
  const int64_t wg = blockIdx.x;
  const int64_t total = nunits * a.groups;
  int64_t lin = wg;
  if ((total & 7) == 0) lin = (wg & 7) * (total >> 3) + (wg >> 3);
  const int g = (int)(lin / nunits);
  const int64_t unit = lin - (int64_t)g * nunits;
  const int t = (int)(unit >> b_hi_bits);
  const uint32_t uhi = (uint32_t)(unit & (((int64_t)1 << b_hi_bits) - 1));
  const int64_t k_per = (a.n_inner + a.groups - 1) / a.groups;
  const int64_t k0 = (int64_t)g * k_per;
  const int64_t k1 = (k0 + k_per) < a.n_inner ? (k0 + k_per) : a.n_inner;
  if (k0 >= k1) return;   // uniform over the work-group

  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t l4 = (lane >> 4) & 1, l5 = (lane >> 5) & 1, l3 = (lane >> 3) & 1;
  const uint32_t base1 = (l4 << 4) | (l5 << 5) | ((lane & 15) << 6) | (w << 10);
  const uint32_t* t1 = a.tab1 + (size_t)t * a.n_rows;
  const uint32_t* t2 = a.tab2 + (size_t)t * a.n_cols;
  // forward gather: byte offsets of the first rows of the thread's buckets
  // (the zero pad when empty) and their folded signs
  uint32_t offA[E], offB[E];
  uint32_t nega = 0, negb = 0;
  {
    const int32_t* f1 = a.planA.first + (size_t)t * BLO + base1;
    const int32_t* f2 = a.planB.first + (size_t)t * BLO + base1;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int32_t r1 = f1[e], r2 = f2[e];
      const uint32_t en1 = t1[r1 >= 0 ? r1 : 0], en2 = t2[r2 >= 0 ? r2 : 0];
      const uint32_t s1 = r1 >= 0 ? (en1 >> 31) ^ (__popc(uhi & ((en1 & kBucketMask) >> LB)) & 1u) : 0u;
      const uint32_t s2 = r2 >= 0 ? (en2 >> 31) ^ (__popc(uhi & ((en2 & kBucketMask) >> LB)) & 1u) : 0u;
      nega |= s1 << e;
      negb |= s2 << e;
      const uint32_t ra = r1 >= 0 ? (uint32_t)r1 : (uint32_t)a.n_rows;
      const uint32_t rb = r2 >= 0 ? (uint32_t)r2 : (uint32_t)a.n_cols;
      offA[e] = (uint32_t)((const unsigned char*)(rowA + ra) - smem);
      offB[e] = (uint32_t)((const unsigned char*)(rowB + rb) - smem);
    }
  }
  // transposed sketch: padded address of lo(h(i)) and the folded sign
  for (int64_t i = threadIdx.x; i < a.n_rows; i += NT) {
    const uint32_t e = t1[i];
    const uint32_t neg = (e >> 31) ^ (__popc(uhi & ((e & kBucketMask) >> LB)) & 1u);
    gA[i] = pad16(e & (uint32_t)(BLO - 1)) | (neg << 31);
  }
  for (int64_t j = threadIdx.x; j < a.n_cols; j += NT) {
    const uint32_t e = t2[j];
    const uint32_t neg = (e >> 31) ^ (__popc(uhi & ((e & kBucketMask) >> LB)) & 1u);
    gB[j] = pad16(e & (uint32_t)(BLO - 1)) | (neg << 31);
  }
  // collision chains, in LDS when they fit
  const int32_t* gcA = a.planA.cstart + (size_t)t * (a.n_rows + 2);
  const int32_t* gcB = a.planB.cstart + (size_t)t * (a.n_cols + 2);
  const int nchA = a.planA.nchains[t], nchB = a.planB.nchains[t];
  const int cntA = gcA[nchA], cntB = gcB[nchB];
  const bool ex_lds = (int64_t)cntA + cntB + (nchA + nchB + 4) / 2 + 1 <= a.ex_cap;
  const uint2* gpA = a.planA.pairs + (size_t)t * a.n_rows;
  const uint2* gpB = a.planB.pairs + (size_t)t * a.n_cols;
  if (ex_lds) {
    for (int q = threadIdx.x; q < cntA; q += NT) exl[q] = gpA[q];
    for (int q = threadIdx.x; q < cntB; q += NT) exl[cntA + q] = gpB[q];
    int32_t* csl = reinterpret_cast<int32_t*>(exl + cntA + cntB);
    for (int q = threadIdx.x; q <= nchA; q += NT) csl[q] = gcA[q];
    for (int q = threadIdx.x; q <= nchB; q += NT) csl[nchA + 1 + q] = gcB[q];
  }
  const uint2* lexA = exl;
  const uint2* lexB = exl + cntA;
  const int32_t* lcsA = reinterpret_cast<const int32_t*>(exl + cntA + cntB);
  const int32_t* lcsB = lcsA + nchA + 1;

  // transpose addresses (as in Compress): L1' <-> L2
  const uint32_t wr_t = pad16(l4 | (l5 << 1) | ((lane & 15) << 6) | (w << 10));
  const uint32_t rd_t = pad16((lane & 7) | (w << 3) | (l4 << 10) | (l5 << 11) | (l3 << 12));
  auto wr_e = [](int e) -> uint32_t {
    return ((uint32_t)(e & 1) << 4) | ((uint32_t)((e >> 1) & 1) << 5) | (uint32_t)(e & 12);
  };
  auto rd_e = [](int e) -> uint32_t { return pad16((uint32_t)e << 6); };
  const T sgn8 = l3 ? T(-1) : T(1);
  const uint32_t nat = pad16(base1);   // + e: the thread's 16 consecutive buckets

  // (r_t / d) on this slice in layout L2' (where the forward passes end)
  T R[E];
  {
    const int64_t b = (int64_t)1 << a.log2b;
    const double* rs = aa.r + (size_t)t * b + ((int64_t)uhi << LB);
    const uint32_t fin_t = (lane & 7) | (w << 3) | (l4 << 6) | (l5 << 7) | (l3 << 12);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t fe = ((uint32_t)(e & 1) << 10) | ((uint32_t)((e >> 1) & 1) << 11) |
                          ((uint32_t)((e >> 2) & 3) << 8);
      R[e] = (T)(rs[fin_t | fe] * aa.scale);
    }
  }

  const T* At = reinterpret_cast<const T*>(a.At);
  const T* Bm = reinterpret_cast<const T*>(a.B);
  T* oA = reinterpret_cast<T*>(aa.partA) + (size_t)unit * a.n_inner * a.n_rows;
  T* oB = reinterpret_cast<T*>(aa.partB) + (size_t)unit * a.n_inner * a.n_cols;
  const bool dma = a.dma != 0;
  stage_row<T, NT>(rowA, At + k0 * a.n_rows, a.n_rows, dma);
  stage_row<T, NT>(rowB, Bm + k0 * a.ldb, a.n_cols, dma);

  // one operand through the transpose buffer: write in one layout, read in
  // the other (barriers around the buffer's reuse)
  auto through = [&](T (&v)[E], bool forward) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[forward ? wr_t + wr_e(e) : rd_t + rd_e(e)] = v[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xbuf[forward ? rd_t + rd_e(e) : wr_t + wr_e(e)];
  };
  // one operand's transposed sketch from the natural-order buffer
  auto scatter_out = [&](const T (&v)[E], const uint32_t* gt, int64_t n, T* o) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[nat + e] = v[e];
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += NT) {
      const uint32_t gi = gt[i];
      o[i] = flip_sign(xbuf[gi & kBucketMask], gi & kSignBit);
    }
  };

  for (int64_t k = k0; k < k1; ++k) {
    if (dma) wait_dma();
    __syncthreads();
    if (nchA + nchB > 0) {
      { if (ex_lds) fix_chains<T, NT>(rowA, lexA, lcsA, nchA, uhi); else fix_chains<T, NT>(rowA, gpA, gcA, nchA, uhi); }
      { if (ex_lds) fix_chains<T, NT>(rowB, lexB, lcsB, nchB, uhi); else fix_chains<T, NT>(rowB, gpB, gcB, nchB, uhi); }
      __syncthreads();
    }
    T X[E], Y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      X[e] = flip_sign(*reinterpret_cast<const T*>(smem + offA[e]), (nega << (31 - e)) & 0x80000000u);
      Y[e] = flip_sign(*reinterpret_cast<const T*>(smem + offB[e]), (negb << (31 - e)) & 0x80000000u);
    }
    __syncthreads();   // the row buffers can be refilled
    if (k + 1 < k1) {
      stage_row<T, NT>(rowA, At + (k + 1) * a.n_rows, a.n_rows, dma);
      stage_row<T, NT>(rowB, Bm + (k + 1) * a.ldb, a.n_cols, dma);
    }
    // forward transforms (as in Compress)
    pass1_16(X);
    pass1_16(Y);
    through(X, true);
    through(Y, true);
    pass2_16(X, sgn8);
    pass2_16(Y, sgn8);
    // dX = (r / d) o Y, dY = (r / d) o X
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const T x = X[e];
      X[e] = R[e] * Y[e];
      Y[e] = R[e] * x;
    }
    // H_lo again, ending in the gather layout
    pass2_16(X, sgn8);
    pass2_16(Y, sgn8);
    through(X, false);
    through(Y, false);
    pass1_16(X);
    pass1_16(Y);
    scatter_out(X, gA, a.n_rows, oA + (size_t)(k - 0) * a.n_rows);
    scatter_out(Y, gB, a.n_cols, oB + (size_t)(k - 0) * a.n_cols);
    // the next iteration's first barrier ends the reads of the buffer
  }
}

// ------------------------------------------------------ partial reduction
// out = sum over p (ascending) of part[p][kk][i], summed in float64:
//   transpose = 0:  out[(kb + kk) * ld + i]     (dB rows)
//   transpose = 1:  out[i * ld + kb + kk]       (dA columns)
// Four consecutive i per thread (one 16- or 32-byte load per partial) when
// n is a multiple of four; otherwise one.
template <typename TP, int VW>
struct VecOf;
template <> struct VecOf<float, 4> { typedef float4 type; };
template <> struct VecOf<double, 4> { typedef double4 type; };

template <typename TP, int VW>
__device__ __forceinline__ void load_vw(const TP* __restrict__ p, double (&v)[VW]) {
  if constexpr (VW == 4) {
    const typename VecOf<TP, 4>::type x = *reinterpret_cast<const typename VecOf<TP, 4>::type*>(p);
    v[0] = (double)x.x; v[1] = (double)x.y; v[2] = (double)x.z; v[3] = (double)x.w;
  } else {
    v[0] = (double)p[0];
  }
}

template <typename TP, typename TO, int VW>
__global__ __launch_bounds__(256) void adjoint_reduce_rows(const TP* __restrict__ part, int P,
                                                           int64_t kc, int64_t n,
                                                           TO* __restrict__ out, int64_t ld,
                                                           int64_t kb) {
  const int64_t kk = blockIdx.y;
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * VW;
  if (i >= n) return;
  double s[VW], v[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) s[q] = 0.0;
  for (int p = 0; p < P; ++p) {
    load_vw<TP, VW>(part + ((size_t)p * kc + kk) * n + i, v);
#pragma unroll
    for (int q = 0; q < VW; ++q) s[q] += v[q];
  }
#pragma unroll
  for (int q = 0; q < VW; ++q) out[(kb + kk) * ld + i + q] = (TO)s[q];
}

template <typename TP, typename TO, int VW>
__global__ __launch_bounds__(256) void adjoint_reduce_cols(const TP* __restrict__ part, int P,
                                                           int64_t kc, int64_t n,
                                                           TO* __restrict__ out, int64_t ld,
                                                           int64_t kb) {
  // tile of 64 k x 64 i; 16 x 16 threads, each 4 i (VW = 4) or 1 i at a stride
  __shared__ double tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, kk0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  for (int r = ty; r < 64; r += 16) {
    const int64_t kk = kk0 + r;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (kk < kc) {
      if constexpr (VW == 4) {
        const int64_t i = i0 + 4 * tx;
        if (i < n) {
          double v[4];
          for (int p = 0; p < P; ++p) {
            load_vw<TP, 4>(part + ((size_t)p * kc + kk) * n + i, v);
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] += v[q];
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t i = i0 + tx + 16 * q;
          if (i < n)
            for (int p = 0; p < P; ++p) s[q] += (double)part[((size_t)p * kc + kk) * n + i];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) tile[r][VW == 4 ? 4 * tx + q : tx + 16 * q] = s[q];
  }
  __syncthreads();
  const int c = threadIdx.x & 63, rr = threadIdx.x >> 6;   // 64 x 4 for the writes
  for (int r = rr; r < 64; r += 4) {
    const int64_t i = i0 + r, kk = kk0 + c;
    if (i < n && kk < kc) out[i * ld + kb + kk] = (TO)tile[c][r];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void zero_matrix_kernel(T* __restrict__ out, int64_t rows,
                                                          int64_t cols, int64_t ld) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
    if (c < cols) out[r * ld + c] = T(0);
}

}  // namespace

// ------------------------------------------------------------ launchers
cmm_status launch_zero_matrix(void* out, cmm_dtype dt, int64_t rows, int64_t cols, int64_t ld,
                              hipStream_t s) {
  const dim3 grid((unsigned)((cols + 255) / 256), (unsigned)(rows < 65535 ? rows : 65535));
  if (dt == CMM_F64)
    hipLaunchKernelGGL(zero_matrix_kernel<double>, grid, dim3(256), 0, s,
                       static_cast<double*>(out), rows, cols, ld);
  else
    hipLaunchKernelGGL(zero_matrix_kernel<float>, grid, dim3(256), 0, s,
                       static_cast<float*>(out), rows, cols, ld);
  return hip_check(hipGetLastError(), "zero fill launch");
}

template <typename TW, typename TA>
static cmm_status launch_wscatter_t(const TW* W, int64_t ldw, const uint32_t* tab1,
                                    const uint32_t* tab2, int d, int64_t n_rows, int64_t n_cols,
                                    int log2b, const ScatterShape& sh, double* part,
                                    hipStream_t s) {
  const size_t qbytes = sizeof(TA) << sh.wb;
  const bool cache = qbytes + sizeof(uint32_t) * (size_t)n_cols <= 160 * 1024;
  const size_t lds = qbytes + (cache ? sizeof(uint32_t) * (size_t)n_cols : 0);
  const dim3 grid((unsigned)(sh.blocks << (log2b - sh.wb)), (unsigned)d);
  auto kern = wscatter_kernel<TW, TA>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "wscatter: set LDS size");
  hipLaunchKernelGGL(kern, grid, dim3(kScatterThreads), lds, s, W, ldw, tab1, tab2, n_rows, n_cols,
                     log2b, sh.wb, sh.rows_per, sh.blocks, (int)cache, part);
  return hip_check(hipGetLastError(), "wscatter kernel launch");
}

cmm_status launch_wscatter(const void* W, cmm_dtype wdt, int64_t ldw, const uint32_t* tab1,
                           const uint32_t* tab2, int d, int64_t n_rows, int64_t n_cols,
                           int log2b, const ScatterShape& sh, double* part, hipStream_t s) {
  ProfScope prof_("wscatter", s);
  if (sh.f32)
    return wdt == CMM_F64
               ? launch_wscatter_t<double, float>(static_cast<const double*>(W), ldw, tab1, tab2,
                                                  d, n_rows, n_cols, log2b, sh, part, s)
               : launch_wscatter_t<float, float>(static_cast<const float*>(W), ldw, tab1, tab2, d,
                                                 n_rows, n_cols, log2b, sh, part, s);
  return wdt == CMM_F64
             ? launch_wscatter_t<double, double>(static_cast<const double*>(W), ldw, tab1, tab2, d,
                                                 n_rows, n_cols, log2b, sh, part, s)
             : launch_wscatter_t<float, double>(static_cast<const float*>(W), ldw, tab1, tab2, d,
                                                n_rows, n_cols, log2b, sh, part, s);
}

size_t adjoint_lds_bytes(cmm_dtype dt, int lb, int64_t n_rows, int64_t n_cols) {
  const size_t es = dtype_size(dt);
  const int64_t pa = (dt == CMM_F64) ? row_pitch<double>(n_rows) : row_pitch<float>(n_rows);
  const int64_t pb = (dt == CMM_F64) ? row_pitch<double>(n_cols) : row_pitch<float>(n_cols);
  size_t s = es * (((size_t)1 << lb) + ((size_t)1 << (lb - 7)) + (size_t)pa + (size_t)pb);
  s += sizeof(uint32_t) * (size_t)((n_rows + n_cols + 1) / 2 * 2);   // gather words
  return s;
}

size_t adjoint16_lds_bytes(cmm_dtype dt, int64_t n_rows, int64_t n_cols) {
  const size_t es = dtype_size(dt);
  const int64_t pa = (dt == CMM_F64) ? row_pitch<double>(n_rows) : row_pitch<float>(n_rows);
  const int64_t pb = (dt == CMM_F64) ? row_pitch<double>(n_cols) : row_pitch<float>(n_cols);
  const size_t xlen = ((size_t)1 << 13) + ((size_t)1 << 7) + 16;
  return es * (xlen + (size_t)pa + (size_t)pb) +
         sizeof(uint32_t) * (size_t)((n_rows + n_cols + 1) / 2 * 2);
}

template <typename T>
static cmm_status launch_adjoint16_t(const AdjointArgs& a0, hipStream_t s) {
  ProfScope prof_("adjoint", s);
  AdjointArgs aa = a0;
  CompressArgs& a = aa.c;
  const int64_t blocks = ((int64_t)a.d << (a.log2b - 13)) * a.groups;
  const size_t kMax = 160 * 1024;
  const size_t base = adjoint16_lds_bytes(sizeof(T) == 8 ? CMM_F64 : CMM_F32, a.n_rows, a.n_cols);
  if (base > kMax) { set_error("adjoint: rows do not fit in LDS"); return CMM_EUNSUPPORTED; }
  int64_t cap = (int64_t)((kMax - base) / sizeof(uint2));
  if (cap > a.n_rows + a.n_cols) cap = a.n_rows + a.n_cols;
  a.ex_cap = cap;
  const size_t lds = base + sizeof(uint2) * (size_t)cap;
  constexpr int V = 16 / sizeof(T);
  a.dma = (a.n_rows % V == 0) && (a.n_cols % V == 0) && (a.ldb % V == 0) &&
          ((uintptr_t)a.At % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
  auto kern = adjoint16_kernel<T>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "adjoint: set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(512), lds, s, aa);
  return hip_check(hipGetLastError(), "adjoint kernel launch");
}

template <typename T, int LB>
static cmm_status launch_adjoint_t(const AdjointArgs& a0, hipStream_t s) {
  ProfScope prof_("adjoint", s);
  AdjointArgs aa = a0;
  CompressArgs& a = aa.c;
  const int64_t blocks = ((int64_t)a.d << (a.log2b - LB)) * a.groups;
  const size_t kMax = 160 * 1024;
  const size_t base = adjoint_lds_bytes(sizeof(T) == 8 ? CMM_F64 : CMM_F32, LB, a.n_rows, a.n_cols);
  if (base > kMax) { set_error("adjoint: rows do not fit in LDS"); return CMM_EUNSUPPORTED; }
  int64_t cap = (int64_t)((kMax - base) / sizeof(uint2));
  const int64_t want = a.n_rows + a.n_cols;
  if (cap > want) cap = want;
  a.ex_cap = cap;
  const size_t lds = base + sizeof(uint2) * (size_t)cap;
  constexpr int V = 16 / sizeof(T);
  a.dma = (a.n_rows % V == 0) && (a.n_cols % V == 0) && (a.ldb % V == 0) &&
          ((uintptr_t)a.At % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
  auto kern = adjoint_kernel<T, LB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "adjoint: set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(Cfg<T, LB>::NT), lds, s, aa);
  return hip_check(hipGetLastError(), "adjoint kernel launch");
}

cmm_status launch_adjoint(const AdjointArgs& a, cmm_dtype dt, int lb, hipStream_t s) {
  // b_lo = 2^13: the 16-element layout when its LDS holds the rows
  if (lb == 13 && adjoint16_lds_bytes(dt, a.c.n_rows, a.c.n_cols) + 2048 <= 160 * 1024) {
    if (dt == CMM_F64) return launch_adjoint16_t<double>(a, s);
    return launch_adjoint16_t<float>(a, s);
  }
  if (dt == CMM_F64) {
    switch (lb) {
      case 11: return launch_adjoint_t<double, 11>(a, s);
      case 12: return launch_adjoint_t<double, 12>(a, s);
      case 13: return launch_adjoint_t<double, 13>(a, s);
    }
  } else {
    switch (lb) {
      case 11: return launch_adjoint_t<float, 11>(a, s);
      case 12: return launch_adjoint_t<float, 12>(a, s);
      case 13: return launch_adjoint_t<float, 13>(a, s);
    }
  }
  set_error("adjoint: unsupported b_lo");
  return CMM_EUNSUPPORTED;
}

template <typename TP, typename TO>
static void reduce_t(const void* part, int P, int64_t kc, int64_t n, void* out, int64_t ld,
                     int64_t kb, bool transpose, hipStream_t s) {
  const TP* pp = static_cast<const TP*>(part);
  TO* o = static_cast<TO*>(out);
  // vector loads need every row of the partials 4-element aligned
  const bool vec = n % 4 == 0 && (uintptr_t)part % (4 * sizeof(TP)) == 0;
  if (transpose) {
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((kc + 63) / 64));
    if (vec)
      hipLaunchKernelGGL((adjoint_reduce_cols<TP, TO, 4>), grid, dim3(256), 0, s, pp, P, kc, n, o, ld, kb);
    else
      hipLaunchKernelGGL((adjoint_reduce_cols<TP, TO, 1>), grid, dim3(256), 0, s, pp, P, kc, n, o, ld, kb);
  } else {
    if (vec) {
      const dim3 grid((unsigned)((n / 4 + 255) / 256), (unsigned)kc);
      hipLaunchKernelGGL((adjoint_reduce_rows<TP, TO, 4>), grid, dim3(256), 0, s, pp, P, kc, n, o, ld, kb);
    } else {
      const dim3 grid((unsigned)((n + 255) / 256), (unsigned)kc);
      hipLaunchKernelGGL((adjoint_reduce_rows<TP, TO, 1>), grid, dim3(256), 0, s, pp, P, kc, n, o, ld, kb);
    }
  }
}

cmm_status launch_adjoint_reduce(const void* part, cmm_dtype part_dt, int P, int64_t kc,
                                 int64_t n, void* out, cmm_dtype out_dt, int64_t ld, int64_t kb,
                                 bool transpose, hipStream_t s) {
  ProfScope prof_("adjoint_reduce", s);
  if (kc > 65535 && !transpose) { set_error("adjoint reduce: chunk too long"); return CMM_EUNSUPPORTED; }
  if (part_dt == CMM_F64 && out_dt == CMM_F64)
    reduce_t<double, double>(part, P, kc, n, out, ld, kb, transpose, s);
  else if (part_dt == CMM_F32 && out_dt == CMM_F32)
    reduce_t<float, float>(part, P, kc, n, out, ld, kb, transpose, s);
  else if (part_dt == CMM_F32 && out_dt == CMM_F64)
    reduce_t<float, double>(part, P, kc, n, out, ld, kb, transpose, s);
  else {
    set_error("adjoint reduce: unsupported types");
    return CMM_EUNSUPPORTED;
  }
  return hip_check(hipGetLastError(), "adjoint reduce launch");
}

}  // namespace cmm
