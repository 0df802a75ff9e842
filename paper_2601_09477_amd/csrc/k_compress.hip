// Fused Compress (Algorithm 1): sketch + forward WHT + accumulation over k.
//
// Kronecker split.  With b = b_hi * b_lo and u = u_hi * b_lo + u_lo,
//   H_b[u][r] = H_hi[u_hi][r_hi] * H_lo[u_lo][r_lo]
// because popcount(u & r) adds over the two bit fields.  Hence the slice
//   X[u_hi * b_lo + u_lo] = (H_lo F)[u_lo],
//   F[r_lo] = sum over rows i with lo(h1(i)) = r_lo of
//             s1(i) * (-1)^popcount(u_hi & hi(h1(i))) * A[i][k],
// a count sketch into b_lo buckets with a folded sign.  A work-group owns
// one (repetition t, slice u_hi, range of k) and keeps its b_lo-slice of
// p_hat = sum_k X o Y in registers; the top log2(b_hi) butterfly stages are
// traded for re-sketching the input once per slice (n adds instead of
// b log2(b_hi)), which is cheaper whenever b >= n.
//
// Sketch without atomics.  The rows of each lo-bucket are known from the
// tables (a per-call plan): the first (lowest) row of every bucket, and a
// list of the other rows ordered by their rank inside the bucket.  Per k
// the input row (A^T[k], B[k]) is staged in LDS, the non-first rows are
// added onto their bucket's first row in rank rounds (ascending row order,
// deterministic), and every thread gathers its buckets straight into
// registers.
//
// Transform layout (E = 32 elements per thread, index bits of u_lo):
//   L1 (gather, pass 1): reg bits -> u_lo bits 0..4, lane bits 4,5 -> 5,6,
//       lane bits 0..3 -> 7..10, wave bits -> 11..LB-1.  Stages 0..4 run
//       in registers; stages 5 and 6 after exchanging lane bit 4 / 5 with
//       register bit 0 / 1 (v_permlane16_swap / v_permlane32_swap).
//   One LDS transpose (XOR-swizzled, conflict free for both sides) to
//   L2: reg bits -> 7..11, lane bits 0..3 -> 0..3, the rest below; the last
//       one or two stages again after permlane swaps.
#include "cmm_internal.h"

namespace cmm {

// ------------------------------------------------------------------- plan
// For operand op (0: rows of A with tab1, 1: columns of B with tab2) and
// repetition t, over the n indices in ascending order:
//   first[t][r]   lowest index whose lo-bucket is r, or -1;
//   extras        (index, first index of its bucket) for every other index,
//                 grouped by rank inside the bucket (rank 1 = second);
//   meta          hi(h(index)) xor hi(h(first)) | (sign(index) xor sign(first)) << 31;
//   roff[t][r]    start of rank r in extras (r = 1 .. maxrank + 1);
//   maxrank[t].
namespace {

constexpr int kPlanThreads = 1024;
constexpr int32_t kNone = 0x7FFFFFFF;

// One work-group per repetition.  LDS: cur[b_lo], nxt[b_lo] (int32) and
// rank[n] (int32).  Rank rounds: round 0 takes the lowest index of every
// lo-bucket (atomicMin, order independent); round r takes the lowest index
// among those not yet ranked.  Hence rank(i) = number of lower indices in
// the same lo-bucket, computed deterministically.  The non-first indices
// are then laid out bucket by bucket (a "chain" per bucket with two or
// more indices), each chain in rank order.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* tmp, int32_t* total) {
  // 1024 threads: inclusive scan within wavefronts, then over wave sums
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int q = 0; q < kPlanThreads / 64; ++q) { const int32_t s = tmp[q]; tmp[q] = acc; acc += s; }
    *total = acc;
  }
  __syncthreads();
  const int32_t r = x - v + tmp[wv];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const uint32_t* __restrict__ tab,
                                                            int64_t n, int lb, PlanView pv) {
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const int blo = 1 << lb;
  const uint32_t lomask = (uint32_t)blo - 1u;
  const uint32_t* tb = tab + (size_t)t * n;
  int32_t* first = pv.first + (size_t)t * blo;
  int32_t* cstart = pv.cstart + (size_t)t * (n + 2);
  uint2* pairs = pv.pairs + (size_t)t * n;
  extern __shared__ int32_t sh[];
  int32_t* cur = sh;                // [b_lo]  first index per bucket
  int32_t* nxt = sh + blo;          // [b_lo]  scratch, then counts, then chain offsets
  int16_t* rank = reinterpret_cast<int16_t*>(sh + 2 * blo);   // [n] (ranks < 2^15)
  int32_t* misc = sh + 2 * blo + (n + 1) / 2;                   // [2 + 16]: more, total, wave sums
  int32_t& s_more = misc[0];
  int32_t* s_total = misc + 1;
  int32_t* wsum = misc + 2;
  for (int r = tid; r < blo; r += kPlanThreads) cur[r] = kNone;
  for (int64_t i = tid; i < n; i += kPlanThreads) rank[i] = -1;
  __syncthreads();
  for (int64_t i = tid; i < n; i += kPlanThreads) atomicMin(&cur[tb[i] & lomask], (int32_t)i);
  __syncthreads();
  for (int r = tid; r < blo; r += kPlanThreads) first[r] = cur[r] == kNone ? -1 : cur[r];
  for (int64_t i = tid; i < n; i += kPlanThreads)
    if (cur[tb[i] & lomask] == (int32_t)i) rank[i] = 0;
  __syncthreads();
  for (int round = 1;; ++round) {
    for (int r = tid; r < blo; r += kPlanThreads) nxt[r] = kNone;
    if (tid == 0) s_more = 0;
    __syncthreads();
    for (int64_t i = tid; i < n; i += kPlanThreads)
      if (rank[i] < 0) atomicMin(&nxt[tb[i] & lomask], (int32_t)i);
    __syncthreads();
    for (int64_t i = tid; i < n; i += kPlanThreads)
      if (rank[i] < 0 && nxt[tb[i] & lomask] == (int32_t)i) { rank[i] = (int16_t)round; s_more = 1; }
    __syncthreads();
    const int more = s_more;
    __syncthreads();   // everyone read s_more before it is reset
    if (!more) break;
  }
  // rows per bucket
  for (int r = tid; r < blo; r += kPlanThreads) nxt[r] = 0;
  __syncthreads();
  for (int64_t i = tid; i < n; i += kPlanThreads) atomicAdd(&nxt[tb[i] & lomask], 1);
  __syncthreads();
  // each thread owns a run of consecutive buckets: chain lengths and count
  const int per = blo / kPlanThreads > 0 ? blo / kPlanThreads : 1;
  const int r0 = tid * per;
  int32_t len_sum = 0, chains = 0;
  for (int r = r0; r < r0 + per && r < blo; ++r) {
    const int32_t c = nxt[r];
    if (c >= 2) { len_sum += c - 1; chains += 1; }
  }
  const int32_t off0 = block_exclusive_scan(len_sum, wsum, s_total);
  const int32_t total_extras = *s_total;
  const int32_t ch0 = block_exclusive_scan(chains, wsum, s_total);
  const int32_t total_chains = *s_total;
  // chain starts and per-bucket offsets (nxt[r] becomes the bucket's offset)
  {
    int32_t off = off0, ch = ch0;
    for (int r = r0; r < r0 + per && r < blo; ++r) {
      const int32_t c = nxt[r];
      if (c >= 2) {
        cstart[ch] = off;
        nxt[r] = off;
        off += c - 1;
        ch += 1;
      }
    }
  }
  if (tid == 0) {
    cstart[total_chains] = total_extras;
    pv.nchains[t] = total_chains;
  }
  __syncthreads();
  for (int64_t i = tid; i < n; i += kPlanThreads) {
    const int rk = rank[i];
    if (rk >= 1) {
      const uint32_t e = tb[i];
      const int32_t f = cur[e & lomask];
      const uint32_t ef = tb[f];
      const uint32_t hx = ((e & kBucketMask) >> lb) ^ ((ef & kBucketMask) >> lb);
      pairs[nxt[e & lomask] + rk - 1] =
          make_uint2((uint32_t)i | ((uint32_t)f << 16), hx | ((e ^ ef) & kSignBit));
    }
  }
}

// ----------------------------------------------------------------- window
// The transform is the same for any order of the bucket bits (the
// Walsh-Hadamard matrix of 2^m points is the Kronecker product of m 2-point
// ones), so a work unit may transform any lb of the m bits and fold the
// others.  Multiply-add-shift hashes of consecutive indices can crowd a
// window of bits onto few values (long collision chains, whose fix-ups
// dominate the unit's time), while another window spreads them.  One
// work-group per repetition counts, for every window s, the rows beyond the
// first in each bucket of the window and (weighted 8) the rows beyond the
// sixth, over both tables; the cheapest window (the lowest s on ties) is
// applied by rotating the bucket bits right by s.  Windows are tried up to
// s = kMaxWindow (the tile of the reduce that restores the order).
__global__ __launch_bounds__(kPlanThreads) void window_kernel(
    const uint32_t* __restrict__ tab1, const uint32_t* __restrict__ tab2, int64_t n1, int64_t n2,
    int log2b, int lb, uint32_t* __restrict__ rtab1, uint32_t* __restrict__ rtab2,
    int32_t* __restrict__ rot) {
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const int blo = 1 << lb;
  const uint32_t lomask = (uint32_t)blo - 1u;
  const uint32_t mmask = (uint32_t)(((uint64_t)1 << log2b) - 1u);
  extern __shared__ int32_t cnt[];   // [b_lo]
  __shared__ int32_t s_part[kPlanThreads / 64];
  __shared__ int32_t s_best;
  const int smax = log2b - lb < kMaxWindow ? log2b - lb : kMaxWindow;
  int32_t best_cost = 0x7FFFFFFF, best_s = 0;
  for (int sh = 0; sh <= smax; ++sh) {
    int32_t cost = 0;
    for (int op = 0; op < 2; ++op) {
      const uint32_t* tb = (op ? tab2 : tab1) + (size_t)t * (op ? n2 : n1);
      const int64_t n = op ? n2 : n1;
      for (int r = tid; r < blo; r += kPlanThreads) cnt[r] = 0;
      __syncthreads();
      for (int64_t i = tid; i < n; i += kPlanThreads)
        atomicAdd(&cnt[((tb[i] & mmask) >> sh) & lomask], 1);
      __syncthreads();
      int32_t mine = 0;
      for (int r = tid; r < blo; r += kPlanThreads) {
        const int32_t c = cnt[r];
        mine += (c > 1 ? c - 1 : 0) + 8 * (c > 6 ? c - 6 : 0);
      }
      for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
      if ((tid & 63) == 0) s_part[tid >> 6] = mine;
      __syncthreads();
      for (int q = 0; q < kPlanThreads / 64; ++q) cost += s_part[q];
      __syncthreads();   // s_part and cnt are reused
    }
    if (cost < best_cost) { best_cost = cost; best_s = sh; }   // uniform
  }
  if (tid == 0) { s_best = best_s; rot[t] = best_s; }
  __syncthreads();
  const int sh = s_best;
  for (int op = 0; op < 2; ++op) {
    const int64_t n = op ? n2 : n1;
    const uint32_t* tb = (op ? tab2 : tab1) + (size_t)t * n;
    uint32_t* ro = (op ? rtab2 : rtab1) + (size_t)t * n;
    for (int64_t i = tid; i < n; i += kPlanThreads) {
      const uint32_t e = tb[i];
      const uint32_t h = e & mmask;
      const uint32_t hr = sh == 0 ? h : ((h >> sh) | (h << (log2b - sh))) & mmask;
      ro[i] = hr | (e & kSignBit);
    }
  }
}

// Sum of the partials of a rotated frame back into natural order.  Natural
// index u = a 2^s + c (c < 2^s) sits at rotated position c 2^(m - s) + a, so
// a tile of 512 consecutive natural indices is, for each of the 2^s values
// of c, a run of 512 / 2^s (>= 16) consecutive rotated positions: read per c
// (coalesced, partials summed in group order, eight loads in flight),
// transposed through LDS, written in natural order.
constexpr int kRedTile = 512;
__global__ __launch_bounds__(256) void reduce_window_kernel(const double* __restrict__ parts,
                                                            int g, int d, int log2b,
                                                            const int32_t* __restrict__ rot,
                                                            double* __restrict__ out) {
  __shared__ double tile[kRedTile + (1 << kMaxWindow)];
  const int t = blockIdx.y;
  const int s = rot[t];
  const int64_t b = (int64_t)1 << log2b;
  const int64_t u0 = (int64_t)blockIdx.x * kRedTile;   // natural tile start
  const int C = 1 << s, A = kRedTile >> s;              // values of c; run length per c
  const int64_t a0 = u0 >> s;
  const size_t len = (size_t)d * b;
  for (int i = threadIdx.x; i < kRedTile; i += 256) {
    const int c = i / A, j = i - c * A;
    const int64_t up = ((int64_t)c << (log2b - s)) + a0 + j;   // rotated position
    const double* src = parts + (size_t)t * b + up;
    double acc = 0.0;
    int q = 0;
    for (; q + 8 <= g; q += 8) {
      double v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = src[(size_t)(q + r) * len];
#pragma unroll
      for (int r = 0; r < 8; ++r) acc += v[r];
    }
    for (; q < g; ++q) acc += src[(size_t)q * len];
    tile[c * (A + 1) + j] = acc;   // padded rows: the transposed reads spread over banks
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kRedTile; i += 256) {
    const int c = i & (C - 1), j = i >> s;
    out[(size_t)t * b + u0 + i] = tile[c * (A + 1) + j];
  }
}

}  // namespace

cmm_status launch_reduce_window(const double* parts, int g, int d, int log2b, const int32_t* rot,
                                double* out, hipStream_t s) {
  const int64_t b = (int64_t)1 << log2b;
  if (!rot) return launch_reduce_partials(parts, g, (size_t)d * b, out, s);
  ProfScope prof_("reduce", s);
  if (b < kRedTile) {
    set_error("reduce (window): needs b >= 512");
    return CMM_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(reduce_window_kernel, dim3((unsigned)(b / kRedTile), d), dim3(256), 0, s,
                     parts, g, d, log2b, rot, out);
  return hip_check(hipGetLastError(), "reduce (window) kernel launch");
}

cmm_status launch_window(const uint32_t* tab1, const uint32_t* tab2, int d, int64_t n_rows,
                         int64_t n_cols, int log2b, int lb, uint32_t* rtab1, uint32_t* rtab2,
                         int32_t* rot, hipStream_t s) {
  ProfScope prof_("plan", s);
  if (lb > log2b || lb > 14 || log2b > 31) {
    set_error("window: needs lb <= log2b, lb <= 14, log2b <= 31");
    return CMM_EUNSUPPORTED;
  }
  const size_t lds = sizeof(int32_t) * ((size_t)1 << lb);
  hipError_t e = hipFuncSetAttribute((const void*)window_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_check(e, "window: set LDS size");
  hipLaunchKernelGGL(window_kernel, dim3(d), dim3(kPlanThreads), lds, s, tab1, tab2, n_rows,
                     n_cols, log2b, lb, rtab1, rtab2, rot);
  return hip_check(hipGetLastError(), "window kernel launch");
}

}  // namespace cmm

#include "wht_regs.h"

namespace cmm {
namespace {

// ------------------------------------------------------------ main kernel
// One work unit: repetition t, slice u_hi, inner indices [k0, k1) (group g
// of the partial p_hat).  Starts by writing LDS, so a caller running units
// back to back separates them with a barrier.
template <typename T, int LB>
__device__ __forceinline__ void compress_unit(const CompressArgs& a, int g, int t, uint32_t uhi,
                                              int64_t k0, int64_t k1, unsigned char* smem) {
  constexpr int E = Cfg<T, LB>::E;
  constexpr int NT = Cfg<T, LB>::NT;
  constexpr int BLO = 1 << LB;
  T* xbuf = reinterpret_cast<T*>(smem);                          // BLO
  T* rowA = xbuf + BLO + BLO / 128;                              // n_rows (16-byte aligned)
  T* rowB = rowA + row_pitch<T>(a.n_rows);                       // n_cols (+ pad)
  uint2* exl = reinterpret_cast<uint2*>(rowB + row_pitch<T>(a.n_cols));
  if (threadIdx.x == 0) { rowA[a.n_rows] = T(0); rowB[a.n_cols] = T(0); }

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t base1 = ((uint32_t)((lane >> 4) & 1) << 5) | ((uint32_t)((lane >> 5) & 1) << 6) |
                         ((uint32_t)(lane & 15) << 7) | ((uint32_t)w << 11);
  // First rows of the thread's 32 consecutive buckets and their folded
  // signs.  Empty buckets point at a zero pad element after the staged row
  // (index n), so the gather below is branch free.
  uint32_t fa[E / 2], fb[E / 2];
  uint32_t nega = 0, negb = 0;
  {
    const int32_t* f1 = a.planA.first + (size_t)t * BLO + base1;
    const int32_t* f2 = a.planB.first + (size_t)t * BLO + base1;
    const uint32_t* t1 = a.tab1 + (size_t)t * a.n_rows;
    const uint32_t* t2 = a.tab2 + (size_t)t * a.n_cols;
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
  // Non-first rows (constant over k): copied once into LDS when they fit.
  const int32_t* gcA = a.planA.cstart + (size_t)t * (a.n_rows + 2);
  const int32_t* gcB = a.planB.cstart + (size_t)t * (a.n_cols + 2);
  const int nchA = a.planA.nchains[t], nchB = a.planB.nchains[t];
  const int cntA = gcA[nchA], cntB = gcB[nchB];
  // entries (8 bytes) plus chain starts (4 bytes each, two per 8-byte slot)
  const bool ex_lds = (int64_t)cntA + cntB + (nchA + nchB + 4) / 2 + 1 <= a.ex_cap;
  const uint2* gA = a.planA.pairs + (size_t)t * a.n_rows;
  const uint2* gB = a.planB.pairs + (size_t)t * a.n_cols;
  if (ex_lds) {
    for (int q = threadIdx.x; q < cntA; q += NT) exl[q] = gA[q];
    for (int q = threadIdx.x; q < cntB; q += NT) exl[cntA + q] = gB[q];
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

  const uint32_t w1 = swz(l1p_lane(lane, w));          // + l1p_reg(e) (additive)
  const uint32_t r2lane = swz(l2_lane<LB>(lane, w, false));   // + swz(l2_reg(e))

  T acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = T(0);

  const T* At = reinterpret_cast<const T*>(a.At);
  const T* Bm = reinterpret_cast<const T*>(a.B);
  const bool dma = a.dma != 0;
  if (k0 < k1) {
    stage_row<T, NT>(rowA, At + k0 * a.n_rows, a.n_rows, dma);
    stage_row<T, NT>(rowB, Bm + k0 * a.ldb, a.n_cols, dma);
  }


  for (int64_t k = k0; k < k1; ++k) {
    if (dma) wait_dma();
    __syncthreads();
    // rank rounds of both operands share the barriers
    if (nchA + nchB > 0) {
      { if (ex_lds) fix_chains<T, NT>(rowA, lexA, lcsA, nchA, uhi); else fix_chains<T, NT>(rowA, gA, gcA, nchA, uhi); }
      { if (ex_lds) fix_chains<T, NT>(rowB, lexB, lcsB, nchB, uhi); else fix_chains<T, NT>(rowB, gB, gcB, nchB, uhi); }
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
    __syncthreads();   // every gather is done: the row buffers can be refilled
    if (k + 1 < k1) {
      stage_row<T, NT>(rowA, At + (k + 1) * a.n_rows, a.n_rows, dma);
      stage_row<T, NT>(rowB, Bm + (k + 1) * a.ldb, a.n_cols, dma);
    }
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
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = fma(X[e], Y[e], acc[e]);
    // xbuf is rewritten next iteration only after the rank-round barriers
  }
  // write the slice of the partial p_hat
  const int64_t b = (int64_t)1 << a.log2b;
  double* dst = a.partial + ((size_t)g * a.d + t) * b + ((int64_t)uhi << LB);
  const uint32_t r2after = l2_lane<LB>(lane, w, true);
#pragma unroll
  for (int e = 0; e < E; ++e) dst[r2after | l2_reg<LB>(e, true)] = (double)acc[e];
}

template <typename T, int LB>
__global__ __launch_bounds__((1 << LB) / 32) void compress_kernel(CompressArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b_hi_bits = a.log2b - LB;
  const int64_t nunits = (int64_t)a.d << b_hi_bits;
  // XCD-aware order: work-groups are dealt to the 8 XCDs round robin, so
  // the groups one XCD runs share a k-range (their input rows hit its L2).
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
  compress_unit<T, LB>(a, g, t, uhi, k0, k1, smem);
}

// Persistent form over a batch of problems: every work-group takes work
// items (pair, repetition, slice, k-range) from a queue, in the order of
// the item list, until the queue is empty.
template <typename T, int LB>
__global__ __launch_bounds__((1 << LB) / 32) void compress_batched_kernel(
    char* __restrict__ ws, const BatchPair* __restrict__ pairs,
    const BatchItem* __restrict__ items, int n_items, int* __restrict__ queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();   // the previous unit is done with LDS and s_item
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;   // uniform: every wave leaves
    const BatchItem bi = items[it];
    const BatchPair bp = pairs[bi.pair];
    CompressArgs a;
    a.At = ws + bp.at;
    a.B = bp.bc >= 0 ? static_cast<const void*>(ws + bp.bc) : bp.B;
    a.ldb = bp.ldb;
    a.n_rows = bp.n_rows;
    a.n_cols = bp.n_cols;
    a.n_inner = bp.n_inner;
    a.tab1 = bp.rtab1 >= 0 ? reinterpret_cast<const uint32_t*>(ws + bp.rtab1) : bp.tab1;
    a.tab2 = bp.rtab2 >= 0 ? reinterpret_cast<const uint32_t*>(ws + bp.rtab2) : bp.tab2;
    a.planA = carve_plan(ws + bp.planA, bp.d, bp.n_rows, LB);
    a.planB = carve_plan(ws + bp.planB, bp.d, bp.n_cols, LB);
    a.d = bp.d;
    a.log2b = bp.log2b;
    a.groups = bp.groups;
    a.partial = reinterpret_cast<double*>(ws + bp.partial);
    a.ex_cap = bp.ex_cap;
    a.dma = bp.dma;
    a.variant = 0;
    const int b_hi_bits = a.log2b - LB;
    const int t = (int)(bi.unit >> b_hi_bits);
    const uint32_t uhi = bi.unit & ((1u << b_hi_bits) - 1u);
    const int64_t k_per = (a.n_inner + a.groups - 1) / a.groups;
    const int64_t k0 = (int64_t)bi.group * k_per;
    const int64_t k1 = (k0 + k_per) < a.n_inner ? (k0 + k_per) : a.n_inner;
    compress_unit<T, LB>(a, (int)bi.group, t, uhi, k0, k1, smem);
  }
}

// ------------------------------------------------ 16 elements per thread
// (layout and transform passes in wht_regs.h)

// SINGLE: one row buffer shared by the two operands (A staged, fixed up and
// gathered before B), for rows too long to stage both at once.
// DESC: collision fix-ups from per-thread descriptors (rows then carry 64
// spare elements after the zero pad); otherwise by walking the plan's chain
// lists.  Separate instances, because the chain-walking code, even when not
// executed, slows the loop it sits in.
constexpr int kSlots16 = 2;   // descriptor slots per thread and operand (512 threads)
// One-word descriptors of two-row chains: slots per thread and operand in
// the same LDS (three words per full slot and operand, plus the partial
// slot's kPairOvf16 positions or more).
constexpr int kPairSlots16 = 7;
constexpr int kPairOvf16 = (kPairSlots16 * 512 - 3 * kSlots16 * 512 + 2) / 3;

template <typename T, bool DESC>
__host__ __device__ constexpr int64_t pitch16(int64_t n) {
  return row_pitch<T>(DESC ? n + 64 : n);
}

// padded transpose buffer of the 16-element layout (pad16 of 2^13 - 1 < it)
constexpr int64_t kXlen16 = (1 << 13) + (1 << 13) / 64 + 16;

// Elements of one row area of the aliased layout: a staged row with its
// spare elements, or one operand's padded transpose.
template <typename T>
__host__ __device__ constexpr int64_t alias_area16(int64_t n) {
  return pitch16<T, true>(n) > kXlen16 ? pitch16<T, true>(n) : kXlen16;
}

// ALIAS: no separate transpose buffer; once a step's rows are gathered into
// registers, A's row area takes the next step's row at once and both
// transposes go through B's row area, whose next row is staged after the
// second transpose.  This keeps both rows and the descriptors in LDS for
// rows too long to sit beside a transpose buffer.
// FIX (descriptor layouts): 1 the general descriptors below; 0 the
// repetition has no collision chains in either operand (no descriptors, no
// fix-ups: a unit without that code runs faster); 2 every chain of both
// operands has two rows and they fit kPairSlots16 one-word descriptors.
template <typename T, bool SINGLE, bool DESC, bool ALIAS = false, int FIX = 1>
__device__ __forceinline__ void compress16_unit(const CompressArgs& a, int g, int t, uint32_t uhi,
                                                int64_t k0, int64_t k1, unsigned char* smem) {
  static_assert(!(SINGLE && DESC), "descriptors need both rows staged");
  static_assert(!ALIAS || DESC, "the aliased layout is a descriptor layout");
  constexpr int LB = 13;
  constexpr int E = 16;
  constexpr int NT = 512;
  constexpr int BLO = 1 << LB;
  constexpr int XLEN = kXlen16;   // padded transpose buffer
  T* xbuf = reinterpret_cast<T*>(smem);
  T* rowA = ALIAS ? xbuf : xbuf + XLEN;
  const int64_t pitch1 = ALIAS ? alias_area16<T>(a.n_rows)
                       : SINGLE ? (row_pitch<T>(a.n_rows) > row_pitch<T>(a.n_cols)
                                       ? row_pitch<T>(a.n_rows) : row_pitch<T>(a.n_cols))
                                : pitch16<T, DESC>(a.n_rows);
  T* rowB = SINGLE ? rowA : rowA + pitch1;
  const int64_t pitch2 = ALIAS ? alias_area16<T>(a.n_cols) : pitch16<T, DESC>(a.n_cols);
  uint2* exl = reinterpret_cast<uint2*>(rowB + (SINGLE ? 0 : pitch2) + (SINGLE ? pitch1 : 0));
  // transpose area of X and Y
  T* xb = ALIAS ? rowB : xbuf;
  if (!SINGLE && threadIdx.x == 0) { rowA[a.n_rows] = T(0); rowB[a.n_cols] = T(0); }

  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t l4 = (lane >> 4) & 1, l5 = (lane >> 5) & 1, l3 = (lane >> 3) & 1;
  const uint32_t base1 = (l4 << 4) | (l5 << 5) | ((lane & 15) << 6) | (w << 10);
  // byte offsets (from the LDS base) of the gather sources of the thread's
  // 16 buckets, and their folded signs
  uint32_t offA[E], offB[E];
  uint32_t nega = 0, negb = 0;
  {
    const int32_t* f1 = a.planA.first + (size_t)t * BLO + base1;
    const int32_t* f2 = a.planB.first + (size_t)t * BLO + base1;
    const uint32_t* t1 = a.tab1 + (size_t)t * a.n_rows;
    const uint32_t* t2 = a.tab2 + (size_t)t * a.n_cols;
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
  const int32_t* gcA = a.planA.cstart + (size_t)t * (a.n_rows + 2);
  const int32_t* gcB = a.planB.cstart + (size_t)t * (a.n_cols + 2);
  const int nchA = a.planA.nchains[t], nchB = a.planB.nchains[t];
  const int cntA = gcA[nchA], cntB = gcB[nchB];
  // entries (8 bytes) plus chain starts (4 bytes each, two per 8-byte slot)
  const bool ex_lds = (int64_t)cntA + cntB + (nchA + nchB + 4) / 2 + 1 <= a.ex_cap;
  const uint2* gA = a.planA.pairs + (size_t)t * a.n_rows;
  const uint2* gB = a.planB.pairs + (size_t)t * a.n_cols;
  if (!DESC && ex_lds) {
    for (int q = threadIdx.x; q < cntA; q += NT) exl[q] = gA[q];
    for (int q = threadIdx.x; q < cntB; q += NT) exl[cntA + q] = gB[q];
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
  // Collision descriptors.  Thread tid owns chains tid + j NT (j < kSlots16);
  // a descriptor (three words in LDS, built once per work unit) holds the
  // chain's target and its next five rows as 15-bit row indices with their
  // signs relative to the target (absent rows: the zero pad index n; an
  // absent chain targets the lane's spare element after the pad):
  //   w0 = target | m1 << 15 | s1 << 30 | more << 31
  //   w1 = m2 | m3 << 15 | s2 << 30 | s3 << 31
  //   w2 = m4 | m5 << 15 | s4 << 30 | s5 << 31
  // A chain with more rows (a bucket of seven or more) and chains beyond
  // the slots are finished from the plan's lists.
  //
  // Slot positions: chain c sits at position p (thread p mod NT, slot
  // p / NT).  When the chains fit the slots they are placed with the chains
  // of three or more rows first (a block scan), so only the waves whose
  // positions hold such chains read words 1 and 2, and waves past the last
  // chain skip a slot (both tests are wave-uniform); otherwise position c
  // holds chain c.  A chain with more than six rows keeps its index in
  // word 2, adds only its first four rows here and is finished in the rare
  // pass; its word 2 then holds where its plan entries start and how many
  // there are (beg | count << 15, both below n).
  // A third, partial slot (positions kSlots16 NT + i, i < ovf, held by
  // threads i < ovf) uses the LDS the launcher found left over.
  uint32_t* dsc = reinterpret_cast<uint32_t*>(exl);   // [word][operand][slot][NT]
  uint32_t* ovf = dsc + 3 * 2 * kSlots16 * NT;         // [word][operand][ovf]
  const int novf = DESC ? a.ovf16 : 0;
  const int npos = kSlots16 * NT + novf;              // descriptor positions per operand
  auto dref = [&](int word, int op, int j) -> uint32_t& {
    if (j < kSlots16) return dsc[((word * 2 + op) * kSlots16 + j) * NT + threadIdx.x];
    return ovf[(word * 2 + op) * novf + threadIdx.x];   // threads below novf only
  };
  auto dslot = [&](int word, int op, int pos) -> uint32_t& {
    if (pos < kSlots16 * NT) return dsc[((word * 2 + op) * kSlots16 + pos / NT) * NT + pos % NT];
    return ovf[(word * 2 + op) * novf + (pos - kSlots16 * NT)];
  };
  // slot j of this thread exists (the partial slot only below novf)
  auto has_slot = [&](int j) -> bool { return j < kSlots16 || (int)threadIdx.x < novf; };
  int nlong[2] = {0, 0};
  if constexpr (DESC && FIX == 1) {
    // the transpose buffer is idle until the k loop: scan scratch
    int32_t* s_scan = reinterpret_cast<int32_t*>(xbuf);
    __syncthreads();   // a previous work unit's last transposed reads are done
    for (int op = 0; op < 2; ++op) {
      const int32_t* gc = op ? gcB : gcA;
      const uint2* gp = op ? gB : gA;
      const int nch = op ? nchB : nchA;
      const uint32_t pad = (uint32_t)(op ? a.n_cols : a.n_rows);
      const bool ordered = nch <= npos;
      const int per = (nch + NT - 1) / NT;
      const int c0 = (int)threadIdx.x * per;
      int mine = 0;
      if (ordered)
        for (int c = c0; c < c0 + per && c < nch; ++c) mine += (gc[c + 1] - gc[c] > 1) ? 1 : 0;
      int incl = mine;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if ((int)lane >= off) incl += y;
      }
      if (lane == 63u) s_scan[w] = incl;
      __syncthreads();
      int wbase = 0, total = 0;
      for (int q = 0; q < NT / 64; ++q) {
        const int x = s_scan[q];
        if (q < (int)w) wbase += x;
        total += x;
      }
      __syncthreads();   // s_scan is reused by the next operand
      nlong[op] = ordered ? total : 0;
      int lpos = wbase + incl - mine;                 // next position of a longer chain
      int ppos = total + c0 - (wbase + incl - mine);  // next position of a two-row chain
      for (int j = 0; j <= kSlots16; ++j) {           // absent chains
        if (has_slot(j) && (int)threadIdx.x + j * NT >= nch) {
          dref(0, op, j) = (pad + 1u + (threadIdx.x & 63u)) | (pad << 15);
          dref(1, op, j) = pad | (pad << 15);
          dref(2, op, j) = pad | (pad << 15);
        }
      }
      const int cb = ordered ? c0 : (int)threadIdx.x;
      const int ce = ordered ? (c0 + per < nch ? c0 + per : nch) : nch;
      for (int c = cb; c < ce; c += ordered ? 1 : NT) {
        const int beg = gc[c], end = gc[c + 1];
        int pos = c;
        if (ordered) pos = (end - beg > 1) ? lpos++ : ppos++;
        if (pos >= npos) continue;
        uint32_t m[6] = {gp[beg].x >> 16, pad, pad, pad, pad, pad};
        uint32_t sg[6] = {0, 0, 0, 0, 0, 0};
        for (int r = 0; r < 5 && beg + r < end; ++r) {
          const uint2 y = gp[beg + r];
          m[r + 1] = y.x & 0xFFFFu;
          sg[r + 1] = (y.y >> 31) ^ (__popc(uhi & (y.y & kBucketMask)) & 1u);
        }
        const uint32_t more = end - beg > 5 ? 1u : 0u;
        dslot(0, op, pos) = m[0] | (m[1] << 15) | (sg[1] << 30) | (more << 31);
        dslot(1, op, pos) = m[2] | (m[3] << 15) | (sg[2] << 30) | (sg[3] << 31);
        dslot(2, op, pos) = more ? (uint32_t)beg | ((uint32_t)(end - beg) << 15)
                                 : m[4] | (m[5] << 15) | (sg[4] << 30) | (sg[5] << 31);
      }
    }
  }
  // Fix-ups of both operands from their descriptors: every live slot adds
  // its target and first row; the rows past those only in the waves whose
  // positions hold longer chains (all waves when the order is the identity).
  // The sum is taken in rank order and stored once into the target; a chain
  // with more rows stores its partial sum (in the row's own type, so no
  // extra rounding) and the rare pass continues from its fifth row.
  const int wave_pos = (int)(threadIdx.x & ~63u);
  // Two-row chains only (FIX = 2): one word per chain, w = target | m1 << 15
  // | s1 << 30, in the descriptor LDS; chain c at slot c / NT of thread
  // c mod NT.  A wave takes a slot when one of its positions holds a chain;
  // an absent position adds the zero pad onto its lane's spare element.
  uint32_t* pdsc = reinterpret_cast<uint32_t*>(exl);   // [operand][slot][NT]
  if constexpr (DESC && FIX == 2) {
    // slots that some wave takes (j NT < nch); the chain starts of all of
    // them, then their entries, are fetched as independent loads
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const int32_t* gc = op ? gcB : gcA;
      const uint2* gp = op ? gB : gA;
      const int nch = op ? nchB : nchA;
      const uint32_t pad = (uint32_t)(op ? a.n_cols : a.n_rows);
      int beg[kPairSlots16];
#pragma unroll
      for (int j = 0; j < kPairSlots16; ++j) {
        const int c = (int)threadIdx.x + j * NT;
        beg[j] = c < nch ? gc[c] : -1;
      }
      uint2 y[kPairSlots16];
#pragma unroll
      for (int j = 0; j < kPairSlots16; ++j) y[j] = beg[j] >= 0 ? gp[beg[j]] : make_uint2(0u, 0u);
#pragma unroll
      for (int j = 0; j < kPairSlots16; ++j) {
        if (j * NT >= nch) continue;   // no wave takes the slot
        uint32_t wd = (pad + 1u + (threadIdx.x & 63u)) | (pad << 15);
        if (beg[j] >= 0) {
          const uint32_t sg = (y[j].y >> 31) ^ (__popc(uhi & (y[j].y & kBucketMask)) & 1u);
          wd = (y[j].x >> 16) | ((y[j].x & 0xFFFFu) << 15) | (sg << 30);
        }
        pdsc[(op * kPairSlots16 + j) * NT + threadIdx.x] = wd;
      }
    }
  }
  // Slots of this wave that hold chains, per operand (slot j is live when
  // one of the wave's positions j NT + lane has a chain), fixed for the
  // unit and kept scalar: with few chains most waves skip the fix-up with
  // one test, and the waves with one live slot per operand take a short path
  // instead of testing every slot on every k.
  int nsl[2] = {0, 0};
  if constexpr (DESC && FIX == 2 && !ALIAS) {
    const int wp = __builtin_amdgcn_readfirstlane(wave_pos);
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const int nch = op ? nchB : nchA;
      const int m = nch > wp ? (nch - wp + NT - 1) / NT : 0;
      nsl[op] = __builtin_amdgcn_readfirstlane(m < kPairSlots16 ? m : kPairSlots16);
    }
  }
  auto fix_pairs = [&]() {
    // (the aliased layout's units hold many chains: there every slot is
    // tested, which keeps the code short)
    if constexpr (!ALIAS) {
      if (nsl[0] + nsl[1] == 0) return;
      if (nsl[0] <= 1 && nsl[1] <= 1) {
        uint32_t q[2];
        T v0[2], v1[2];
#pragma unroll
        for (int op = 0; op < 2; ++op) {
          if (nsl[op] == 0) continue;
          const T* row = op ? rowB : rowA;
          q[op] = pdsc[(op * kPairSlots16) * NT + threadIdx.x];
          v0[op] = row[q[op] & 0x7FFFu];
          v1[op] = row[(q[op] >> 15) & 0x7FFFu];
        }
#pragma unroll
        for (int op = 0; op < 2; ++op) {
          if (nsl[op] == 0) continue;
          T* row = op ? rowB : rowA;
          row[q[op] & 0x7FFFu] = v0[op] + flip_sign(v1[op], ((q[op] >> 30) & 1u) << 31);
        }
        return;
      }
    }
    uint32_t q[2][kPairSlots16];
    T v0[2][kPairSlots16], v1[2][kPairSlots16];
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const T* row = op ? rowB : rowA;
      const int nch = op ? nchB : nchA;
#pragma unroll
      for (int j = 0; j < kPairSlots16; ++j) {
        if (ALIAS ? wave_pos + j * NT >= nch : j >= nsl[op]) continue;   // wave-uniform
        q[op][j] = pdsc[(op * kPairSlots16 + j) * NT + threadIdx.x];
        v0[op][j] = row[q[op][j] & 0x7FFFu];
        v1[op][j] = row[(q[op][j] >> 15) & 0x7FFFu];
      }
    }
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      T* row = op ? rowB : rowA;
      const int nch = op ? nchB : nchA;
#pragma unroll
      for (int j = 0; j < kPairSlots16; ++j) {
        if (ALIAS ? wave_pos + j * NT >= nch : j >= nsl[op]) continue;
        row[q[op][j] & 0x7FFFu] = v0[op][j] + flip_sign(v1[op][j], ((q[op][j] >> 30) & 1u) << 31);
      }
    }
  };
  constexpr int kJ = kSlots16 + 1;   // full slots and the partial one
  auto fix_desc = [&]() {
    bool rare = false;
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      T* row = op ? rowB : rowA;
      const int nch_op = op ? nchB : nchA;
      const bool all = nch_op > npos;   // identity order
      const int nl = nlong[op];
      const uint32_t pad = (uint32_t)(op ? a.n_cols : a.n_rows);
      const uint32_t absent0 = (pad + 1u + (threadIdx.x & 63u)) | (pad << 15);
      const uint32_t padw = pad | (pad << 15);
      // a wave takes a slot when the slot's positions in the wave hold chains
      // (wave-uniform); a lane without the partial slot sums its spare
      bool live[kJ];
      uint32_t q0[kJ];
      T sum[kJ];
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) {
        live[jj] = (jj < kSlots16 || wave_pos < novf) && (all || wave_pos + jj * NT < nch_op);
        q0[jj] = (live[jj] && has_slot(jj)) ? dref(0, op, jj) : absent0;
      }
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) {
        if (!live[jj]) continue;
        const uint32_t w0 = q0[jj];
        const T v1 = row[(w0 >> 15) & 0x7FFFu];
        T acc_ = row[w0 & 0x7FFFu] + flip_sign(v1, ((w0 >> 30) & 1u) << 31);
        if (all || wave_pos + jj * NT < nl) {                  // wave-uniform
          const bool hs = has_slot(jj);
          const uint32_t w1 = hs ? dref(1, op, jj) : padw, w2 = hs ? dref(2, op, jj) : padw;
          const T v2 = row[w1 & 0x7FFFu], v3 = row[(w1 >> 15) & 0x7FFFu];
          // word 2 of a chain with more rows is beg | count << 15 (both < n:
          // the reads stay in the row)
          const bool mr = (w0 >> 31) != 0u;
          const T v4 = row[w2 & 0x7FFFu], v5 = row[(w2 >> 15) & 0x7FFFu];
          acc_ = acc_ + flip_sign(v2, ((w1 >> 30) & 1u) << 31);
          acc_ = acc_ + flip_sign(v3, ((w1 >> 31) & 1u) << 31);
          if (!mr) {
            acc_ = acc_ + flip_sign(v4, ((w2 >> 30) & 1u) << 31);
            acc_ = acc_ + flip_sign(v5, ((w2 >> 31) & 1u) << 31);
          }
        }
        sum[jj] = acc_;
      }
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) {
        if (!live[jj]) continue;
        rare = rare || (q0[jj] >> 31) != 0u;
        row[q0[jj] & 0x7FFFu] = sum[jj];
      }
    }
    const bool extra = nchA > npos || nchB > npos;
    if (rare || extra) {
#pragma unroll
      for (int op = 0; op < 2; ++op) {
        T* row = op ? rowB : rowA;
        const int32_t* gc = op ? gcB : gcA;
        const uint2* gp = op ? gB : gA;
        for (int jj = 0; jj < kJ; ++jj) {
          if (!has_slot(jj)) continue;
          const uint32_t w0 = dref(0, op, jj);
          if (!(w0 >> 31)) continue;
          // rows four onwards, eight plan entries per round trip
          const uint32_t w2 = dref(2, op, jj);
          const int beg = (int)(w2 & 0x7FFFu), end = beg + (int)((w2 >> 15) & 0x7FFFu);
          row[w0 & 0x7FFFu] = chain_sum<T, T, 8>(row, gp, beg + 3, end, uhi, row[w0 & 0x7FFFu]);
        }
        // chains beyond the slots (identity order: disjoint targets), four
        // per thread at a time: their starts, first entries and first two
        // rows are each fetched as independent loads
        const int nch = op ? nchB : nchA;
        for (int c0 = npos + (int)threadIdx.x; c0 < nch; c0 += 4 * NT) {
          int beg[4], end[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int c = c0 + j * NT;
            beg[j] = c < nch ? gc[c] : 0;
            end[j] = c < nch ? gc[c + 1] : 0;
          }
          uint2 y[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) y[j] = beg[j] < end[j] ? gp[beg[j]] : make_uint2(0u, 0u);
          T v0[4], v1[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            v0[j] = beg[j] < end[j] ? row[y[j].x >> 16] : T(0);
            v1[j] = beg[j] < end[j] ? row[y[j].x & 0xFFFFu] : T(0);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (beg[j] >= end[j]) continue;
            const uint32_t neg = (y[j].y >> 31) ^ (__popc(uhi & (y[j].y & kBucketMask)) & 1u);
            T acc_ = v0[j] + flip_sign(v1[j], neg << 31);
            if (end[j] - beg[j] > 1) acc_ = chain_sum<T, T, 4>(row, gp, beg[j] + 1, end[j], uhi, acc_);
            row[y[j].x >> 16] = acc_;
          }
        }
      }
    }
  };
  // transpose addresses: thread part (padded) + register part
  const uint32_t wr_t = pad16(l4 | (l5 << 1) | ((lane & 15) << 6) | (w << 10));
  const uint32_t rd_t = pad16((lane & 7) | (w << 3) | (l4 << 10) | (l5 << 11) | (l3 << 12));
  // register parts: L1' reg bit0 -> 4, bit1 -> 5, bits 2,3 -> 2,3;  L2 reg bits -> 6..9
  auto wr_e = [](int e) -> uint32_t {
    return ((uint32_t)(e & 1) << 4) | ((uint32_t)((e >> 1) & 1) << 5) | (uint32_t)(e & 12);
  };
  auto rd_e = [](int e) -> uint32_t { return pad16((uint32_t)e << 6); };
  const T sgn8 = l3 ? T(-1) : T(1);

  T acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = T(0);

  const T* At = reinterpret_cast<const T*>(a.At);
  const T* Bm = reinterpret_cast<const T*>(a.B);
  const bool dma = a.dma != 0;
  T X[E], Y[E];
  // Rows of k are staged, fixed up and gathered into X, Y before the
  // iteration that transforms them; the gather of k + 1 closes iteration k.
  auto load_k = [&](int64_t kk) {
    stage_row<T, NT>(rowA, At + kk * a.n_rows, a.n_rows, dma);
    if (!SINGLE) stage_row<T, NT>(rowB, Bm + kk * a.ldb, a.n_cols, dma);
  };
  auto fixups = [&]() {
    if constexpr (DESC && FIX == 0) return;
    if constexpr (DESC && FIX == 2) {
      fix_pairs();
      return;
    }
    if constexpr (DESC) {
      fix_desc();
      return;
    }
    { if (ex_lds) fix_chains<T, NT>(rowA, lexA, lcsA, nchA, uhi); else fix_chains<T, NT>(rowA, gA, gcA, nchA, uhi); }
    if (!SINGLE) { if (ex_lds) fix_chains<T, NT>(rowB, lexB, lcsB, nchB, uhi); else fix_chains<T, NT>(rowB, gB, gcB, nchB, uhi); }
  };
  auto gather = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      X[e] = flip_sign(*reinterpret_cast<const T*>(smem + offA[e]), (nega << (31 - e)) & 0x80000000u);
      if (!SINGLE)
        Y[e] = flip_sign(*reinterpret_cast<const T*>(smem + offB[e]), (negb << (31 - e)) & 0x80000000u);
    }
  };
  // SINGLE: B of step kk through the shared buffer (after X is gathered)
  auto single_b = [&](int64_t kk) {
    __syncthreads();   // X gathered: the buffer can take B
    if (threadIdx.x == 0) rowB[a.n_cols] = T(0);
    stage_row<T, NT>(rowB, Bm + kk * a.ldb, a.n_cols, dma);
    if (dma) wait_dma();
    __syncthreads();
    { if (ex_lds) fix_chains<T, NT>(rowB, lexB, lcsB, nchB, uhi); else fix_chains<T, NT>(rowB, gB, gcB, nchB, uhi); }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
      Y[e] = flip_sign(*reinterpret_cast<const T*>(smem + offB[e]), (negb << (31 - e)) & 0x80000000u);
  };
  if (k0 < k1) {
    if (SINGLE && threadIdx.x == 0) rowA[a.n_rows] = T(0);
    load_k(k0);
    if (dma) wait_dma();
    __syncthreads();
    if (!DESC || FIX != 0) {
      fixups();
      __syncthreads();
    }
    gather();
    if (SINGLE) single_b(k0);
  }
  for (int64_t k = k0; k < k1 && ALIAS; ++k) {
    const bool more = k + 1 < k1;
    pass1_16(X);
    __syncthreads();   // every thread's gathers of k are done: the row areas are free
    // The row of A for k + 1 is copied while both transforms run; both
    // transposes go through B's row area, one operand after the other, and
    // the row of B for k + 1 follows the second transpose.
    if (more) stage_row<T, NT>(rowA, At + (k + 1) * a.n_rows, a.n_rows, dma);
#pragma unroll
    for (int e = 0; e < E; ++e) xb[wr_t + wr_e(e)] = X[e];
    pass1_16(Y);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) X[e] = xb[rd_t + rd_e(e)];
    __syncthreads();   // the transposed reads of X are done
#pragma unroll
    for (int e = 0; e < E; ++e) xb[wr_t + wr_e(e)] = Y[e];
    pass2_16(X, sgn8);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) Y[e] = xb[rd_t + rd_e(e)];
    __syncthreads();   // the transposed reads of Y are done: the area takes B's row of k + 1
    if (more) {
      if (threadIdx.x == 0) rowB[a.n_cols] = T(0);   // the transposes overwrote the pad
      stage_row<T, NT>(rowB, Bm + (k + 1) * a.ldb, a.n_cols, dma);
    }
    pass2_16(Y, sgn8);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = fma(X[e], Y[e], acc[e]);
    if (more) {
      if (dma) wait_dma();
      __syncthreads();   // rows of k + 1 and the pad are in place
      if (FIX != 0) {
        fixups();
        __syncthreads();
      }
      gather();
    }
  }
  for (int64_t k = k0; k < k1 && !ALIAS; ++k) {
    const bool more = k + 1 < k1;
    pass1_16(X);
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[wr_t + wr_e(e)] = X[e];
    __syncthreads();
    // every thread has passed its gathers of k (they fed pass 1): the row
    // buffers can be refilled with k + 1
    if (more) {
      if (SINGLE && threadIdx.x == 0) rowA[a.n_rows] = T(0);
      load_k(k + 1);
    }
    // the transposed reads of X overlap pass 1 of Y
#pragma unroll
    for (int e = 0; e < E; ++e) X[e] = xbuf[rd_t + rd_e(e)];
    pass1_16(Y);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[wr_t + wr_e(e)] = Y[e];
    // pass 2 of X overlaps the LDS writes of Y and the row copies of k + 1
    pass2_16(X, sgn8);
    if (more && dma) wait_dma();
    __syncthreads();   // Y transposed and the rows of k + 1 have landed
#pragma unroll
    for (int e = 0; e < E; ++e) Y[e] = xbuf[rd_t + rd_e(e)];
    // the chain-walking fix-ups of k + 1 run while other waves do pass 2 of
    // k; the descriptor fix-ups after it, when X and Y are no longer live
    if (!DESC && more) fixups();
    pass2_16(Y, sgn8);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = fma(X[e], Y[e], acc[e]);
    if (DESC && more) fixups();
    if (more) {
      __syncthreads();
      gather();
      if (SINGLE) single_b(k + 1);
    }
  }
  // final layout L2': reg bit0 -> 10, bit1 -> 11, bits 2,3 -> 8,9;
  // lane bit4 -> 6, bit5 -> 7, bit3 -> 12, bits 0..2 -> 0..2; waves -> 3..5
  const int64_t b = (int64_t)1 << a.log2b;
  double* dst = a.partial + ((size_t)g * a.d + t) * b + ((int64_t)uhi << LB);
  const uint32_t fin_t = (lane & 7) | (w << 3) | (l4 << 6) | (l5 << 7) | (l3 << 12);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t fe = ((uint32_t)(e & 1) << 10) | ((uint32_t)((e >> 1) & 1) << 11) |
                        ((uint32_t)((e >> 2) & 3) << 8);
    dst[fin_t | fe] = (double)acc[e];
  }
}

// Two waves per SIMD for both types: at four (128 registers) the float32
// variant spills, which costs more than the extra occupancy gains.
template <typename T>
constexpr int waves16() { return 2; }

template <typename T, bool SINGLE, bool DESC, bool ALIAS>
__global__ __launch_bounds__(512, waves16<T>()) void compress16_kernel(CompressArgs a) {
  // units of a repetition without collision chains take the instance
  // without fix-ups
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int LB = 13;
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
  if constexpr (DESC) {
    const int nA = a.planA.nchains[t], nB = a.planB.nchains[t];
    if (nA == 0 && nB == 0) {
      compress16_unit<T, SINGLE, DESC, ALIAS, 0>(a, g, t, uhi, k0, k1, smem);
      return;
    }
    // extras equal chains: every chain has two rows
    const int xA = a.planA.cstart[(size_t)t * (a.n_rows + 2) + nA];
    const int xB = a.planB.cstart[(size_t)t * (a.n_cols + 2) + nB];
    if (xA == nA && xB == nB && nA <= kPairSlots16 * 512 && nB <= kPairSlots16 * 512 &&
        a.ovf16 >= kPairOvf16) {
      compress16_unit<T, SINGLE, DESC, ALIAS, 2>(a, g, t, uhi, k0, k1, smem);
      return;
    }
  }
  compress16_unit<T, SINGLE, DESC, ALIAS, 1>(a, g, t, uhi, k0, k1, smem);
}

// The persistent batched form with the 16-element layout (b_lo = 2^13).
template <typename T, bool DESC>
__global__ __launch_bounds__(512, waves16<T>()) void compress16_batched_kernel(
    char* __restrict__ ws, const BatchPair* __restrict__ pairs,
    const BatchItem* __restrict__ items, int n_items, int* __restrict__ queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  constexpr int LB = 13;
  for (;;) {
    __syncthreads();   // the previous unit is done with LDS and s_item
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;   // uniform: every wave leaves
    const BatchItem bi = items[it];
    const BatchPair bp = pairs[bi.pair];
    CompressArgs a;
    a.At = ws + bp.at;
    a.B = bp.bc >= 0 ? static_cast<const void*>(ws + bp.bc) : bp.B;
    a.ldb = bp.ldb;
    a.n_rows = bp.n_rows;
    a.n_cols = bp.n_cols;
    a.n_inner = bp.n_inner;
    a.tab1 = bp.rtab1 >= 0 ? reinterpret_cast<const uint32_t*>(ws + bp.rtab1) : bp.tab1;
    a.tab2 = bp.rtab2 >= 0 ? reinterpret_cast<const uint32_t*>(ws + bp.rtab2) : bp.tab2;
    a.planA = carve_plan(ws + bp.planA, bp.d, bp.n_rows, LB);
    a.planB = carve_plan(ws + bp.planB, bp.d, bp.n_cols, LB);
    a.d = bp.d;
    a.log2b = bp.log2b;
    a.groups = bp.groups;
    a.partial = reinterpret_cast<double*>(ws + bp.partial);
    a.ex_cap = bp.ex_cap;
    a.dma = bp.dma;
    a.variant = 0;
    a.ovf16 = DESC ? bp.ovf16 : 0;
    const int b_hi_bits = a.log2b - LB;
    const int t = (int)(bi.unit >> b_hi_bits);
    const uint32_t uhi = bi.unit & ((1u << b_hi_bits) - 1u);
    const int64_t k_per = (a.n_inner + a.groups - 1) / a.groups;
    const int64_t k0 = (int64_t)bi.group * k_per;
    const int64_t k1 = (k0 + k_per) < a.n_inner ? (k0 + k_per) : a.n_inner;
    if constexpr (DESC) {
      // as in the single-problem kernel: repetitions without chains, or
      // with two-row chains only, take the shorter instances
      const int nA = a.planA.nchains[t], nB = a.planB.nchains[t];
      if (nA == 0 && nB == 0) {
        compress16_unit<T, false, DESC, false, 0>(a, (int)bi.group, t, uhi, k0, k1, smem);
        continue;
      }
      const int xA = a.planA.cstart[(size_t)t * (a.n_rows + 2) + nA];
      const int xB = a.planB.cstart[(size_t)t * (a.n_cols + 2) + nB];
      if (xA == nA && xB == nB && nA <= kPairSlots16 * 512 && nB <= kPairSlots16 * 512 &&
          a.ovf16 >= kPairOvf16) {
        compress16_unit<T, false, DESC, false, 2>(a, (int)bi.group, t, uhi, k0, k1, smem);
        continue;
      }
    }
    compress16_unit<T, false, DESC>(a, (int)bi.group, t, uhi, k0, k1, smem);
  }
}

}  // namespace

// Host-side helpers used by the estimate driver.
size_t plan_bytes(int d, int64_t n, int lb) {
  const size_t blo = (size_t)1 << lb;
  size_t s = 0;
  s += align_up(sizeof(int32_t) * d * blo, 256);               // first
  s += align_up(sizeof(uint2) * d * (size_t)n, 256);           // pairs
  s += align_up(sizeof(int32_t) * d * (size_t)(n + 2), 256);   // cstart
  s += align_up(sizeof(int32_t) * d, 256);                     // nchains
  return s;
}

size_t plan_lds_bytes(int64_t n, int lb) {
  return sizeof(int32_t) * (2 * ((size_t)1 << lb) + ((size_t)n + 1) / 2 + 2 + kPlanThreads / 64);
}

cmm_status launch_plan(const uint32_t* tab, int d, int64_t n, int lb, const PlanView& pv,
                       hipStream_t s) {
  ProfScope prof_("plan", s);
  const size_t lds = plan_lds_bytes(n, lb);
  if (lds > 160 * 1024) {
    set_error("plan: too many indices for the LDS rank arrays");
    return CMM_EUNSUPPORTED;
  }
  hipError_t e = hipFuncSetAttribute((const void*)plan_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_check(e, "plan: set LDS size");
  hipLaunchKernelGGL(plan_kernel, dim3(d), dim3(kPlanThreads), lds, s, tab, n, lb, pv);
  return hip_check(hipGetLastError(), "plan kernel launch");
}

template <typename T, int LB>
static cmm_status launch_compress_t(const CompressArgs& a0, hipStream_t s) {
  ProfScope prof_("compress", s);
  CompressArgs a = a0;
  const int64_t blocks = ((int64_t)a.d << (a.log2b - LB)) * a.groups;
  const size_t base = sizeof(T) * (((size_t)1 << LB) + ((size_t)1 << (LB - 7)) +
                                   (size_t)row_pitch<T>(a.n_rows) + (size_t)row_pitch<T>(a.n_cols));
  const size_t kMax = 160 * 1024;
  if (base > kMax) { set_error("compress: rows do not fit in LDS"); return CMM_EUNSUPPORTED; }
  // LDS left for the non-first-row lists (8 bytes per entry)
  int64_t cap = (int64_t)((kMax - base) / sizeof(uint2));
  const int64_t want = a.n_rows + a.n_cols;
  if (cap > want) cap = want;
  a.ex_cap = cap;
  const size_t lds = base + sizeof(uint2) * (size_t)cap;
  // 16-byte asynchronous row copies need 16-byte aligned rows
  constexpr int V = 16 / sizeof(T);
  a.dma = (a.n_rows % V == 0) && (a.n_cols % V == 0) && (a.ldb % V == 0) &&
          ((uintptr_t)a.At % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
  auto kern = compress_kernel<T, LB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress: set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(Cfg<T, LB>::NT), lds, s, a);
  return hip_check(hipGetLastError(), "compress kernel launch");
}

template <typename T>
static cmm_status launch_compress16(const CompressArgs& a0, hipStream_t s) {
  ProfScope prof_("compress", s);
  CompressArgs a = a0;
  constexpr int LB = 13;
  const int64_t blocks = ((int64_t)a.d << (a.log2b - LB)) * a.groups;
  const size_t xlen = ((size_t)1 << LB) + ((size_t)1 << (LB - 6)) + 16;
  const size_t kMax = 160 * 1024;
  // descriptor fix-ups when both rows (with their spare elements) and the
  // descriptors fit; else chain lists, with one time-shared row buffer when
  // two rows do not fit
  const size_t desc_lds = sizeof(uint32_t) * 3 * 2 * kSlots16 * 512;
  const size_t base_desc = sizeof(T) * (xlen + (size_t)pitch16<T, true>(a.n_rows) +
                                        (size_t)pitch16<T, true>(a.n_cols));
  const bool idx15 = a.n_rows + 64 < 32768 && a.n_cols + 64 < 32768;
  const bool desc = base_desc + desc_lds <= kMax && idx15;
  // rows too long for a transpose buffer beside them: transposes through
  // the row areas
  const size_t base_alias = sizeof(T) * (size_t)(alias_area16<T>(a.n_rows) + alias_area16<T>(a.n_cols));
  const bool alias = !desc && idx15 && base_alias + desc_lds <= kMax;
  size_t base = desc ? base_desc
              : alias ? base_alias
                      : sizeof(T) * (xlen + (size_t)row_pitch<T>(a.n_rows) + (size_t)row_pitch<T>(a.n_cols));
  bool single = false;
  if (base > kMax) {
    const size_t p1 = (size_t)(row_pitch<T>(a.n_rows) > row_pitch<T>(a.n_cols)
                                   ? row_pitch<T>(a.n_rows) : row_pitch<T>(a.n_cols));
    base = sizeof(T) * (xlen + p1);
    single = true;
  }
  if (base > kMax) { set_error("compress: rows do not fit in LDS"); return CMM_EUNSUPPORTED; }
  // the descriptor slots, and a partial third slot in whatever LDS is left
  // (three words per position and operand)
  a.ovf16 = 0;
  if ((desc || alias) && !single) {
    size_t left = kMax - base - desc_lds;
    size_t ovf = left / (sizeof(uint32_t) * 3 * 2);
    if (ovf > 512) ovf = 512;
    a.ovf16 = (int)ovf;
  }
  int64_t cap = (int64_t)((kMax - base) / sizeof(uint2));
  const int64_t want = (desc || alias) ? (int64_t)((desc_lds + sizeof(uint32_t) * 3 * 2 * (size_t)a.ovf16) /
                                        sizeof(uint2))
                            : a.n_rows + a.n_cols;
  if (cap > want) cap = want;
  a.ex_cap = cap;
  const size_t lds = base + sizeof(uint2) * (size_t)cap;
  constexpr int V = 16 / sizeof(T);
  a.dma = (a.n_rows % V == 0) && (a.n_cols % V == 0) && (a.ldb % V == 0) &&
          ((uintptr_t)a.At % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
  auto kern = single ? compress16_kernel<T, true, false, false>
             : alias  ? compress16_kernel<T, false, true, true>
             : desc   ? compress16_kernel<T, false, true, false>
                      : compress16_kernel<T, false, false, false>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress: set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(512), lds, s, a);
  return hip_check(hipGetLastError(), "compress kernel launch");
}

size_t compress16_desc_lds(cmm_dtype dt, int64_t n_rows, int64_t n_cols) {
  const size_t xlen = ((size_t)1 << 13) + ((size_t)1 << 7) + 16;
  const size_t desc = sizeof(uint32_t) * 3 * 2 * kSlots16 * 512;
  if (dt == CMM_F64)
    return sizeof(double) * (xlen + (size_t)pitch16<double, true>(n_rows) +
                             (size_t)pitch16<double, true>(n_cols)) + desc;
  return sizeof(float) * (xlen + (size_t)pitch16<float, true>(n_rows) +
                          (size_t)pitch16<float, true>(n_cols)) + desc;
}

size_t compress16_lds_base(cmm_dtype dt, int64_t n_rows, int64_t n_cols) {
  const size_t xlen = ((size_t)1 << 13) + ((size_t)1 << 7) + 16;
  if (dt == CMM_F64)
    return sizeof(double) * (xlen + (size_t)row_pitch<double>(n_rows) + (size_t)row_pitch<double>(n_cols));
  return sizeof(float) * (xlen + (size_t)row_pitch<float>(n_rows) + (size_t)row_pitch<float>(n_cols));
}

size_t compress_lds_base(cmm_dtype dt, int lb, int64_t n_rows, int64_t n_cols) {
  if (dt == CMM_F64)
    return sizeof(double) * (((size_t)1 << lb) + ((size_t)1 << (lb - 7)) +
                             (size_t)row_pitch<double>(n_rows) + (size_t)row_pitch<double>(n_cols));
  return sizeof(float) * (((size_t)1 << lb) + ((size_t)1 << (lb - 7)) +
                          (size_t)row_pitch<float>(n_rows) + (size_t)row_pitch<float>(n_cols));
}

template <typename T, int LB>
static cmm_status launch_batched_t(char* ws, const BatchPair* pairs, const BatchItem* items,
                                   int n_items, int* queue, int wgs, size_t lds, hipStream_t s) {
  ProfScope prof_("compress", s);
  auto kern = compress_batched_kernel<T, LB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress (batched): set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)wgs), dim3(Cfg<T, LB>::NT), lds, s, ws, pairs, items,
                     n_items, queue);
  return hip_check(hipGetLastError(), "compress (batched) launch");
}

template <typename T>
static cmm_status launch_batched16_t(char* ws, const BatchPair* pairs, const BatchItem* items,
                                     int n_items, int* queue, bool desc, int wgs, size_t lds,
                                     hipStream_t s) {
  ProfScope prof_("compress", s);
  auto kern = desc ? compress16_batched_kernel<T, true> : compress16_batched_kernel<T, false>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress (batched): set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)wgs), dim3(512), lds, s, ws, pairs, items, n_items, queue);
  return hip_check(hipGetLastError(), "compress (batched) launch");
}

cmm_status launch_compress_batched(char* ws, const BatchPair* pairs, const BatchItem* items,
                                   int n_items, int* queue, cmm_dtype dt, int lb, int radix,
                                   bool desc, int wgs, size_t lds, hipStream_t s) {
  if (radix == 16) {
    if (lb != 13) {
      set_error("compress (batched): the 16-element layout needs b_lo = 2^13");
      return CMM_EUNSUPPORTED;
    }
    if (dt == CMM_F64)
      return launch_batched16_t<double>(ws, pairs, items, n_items, queue, desc, wgs, lds, s);
    return launch_batched16_t<float>(ws, pairs, items, n_items, queue, desc, wgs, lds, s);
  }
  if (dt == CMM_F64) {
    switch (lb) {
      case 11: return launch_batched_t<double, 11>(ws, pairs, items, n_items, queue, wgs, lds, s);
      case 12: return launch_batched_t<double, 12>(ws, pairs, items, n_items, queue, wgs, lds, s);
      case 13: return launch_batched_t<double, 13>(ws, pairs, items, n_items, queue, wgs, lds, s);
    }
  } else {
    switch (lb) {
      case 11: return launch_batched_t<float, 11>(ws, pairs, items, n_items, queue, wgs, lds, s);
      case 12: return launch_batched_t<float, 12>(ws, pairs, items, n_items, queue, wgs, lds, s);
      case 13: return launch_batched_t<float, 13>(ws, pairs, items, n_items, queue, wgs, lds, s);
    }
  }
  set_error("compress (batched): unsupported b_lo");
  return CMM_EUNSUPPORTED;
}

cmm_status launch_compress(const CompressArgs& a, cmm_dtype dt, int lb, hipStream_t s) {
  if (dt == CMM_F64) {
    switch (lb) {
      case 11: return launch_compress_t<double, 11>(a, s);
      case 12: return launch_compress_t<double, 12>(a, s);
      case 13:
        if (a.variant == 1) return launch_compress_t<double, 13>(a, s);
        return launch_compress16<double>(a, s);
    }
  } else {
    switch (lb) {
      case 11: return launch_compress_t<float, 11>(a, s);
      case 12: return launch_compress_t<float, 12>(a, s);
      case 13:
        if (a.variant == 1) return launch_compress_t<float, 13>(a, s);
        return launch_compress16<float>(a, s);
      case 14: return launch_compress_t<float, 14>(a, s);
    }
  }
  set_error("compress: unsupported b_lo");
  return CMM_EUNSUPPORTED;
}

// ------------------------------------------------------------ transpose
namespace {
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void transpose_kernel(const TI* __restrict__ in, int64_t rows,
                                                        int64_t cols, int64_t ld,
                                                        TO* __restrict__ out) {
  // out[c][r] = in[r][c]; 64 x 64 tiles through LDS
  __shared__ TO tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y, c = c0 + tx;
    if (r < rows && c < cols) tile[y][tx] = (TO)in[r * ld + c];
  }
  __syncthreads();
  for (int y = ty; y < 64; y += 4) {
    const int64_t c = c0 + y, r = r0 + tx;
    if (r < rows && c < cols) out[c * rows + r] = tile[tx][y];
  }
}
}  // namespace

namespace {
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void convert_kernel(const TI* __restrict__ in, int64_t rows,
                                                      int64_t cols, int64_t ld,
                                                      TO* __restrict__ out) {
  const int64_t n = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const int64_t r = q / cols, c = q - r * cols;
    out[q] = (TO)in[r * ld + c];
  }
}
}  // namespace

cmm_status launch_convert(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols,
                          int64_t ld, void* out, cmm_dtype out_dt, hipStream_t s) {
  const int64_t n = rows * cols;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  if (in_dt == CMM_F64 && out_dt == CMM_F32)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3((unsigned)g), dim3(256), 0, s,
                       (const double*)in, rows, cols, ld, (float*)out);
  else if (in_dt == CMM_F64 && out_dt == CMM_F64)
    hipLaunchKernelGGL((convert_kernel<double, double>), dim3((unsigned)g), dim3(256), 0, s,
                       (const double*)in, rows, cols, ld, (double*)out);
  else if (in_dt == CMM_F32 && out_dt == CMM_F32)
    hipLaunchKernelGGL((convert_kernel<float, float>), dim3((unsigned)g), dim3(256), 0, s,
                       (const float*)in, rows, cols, ld, (float*)out);
  else { set_error("convert: dtype pair"); return CMM_EUNSUPPORTED; }
  return hip_check(hipGetLastError(), "convert kernel launch");
}

cmm_status launch_transpose(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols,
                            int64_t ld, void* out, cmm_dtype out_dt, hipStream_t s) {
  ProfScope prof_("transpose", s);
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
  if (grid.y > 65535) { set_error("transpose: too many rows"); return CMM_EUNSUPPORTED; }
  if (in_dt == CMM_F64 && out_dt == CMM_F64)
    hipLaunchKernelGGL((transpose_kernel<double, double>), grid, dim3(256), 0, s,
                       (const double*)in, rows, cols, ld, (double*)out);
  else if (in_dt == CMM_F64 && out_dt == CMM_F32)
    hipLaunchKernelGGL((transpose_kernel<double, float>), grid, dim3(256), 0, s,
                       (const double*)in, rows, cols, ld, (float*)out);
  else if (in_dt == CMM_F32 && out_dt == CMM_F32)
    hipLaunchKernelGGL((transpose_kernel<float, float>), grid, dim3(256), 0, s,
                       (const float*)in, rows, cols, ld, (float*)out);
  else { set_error("transpose: dtype pair"); return CMM_EUNSUPPORTED; }
  return hip_check(hipGetLastError(), "transpose kernel launch");
}

}  // namespace cmm
