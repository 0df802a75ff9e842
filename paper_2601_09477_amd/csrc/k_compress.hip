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

constexpr int kPlanWave = 64;

__global__ __launch_bounds__(kPlanWave) void plan_kernel(const uint32_t* __restrict__ tab,
                                                         int64_t n, int lb, PlanView pv) {
  const int t = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t blo = (int64_t)1 << lb;
  const uint32_t lomask = (uint32_t)blo - 1u;
  const uint32_t* tb = tab + (size_t)t * n;
  int32_t* first = pv.first + (size_t)t * blo;
  int32_t* rank = pv.rank + (size_t)t * n;
  int32_t* roff = pv.roff + (size_t)t * (n + 2);
  // cnt[r]: indices seen so far in lo-bucket r (LDS holds max(b_lo, n + 2)
  // counters so that it can be reused as the per-rank cursor below).
  extern __shared__ int32_t cnt[];
  for (int64_t r = lane; r < blo; r += kPlanWave) { cnt[r] = 0; first[r] = -1; }
  for (int64_t r = lane; r < n + 2; r += kPlanWave) roff[r] = 0;
  __syncthreads();
  int maxr = 0;
  for (int64_t g0 = 0; g0 < n; g0 += kPlanWave) {
    const int64_t i = g0 + lane;
    const uint32_t key = i < n ? (tb[i] & lomask) : 0xFFFFFFFFu;
    int below = 0, above = 0;
    for (int j = 0; j < kPlanWave; ++j) {
      const uint32_t kj = (uint32_t)__builtin_amdgcn_readlane((int)key, j);
      below += (j < lane && kj == key) ? 1 : 0;
      above += (j > lane && kj == key) ? 1 : 0;
    }
    int rk = 0;
    if (i < n) {
      rk = cnt[key] + below;
      rank[i] = rk;
      if (rk == 0) first[key] = (int32_t)i;
      maxr = rk > maxr ? rk : maxr;
    }
    __syncthreads();   // all reads of cnt for this group precede the updates
    if (i < n && above == 0) cnt[key] = rk + 1;
    __syncthreads();
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(maxr, off);
    maxr = o > maxr ? o : maxr;
  }
  if (lane == 0) pv.maxrank[t] = maxr;
  // histogram of ranks >= 1 into roff[rank + 1], then prefix sum
  for (int64_t i = lane; i < n; i += kPlanWave) {
    const int rk = rank[i];
    if (rk >= 1) atomicAdd(&roff[rk + 1], 1);
  }
  __syncthreads();
  if (lane == 0) {
    int32_t acc = 0;
    for (int r = 0; r <= maxr + 1 && r < n + 2; ++r) { acc += roff[r]; roff[r] = acc; }
  }
  __syncthreads();
  // roff[r] now = number of entries with rank < r (r >= 1).  Place the
  // entries of each rank through a per-rank cursor; the order inside a rank
  // is irrelevant because the targets of one rank are distinct buckets.
  for (int r = lane; r <= maxr + 1; r += kPlanWave) cnt[r] = 0;
  __syncthreads();
  for (int64_t i = lane; i < n; i += kPlanWave) {
    const int rk = rank[i];
    if (rk >= 1) {
      const uint32_t e = tb[i];
      const int32_t f = first[e & lomask];
      const uint32_t ef = tb[f];
      const int pos = roff[rk] + atomicAdd(&cnt[rk], 1);
      pv.extras[(size_t)t * n + pos] = (uint32_t)i | ((uint32_t)f << 16);
      const uint32_t hx = ((e & kBucketMask) >> lb) ^ ((ef & kBucketMask) >> lb);
      pv.meta[(size_t)t * n + pos] = hx | ((e ^ ef) & kSignBit);
    }
  }
}

// ------------------------------------------------------------- helpers
__device__ __forceinline__ void bfly(double& a, double& b) {
  const double x = a, y = b;
  a = x + y;
  b = x - y;
}
__device__ __forceinline__ void bfly(float& a, float& b) {
  const float x = a, y = b;
  a = x + y;
  b = x - y;
}

// Exchange lane bit 4 (16-lane rows) of x with the register bit that
// distinguishes x (bit clear) from y (bit set).
__device__ __forceinline__ void xswap16(double& x, double& y) {
  const uint64_t ux = __double_as_longlong(x), uy = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ux, (uint32_t)uy, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ux >> 32), (uint32_t)(uy >> 32),
                                                   false, false);
  x = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void xswap32(double& x, double& y) {
  const uint64_t ux = __double_as_longlong(x), uy = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ux, (uint32_t)uy, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ux >> 32), (uint32_t)(uy >> 32),
                                                   false, false);
  x = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void xswap16(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void xswap32(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}

// Butterfly stage on register bit j of a 32-element array.
template <int J, typename T>
__device__ __forceinline__ void stage_reg(T (&v)[32]) {
#pragma unroll
  for (int e = 0; e < 32; ++e)
    if ((e & (1 << J)) == 0) bfly(v[e], v[e | (1 << J)]);
}
// Exchange lane bit 4 (S = 16) or 5 (S = 32) with register bit J.
template <int J, int S, typename T>
__device__ __forceinline__ void swap_reg(T (&v)[32]) {
#pragma unroll
  for (int e = 0; e < 32; ++e)
    if ((e & (1 << J)) == 0) {
      if (S == 16) xswap16(v[e], v[e | (1 << J)]);
      else xswap32(v[e], v[e | (1 << J)]);
    }
}

// Pass 1 on layout L1: stages on u_lo bits 0..6.
template <typename T>
__device__ __forceinline__ void pass1(T (&v)[32]) {
  stage_reg<0>(v); stage_reg<1>(v); stage_reg<2>(v); stage_reg<3>(v); stage_reg<4>(v);
  swap_reg<0, 16>(v); stage_reg<0>(v);   // lane bit 4 (u_lo bit 5) <-> reg bit 0
  swap_reg<1, 32>(v); stage_reg<1>(v);   // lane bit 5 (u_lo bit 6) <-> reg bit 1
}
// Pass 2 on layout L2: stages on u_lo bits 7..LB-1.
template <int LB, typename T>
__device__ __forceinline__ void pass2(T (&v)[32]) {
  if (LB >= 8) stage_reg<0>(v);
  if (LB >= 9) stage_reg<1>(v);
  if (LB >= 10) stage_reg<2>(v);
  if (LB >= 11) stage_reg<3>(v);
  if (LB >= 12) stage_reg<4>(v);
  if (LB >= 13) { swap_reg<0, 16>(v); stage_reg<0>(v); }   // lane bit 4 <-> u_lo bit 12
  if (LB >= 14) { swap_reg<1, 32>(v); stage_reg<1>(v); }   // lane bit 5 <-> u_lo bit 13
}

// u_lo index of (thread, register e) in each layout.  l = lane, w = wave.
//  L1' (after pass 1): reg bit0 -> 5, bit1 -> 6, bits 2..4 -> 2..4;
//                      lane bit4 -> 0, bit5 -> 1, bits 0..3 -> 7..10; wave -> 11..
__device__ __forceinline__ uint32_t l1p_lane(int l, int w) {
  return ((uint32_t)((l >> 4) & 1) << 0) | ((uint32_t)((l >> 5) & 1) << 1) |
         ((uint32_t)(l & 15) << 7) | ((uint32_t)w << 11);
}
__host__ __device__ constexpr uint32_t l1p_reg(int e) {
  return ((uint32_t)(e & 1) << 5) | ((uint32_t)((e >> 1) & 1) << 6) | ((uint32_t)(e & 28));
}
// L2: reg bits 0..4 -> 7..11 (only bits < LB are real; for LB < 12 the
// spare register bits take the free low bits 4, 5, 6);
//     lane bits 0..3 -> 0..3; lane bit 4 -> 12 (LB >= 13) else a free low bit;
//     lane bit 5 -> 13 (LB >= 14) else a free low bit; waves -> remaining.
// For the LB values used (11..14) the free low bits are assigned in order.
template <int LB>
struct L2Map {
  // target u_lo bit of reg bits 0..4, lane bits 4,5, wave bits 0..3
  static constexpr int reg(int k) {
    return (7 + k < LB) ? 7 + k : free_bit(k - (LB - 7));
  }
  static constexpr int lane4() { return LB >= 13 ? 12 : free_bit(spare_regs()); }
  static constexpr int lane5() { return LB >= 14 ? 13 : free_bit(spare_regs() + (LB >= 13 ? 0 : 1)); }
  static constexpr int wave(int k) {
    return free_bit(spare_regs() + (LB >= 13 ? 0 : 1) + (LB >= 14 ? 0 : 1) + k);
  }
  static constexpr int spare_regs() { return (LB - 7) >= 5 ? 0 : 5 - (LB - 7); }
  static constexpr int free_bit(int q) { return 4 + q; }   // 4, 5, 6
};
// After pass 2's swaps: reg bit 0 <-> lane bit 4 exchanged (LB >= 13),
// reg bit 1 <-> lane bit 5 exchanged (LB >= 14).
template <int LB>
__host__ __device__ constexpr uint32_t l2_reg(int e, bool after) {
  uint32_t r = 0;
  for (int k = 0; k < 5; ++k) {
    int bit = L2Map<LB>::reg(k);
    if (after && k == 0 && LB >= 13) bit = L2Map<LB>::lane4();
    if (after && k == 1 && LB >= 14) bit = L2Map<LB>::lane5();
    r |= (uint32_t)((e >> k) & 1) << bit;
  }
  return r;
}
template <int LB>
__device__ __forceinline__ uint32_t l2_lane(int l, int w, bool after) {
  uint32_t r = (uint32_t)(l & 15);
  const int b4 = (after && LB >= 13) ? L2Map<LB>::reg(0) : L2Map<LB>::lane4();
  const int b5 = (after && LB >= 14) ? L2Map<LB>::reg(1) : L2Map<LB>::lane5();
  r |= (uint32_t)((l >> 4) & 1) << b4;
  r |= (uint32_t)((l >> 5) & 1) << b5;
  for (int k = 0; k < LB - 11; ++k) r |= (uint32_t)((w >> k) & 1) << L2Map<LB>::wave(k);
  return r;
}
// XOR swizzle of the transpose buffer: low 4 bits ^= bits 7..10.
__device__ __forceinline__ uint32_t swz(uint32_t x) { return x ^ ((x >> 7) & 15u); }

}  // namespace

// ------------------------------------------------------------ main kernel
namespace {

template <typename T, int LB>
struct Cfg {
  static constexpr int E = 32;
  static constexpr int NT = (1 << LB) / E;
};

// Stage row `k` of the operand (n values) into LDS.
template <typename T, int NT>
__device__ __forceinline__ void stage_row(T* __restrict__ dst, const T* __restrict__ src,
                                          int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
}

// Apply the rank rounds of extras onto the staged row (folded signs).
template <typename T, int NT>
__device__ __forceinline__ void fixups(T* __restrict__ row, const uint32_t* __restrict__ ex,
                                       const uint32_t* __restrict__ meta,
                                       const int32_t* __restrict__ roff, int maxr,
                                       uint32_t uhi) {
  for (int r = 1; r <= maxr; ++r) {
    const int beg = roff[r], end = roff[r + 1];
    for (int q = beg + (int)threadIdx.x; q < end; q += NT) {
      const uint32_t x = ex[q], m = meta[q];
      const uint32_t idx = x & 0xFFFFu, tgt = x >> 16;
      const uint32_t neg = (m >> 31) ^ (__popc(uhi & (m & kBucketMask)) & 1u);
      const T v = row[idx];
      row[tgt] = row[tgt] + (neg ? -v : v);
    }
    __syncthreads();
  }
}

template <typename T, int LB>
__global__ __launch_bounds__((1 << LB) / 32) void compress_kernel(CompressArgs a) {
  constexpr int E = Cfg<T, LB>::E;
  constexpr int NT = Cfg<T, LB>::NT;
  constexpr int BLO = 1 << LB;
  extern __shared__ __align__(16) unsigned char smem[];
  T* xbuf = reinterpret_cast<T*>(smem);                 // BLO
  T* rowA = xbuf + BLO;                                 // n_rows
  T* rowB = rowA + a.n_rows;                            // n_cols

  const int b_hi_bits = a.log2b - LB;
  const int64_t nunits = (int64_t)a.d << b_hi_bits;
  // XCD-aware order: work-groups are dealt to the 8 XCDs round robin, so
  // give consecutive groups of the same XCD the same k-range.
  const int64_t wg = blockIdx.x;
  const int64_t total = nunits * a.groups;
  const int64_t xcd = wg & 7, slot = wg >> 3;
  const int64_t per_xcd = (total + 7) >> 3;
  int64_t lin = xcd * per_xcd + slot;                   // a permutation when total % 8 == 0
  if ((total & 7) != 0) lin = wg;
  const int g = (int)(lin / nunits);
  const int64_t unit = lin - (int64_t)g * nunits;
  const int t = (int)(unit >> b_hi_bits);
  const uint32_t uhi = (uint32_t)(unit & (((int64_t)1 << b_hi_bits) - 1));
  const int64_t k_per = (a.n_inner + a.groups - 1) / a.groups;
  const int64_t k0 = (int64_t)g * k_per;
  const int64_t k1 = (k0 + k_per) < a.n_inner ? (k0 + k_per) : a.n_inner;

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // L1: this thread's 32 consecutive buckets start at base1.
  const uint32_t base1 = ((uint32_t)((lane >> 4) & 1) << 5) | ((uint32_t)((lane >> 5) & 1) << 6) |
                         ((uint32_t)(lane & 15) << 7) | ((uint32_t)w << 11);
  // First rows of the thread's buckets (0xFFFF = empty) and folded signs.
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
      uint32_t s1 = 0, s2 = 0;
      if (r1 >= 0) {
        const uint32_t en = t1[r1];
        s1 = (en >> 31) ^ (__popc(uhi & ((en & kBucketMask) >> LB)) & 1u);
      }
      if (r2 >= 0) {
        const uint32_t en = t2[r2];
        s2 = (en >> 31) ^ (__popc(uhi & ((en & kBucketMask) >> LB)) & 1u);
      }
      nega |= s1 << e;
      negb |= s2 << e;
      const uint32_t ra = r1 >= 0 ? (uint32_t)r1 : 0xFFFFu;
      const uint32_t rb = r2 >= 0 ? (uint32_t)r2 : 0xFFFFu;
      if (e & 1) { fa[e >> 1] |= ra << 16; fb[e >> 1] |= rb << 16; }
      else { fa[e >> 1] = ra; fb[e >> 1] = rb; }
    }
  }
  const uint32_t* exA = a.planA.extras + (size_t)t * a.n_rows;
  const uint32_t* mtA = a.planA.meta + (size_t)t * a.n_rows;
  const int32_t* roA = a.planA.roff + (size_t)t * (a.n_rows + 2);
  const int maxrA = a.planA.maxrank[t];
  const uint32_t* exB = a.planB.extras + (size_t)t * a.n_cols;
  const uint32_t* mtB = a.planB.meta + (size_t)t * a.n_cols;
  const int32_t* roB = a.planB.roff + (size_t)t * (a.n_cols + 2);
  const int maxrB = a.planB.maxrank[t];

  const uint32_t w1 = l1p_lane(lane, w);
  const uint32_t r2lane = l2_lane<LB>(lane, w, false);

  T acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = T(0);

  const T* At = reinterpret_cast<const T*>(a.At);
  const T* Bm = reinterpret_cast<const T*>(a.B);

  for (int64_t k = k0; k < k1; ++k) {
    stage_row<T, NT>(rowA, At + k * a.n_rows, a.n_rows);
    stage_row<T, NT>(rowB, Bm + k * a.ldb, a.n_cols);
    __syncthreads();
    // rank rounds of both operands share the barriers
    const int maxr = maxrA > maxrB ? maxrA : maxrB;
    for (int r = 1; r <= maxr; ++r) {
      if (r <= maxrA) {
        for (int q = roA[r] + (int)threadIdx.x; q < roA[r + 1]; q += NT) {
          const uint32_t x = exA[q], m = mtA[q];
          const uint32_t neg = (m >> 31) ^ (__popc(uhi & (m & kBucketMask)) & 1u);
          const T v = rowA[x & 0xFFFFu];
          rowA[x >> 16] = rowA[x >> 16] + (neg ? -v : v);
        }
      }
      if (r <= maxrB) {
        for (int q = roB[r] + (int)threadIdx.x; q < roB[r + 1]; q += NT) {
          const uint32_t x = exB[q], m = mtB[q];
          const uint32_t neg = (m >> 31) ^ (__popc(uhi & (m & kBucketMask)) & 1u);
          const T v = rowB[x & 0xFFFFu];
          rowB[x >> 16] = rowB[x >> 16] + (neg ? -v : v);
        }
      }
      __syncthreads();
    }
    T X[E], Y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t ra = (e & 1) ? (fa[e >> 1] >> 16) : (fa[e >> 1] & 0xFFFFu);
      const uint32_t rb = (e & 1) ? (fb[e >> 1] >> 16) : (fb[e >> 1] & 0xFFFFu);
      T va = ra != 0xFFFFu ? rowA[ra] : T(0);
      T vb = rb != 0xFFFFu ? rowB[rb] : T(0);
      X[e] = ((nega >> e) & 1u) ? -va : va;
      Y[e] = ((negb >> e) & 1u) ? -vb : vb;
    }
    pass1(X);
    pass1(Y);
    // transpose X through LDS
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[swz(w1 | l1p_reg(e))] = X[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) X[e] = xbuf[swz(r2lane | l2_reg<LB>(e, false))];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xbuf[swz(w1 | l1p_reg(e))] = Y[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) Y[e] = xbuf[swz(r2lane | l2_reg<LB>(e, false))];
    pass2<LB>(X);
    pass2<LB>(Y);
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = fma(X[e], Y[e], acc[e]);
    // rowA/rowB and xbuf are rewritten next iteration only after this barrier
    __syncthreads();
  }
  // write the slice of the partial p_hat
  const int64_t b = (int64_t)1 << a.log2b;
  double* dst = a.partial + ((size_t)g * a.d + t) * b + ((int64_t)uhi << LB);
  const uint32_t r2after = l2_lane<LB>(lane, w, true);
#pragma unroll
  for (int e = 0; e < E; ++e) dst[r2after | l2_reg<LB>(e, true)] = (double)acc[e];
}

}  // namespace

// Host-side helpers used by the estimate driver.
size_t plan_bytes(int d, int64_t n, int lb) {
  const size_t blo = (size_t)1 << lb;
  size_t s = 0;
  s += align_up(sizeof(int32_t) * d * blo, 256);          // first
  s += align_up(sizeof(uint32_t) * d * (size_t)n, 256);   // extras
  s += align_up(sizeof(uint32_t) * d * (size_t)n, 256);   // meta
  s += align_up(sizeof(int32_t) * d * (size_t)(n + 2), 256);  // roff
  s += align_up(sizeof(int32_t) * d, 256);                // maxrank
  s += align_up(sizeof(int32_t) * d * (size_t)n, 256);    // rank
  return s;
}

PlanView carve_plan(char* p, int d, int64_t n, int lb) {
  const size_t blo = (size_t)1 << lb;
  PlanView v;
  v.first = reinterpret_cast<int32_t*>(p); p += align_up(sizeof(int32_t) * d * blo, 256);
  v.extras = reinterpret_cast<uint32_t*>(p); p += align_up(sizeof(uint32_t) * d * (size_t)n, 256);
  v.meta = reinterpret_cast<uint32_t*>(p); p += align_up(sizeof(uint32_t) * d * (size_t)n, 256);
  v.roff = reinterpret_cast<int32_t*>(p); p += align_up(sizeof(int32_t) * d * (size_t)(n + 2), 256);
  v.maxrank = reinterpret_cast<int32_t*>(p); p += align_up(sizeof(int32_t) * d, 256);
  v.rank = reinterpret_cast<int32_t*>(p);
  return v;
}

cmm_status launch_plan(const uint32_t* tab, int d, int64_t n, int lb, const PlanView& pv,
                       hipStream_t s) {
  ProfScope prof_("plan", s);
  const size_t lds = sizeof(int32_t) * (((size_t)1 << lb) > (size_t)(n + 2) ? ((size_t)1 << lb)
                                                                           : (size_t)(n + 2));
  if (lds > 160 * 1024) {
    set_error("plan: too many indices for the LDS counters");
    return CMM_EUNSUPPORTED;
  }
  hipError_t e = hipFuncSetAttribute((const void*)plan_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_check(e, "plan: set LDS size");
  hipLaunchKernelGGL(plan_kernel, dim3(d), dim3(kPlanWave), lds, s, tab, n, lb, pv);
  return hip_check(hipGetLastError(), "plan kernel launch");
}

template <typename T, int LB>
static cmm_status launch_compress_t(const CompressArgs& a, hipStream_t s) {
  ProfScope prof_("compress", s);
  const int64_t blocks = ((int64_t)a.d << (a.log2b - LB)) * a.groups;
  const size_t lds = sizeof(T) * (((size_t)1 << LB) + (size_t)a.n_rows + (size_t)a.n_cols);
  auto kern = compress_kernel<T, LB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress: set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(Cfg<T, LB>::NT), lds, s, a);
  return hip_check(hipGetLastError(), "compress kernel launch");
}

cmm_status launch_compress(const CompressArgs& a, cmm_dtype dt, int lb, hipStream_t s) {
  if (dt == CMM_F64) {
    switch (lb) {
      case 11: return launch_compress_t<double, 11>(a, s);
      case 12: return launch_compress_t<double, 12>(a, s);
      case 13: return launch_compress_t<double, 13>(a, s);
    }
  } else {
    switch (lb) {
      case 11: return launch_compress_t<float, 11>(a, s);
      case 12: return launch_compress_t<float, 12>(a, s);
      case 13: return launch_compress_t<float, 13>(a, s);
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
