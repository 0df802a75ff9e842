// Precision form of the fused Compress: sketches rounded to bf16 / fp16,
// the Walsh-Hadamard transform on the matrix cores (MFMA) with float32
// accumulation, the sum over k flushed into float64 every kFlush steps.
//
// Transform.  b_lo = 2^14 per work-group (512 threads, 8 wavefronts, each
// holding 8 tiles of 16 x 16).  For a tile Z with row index a and column
// index b (4 bits each),
//   pass 1:  D1 = Z  . H16   (Z as the A operand)  transforms b;
//   pass 2:  D2 = H16 . D1   (D1 as the B operand) transforms a.
// The D layout of v_mfma_f32_16x16x16 (lane l holds rows 4(l/16)+v of column
// l%16) is exactly its B layout, so pass 2 consumes pass 1's output after a
// float32 -> bf16/fp16 conversion in place: 8 index bits per tile with no
// data movement.  One LDS transpose (bf16, 8-byte reads) regroups the bits
// and a second chained pair (H16, then H4 x I4 on the two top bits) does
// the remaining six.  H16 and H4 are exact in bf16 / fp16; only the data
// operand rounds.
//
// u_lo index bits:
//   gather / pass 1 (A layout): v -> 0,1  g=l/16 -> 2,3  m=l%16 -> 4..7
//                               tile c -> 8..10  wave w -> 11..13
//   after pass 2:               n=l%16 -> 0..3  (4g+v) -> 4..7  c, w as above
//   pass 3 (A layout):          m=l%16 -> {0,1,12,13}  (4g+v) -> 8..11
//                               tile c -> 2..4  wave w -> 5..7
//   after pass 4 (final):       v -> 0,1  g -> 12,13  n=l%16 -> 8..11
//                               c -> 2..4  w -> 5..7
// The sketch (fold, gather, collision chains) is the one of the float64
// kernel, on rows staged in the low precision.
#include "cmm_internal.h"
#include "wht_regs.h"

namespace cmm {
namespace {

typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) _Float16 f16x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

template <typename IN> struct Mf;
template <> struct Mf<__bf16> {
  typedef bf16x4 vec;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
template <> struct Mf<_Float16> {
  typedef f16x4 vec;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

constexpr int kLB = 14;
constexpr int kNT = 512;
constexpr int kTiles = 8;
constexpr int kFlush = 128;   // k steps summed in float32 before the float64 flush

template <typename IN>
__device__ __forceinline__ IN neg_if(IN x, uint32_t neg) {
  return neg ? -x : x;
}

// Transpose-buffer address (in elements) of index u, a bit permutation:
//   a0,a1 <- u8,u9   (a pass-3 lane's four values: one 8-byte load)
//   a2,a3 <- u0,u1   a4,a5 <- u12,u13   (the 16 lanes of a pass-3 read
//                                        phase hit 16 distinct bank pairs)
//   a6..a11 <- u2..u7   a12 <- u10   a13 <- u11
// The bits a thread varies (tile c, value v) land on bits no thread bit
// uses, so every access is a per-thread base plus an immediate offset.
__host__ __device__ constexpr uint32_t taddr(uint32_t u) {
  return ((u >> 8) & 3u) | ((u & 3u) << 2) | (((u >> 12) & 3u) << 4) | (((u >> 2) & 63u) << 6) |
         (((u >> 10) & 1u) << 12) | (((u >> 11) & 1u) << 13);
}

template <typename IN>
__device__ __forceinline__ float to_f(IN x) { return (float)x; }

// Collision chains on a low-precision staged row: the sum is formed in
// float32 in ascending index order and rounded once.
template <typename IN, int NT>
__device__ __forceinline__ void fix_chains_lp(IN* __restrict__ row, const uint2* __restrict__ ex,
                                              const int32_t* __restrict__ cs, int nch,
                                              uint32_t uhi) {
  for (int c = threadIdx.x; c < nch; c += NT) {
    const int beg = cs[c], end = cs[c + 1];
    const uint32_t tgt = ex[beg].x >> 16;
    float acc = to_f(row[tgt]);
    for (int q0 = beg; q0 < end; q0 += 4) {
      uint2 x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = (q0 + j < end) ? ex[q0 + j] : make_uint2(0u, 0u);
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (q0 + j < end) ? to_f(row[x[j].x & 0xFFFFu]) : 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (q0 + j < end) {
          const uint32_t neg = (x[j].y >> 31) ^ (__popc(uhi & (x[j].y & kBucketMask)) & 1u);
          acc = acc + (neg ? -v[j] : v[j]);
        }
    }
    row[tgt] = (IN)acc;
  }
}

// Copy a row of n low-precision values into LDS (16-byte asynchronous
// global->LDS loads when possible, else a plain loop).
template <typename IN, int NT>
__device__ __forceinline__ void stage_row_lp(IN* __restrict__ dst, const IN* __restrict__ src,
                                             int64_t n, bool dma) {
  if (dma) {
    // the wave's first chunk is wave-uniform (readfirstlane), so the LDS
    // destination of every load is a scalar value; rounds with all 64
    // chunks in the row skip the per-lane test; chunks < 2^31 (n < 2^34)
    const int chunks = (int)(n / 8);
    const int lane = threadIdx.x & 63;
    const int wbase = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * 64;
    int c0 = wbase;
    for (; c0 + 64 <= chunks; c0 += NT)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + (size_t)(c0 + lane) * 8),
          (__attribute__((address_space(3))) void*)(dst + (size_t)c0 * 8), 16, 0, 0);
    if (c0 < chunks && c0 + lane < chunks)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + (size_t)(c0 + lane) * 8),
          (__attribute__((address_space(3))) void*)(dst + (size_t)c0 * 8), 16, 0, 0);
  } else {
    for (int64_t i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
  }
}

// Pack two float32 into the low precision (round to nearest even).
__device__ __forceinline__ uint32_t pack2(float x, float y, __bf16*) {
  typedef __attribute__((ext_vector_type(2))) float f2;
  typedef __attribute__((ext_vector_type(2))) __bf16 b2;
  const b2 r = __builtin_convertvector((f2){x, y}, b2);
  return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ uint32_t pack2(float x, float y, _Float16*) {
  typedef __attribute__((ext_vector_type(2))) float f2;
  typedef __attribute__((ext_vector_type(2))) _Float16 h2;
  const h2 r = __builtin_convertvector((f2){x, y}, h2);
  return __builtin_bit_cast(uint32_t, r);
}

// Collision fix-ups: DESC = true uses per-thread descriptors (the common
// case, when their LDS fits); DESC = false walks the plan's chain lists.
// They are separate instances because the chain-walking code alone, even
// unexecuted, costs the loop a quarter of its speed.
// Descriptor slots per thread and operand.  Two keep 24 KB of LDS for them;
// the rest of the LDS stages merged two-row chains, which at n = 8192 hold
// every chain the transform windows leave, so no descriptor is used there.
constexpr int kSlots = 2;

struct RareLists {
  const int32_t* gc[2];   // chain starts per operand
  const uint2* gp[2];     // chain entries per operand
  int nch[2];             // chains per operand
};
constexpr int kDescLds = 2 * kSlots * kNT * 12;   // three words per descriptor

template <typename IN, bool DESC>
__global__ __launch_bounds__(kNT) void compress_mfma_kernel(CompressArgs a) {
  typedef typename Mf<IN>::vec vec;
  typedef __attribute__((ext_vector_type(2))) uint32_t u2;
  constexpr int BLO = 1 << kLB;
  constexpr int NS = kTiles * 4;   // gather slots per thread and operand
  extern __shared__ __align__(16) unsigned char smem[];
  // rows first (small LDS offsets), then the two transpose buffers
  // 16-byte aligned rows: the row, a zero pad at index n, then 64 spare
  // elements (per-lane targets of absent collision slots)
  // then, when the launcher reserved them, the sums of merged two-row
  // chains (2 cap values)
  const int64_t pbaseA = (a.n_rows + 1 + 64 + 7) / 8 * 8;
  const int64_t pbaseB = (a.n_cols + 1 + 64 + 7) / 8 * 8;
  const int64_t pitchA = pbaseA + 2 * (int64_t)a.pair_capA;
  const int64_t pitchB = pbaseB + 2 * (int64_t)a.pair_capB;
  IN* rowA = reinterpret_cast<IN*>(smem);
  IN* rowB = rowA + pitchA;
  IN* tbufX = rowB + pitchB;                             // BLO
  IN* tbufY = tbufX + BLO;                               // BLO
  uint2* exl = reinterpret_cast<uint2*>(tbufY + BLO);
  const uint16_t* rowA16 = reinterpret_cast<const uint16_t*>(rowA);
  const uint16_t* rowB16 = reinterpret_cast<const uint16_t*>(rowB);
  if (threadIdx.x == 0) { rowA[a.n_rows] = (IN)0.f; rowB[a.n_cols] = (IN)0.f; }

  const int b_hi_bits = a.log2b - kLB;
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

  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t lg = lane >> 4, lm = lane & 15;
  // gather slots e = 4 c + v -> bucket v | lg << 2 | lm << 4 | c << 8 | w << 11.
  // Two 16-bit words per register: byte offset of the row element in bits
  // 0..14 (empty bucket -> the zero pad at index n), folded sign in bit 15.
  uint32_t idxA[NS / 2], idxB[NS / 2];     // first rows of the buckets
  const uint32_t* t1 = a.tab1 + (size_t)t * a.n_rows;
  const uint32_t* t2 = a.tab2 + (size_t)t * a.n_cols;
  const int nchA = a.planA.nchains[t], nchB = a.planB.nchains[t];
  // Merged two-row chains: used by this work unit when the chains left to
  // the descriptors (the longer ones and the two-row chains past the cap)
  // fit their slots.  npair: merged chains; ndesc: descriptor positions.
  int npair[2] = {0, 0}, ndesc[2] = {nchA, nchB};
  if (DESC) {
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const int cap = op ? a.pair_capB : a.pair_capA;
      if (cap > 0) {
        const int n2 = (op ? a.pair_countB : a.pair_countA)[t];
        const int m = n2 < cap ? n2 : cap;
        const int nd = (op ? nchB : nchA) - m;
        if (nd <= kSlots * kNT) {
          npair[op] = m;
          ndesc[op] = nd;
        }
      }
    }
  }
  // bucket -> 2 p + relative sign of merged chain p, in the transpose
  // buffers (idle until the k loop), one operand at a time
  int32_t* pmap = reinterpret_cast<int32_t*>(tbufX);   // [BLO]
  auto gather_offsets = [&](int op, uint32_t (&idx)[NS / 2]) {
    const int np = npair[op];
    if (np > 0) {
      for (int r = threadIdx.x; r < BLO; r += kNT) pmap[r] = -1;
      __syncthreads();
      const uint2* pl = (op ? a.pair_listB : a.pair_listA) +
                        (size_t)t * ((op ? a.n_cols : a.n_rows) / 2 + 1);
      const uint32_t* tb = op ? t2 : t1;
      for (int q = threadIdx.x; q < np; q += kNT) {
        const uint2 y = pl[q];
        const uint32_t rel = (y.y >> 31) ^ (__popc(uhi & (y.y & kBucketMask)) & 1u);
        pmap[tb[y.x >> 16] & (uint32_t)(BLO - 1)] = 2 * q + (int32_t)rel;
      }
      __syncthreads();
    }
    const int32_t* f = (op ? a.planB.first : a.planA.first) + (size_t)t * BLO;
    const uint32_t* tb = op ? t2 : t1;
    const uint32_t pad = (uint32_t)(op ? a.n_cols : a.n_rows);
    const uint32_t pbase = (uint32_t)(op ? pbaseB : pbaseA);
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const uint32_t c = (uint32_t)e >> 2, v = (uint32_t)e & 3u;
      const uint32_t r = v | (lg << 2) | (lm << 4) | (c << 8) | (w << 11);
      const int32_t r1 = f[r];
      const uint32_t en = tb[r1 >= 0 ? r1 : 0];
      const uint32_t s1 = r1 >= 0 ? (en >> 31) ^ (__popc(uhi & ((en & kBucketMask) >> kLB)) & 1u) : 0u;
      uint32_t el = r1 >= 0 ? (uint32_t)r1 : pad;
      if (np > 0) {
        const int32_t m = pmap[r];
        if (m >= 0) el = pbase + (uint32_t)m;   // the merged sum, same folded sign
      }
      const uint32_t ix = 2u * el | (s1 << 15);
      if (e & 1) idx[e >> 1] |= ix << 16;
      else idx[e >> 1] = ix;
    }
    if (np > 0) __syncthreads();   // the map is rebuilt for the next operand
  };
  gather_offsets(0, idxA);
  gather_offsets(1, idxB);
  const int32_t* gcA = a.planA.cstart + (size_t)t * (a.n_rows + 2);
  const int32_t* gcB = a.planB.cstart + (size_t)t * (a.n_cols + 2);
  const int cntA = gcA[nchA], cntB = gcB[nchB];
  const bool ex_lds = (int64_t)cntA + cntB + (nchA + nchB + 4) / 2 + 1 <= a.ex_cap;
  const uint2* gA = a.planA.pairs + (size_t)t * a.n_rows;
  const uint2* gB = a.planB.pairs + (size_t)t * a.n_cols;
  if (!DESC && ex_lds) {
    for (int q = threadIdx.x; q < cntA; q += kNT) exl[q] = gA[q];
    for (int q = threadIdx.x; q < cntB; q += kNT) exl[cntA + q] = gB[q];
    int32_t* csl = reinterpret_cast<int32_t*>(exl + cntA + cntB);
    for (int q = threadIdx.x; q <= nchA; q += kNT) csl[q] = gcA[q];
    for (int q = threadIdx.x; q <= nchB; q += kNT) csl[nchA + 1 + q] = gcB[q];
  }
  // LDS views of the lists; each fix-up call below takes either these or the
  // global lists, so the compiler knows every pointer's memory space
  const uint2* lexA = exl;
  const uint2* lexB = exl + cntA;
  const int32_t* lcsA = reinterpret_cast<const int32_t*>(exl + cntA + cntB);
  const int32_t* lcsB = lcsA + nchA + 1;
  // Collision descriptors.  A descriptor (three words in LDS, built once per
  // work unit) holds a chain's target and its next five rows as 15-bit row
  // indices with their signs relative to the target (absent rows: the zero
  // pad index n; an absent chain targets the lane's spare element after the
  // pad):
  //   w0 = target | m1 << 15 | s1 << 30 | more << 31
  //   w1 = m2 | m3 << 15 | s2 << 30 | s3 << 31
  //   w2 = m4 | m5 << 15 | s4 << 30 | s5 << 31, or, when the chain has more
  //        rows (more = 1; the rare pass adds rows 4 onwards), where its
  //        plan entries start and how many there are: beg | count << 15
  // Slot position pos = tid + j kNT (j < kSlots) takes the chains in an
  // order with the chains of three or more rows first (stable), so that the
  // fix-up can read and add the rows past the first two only in the waves
  // whose positions hold such chains (a wave-uniform test).  A chain with
  // more than six rows (about one in a million buckets) and chains beyond
  // the slots are finished from the plan's lists.
  uint32_t* dsc = reinterpret_cast<uint32_t*>(exl);   // [word][operand][slot][kNT]
  auto dslot = [&](int word, int op, int pos) -> uint32_t& {
    return dsc[((word * 2 + op) * kSlots + pos / kNT) * kNT + pos % kNT];
  };
  auto dref = [&](int word, int op, int j) -> uint32_t& {
    return dsc[((word * 2 + op) * kSlots + j) * kNT + threadIdx.x];
  };
  __shared__ int32_t s_scan[kNT / 64 + 1];
  int nlong[2] = {0, 0};
  // position of every chain (longer chains first) by a block-wide scan over
  // contiguous runs of chains; identity order when the chains exceed the slots
  auto build_desc = [&](int op, const int32_t* gc, const uint2* gp, int nch, uint32_t pad) {
    // merged two-row chains (the first npair in chain order) take no slot
    const int np = npair[op];
    const int nd = ndesc[op];
    const bool ordered = nd <= kSlots * kNT;
    const int per = (nch + kNT - 1) / kNT;
    const int c0 = (int)threadIdx.x * per;
    int mine = 0;
    if (ordered)
      for (int c = c0; c < c0 + per && c < nch; ++c) mine += (gc[c + 1] - gc[c] > 1) ? 1 : 0;
    // exclusive scan of `mine` over the block
    const uint32_t lane_ = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if ((int)lane_ >= off) incl += y;
    }
    if (lane_ == 63u) s_scan[wv] = incl;
    __syncthreads();
    int wbase_ = 0, total = 0;
    for (int q = 0; q < kNT / 64; ++q) {
      const int x = s_scan[q];
      if (q < (int)wv) wbase_ += x;
      total += x;
    }
    __syncthreads();   // s_scan is reused by the next operand
    nlong[op] = ordered ? total : 0;
    int lpos = wbase_ + incl - mine;                 // next long position
    int ppos = total + c0 - (wbase_ + incl - mine);  // next pair position
    // empty slots first: absent chains
    for (int j = 0; j < kSlots; ++j) {
      const int pos = (int)threadIdx.x + j * kNT;
      if (pos >= nd) {
        dref(0, op, j) = (pad + 1u + (threadIdx.x & 63u)) | (pad << 15);
        dref(1, op, j) = pad | (pad << 15);
        dref(2, op, j) = pad | (pad << 15);
      }
    }
    const int cb = ordered ? c0 : (int)threadIdx.x;
    const int ce = ordered ? (c0 + per < nch ? c0 + per : nch) : nch;
    for (int c = cb; c < ce; c += ordered ? 1 : kNT) {
      const int beg = gc[c], end = gc[c + 1];
      int pos = c;
      if (ordered) {
        if (end - beg > 1) {
          pos = lpos++;
        } else {
          const int q = ppos++ - total;   // index among the two-row chains
          if (q < np) continue;           // merged ahead of the kernel
          pos = total + q - np;
        }
      }
      if (pos >= kSlots * kNT) continue;
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
  };
  if (DESC) {
    build_desc(0, gcA, gA, nchA, (uint32_t)a.n_rows);
    build_desc(1, gcB, gB, nchB, (uint32_t)a.n_cols);
  }
  // Fix-ups of both operands from their descriptors: every slot adds its
  // target and first row; the rows past those only in waves whose positions
  // hold longer chains (all of them when the order is the identity).  The
  // sum is in float32, in rank order, stored once; a slot with more rows
  // stores to its lane's spare element and is finished, still rounded once,
  // in the rare pass.
  const int wave_pos = (int)(threadIdx.x & ~63u);
  // First descriptor words of the thread's slots, kept in registers for the
  // whole k loop (the descriptors do not change with k), so a fix-up starts
  // with the row reads.
  uint32_t q0[2][kSlots];
  if (DESC) {
    __syncthreads();   // every thread's descriptors are written
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        q0[op][j] = dref(0, op, j);
        asm volatile("" : "+v"(q0[op][j]));
      }
  }
  // The chain lists the rare pass of the fix-ups walks, kept in LDS rather
  // than in scalar registers for the whole k loop (read through volatile
  // loads there, so they are not hoisted back into registers).
  __shared__ RareLists s_rare;
  if (threadIdx.x == 0) {
    s_rare.gc[0] = gcA; s_rare.gc[1] = gcB;
    s_rare.gp[0] = gA; s_rare.gp[1] = gB;
    s_rare.nch[0] = nchA; s_rare.nch[1] = nchB;
  }
  auto fix_desc = [&]() {
    // A slot is live in a wave when one of the wave's positions in it holds
    // a chain (wave-uniform; every position is live when the chains exceed
    // the slots).  Every live slot's target and first row are read
    // straight-line so that all the reads are in flight together (an absent
    // position of a live slot reads its lane's spare element and the zero
    // pad, and writes the spare back unchanged).
    bool live[2][kSlots];
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int j = 0; j < kSlots; ++j)
        live[op][j] = ndesc[op] > kSlots * kNT || wave_pos + j * kNT < ndesc[op];
    IN r0[2][kSlots], r1[2][kSlots];
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const IN* row = op ? rowB : rowA;
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        if (!live[op][j]) continue;
        r0[op][j] = row[q0[op][j] & 0x7FFFu];
        r1[op][j] = row[(q0[op][j] >> 15) & 0x7FFFu];
      }
    }
    float sum[2][kSlots];
#pragma unroll
    for (int op = 0; op < 2; ++op)
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        if (!live[op][j]) continue;
        const float v1 = to_f(r1[op][j]);
        sum[op][j] = to_f(r0[op][j]) + (((q0[op][j] >> 30) & 1u) ? -v1 : v1);
      }
    // rows three to six: only the waves whose positions hold longer chains
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      const IN* row = op ? rowB : rowA;
      const int nl = DESC ? nlong[op] : 0;
      const bool all_long = ndesc[op] > kSlots * kNT;
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        if (live[op][j] && (all_long || wave_pos + j * kNT < nl)) {   // wave-uniform
          const uint32_t w0 = q0[op][j];
          const uint32_t w1 = dref(1, op, j), w2 = dref(2, op, j);
          const float v2 = to_f(row[w1 & 0x7FFFu]), v3 = to_f(row[(w1 >> 15) & 0x7FFFu]);
          // w2 of a slot with more rows is beg | count << 15 (both < n, so
          // the reads stay in the row): its values are not added here
          const bool mr = (w0 >> 31) != 0u;
          float v4 = to_f(row[w2 & 0x7FFFu]), v5 = to_f(row[(w2 >> 15) & 0x7FFFu]);
          v4 = mr ? 0.f : v4;
          v5 = mr ? 0.f : v5;
          float acc_ = sum[op][j];
          acc_ = acc_ + (((w1 >> 30) & 1u) ? -v2 : v2);
          acc_ = acc_ + (((w1 >> 31) & 1u) ? -v3 : v3);
          acc_ = acc_ + ((!mr && ((w2 >> 30) & 1u)) ? -v4 : v4);
          acc_ = acc_ + ((!mr && ((w2 >> 31) & 1u)) ? -v5 : v5);
          sum[op][j] = acc_;
        }
      }
    }
    bool rare = false;
#pragma unroll
    for (int op = 0; op < 2; ++op) {
      IN* row = op ? rowB : rowA;
      const uint32_t spare = (uint32_t)(op ? a.n_cols : a.n_rows) + 1u + (threadIdx.x & 63u);
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        if (!live[op][j]) continue;
        const bool more = (q0[op][j] >> 31) != 0u;
        rare = rare || more;
        row[more ? spare : (q0[op][j] & 0x7FFFu)] = (IN)sum[op][j];
      }
    }
    const bool extra = ndesc[0] > kSlots * kNT || ndesc[1] > kSlots * kNT;
    if (rare || extra) {
      const volatile RareLists* rl = &s_rare;
#pragma unroll
      for (int op = 0; op < 2; ++op) {
        IN* row = op ? rowB : rowA;
        const int32_t* gc = rl->gc[op];
        const uint2* gp = rl->gp[op];
        for (int j = 0; j < kSlots; ++j) {
          if (!(q0[op][j] >> 31)) continue;
          // a bucket of seven or more rows: the target and rows 1..3 are
          // summed; rows four onwards, eight plan entries per round trip
          const uint32_t tgt = q0[op][j] & 0x7FFFu;
          const uint32_t w2 = dref(2, op, j);
          const int beg = (int)(w2 & 0x7FFFu), end = beg + (int)((w2 >> 15) & 0x7FFFu);
          row[tgt] = (IN)chain_sum<IN, float, 8>(row, gp, beg + 3, end, uhi, sum[op][j]);
        }
        // chains beyond the slots (identity order; disjoint targets), four
        // per thread at a time: their starts, first entries and first two
        // rows are each fetched as independent loads.  Only an operand in
        // identity order has them: in slot order every chain is either
        // merged or in a slot, however many chains the operand has.
        const int nch = ndesc[op] > kSlots * kNT ? rl->nch[op] : 0;
        for (int c0 = kSlots * kNT + (int)threadIdx.x; c0 < nch; c0 += 4 * kNT) {
          int beg[4], end[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c = c0 + q * kNT;
            beg[q] = c < nch ? gc[c] : 0;
            end[q] = c < nch ? gc[c + 1] : 0;
          }
          uint2 y[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) y[q] = beg[q] < end[q] ? gp[beg[q]] : make_uint2(0u, 0u);
          float v0[4], v1[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            v0[q] = beg[q] < end[q] ? to_f(row[y[q].x >> 16]) : 0.f;
            v1[q] = beg[q] < end[q] ? to_f(row[y[q].x & 0xFFFFu]) : 0.f;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (beg[q] >= end[q]) continue;
            const uint32_t neg = (y[q].y >> 31) ^ (__popc(uhi & (y[q].y & kBucketMask)) & 1u);
            float acc_ = v0[q] + (neg ? -v1[q] : v1[q]);
            if (end[q] - beg[q] > 1)
              acc_ = chain_sum<IN, float, 4>(row, gp, beg[q] + 1, end[q], uhi, acc_);
            row[y[q].x >> 16] = (IN)acc_;
          }
        }
      }
    }
  };

  // H16 as the B operand (passes 1, 3) and as the A operand (pass 2): lane
  // holds H[4 lg + v][lm] = H[lm][4 lg + v].  Pass 4: M4 = H4 x I4 on the
  // two top bits, as the A operand: M4[lm][4 lg + v] = H4[lm >> 2][lg] [lm & 3 == v].
  vec h16, m4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t k = 4u * lg + (uint32_t)v;
    h16[v] = (IN)((__popc(k & lm) & 1u) ? -1.f : 1.f);
    const float h4 = (__popc((lm >> 2) & lg) & 1u) ? -1.f : 1.f;
    m4[v] = (IN)(((lm & 3u) == (uint32_t)v) ? h4 : 0.f);
  }
  // pass-2 output index base (+ (4 lg + v) << 4 + c << 8) and pass-3 read
  // index base (+ c << 2; the four v at bits 8, 9 are one 8-byte load)
  const uint32_t wbase = taddr(lm | ((4u * lg) << 4) | (w << 11));   // + taddr of (v, c)
  const uint32_t rbase = taddr((lm & 3u) | ((lm >> 2) << 12) | (lg << 10) | (w << 5));   // + taddr(c << 2)
  IN* const dummy = nullptr;

  const IN* At = reinterpret_cast<const IN*>(a.At);
  const IN* Bm = reinterpret_cast<const IN*>(a.B);
  const bool dma = a.dma != 0;
  // the merged chains' sums of k follow each row (whole 16-byte chunks,
  // inside the 2 cap values reserved per k)
  const IN* pvA = reinterpret_cast<const IN*>(a.pair_valsA);
  const IN* pvB = reinterpret_cast<const IN*>(a.pair_valsB);
  const int64_t plenA = (2 * (int64_t)npair[0] + 7) / 8 * 8;
  const int64_t plenB = (2 * (int64_t)npair[1] + 7) / 8 * 8;
  auto load_k = [&](int64_t kk) {
    stage_row_lp<IN, kNT>(rowA, At + kk * a.n_rows, a.n_rows, dma);
    stage_row_lp<IN, kNT>(rowB, Bm + kk * a.ldb, a.n_cols, dma);
    if (plenA > 0)
      stage_row_lp<IN, kNT>(rowA + pbaseA, pvA + ((size_t)t * a.n_inner + kk) * (2 * a.pair_capA),
                            plenA, dma);
    if (plenB > 0)
      stage_row_lp<IN, kNT>(rowB + pbaseB, pvB + ((size_t)t * a.n_inner + kk) * (2 * a.pair_capB),
                            plenB, dma);
  };
  // passes 1-2 of one operand from its staged row, each phase over all
  // tiles (independent MFMAs); result written (rounded) to the transpose buffer
  auto gather_tiles = [&](const unsigned char* rb, const uint32_t (&idx)[NS / 2],
                          vec (&av)[kTiles]) {
    // the two 16-bit values of a slot pair go straight into the low and
    // high halves of one register (d16 loads), then take their signs
    typedef __attribute__((ext_vector_type(2))) uint16_t h2;
    h2 raw[NS / 2];
#pragma unroll
    for (int q = 0; q < NS / 2; ++q) {
      raw[q].x = *reinterpret_cast<const uint16_t*>(rb + (idx[q] & 0x7FFFu));
      raw[q].y = *reinterpret_cast<const uint16_t*>(rb + ((idx[q] >> 16) & 0x7FFFu));
    }
#pragma unroll
    for (int c = 0; c < kTiles; ++c) {
      u2 pk;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = c * 2 + h;
        pk[h] = __builtin_bit_cast(uint32_t, raw[q]) ^ (idx[q] & 0x80008000u);   // folded signs
      }
      av[c] = __builtin_bit_cast(vec, pk);
    }
  };
  // passes 1-2 of one operand from its gathered tiles; each phase runs over
  // all tiles (independent MFMAs); the result is written, rounded, to the
  // transpose buffer
  auto front = [&](vec (&av)[kTiles], IN* tb) {
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 d[kTiles];
#pragma unroll
    for (int c = 0; c < kTiles; ++c) d[c] = Mf<IN>::mma(av[c], h16, z);
#pragma unroll
    for (int c = 0; c < kTiles; ++c) {
      u2 pk;
      pk[0] = pack2(d[c][0], d[c][1], dummy);
      pk[1] = pack2(d[c][2], d[c][3], dummy);
      av[c] = __builtin_bit_cast(vec, pk);
    }
#pragma unroll
    for (int c = 0; c < kTiles; ++c) d[c] = Mf<IN>::mma(h16, av[c], z);
    uint16_t* tb16 = reinterpret_cast<uint16_t*>(tb) + wbase;
#pragma unroll
    for (int c = 0; c < kTiles; ++c) {
      const uint32_t p01 = pack2(d[c][0], d[c][1], dummy);
      const uint32_t p23 = pack2(d[c][2], d[c][3], dummy);
      tb16[taddr((0u << 4) | ((uint32_t)c << 8))] = (uint16_t)p01;
      tb16[taddr((1u << 4) | ((uint32_t)c << 8))] = (uint16_t)(p01 >> 16);
      tb16[taddr((2u << 4) | ((uint32_t)c << 8))] = (uint16_t)p23;
      tb16[taddr((3u << 4) | ((uint32_t)c << 8))] = (uint16_t)(p23 >> 16);
    }
  };
  // the transposed tiles of one operand (8-byte reads)
  auto load_back = [&](const IN* tb, vec (&av)[kTiles]) {
#pragma unroll
    for (int c = 0; c < kTiles; ++c)
      av[c] = *reinterpret_cast<const vec*>(tb + rbase + taddr((uint32_t)c << 2));
  };
  // passes 3-4 into the final float32 layout
  auto back = [&](vec (&av)[kTiles], f32x4 (&out)[kTiles]) {
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 d[kTiles];
#pragma unroll
    for (int c = 0; c < kTiles; ++c) d[c] = Mf<IN>::mma(av[c], h16, z);
#pragma unroll
    for (int c = 0; c < kTiles; ++c) {
      u2 pk;
      pk[0] = pack2(d[c][0], d[c][1], dummy);
      pk[1] = pack2(d[c][2], d[c][3], dummy);
      av[c] = __builtin_bit_cast(vec, pk);
    }
#pragma unroll
    for (int c = 0; c < kTiles; ++c) out[c] = Mf<IN>::mma(m4, av[c], z);
  };

  // partial p_hat slice of this work-group: final index of (thread, c, v)
  const int64_t b = (int64_t)1 << a.log2b;
  double* dst = a.partial + ((size_t)g * a.d + t) * b + ((int64_t)uhi << kLB);
  const uint32_t fin = (lg << 12) | (lm << 8) | (w << 5);   // + v + c << 2
  f32x4 acc[kTiles];
#pragma unroll
  for (int c = 0; c < kTiles; ++c) acc[c] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // the float64 sums of the flushes stay in registers; the slice of the
  // partials is written once, after the last flush
  double acc64[kTiles][4];
#pragma unroll
  for (int c = 0; c < kTiles; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc64[c][v] = 0.0;
  int pending = 0;
  auto flush = [&]() {
#pragma unroll
    for (int c = 0; c < kTiles; ++c) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[c][v] = acc64[c][v] + (double)acc[c][v];
      acc[c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
    pending = 0;
  };

  if (k0 < k1) load_k(k0);
  for (int64_t k = k0; k < k1; ++k) {
    if (dma) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();   // rows of k staged; the transpose buffers are free
    if ((DESC ? ndesc[0] + ndesc[1] : nchA + nchB) > 0) {
      if constexpr (DESC) {
        fix_desc();
      } else {
        { if (ex_lds) fix_chains_lp<IN, kNT>(rowA, lexA, lcsA, nchA, uhi); else fix_chains_lp<IN, kNT>(rowA, gA, gcA, nchA, uhi); }
        { if (ex_lds) fix_chains_lp<IN, kNT>(rowB, lexB, lcsB, nchB, uhi); else fix_chains_lp<IN, kNT>(rowB, gB, gcB, nchB, uhi); }
      }
      __syncthreads();
    }
    // both operands' gathers are issued before either's matrix passes, so
    // the loads of one overlap the MFMAs of the other
    {
      vec avX[kTiles], avY[kTiles];
      gather_tiles(reinterpret_cast<const unsigned char*>(rowA16), idxA, avX);
      gather_tiles(reinterpret_cast<const unsigned char*>(rowB16), idxB, avY);
      front(avX, tbufX);
      front(avY, tbufY);
    }
    __syncthreads();   // gathers done (rows free), transpose buffers written
    if (k + 1 < k1) load_k(k + 1);
    f32x4 X[kTiles], Y[kTiles];
    {
      vec bvX[kTiles], bvY[kTiles];
      load_back(tbufX, bvX);
      load_back(tbufY, bvY);
      back(bvX, X);
      back(bvY, Y);
    }
#pragma unroll
    for (int c = 0; c < kTiles; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[c][v] = fmaf(X[c][v], Y[c][v], acc[c][v]);
    // keep the per-slot offsets in their packed form (no hoisted copies)
#pragma unroll
    for (int q = 0; q < NS / 2; ++q) {
      asm volatile("" : "+v"(idxA[q]));
      asm volatile("" : "+v"(idxB[q]));
    }
    if (++pending == kFlush) flush();
  }
  if (pending > 0) flush();
#pragma unroll
  for (int c = 0; c < kTiles; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[fin | (uint32_t)v | ((uint32_t)c << 2)] = acc64[c][v];
}

}  // namespace

namespace {

// Two-row chains of one repetition in chain order (one work-group per
// repetition): a block scan over contiguous runs of chains numbers them.
__global__ __launch_bounds__(kNT) void pair_list_kernel(PlanView pv, int64_t n, uint2* list,
                                                        int32_t* count) {
  __shared__ int32_t s_scan[kNT / 64];
  const int t = blockIdx.x;
  const int32_t* gc = pv.cstart + (size_t)t * (n + 2);
  const uint2* gp = pv.pairs + (size_t)t * n;
  uint2* out = list + (size_t)t * (n / 2 + 1);
  const int nch = pv.nchains[t];
  const int per = (nch + kNT - 1) / kNT;
  const int c0 = (int)threadIdx.x * per;
  const int c1 = c0 + per < nch ? c0 + per : nch;
  int mine = 0;
  for (int c = c0; c < c1; ++c) mine += (gc[c + 1] - gc[c] == 1) ? 1 : 0;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  int incl = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if ((int)lane >= off) incl += y;
  }
  if (lane == 63u) s_scan[wv] = incl;
  __syncthreads();
  int q = incl - mine, total = 0;
  for (int v = 0; v < kNT / 64; ++v) {
    if (v < (int)wv) q += s_scan[v];
    total += s_scan[v];
  }
  for (int c = c0; c < c1; ++c)
    if (gc[c + 1] - gc[c] == 1) out[q++] = gp[gc[c]];
  if (threadIdx.x == 0) count[t] = total;
}

// Sums of the two rows of every listed chain: one work-group per k copies
// row k into LDS (coalesced) and forms every repetition's sums from it:
// vals[t][k][2 q + 0] = x + y, [2 q + 1] = x - y, with x the chain's first
// row and y its second, added in float32 and rounded once (what the
// in-kernel fix-up of such a chain computes).
template <typename IN>
__global__ __launch_bounds__(256) void pair_sums_kernel(const IN* __restrict__ rows, int64_t ld,
                                                        int64_t n_inner, int64_t n, int d,
                                                        const uint2* __restrict__ list,
                                                        const int32_t* __restrict__ count,
                                                        int cap, IN* __restrict__ vals) {
  extern __shared__ __align__(16) unsigned char psm[];
  IN* row = reinterpret_cast<IN*>(psm);
  const int64_t kk = blockIdx.x;
  const IN* src = rows + kk * ld;
  for (int64_t i = threadIdx.x; i < n; i += 256) row[i] = src[i];
  __syncthreads();
  for (int t = 0; t < d; ++t) {
    const int n2 = count[t] < cap ? count[t] : cap;
    const uint2* pl = list + (size_t)t * (n / 2 + 1);
    uint32_t* out = reinterpret_cast<uint32_t*>(vals + ((size_t)t * n_inner + kk) * (2 * (size_t)cap));
    for (int q = threadIdx.x; q < n2; q += 256) {
      const uint2 y = pl[q];
      const float x0 = (float)row[y.x >> 16], x1 = (float)row[y.x & 0xFFFFu];
      out[q] = pack2(x0 + x1, x0 - x1, (IN*)nullptr);
    }
  }
}

}  // namespace

int mfma_pair_cap(int64_t n_rows, int64_t n_cols, int operand) {
  if (n_rows > 16383 || n_cols > 16383 || n_rows < 1 || n_cols < 1) return 0;
  const int64_t pA = (n_rows + 1 + 64 + 7) / 8 * 8, pB = (n_cols + 1 + 64 + 7) / 8 * 8;
  const int64_t base = 2 * (2 * ((int64_t)1 << kLB) + pA + pB);   // 16-bit elements
  const int64_t kMax = 160 * 1024 - 256;
  if (base + kDescLds > kMax) return 0;   // the chain-list instance: nothing merged
  // each operand's share of what is left, 2 values of 2 bytes per chain;
  // every element of the row region addressable with 15-bit byte offsets
  int64_t cap = (kMax - base - kDescLds) / 8;
  const int64_t n = operand ? n_cols : n_rows;
  const int64_t p0 = operand ? pB : pA;
  if (cap > n / 2) cap = n / 2;
  if (cap > (16384 - p0) / 2) cap = (16384 - p0) / 2;
  cap &= ~(int64_t)3;
  return cap > 0 ? (int)cap : 0;
}

cmm_status launch_pair_list(const PlanView& pv, int d, int64_t n, uint2* list, int32_t* count,
                            hipStream_t s) {
  ProfScope prof_("pairs", s);
  hipLaunchKernelGGL(pair_list_kernel, dim3((unsigned)d), dim3(kNT), 0, s, pv, n, list, count);
  return hip_check(hipGetLastError(), "pair list launch");
}

cmm_status launch_pair_sums(const void* rows, int64_t ld, cmm_dtype lp, int d, int64_t n_inner,
                            int64_t n, const uint2* list, const int32_t* count, int cap,
                            void* vals, hipStream_t s) {
  ProfScope prof_("pairs", s);
  if (cap <= 0 || n_inner <= 0) return CMM_OK;
  if (n_inner > 0x7FFFFFFF || n > 16383) return invalid("pair sums: size out of range");
  const size_t lds = 2 * (size_t)n;   // one row of 16-bit values
  if (lp == CMM_BF16)
    hipLaunchKernelGGL(pair_sums_kernel<__bf16>, dim3((unsigned)n_inner), dim3(256), lds, s,
                       (const __bf16*)rows, ld, n_inner, n, d, list, count, cap, (__bf16*)vals);
  else
    hipLaunchKernelGGL(pair_sums_kernel<_Float16>, dim3((unsigned)n_inner), dim3(256), lds, s,
                       (const _Float16*)rows, ld, n_inner, n, d, list, count, cap,
                       (_Float16*)vals);
  return hip_check(hipGetLastError(), "pair sums launch");
}

template <typename IN>
static cmm_status launch_mfma_t(const CompressArgs& a0, hipStream_t s) {
  ProfScope prof_("compress", s);
  CompressArgs a = a0;
  const int64_t blocks = ((int64_t)a.d << (a.log2b - kLB)) * a.groups;
  if (a.n_rows > 16383 || a.n_cols > 16383) {   // byte offset of the zero pad in 15 bits
    set_error("compress (mfma): needs n_rows, n_cols <= 16383");
    return CMM_EUNSUPPORTED;
  }
  if (a.pair_capA < 0 || a.pair_capB < 0 || a.pair_capA > mfma_pair_cap(a.n_rows, a.n_cols, 0) ||
      a.pair_capB > mfma_pair_cap(a.n_rows, a.n_cols, 1) || (a.pair_capA & 3) || (a.pair_capB & 3)) {
    set_error("compress (mfma): merged-chain capacity out of range");
    return CMM_EINVAL;
  }
  const size_t pitch = ((size_t)a.n_rows + 1 + 64 + 7) / 8 * 8 + 2 * (size_t)a.pair_capA +
                       ((size_t)a.n_cols + 1 + 64 + 7) / 8 * 8 + 2 * (size_t)a.pair_capB;
  const size_t base = sizeof(IN) * (2 * ((size_t)1 << kLB) + pitch);
  const size_t kMax = 160 * 1024 - 256;   // the kernel's own counters take a few bytes more
  if (base > kMax) { set_error("compress (mfma): rows do not fit in LDS"); return CMM_EUNSUPPORTED; }
  const bool desc = base + kDescLds <= kMax;
  int64_t cap = (int64_t)((kMax - base) / sizeof(uint2));
  const int64_t want = desc ? kDescLds / 8 : a.n_rows + a.n_cols;
  if (cap > want) cap = want;
  a.ex_cap = cap;
  const size_t lds = base + sizeof(uint2) * (size_t)cap;
  a.dma = (a.n_rows % 8 == 0) && (a.n_cols % 8 == 0) && (a.ldb % 8 == 0) &&
          ((uintptr_t)a.At % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
  auto kern = desc ? compress_mfma_kernel<IN, true> : compress_mfma_kernel<IN, false>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return hip_check(e, "compress (mfma): set LDS size");
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kNT), lds, s, a);
  return hip_check(hipGetLastError(), "compress (mfma) kernel launch");
}

cmm_status launch_compress_mfma(const CompressArgs& a, cmm_dtype lp, hipStream_t s) {
  if (a.log2b < kLB) {
    set_error("compress (mfma): needs log2b >= 14");
    return CMM_EUNSUPPORTED;
  }
  if (lp == CMM_BF16) return launch_mfma_t<__bf16>(a, s);
  return launch_mfma_t<_Float16>(a, s);
}

// Low-precision copies of the operands: out[c][r] = in[r][c] (transpose)
// or out[r][c] = in[r][c], rounded to nearest even.
namespace {
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void lp_transpose_kernel(const TI* __restrict__ in, int64_t rows,
                                                           int64_t cols, int64_t ld,
                                                           TO* __restrict__ out) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y, c = c0 + tx;
    if (r < rows && c < cols) tile[y][tx] = (float)in[r * ld + c];
  }
  __syncthreads();
  for (int y = ty; y < 64; y += 4) {
    const int64_t c = c0 + y, r = r0 + tx;
    if (r < rows && c < cols) out[c * rows + r] = (TO)tile[tx][y];
  }
}
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void lp_convert_kernel(const TI* __restrict__ in, int64_t rows,
                                                         int64_t cols, int64_t ld,
                                                         TO* __restrict__ out) {
  const int64_t n = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const int64_t r = q / cols, c = q - r * cols;
    out[q] = (TO)(float)in[r * ld + c];
  }
}
template <typename TO>
cmm_status lp_copy_t(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols, int64_t ld,
                     void* out, bool transpose, hipStream_t s) {
  if (transpose) {
    dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    if (in_dt == CMM_F64)
      hipLaunchKernelGGL((lp_transpose_kernel<double, TO>), grid, dim3(256), 0, s,
                         (const double*)in, rows, cols, ld, (TO*)out);
    else
      hipLaunchKernelGGL((lp_transpose_kernel<float, TO>), grid, dim3(256), 0, s,
                         (const float*)in, rows, cols, ld, (TO*)out);
  } else {
    int64_t gsz = (rows * cols + 255) / 256;
    if (gsz > 65536) gsz = 65536;
    if (gsz < 1) gsz = 1;
    if (in_dt == CMM_F64)
      hipLaunchKernelGGL((lp_convert_kernel<double, TO>), dim3((unsigned)gsz), dim3(256), 0, s,
                         (const double*)in, rows, cols, ld, (TO*)out);
    else
      hipLaunchKernelGGL((lp_convert_kernel<float, TO>), dim3((unsigned)gsz), dim3(256), 0, s,
                         (const float*)in, rows, cols, ld, (TO*)out);
  }
  return hip_check(hipGetLastError(), "low-precision copy launch");
}
}  // namespace

cmm_status launch_lp_copy(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols, int64_t ld,
                          void* out, cmm_dtype lp, bool transpose, hipStream_t s) {
  ProfScope prof_("transpose", s);
  if (lp == CMM_BF16) return lp_copy_t<__bf16>(in, in_dt, rows, cols, ld, out, transpose, s);
  return lp_copy_t<_Float16>(in, in_dt, rows, cols, ld, out, transpose, s);
}

}  // namespace cmm
