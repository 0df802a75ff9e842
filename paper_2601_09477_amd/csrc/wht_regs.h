// Register-resident Walsh-Hadamard transform pieces shared by the fused
// Compress kernel and its adjoint: butterflies, cross-lane exchanges, the
// two E = 32 transform passes and their index layouts, row staging into
// LDS and the collision-chain sums of the gather-form count sketch.
#pragma once
#include "cmm_internal.h"

namespace cmm {
namespace {

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
// Padded transpose buffer: one spare element after every 128.  Writes (L1',
// lanes 0..15 stepping u_lo bit 7) then hit 16 distinct bank pairs, reads
// (L2, lanes 0..15 stepping bits 0..3) are contiguous; and the padding is
// additive in the register part of the index, so every access is a base
// address plus an immediate offset.
__device__ __forceinline__ uint32_t swz(uint32_t x) { return x + (x >> 7); }

template <typename T, int LB>
struct Cfg {
  static constexpr int E = 32;
  static constexpr int NT = (1 << LB) / E;
};

// Copy a row of n values into LDS.  With `dma` the copy is issued as
// asynchronous 16-byte global->LDS loads (global_load_lds_dwordx4): each
// wavefront moves 64 consecutive 16-byte chunks per instruction, lane L to
// LDS offset 16 L; completion is awaited with s_waitcnt vmcnt(0) before the
// next barrier.  Without `dma` it is a plain load/store loop.
template <typename T, int NT>
__device__ __forceinline__ void stage_row(T* __restrict__ dst, const T* __restrict__ src,
                                          int64_t n, bool dma) {
  if (dma) {
    // the wave's first chunk is wave-uniform (readfirstlane), so the LDS
    // destination of every load is a scalar value; rounds with all 64
    // chunks in the row skip the per-lane test; chunks < 2^31
    constexpr int V = 16 / sizeof(T);
    const int chunks = (int)(n / V);
    const int lane = threadIdx.x & 63;
    const int wbase = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * 64;
    int c0 = wbase;
    for (; c0 + 64 <= chunks; c0 += NT)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + (size_t)(c0 + lane) * V),
          (__attribute__((address_space(3))) void*)(dst + (size_t)c0 * V), 16, 0, 0);
    if (c0 < chunks && c0 + lane < chunks)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + (size_t)(c0 + lane) * V),
          (__attribute__((address_space(3))) void*)(dst + (size_t)c0 * V), 16, 0, 0);
  } else {
    for (int64_t i = threadIdx.x; i < n; i += NT) dst[i] = src[i];
  }
}

// Elements of a staged row, rounded up so the next row stays 16-byte
// aligned, plus one zero pad element.
template <typename T>
__host__ __device__ constexpr int64_t row_pitch(int64_t n) {
  return (n + 1 + (16 / (int64_t)sizeof(T)) - 1) / (16 / (int64_t)sizeof(T)) * (16 / (int64_t)sizeof(T));
}

// x with its sign bit flipped when bit 31 of m is set.
__device__ __forceinline__ double flip_sign(double x, uint32_t m) {
  const uint64_t u = (uint64_t)__double_as_longlong(x) ^ ((uint64_t)m << 32);
  return __longlong_as_double((long long)u);
}
__device__ __forceinline__ float flip_sign(float x, uint32_t m) {
  return __uint_as_float(__float_as_uint(x) ^ m);
}

__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The non-first rows of one operand, bucket by bucket: a thread takes one
// bucket's chain and adds its rows onto the bucket's first row in rank
// (ascending index) order, row[first] += +-row[index], so every bucket
// receives its rows left to right without atomics.  Entries are fetched
// KB at a time (independent loads) and two chains are in flight per
// thread, so a chain costs a few round trips instead of two per row.  The
// sum is formed in A (the row's type, or float32 for low-precision rows).
template <typename T, typename A = T, int KB = 4>
__device__ __forceinline__ A chain_sum(const T* __restrict__ row, const uint2* __restrict__ ex,
                                       int beg, int end, uint32_t uhi, A accv) {
  for (int q0 = beg; q0 < end; q0 += KB) {
    uint2 x[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) x[j] = (q0 + j < end) ? ex[q0 + j] : make_uint2(0u, 0u);
    A v[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) v[j] = (q0 + j < end) ? (A)row[x[j].x & 0xFFFFu] : A(0);
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (q0 + j < end) {
        const uint32_t neg = (x[j].y >> 31) ^ (__popc(uhi & (x[j].y & kBucketMask)) & 1u);
        accv = accv + (neg ? -v[j] : v[j]);
      }
    }
  }
  return accv;
}

template <typename T, int NT>
__device__ __forceinline__ void fix_chains(T* __restrict__ row, const uint2* __restrict__ ex,
                                           const int32_t* __restrict__ cs, int nch,
                                           uint32_t uhi) {
  for (int c = threadIdx.x; c < nch; c += 2 * NT) {
    const int c2 = c + NT;
    const int b1 = cs[c], e1 = cs[c + 1];
    const int b2 = c2 < nch ? cs[c2] : 0, e2 = c2 < nch ? cs[c2 + 1] : 0;
    const uint32_t t1 = ex[b1].x >> 16;
    const uint32_t t2 = c2 < nch ? ex[b2].x >> 16 : 0u;
    const T a1 = row[t1];
    const T a2 = c2 < nch ? row[t2] : T(0);
    const T s1 = chain_sum(row, ex, b1, e1, uhi, a1);
    const T s2 = chain_sum(row, ex, b2, e2, uhi, a2);
    row[t1] = s1;
    if (c2 < nch) row[t2] = s2;
  }
}

// ------------------------------------------------ 16 elements per thread
// Layout for b_lo = 2^13 with 512 threads (two wavefronts per SIMD):
// 4 register bits, 6 lane bits, 3 wave bits.
//   L1 (gather, pass 1): reg -> u_lo bits 0..3, lane bits 4,5 -> 4,5,
//       lane bits 0..3 -> 6..9, waves -> 10..12.  Pass 1: stages 0..3 in
//       registers, stages 4 and 5 after permlane16/32 swaps with reg bits 0/1.
//   L2 (pass 2): reg -> 6..9, lane bits 4,5 -> 10,11 (permlane swaps),
//       lane bit 3 -> 12 (a DPP row_ror:8 butterfly, i.e. partner lane
//       xor 8), lane bits 0..2 -> 0..2, waves -> 3..5.
// Transpose buffer padding g(x) = x + (x >> 6) + 8 * bit12(x) makes both
// the L1' writes and the L2 reads free of bank conflicts and is additive in
// the register part of the index.

__device__ __forceinline__ uint32_t pad16(uint32_t x) { return x + (x >> 6) + ((x >> 9) & 8u); }

// Butterfly across lane bit 3: lanes with bit 3 clear keep a + b, lanes
// with it set b' = a - b, where the partner value comes from lane xor 8
// (row_ror:8 within 16-lane rows).  The rotation gives every lane a
// source, so the move needs no prior value in its destination (mov_dpp;
// update_dpp with an explicit old value costs one extra move per dword).
__device__ __forceinline__ double dpp_xor8(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x128, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x128, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float dpp_xor8(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x128, 0xF, 0xF, false));
}

template <int J, typename T>
__device__ __forceinline__ void stage_reg16(T (&v)[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e)
    if ((e & (1 << J)) == 0) bfly(v[e], v[e | (1 << J)]);
}
template <int J, int S, typename T>
__device__ __forceinline__ void swap_reg16(T (&v)[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e)
    if ((e & (1 << J)) == 0) {
      if (S == 16) xswap16(v[e], v[e | (1 << J)]);
      else xswap32(v[e], v[e | (1 << J)]);
    }
}
template <typename T>
__device__ __forceinline__ void pass1_16(T (&v)[16]) {
  stage_reg16<0>(v); stage_reg16<1>(v); stage_reg16<2>(v); stage_reg16<3>(v);
  swap_reg16<0, 16>(v); stage_reg16<0>(v);
  swap_reg16<1, 32>(v); stage_reg16<1>(v);
}
template <typename T>
__device__ __forceinline__ void pass2_16(T (&v)[16], T sgn8) {
  stage_reg16<0>(v); stage_reg16<1>(v); stage_reg16<2>(v); stage_reg16<3>(v);
  swap_reg16<0, 16>(v); stage_reg16<0>(v);
  swap_reg16<1, 32>(v); stage_reg16<1>(v);
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = fma(v[e], sgn8, dpp_xor8(v[e]));
}

}  // namespace
}  // namespace cmm
