// Standalone count sketch (Algorithm 1, the two sketch loops of Compress).
//
// A work-group owns one repetition t, one window of W <= 1024 consecutive
// buckets and a run of tiles of KT consecutive inner indices k.  It scans
// the hash table of t once, keeps the indices that land in its window as a
// list in LDS (ascending index order), and ranks equal buckets in that
// order.  Each tile then accumulates its KT x W sketch values in LDS, rank
// level by rank level (the terms of one bucket are added in ascending index
// order, so the result equals a sequential left-to-right sum and does not
// depend on scheduling), and streams them to HBM with coalesced stores.
// The list is built once per work-group when the window's hits fit it
// (always, unless b is small against n); otherwise it is rebuilt segment by
// segment for every tile.
#include <type_traits>

#include "cmm_internal.h"

namespace cmm {
namespace {

constexpr int kSkThreads = 256;
constexpr int kSkLogW = 10;       // at most 1024 buckets per window
constexpr int kSkHC = 2048;       // hit-list capacity
constexpr int kSkChunk = 1024;    // indices scanned per step (4 per thread)
constexpr int kSkTarget = 2048;   // work-groups aimed for (the tiles are split to reach it)
constexpr int32_t kSkNone = 0x7FFFFFFF;

template <typename T>
struct SkTile { static constexpr int value = sizeof(T) == 8 ? 4 : 8; };   // 32 KB of LDS

// Input type T, output type O; the sums are formed in float64 when either
// is float64 (float32 inputs widen exactly), and rounded once to O.
template <typename T, typename O>
struct SkAcc { typedef typename std::conditional<sizeof(T) == 8 || sizeof(O) == 8, double, float>::type type; };

template <typename T, typename O>
__global__ __launch_bounds__(kSkThreads) void sketch_kernel(
    int side, const T* __restrict__ M, int64_t ld, const uint32_t* __restrict__ tab,
    int64_t n_idx, int log2b, int log2w, int64_t nwin, int64_t tiles_per_group, int64_t k0,
    int64_t kc, int d, O* __restrict__ out) {
  typedef typename SkAcc<T, O>::type A;
  constexpr int KT = SkTile<A>::value;
  __shared__ A acc[KT << kSkLogW];           // [kk][bucket in window]
  __shared__ uint32_t hidx[kSkHC];           // hit index
  __shared__ uint32_t hkey[kSkHC];           // bucket in window | rank << 16 | sign bit
  __shared__ int32_t tag[1 << kSkLogW];
  __shared__ int32_t wsum[4][kSkThreads / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t lin = blockIdx.x;
  const int64_t w = lin % nwin;
  const int t = (int)((lin / nwin) % d);
  const int64_t grp = lin / (nwin * d);
  const int W = 1 << log2w;
  const int64_t b = (int64_t)1 << log2b;
  const uint32_t bmask = (uint32_t)(b - 1);
  const uint32_t* tb = tab + (size_t)t * n_idx;
  const int64_t ntiles = (kc + KT - 1) / KT;
  const int64_t kt0 = grp * tiles_per_group;
  const int64_t kt1 = kt0 + tiles_per_group < ntiles ? kt0 + tiles_per_group : ntiles;

  for (int e = tid; e < (KT << log2w); e += kSkThreads) acc[e] = A(0);
  for (int e = tid; e < W; e += kSkThreads) tag[e] = kSkNone;
  __syncthreads();

  // Hit list of the indices from pos on, in ascending order, until it could
  // overflow; cnt is the list length (the same in every thread).  Returns the
  // first index not scanned.
  auto build = [&](int64_t pos, int& cnt) -> int64_t {
    cnt = 0;
    int64_t c0 = pos;
    for (; c0 < n_idx && cnt + kSkChunk <= kSkHC; c0 += kSkChunk) {
      uint32_t e[4];
      bool hit[4];
      unsigned long long m[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t idx = c0 + q * kSkThreads + tid;
        e[q] = idx < n_idx ? tb[idx] : 0u;
        hit[q] = idx < n_idx && (int64_t)((e[q] & bmask) >> log2w) == w;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        m[q] = __ballot(hit[q]);
        if (lane == 0) wsum[q][wv] = __popcll(m[q]);
      }
      __syncthreads();
      int base = cnt;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int off = base;
        for (int v = 0; v < wv; ++v) off += wsum[q][v];
        for (int v = 0; v < kSkThreads / 64; ++v) base += wsum[q][v];
        if (hit[q]) {
          const int h = off + __popcll(m[q] & ((1ull << lane) - 1ull));
          hidx[h] = (uint32_t)(c0 + q * kSkThreads + tid);
          hkey[h] = ((e[q] & bmask) & (uint32_t)(W - 1)) | (e[q] & kSignBit);
        }
      }
      cnt = base;
      __syncthreads();   // wsum read everywhere before the next step writes it
    }
    return c0 < n_idx ? c0 : n_idx;
  };

  // Ranks the list: the rank of an entry is the number of earlier entries
  // with the same bucket.  Round r gives rank r to the first unranked entry
  // of every bucket.  Returns the number of ranks.
  auto rank_list = [&](int cnt) -> int {
    if (cnt == 0) return 0;
    uint32_t pend = 0;   // bit s: entry tid + s * kSkThreads is unranked
    for (int s = 0; tid + s * kSkThreads < cnt; ++s) pend |= 1u << s;
    for (int round = 0;; ++round) {
      for (int s = 0; tid + s * kSkThreads < cnt; ++s)
        if ((pend >> s) & 1u) {
          const int h = tid + s * kSkThreads;
          atomicMin(&tag[hkey[h] & 0xFFFFu], h);
        }
      __syncthreads();
      uint32_t won = 0;
      for (int s = 0; tid + s * kSkThreads < cnt; ++s)
        if ((pend >> s) & 1u) {
          const int h = tid + s * kSkThreads;
          if (tag[hkey[h] & 0xFFFFu] == h) won |= 1u << s;
        }
      __syncthreads();   // every thread read its tags before they are reset
      for (int s = 0; tid + s * kSkThreads < cnt; ++s)
        if ((won >> s) & 1u) {
          const int h = tid + s * kSkThreads;
          tag[hkey[h] & 0xFFFFu] = kSkNone;
          hkey[h] |= (uint32_t)round << 16;
        }
      pend &= ~won;
      if (!__syncthreads_or(pend != 0u)) return round + 1;
    }
  };

  const int64_t kdim = side == 0 ? 1 : ld;   // stride of M along k
  const int64_t idim = side == 0 ? ld : 1;   // stride of M along the sketched index
  bool single = false;
  int cnt = 0, levels = 0;
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    const int64_t kb = kt * KT;
    int64_t pos = 0;
    do {
      if (!single) {
        const int64_t next = build(pos, cnt);
        levels = rank_list(cnt);
        single = pos == 0 && next >= n_idx;
        pos = next;
      } else {
        pos = n_idx;
      }
      for (int r = 0; r < levels; ++r) {
        for (int e = tid; e < cnt * KT; e += kSkThreads) {
          const int h = e / KT;
          const int kk = e - h * KT;
          const uint32_t hk = hkey[h];
          if ((int)((hk >> 16) & 0x7FFFu) != r || kb + kk >= kc) continue;
          const A m = (A)M[(int64_t)hidx[h] * idim + (k0 + kb + kk) * kdim];
          acc[(kk << log2w) + (hk & 0xFFFFu)] += (hk & kSignBit) ? -m : m;
        }
        __syncthreads();
      }
    } while (pos < n_idx);
    // stream the tile out and clear it for the next one
    for (int e = tid; e < (KT << log2w); e += kSkThreads) {
      const int kk = e >> log2w;
      const int x = e & (W - 1);
      const A v = acc[e];
      acc[e] = A(0);
      if (kb + kk < kc) out[((size_t)t * kc + kb + kk) * b + w * W + x] = (O)v;
    }
    __syncthreads();
  }
}

}  // namespace

template <typename T, typename O>
static void launch_sketch_t(dim3 grid, hipStream_t s, int side, const void* M, int64_t ld,
                            const uint32_t* tab, int64_t n_idx, int log2b, int log2w,
                            int64_t nwin, int64_t per, int64_t k0, int64_t kc, int d, void* out) {
  hipLaunchKernelGGL((sketch_kernel<T, O>), grid, dim3(kSkThreads), 0, s, side,
                     (const T*)M, ld, tab, n_idx, log2b, log2w, nwin, per, k0, kc, d, (O*)out);
}

cmm_status launch_sketch(int side, const void* M, cmm_dtype dt, int64_t rows, int64_t cols,
                         int64_t ld, const uint32_t* tab, int d, int log2b, int64_t k0,
                         int64_t kc, void* out, cmm_dtype out_dt, hipStream_t s) {
  ProfScope prof_("sketch", s);
  const int64_t n_idx = side == 0 ? rows : cols;
  const int log2w = log2b < kSkLogW ? log2b : kSkLogW;
  const int64_t nwin = (int64_t)1 << (log2b - log2w);
  // the tile follows the accumulation type (float64 when either side is)
  const int kt = (dt == CMM_F64 || out_dt == CMM_F64) ? SkTile<double>::value
                                                     : SkTile<float>::value;
  const int64_t ntiles = (kc + kt - 1) / kt;
  const int64_t base = (int64_t)d * nwin;
  int64_t groups = (kSkTarget + base - 1) / base;
  if (groups > ntiles) groups = ntiles;
  const int64_t per = (ntiles + groups - 1) / groups;
  groups = (ntiles + per - 1) / per;
  const int64_t blocks = base * groups;
  if (blocks > 0x7FFFFFFF) return invalid("cmm_sketch: d * 2^log2b too large");
  const dim3 grid((unsigned)blocks);
  if (dt == CMM_F64 && out_dt == CMM_F64)
    launch_sketch_t<double, double>(grid, s, side, M, ld, tab, n_idx, log2b, log2w, nwin, per, k0, kc, d, out);
  else if (dt == CMM_F64)
    launch_sketch_t<double, float>(grid, s, side, M, ld, tab, n_idx, log2b, log2w, nwin, per, k0, kc, d, out);
  else if (out_dt == CMM_F64)
    launch_sketch_t<float, double>(grid, s, side, M, ld, tab, n_idx, log2b, log2w, nwin, per, k0, kc, d, out);
  else
    launch_sketch_t<float, float>(grid, s, side, M, ld, tab, n_idx, log2b, log2w, nwin, per, k0, kc, d, out);
  return hip_check(hipGetLastError(), "sketch kernel launch");
}

}  // namespace cmm
