// Internal declarations shared by the HIP translation units of libcmm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "cmm.h"

namespace cmm {

constexpr uint32_t kSignBit = 0x80000000u;
constexpr uint32_t kBucketMask = 0x7FFFFFFFu;

// Thread-local message for cmm_last_error().
void set_error(const std::string& msg);

// Host checks shared by every entry point that takes a cmm_problem.
cmm_status validate_problem(const cmm_problem* pr, const char* fn);

// Returns CMM_EINVAL after recording msg.
cmm_status invalid(const std::string& msg);

// Maps a HIP error to CMM_EHIP (recording where it happened) or CMM_OK.
cmm_status hip_check(hipError_t e, const char* what);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t dtype_size(cmm_dtype t) {
  switch (t) {
    case CMM_F64: return 8;
    case CMM_F32: return 4;
    case CMM_BF16: return 2;
    case CMM_F16: return 2;
  }
  return 0;
}

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------ kernel timing
// While timing is enabled (cmm_profile_enable), launchers bracket their
// kernels with HIP events recorded on the launch stream; cmm_profile_query
// sums the elapsed times per kernel name.  Disabled, a scope costs one
// relaxed atomic load.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t stream_;
  hipEvent_t start_ = nullptr;
};

// ---------------------------------------------------------------- launchers
// Every launcher only enqueues work; arguments were validated by the caller.
cmm_status launch_hash(const uint64_t* keys, int d, int64_t n_rows, int64_t n_cols, int log2b,
                       uint32_t* tab1, uint32_t* tab2, hipStream_t s);
cmm_status launch_hash_family(cmm_hash_kind kind, const uint64_t* keys, int d, int64_t n_rows,
                              int64_t n_cols, int log2b, uint32_t* tab1, uint32_t* tab2,
                              hipStream_t s);

cmm_status launch_sketch(int side, const void* M, cmm_dtype dt, int64_t rows, int64_t cols,
                         int64_t ld, const uint32_t* tab, int d, int log2b, int64_t k0,
                         int64_t kc, void* out, cmm_dtype out_dt, hipStream_t s);

cmm_status launch_fwht(void* x, cmm_dtype dt, int64_t batch, int log2b, double scale,
                       hipStream_t s);

cmm_status launch_accumulate(const void* X, const void* Y, cmm_dtype dt, int d, int64_t kc,
                             int log2b, double* p_hat, hipStream_t s);

// cyclic: Pagh's FFT form, buckets combined as (h1 + h2) mod b
cmm_status launch_extract(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                          int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                          void* C_hat, cmm_dtype out_dt, int64_t ldc, hipStream_t s,
                          bool cyclic = false);

// Pagh's FFT form: batched complex float64 transform (natural order; in and
// out distinct when log2n > 12), its staged Compress helpers
cmm_status launch_fft(const void* in, void* out, int64_t batch, int log2n, int inverse,
                      double scale, hipStream_t s);
cmm_status launch_pack(const double* X, const double* Y, void* Z, size_t n, hipStream_t s);
cmm_status launch_accumulate_cyclic(const void* Z, int d, int64_t kc, int log2b, void* P,
                                    hipStream_t s);
cmm_status launch_zero_complex(void* x, size_t n, hipStream_t s);
cmm_status launch_real_part(const void* Z, double* p, size_t n, hipStream_t s);

cmm_status launch_extract_entries(const double* p, const uint32_t* tab1, const uint32_t* tab2,
                                  int d, int64_t n_rows, int64_t n_cols, int log2b,
                                  cmm_estimator est, const int64_t* rows, const int64_t* cols,
                                  int64_t count, void* out, cmm_dtype out_dt, hipStream_t s);
cmm_status launch_extract_heavy(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                                int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                                double threshold, int64_t* rows, int64_t* cols, void* vals,
                                cmm_dtype out_dt, int64_t capacity, int64_t* count,
                                hipStream_t s);
// Top-K Decompress (k_topk): workspace bytes for k, and the launch sequence.
cmm_status topk_workspace_bytes(int64_t k, size_t* bytes);
cmm_status launch_extract_topk(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                               int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator est,
                               int64_t k, int64_t* rows, int64_t* cols, void* vals,
                               cmm_dtype out_dt, void* workspace, size_t ws_bytes, hipStream_t s);
cmm_status launch_extract_reps(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                               int64_t n_rows, int64_t n_cols, int log2b, const int64_t* rows,
                               const int64_t* cols, int64_t count, void* out, cmm_dtype out_dt,
                               hipStream_t s);
cmm_status launch_correctness(const void* C_hat, cmm_dtype dt, int64_t ldh, const double* C,
                              int64_t ldc, int64_t n_rows, int64_t n_cols, const int64_t* rows,
                              const int64_t* cols, int64_t n_big, double thr, double tol,
                              int64_t* counts, hipStream_t s);

// Fill n doubles with zero (a kernel, not hipMemsetAsync, so that the
// sequence stays valid under stream capture).
cmm_status launch_zero(double* x, size_t n, hipStream_t s);

// Sum g partial float64 vectors of length len (stored back to back) into
// out, in ascending partial order.
cmm_status launch_reduce_partials(const double* parts, int g, size_t len, double* out,
                                  hipStream_t s);

// ------------------------------------------------------ fused compress
// Per-call plan of the lo-bucket membership of one operand (see k_compress).
struct PlanView {
  int32_t* first;     // [d][b_lo]  lowest index in each lo-bucket, or -1
  uint2* pairs;       // [d][n]     (index | first << 16, hi-bits xor | sign xor << 31)
                      //            of every non-first index, bucket by bucket,
                      //            each bucket's chain in ascending index order
  int32_t* cstart;    // [d][n + 2] start of each chain in pairs (+ end sentinel)
  int32_t* nchains;   // [d]        number of buckets with two or more indices
};

struct CompressArgs {
  const void* At;          // A^T: n_inner x n_rows, dense
  const void* B;           // n_inner x n_cols, leading dimension ldb
  int64_t ldb;
  int64_t n_rows, n_cols, n_inner;
  const uint32_t* tab1;    // [d][n_rows]
  const uint32_t* tab2;    // [d][n_cols]
  PlanView planA, planB;
  int d, log2b, groups;
  double* partial;         // [groups][d][2^log2b]
  int64_t ex_cap;          // set by the launcher: LDS entries for the extras
  int dma;                 // set by the launcher: asynchronous row copies
  int variant;             // 0: default kernel for (dtype, b_lo); 1: 32 elements per thread
  int ovf16 = 0;           // set by the launcher: positions of the partial third
                           // descriptor slot of the 16-element kernel (<= 512)
  // Precision form only: the two-row chains of each repetition merged ahead
  // of the kernel.  list [d][n / 2 + 1] holds a chain's plan entry (member |
  // first << 16, hi-bits xor | sign xor << 31) in chain order, count [d] their
  // number, vals [d][n_inner][2 cap] the low-precision sums x + y and x - y
  // of the chain's two rows for every k.  cap = 0: no merged chains.
  const uint2* pair_listA = nullptr;
  const uint2* pair_listB = nullptr;
  const int32_t* pair_countA = nullptr;
  const int32_t* pair_countB = nullptr;
  const void* pair_valsA = nullptr;
  const void* pair_valsB = nullptr;
  int pair_capA = 0, pair_capB = 0;
};

// Transform window per repetition for the fused Compress with b_lo = 2^lb:
// the window s (0 <= s <= min(log2b - lb, kMaxWindow)) whose bits s .. s +
// lb - 1 of the bucket index leave the fewest collisions in both tables,
// and the tables with their bucket bits rotated right by s (rtab1
// [d][n_rows], rtab2 [d][n_cols], rot [d]).  A compress on the rotated
// tables yields p_hat in the rotated frame; launch_reduce_window sums its
// partials and restores the natural order.
constexpr int kMaxWindow = 5;
cmm_status launch_window(const uint32_t* tab1, const uint32_t* tab2, int d, int64_t n_rows,
                         int64_t n_cols, int log2b, int lb, uint32_t* rtab1, uint32_t* rtab2,
                         int32_t* rot, hipStream_t s);
// out[t][u] = sum over q < g, in order, of parts[q][t][rotr(u, rot[t])]
// (rotation of the log2b bucket bits; rot = nullptr: none).
cmm_status launch_reduce_window(const double* parts, int g, int d, int log2b, const int32_t* rot,
                                double* out, hipStream_t s);

size_t plan_bytes(int d, int64_t n, int lb);
size_t plan_lds_bytes(int64_t n, int lb);
// The plan's arrays at p (plan_bytes(d, n, lb) bytes), in this order.
__host__ __device__ inline PlanView carve_plan(char* p, int d, int64_t n, int lb) {
  const size_t blo = (size_t)1 << lb;
  PlanView v;
  v.first = reinterpret_cast<int32_t*>(p); p += align_up(sizeof(int32_t) * d * blo, 256);
  v.pairs = reinterpret_cast<uint2*>(p); p += align_up(sizeof(uint2) * d * (size_t)n, 256);
  v.cstart = reinterpret_cast<int32_t*>(p); p += align_up(sizeof(int32_t) * d * (size_t)(n + 2), 256);
  v.nchains = reinterpret_cast<int32_t*>(p);
  return v;
}
cmm_status launch_plan(const uint32_t* tab, int d, int64_t n, int lb, const PlanView& pv,
                       hipStream_t s);
cmm_status launch_compress(const CompressArgs& a, cmm_dtype dt, int lb, hipStream_t s);
// fused FFT-form Compress (b_lo = 2^12 complex, partials [groups][d][b]
// complex), its LDS size and shape limits, and the reduction of its partials
// into the full transformed accumulator
size_t compress_fft_lds(int64_t n_rows, int64_t n_cols, int log2b);
bool compress_fft_supported(int64_t n_rows, int64_t n_cols, int log2b);
cmm_status launch_compress_fft(const CompressArgs& a, hipStream_t s);
cmm_status launch_reduce_fft_partials(const void* part, int groups, int d, int log2b, void* P,
                                      hipStream_t s);
// LDS bytes of the fused kernel (b_lo = 2^lb, 32 elements per thread)
// before the collision lists.
size_t compress_lds_base(cmm_dtype dt, int lb, int64_t n_rows, int64_t n_cols);
// The same for the 16-element layout (b_lo = 2^13, 512 threads).
size_t compress16_lds_base(cmm_dtype dt, int64_t n_rows, int64_t n_cols);
// LDS of the 16-element kernel with descriptor fix-ups (rows with their 64
// spare elements, the descriptors); usable when n_rows, n_cols + 64 < 2^15
size_t compress16_desc_lds(cmm_dtype dt, int64_t n_rows, int64_t n_cols);

// ------------------------------------------------------------ batched form
// One problem of a batch as the persistent kernel reads it: workspace
// buffers as byte offsets from the workspace base (so that the table does
// not depend on where the workspace lives), caller buffers as pointers.
struct BatchPair {
  int64_t at;              // A^T in the compute type
  int64_t bc;              // converted B, or -1 to read the caller's B
  const void* B;
  int64_t ldb, n_rows, n_cols, n_inner;
  const uint32_t* tab1;
  const uint32_t* tab2;
  int64_t planA, planB;    // plans (carve_plan layout)
  // per-repetition transform windows: the tables rotated to them
  // ([d][n_rows], [d][n_cols] u32) and the rotations ([d] i32), or -1 when
  // the bucket has no bits beyond the slice
  int64_t rtab1, rtab2, rot;
  int64_t partial;         // [groups][d][2^log2b] float64, in the rotated frame
  int64_t ex_cap;
  int d, log2b, groups, dma;
  int ovf16;               // partial third descriptor slot (16-element layout)
};
struct BatchItem {
  uint32_t pair, unit, group;   // unit = t * b_hi + u_hi
};
// Persistent Compress over all items: `wgs` work-groups take items from
// the queue counter (zeroed before the launch) until none are left.
// radix: elements per thread of the transform layout (32: b_lo from 2^11
// to 2^13; 16: b_lo = 2^13).
cmm_status launch_compress_batched(char* ws, const BatchPair* pairs, const BatchItem* items,
                                   int n_items, int* queue, cmm_dtype dt, int lb, int radix,
                                   bool desc,
                                   int wgs, size_t lds, hipStream_t s);

// Precision form: MFMA compress (b_lo = 2^14) on bf16 / fp16 rows.
cmm_status launch_compress_mfma(const CompressArgs& a, cmm_dtype lp, hipStream_t s);
// Merged two-row chains of the precision form: the largest number of chains
// per repetition whose sums the kernel can stage beside a row of n values
// (0 when none fit), the chain lists from the plans, and the sums of the
// rows of At (n_inner x n_rows) or B (n_inner x n_cols, leading dimension
// ld) in the low precision lp.
int mfma_pair_cap(int64_t n_rows, int64_t n_cols, int operand);
cmm_status launch_pair_list(const PlanView& pv, int d, int64_t n, uint2* list, int32_t* count,
                            hipStream_t s);
cmm_status launch_pair_sums(const void* rows, int64_t ld, cmm_dtype lp, int d, int64_t n_inner,
                            int64_t n, const uint2* list, const int32_t* count, int cap,
                            void* vals, hipStream_t s);
// ------------------------------------------------ differentiation form
// Shape of the W scatter (extract^T): row blocks of rows_per rows, windows
// of 2^wb buckets (at most 128 KB of LDS).
struct ScatterShape {
  int wb;
  int64_t rows_per;
  int64_t blocks;
  bool f32;          // window sums in float32 (the float32 form), else float64
};
// q partials [blocks][d][2^log2b] (float64) of the bucket sums of W.
cmm_status launch_wscatter(const void* W, cmm_dtype wdt, int64_t ldw, const uint32_t* tab1,
                           const uint32_t* tab2, int d, int64_t n_rows, int64_t n_cols,
                           int log2b, const ScatterShape& sh, double* part, hipStream_t s);

struct AdjointArgs {
  CompressArgs c;    // operands of one k-chunk (c.n_inner = chunk length), tables, plans
  const double* r;   // [d][2^log2b]  2^-log2b H q
  double scale;      // 1 / d
  void* partA;       // [d * b_hi][chunk][n_rows]  per-(t, u_hi) columns of dA
  void* partB;       // [d * b_hi][chunk][n_cols]  per-(t, u_hi) rows of dB
};
// out[r][c] = 0 for a rows x cols matrix (leading dimension ld) of dt.
cmm_status launch_zero_matrix(void* out, cmm_dtype dt, int64_t rows, int64_t cols, int64_t ld,
                              hipStream_t s);
size_t adjoint_lds_bytes(cmm_dtype dt, int lb, int64_t n_rows, int64_t n_cols);
cmm_status launch_adjoint(const AdjointArgs& a, cmm_dtype dt, int lb, hipStream_t s);
// Sum P partials [P][kc][n] into out rows kb.. (transpose = false) or
// columns kb.. (transpose = true), ascending p, in float64.
cmm_status launch_adjoint_reduce(const void* part, cmm_dtype part_dt, int P, int64_t kc,
                                 int64_t n, void* out, cmm_dtype out_dt, int64_t ld, int64_t kb,
                                 bool transpose, hipStream_t s);

// bf16 / fp16 copy of a float64 / float32 matrix, transposed or not.
cmm_status launch_lp_copy(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols, int64_t ld,
                          void* out, cmm_dtype lp, bool transpose, hipStream_t s);

// out[c][r] = in[r][c] (dense out, leading dimension rows), with conversion.
cmm_status launch_transpose(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols,
                            int64_t ld, void* out, cmm_dtype out_dt, hipStream_t s);
// out[r][c] = in[r][c] (dense out), with conversion.
cmm_status launch_convert(const void* in, cmm_dtype in_dt, int64_t rows, int64_t cols,
                          int64_t ld, void* out, cmm_dtype out_dt, hipStream_t s);

}  // namespace cmm
