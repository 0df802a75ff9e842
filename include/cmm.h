/*
 * cmm.h -- C ABI of the MI355X (gfx950) library for compressed matrix
 * multiplication in the Fast Walsh-Hadamard Transform form (Pagh's
 * Compress / Decompress with the FFT replaced by the FWHT; Andersson &
 * Karppa, "Engineering Compressed Matrix Multiplication with the Fast
 * Walsh-Hadamard Transform", Algorithm 1 and Section 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrix and vector pointers are DEVICE pointers owned by the caller.
 *   The library keeps no pointer after a call returns (except a batch
 *   plan, which keeps its problems) and allocates no device memory in any
 *   entry point; scratch memory comes from an explicit workspace argument
 *   where one is needed.
 * - `stream` is a hipStream_t passed as void*; NULL means the default
 *   stream.  Every call only enqueues work on that stream and returns; the
 *   results are valid once the stream has reached that point.
 * - Dense matrices are row-major with a leading dimension (elements
 *   between consecutive rows), ld >= number of columns (not checked for a
 *   matrix with no elements).
 * - Indices are 0-based.  h1/s1 hash the row index i of A, h2/s2 the column
 *   index j of B (Section 3.1).
 * - A hash TABLE entry is a uint32: bits [0, log2b) hold the bucket, bit 31
 *   the sign (1 means -1); bits [log2b, 31) are ignored.  Hence
 *   1 <= log2b <= 30.
 * - The Walsh-Hadamard transform is unnormalised and in natural (Sylvester)
 *   order, H[u][r] = (-1)^popcount(u & r), so H H = b I.  The inverse
 *   transform of Compress is applied with the exact scale 2^-log2b; p is
 *   then exactly the XOR convolution of eq. (fwhtxorconvolution).
 * - Errors are returned as status codes; nothing is thrown or aborted across
 *   the ABI.  Argument checks run on the host before anything is enqueued;
 *   on CMM_EINVAL nothing was launched.  cmm_last_error() gives a message
 *   for the last non-OK status returned on the calling host thread.
 *   Sizes of zero are a no-op returning CMM_OK.
 */
#ifndef CMM_H
#define CMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CMM_OK = 0,
  CMM_EINVAL = 1,       /* an argument check failed; nothing was launched   */
  CMM_ENOMEM = 2,       /* the workspace passed in is smaller than required */
  CMM_EHIP = 3,         /* a HIP runtime call or a kernel launch failed     */
  CMM_EUNSUPPORTED = 4  /* valid arguments, combination not implemented     */
} cmm_status;

typedef enum { CMM_F64 = 0, CMM_F32 = 1, CMM_BF16 = 2, CMM_F16 = 3 } cmm_dtype;

/* Decompress: median over the d repetitions (Algorithm 1; needs odd d) or
 * the mean over d (each repetition is unbiased, Section 3.1). */
typedef enum { CMM_MEDIAN = 0, CMM_MEAN = 1 } cmm_estimator;

/* ------------------------------------------------------------------ hash */
/* Section 4.2 multiply-add-shift family, drawn once per repetition as in
 * Algorithm 1: h(x) = floor(((a x + c) mod 2^64) / 2^(64 - log2b)) for the
 * buckets, the same with one output bit for the signs.
 *   keys  device uint64[d][4][2]: (a, c) for h1, h2, s1, s2 of repetition t.
 *   tab1  device uint32[d][n_rows] out: entry of row i of A, repetition t.
 *   tab2  device uint32[d][n_cols] out: entry of column j of B.
 * n_rows, n_cols <= 2^32 (the family's domain).  Bit-exact. */
cmm_status cmm_hash(const uint64_t* keys, int d, int64_t n_rows, int64_t n_cols, int log2b,
                    uint32_t* tab1, uint32_t* tab2, void* stream);

/* Alternative hash families.  Section 4.2 reports results for the
 * multiply-add-shift family only and names a simpler and a more complex one
 * that it does not define; this library reads them as:
 *   CMM_HASH_MULTIPLY_ADD_SHIFT  the Section 4.2 family (same as cmm_hash);
 *   CMM_HASH_MULTIPLY_SHIFT      h(x) = floor(((a x) mod 2^64) / 2^(64 - log2b))
 *                                with the low bit of a set (Dietzfelbinger et
 *                                al.; universal, not 2-wise independent: x = 0
 *                                is always bucket 0, sign +1);
 *   CMM_HASH_TABULATION          simple tabulation (Patrascu and Thorup):
 *                                h(x) = T0[x_0] ^ T1[x_1] ^ T2[x_2] ^ T3[x_3]
 *                                over the bytes of x (x_0 least significant),
 *                                log2b top bits of the 64-bit word; the sign
 *                                is the top bit of the sign function's word.
 * keys (device):
 *   multiply families  uint64[d][4][2], (a, c) for h1, h2, s1, s2 (c unused
 *                      by multiply-shift);
 *   tabulation         uint64[d][4][4][256]: for h1, h2, s1, s2 the tables
 *                      T0..T3 of 256 words each.
 * Tables as for cmm_hash (bucket | sign << 31); they feed every entry point
 * that takes tab1 / tab2 with keys NULL.  Bit-exact.  An unknown kind is
 * CMM_EINVAL. */
typedef enum {
  CMM_HASH_MULTIPLY_ADD_SHIFT = 0,
  CMM_HASH_MULTIPLY_SHIFT = 1,
  CMM_HASH_TABULATION = 2
} cmm_hash_kind;

cmm_status cmm_hash_family(cmm_hash_kind kind, const uint64_t* keys, int d, int64_t n_rows,
                           int64_t n_cols, int log2b, uint32_t* tab1, uint32_t* tab2,
                           void* stream);

/* ---------------------------------------------------------------- sketch */
/* Algorithm 1, the count-sketch loops of Compress, for kc consecutive values
 * of the inner index starting at k0:
 *   side 0 (M = A, rows x cols, ld):  out[t][kk][x] = sum over i with
 *          bucket(tab[t][i]) = x of sign(tab[t][i]) * A[i][k0 + kk]
 *          (tab is tab1, uint32[d][rows]);
 *   side 1 (M = B, rows x cols, ld):  out[t][kk][x] = sum over j with
 *          bucket(tab[t][j]) = x of sign(tab[t][j]) * B[k0 + kk][j]
 *          (tab is tab2, uint32[d][cols]).
 * dtype (of M) and out_dtype (of out) are each CMM_F64 or CMM_F32; out is
 * [d][kc][2^log2b], fully overwritten.  Terms are added in ascending index
 * order, in float64 when either type is float64 (float32 inputs widen
 * exactly), and each sum is rounded once to out_dtype, so results are
 * deterministic. */
cmm_status cmm_sketch(int side, const void* M, cmm_dtype dtype, int64_t rows, int64_t cols,
                      int64_t ld, const uint32_t* tab, int d, int log2b, int64_t k0, int64_t kc,
                      void* out, cmm_dtype out_dtype, void* stream);

/* ------------------------------------------------------------------ FWHT */
/* Section 3.2: in-place Walsh-Hadamard transform of `batch` contiguous
 * vectors of length 2^log2b (natural order, unnormalised butterflies), then
 * x *= scale.  dtype CMM_F64 or CMM_F32.  scale must be a power of two
 * (1.0 for the forward transform, 2^-log2b for the inverse of Compress) so
 * that it is exact. */
cmm_status cmm_fwht(void* x, cmm_dtype dtype, int64_t batch, int log2b, double scale,
                    void* stream);

/* ------------------------------------------------------------ accumulate */
/* Algorithm 1, p[t] <- p[t] + H{p_A} o H{p_B}, over kc values of k:
 *   p_hat[t][u] += sum_kk X[t][kk][u] * Y[t][kk][u]   (kk ascending,
 *   product rounded, then added: no fused multiply-add).
 * X, Y: [d][kc][2^log2b] of dtype CMM_F64 or CMM_F32; p_hat: float64
 * [d][2^log2b], accumulated into (the caller zeroes it first). */
cmm_status cmm_accumulate(const void* X, const void* Y, cmm_dtype dtype, int d, int64_t kc,
                          int log2b, double* p_hat, void* stream);

/* --------------------------------------------------------------- extract */
/* Algorithm 1, Decompress, for the dense n_rows x n_cols block:
 *   C_hat[i][j] = Median_t ( s1_t(i) s2_t(j) p[t][h1_t(i) xor h2_t(j)] )
 * (or the mean over t).  p: float64 [d][2^log2b]; tables as above.
 * out_dtype CMM_F64 or CMM_F32; C_hat row-major with leading dimension ldc.
 * CMM_MEDIAN requires odd d.  The median is the exact middle value. */
cmm_status cmm_extract(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                       int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                       void* C_hat, cmm_dtype out_dtype, int64_t ldc, void* stream);

/* ---------------------------------------------------------- sparse queries */
/* Decompress at a list of entries (Algorithm 1's Decompress, one pair at a
 * time, without the dense output):
 *   out[q] = Median_t ( s1_t(rows[q]) s2_t(cols[q]) p[t][h1_t(rows[q]) xor h2_t(cols[q])] )
 * (or the mean) for q < count.  rows, cols: device int64[count]; an index
 * outside [0, n_rows) x [0, n_cols) gives NaN.  out: device out_dtype[count]. */
cmm_status cmm_extract_entries(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                               int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                               const int64_t* rows, const int64_t* cols, int64_t count, void* out,
                               cmm_dtype out_dtype, void* stream);

/* Heavy hitters: every (i, j) of the n_rows x n_cols grid whose estimate has
 * |C_hat[i][j]| >= threshold (the large entries of the product, which the
 * compressed product is meant to find, Section 1), without writing the
 * dense C_hat.  The hits are written to out_rows / out_cols (device int64)
 * and out_vals (device out_dtype) in no particular order; *count (device
 * int64, zeroed by the call) receives the number of hits.  When it exceeds
 * capacity only `capacity` of them (an arbitrary subset) are written.
 * The values are those cmm_extract gives, bit for bit. */
cmm_status cmm_extract_heavy(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                             int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                             double threshold, int64_t* out_rows, int64_t* out_cols,
                             void* out_vals, cmm_dtype out_dtype, int64_t capacity,
                             int64_t* count, void* stream);

/* Top-K heavy hitters: the k entries of largest |C_hat| over the dense
 * n_rows x n_cols block (Algorithm 1's Decompress at every entry, keeping
 * only the largest ones: the large entries of the product are what the
 * method is for, Section 1), without writing the dense C_hat.  out_rows,
 * out_cols (device int64[k]) and out_vals (device out_dtype[k]) receive them
 * sorted by |C_hat| descending, ties by the smaller row-major index
 * i * n_cols + j; the values are those cmm_extract gives, bit for bit (a NaN
 * estimate ranks above every number).  0 <= k <= n_rows * n_cols (k = 0 is a
 * no-op), k < 2^31 - 2^15; CMM_MEDIAN needs odd d <= 63.  An exact radix
 * selection on 12-bit digits of the key (|C_hat|, index), all on the device
 * with no host synchronisation: a few passes that evaluate the estimates
 * (two at the benchmark sizes, at most eight), one that collects at most
 * k + 16384 candidates, and a stable sort of those.  The workspace, from
 * cmm_topk_workspace_size, holds the selection state and the candidates;
 * the size query reads the current device's sort configuration, so it needs
 * a current device (CMM_EHIP otherwise). */
cmm_status cmm_topk_workspace_size(int64_t k, size_t* bytes);
cmm_status cmm_extract_topk(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                            int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                            int64_t k, int64_t* out_rows, int64_t* out_cols, void* out_vals,
                            cmm_dtype out_dtype, void* workspace, size_t workspace_bytes,
                            void* stream);

/* The d single-repetition estimates at a list of entries, before the median
 * or mean of Decompress (Algorithm 1):
 *   out[t][q] = s1_t(rows[q]) s2_t(cols[q]) p[t][h1_t(rows[q]) xor h2_t(cols[q])]
 * Each is unbiased with variance at most ||A B||_F^2 / b over the hash draw
 * (Section 3.1); the variance experiment of Section 5.3 samples them with
 * one independent draw per repetition.  rows, cols: device int64[count];
 * out: device out_dtype[d][count] (CMM_F64 or CMM_F32); NaN for an index
 * outside [0, n_rows) x [0, n_cols).  Any d in [1, 65535]. */
cmm_status cmm_extract_reps(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                            int64_t n_rows, int64_t n_cols, int log2b, const int64_t* rows,
                            const int64_t* cols, int64_t count, void* out, cmm_dtype out_dtype,
                            void* stream);

/* ------------------------------------------------------ evaluation counters */
/* The correctness counters of Section 5.4 for one estimate: with B the set
 * of big entries (big_rows / big_cols, device int64[n_big], distinct; an
 * entry outside the matrix is skipped) and S every other entry of the
 * n_rows x n_cols grid,
 *   counts[0] = #{(i,j) in B : |C_hat[i][j]| >= threshold}
 *   counts[1] = #{(i,j) in S : |C_hat[i][j]| <= threshold}
 *   counts[2] = #{(i,j) in B : |C_hat[i][j] - C[i][j]| <= tolerance}
 *   counts[3] = #{(i,j) in S : |C_hat[i][j] - C[i][j]| <= tolerance}
 * (the paper uses threshold 0.5 and tolerance 0.1).  C_hat: device
 * C_hat_dtype (CMM_F64 or CMM_F32), leading dimension ldh; C: the exact
 * product, device float64, leading dimension ldc.  counts: device int64[4],
 * overwritten.  A NaN estimate satisfies no condition.  Exact integers. */
cmm_status cmm_correctness_counts(const void* C_hat, cmm_dtype C_hat_dtype, int64_t ldh,
                                  const double* C, int64_t ldc, int64_t n_rows, int64_t n_cols,
                                  const int64_t* big_rows, const int64_t* big_cols, int64_t n_big,
                                  double threshold, double tolerance, int64_t* counts,
                                  void* stream);

/* ------------------------------------------------------ Pagh's FFT form */
/* Section 3.1: Pagh's original Compress sketches with h(i, j) = h1(i) + h2(j)
 * mod b and takes the cyclic convolution p_A * p_B through the discrete
 * Fourier transform; the FWHT form of Section 3.2 replaces both.  This form
 * is here to compare the two transforms on the same GPU.
 *
 * cmm_fft: batched complex float64 DFT of `batch` vectors of length
 * 2^log2n (1 <= log2n <= 24), interleaved (re, im), natural order:
 *   out[v][k] = scale * sum_n in[v][n] exp(-+ 2 pi i n k / 2^log2n)
 * (minus for inverse = 0, plus for inverse = 1).  in and out are device
 * buffers; they may be the same buffer only when log2n <= 12. */
cmm_status cmm_fft(const void* in, void* out, int64_t batch, int log2n, int inverse, double scale,
                   void* stream);

/* Decompress for the FFT form: C_hat[i][j] = Median_t s1 s2 p[t][(h1_t(i) +
 * h2_t(j)) mod b] (or the mean).  Arguments as for cmm_extract. */
cmm_status cmm_extract_cyclic(const double* p, const uint32_t* tab1, const uint32_t* tab2, int d,
                              int64_t n_rows, int64_t n_cols, int log2b, cmm_estimator estimator,
                              void* C_hat, cmm_dtype out_dtype, int64_t ldc, void* stream);

/* ------------------------------------------------------------- end to end */
/* One compressed product C_hat ~ A B (Algorithm 1 Compress + dense
 * Decompress).
 *   A: n_rows x n_inner (lda), B: n_inner x n_cols (ldb), both of in_dtype.
 *   compute: CMM_F64 -- sketches, transforms, accumulation in float64;
 *            CMM_F32 -- sketches and transforms in float32, products summed
 *                       in float32 per k-group, groups added in float64;
 *            CMM_BF16 / CMM_F16 -- precision form: sketches rounded to
 *                       bf16 / f16, transforms on the matrix cores (MFMA) with
 *                       float32 accumulation, cross-k accumulation and the
 *                       inverse transform in float64.  Needs log2b >= 14 and
 *                       n_rows, n_cols <= 16383 (else CMM_EUNSUPPORTED).
 *   in_dtype: CMM_F64 or CMM_F32 (CMM_F64 required when compute = CMM_F64).
 *   keys: device uint64[d][4][2] or NULL.  If non-NULL the tables are
 *         computed from the keys into tab1 / tab2 (outputs).  If NULL,
 *         tab1 / tab2 are read as given (explicit tables).
 *   p:    device float64[d][2^log2b] out (the compressed product returned
 *         by Compress), or NULL to keep it in the workspace only.
 *   C_hat: device out_dtype (CMM_F64 / CMM_F32) n_rows x n_cols (ldc), or
 *         NULL to run Compress only.
 * Requires n_rows, n_cols <= 2^32 and the workspace size reported by
 * cmm_workspace_size for the same problem, asked with the same device
 * current: the split of the inner dimension over work-groups follows the
 * device's compute-unit count, so the size can differ between devices.  A
 * workspace smaller than the plan at call time is rejected with
 * CMM_ENOMEM before anything is launched. */
typedef struct {
  int64_t n_rows, n_inner, n_cols;
  const void* A; int64_t lda;
  const void* B; int64_t ldb;
  cmm_dtype in_dtype;
  cmm_dtype compute;
  int d;
  int log2b;
  cmm_estimator estimator;
  const uint64_t* keys;
  uint32_t* tab1;
  uint32_t* tab2;
  double* p;
  void* C_hat; cmm_dtype out_dtype; int64_t ldc;
} cmm_problem;

cmm_status cmm_workspace_size(const cmm_problem* prob, size_t* bytes);
cmm_status cmm_estimate(const cmm_problem* prob, void* workspace, size_t workspace_bytes,
                        void* stream);

/* cmm_estimate without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same problem, outputs, kernels and results as
 * cmm_estimate; the scratch the workspace would hold comes from a static
 * device array of CMM_STATIC_SCRATCH_BYTES per device, so the call allocates
 * nothing (and creates no timing events: kernels run untimed even while
 * cmm_profile_enable is on).  A problem whose cmm_workspace_size exceeds
 * CMM_STATIC_SCRATCH_BYTES is rejected with CMM_EUNSUPPORTED before any
 * launch (about n <= 1024 at b = 16 n, d = 7 in float64).  Every call on
 * one device shares that device's array and finds the previous call's
 * contents in it (every kernel writes what it reads first): calls that
 * overlap in time on one device, on any streams or threads, race and must be
 * serialised by the caller.  The array is taken from the device current at
 * the call. */
#define CMM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
cmm_status cmm_estimate_static(const cmm_problem* prob, void* stream);

/* Pagh's FFT form end to end (Section 3.1): the same problem description,
 * float64 only (compute and in_dtype CMM_F64, else CMM_EUNSUPPORTED); p
 * receives the cyclic sketch and C_hat the cyclic Decompress.  Composed of
 * count sketches, one complex transform per (t, k) of p_A + i p_B, the
 * products accumulated in the transform domain, and one inverse transform
 * per repetition.  Workspace from cmm_fft_workspace_size. */
cmm_status cmm_fft_workspace_size(const cmm_problem* prob, size_t* bytes);
cmm_status cmm_estimate_fft(const cmm_problem* prob, void* workspace, size_t workspace_bytes,
                            void* stream);

/* ---------------------------------------------------------- batched form */
/* Many independent problems (Algorithm 1 each, uneven sizes) with all their
 * Compress work in ONE persistent kernel launch: work-groups take work items
 * (problem, repetition, slice of the transform, range of k) from a queue.
 * The rest of each problem (tables, operand copies, plans, sums of partials,
 * inverse transform, extract) is enqueued per problem around it; nothing in
 * cmm_estimate_batched allocates or synchronises, so the whole call can be
 * captured into a HIP graph and replayed.
 *   cmm_batch_create: plans a batch of `count` problems (each as for
 *     cmm_estimate; compute CMM_F64 or CMM_F32, the same for all; log2b >= 11;
 *     n_rows, n_cols <= 65534).  The problems' pointers are kept and used by
 *     every later call: the buffers must stay valid while the batch exists.
 *     Needs a device (pinned host memory holds the work-item table).
 *   cmm_batch_workspace_size: bytes of workspace (valid for every launch
 *     configuration, so autotuning never needs more); the workspace must be
 *     256-byte aligned.
 *   cmm_batch_autotune: a project-written tuner.  Times the persistent
 *     launch over candidate configurations -- tile b_lo = 2^11..2^13, radix
 *     (16 elements per thread, b_lo = 2^13, or 32), inner indices per work
 *     item 32..256, one or two work-groups per compute unit (LDS share),
 *     item order (largest problems first / round robin) -- by coordinate
 *     descent from the default, and keeps the fastest.  Results
 *     are cached per device and batch signature for the process, and in the
 *     file named by the environment variable CMM_TUNE_CACHE when set (read,
 *     then appended).  Synchronises the stream; not for use under capture.
 *   cmm_batch_set_config / cmm_batch_get_config: choose or read the
 *     configuration (source: 0 default, 1 tuned, 2 from the cache, 3 set).
 *     Graphs captured earlier keep the configuration they were captured with.
 *   cmm_estimate_batched: one estimate of every problem (outputs as for
 *     cmm_estimate). */
typedef struct cmm_batch cmm_batch;
cmm_status cmm_batch_create(const cmm_problem* probs, int count, cmm_batch** batch);
cmm_status cmm_batch_destroy(cmm_batch* batch);
cmm_status cmm_batch_workspace_size(const cmm_batch* batch, size_t* bytes);
cmm_status cmm_batch_autotune(cmm_batch* batch, void* workspace, size_t workspace_bytes,
                              void* stream);
cmm_status cmm_batch_set_config(cmm_batch* batch, int log2_blo, int k_per_item, int wg_per_cu,
                                int order, int radix);
cmm_status cmm_batch_get_config(const cmm_batch* batch, int* log2_blo, int* k_per_item,
                                int* wg_per_cu, int* order, int* radix, int* source);
cmm_status cmm_estimate_batched(cmm_batch* batch, void* workspace, size_t workspace_bytes,
                                void* stream);

/* ------------------------------------------------------ differentiation */
/* Gradient of L = sum_ij W[i][j] C_hat[i][j] for the mean-over-d estimator
 * C_hat = (1/d) sum_t L_t(A B) of the same problem (Section 3.1: each
 * repetition is an unbiased linear estimate; L_t(C)[i][j] is
 * s1(i) s2(j) times the bucket sum of C at h1(i) xor h2(j), which Algorithm 1
 * computes through the transforms of Section 3.2):
 *   dA = dL/dA  (n_rows x n_inner, leading dimension ldda)
 *   dB = dL/dB  (n_inner x n_cols, leading dimension lddb)
 * by the adjoint of every step of the forward pass (bucket sums of W, the
 * transforms, the pointwise products, the transposed count sketch), with the
 * same tables as the forward call.
 *   prob: as for cmm_estimate, with estimator = CMM_MEAN and compute CMM_F64 or
 *         CMM_F32 (else CMM_EUNSUPPORTED); keys NULL to read tab1 / tab2, or the
 *         forward's keys (the tables are then recomputed, identically);
 *         p, C_hat are ignored.  Needs log2b >= 11 and n_rows, n_cols <= 65534.
 *   W: n_rows x n_cols (ldw) of in_dtype; dA, dB of in_dtype, overwritten.
 * The workspace size comes from cmm_backward_workspace_size.  With compute =
 * CMM_F32 the transforms run in float32 and the sums over repetitions and
 * slices in float64; the bucket sums of W are float64 (their order of
 * addition within a block is not fixed). */
cmm_status cmm_backward_workspace_size(const cmm_problem* prob, size_t* bytes);
cmm_status cmm_estimate_backward(const cmm_problem* prob, const void* W, int64_t ldw, void* dA,
                                 int64_t ldda, void* dB, int64_t lddb, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------- kernel timing */
/* Tracing for measurement: while enabled, every launch of the library is
 * bracketed by two HIP events recorded on the caller's stream, and
 * cmm_profile_query returns the summed elapsed time and the number of
 * launches of one kernel ("hash", "transpose", "plan", "compress",
 * "reduce", "fwht", "extract", "sketch", "accumulate", "wscatter",
 * "adjoint", "adjoint_reduce", "extract_entries", "extract_heavy",
 * "extract_reps", "extract_topk", "correctness", "fft", "pairs") since the last
 * cmm_profile_enable call.  Enabling or disabling discards the records.
 * query waits for the recorded events.  Off by default.
 *
 * Each event record delays the stream's next launch by a few microseconds.
 * cmm_profile_only(kernel) brackets only the launches of that kernel (one of
 * the names above; NULL brackets every kernel again, the default), so that a
 * timed loop pays for two events per launch of the kernel it measures and
 * no others.  It discards the records; an unknown name returns CMM_EINVAL
 * and leaves the setting as it was.  The setting is process-wide. */
void cmm_profile_enable(int on);
cmm_status cmm_profile_only(const char* kernel);
cmm_status cmm_profile_query(const char* kernel, double* total_ms, int* launches);

/* ------------------------------------------------------ gather probe */
/* A measurement aid, not a step of the method.  Decompress (Algorithm 1)
 * reads p at h1(i) XOR h2(j) for every entry and repetition: d n_rows n_cols
 * random 8-byte gathers over the d 2^log2b values of p, whose rate, not HBM
 * bandwidth, bounds the dense extract.  cmm_gather_probe issues at least
 * `gathers` such gathers, at positions drawn uniformly (a hash of a counter
 * and `seed`) from table[0, len), so that the extract's gather rate can be
 * set against what the memory hierarchy gives at the same footprint.
 *   table   device, len float64 values (read only; the caller's, e.g. p)
 *   len     in [1, 2^32]
 *   gathers in [1, 2^40]; rounded up to whole work-groups of 16384
 *   sink    device, one float64; written only if the gathered values sum to
 *           one fixed value (it keeps the loads live)
 *   issued  host, may be NULL: receives the number of gathers issued
 * Launches one kernel on `stream` and returns; CMM_EINVAL for a null table
 * or sink or a size out of range. */
cmm_status cmm_gather_probe(const double* table, int64_t len, int64_t gathers, uint32_t seed,
                            double* sink, int64_t* issued, void* stream);

/* ---------------------------------------------------------------- status */
const char* cmm_status_string(cmm_status s);
const char* cmm_last_error(void);
/* 2 since cmm_sketch takes out_dtype. */
int cmm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CMM_H */
