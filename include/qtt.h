/*
 * qtt.h -- C ABI of the MI355X QTT denoising-convolution library.
 *
 * The library implements the hot path of Chertock, Leonard, Tsynkov and
 * Utyuzhnikov, "Denoising Convolution Algorithms and Applications to SAR
 * Signal Processing" (arXiv 2301.13339): decomposition of a 2^d-sample signal
 * or image into quantized tensor-train (QTT) cores by TT-SVD with truncation
 * at a tolerance (Algorithm 1, with the max-rank modification (1) of
 * Section 5), an exact convolution with a sinc kernel (GAF (3.1), kernels
 * (7.2)/(7.3), discrete convolution (2.2)) carried out in QTT format,
 * TT-rounding of the result, and reconstruction of the full array
 * (Algorithm 3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  * All array arguments are DEVICE pointers (HIP global memory) owned by the
 *    caller unless stated otherwise.  The library never allocates device
 *    memory; every call takes a caller-owned workspace `ws` of `ws_bytes`
 *    bytes whose required size is returned by the matching qtt_query_* call.
 *  * Every call is asynchronous on `stream` (0 = the default stream) and
 *    performs no host/device synchronisation.  Ranks that depend on the data
 *    live in device memory (`qtt_tensor.ranks`); the host only knows their
 *    capacities.
 *  * QTT index map (Section 4): a vector v of length 2^d is the d-mode tensor
 *    V(i_1..i_d) = v(i), i = sum_k i_k 2^(k-1); i_1 is the least significant
 *    bit.  A row-major 2^dy x 2^dx image is its flattened row-major vector,
 *    so modes 1..dx are the column bits and modes dx+1..dx+dy the row bits.
 *  * Core k (k = 1..d) has shape (r_{k-1}, 2, r_k), r_0 = r_d = 1, stored
 *    C-contiguously with the ACTUAL ranks: entry (a, i, b) at element offset
 *    off_k + (a*2 + i)*r_k + b, where off_k = sum_{j<k} cap_j * 2 * cap_{j+1}
 *    is fixed by the host-side capacities (0-based arrays below).
 *  * Return value: QTT_OK (0) or a negative error code (see below).  Codes
 *    are returned synchronously, before anything is enqueued, for invalid
 *    arguments and undersized workspaces.  Conditions found on the device
 *    (non-finite input, a rank limited by a capacity) are OR-ed into the
 *    tensor's `status` word, which the caller reads after synchronising.
 *  * No C++ exception crosses this boundary.  The library keeps no pointer
 *    after a call returns.  Concurrent calls on different streams must use
 *    different workspaces and output tensors.
 */
#ifndef QTT_H
#define QTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define QTT_OK 0
#define QTT_EINVAL (-1)   /* invalid argument                                  */
#define QTT_ENOSPC (-2)   /* workspace or tensor capacity too small            */
#define QTT_ENOTSUP (-3)  /* valid but unsupported size or option              */
#define QTT_EHIP (-4)     /* a HIP runtime call failed (see qtt_last_hip_error) */

/* device status bits (OR-ed into *status) */
#define QTT_STATUS_NONFINITE 1  /* the input held NaN or Inf                    */
#define QTT_STATUS_RANKCAP 2    /* an eps-rank exceeded the rank capacity       */
#define QTT_STATUS_FFT_RANK 4   /* a QTT-FFT input rank above QTT_FFT_MAX_RANK  */

/* element types */
#define QTT_F32 0
#define QTT_F64 1
#define QTT_C128 2  /* complex, FP64 (re, im) pairs; QTT-FFT tensors only */

/* rounding methods for qtt_round */
#define QTT_ROUND_EXACT 0       /* TT-SVD of the represented tensor, FP64 sums  */
#define QTT_ROUND_SKETCH_F32 1  /* randomized range finder, FP32 sketch GEMM    */
#define QTT_ROUND_SKETCH_BF16 2 /* randomized range finder, BF16-operand sketch */

#define QTT_SKETCH_ELL 32       /* sketch width of qtt_round's sketch methods   */
#define QTT_SKETCH_MAX_ELL 64   /* largest sketch width                         */
#define QTT_MAXD 48             /* largest number of binary modes               */
#define QTT_MAX_RANK 64         /* largest TT-rank a decomposition can produce  */

/*
 * A QTT tensor.  `d`, `dtype` and `cap` are host values written by the
 * caller (normally copied from a qtt_query_* result); `ranks`, `cores` and
 * `status` point to device memory of at least (d+1) int32, qtt_core_elems()
 * elements of `dtype`, and one int32.  Producers write `ranks` (r_0..r_d) and
 * the cores; `status` may be NULL, in which case device conditions are
 * dropped.
 */
typedef struct {
  int32_t d;
  int32_t dtype;
  int32_t cap[QTT_MAXD + 1];
  int32_t* ranks;
  void* cores;
  int32_t* status;
} qtt_tensor;

/* Number of core elements for the capacities cap[0..d]. */
size_t qtt_core_elems(int d, const int32_t* cap);

/* Text for an error code or status bit set (static storage). */
const char* qtt_strerror(int code);

/* Text of the last HIP error seen by the calling thread ("" if none). */
const char* qtt_last_hip_error(void);

/* ------------------------------------------------------------- decompose */
/*
 * Sizes for qtt_decompose / qtt_kernel_sinc.
 *   d         number of modes of the decomposed tensor (N = 2^d samples)
 *   max_rank  rank cap R of modification (1); 0 = no cap.  The effective cap
 *             is min(R, QTT_MAX_RANK); an eps-rank above it is truncated and
 *             flagged with QTT_STATUS_RANKCAP.
 *   dtype     element type of the data and of the cores
 * Outputs (any may be NULL): cap[0..d] = min(2^k, 2^(d-k), effective cap)
 * with cap[0] = cap[d] = 1, the workspace size and the core element count.
 */
int qtt_query_decompose(int d, int max_rank, int dtype, int32_t* cap, size_t* ws_bytes,
                        size_t* core_elems);

/*
 * TT-SVD of a vector (Algorithm 1 with modification (1); Lemma 5.1 shapes).
 *   x         device, 2^d elements of `dtype`, read only
 *   eps       relative tolerance >= 0: each unfolding k is truncated to the
 *             smallest rank r >= 1 whose discarded tail satisfies
 *             sum_{i>r} sigma_i^2 <= tau^2, tau = eps*||x||_F/sqrt(d-1), then
 *             to min(r, cap_k)
 *   max_rank  as in qtt_query_decompose
 *   out       tensor with out->d == d, out->dtype == dtype and capacities at
 *             least those returned by qtt_query_decompose
 *   sv        optional device buffer (NULL to skip) of (d-1)*2*QTT_MAX_RANK
 *             doubles: row k-1 receives the singular values of unfolding k in
 *             non-increasing order, zero padded
 * Singular values and vectors come from FP64 Gram sums of the unfoldings
 * (wavefront-shuffle reductions) and a one-workgroup FP64 symmetric
 * eigensolver (Householder tridiagonalisation, multisection, twisted
 * factorisation), whatever `dtype` is.
 */
int qtt_decompose(const void* x, int d, int dtype, double eps, int max_rank, qtt_tensor* out,
                  double* sv, void* ws, size_t ws_bytes, void* stream);

/*
 * TT-SVD with the singular-value drop-off rule, modification (3) of Section 5
 * ("SV drop off TT-SVD"), on top of the tolerance rule and the cap of
 * qtt_decompose.  With s the singular values of unfolding k (non-increasing),
 * the drop-off rank is the smallest j >= 1 with s_{j+1} < delta * s_j (the
 * first relative drop below delta cuts every later value; two zero values
 * are not a drop); the kept rank is min(eps-rank, drop-off rank, cap_k), or
 * min(eps-rank, cap_k) when no ratio falls below delta.  eps = 0 and
 * max_rank = 0 give the drop-off rule alone; delta = 0 is qtt_decompose.
 * The ratios come from the FP64 Gram eigenvalues (s^2), so a decision on
 * singular values below about 1e-7 of the largest is not reliable.
 *   delta     threshold, 0 <= delta < 1 (else QTT_EINVAL)
 * Everything else (sizes, workspace, outputs, errors) as qtt_decompose;
 * QTT_STATUS_RANKCAP is set only when the cap, not the drop-off, decided.
 */
int qtt_decompose_dropoff(const void* x, int d, int dtype, double eps, double delta, int max_rank,
                          qtt_tensor* out, double* sv, void* ws, size_t ws_bytes, void* stream);

/*
 * TT-SVD and max-rank TT-RSVD of a tensor with K modes of size M (Section 5,
 * modifications (1) and (2); Algorithms 1, 4 and 5), FP64.  The tensor is the
 * vector x of M^K entries with index i = i_1 + M (i_2 + M (...)); step k
 * unfolds the remainder column-major into m_k = M r_{k-1} rows and
 * n_k = M^(K-k) columns.
 *   K, M        modes (1 <= K <= QTT_MAXD) and mode size (2..64), M^K <= 2^31
 *   max_rank    rank cap R (0 = QTT_MAX_RANK); the effective cap is lowered
 *               to 128 / M so that every unfolding has at most 128 rows
 *   method      0: exact truncated SVDs (Gram matrix and the FP64
 *               eigensolver); 1: max-rank TT-RSVD, the step's SVD taken by
 *               the range finder with ell = R + oversample columns
 *               (R + oversample <= 64, max_rank > 0), reverting to the exact
 *               step where min(M cap_{k-1}, n_k) <= ell
 *   seed        Omega[row][col] of step k is the standard normal of
 *               Philox-4x32-10 with counter (row, col, k, 0) and key
 *               (seed mod 2^32, seed >> 32), Box-Muller of its first two words
 * Outputs (query): cap[0..K] = min(M^k, M^(K-k), effective cap), the
 * workspace size and the number of core elements.
 * Call: x (device, read only); cap = the query's capacities; ranks (device,
 * K+1 int32) receives r_0..r_K; cores (device) receives core k (1-based) as
 * C-contiguous (r_{k-1}, M, r_k) with the actual ranks, at element offset
 * sum_{j<k} cap[j-1] M cap[j].  The rank of step k is Algorithm 1's rule at
 * eps (tau = eps ||x|| / sqrt(K-1)) on the step's singular values, then the
 * cap.  status (device int32, may be NULL) receives, OR-ed in,
 * QTT_STATUS_RANKCAP when an eps-rank exceeded a cap that the library's
 * capacity (128 / M, at most QTT_MAX_RANK) set below the caller's max_rank
 * (or with max_rank = 0), and QTT_STATUS_NONFINITE for non-finite input.
 * Errors: QTT_EINVAL for invalid arguments or capacities other than the
 * query's, QTT_ENOSPC for a short workspace.
 */
int qtt_query_decompose_modes(int K, int M, int max_rank, int method, int oversample,
                              int32_t* cap, size_t* ws_bytes, size_t* core_elems);
int qtt_decompose_modes(const double* x, int K, int M, double eps, int max_rank, int method,
                        int oversample, uint64_t seed, const int32_t* cap, int32_t* ranks,
                        double* cores, int32_t* status, void* ws, size_t ws_bytes,
                        void* stream);

/*
 * QTT of the Toeplitz generator of the normalised sinc kernel.
 * For N = 2^d the kernel is g_m = sinc(B x_m)/Z on x_m = -1/2 + m/N
 * (sinc(t) = sin(pi t)/(pi t), kernel (7.2) with B = 1/Delta_x and Z the
 * midpoint sum dx*sum_m sinc(B x_m)); the generator w has 2N entries,
 * w_u = dx*g_{u-N/2} for N/2 <= u < 3N/2 and 0 otherwise, so that (2.2) is
 * y_j = sum_i w_{j-i+N} f_i.  The samples are computed on the device (no
 * input array) and decomposed like qtt_decompose on d+1 modes at tolerance
 * eps_w, uncapped (up to QTT_MAX_RANK).
 *   w_out     tensor with d+1 modes and capacities from
 *             qtt_query_decompose(d+1, 0, dtype, ...)
 */
int qtt_kernel_sinc(int d, double B, double eps_w, int dtype, qtt_tensor* w_out, void* ws,
                    size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ conv */
/*
 * Sizes for qtt_conv.  `f_cap` are the capacities of the signal (d modes),
 * `w_caps[a]` those of the kernel generator of axis a (d_a + 1 modes, axes
 * ordered column axis first), n_axes = 1 (signal) or 2 (image, d = d_0 + d_1).
 * Returns the output capacities y_cap[0..d] (y_cap[k] = 2*capW*capF inside an
 * axis, capF at an axis boundary) and the sizes.
 */
int qtt_query_conv(int d, int n_axes, const int32_t* axis_modes, const int32_t* f_cap,
                   const int32_t* const* w_caps, int dtype, int32_t* y_cap, size_t* ws_bytes,
                   size_t* core_elems);

/*
 * Exact convolution (2.2) in QTT format: y = T(w) f with T(j,i) = w_{j-i+N}
 * per axis.  The index u = j + (N-1-i) + 1 is a binary addition with carry,
 * so each mode of the Toeplitz operator is a QTT-matrix core whose bond is
 * (kernel bond, carry bit); the output cores are the mode-wise products with
 * the signal cores (bond 2*rho_k*r_k).  No truncation.
 *   f         signal tensor (d modes)
 *   w         array of n_axes kernel tensors, w[a] with axis_modes[a]+1 modes
 *   y         output tensor with capacities from qtt_query_conv
 */
int qtt_conv(const qtt_tensor* f, const qtt_tensor* w, int n_axes, const int32_t* axis_modes,
             qtt_tensor* y, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------- round */
/*
 * Sizes for qtt_round of a tensor with capacities y_cap into a tensor with
 * capacities z_cap = qtt_query_decompose(d, max_rank, ...).
 */
int qtt_query_round(int d, const int32_t* y_cap, int max_rank, int dtype, int method,
                    int32_t* z_cap, size_t* ws_bytes, size_t* core_elems);

/*
 * TT-rounding of y at tolerance eps (the paper gives no rounding algorithm;
 * TT-rounding of an exact TT returns the TT-SVD of the tensor it represents).
 *   method QTT_ROUND_EXACT: the result is the TT-SVD (Algorithm 1, same
 *          truncation rule and threshold with ||y||_F) of the represented
 *          tensor; it is computed by reconstructing the tensor into the
 *          workspace (Algorithm 3) and running the qtt_decompose sweep.
 *   method QTT_ROUND_SKETCH_F32 / _BF16: the same sweep with every
 *          truncated SVD taken by Algorithms 4 and 5 (qtt_round_sketch with
 *          ell = QTT_SKETCH_ELL and the given seed).
 *   z      output tensor with capacities from qtt_query_round
 */
int qtt_round(const qtt_tensor* y, double eps, int max_rank, int method, uint64_t seed,
              qtt_tensor* z, void* ws, size_t ws_bytes, void* stream);

/* Capacities and workspace of qtt_round_sketch (2 <= ell <= QTT_SKETCH_MAX_ELL: the first
 * unfolding has two rows, so its step is exact and gives the norm). */
int qtt_query_round_sketch(int d, const int32_t* y_cap, int max_rank, int dtype, int ell,
                           int32_t* z_cap, size_t* ws_bytes, size_t* core_elems);

/*
 * Randomised rounding (Algorithms 4 and 5 of Appendix A inside the TT-SVD
 * sweep of the represented tensor): at every step whose unfolding A (m x n)
 * has more rows than the sketch width (m > ell), Y = A Omega (m x ell,
 * Omega Gaussian from Philox-4x32-10, counter (row, col, step, 0), key =
 * seed, Box-Muller of the first two words), Q = qr(Y) and B = Q^T A give the
 * truncated SVD through the eigendecomposition of B B^T, whose rank follows
 * the rule of Algorithm 1 at eps (cap max_rank); the next remainder is
 * U^T A with U = Q U~.  The range-finder product Y = A Omega runs on the
 * matrix cores with single-precision operands (bf16 = 0,
 * v_mfma_f32_16x16x4f32) or operands rounded to bfloat16 (bf16 = 1,
 * v_mfma_f32_16x16x32_bf16); B = Q^T A and B B^T run on the FP32 matrix
 * cores with single-precision operands; all accumulate in FP32 with an FP64
 * combine of the partial sums; QR, the small eigenproblem and the
 * projection stay in FP64.  No Gram of A is formed on these steps.
 * A step with ell >= m is the exact SVD (FP64 Gram).  qtt_round's
 * QTT_ROUND_SKETCH_* methods are this call with ell = QTT_SKETCH_ELL.
 */
int qtt_round_sketch(const qtt_tensor* y, double eps, int max_rank, int ell, int bf16,
                     uint64_t seed, qtt_tensor* z, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ full */
/* Workspace for qtt_full of a tensor with capacities cap[0..d]. */
int qtt_query_full(int d, const int32_t* cap, int dtype, size_t* ws_bytes);

/*
 * Full (Algorithm 3): out[i] = G_1[:, i_1, :] ... G_d[:, i_d, :] for all
 * i < 2^d, written as 2^d elements of t->dtype.  Computed as two half
 * chains (left and right interface matrices) and one tiled product.
 */
int qtt_full(const qtt_tensor* t, void* out, void* ws, size_t ws_bytes, void* stream);

/*
 * qtt_full without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc).  Same result as qtt_full (the same kernels); the interface
 * matrices of the two half chains live in a fixed device array of the
 * library, QTT_NOALLOC_SCRATCH_MIB MiB per device, held until the process
 * ends.  Nothing is allocated or freed by the call.
 *   t, out    as qtt_full
 * Errors: as qtt_full; QTT_ENOSPC when the interface matrices need more than
 * the array (qtt_query_full's workspace size above QTT_NOALLOC_SCRATCH_MIB
 * MiB).  Every call on one device shares that device's array, so calls that
 * overlap in time on one device (different streams or host threads without
 * ordering) race and must be serialised by the caller.
 */
#define QTT_NOALLOC_SCRATCH_MIB 32
int qtt_full_noalloc(const qtt_tensor* t, void* out, void* stream);

/* --------------------------------------------------------------- adjoint */
/*
 * Building blocks of the backward of y = T(w) full(F) (the convolution (2.2)
 * of the reconstruction of Algorithm 3 with the kernel generator w), at fixed
 * ranks.  The paper gives no derivative; these follow from the chain rule.
 */

/* Workspace of qtt_toeplitz_apply for a signal of d modes and a generator
 * with capacities w_cap[0..d+1]. */
int qtt_query_toeplitz(int d, const int32_t* w_cap, int dtype, size_t* ws_bytes);

/*
 * Toeplitz product on full vectors of N = 2^(w->d - 1) elements (w->dtype):
 *   transpose = 0:  y_j = sum_i w_{j-i+N} x_i      (y = T(w) x, eq. (2.2))
 *   transpose = 1:  y_i = sum_j w_{j-i+N} x_j      (y = T(w)^T x, its adjoint)
 * with w the QTT generator (d+1 modes, e.g. from qtt_kernel_sinc).  The
 * operator is applied in its QTT-matrix form (the binary adder of qtt_conv)
 * one mode per pass, so the cost is O(N d rho^2) for generator ranks rho.
 * x and y are device arrays that must not overlap; ws holds two FP64 states
 * of 2 max_k(w_cap[k]) N doubles (size from qtt_query_toeplitz): the
 * intermediate sums stay in FP64 whatever the dtype.
 * Errors: QTT_EINVAL (null pointers, w with fewer than 2 modes, a transpose
 * flag other than 0/1, capacities above QTT_MAX_RANK), QTT_ENOSPC.
 */
int qtt_toeplitz_apply(const qtt_tensor* w, const void* x, void* y, int transpose, void* ws,
                       size_t ws_bytes, void* stream);

/* Capacities (d+2 entries) and workspace for qtt_kernel_sinc_dB. */
int qtt_query_kernel_sinc_dB(int d, int dtype, int32_t* cap, size_t* ws_bytes,
                             size_t* core_elems);

/*
 * QTT (d+1 modes, uncapped, tolerance eps_w) of the derivative with respect
 * to the bandwidth B of the normalised generator of qtt_kernel_sinc:
 *   dw_u/dB = s'_m / S - s_m S' / S^2,  s_m = sinc(B x_m),
 *   s'_m = (cos(pi B x_m) - s_m) / B  (0 at x_m = 0),  S = sum s, S' = sum s'
 * (kernel (3.1) normalised as in (7.2) by the discrete sum).  S and S' are
 * summed on the device; the samples are generated on the fly.
 */
int qtt_kernel_sinc_dB(int d, double B, double eps_w, int dtype, qtt_tensor* w_out, void* ws,
                       size_t ws_bytes, void* stream);

/* Workspace of qtt_full_adjoint (capacities of F, each <= QTT_MAX_RANK). */
int qtt_query_full_adjoint(int d, const int32_t* cap, int dtype, size_t* ws_bytes);

/*
 * Adjoint of qtt_full: grad->cores[k] = d<g, full(f)>/d f_k for every core,
 * at the ranks of f (written to grad->ranks).  g: 2^d elements of f->dtype.
 * grad must have f's d, dtype and capacities.  The right interface matrices
 * of f are recomputed, and g is contracted from the left mode by mode;
 * every sum runs in FP64 in a fixed order (bit-reproducible).
 */
int qtt_full_adjoint(const qtt_tensor* f, const void* g, qtt_tensor* grad, void* ws,
                     size_t ws_bytes, void* stream);

/*
 * Workspace of qtt_conv_full_backward (wdb_cap may be NULL; want_w = 1 when
 * the kernel-core gradient grad_w will be asked for).  With want_w the
 * workspace holds the d forward-product states Q_1..Q_d of
 * 2 w_cap[k] 2^d doubles each, so pass a generator whose capacities equal
 * its ranks (about 14 GB at d = 22 and ranks near 10).
 */
int qtt_query_conv_full_backward(int d, const int32_t* f_cap, const int32_t* w_cap,
                                 const int32_t* wdb_cap, int want_w, int dtype,
                                 size_t* ws_bytes);

/*
 * Backward of y = T(w) full(f) = full(qtt_conv(f, w)) for an upstream
 * gradient grad_y = dL/dy (2^d elements), at the ranks of f and w:
 *   grad_f  = qtt_full_adjoint(f, T(w)^T grad_y)  (every signal core);
 *   grad_w  (optional, NULL to skip; w's d, dtype and capacities): the
 *             gradient with respect to every core of the generator QTT w
 *             (d+1 modes).  Core k contracts the state of the transposed
 *             product before mode k (grad_y pushed through modes 1..k-1 of
 *             T(w)^T) with the state of the forward product after it (full(f)
 *             pushed through modes k+1..d of T(w) from the top), through the
 *             carry structure of the binary adder of mode k; ranks copied
 *             from w;
 *   *grad_B  (one device double, with w_dB from qtt_kernel_sinc_dB) =
 *             <grad_y, T(w_dB) full(f)>.
 * full(f) is recomputed, not taken from the forward; every sum is FP64 in a
 * fixed order.  w_dB and grad_B are both NULL or both non-NULL.  The paper
 * gives no derivative: these follow from the chain rule applied to the
 * convolution (2.2) and Algorithm 3.
 */
int qtt_conv_full_backward(const qtt_tensor* f, const qtt_tensor* w, const qtt_tensor* w_dB,
                           const void* grad_y, qtt_tensor* grad_f, qtt_tensor* grad_w,
                           double* grad_B, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- batched */
/*
 * Many independent lines (e.g. SAR range lines) through the whole pipeline
 * of qtt_decompose / qtt_kernel_sinc / exact convolution / rounding /
 * qtt_full, each line with its own length 2^d[l] and bandwidth B[l], in a
 * handful of launches over the whole batch that qtt_batch_run can capture
 * in one hipGraph (replayed by later calls with the same pointers).
 * Per line the result equals the single-signal pipeline with the same
 * parameters: signal TT-SVD at eps with rank cap max_rank, kernel QTT at
 * eps_w (rank cap w_max_rank, 0 = 16), y = T(w) full(F) exactly, rounding =
 * TT-SVD of y at eps (cap round_max_rank, 0 = QTT_MAX_RANK), out = full.
 */
#define QTT_BATCH_MAXD 18       /* largest d of a line in a batch               */

typedef struct qtt_batch qtt_batch;  /* host-side plan (line tables, graph) */

/*
 * Plan a batch: d[l] (1..QTT_BATCH_MAXD) and B[l] > 0 are host arrays of
 * n_lines entries.  The lines are stored back to back (line l at offset
 * sum_{j<l} 2^d[j]) in x and out.  *ws_bytes receives the workspace size
 * (tables, cores, ranks, full vectors, the Toeplitz state of
 * 2 w_max_rank 2^d[l] elements per line and per-workgroup scratch).  The
 * plan is host memory owned by the library; free it with qtt_batch_destroy.
 * Errors: QTT_EINVAL (bad sizes, eps, ranks or bandwidths), QTT_ENOTSUP
 * (w_max_rank above 24).
 */
int qtt_batch_create(int n_lines, const int32_t* d, const double* B, int dtype, double eps,
                     int max_rank, double eps_w, int w_max_rank, int round_max_rank,
                     qtt_batch** plan, size_t* ws_bytes);

int qtt_batch_destroy(qtt_batch* plan);

/*
 * Run the batch: x (input samples) and out (results) are device arrays of
 * sum 2^d[l] elements of the plan's dtype; ws is the workspace.  The first
 * call tunes the chunk width of the Toeplitz stage by timing the candidates
 * (it synchronises the stream once) and uploads the line tables into ws;
 * with use_graph = 1 the stage launches are captured in a hipGraph on the
 * first call for these pointers and replayed afterwards.  Per-line status
 * words (non-finite input, rank capacity reached) are in the workspace (see
 * qtt_batch_status_offset): 3 per line (signal, kernel, rounding).
 */
int qtt_batch_run(qtt_batch* plan, const void* x, void* out, void* ws, size_t ws_bytes,
                  int use_graph, void* stream);

/*
 * Where line `line`'s tensors live in the workspace: which = 0 signal cores
 * F, 1 kernel cores W (d+1 modes), 2 rounded cores Z.  Byte offsets of its
 * int32 ranks (d+1 or d+2 entries) and of its capacity-strided cores, the
 * rank cap of that family and the element offset of the line's samples.
 */
int qtt_batch_info(const qtt_batch* plan, int line, int which, int64_t* rank_off_bytes,
                   int64_t* core_off_bytes, int32_t* rank_cap, int64_t* sample_off);

/* Byte offset of the 3 x n_lines status words and the tuned chunk width. */
int qtt_batch_status_offset(const qtt_batch* plan, int64_t* status_off_bytes,
                            int32_t* chunk_bits);

/* ------------------------------------------------------------ measurement */
/* ------------------------------------------------------------- QTT-FFT */
#define QTT_FFT_MAX_RANK 16  /* largest rank into and out of a QTT-FFT          */
#define QTT_FFT_MAX_ELL 32   /* largest sketch width R^_max + p of qtt_conv_fft  */

/*
 * Sizes for qtt_fft.  Outputs (either may be NULL): cap[0..d] =
 * min(2^k, 2^(d-k), max_rank or QTT_FFT_MAX_RANK), the capacities the output
 * tensor needs, and the workspace size.
 */
int qtt_query_fft(int d, int max_rank, int32_t* cap, size_t* ws_bytes);

/*
 * QTT-FFT (Section 4; the truncated transform of Section 5): the DFT
 * X(b) = sum_a x(a) exp(-2 pi i a b / 2^d) of a complex QTT tensor, computed
 * in QTT format as the d radix-2 decimation-in-frequency stages (stage s sums
 * over digit a_m, m = d + 1 - s, and doubles bonds 1..m-1), each followed by
 * the rounding of the doubled bonds: Householder QR from the left, then
 * one-sided Jacobi SVDs from core m down to core 2, truncated to
 * min(r_eps, r_drop, cap) as in Algorithm 1 with modifications (1) and (3),
 * tau = eps ||Y_s|| / sqrt(d-1).  The output is in BIT-REVERSED mode order:
 * mode p of y holds digit b_(d+1-p).
 * inverse != 0: QTT-iFFT, x(a) = 2^-d sum_b X(b) exp(+2 pi i a b / 2^d), with
 * the input in the bit-reversed order a forward transform returns and the
 * output in natural order.
 *   x         complex tensor (dtype QTT_C128); its actual ranks must not exceed
 *             QTT_FFT_MAX_RANK, otherwise the output is the zero tensor and
 *             QTT_STATUS_FFT_RANK is set in y->status
 *   eps       tolerance of each rounding (0 = off); delta: drop-off threshold
 *             in [0, 1) (0 = off); max_rank: cap R^_max in 0..QTT_FFT_MAX_RANK
 *             (0 = QTT_FFT_MAX_RANK, with QTT_STATUS_RANKCAP set when the
 *             tolerance or drop-off rank exceeded it)
 *   y         complex tensor, d modes, capacities from qtt_query_fft
 * All arithmetic is FP64.  Errors: QTT_EINVAL (arguments, d > 31),
 * QTT_ENOSPC (y or workspace).
 */
int qtt_fft(const qtt_tensor* x, int inverse, double eps, int max_rank, double delta,
            qtt_tensor* y, void* ws, size_t ws_bytes, void* stream);

/*
 * Sizes for qtt_conv_fft (arguments as there): y_cap[0..d] = 2 R^ bounded
 * by the bond's full rank, 1 at the ends, and the workspace size.  Requires
 * 1 <= max_rank_hat <= QTT_FFT_MAX_RANK, max_rank_hat + oversample <=
 * QTT_FFT_MAX_ELL and d + n_axes <= 31.
 */
int qtt_query_conv_fft(int d, int n_axes, const int32_t* axis_modes, int max_rank_hat,
                       int oversample, int32_t* y_cap, size_t* ws_bytes);

/*
 * The QTT-FFT convolution route, Step 3 of Algorithm 2:
 * I = QiFFT(QFFT(F) . QFFT(G)), truncated by R^_max (and optionally a
 * tolerance and the drop-off threshold) in every transform.
 *   f         real data tensor, d modes (f32 or f64); each axis is
 *             zero-padded by one mode (the data in the lower half)
 *   w, n_axes, axis_modes   as in qtt_conv: n_axes = 1 (a signal, w[0] with
 *             d + 1 modes) or 2 (a row-major image, axis_modes = {dx, dy},
 *             dx + dy = d, w[0] the column axis with dx + 1 modes, w[1] the
 *             row axis with dy + 1 modes); each w is a Toeplitz generator as
 *             written by qtt_kernel_sinc (lag u - 2^k at index u), rotated
 *             here by 2^k (lag 0 at index 0, the negative lags at the top),
 *             so that the lower half of the circular convolution is the
 *             discrete convolution (2.2), the product of qtt_conv.  For an
 *             image both transforms are two-dimensional: each axis's digits
 *             form a block transformed on its own (bit-reversed inside it)
 *   eps_hat, max_rank_hat, delta_hat   the rule of every rounding, as in
 *             qtt_fft (max_rank_hat >= 1)
 *   oversample, seed   the product of the two spectra (ranks r_F r_G) is
 *             rounded by a randomised TT rounding: Gaussian sketch TT of
 *             ranks ell = max_rank_hat + oversample (Philox-4x32-10, counter
 *             (2t + i, u, p, 0) for entry (t, i, u) of core p, key = seed),
 *             orthogonalisation left to right, then the truncation sweep
 *   y         real tensor, d modes, dtype of f, capacities from
 *             qtt_query_conv_fft: the real part of the inverse transform with
 *             every padding digit 0, as a real TT (complex ranks doubled)
 * The actual ranks of f and w must not exceed QTT_FFT_MAX_RANK; otherwise y
 * is the zero tensor and QTT_STATUS_FFT_RANK is set in y->status.  The
 * transforms run in FP64 complex arithmetic whatever the dtype of f.
 */
int qtt_conv_fft(const qtt_tensor* f, const qtt_tensor* w, int n_axes, const int32_t* axis_modes,
                 double eps_hat, int max_rank_hat, double delta_hat, int oversample,
                 uint64_t seed, qtt_tensor* y, void* ws, size_t ws_bytes, void* stream);

/*
 * Kernel classes for the launch probe.  Between qtt_probe_start and
 * qtt_probe_stop the library records a HIP event pair on the launch stream
 * around every launch of kernels of class `cls` (at most `max_launches`
 * pairs); qtt_probe_stop waits for the recorded events and returns the summed
 * GPU time (ms) and the number of launches.  Measurement aid only: one probe
 * per process, not thread-safe, events are created and destroyed by these
 * two calls (no device memory is allocated).
 */
#define QTT_K_LEVEL_GRAM 1   /* streaming Gram of the samples (first pass)     */
#define QTT_K_REDUCE 2       /* fixed-order sum of partial Gram matrices       */
#define QTT_K_LEVEL_EIG 3    /* steps 1..6 from the level Gram                  */
#define QTT_K_PROJECT 4      /* streaming projection + Gram of the remainder   */
#define QTT_K_EIG_STEP 5     /* one truncated SVD step (FP64 eigensolver)      */
#define QTT_K_TAIL 6         /* last steps of the sweep in one workgroup       */
#define QTT_K_CONV 7         /* Toeplitz-operator x signal cores               */
#define QTT_K_FULL_CHAIN 8   /* half-chain products of Full                    */
#define QTT_K_FULL_FINAL 9   /* final product of Full (writes the 2^d outputs) */
#define QTT_K_OTHER 10       /* bookkeeping kernels                            */
#define QTT_K_ADJOINT 11     /* Toeplitz products on full vectors, adjoint of Full */
#define QTT_K_BATCH 12       /* batched (many-line) kernels                     */
#define QTT_K_SKETCH 13      /* randomised rounding: QR of the sketch, eigensteps */
#define QTT_K_SKETCH_GEMM 14 /* sketch GEMMs Y = A Omega, B = Q^T A, B B^T (MFMA) */
#define QTT_K_QFFT 15        /* QTT-FFT stages and their rounding (one workgroup each) */
#define QTT_K_QFFT_HADAMARD 16 /* randomised rounding of the spectra's product    */

int qtt_probe_start(int cls, int max_launches);
int qtt_probe_stop(double* total_ms, int* launches);

#ifdef __cplusplus
}
#endif

#endif /* QTT_H */
