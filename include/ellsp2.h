/*
 * ellsp2.h -- C ABI of the MI355X (gfx950) thresholded ELLPACK X^2 and SP2
 * density-matrix purification library (libellsp2.so).
 *
 * Source: arXiv 2102.08505, "Performance Optimizations of Recursive Electronic
 * Structure Solvers targeting Multi-Core Architectures".  The paper's problem
 * statement for a BML operation is: allocate and initialise the ELLPACK
 * matrix, run the linear-algebra step, de-allocate (section "Micro-Kernel
 * Performance Evaluation - NUMA Aware Data", its allocation listings give the
 * ELLPACK fields N, M, nnz, index, value).  The benchmarked operation is the
 * BML ELLPACK matrix-matrix multiply X.X (section "Performance Evaluation using
 * System Matrices"), and the application loop around it is ExaSP2's SP2-Basic
 * algorithm: initialisation, then per iteration an X^2 product, a matrix norm
 * and the remaining update steps (section "Performance Evaluation using an
 * ExaSP2 Application").  The paper prints no formula for these steps; the
 * conventions below are this library's reading and are the same ones the
 * test oracle implements:
 *
 *   X^2     row-wise (Gustavson) product; each output entry is a chain of
 *           fused multiply-adds in ascending k.  Bit-for-bit reproducible.
 *   prune   an entry is kept iff |v| > tau (strict); exact zeros never stored.
 *   trace   Tr X = pairwise tree over i of X_ii (0 if absent); Tr X^2 uses the
 *           diagonal of the product before pruning.
 *   pairwise tree   while n > 1: d'[i] = d[2i] + d[2i+1], an odd last element
 *           passes through.
 *   norm    eta^2 = ||X^2 - X||_F^2 with the pruned X^2 and the stored X.  Row
 *           term e_i: the pairwise tree over all N column positions j of
 *           q_j = d*d, d = X^2_ij - X_ij (a value absent from a matrix is 0,
 *           so q_j = +0 where neither stores column j), each square rounded
 *           to double (FP32 values are widened exactly first); eta^2 = the
 *           pairwise tree of the e_i.  The tree over N leaves is the perfect
 *           tree over the next power of two with +0 leaves past N.
 *   X0      Gershgorin bounds emin, emax of H (row sums of |H_ij|, j != i, in
 *           ascending j); X0 = (emax I - H) * (1 / (emax - emin)), pruned.
 *   branch  up = |2 TrX - TrX^2 - n_occ| < |TrX^2 - n_occ| (a tie takes X^2);
 *           up: X <- prune(2X - X^2), else X <- X^2.
 *   stop    eta^2 < idem_target^2 returns the X whose eta was measured.
 *
 * Device storage (this library's layout): row-major ELLPACK.  Row i occupies
 * slots [i*M, i*M + nnz[i]) of index[] and value[]; columns strictly
 * ascending; slots >= nnz[i] are unspecified.  Values are double (ELL_F64) or
 * float (ELL_F32), indices int32.
 *
 * Streams: every call is ordered on the handle's HIP stream (NULL = the
 * default stream).  Calls that return host scalars synchronise that stream
 * before returning.  Handles are not thread-safe.
 *
 * Errors: every function returns an int status, 0 = ELL_OK, < 0 = error.
 * Arguments are validated on the host before any device call, so argument
 * errors are reported without touching a GPU.
 */
#ifndef ELLSP2_H
#define ELLSP2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ellpack ellpack_t; /* opaque handle */

typedef enum { ELL_F64 = 0, ELL_F32 = 1 } ell_prec_t;

enum {
  ELL_OK = 0,
  ELL_EINVAL = -1,      /* bad argument or malformed matrix */
  ELL_ENOMEM = -2,      /* device or host allocation failed */
  ELL_EOVERFLOW = -3,   /* a result row needs more than the capacity M */
  ELL_ENOCONV = -4,     /* SP2: max_iter reached or stalled */
  ELL_EDEVICE = -5,     /* HIP runtime failure; see ellpack_last_device_error */
  ELL_ENODEV = -6,      /* no usable GPU */
  ELL_ENONFINITE = -7,  /* NaN or Inf in an input */
  ELL_EDEGENERATE = -8  /* emax == emin, or n_occ outside (0, N) */
};

enum { SP2_F64 = 0, SP2_MIXED = 1 };
enum { DENSE_F64 = 0, DENSE_BF16X3 = 1 };

/* Host-only structural check of a row-major ELLPACK matrix: N > 0, M > 0,
 * 0 <= nnz[i] <= M, 0 <= index < N strictly ascending per row, values finite
 * (value may be NULL to skip that check).  Returns ELL_OK, ELL_EINVAL or
 * ELL_ENONFINITE.  Never touches a device. */
int ellpack_check_host(int32_t N, int32_t M, const int32_t *nnz, const int32_t *index_rowmajor,
                       const double *value_rowmajor);

/* Allocate an N x N matrix with capacity M slots per row on the current
 * device, every row empty.  The library owns the device buffers (released by
 * ellpack_free).  hip_stream: a hipStream_t, or NULL.
 * Limits: 1 <= N <= 2^20, 1 <= M <= 65536.
 * Errors: ELL_EINVAL (N or M out of range, bad prec), ELL_ENODEV, ELL_ENOMEM. */
int ellpack_alloc(ellpack_t **A, int32_t N, int32_t M, ell_prec_t prec, void *hip_stream);

/* Wrap caller-owned device buffers in the layout above (for example the
 * storage of torch tensors): d_nnz int32[N], d_index int32[N*M], d_value
 * double or float [N*M].  The caller keeps them alive; ellpack_free releases
 * only the handle.  The contents are validated on the device before first use
 * by a computing call. */
int ellpack_wrap(ellpack_t **A, int32_t N, int32_t M, ell_prec_t prec, int32_t *d_nnz,
                 int32_t *d_index, void *d_value, void *hip_stream);

/* Release a handle (and its buffers if the library owns them).  NULL is a no-op. */
int ellpack_free(ellpack_t *A);

/* N, capacity M and precision of a handle (any pointer may be NULL). */
int ellpack_info(const ellpack_t *A, int32_t *N, int32_t *M, int32_t *prec);

/* Copy a host row-major matrix (stride = the handle's M) to the device.  The
 * host arrays are validated first (ellpack_check_host); values are given in
 * double and rounded to float for an ELL_F32 handle.  Synchronous. */
int ellpack_upload(ellpack_t *A, const int32_t *nnz, const int32_t *index_rowmajor,
                   const double *value_rowmajor);

/* Copy the device matrix to host row-major arrays of N*M (stride M).  Unused
 * slots are written as index -1, value 0.  ELL_F32 values are widened
 * exactly.  Synchronous. */
int ellpack_download(const ellpack_t *A, int32_t *nnz, int32_t *index_rowmajor,
                     double *value_rowmajor);

/* X2 = prune(X . X, tau) ("SP2 Loop X2" of the paper's SP2-Basic breakdown).
 * X and X2 must have the same N and precision and must not alias.
 * trace_out[0] = Tr X, trace_out[1] = Tr(X.X) before pruning (may be NULL).
 * *max_row_width_out = widest row of the pruned product (may be NULL), also
 * on overflow.  If a row needs more than X2's capacity the call returns
 * ELL_EOVERFLOW and X2's contents are unspecified; nothing is truncated
 * silently.  tau must be >= 0 (rounded to float for ELL_F32). */
int ellpack_x2_threshold(const ellpack_t *X, ellpack_t *X2, double tau, double trace_out[2],
                         int32_t *max_row_width_out);

/* The fused SP2 step kernel exposed whole: X2 = prune(X.X, tau) as above,
 * plus (if U != NULL) U = prune(2X - X2, tau) over the union of the patterns,
 * and the idempotency norm ("SP2 Loop Norm").  out[0] = Tr X, out[1] = Tr X^2
 * (unpruned diagonal), out[2] = eta^2 = ||X2 - X||_F^2 (any may be NULL via
 * out == NULL).  widths[0], widths[1] = widest row of X2 and U.  Overflow of
 * either output returns ELL_EOVERFLOW. */
int ellpack_x2_step(const ellpack_t *X, ellpack_t *X2, ellpack_t *U, double tau, double out[3],
                    int32_t widths[2]);

/* ellpack_x2_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results, errors and bits as ellpack_x2_step, computed
 * by the ELLPACK step kernel only, with every intermediate (per-row outputs,
 * reduction partials, the validation flag) in a fixed device array of the
 * library, about 4 MiB per device, kept until the process ends.  Calls no
 * hipMalloc / hipFree.  N must be <= 131072 (ELL_EINVAL beyond, with a
 * message in ellpack_last_device_error).  The first call on a device resolves
 * that device's copy of the array (the current device, which must be the
 * handles' device).  Every call on one device shares that array: calls that
 * overlap on one device (other host threads, or other streams still running
 * an earlier call) race and give undefined results. */
int ellpack_x2_step_noalloc(const ellpack_t *X, ellpack_t *X2, ellpack_t *U, double tau, double out[3],
                            int32_t widths[2]);

/* Tr A by the pairwise tree. */
int ellpack_trace(const ellpack_t *A, double *trace_out);

/* Tr(AB) = sum_i sum_j A_ij B_ji of two validated N x N handles of either
 * precision: the energy Tr(DH) of a density matrix D and its Hamiltonian H
 * (the output of the paper's "ExaSP2 Application").  Row term t_i: fused
 * multiply-adds over the stored entries of row i of A in ascending column j,
 * t = fma(A_ij, B_ji, t), with B_ji from row j of B (skipped where B stores no
 * (j, i) entry) and FP32 values widened exactly to double; Tr(AB) = pairwise
 * tree of the t_i.  trace_out: host double.  Runs on A's stream after
 * synchronising B's.  Errors: ELL_EINVAL (NULL, different N, malformed
 * matrix), ELL_ENONFINITE, ELL_EDEVICE. */
int ellpack_trace_product(const ellpack_t *A, const ellpack_t *B, double *trace_out);

typedef struct {
  double n_occ;            /* target occupation Tr P, in (0, N) */
  double tau;              /* FP64 drop tolerance, >= 0 */
  double idem_target;      /* stop when ||X^2 - X||_F < idem_target */
  int32_t max_iter;        /* maximum number of X^2 products, >= 1 */
  int32_t precision;       /* SP2_F64 or SP2_MIXED */
  int32_t fp64_tail_steps; /* mixed: FP64 updates required before the stop test may pass (2) */
  int32_t poll_every;      /* host reads the device flags every poll_every iterations (4) */
  double tau_fp32;         /* mixed: FP32 drop tolerance */
  double switch_eta;       /* mixed: switch to FP64 once eta < switch_eta (or on a stall) */
  int32_t stall_stop;      /* nonzero: once eta < 1e-2, stop (ENOCONV) when the best eta of
                              the last two steps is no better than that of the two before */
  int32_t profile;         /* nonzero: time every X^2 step kernel with hipEvents (report x2_*) */
  int32_t prune_once;      /* 0: two prunings per iteration -- X^2 is pruned, and 2X - X^2 and the
                              norm ||X^2 - X||_F are formed from the pruned X^2, then 2X - X^2 is
                              pruned again; nonzero: one pruning -- 2X - X^2 and the norm are formed
                              from the unpruned X^2, and only the iterate taken is pruned (the
                              paper's "SP2 Loop X2", "Norm" and "Misc" steps fused into one pass;
                              its text does not say where the pruning falls).  Branch, traces and
                              every other rule are the same. */
} sp2_params_t;

typedef struct {
  int32_t status;          /* same as the return value */
  int32_t iterations;      /* X^2 products computed */
  int32_t fp32_iterations; /* of which in FP32 (mixed) */
  int32_t final_M;         /* capacity the working matrices ended with */
  double eta, trace_x, emin, emax;
  double seconds;          /* device time from X0 to stop (hipEvent) */
  /* caller-owned host arrays of length max_iter, or NULL */
  double *hist_trx, *hist_trx2, *hist_eta2;
  int8_t *hist_up;         /* 1: 2X - X^2 taken, 0: X^2 taken, -1: no update (stop) */
  int32_t *hist_maxw;      /* widest row of the pruned X^2 */
  int8_t *hist_prec;       /* 1: FP32 step, 0: FP64 step */
  double x2_seconds;       /* p->profile != 0: summed duration of the X^2 step kernels that did
                              work (hipEvents around each launch); else 0 */
  int64_t x2_bytes;        /* algorithmic bytes of the X^2 products: every stored entry of X read
                              once and of the pruned X^2 written once, value + index, plus nnz arrays */
  int32_t x2_launches;     /* p->profile != 0: number of those kernels; else 0 */
  /* caller-owned host arrays of length max_iter, or NULL: per iteration, the duration of its
     X^2 step kernel (p->profile != 0 only) and its algorithmic bytes as counted in x2_bytes
     (dense_sp2_solve: the duration of each product and its bytes, p->profile != 0 only) */
  double *hist_x2_seconds;
  int64_t *hist_x2_bytes;
  int32_t batch_k;         /* sp2_solve_batched: iterations per graph replay it used; else 0 */
  int32_t batch_kernel;    /* sp2_solve_batched: its step kernel, 0 matrix cores, 1 register-tiled
                              VALU (the same results); else 0 */
} sp2_report_t;

/* SP2 purification of the FP64 Hamiltonian H into the density matrix D
 * (FP64).  Runs entirely on the device: X0, then per iteration the fused
 * X^2/trace/norm/update kernel, a deterministic reduction and a device-side
 * decision; the host only polls flags every poll_every iterations.  Working
 * matrices grow their capacity on overflow (to a multiple of 32) and redo the
 * step, so the result never depends on M.  If D is library-owned it is
 * reallocated when too narrow; a wrapped D that is too narrow gives
 * ELL_EOVERFLOW with r->final_M = the width needed.  On ELL_ENOCONV, D holds
 * the last X and the report is filled.  r may be NULL. */
int sp2_solve(const ellpack_t *H, ellpack_t *D, const sp2_params_t *p, sp2_report_t *r);

/* n independent SP2 solves of uneven sizes, run together: the instances' rows
 * are stacked in one matrix and every iteration is one launch of the step
 * kernel over all of them, replayed from a captured HIP graph of K iterations,
 * with per-instance state (buffers, precision phase, stop) on the device.
 * p: n parameter sets (one per instance); p[0].poll_every = K, or 0 to pick K
 * and then the step kernel (matrix cores or register-tiled VALU) by timing the
 * first graph replays; that choice is kept for the life of the process per
 * device architecture, precision mix and size class (log2 of the stacked rows
 * and of the row stride), and later calls of the same class replay at once.  Each instance's result, history and
 * status are bit-identical to sp2_solve on it alone; an instance the stacked
 * form cannot hold (X0 with exact zeros or rows wider than 65536 columns, or a
 * stride overflow beyond that) is finished by sp2_solve on its own.  r: n
 * reports (may be NULL); `seconds` is the whole batch's device time, and the
 * x2 timing fields are 0 (the step kernel serves all instances at once).
 * Returns ELL_OK or the most negative instance status. */
int sp2_solve_batched(int32_t n, const ellpack_t *const *H, ellpack_t *const *D,
                      const sp2_params_t *p, sp2_report_t *r);

/* Dense variant on device arrays: d_H, d_D row-major N x N double.  mode
 * DENSE_F64: FP64 X^2 throughout; DENSE_BF16X3: X held in float and X^2 from
 * three bf16 MFMA products (hi.hi + hi.lo + lo.hi, FP32 accumulate) until the
 * switch rule fires, then FP64 with p->fp64_tail_steps FP64 updates before
 * the stop test may pass. */
int dense_sp2_solve(const double *d_H, int32_t N, double *d_D, int32_t mode, const sp2_params_t *p,
                    sp2_report_t *r, void *hip_stream);

/* Dense X^2 on device arrays (the MFMA kernels exposed for testing):
 * mode DENSE_F64: d_C = d_A.d_A in double (d_A, d_C double N x N);
 * mode DENSE_BF16X3: float in, float out. */
int dense_x2(const void *d_A, void *d_C, int32_t N, int32_t mode, void *hip_stream);

/* Text of a status code. */
const char *ellpack_strerror(int status);
/* Text of the last HIP error seen by this library (thread-local). */
const char *ellpack_last_device_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ELLSP2_H */
