/*
 * CPU oracle for the thresholded ELLPACK X^2 and the SP2 purification loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this code.  The GPU library
 * shares no code, header, table or helper with it.
 *
 * Plain C11, every step written in the order the definition states it; no
 * blocking, fusion or reordering.  The row loops of X^2 and of the update
 * are shared out over OpenMP threads, row by row: a row's result depends on
 * the inputs alone, so it is the same for any thread count.  Matrices are row-major
 * ELLPACK (the field set of the paper's ELLPACK listings, section "NUMA Aware
 * Data": N, M, nnz[N], index[N*M], value[N*M]); row i occupies slots
 * i*M .. i*M + nnz[i] - 1 with strictly ascending columns.
 *
 * The paper (arXiv 2102.08505) names the operations on this path -- the BML
 * ELLPACK matrix-matrix multiply and the SP2-Basic loop with its X2, Norm and
 * Misc steps (section "Performance Evaluation using an ExaSP2 Application") --
 * but prints no formula for any of them.  The conventions fixed here are:
 *
 *   X^2    Gustavson's row-wise product with a dense accumulator; for every
 *          output entry the products are added with fma() in ascending k.
 *   prune  an entry is kept iff |v| > tau (strict); exact zeros never stored.
 *   traces d1[i] = X_ii (0 if absent), d2[i] = (X.X)_ii before pruning;
 *          a trace is the pairwise tree sum of the vector (orc_pairwise).
 *   norm   eta^2 = ||X2 - X||_F^2: e_i = pairwise tree over the row's N
 *          column positions of the rounded squares d*d (d = 0 where neither
 *          matrix stores the column), eta^2 = pairwise tree of the e_i.
 *   X0     Gershgorin bounds; X0 = (emax I - H) / (emax - emin), pruned.
 *   branch up = |2 TrX - TrX2 - n_occ| < |TrX2 - n_occ|  (tie -> X^2);
 *          up: X <- prune(2X - X^2); else X <- X^2.
 *   stop   eta^2 < target^2 returns the X whose eta was measured.
 * Parity status of each function is stated beside it.
 */
#ifndef ELLSP2_ORACLE_H
#define ELLSP2_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EOVERFLOW = -3,
  ORC_ENOCONV = -4, ORC_ENONFINITE = -7, ORC_EDEGENERATE = -8
};

enum { ORC_PREC_F64 = 0, ORC_PREC_MIXED = 1 };
enum { ORC_DENSE_F64 = 0, ORC_DENSE_BF16X3 = 1 };

/* Pairwise tree sum: while n > 1, d'[i] = d[2i] + d[2i+1] for i < n/2, an odd
 * last element passes through unchanged.  Empty sum is +0. */
double orc_pairwise(int64_t n, const double *d);

/* Structural checks: nnz in [0,M], columns in [0,N) strictly ascending; values finite. */
int orc_check_ell(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx);
int orc_check_finite_f64(int32_t N, int32_t M, const int32_t *nnz, const double *val);

/* Number of scalar FMAs of X.X: sum over rows i, over k in row i, of nnz[k]. */
int64_t orc_x2_fma_count(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx);

/* Sets the OpenMP thread count when n > 0; returns the count in use. */
int32_t orc_threads(int32_t n);

/* Fills rows of an N x M ELLPACK matrix with nothing stored (nnz 0, index -1,
 * value 0; val_size bytes per value) in the row loops' static schedule, so
 * that first touch places each row's pages with the thread that writes it. */
void orc_rows_init(int32_t N, int32_t M, int32_t *nnz, int32_t *idx, void *val, int32_t val_size);

/* Host memory bandwidth in GB/s: the best of `reps` runs of the STREAM triad
 * a = b + s c over arrays of n doubles (24 bytes per element counted), on the
 * OpenMP threads, arrays first touched in the same static schedule.  Returns
 * a negative value when the arrays cannot be allocated.  (host_stream.c; not
 * part of the oracle's arithmetic: it sizes the CPU baseline.) */
double orc_stream_triad(int64_t n, int32_t reps);

/* X2 = prune(X.X, tau).  d1, d2 (length N, may be NULL) receive X_ii and the
 * unpruned (X.X)_ii.  *maxw receives the largest surviving row width (also on
 * overflow).  Returns ORC_EOVERFLOW if a row needs more than M2 slots. */
int orc_x2_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
               double tau, int32_t M2, int32_t *nnz2, int32_t *idx2, double *val2,
               double *d1, double *d2, int32_t *maxw);
/* FP32 values, fmaf accumulation, float threshold; d1/d2 promoted to double. */
int orc_x2_f32(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const float *val,
               float tau, int32_t M2, int32_t *nnz2, int32_t *idx2, float *val2,
               double *d1, double *d2, int32_t *maxw);

/* Trace (pairwise tree over the diagonal). */
double orc_trace_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val);
/* Tr(AB) = sum_i sum_j A_ij B_ji: per row of A an ascending-j fma chain of
 * A_ij * B_ji over the stored (j, i) entries of B, then the pairwise tree over
 * rows.  FP64 values (FP32 inputs are widened exactly by the caller). */
double orc_trace_product_f64(int32_t N, int32_t MA, const int32_t *nnzA, const int32_t *idxA, const double *valA,
                             int32_t MB, const int32_t *nnzB, const int32_t *idxB, const double *valB);

/* eta^2 = ||X2 - X||_F^2; e (length N, may be NULL) receives the row terms. */
double orc_norm2_f64(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const double *valX,
                     int32_t M2, const int32_t *nnz2, const int32_t *idx2, const double *val2, double *e);
/* FP32 matrices; differences taken in double after exact widening. */
double orc_norm2_f32(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const float *valX,
                     int32_t M2, const int32_t *nnz2, const int32_t *idx2, const float *val2, double *e);

/* Out = prune(2X - X2, tau), sorted union of the two rows. */
int orc_update_f64(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const double *valX,
                   int32_t M2, const int32_t *nnz2, const int32_t *idx2, const double *val2, double tau,
                   int32_t Mo, int32_t *nnzo, int32_t *idxo, double *valo, int32_t *maxw);
int orc_update_f32(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const float *valX,
                   int32_t M2, const int32_t *nnz2, const int32_t *idx2, const float *val2, float tau,
                   int32_t Mo, int32_t *nnzo, int32_t *idxo, float *valo, int32_t *maxw);

/* Rows rows[0 .. nr) of prune(X.X, tau) in FP64, computed as orc_x2_f64
 * computes them, into output rows 0 .. nr (capacity M2), and the unpruned
 * diagonal entries (X.X)_ii of those rows in d2 (may be NULL): for checking
 * sampled rows of products too large to form whole. */
int orc_x2_rows_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
                    double tau, int32_t nr, const int32_t *rows, int32_t M2, int32_t *nnz2, int32_t *idx2,
                    double *val2, double *d2);

/* A = prune(Y, tau): the entries of Y with |v| > tau, in order. */
int orc_prune_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val, double tau,
                  int32_t Mo, int32_t *nnzo, int32_t *idxo, double *valo, int32_t *maxw);
int orc_prune_f32(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const float *val, float tau,
                  int32_t Mo, int32_t *nnzo, int32_t *idxo, float *valo, int32_t *maxw);

/* Gershgorin interval of H. */
int orc_gershgorin(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
                   double *emin, double *emax);
/* X0 = prune((emax I - H) * (1/(emax - emin)), tau).  The diagonal is inserted if absent. */
int orc_x0_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
               double emin, double emax, double tau,
               int32_t Mo, int32_t *nnzo, int32_t *idxo, double *valo, int32_t *maxw);
/* FP32 X0: the FP64 value rounded to float, then kept iff |x| > tau (float). */
int orc_x0_f32(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
               double emin, double emax, float tau,
               int32_t Mo, int32_t *nnzo, int32_t *idxo, float *valo, int32_t *maxw);

typedef struct {
  double n_occ;          /* target occupation, in (0, N) */
  double tau;            /* FP64 drop tolerance */
  double idem_target;    /* stop when ||X^2 - X||_F < idem_target */
  int32_t max_iter;      /* maximum number of X^2 products */
  int32_t precision;     /* ORC_PREC_F64 or ORC_PREC_MIXED */
  int32_t fp64_tail_steps; /* mixed: FP64 updates before the stop test may pass */
  int32_t stall_stop;    /* nonzero: apply the stall rule */
  double tau_fp32;       /* mixed: FP32 drop tolerance (rounded to float) */
  double switch_eta;     /* mixed: switch to FP64 when eta < switch_eta */
  int32_t prune_once;    /* 0: X2 = prune(X.X) enters the norm and 2X - X2, which is pruned
                            again (two prunings); nonzero: the unpruned product Y = X.X enters
                            the norm and 2X - Y, and only the iterate taken is pruned:
                            prune(Y) or prune(2X - Y) (one pruning) */
} orc_sp2_params;

typedef struct {
  int32_t status, iterations, fp32_iterations, final_M;
  double eta, trace_x, emin, emax;
  /* caller-owned arrays of length max_iter, or NULL */
  double *hist_trx, *hist_trx2, *hist_eta2;
  int8_t *hist_up;       /* 1: 2X - X^2, 0: X^2, -1: no update (stop) */
  int32_t *hist_maxw;    /* max row width of the pruned X^2 */
  int8_t *hist_prec;     /* 0: FP64 step, 1: FP32 step */
} orc_sp2_report;

/* Full SP2 from H.  D receives the returned X (FP64, capacity Mo); if its
 * widest row exceeds Mo the call returns ORC_EOVERFLOW with r->final_M set. */
int orc_sp2(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
            const orc_sp2_params *p, int32_t Mo, int32_t *nnzD, int32_t *idxD, double *valD,
            orc_sp2_report *r);

/* ---- dense variant -------------------------------------------------------- */
/* C = A.A, every entry an fma chain in ascending k (row-major N x N). */
void orc_dense_x2_f64(int32_t N, const double *A, double *C);
/* bf16 round-to-nearest-even of a float (returned as float). */
float orc_bf16_rne(float x);
/* Three-product split: hi = bf16(x), lo = bf16(x - hi);
 * C = hi.hi + hi.lo + lo.hi with float accumulation. */
void orc_dense_x2_bf16x3(int32_t N, const float *A, float *C);
/* Dense SP2 (no pruning).  mode ORC_DENSE_F64 runs in FP64 throughout;
 * ORC_DENSE_BF16X3 keeps X in float with the split product until the switch
 * rule fires, then finishes in FP64 as the mixed ELLPACK mode does. */
int orc_dense_sp2(int32_t N, const double *H, int32_t mode, const orc_sp2_params *p,
                  double *D, orc_sp2_report *r);

#ifdef __cplusplus
}
#endif
#endif
