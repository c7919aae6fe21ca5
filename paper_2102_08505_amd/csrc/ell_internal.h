// Internal declarations of libellsp2: device views, the device-resident SP2
// control block, and the kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ellsp2 {

// Row-major ELLPACK on the device: row i at [i*M, i*M + nnz[i]).
template <typename T>
struct EllView {
  int32_t *nnz;
  int32_t *idx;
  T *val;
  int32_t M;
};

// Three working matrices of one precision; during SP2 the current X is
// buffer `cur`, X^2 goes to (cur+1)%3 and 2X - X^2 to (cur+2)%3.
template <typename T>
struct Rot3 {
  EllView<T> b[3];
};

// Internal status values beyond the public ELL_* codes.
enum { ST_RUNNING = 1, ST_SWITCH = 2 };

// Device-resident state of one SP2 solve.  Written only by the single-thread
// decision kernel (and by the host between polls while the stream is idle).
struct SP2State {
  int32_t cur;          // index of the current X buffer
  int32_t iter;         // X^2 products completed and accepted
  int32_t stop;         // nonzero: every further kernel of this solve returns at once
  int32_t status;       // ST_RUNNING, ST_SWITCH or an ELL_* code
  int32_t phase32;      // 1 while iterating in FP32 (mixed mode)
  int32_t fp64_updates; // FP64-phase updates applied
  int32_t phase_start;  // iteration index where the current phase began
  int32_t need_width;   // on overflow: the width required
  int32_t cap;          // capacity M of the working matrices
  int32_t wy_max, wu_max;
  int32_t pad;
  double trx, trx2, eta2;
};

struct SP2Cfg {
  double n_occ, target2, switch2;
  int32_t max_iter, tail, stall, mixed;
};

struct SP2Hist {
  double *trx, *trx2, *eta2;
  int8_t *up, *prec;
  int32_t *maxw;
  int64_t *nnzx, *nnzy;  // total stored entries of X and of the pruned X^2
};

// Per-call scratch of the fused step: per-row outputs and reduction partials.
struct StepScratch {
  double *d1, *d2, *e;      // N
  int32_t *wy, *wu;         // N: true survivor counts (may exceed capacity)
  double *part;             // 3 * nb partial sums
  int32_t *partw;           // 2 * nb partial maxima
  int64_t *partn;           // 2 * nb partial nnz totals
  double *out;              // 3: TrX, TrX2, eta2
  int32_t *outw;            // 2: widest X2 row, widest U row
  int64_t *outn;            // 2: nnz(X), nnz(X2)
  int32_t nb;               // number of 1024-row reduction blocks
};

constexpr int kRedBlock = 1024;  // rows per partial-reduction block
constexpr int kMaxFinal = 1024;  // partials the final reduction handles in one block
constexpr int kMaxCap = 4096;    // largest supported capacity M
constexpr int kMaxN = kRedBlock * kMaxFinal;  // two reduction levels cover every row

// ---- launchers (ell_kernels.hip) ---------------------------------------------------
template <typename T>
hipError_t launch_x2_step(int N, Rot3<T> bufs, const SP2State *st, bool with_u, T tau,
                          const StepScratch &s, hipStream_t stream);
hipError_t launch_reduce(int N, const SP2State *st, const StepScratch &s, hipStream_t stream,
                         const int32_t *nnzx_rows, const int32_t *nnzy_rows_a,
                         const int32_t *nnzy_rows_b);
hipError_t launch_decide(SP2State *st, SP2Cfg cfg, SP2Hist hist, const StepScratch &s,
                         hipStream_t stream);
hipError_t launch_final_only(const StepScratch &s, hipStream_t stream);

hipError_t launch_gershgorin(int N, EllView<double> H, double *rowlo, double *rowhi,
                             double *emin_emax, int32_t *flags, hipStream_t stream);
template <typename T>
hipError_t launch_x0(int N, EllView<double> H, EllView<T> X, double emax, double inv, T tau,
                     int32_t *wmax, hipStream_t stream);
template <typename TS, typename TD>
hipError_t launch_copy(int N, EllView<TS> src, EllView<TD> dst, hipStream_t stream);
template <typename T>
hipError_t launch_validate(int N, EllView<T> A, int32_t *flags, hipStream_t stream);
template <typename T>
hipError_t launch_trace_rows(int N, EllView<T> A, double *d, hipStream_t stream);
hipError_t launch_tree_sum(int n, const double *d, double *part, double *out, hipStream_t stream);

}  // namespace ellsp2
