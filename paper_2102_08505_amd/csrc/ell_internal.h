// Internal declarations of libellsp2: device views, the device-resident SP2
// control block, and the kernel launchers.  Not part of the public ABI.
#pragma once

#include <algorithm>
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

// Span form: row i stored densely over columns [base[i], base[i] + len[i]) at
// val[i*SW ...] (zeros at pruned positions).  val points kSpanGuard elements
// into its allocation, which has kSpanGuard spare elements at both ends.
template <typename T>
struct SpanView {
  T *val;
  int32_t *base;
  int32_t *len;
  int32_t SW;
};

template <typename T>
struct SpanRot3 {
  SpanView<T> b[3];
};

constexpr int kSpanGuard = 1024;  // elements; larger than any window the band kernel reads across
constexpr int kSpanPadRows = 64;  // base/len entries past N (zero): batched loads may run past the last row

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
  int32_t cap;          // capacity M of the working matrices (ELLPACK pipeline)
  int32_t sw;           // row stride SW of the working matrices (span pipeline)
  int32_t wy_max, wu_max;
  int64_t nnz_cur;      // stored entries of the current X
  double trx, trx2, eta2;
  // symmetric span iteration: the branch of the next product (1: 2X - X^2),
  // fixed from the traces of the current X that the step which wrote it
  // predicted, Tr X and the unpruned Tr X^2; the next step checks them
  int32_t up_next;
  int32_t once;         // 1: 2X - X^2 and the norm from the unpruned X^2 (one pruning per iteration)
  double ptrx, ptrx2;
};

enum { ST_FALLBACK = 3 };  // span pipeline cannot take a row group: continue on ELLPACK
enum { ST_MISPREDICT = 4 };  // symmetric iteration: the traces of X differ from those predicted

struct SP2Cfg {
  double n_occ, target2, switch2;
  int32_t max_iter, tail, stall, mixed;
  int32_t span;  // 1: working matrices are in span form (capacity = SW, not M)
  int32_t pad;
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
  int32_t *ly, *lu;         // N: interval lengths of X2 and U rows (span pipeline), or NULL
  double *part;             // 3 * nb partial sums (symmetric span iteration: 5 * nq + 256 L, L >= nq / 256 a power of two)
  int32_t *partw;           // 4 * nb partial maxima (wy, wu, ly, lu)
  int64_t *partn;           // 2 * nb partial nnz totals (X2, U)
  double *out;              // 3: TrX, TrX2, eta2 (symmetric span iteration: 5, with Tr X', Tr X'^2)
  int32_t *outw;            // 4: widest X2 row, widest U row, longest X2 / U interval
  int64_t *outn;            // 2: nnz(X2), nnz(U)
  int32_t *flags;           // bit 0: a row group needs the ELLPACK pipeline
  uint32_t *ticket;         // workgroups of the symmetric step finished so far (0 between launches)
  int32_t nb;               // number of 1024-row reduction blocks
  int32_t nq;               // number of 64-row partials (span iteration on the matrix cores; part* hold 5 / 4 / 2 * nq)
};

constexpr int kRedBlock = 1024;  // rows per partial-reduction block
constexpr int kMaxFinal = 1024;  // partials the final reduction handles in one block
constexpr int kMaxCap = 1 << 16;  // largest supported capacity M (entries per row)
constexpr int kMaxN = kRedBlock * kMaxFinal;  // two reduction levels cover every row

// Record a failed HIP call as the library's last device error; returns the
// matching ELL_* status (ELL_ENOMEM for out-of-memory, else ELL_EDEVICE).
int device_error(hipError_t e, const char *what);
void set_device_error(const char *what);

// ---- launchers (ell_kernels.hip) ---------------------------------------------------
template <typename T>
hipError_t launch_x2_step(int N, Rot3<T> bufs, const SP2State *st, bool with_u, T tau,
                          const StepScratch &s, hipStream_t stream);
// The standalone step with the hashed row accumulator (ell_kernels.hip) for
// rows with at most 512 products, then the window kernel on the rows left in
// `left` (N entries) / *nleft (one word, cleared here).
template <typename T>
hipError_t launch_x2_hash(int N, Rot3<T> bufs, bool with_u, T tau, const StepScratch &s, int32_t *left,
                          int32_t *nleft, hipStream_t stream);
hipError_t launch_reduce(int N, const SP2State *st, const StepScratch &s, hipStream_t stream);
hipError_t launch_decide(SP2State *st, SP2Cfg cfg, SP2Hist hist, const StepScratch &s,
                         hipStream_t stream);
hipError_t launch_final_only(const StepScratch &s, hipStream_t stream);
// batched: nblocks reduction blocks over all instances; one decision block per instance
hipError_t launch_reduce_batch(int nblocks, const int32_t *blk_inst, const int32_t *blk_local,
                               const int32_t *inst_rows, const StepScratch *ss, const SP2State *states,
                               hipStream_t stream);
hipError_t launch_decide_batch(int n, SP2State *states, const SP2Cfg *cfgs, const SP2Hist *hists,
                               const StepScratch *ss, hipStream_t stream);

// Workgroups of the initialisation kernels (one wavefront per row, 4 per
// workgroup, rows strided over at most kInitBlocks workgroups).
constexpr int kInitBlocks = 1024;
inline int init_blocks(int N) { return N < 4 * kInitBlocks ? (N + 3) / 4 : kInitBlocks; }
// One instance of a multi-instance initialisation launch (the batched solve's
// Gershgorin bounds, symmetry checks and X0s, one launch each for all).
struct InitInst {
  EllView<double> H;  // its Hamiltonian
  int32_t N;
  int32_t w0, nw;     // its workgroups in the launch: w0 .. w0 + nw - 1
  int32_t r0;         // its first row in the packed X0 buffers
  int32_t f32;        // 1: its X0 is FP32
  double emax, inv;   // X0 = (emax I - H) inv
  double tau;         // X0's drop tolerance (rounded to its precision by the kernel)
};
// Gershgorin bounds of every instance (workgroups w0 = sum of gersh_blocks(N)
// of the instances before, nw = gersh_blocks(N); ws: their w0): out[2m],
// out[2m + 1] = emin, emax of instance m, flags[m] |= 2 if its H holds a
// non-finite value; plo, phi: the launch's per-workgroup partials.
hipError_t launch_gershgorin_multi(const InitInst *in, const int32_t *ws, int n, int nwork, double *plo,
                                   double *phi, double *out, int32_t *flags, hipStream_t stream);
// Bitwise symmetry of every instance (w0 = sum of sym_blocks(N) of the
// instances before, nw = sym_blocks(N)): flag[4m] |= 1 and the balance at
// flag + 4m + 2 (64 bits) as launch_check_symmetric's, all zeroed by the caller.
inline int sym_blocks(int N) { return (N + 3) / 4; }
hipError_t launch_check_symmetric_multi(const InitInst *in, const int32_t *ws, int n, int nwork, int32_t *flag,
                                        hipStream_t stream);
// X0 of every instance whose precision is T's into the packed rows X[r0 ..
// r0 + N) (rows: the packed rows; rs: the instances' r0, ascending); rowc[r]
// = the kept count of packed row r before the capacity cut (rows of other
// instances untouched).
template <typename T>
hipError_t launch_x0_multi(const InitInst *in, const int32_t *rs, int n, int rows, EllView<T> X, int32_t *rowc,
                           hipStream_t stream);

// Workgroups of the Gershgorin kernel: one wavefront per kGershRows rows.
constexpr int kGershRows = 16, kGershMaxBlocks = 8192;
inline int gersh_blocks(int N) { return std::min((N + kGershRows - 1) / kGershRows, kGershMaxBlocks); }
// Gershgorin bounds of H into emin_emax[0..1] (rowlo, rowhi: gersh_blocks(N)
// doubles of per-workgroup partials); flags |= 2 if H holds a non-finite value
hipError_t launch_gershgorin(int N, EllView<double> H, double *rowlo, double *rowhi,
                             double *emin_emax, int32_t *flags, hipStream_t stream);
// X0 of H into X: *wmax (zeroed by the caller) gets the widest row's count
// of kept entries, *total (zeroed, or null) their sum
template <typename T>
hipError_t launch_x0(int N, EllView<double> H, EllView<T> X, double emax, double inv, T tau,
                     int32_t *wmax, unsigned long long *total, hipStream_t stream);
// the same with the bounds read on the device (emin_emax[0..1], as written by
// launch_gershgorin); inv = 1 / (emax - emin) is formed there
template <typename T>
hipError_t launch_x0(int N, EllView<double> H, EllView<T> X, const double *emin_emax, T tau, int32_t *wmax,
                     unsigned long long *total, hipStream_t stream);
template <typename TS, typename TD>
hipError_t launch_copy(int N, EllView<TS> src, EllView<TD> dst, hipStream_t stream);
template <typename T>
hipError_t launch_validate(int N, EllView<T> A, int32_t *flags, hipStream_t stream);
hipError_t launch_zero_words(int n, int32_t *p, hipStream_t stream);
// up to eight int32 arrays cleared by one launch (the setup's interval arrays,
// which separate fills would each pay a host call and a device idle for)
struct ZeroList {
  int32_t *p[8];
  int n[8];
  int count;
};
hipError_t launch_zero_list(const ZeroList &z, hipStream_t stream);
template <typename T>
hipError_t launch_trace_rows(int N, EllView<T> A, double *d, hipStream_t stream);
// Bitwise symmetry of H: *flag |= 1 when a stored H_ij above the diagonal has
// no stored H_ji with the same bits, and *balance (both zeroed by the caller)
// gains the entries above the diagonal minus those below it.  H is bitwise
// symmetric iff neither is nonzero afterwards.
hipError_t launch_check_symmetric(int N, EllView<double> H, int32_t *flag, unsigned long long *balance,
                                  hipStream_t stream);
hipError_t launch_tree_sum(int n, const double *d, double *part, double *out, hipStream_t stream);
// row terms of Tr(AB): d[i] = ascending-j fma chain of A_ij * B_ji
template <typename TA, typename TB>
hipError_t launch_trace_product_rows(int N, EllView<TA> A, EllView<TB> B, double *d, hipStream_t stream);

// ---- span pipeline (ell_band.hip) ------------------------------------------------------
template <typename T>
hipError_t launch_x2_band(int N, SpanRot3<T> spans, Rot3<T> ells, const SP2State *st, bool with_u, bool out_ell,
                          T tau, const StepScratch &s, int32_t *fallback, hipStream_t stream);
// Span-form X^2 on the matrix cores (ell_band16.hip): the kernel of the SP2
// iteration when every matrix of the rotation fits 2^31 bytes; with_u false:
// X^2 only (a standalone product without the 2X - X^2 output)
bool x2_band16_fits(int N, int SW, int elem_bytes);
template <typename T>
hipError_t launch_x2_band16(int N, SpanRot3<T> spans, const SP2State *st, T tau, const StepScratch &s,
                            int32_t *fallback, hipStream_t stream, bool with_u = true);
// The SP2 iteration on the span form in two launches (ell_band16.hip): X^2,
// the row outputs and 64-row partial sums (needs x2_band16_fits and s sized for
// N rows: s.nq == ceil(N / 64) <= 16384); then the upper reduction levels and
// the decision in one workgroup, `publish` (mapped pinned host memory or null)
// receiving the state afterwards.
template <typename T>
hipError_t launch_x2_band16_part(int N, SpanRot3<T> spans, const SP2State *st, T tau, const StepScratch &s,
                                 hipStream_t stream);
hipError_t launch_step_final64(SP2State *st, const SP2Cfg &cfg, const SP2Hist &h, const StepScratch &s,
                               SP2State *publish, hipStream_t stream);
// The symmetric span iteration on the matrix cores in one launch
// (ell_sym16.hip): the product writes only the iterate of the branch fixed
// beforehand (st->up_next); the workgroup that finishes last reduces the
// traces, the norm and Tr X', Tr X'^2 of that iterate and takes the decision,
// publishing the state to `publish` (mapped pinned host memory, or null).
// Needs x2_band16_fits, spans whose rows start on a multiple of
// 16 / sizeof(T) columns and hold a multiple of that, X bitwise symmetric, s
// sized for N rows with s.ticket zero.  The seed sets the branch of the first
// product of the current X from its traces.
template <typename T>
hipError_t launch_x2_sym_step(int N, SpanRot3<T> spans, SP2State *st, T tau, const StepScratch &s,
                              const SP2Cfg &cfg, const SP2Hist &h, SP2State *publish, hipStream_t stream);
template <typename T>
hipError_t launch_sym_seed(int N, SpanRot3<T> spans, SP2State *st, const SP2Cfg &cfg, const StepScratch &s,
                           hipStream_t stream);
template <typename T>
hipError_t launch_x2_band16_batch(int ngroups16, SpanRot3<T> spans, const int32_t *grp_inst, const int32_t *inst_r0,
                                  const int32_t *inst_rows, const SP2State *states, int32_t phase32, const T *taus,
                                  const StepScratch *ss, int32_t *flags, bool sym, hipStream_t stream);
// Row intervals of an ELLPACK matrix: len[i] (or null), flags |= 4 when a value
// is an exact zero; with maxlen: the longest interval, and with sums:
// sums[0] += stored entries, sums[1] += interval lengths.
template <typename T>
hipError_t launch_ell_extent(int N, EllView<T> A, int32_t *len, int32_t *flags, int32_t *maxlen,
                             unsigned long long *sums, hipStream_t stream);
// Span form pays for every position of a row's interval; a standalone product
// whose operand fills less than this share of its intervals (stored entries /
// interval positions) goes to the ELLPACK kernels.  (Not so in SP2, whose
// iterates fill their intervals.)
constexpr int kMinSpanFillInv = 64;
// (rows start on a multiple of `align` columns and hold a multiple of `align`
// positions, zeros filling the ends; align a power of two)
template <typename T>
hipError_t launch_ell_to_span(int N, EllView<T> A, SpanView<T> S, hipStream_t stream, int align = 1);
// Span alignment of the symmetric iteration: 16-byte runs of either precision
constexpr int kSymAlign = 4;
template <typename TS, typename TD>
hipError_t launch_span_to_ell(int N, SpanView<TS> S, EllView<TD> A, int32_t *wmax, hipStream_t stream);
// batched step: ngroups groups of kGroupRows rows; group -> instance; instance m's
// rows start at inst_r0[m] (a multiple of kBatchAlign) and it has inst_rows[m]
// of them (local columns); per-instance state, drop tolerance, row-output
// scratch view and fallback flag.  Takes the matrix-core kernel when the stack
// fits its 2^31-byte buffer range and matrix_cores is set, else the
// register-tiled VALU kernel (the same results).  sym: every instance's X is
// bitwise symmetric (the matrix-core kernel then reads its A operand through
// the symmetry).
template <typename T>
hipError_t launch_x2_band_batch(int ngroups, SpanRot3<T> spans, const int32_t *grp_inst, const int32_t *inst_r0,
                                const int32_t *inst_rows, const SP2State *states, int32_t phase32, const T *taus,
                                const StepScratch *ss, int32_t *flags, hipStream_t stream,
                                bool matrix_cores = true, bool sym = false);
constexpr int kGroupRows = 8;   // rows per wavefront of the register-tiled span step kernel
constexpr int kBatchAlign = 16; // instance alignment in a batch: a whole number of both kernels' row groups
template <typename TS, typename TD>
hipError_t launch_span_copy(int N, SpanView<TS> S, SpanView<TD> D, hipStream_t stream);

}  // namespace ellsp2
