// The SP2 loop's decision after each X^2 product, taken on the device by one
// thread: record the iteration's traces and norm, stop on convergence,
// stagnation, the iteration limit, a phase switch (mixed precision) or an
// overflow, else choose the branch and rotate the buffers.  Shared by the
// separate decision kernel and the fused span-form iteration.  Device-only.
#pragma once

#include <hip/hip_runtime.h>

#include "ell_internal.h"
#include "../../include/ellsp2.h"

namespace ellsp2 {
namespace sp2dev {

__device__ inline bool stalled(const double *h, int n)
{
  if (n < 3) return false;
  if (!(h[n - 3] < 1e-4)) return false;
  const double now = h[n] < h[n - 1] ? h[n] : h[n - 1];
  const double before = h[n - 2] < h[n - 3] ? h[n - 2] : h[n - 3];
  return now >= before;
}

// One decision of the SP2 loop, taken on the device by a single thread.
__device__ inline void decide(SP2State *st, const SP2Cfg &cfg, const SP2Hist &h, const StepScratch &s)
{
  const int n = st->iter;
  if (s.flags && (*s.flags & 1)) {  // some row group was not computed: redo on the ELLPACK pipeline
    st->status = ST_FALLBACK;
    st->stop = 1;
    return;
  }
  const double trx = s.out[0], trx2 = s.out[1], eta2 = s.out[2];
  st->trx = trx;
  st->trx2 = trx2;
  st->eta2 = eta2;
  st->wy_max = s.outw[0];
  st->wu_max = s.outw[1];
  h.trx[n] = trx;
  h.trx2[n] = trx2;
  h.eta2[n] = eta2;
  h.maxw[n] = s.outw[0];
  h.prec[n] = (int8_t)st->phase32;
  h.up[n] = -1;
  h.nnzx[n] = st->nnz_cur;
  h.nnzy[n] = s.outn[0];
  const bool stall = cfg.stall && stalled(h.eta2 + st->phase_start, n - st->phase_start);
  if (st->phase32) {
    if (eta2 < cfg.switch2 || stall) {
      st->phase_start = n + 1;
      st->iter = n + 1;
      st->stop = 1;
      st->status = (n + 1 == cfg.max_iter) ? ELL_ENOCONV : ST_SWITCH;
      return;
    }
  } else {
    if (eta2 < cfg.target2 && st->fp64_updates >= (cfg.mixed ? cfg.tail : 0)) {
      st->status = ELL_OK;
      st->stop = 1;
      st->iter = n + 1;
      return;
    }
    if (stall) {
      st->status = ELL_ENOCONV;
      st->stop = 1;
      st->iter = n + 1;
      return;
    }
  }
  if (n + 1 == cfg.max_iter) {
    st->status = ELL_ENOCONV;
    st->stop = 1;
    st->iter = n + 1;
    return;
  }
  const double a = fabs(2.0 * trx - trx2 - cfg.n_occ);
  const double b = fabs(trx2 - cfg.n_occ);
  const bool up = a < b;
  const int need = cfg.span ? (up ? s.outw[3] : s.outw[2]) : (up ? s.outw[1] : s.outw[0]);
  if (need > (cfg.span ? st->sw : st->cap)) {
    st->status = ELL_EOVERFLOW;
    st->need_width = need;
    st->stop = 1;
    return;
  }
  h.up[n] = up ? 1 : 0;
  const int c = st->cur;
  st->cur = up ? (c == 0 ? 2 : c - 1) : (c == 2 ? 0 : c + 1);
  if (!st->phase32) st->fp64_updates += 1;
  st->nnz_cur = up ? s.outn[1] : s.outn[0];
  st->iter = n + 1;
}

__device__ inline bool closer_up(double trx, double trx2, double n_occ)
{
  return fabs(2.0 * trx - trx2 - n_occ) < fabs(trx2 - n_occ);
}

__device__ inline bool same_bits(double a, double b) { return __double_as_longlong(a) == __double_as_longlong(b); }

// The branch of the next product from the traces of the current X (Tr X and
// the unpruned Tr X^2, the latter from the chains of squares of its rows).
__device__ inline void seed_sym(SP2State *st, const SP2Cfg &cfg, double trx, double trx2)
{
  st->ptrx = trx;
  st->ptrx2 = trx2;
  st->up_next = closer_up(trx, trx2, cfg.n_occ) ? 1 : 0;
}

// decide() for the symmetric span iteration, whose product wrote only the
// iterate of the branch st->up_next: the same record, stop, stall, switch,
// limit and overflow rules; the branch taken is the one fixed beforehand,
// which equals the rule's choice on this product's traces because those
// traces equal the predicted ones (checked: a difference stops the solve
// with ST_MISPREDICT).  s.out[3], s.out[4]: Tr X', Tr X'^2 of the written
// iterate, which fix the next branch.  s.outw: widest pruned X^2 row, widest
// iterate row, longest iterate interval; s.outn: entries of the pruned X^2
// and of the iterate.  The deciding thread holds them in registers (SymOut),
// with the norms of the three products before this one, loaded ahead for the
// stall rule.
struct SymOut {
  double sum[5];    // Tr X, Tr X^2 (unpruned), eta^2, Tr X', Tr X'^2
  int32_t w[3];     // widest pruned X^2 row, widest iterate row, longest iterate interval
  int64_t n[2];     // entries of the pruned X^2 and of the iterate
  double prev[3];   // eta^2 of products n - 1, n - 2, n - 3 (when within the phase)
};

// stalled() with the current norm and the three before it from registers;
// m = products of the phase before this one
__device__ inline bool stalled_sym(const SymOut &o, int m)
{
  if (m < 3) return false;
  if (!(o.prev[2] < 1e-4)) return false;
  const double now = o.sum[2] < o.prev[0] ? o.sum[2] : o.prev[0];
  const double before = o.prev[1] < o.prev[2] ? o.prev[1] : o.prev[2];
  return now >= before;
}

__device__ inline void decide_sym(SP2State *st, const SP2Cfg &cfg, const SP2Hist &h, const SymOut &o)
{
  const int n = st->iter;
  const double trx = o.sum[0], trx2 = o.sum[1], eta2 = o.sum[2];
  if (!same_bits(trx, st->ptrx) || !same_bits(trx2, st->ptrx2)) {
    // the product's own traces are recorded; D keeps X_n
    h.trx[n] = trx;
    h.trx2[n] = trx2;
    h.eta2[n] = eta2;
    h.maxw[n] = o.w[0];
    h.prec[n] = (int8_t)st->phase32;
    h.up[n] = -1;
    h.nnzx[n] = st->nnz_cur;
    h.nnzy[n] = o.n[0];
    st->trx = trx;
    st->trx2 = trx2;
    st->eta2 = eta2;
    st->iter = n + 1;
    st->status = ST_MISPREDICT;
    st->stop = 1;
    return;
  }
  st->trx = trx;
  st->trx2 = trx2;
  st->eta2 = eta2;
  st->wy_max = o.w[0];
  st->wu_max = o.w[1];
  h.trx[n] = trx;
  h.trx2[n] = trx2;
  h.eta2[n] = eta2;
  h.maxw[n] = o.w[0];
  h.prec[n] = (int8_t)st->phase32;
  h.up[n] = -1;
  h.nnzx[n] = st->nnz_cur;
  h.nnzy[n] = o.n[0];
  const bool stall = cfg.stall && stalled_sym(o, n - st->phase_start);
  if (st->phase32) {
    if (eta2 < cfg.switch2 || stall) {
      st->phase_start = n + 1;
      st->iter = n + 1;
      st->stop = 1;
      st->status = (n + 1 == cfg.max_iter) ? ELL_ENOCONV : ST_SWITCH;
      return;
    }
  } else {
    if (eta2 < cfg.target2 && st->fp64_updates >= (cfg.mixed ? cfg.tail : 0)) {
      st->status = ELL_OK;
      st->stop = 1;
      st->iter = n + 1;
      return;
    }
    if (stall) {
      st->status = ELL_ENOCONV;
      st->stop = 1;
      st->iter = n + 1;
      return;
    }
  }
  if (n + 1 == cfg.max_iter) {
    st->status = ELL_ENOCONV;
    st->stop = 1;
    st->iter = n + 1;
    return;
  }
  const bool up = st->up_next != 0;
  if (o.w[2] > st->sw) {
    st->status = ELL_EOVERFLOW;
    st->need_width = o.w[2];
    st->stop = 1;
    return;
  }
  h.up[n] = up ? 1 : 0;
  const int c = st->cur;
  st->cur = up ? (c == 0 ? 2 : c - 1) : (c == 2 ? 0 : c + 1);
  if (!st->phase32) st->fp64_updates += 1;
  st->nnz_cur = o.n[1];
  st->iter = n + 1;
  seed_sym(st, cfg, o.sum[3], o.sum[4]);
}

}  // namespace sp2dev
}  // namespace ellsp2
