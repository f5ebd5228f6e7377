// Host loops of the multi-rhs even-odd CG solvers.
//
// The whole solve stays on the device; the host enqueues the iteration and only looks at the
// per-rhs residual state at polls (Section 2 keeps the solver on the GPU and moves only the set
// of residuals to the host per iteration; here a poll every `check_every` iterations, with the
// per-rhs decisions taken on the device between polls).
//
// Plain FP64 CG: textbook CG per rhs on M = m^2 - D_eo D_oe.  When a rhs's iterated residual
// drops below tol its true residual is recomputed in FP64; it stops if that meets tol and
// restarts from its current x otherwise.
//
// Mixed precision: FP32 Dslash (FP32 or FP16 link storage) and FP32 vectors in the body, FP64
// solution x, FP64 reductions, and every `reliable_every` iterations (and whenever a rhs's
// iterated residual reaches tol) a reliable update: x += xhat in FP64, r = b - M x with FP64
// links, the body residual replaced by (float) r, xhat = 0, search direction kept (Sleijpen and
// van der Vorst 1996).  A rhs stops when its FP64 true residual meets tol.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "cg_state.hpp"
#include "internal.hpp"

int fcg_nn_solve(hisq_ctx *ctx, double mass, int n, const void *b, void *x, const hisq_cg_params *p,
                 hisq_cg_stats *st, CGState *S, CGState *hS, double *partial);

namespace {

bool cg_trace() {
  static const bool on = [] {
    const char *e = getenv("HISQ_CG_TRACE");
    return e && atoi(e) != 0;
  }();
  return on;
}

// HISQ_CG_FUSED_REDUCTIONS=0 keeps the alpha and beta reductions as launches of their own on
// every lattice (read at each solve; the results are the same bits either way).
bool fused_reductions() {
  const char *e = getenv("HISQ_CG_FUSED_REDUCTIONS");
  return !(e && e[0] == '0' && e[1] == 0);
}

// What the final residual needs of a rhs that left the bundle.
struct SlotRecord {
  int iters = 0, replacements = 0, status = 0;
  double bnorm2 = 0.0;
};

// Slot src[j] of the state moves to slot j for j < m; the slots from m on are cleared.
void permute_state(CGState &s, const int *src, int m) {
  const CGState o = s;
  for (int j = 0; j < HISQ_MAX_RHS; ++j) {
    if (j >= m) {
      s.active[j] = s.hit[j] = s.sel[j] = s.fin[j] = 0;
      continue;
    }
    const int k = src[j];
    s.rho[j] = o.rho[k];
    s.pq[j] = o.pq[k];
    s.alpha[j] = o.alpha[k];
    s.beta[j] = o.beta[k];
    s.bnorm2[j] = o.bnorm2[k];
    s.rr[j] = o.rr[k];
    s.rr_true[j] = o.rr_true[k];
    s.drift[j] = o.drift[k];
    for (int c = 0; c < 2; ++c) {
      s.calpha[2 * j + c] = o.calpha[2 * k + c];
      s.cbeta[2 * j + c] = o.cbeta[2 * k + c];
    }
    s.active[j] = o.active[k];
    s.hit[j] = o.hit[k];
    s.sel[j] = o.sel[k];
    s.fin[j] = o.fin[k];
    s.status[j] = o.status[k];
    s.iters[j] = o.iters[k];
    s.replacements[j] = o.replacements[k];
  }
}

// The state of rhs 0..n-1 in the caller's order from the records of the rhs that left the bundle,
// ready for the final residual of every rhs.
void restore_state(CGState &s, const SlotRecord *done, int n) {
  for (int i = 0; i < HISQ_MAX_RHS; ++i) {
    s.active[i] = s.hit[i] = s.sel[i] = 0;
    s.fin[i] = i < n;
    if (i >= n) continue;
    s.iters[i] = done[i].iters;
    s.replacements[i] = done[i].replacements;
    s.status[i] = done[i].status;
    s.bnorm2[i] = done[i].bnorm2;
  }
}

struct Vecs {
  void *r = nullptr, *p = nullptr, *q = nullptr, *t = nullptr, *xh = nullptr;
  void *mx64 = nullptr, *t64 = nullptr;
};

}  // namespace

int cg_poll(hisq_ctx *ctx, CGState *S, CGState *hS) {
  HIPCHK(ctx, hipMemcpyAsync(hS, S, sizeof(CGState), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return HISQ_OK;
}
#define poll cg_poll

// mx64 = M x64 (FP64 links) for the rhs selected by mask.
int apply_m64(hisq_ctx *ctx, double mass, int n, const void *x64, void *t64, void *mx64,
              const int *mask) {
  RETCHK(launch_dslash(ctx, 1, HISQ_F64, n, x64, t64, false, 0.0, nullptr, nullptr, nullptr, mask));
  RETCHK(launch_dslash(ctx, 0, HISQ_F64, n, t64, mx64, true, mass * mass, x64, nullptr, nullptr, mask));
  return HISQ_OK;
}

// One bundle iteration of (F)CG's operator part: t = D_oe p; q = m^2 p - D_eo t; <p, q>.
int cg_apply_op(hisq_ctx *ctx, int op_prec, double mass, int n, const void *p, void *t, void *q,
                double *partial, int *nblk, const int *active) {
  RETCHK(launch_dslash(ctx, 1, op_prec, n, p, t, false, 0.0, nullptr, nullptr, nullptr, active));
  RETCHK(launch_dslash(ctx, 0, op_prec, n, t, q, true, mass * mass, p, partial, nblk, active));
  return HISQ_OK;
}

// Final bookkeeping shared by all solvers: FP64 true residual of every rhs, stats.
int cg_finish(hisq_ctx *ctx, double mass, int n, const void *b, void *x, double tol, CGState *S,
              CGState *hS, double *partial, hisq_cg_stats *st, bool *all_conv) {
  const Geometry &g = ctx->g;
  void *t64, *mx64;
  RETCHK(ws_get(ctx, WS_CG5, size_t(n) * 3 * g.vh * 16, &mx64));
  RETCHK(ws_get(ctx, WS_CG6, size_t(n) * 3 * g.vh * 16, &t64));
  RETCHK(apply_m64(ctx, mass, n, x, t64, mx64, S->fin));
  RETCHK(cg_replace_r(ctx, HISQ_F64, b, mx64, nullptr, nullptr, S, S->fin, n, partial));
  RETCHK(cg_reduce_true(ctx, partial, S, n, tol * tol, 1));
  RETCHK(poll(ctx, S, hS));
  bool ok = true;
  long long site_rhs = 0;
  for (int i = 0; i < n; ++i) {
    double res = hS->bnorm2[i] > 0 ? std::sqrt(hS->rr_true[i] / hS->bnorm2[i]) : std::sqrt(hS->rr_true[i]);
    bool conv = std::isfinite(res) && res <= tol;
    ok = ok && conv;
    if (st) {
      if (st->iters) st->iters[i] = hS->iters[i];
      if (st->true_resid) st->true_resid[i] = res;
      if (st->converged) st->converged[i] = conv ? 1 : 0;
    }
    site_rhs += 2LL * g.vh * (hS->iters[i] + hS->replacements[i]);
  }
  if (st) {
    st->dslash_site_rhs = site_rhs;
    st->peak_bytes = ctx->dev_peak;
  }
  *all_conv = ok;
  return HISQ_OK;
}

// A bundle that shrinks from n_from to n_to right-hand sides gives (prec, n_to), plain and fused
// forms, the launch configuration of (prec, n_from) where n_to has none yet, so that the shrunk
// bundle does not autotune in the middle of the solve (one autotune takes seconds on large
// lattices).  A configuration that serves n_from rhs serves fewer (the launch only skips the
// missing rhs); entries n_to already has (tuned, loaded, forced) are kept, and the borrowed ones
// are not saved by hisq_save_tuning.
static void borrow_launch(hisq_ctx *ctx, int prec, int n_from, int n_to) {
  if (n_to < 1 || n_to >= n_from || n_from > HISQ_MAX_RHS) return;
  for (int e = 0; e < 2; ++e) {
    TuneEntry &to = ctx->tune[prec][n_to][e];
    const TuneEntry &from = ctx->tune[prec][n_from][e];
    if (to.state != TuneEntry::NONE || from.state == TuneEntry::NONE) continue;
    to.cfg = from.cfg;
    to.state = TuneEntry::HEURISTIC;
    to.ms = 0.f;
  }
}

// snap_x: optional device [n_snap][n][3][V/2] complex128 receiving x after iterations
// 0, snap_every, 2 snap_every, ... (plain FP64 solver only); *n_taken = snapshots written.
int cg_solve(hisq_ctx *ctx, double mass, int n, const void *b, void *x, const hisq_cg_params *prm,
             hisq_cg_stats *st, CGState *S, CGState *hS, double *partial, void *snap_x,
             int n_snap, int snap_every, int *n_taken) {
  const Geometry &g = ctx->g;
  const bool mixed = prm->kind == HISQ_CG_MIXED;
  const int body = mixed ? HISQ_F32 : HISQ_F64;
  int op_prec = mixed ? prm->link_prec : HISQ_F64;
  const size_t vb = size_t(n) * 3 * g.vh * cplx_bytes(body);
  const double tol2 = prm->tol * prm->tol;
  const bool fuse_beta = fused_reductions() && cg_fuse_beta(ctx);
  const bool fuse_alpha = fused_reductions() && cg_fuse_alpha(ctx);
  // the r pass's ||r||^2 partials, apart from the <p, Mp> partials when it also sums those
  double *rr_partial = fuse_alpha ? partial + size_t(n) * dslash_partials(g) : partial;
  const int check_every = prm->check_every > 0 ? prm->check_every : 8;
  const int reliable_every = prm->reliable_every > 0 ? prm->reliable_every : 50;
  Vecs v;
  RETCHK(ws_get(ctx, WS_CG0, vb, &v.r));
  RETCHK(ws_get(ctx, WS_CG1, vb, &v.p));
  RETCHK(ws_get(ctx, WS_CG2, vb, &v.q));
  RETCHK(ws_get(ctx, WS_CG3, vb, &v.t));
  if (mixed) {
    RETCHK(ws_get(ctx, WS_CG4, vb, &v.xh));
    RETCHK(ws_get(ctx, WS_CG5, size_t(n) * 3 * g.vh * 16, &v.mx64));
    RETCHK(ws_get(ctx, WS_CG6, size_t(n) * 3 * g.vh * 16, &v.t64));
  }

  // ---- initial residual ----
  RETCHK(cg_init_state(ctx, b, S, n, partial));
  RETCHK(cg_select(ctx, S, n, 1));
  RETCHK(cg_zero(ctx, HISQ_F64, x, S->sel, 1, n));  // x = 0 where b = 0
  if (prm->use_x0) {
    void *mx = mixed ? v.mx64 : v.q;
    void *tt = mixed ? v.t64 : v.t;
    RETCHK(apply_m64(ctx, mass, n, x, tt, mx, S->sel));
    RETCHK(cg_replace_r(ctx, body, b, mx, v.r, v.p, S, S->sel, n, partial));
  } else {
    RETCHK(cg_zero(ctx, HISQ_F64, x, nullptr, 0, n));
    void *zero64 = mixed ? v.mx64 : v.q;
    RETCHK(cg_zero(ctx, HISQ_F64, zero64, nullptr, 0, n));
    RETCHK(cg_replace_r(ctx, body, b, zero64, v.r, v.p, S, S->sel, n, partial));
  }
  RETCHK(cg_set_rho(ctx, partial, S, n, tol2));
  if (mixed) RETCHK(cg_zero(ctx, HISQ_F32, v.xh, nullptr, 0, n));
  RETCHK(poll(ctx, S, hS));
  for (int i = 0; i < n; ++i)
    if (hS->status[i] == CG_NONFINITE)
      return set_err(ctx, HISQ_ERR_NONFINITE, "hisq_cg_mrhs: non-finite source %d", i);

  // host-side stagnation bookkeeping (mixed): best true residual and polls without progress
  double best[HISQ_MAX_RHS];
  int stale[HISQ_MAX_RHS], drifting[HISQ_MAX_RHS];
  int last_rep[HISQ_MAX_RHS];
  for (int i = 0; i < n; ++i) {
    best[i] = hS->rr_true[i];
    stale[i] = drifting[i] = 0;
    last_rep[i] = 0;
  }
  int switch_iter = -1;
  // FP16-link rate test: (iteration, mean log relative true residual of the live rhs) at the
  // periodic replacements, and the best rate so far
  int rate_it[kRateWindow + 1];
  double rate_l[kRateWindow + 1];
  int rate_len = 0, rate_reps = 0, rate_live = -1;
  double rate_best = 0.0;

  // Compaction of the bundle (converged rhs stop costing work, Section 2): the iteration runs on
  // ns slots, slot k holding rhs map[k].  Once a quarter of the slots have finished, the finished
  // ones hand their solution to the caller's x and the live ones move to the front, so every
  // kernel runs on a bundle of live rhs only (with the launch configuration tuned for its size).
  // Until the first repack the slots are the caller's rhs and xw, bw are the caller's x, b; from
  // then on they are slot-ordered copies in the workspace.  Each rhs's arithmetic does not depend
  // on its slot or on the bundle size, so a repack does not change any result.
  const bool can_compact = !prm->no_compaction && !snap_x;
  int map[HISQ_MAX_RHS];
  for (int i = 0; i < n; ++i) map[i] = i;
  int ns = n;
  void *xw = x;
  const void *bw = b;
  SlotRecord done[HISQ_MAX_RHS];
  int compactions = 0;
  const size_t xb1 = size_t(3) * g.vh * 16;                // one FP64 rhs
  const size_t vb1 = size_t(3) * g.vh * cplx_bytes(body);  // one rhs of a body vector
  auto slot_copy = [&](void *base, size_t bytes, int from, int to) -> int {
    char *c = static_cast<char *>(base);
    HIPCHK(ctx, hipMemcpyAsync(c + size_t(to) * bytes, c + size_t(from) * bytes, bytes,
                               hipMemcpyDeviceToDevice, ctx->stream));
    return HISQ_OK;
  };
  auto hand_back = [&](int k) -> int {  // slot k's solution to the caller's x, its statistics kept
    HIPCHK(ctx, hipMemcpyAsync(static_cast<char *>(x) + size_t(map[k]) * xb1,
                               static_cast<const char *>(xw) + size_t(k) * xb1, xb1,
                               hipMemcpyDeviceToDevice, ctx->stream));
    done[map[k]] = SlotRecord{hS->iters[k], hS->replacements[k], hS->status[k], hS->bnorm2[k]};
    return HISQ_OK;
  };
  auto repack = [&]() -> int {
    if (xw == x) {  // first repack: slot-ordered copies of x and b
      void *xc, *bc;
      RETCHK(ws_get(ctx, WS_CMPX, size_t(n) * xb1, &xc));
      RETCHK(ws_get(ctx, WS_CMPB, size_t(n) * xb1, &bc));
      HIPCHK(ctx, hipMemcpyAsync(xc, x, size_t(ns) * xb1, hipMemcpyDeviceToDevice, ctx->stream));
      HIPCHK(ctx, hipMemcpyAsync(bc, b, size_t(ns) * xb1, hipMemcpyDeviceToDevice, ctx->stream));
      xw = xc;
      bw = bc;
    }
    if (mixed) {  // finished slots: x += xhat (live slots keep their xhat, which moves with them)
      for (int k = 0; k < HISQ_MAX_RHS; ++k) hS->sel[k] = k < ns && !hS->active[k];
      HIPCHK(ctx, hipMemcpyAsync(S, hS, sizeof(CGState), hipMemcpyHostToDevice, ctx->stream));
      RETCHK(cg_accum_x(ctx, xw, v.xh, S->sel, ns));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));  // the upload has read hS before it changes
    }
    int src[HISQ_MAX_RHS], m = 0;
    for (int k = 0; k < ns; ++k) {
      if (hS->active[k])
        src[m++] = k;
      else
        RETCHK(hand_back(k));
    }
    // live slots to the front, in order (slot src[j] >= j, so the in-place moves never overwrite
    // a slot that is still to be moved)
    int newmap[HISQ_MAX_RHS];
    for (int j = 0; j < m; ++j) {
      const int k = src[j];
      newmap[j] = map[k];
      best[j] = best[k];
      stale[j] = stale[k];
      drifting[j] = drifting[k];
      last_rep[j] = last_rep[k];
      if (k == j) continue;
      RETCHK(slot_copy(v.r, vb1, k, j));
      RETCHK(slot_copy(v.p, vb1, k, j));
      if (mixed) RETCHK(slot_copy(v.xh, vb1, k, j));
      RETCHK(slot_copy(xw, xb1, k, j));
      RETCHK(slot_copy(const_cast<void *>(bw), xb1, k, j));
    }
    for (int j = 0; j < m; ++j) map[j] = newmap[j];
    for (int pr : {HISQ_F64, HISQ_F32, HISQ_F16}) borrow_launch(ctx, pr, ns, m);
    permute_state(*hS, src, m);
    HIPCHK(ctx, hipMemcpyAsync(S, hS, sizeof(CGState), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));  // hS is read and written by the host again
    ns = m;
    ++compactions;
    return HISQ_OK;
  };

  auto reliable = [&](int all) -> int {
    RETCHK(cg_select(ctx, S, ns, all));
    if (mixed) {
      RETCHK(cg_accum_x(ctx, xw, v.xh, S->sel, ns));
      RETCHK(apply_m64(ctx, mass, ns, xw, v.t64, v.mx64, S->sel));
      RETCHK(cg_replace_r(ctx, body, bw, v.mx64, v.r, nullptr, S, S->sel, ns, partial));
    } else {  // verify, restart from x if the true residual misses tol
      RETCHK(apply_m64(ctx, mass, ns, xw, v.t, v.q, S->sel));
      RETCHK(cg_replace_r(ctx, body, bw, v.q, v.r, v.p, S, S->sel, ns, partial));
    }
    RETCHK(cg_reduce_true(ctx, partial, S, ns, tol2, 0));
    return HISQ_OK;
  };

  int it = 0;
  int trace_rep = 0;
  int nactive = 0;
  for (int i = 0; i < n; ++i) nactive += hS->active[i];
  int reps = 0;
  int taken = 0;
  const size_t xbytes = size_t(n) * 3 * g.vh * 16;
  auto snapshot = [&]() -> int {
    if (snap_x && !mixed && taken < n_snap && snap_every > 0 && it % snap_every == 0) {
      HIPCHK(ctx, hipMemcpyAsync(static_cast<char *>(snap_x) + taken * xbytes, x, xbytes,
                                 hipMemcpyDeviceToDevice, ctx->stream));
      ++taken;
    }
    return HISQ_OK;
  };
  RETCHK(snapshot());
  while (nactive > 0 && it < prm->max_iter) {
    int nblk_d = 0;
    RETCHK(cg_apply_op(ctx, op_prec, mass, ns, v.p, v.t, v.q, partial, &nblk_d, S->active));
    if (fuse_alpha) {
      RETCHK(cg_update_r_alpha(ctx, body, v.r, v.q, S, ns, partial, nblk_d, rr_partial));
    } else {
      RETCHK(cg_reduce_alpha(ctx, partial, nblk_d, S, ns));
      RETCHK(cg_update_r(ctx, body, v.r, v.q, S, ns, rr_partial));
    }
    if (fuse_beta) {
      RETCHK(cg_update_px_beta(ctx, body, !mixed, mixed ? v.xh : xw, v.r, v.p, S, ns, rr_partial, tol2));
    } else {
      RETCHK(cg_reduce_beta(ctx, rr_partial, cg_pass_nblk(ctx), S, ns, tol2));
      RETCHK(cg_update_px(ctx, body, !mixed, mixed ? v.xh : xw, v.r, v.p, S, ns));
    }
    ++it;
    RETCHK(snapshot());
    if (mixed && it % reliable_every == 0) {
      RETCHK(reliable(1));
      ++reps;
    }
    if (it % check_every == 0 || it == prm->max_iter) {
      RETCHK(poll(ctx, S, hS));
      bool any_hit = false;
      for (int i = 0; i < ns; ++i) any_hit = any_hit || (hS->active[i] && hS->hit[i]);
      if (any_hit) {
        RETCHK(reliable(0));
        ++reps;
        RETCHK(poll(ctx, S, hS));
      }
      nactive = 0;
      for (int i = 0; i < ns; ++i) nactive += hS->active[i];
      if (cg_trace() && hS->replacements[0] != trace_rep) {
        // diagnostic (HISQ_CG_TRACE=1): the true residual and the true / iterated residual ratio
        // of slot 0 at each of its residual replacements
        trace_rep = hS->replacements[0];
        fprintf(stderr, "hisq cg trace: it %d links %s rhs0 true %.4e drift %.4f active %d\n", it,
                op_prec == HISQ_F16 ? "f16" : (op_prec == HISQ_F32 ? "f32" : "f64"),
                std::sqrt(hS->rr_true[0] / (hS->bnorm2[0] > 0 ? hS->bnorm2[0] : 1.0)),
                std::sqrt(hS->drift[0]), nactive);
      }
      if (mixed && op_prec == HISQ_F16 && ctx->links[HISQ_F32].base) {
        // FP16-link error dominating (the true residual drifts away from the iterated one well
        // above the FP32 floor) or a stalled true residual: the inner operator moves to the FP32
        // links for the rest of the solve (the FP16 rounding of ~5e-4 can slow CG a lot on
        // ill-conditioned systems).
        bool to_f32 = false;
        for (int i = 0; i < ns; ++i) {
          if (!hS->active[i] || hS->replacements[i] == last_rep[i]) continue;
          last_rep[i] = hS->replacements[i];
          if (hS->drift[i] > kDriftRatio && hS->rr_true[i] > kDriftFloor2 * hS->bnorm2[i]) {
            to_f32 = to_f32 || ++drifting[i] >= kDriftUpdates;
          } else {
            drifting[i] = 0;
          }
          if (hS->rr_true[i] < kStallDrop * best[i]) {
            best[i] = hS->rr_true[i];
            stale[i] = 0;
          } else if (++stale[i] >= kStallUpdates) {
            to_f32 = true;
          }
        }
        if (reps != rate_reps && nactive > 0) {  // a periodic replacement since the last poll
          rate_reps = reps;
          double l = 0.0;
          for (int i = 0; i < ns; ++i)
            if (hS->active[i]) l += 0.5 * std::log(hS->rr_true[i] / hS->bnorm2[i]);
          l /= nactive;
          if (nactive != rate_live) rate_len = 0;  // the set of live rhs changed: start again
          rate_live = nactive;
          if (rate_len == kRateWindow + 1) {
            for (int k = 0; k < kRateWindow; ++k) {
              rate_it[k] = rate_it[k + 1];
              rate_l[k] = rate_l[k + 1];
            }
            --rate_len;
          }
          rate_it[rate_len] = it;
          rate_l[rate_len] = l;
          ++rate_len;
          if (rate_len == kRateWindow + 1) {
            const double rate = (rate_l[0] - rate_l[kRateWindow]) / double(rate_it[kRateWindow] - rate_it[0]);
            rate_best = std::max(rate_best, rate);
            if (rate < kRateFrac * rate_best && l > std::log(kRateNearTol * prm->tol)) to_f32 = true;
          }
        }
        if (to_f32) {
          op_prec = HISQ_F32;
          switch_iter = it;
        }
      }
      if (can_compact && nactive > 0 && ns - nactive >= std::max(1, ns / 4)) RETCHK(repack());
    }
  }
  if (mixed) {  // fold the last FP32 correction of every rhs into x
    RETCHK(cg_accum_x(ctx, xw, v.xh, S->fin, ns));
  }
  if (xw != x) {
    // compacted: the remaining slots' solutions to the caller's x, and the per-rhs state in the
    // caller's order for the final residual
    RETCHK(poll(ctx, S, hS));
    for (int k = 0; k < ns; ++k) RETCHK(hand_back(k));
    restore_state(*hS, done, n);
    HIPCHK(ctx, hipMemcpyAsync(S, hS, sizeof(CGState), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  if (n_taken) *n_taken = taken;
  bool ok = false;
  RETCHK(cg_finish(ctx, mass, n, b, x, prm->tol, S, hS, partial, st, &ok));
  if (st) {
    st->total_iters = it;
    st->reliable_updates = reps;
    st->link_switch_iter = switch_iter;
    st->compactions = compactions;
    if (st->fell_back)
      for (int i = 0; i < n; ++i) st->fell_back[i] = 0;
  }
  if (!ok) return set_err(ctx, HISQ_ERR_NOCONV, "hisq_cg_mrhs: some rhs missed tol %.3g", prm->tol);
  return HISQ_OK;
}

extern "C" int hisq_cg_mrhs(hisq_ctx *ctx, double mass, int n, const void *b, void *x,
                            const hisq_cg_params *prm, hisq_cg_stats *st) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!b || !x || !prm) return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: null pointer");
  if (b == x) return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: b and x alias");
  if (!elem_aligned(b, 16) || !elem_aligned(x, 16))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: b and x must be aligned to 16 bytes");
  if (n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: n = %d outside 1..%d", n, HISQ_MAX_RHS);
  if (!(prm->tol > 0) || prm->max_iter < 1 || !std::isfinite(mass))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: need tol > 0, max_iter >= 1, finite mass");
  if (prm->kind != HISQ_CG_F64 && prm->kind != HISQ_CG_MIXED && prm->kind != HISQ_FCG_NN)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: bad solver kind %d", prm->kind);
  if (prm->kind != HISQ_CG_F64 && prm->link_prec != HISQ_F32 && prm->link_prec != HISQ_F16)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_cg_mrhs: link_prec must be HISQ_F32 or HISQ_F16");
  if (!ctx->links_loaded) return set_err(ctx, HISQ_ERR_STATE, "hisq_cg_mrhs: no links loaded");
  if (!ctx->links[HISQ_F64].base)
    return set_err(ctx, HISQ_ERR_STATE, "hisq_cg_mrhs: the FP64 link copy is required");
  if (prm->kind != HISQ_CG_F64 && !ctx->links[prm->link_prec].base)
    return set_err(ctx, HISQ_ERR_STATE, "hisq_cg_mrhs: link copy of the requested precision missing");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (st) {
    st->link_switch_iter = -1;
    st->compactions = 0;
  }
  ctx->dev_peak = ctx->dev_bytes;  // peak_bytes: the most the context holds during this solve
  auto t0 = std::chrono::steady_clock::now();
  void *sp, *pp, *hp;
  RETCHK(ws_get(ctx, WS_SCAL, sizeof(CGState), &sp));
  RETCHK(ws_get(ctx, WS_PARTIAL, cg_partial_doubles(ctx, n) * sizeof(double), &pp));
  RETCHK(pinned_get(ctx, sizeof(CGState), &hp));
  CGState *S = static_cast<CGState *>(sp);
  CGState *hS = static_cast<CGState *>(hp);
  double *partial = static_cast<double *>(pp);
  int rc;
  if (prm->kind == HISQ_FCG_NN)
    rc = fcg_nn_solve(ctx, mass, n, b, x, prm, st, S, hS, partial);
  else
    rc = cg_solve(ctx, mass, n, b, x, prm, st, S, hS, partial, nullptr, 0, 0, nullptr);
  if (st)
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

extern "C" int hisq_nn_harvest(hisq_ctx *ctx, double mass, int n, const void *b, double tol,
                               int n_snap, int snap_every, void *r_out, void *y_out, int *n_pairs) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!b || !r_out || !y_out || n < 1 || n > HISQ_MAX_RHS || n_snap < 1 || snap_every < 1 || !(tol > 0))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_harvest: bad argument");
  if (!elem_aligned(b, 16) || !elem_aligned(r_out, 16) || !elem_aligned(y_out, 16))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_harvest: b, r_out and y_out must be aligned to 16 bytes");
  if (!ctx->links_loaded || !ctx->links[HISQ_F64].base)
    return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_harvest: the FP64 link copy is required");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const Geometry &g = ctx->g;
  const size_t vbytes = size_t(n) * 3 * g.vh * 16;
  void *sp, *pp, *hp, *xstar, *t64;
  RETCHK(ws_get(ctx, WS_SCAL, sizeof(CGState), &sp));
  RETCHK(ws_get(ctx, WS_PARTIAL, cg_partial_doubles(ctx, n) * sizeof(double), &pp));
  RETCHK(pinned_get(ctx, sizeof(CGState), &hp));
  RETCHK(ws_get(ctx, WS_CG7, vbytes, &xstar));
  CGState *S = static_cast<CGState *>(sp);
  CGState *hS = static_cast<CGState *>(hp);
  double *partial = static_cast<double *>(pp);
  // the snapshots need the bundle in the caller's order: no repacking (cg_solve also skips it
  // whenever it takes snapshots)
  hisq_cg_params prm{HISQ_CG_F64, tol, 1000000, 50, HISQ_F32, 0, 8, 1};
  int taken = 0;
  // x snapshots go straight into y_out; r_k and y_k = x* - x_k are formed afterwards
  int rc = cg_solve(ctx, mass, n, b, xstar, &prm, nullptr, S, hS, partial, y_out, n_snap,
                    snap_every, &taken);
  if (rc != HISQ_OK) return rc;
  RETCHK(ws_get(ctx, WS_CG6, vbytes, &t64));
  for (int k = 0; k < taken; ++k) {
    char *xk = static_cast<char *>(y_out) + k * vbytes;
    char *rk = static_cast<char *>(r_out) + k * vbytes;
    RETCHK(cg_select(ctx, S, n, 1));
    RETCHK(cg_init_state(ctx, b, S, n, partial));  // fin = 1 for every rhs
    RETCHK(apply_m64(ctx, mass, n, xk, t64, rk, S->fin));
    RETCHK(cg_replace_r(ctx, HISQ_F64, b, rk, rk, nullptr, S, S->fin, n, partial));
    RETCHK(cg_snapshot_pairs(ctx, xstar, xk, xk, n));
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (n_pairs) *n_pairs = taken * n;
  return HISQ_OK;
}
