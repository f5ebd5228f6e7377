// Per-rhs device state of the multi-rhs CG solvers (one instance in device memory per solve,
// mirrored to pinned host memory at the host's convergence polls).
#pragma once

#include "hisq.h"

enum { CG_RUNNING = 0, CG_CONVERGED = 1, CG_BREAKDOWN = 2, CG_NONFINITE = 3 };

// Stagnation test of the solvers with reliable updates: a rhs stalls when kStallUpdates
// consecutive true-residual recomputations bring ||b - Mx||^2 no lower than kStallDrop times
// its best value so far.  The drop is mild (10 %): at m = 0.005 on 64^3 x 16 plain CG lowers the
// residual only ~1.5x per 300 iterations, so a stronger demand would flag normal progress.
constexpr double kStallDrop = 0.9;
constexpr int kStallUpdates = 6;
// FP16-link error test of the mixed solver: the true residual exceeds the iterated one by more
// than 2x in norm (4x squared) at kDriftUpdates replacements in a row while ||b - Mx|| / ||b||
// is above 1e-5 (where FP32 vectors still track it closely).
constexpr double kDriftRatio = 4.0;
constexpr double kDriftFloor2 = 1e-10;
constexpr int kDriftUpdates = 2;
// FP16-link rate test of the mixed solver: on ill-conditioned systems the FP16 rounding of the
// links slows CG more and more as the residual falls while the true and the iterated residual
// stay together (measured on 48^3 x 12 at m = 0.01: the true residual falls 3.6x per 500
// iterations at its best and 1.3x at the end, against a steady 3.8x with FP32 links; on 32^3 x 8
// at m = 0.02 it stays within 0.96 of its best).  The convergence rate, d(mean over the live rhs
// of log ||b - Mx|| / ||b||) per iteration over the last kRateWindow periodic residual
// replacements, below kRateFrac of the best such rate of the solve moves the operator to the
// FP32 links, unless the residual is already within kRateNearTol of tol (0.8 switched on
// 48^3 x 12 at iteration 4704, 22 % more iterations than FP32 links throughout; 0.9 leaves
// 32^3 x 8, whose rate stays within 0.96 of its best, on FP16 links).
constexpr int kRateWindow = 8;
constexpr double kRateFrac = 0.9;
constexpr double kRateNearTol = 100.0;

struct CGState {
  double rho[HISQ_MAX_RHS];      // <r, r> of the iterated residual (or <z, r> for FCG)
  double rho_prev[HISQ_MAX_RHS]; // rho as the iteration's alpha reduction read it (for beta)
  double pq[HISQ_MAX_RHS];       // Re <p, M p>
  double alpha[HISQ_MAX_RHS];
  double beta[HISQ_MAX_RHS];
  double bnorm2[HISQ_MAX_RHS];   // ||b||^2
  double rr[HISQ_MAX_RHS];       // ||r||^2 of the iterated residual
  double rr_true[HISQ_MAX_RHS];  // ||b - M x||^2 at the last FP64 recomputation
  double drift[HISQ_MAX_RHS];    // ||b - M x||^2 / iterated ||r||^2 at the last recomputation
  double calpha[2 * HISQ_MAX_RHS]; // FCG: complex alpha = <p, r> / <p, q>  (re, im)
  double cbeta[2 * HISQ_MAX_RHS];  // FCG: complex beta = -<q, z> / <p, q>  (re, im)
  int active[HISQ_MAX_RHS];      // 1 while the rhs iterates
  int hit[HISQ_MAX_RHS];         // iterated residual below tol since the last true residual
  int sel[HISQ_MAX_RHS];         // rhs selected for the current true-residual recomputation
  int fin[HISQ_MAX_RHS];         // rhs included in the final residual report
  int status[HISQ_MAX_RHS];      // CG_RUNNING / CG_CONVERGED / CG_BREAKDOWN / CG_NONFINITE
  int iters[HISQ_MAX_RHS];
  int replacements[HISQ_MAX_RHS];
};

// launchers in blas.hip
struct hisq_ctx;
int blas_nblk(const hisq_ctx *ctx);
int cg_reduce_alpha(hisq_ctx *ctx, const double *partial, int nblk, CGState *S, int n);
int cg_reduce_beta(hisq_ctx *ctx, const double *partial, int nblk, CGState *S, int n, double tol2);
// The unfused r pass writes cg_pass_nblk partials per rhs (finer workgroups on large lattices).
int cg_pass_nblk(const hisq_ctx *ctx);
int cg_update_r(hisq_ctx *ctx, int body_prec, void *r, const void *q, CGState *S, int n, double *partial);
// k_reduce_alpha folded into k_update_r the same way (cg_fuse_alpha): every workgroup of a rhs
// sums its <p, Mp> partials (pq_partial, nblk_pq per rhs) and the ||r||^2 partials go to
// `partial`, which must not overlap pq_partial.
bool cg_fuse_alpha(const hisq_ctx *ctx);
int cg_update_r_alpha(hisq_ctx *ctx, int body_prec, void *r, const void *q, CGState *S, int n,
                      const double *pq_partial, int nblk_pq, double *partial);
// Size of the CG's partials buffer in doubles: the Dslash's <p, Mp> partials and, after them,
// the BLAS kernels' partials, for n rhs.
size_t cg_partial_doubles(const hisq_ctx *ctx, int n);
int cg_update_px(hisq_ctx *ctx, int body_prec, bool x64, void *x, const void *r, void *p, const CGState *S, int n);
// k_reduce_beta folded into k_update_px: every workgroup of a rhs sums that rhs's ||r||^2
// partials itself (the same fixed order, so the same beta), and the first one records the scalars
// k_reduce_beta would; used where the partials are few (cg_fuse_beta), as the redundant sums then
// cost less than a launch.
bool cg_fuse_beta(const hisq_ctx *ctx);
int cg_update_px_beta(hisq_ctx *ctx, int body_prec, bool x64, void *x, const void *r, void *p, CGState *S, int n,
                      const double *partial, double tol2);
int cg_select(hisq_ctx *ctx, CGState *S, int n, int all);
int cg_accum_x(hisq_ctx *ctx, void *x64, void *xh32, const int *mask, int n);
int cg_replace_r(hisq_ctx *ctx, int body_prec, const void *b, const void *mx, void *r, void *p,
                 const CGState *S, const int *sel, int n, double *partial);
int cg_reduce_true(hisq_ctx *ctx, const double *partial, CGState *S, int n, double tol2, int final_only);
int cg_init_state(hisq_ctx *ctx, const void *b, CGState *S, int n, double *partial);
int cg_set_rho(hisq_ctx *ctx, const double *partial, CGState *S, int n, double tol2);
int cg_zero(hisq_ctx *ctx, int prec, void *v, const int *sel, int invert, int n);

// solver pieces shared by the CG host loops (cg.cpp) and the flexible CG (nn.hip)
int cg_poll(hisq_ctx *ctx, CGState *S, CGState *hS);
int apply_m64(hisq_ctx *ctx, double mass, int n, const void *x64, void *t64, void *mx64, const int *mask);
int cg_apply_op(hisq_ctx *ctx, int op_prec, double mass, int n, const void *p, void *t, void *q,
                double *partial, int *nblk, const int *active);
int cg_finish(hisq_ctx *ctx, double mass, int n, const void *b, void *x, double tol, CGState *S,
              CGState *hS, double *partial, hisq_cg_stats *st, bool *all_conv);
int cg_solve(hisq_ctx *ctx, double mass, int n, const void *b, void *x, const hisq_cg_params *prm,
             hisq_cg_stats *st, CGState *S, CGState *hS, double *partial, void *snap_x, int n_snap,
             int snap_every, int *n_taken);

// flexible CG (complex scalars) building blocks
int fcg_alpha(hisq_ctx *ctx, const double *pq_partial, int nblk_pq, const double *pr_partial,
              int nblk_pr, CGState *S, int n);
int fcg_update_xr(hisq_ctx *ctx, void *xh, void *r, const void *p, const void *q, CGState *S, int n,
                  double *partial);
int fcg_beta(hisq_ctx *ctx, const double *qz_partial, int nblk_qz, CGState *S, int n);
int fcg_update_p(hisq_ctx *ctx, const void *z, void *p, const CGState *S, int n);
int cg_snapshot_pairs(hisq_ctx *ctx, const void *xstar, const void *xk, void *y, int n);
