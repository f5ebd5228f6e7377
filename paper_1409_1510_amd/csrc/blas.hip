// Multi-rhs reductions and the CG linear algebra for gfx950.
//
// Every per-rhs reduction is a deterministic two-stage tree in FP64: each workgroup reduces its
// elements (per thread in a fixed order, then 64-lane shuffles, then the 4 waves in a fixed
// order) into one partial per (rhs, workgroup); a second kernel sums the partials of a rhs in a
// fixed order.  No atomics, so results are reproducible run to run.
//
// The CG kernels act on a bundle of n right-hand sides with separate scalars per rhs and skip a
// rhs whose `active` flag is 0 (Section 2: the linear algebra is kept separate per rhs so that
// converged rhs stop).  Vectors are [n][3][V/2] complex; a rhs is a contiguous run of 3*V/2
// complex numbers.
#include "internal.hpp"
#include "cg_state.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;  // complex elements per thread in the streaming kernels
constexpr int kPerBlock = kThreads * kItems;

__device__ inline double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return s;
}

// Complex loads and stores with the non-temporal hint, for operands a pass touches for the last
// time before the next Dslash pair: they should not push the links and the Dslash's input out of
// the caches (the same values, so the same bits).
template <typename C>
__device__ inline C load_nt(const C *p) {
  using R = decltype(C{}.x);
  typedef R v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  C c;
  c.x = v.x;
  c.y = v.y;
  return c;
}
template <typename C>
__device__ inline void store_nt(C *p, C c) {
  using R = decltype(C{}.x);
  typedef R v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = c.x;
  v.y = c.y;
  __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
}

// This thread's share of sum_b row[b] (b = threadIdx.x, threadIdx.x + kThreads, ...), added in
// ascending b.  The loads are issued eight at a time before their adds, so a long row is not one
// load latency per element (the summation order, and so every bit of the result, is that of the
// plain loop).
__device__ inline double strided_sum(const double *__restrict__ row, int nblk) {
  double v = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * kThreads < nblk; b += 8 * kThreads) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = row[b + k * kThreads];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += t[k];
  }
  for (; b < nblk; b += kThreads) v += row[b];
  return v;
}

// res[row] = sum_b partial[row * nblk + b], rows = n * width.
__global__ void __launch_bounds__(kThreads)
k_reduce_rows(const double *__restrict__ partial, int nblk, double *__restrict__ res) {
  __shared__ double red[4];
  const int row = blockIdx.x;
  double v = strided_sum(partial + size_t(row) * nblk, nblk);
  v = block_sum(v, red);
  if (threadIdx.x == 0) res[row] = v;
}

template <typename C>
__global__ void __launch_bounds__(kThreads)
k_dot_partials(const C *__restrict__ a, const C *__restrict__ b, unsigned len, int nblk,
               double *__restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  const size_t off = size_t(r) * len;
  double re = 0.0, im = 0.0;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      C u = a[off + j], v = b[off + j];
      re = fma(double(u.x), double(v.x), re);
      re = fma(double(u.y), double(v.y), re);
      im = fma(double(u.x), double(v.y), im);
      im = fma(-double(u.y), double(v.x), im);
    }
  }
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) {
    partial[size_t(2 * r) * nblk + blockIdx.x] = re;
    partial[size_t(2 * r + 1) * nblk + blockIdx.x] = im;
  }
}

template <typename C>
__global__ void __launch_bounds__(kThreads)
k_norm2_partials(const C *__restrict__ a, unsigned len, int nblk, double *__restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  const size_t off = size_t(r) * len;
  double v = 0.0;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      C u = a[off + j];
      v = fma(double(u.x), double(u.x), v);
      v = fma(double(u.y), double(u.y), v);
    }
  }
  v = block_sum(v, red);
  if (threadIdx.x == 0) partial[size_t(r) * nblk + blockIdx.x] = v;
}

// ------------------------------------------------------------------------------------------
// CG kernels.  S: device CGState (per-rhs scalars and flags).

__global__ void k_reduce_alpha(const double *__restrict__ partial, int nblk, CGState *S) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (!S->active[r]) return;
  double v = strided_sum(partial + size_t(r) * nblk, nblk);
  v = block_sum(v, red);
  if (threadIdx.x == 0) {
    S->pq[r] = v;
    S->rho_prev[r] = S->rho[r];
    if (!(v > 0.0) || !isfinite(v)) {  // M is HPD: <p, Mp> <= 0 means breakdown
      S->alpha[r] = 0.0;
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
    } else {
      S->alpha[r] = S->rho[r] / v;
    }
  }
}

__global__ void k_reduce_beta(const double *__restrict__ partial, int nblk, CGState *S, double tol2) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (!S->active[r]) return;
  double v = strided_sum(partial + size_t(r) * nblk, nblk);
  v = block_sum(v, red);
  if (threadIdx.x == 0) {
    S->iters[r] += 1;
    if (!isfinite(v)) {
      S->beta[r] = 0.0;
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
      return;
    }
    S->beta[r] = v / S->rho[r];
    S->rho[r] = v;
    S->rr[r] = v;
    if (v <= tol2 * S->bnorm2[r]) S->hit[r] = 1;
  }
}

// r -= a q for rhs r and this workgroup's partial of ||r||^2 (ITEMS complex per thread)
template <int ITEMS, typename C>
__device__ inline void update_r_body(C *__restrict__ rv, const C *__restrict__ q, unsigned len, int nblk, int r,
                                     double alpha, double *__restrict__ partial, double *red) {
  using R = decltype(C{}.x);
  const R a = R(alpha);
  const size_t off = size_t(r) * len;
  double rr = 0.0;
  const unsigned base = blockIdx.x * (kThreads * ITEMS) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      C qj = load_nt(q + off + j), rj = rv[off + j];
      rj.x = fma(-a, qj.x, rj.x);
      rj.y = fma(-a, qj.y, rj.y);
      rv[off + j] = rj;
      rr = fma(double(rj.x), double(rj.x), rr);
      rr = fma(double(rj.y), double(rj.y), rr);
    }
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) partial[size_t(r) * nblk + blockIdx.x] = rr;
}

// r -= alpha q and the partials of ||r||^2 (the solution update is left to k_update_px)
template <int ITEMS, typename C>
__global__ void __launch_bounds__(kThreads)
k_update_r(C *__restrict__ rv, const C *__restrict__ q, unsigned len, int nblk, const CGState *S,
           double *__restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (!S->active[r]) return;
  update_r_body<ITEMS>(rv, q, len, nblk, r, S->alpha[r], partial, red);
}

// k_update_r with the alpha reduction of k_reduce_alpha done by every workgroup of the rhs: the
// same <p, Mp> partials summed in the same order, so every workgroup and the separate kernel get
// the same alpha.  The first workgroup of a rhs records what k_reduce_alpha records; no workgroup
// reads those fields here.  A breakdown (<p, Mp> <= 0 or not finite) is seen by every workgroup
// alike: none updates, and the first deactivates the rhs.  The ||r||^2 partials go to a buffer
// apart from the <p, Mp> ones, which other workgroups may still be reading.
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_update_r_alpha(C *__restrict__ rv, const C *__restrict__ q, unsigned len, int nblk, CGState *S,
                 const double *__restrict__ pq_partial, int nblk_pq, double *__restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (!S->active[r]) return;
  double v = strided_sum(pq_partial + size_t(r) * nblk_pq, nblk_pq);
  v = block_sum(v, red);
  const bool ok = v > 0.0 && isfinite(v);  // M is HPD: <p, Mp> <= 0 means breakdown
  const double alpha = ok ? S->rho[r] / v : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->pq[r] = v;
    S->rho_prev[r] = S->rho[r];
    S->alpha[r] = alpha;
    if (!ok) {
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
    }
  }
  if (ok) update_r_body<kItems>(rv, q, len, nblk, r, alpha, partial, red);
}

// x += alpha p; p = r + beta p: the solution update of the step, deferred to the pass that
// rewrites p anyway (one read of p instead of two)
template <int ITEMS, typename C, typename CX>
__global__ void __launch_bounds__(kThreads)
k_update_px(CX *__restrict__ x, const C *__restrict__ rv, C *__restrict__ p, unsigned len, const CGState *S) {
  const int r = blockIdx.y;
  if (!S->active[r]) return;
  using R = decltype(C{}.x);
  using RX = decltype(CX{}.x);
  const R b = R(S->beta[r]);
  const RX ax = RX(S->alpha[r]);
  const size_t off = size_t(r) * len;
  const unsigned base = blockIdx.x * (kThreads * ITEMS) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      C pj = p[off + j], rj = rv[off + j];
      CX xj = load_nt(x + off + j);
      xj.x = fma(ax, RX(pj.x), xj.x);
      xj.y = fma(ax, RX(pj.y), xj.y);
      store_nt(x + off + j, xj);
      pj.x = fma(b, pj.x, rj.x);
      pj.y = fma(b, pj.y, rj.y);
      p[off + j] = pj;
    }
  }
}

// k_update_px with the beta reduction of k_reduce_beta done by every workgroup of the rhs (the
// same partials in the same order, so every workgroup and the separate kernel get the same bits).
// The first workgroup of a rhs records what k_reduce_beta records; the others read only the
// iteration's snapshot rho_prev, which no workgroup writes here.  A non-finite ||r||^2 is seen by
// every workgroup alike: none updates, and the first marks the breakdown.
template <typename C, typename CX>
__global__ void __launch_bounds__(kThreads)
k_update_px_beta(CX *__restrict__ x, const C *__restrict__ rv, C *__restrict__ p, unsigned len, CGState *S,
                 const double *__restrict__ partial, int nblk, double tol2) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (!S->active[r]) return;
  double v = strided_sum(partial + size_t(r) * nblk, nblk);
  v = block_sum(v, red);
  const bool first = blockIdx.x == 0 && threadIdx.x == 0;
  if (!isfinite(v)) {
    if (first) {
      S->iters[r] += 1;
      S->beta[r] = 0.0;
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
    }
    return;
  }
  const double beta = v / S->rho_prev[r];
  if (first) {
    S->iters[r] += 1;
    S->beta[r] = beta;
    S->rho[r] = v;
    S->rr[r] = v;
    if (v <= tol2 * S->bnorm2[r]) S->hit[r] = 1;
  }
  using R = decltype(C{}.x);
  using RX = decltype(CX{}.x);
  const R b = R(beta);
  const RX ax = RX(S->alpha[r]);
  const size_t off = size_t(r) * len;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      C pj = p[off + j], rj = rv[off + j];
      CX xj = load_nt(x + off + j);
      xj.x = fma(ax, RX(pj.x), xj.x);
      xj.y = fma(ax, RX(pj.y), xj.y);
      store_nt(x + off + j, xj);
      pj.x = fma(b, pj.x, rj.x);
      pj.y = fma(b, pj.y, rj.y);
      p[off + j] = pj;
    }
  }
}

// sel[r] = active[r] && (all || hit[r])
__global__ void k_select(CGState *S, int n, int all) {
  const int r = threadIdx.x;
  if (r < n) S->sel[r] = S->active[r] && (all || S->hit[r]);
}

// x64 += xhat; xhat = 0 for the rhs selected by mask.
__global__ void __launch_bounds__(kThreads)
k_accum_x(double2 *__restrict__ x, float2 *__restrict__ xh, unsigned len, const int *mask) {
  const int r = blockIdx.y;
  if (!mask[r]) return;
  const size_t off = size_t(r) * len;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      double2 xj = x[off + j];
      float2 h = xh[off + j];
      xj.x += double(h.x);
      xj.y += double(h.y);
      x[off + j] = xj;
      xh[off + j] = make_float2(0.f, 0.f);
    }
  }
}

// r = b - mx for selected rhs (FP64), stored in the body precision, and ||r||^2 partials.
// With copy_p, also p = r (restart).
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_replace_r(const double2 *__restrict__ b, const double2 *__restrict__ mx, C *__restrict__ rv,
            C *__restrict__ p, unsigned len, int nblk, const CGState *S, const int *sel,
            double *__restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (!sel[r]) return;
  using R = decltype(C{}.x);
  const size_t off = size_t(r) * len;
  double rr = 0.0;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      double2 bj = b[off + j], mj = mx[off + j];
      double re = bj.x - mj.x, im = bj.y - mj.y;
      rr = fma(re, re, rr);
      rr = fma(im, im, rr);
      C o;
      o.x = R(re);
      o.y = R(im);
      if (rv) rv[off + j] = o;
      if (p) p[off + j] = o;
    }
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) partial[size_t(r) * nblk + blockIdx.x] = rr;
}

// After a true-residual recomputation of the selected rhs: converged ones stop, the others
// continue with rho = ||r_true||^2.  final_only: only record rr_true.
__global__ void k_reduce_true(const double *__restrict__ partial, int nblk, CGState *S, double tol2,
                              int final_only) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (!(final_only ? S->fin[r] : S->sel[r])) return;
  double v = strided_sum(partial + size_t(r) * nblk, nblk);
  v = block_sum(v, red);
  if (threadIdx.x == 0) {
    S->rr_true[r] = v;
    if (final_only) return;
    S->drift[r] = S->rr[r] > 0.0 ? v / S->rr[r] : 1.0;
    S->hit[r] = 0;
    S->replacements[r] += 1;
    if (!isfinite(v)) {
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
    } else if (v <= tol2 * S->bnorm2[r]) {
      S->status[r] = CG_CONVERGED;
      S->active[r] = 0;
    } else {
      S->rho[r] = v;
      S->rr[r] = v;
    }
  }
}

// ||b||^2 partials for all rhs (sel = null) and the initialisation of the per-rhs state.
__global__ void k_init_state(const double *__restrict__ partial, int nblk, CGState *S, int n) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  double v = strided_sum(partial + size_t(r) * nblk, nblk);
  v = block_sum(v, red);
  if (threadIdx.x == 0) {
    S->bnorm2[r] = v;
    S->iters[r] = 0;
    S->hit[r] = 0;
    S->replacements[r] = 0;
    S->alpha[r] = S->beta[r] = 0.0;
    S->rr_true[r] = 0.0;
    S->fin[r] = 1;
    if (!isfinite(v)) {
      S->status[r] = CG_NONFINITE;
      S->active[r] = 0;
    } else if (v == 0.0) {
      S->status[r] = CG_CONVERGED;
      S->active[r] = 0;
    } else {
      S->status[r] = CG_RUNNING;
      S->active[r] = 1;
    }
  }
}

// rho = ||r||^2 from partials for active rhs (start of an iteration sequence).
__global__ void k_set_rho(const double *__restrict__ partial, int nblk, CGState *S, double tol2) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (!S->sel[r]) return;
  double v = strided_sum(partial + size_t(r) * nblk, nblk);
  v = block_sum(v, red);
  if (threadIdx.x == 0) {
    S->rho[r] = v;
    S->rr[r] = v;
    S->rr_true[r] = v;
    if (v <= tol2 * S->bnorm2[r]) {  // the initial guess already solves it
      S->status[r] = CG_CONVERGED;
      S->active[r] = 0;
    }
  }
}

// zero the selected rhs of a vector (x = 0 for b = 0, or xhat = 0)
template <typename C>
__global__ void __launch_bounds__(kThreads)
k_zero_sel(C *__restrict__ v, unsigned len, const int *sel, int invert) {
  const int r = blockIdx.y;
  if (sel && (bool(sel[r]) == bool(invert))) return;
  const size_t off = size_t(r) * len;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      C z;
      z.x = 0;
      z.y = 0;
      v[off + j] = z;
    }
  }
}

// ---- flexible CG with complex step sizes --------------------------------------------------

// alpha = <p, r> / Re<p, q>; pq partials [n][nblk_pq] (real), pr partials [2n][nblk_pr]
__global__ void k_fcg_alpha(const double *__restrict__ pqp, int nblk_pq, const double *__restrict__ prp,
                            int nblk_pr, CGState *S) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (!S->active[r]) return;
  double pq = strided_sum(pqp + size_t(r) * nblk_pq, nblk_pq);
  double pre = strided_sum(prp + size_t(2 * r) * nblk_pr, nblk_pr);
  double pim = strided_sum(prp + size_t(2 * r + 1) * nblk_pr, nblk_pr);
  pq = block_sum(pq, red);
  pre = block_sum(pre, red);
  pim = block_sum(pim, red);
  if (threadIdx.x == 0) {
    S->pq[r] = pq;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(pre) || !isfinite(pim)) {
      S->calpha[2 * r] = S->calpha[2 * r + 1] = 0.0;
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
    } else {
      S->calpha[2 * r] = pre / pq;
      S->calpha[2 * r + 1] = pim / pq;
    }
  }
}

// xh += alpha p; r -= alpha q (complex alpha, FP32 vectors); ||r||^2 partials
__global__ void __launch_bounds__(kThreads)
k_fcg_update_xr(float2 *__restrict__ x, float2 *__restrict__ rv, const float2 *__restrict__ p,
                const float2 *__restrict__ q, unsigned len, int nblk, const CGState *S,
                double *__restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  if (!S->active[r]) return;
  const float ar = float(S->calpha[2 * r]), ai = float(S->calpha[2 * r + 1]);
  const size_t off = size_t(r) * len;
  double rr = 0.0;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      float2 pj = p[off + j], qj = q[off + j], rj = rv[off + j], xj = x[off + j];
      xj.x = fmaf(ar, pj.x, fmaf(-ai, pj.y, xj.x));
      xj.y = fmaf(ar, pj.y, fmaf(ai, pj.x, xj.y));
      rj.x = fmaf(-ar, qj.x, fmaf(ai, qj.y, rj.x));
      rj.y = fmaf(-ar, qj.y, fmaf(-ai, qj.x, rj.y));
      x[off + j] = xj;
      rv[off + j] = rj;
      rr = fma(double(rj.x), double(rj.x), rr);
      rr = fma(double(rj.y), double(rj.y), rr);
    }
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) partial[size_t(r) * nblk + blockIdx.x] = rr;
}

// beta = -<q, z> / Re<p, q>; qz partials [2n][nblk]
__global__ void k_fcg_beta(const double *__restrict__ qzp, int nblk, CGState *S) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (!S->active[r]) return;
  double re = strided_sum(qzp + size_t(2 * r) * nblk, nblk);
  double im = strided_sum(qzp + size_t(2 * r + 1) * nblk, nblk);
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) {
    const double pq = S->pq[r];
    if (!isfinite(re) || !isfinite(im)) {
      S->status[r] = CG_BREAKDOWN;
      S->active[r] = 0;
      return;
    }
    S->cbeta[2 * r] = -re / pq;
    S->cbeta[2 * r + 1] = -im / pq;
  }
}

// p = z + beta p (complex beta)
__global__ void __launch_bounds__(kThreads)
k_fcg_update_p(const float2 *__restrict__ z, float2 *__restrict__ p, unsigned len, const CGState *S) {
  const int r = blockIdx.y;
  if (!S->active[r]) return;
  const float br = float(S->cbeta[2 * r]), bi = float(S->cbeta[2 * r + 1]);
  const size_t off = size_t(r) * len;
  const unsigned base = blockIdx.x * kPerBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    unsigned j = base + k * kThreads;
    if (j < len) {
      float2 pj = p[off + j], zj = z[off + j];
      float2 o;
      o.x = fmaf(br, pj.x, fmaf(-bi, pj.y, zj.x));
      o.y = fmaf(br, pj.y, fmaf(bi, pj.x, zj.y));
      p[off + j] = o;
    }
  }
}

// y = xstar - xk (training targets of harvested pairs)
__global__ void __launch_bounds__(kThreads)
k_sub64(const double2 *__restrict__ a, const double2 *__restrict__ b, double2 *__restrict__ y, size_t len) {
  for (size_t j = size_t(blockIdx.x) * kThreads + threadIdx.x; j < len; j += size_t(gridDim.x) * kThreads) {
    double2 u = a[j], v = b[j];
    y[j] = make_double2(u.x - v.x, u.y - v.y);
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------
// host launchers

int blas_nblk(const hisq_ctx *ctx) { return (3 * ctx->g.vh + kPerBlock - 1) / kPerBlock; }

int launch_reduce_partials(hisq_ctx *ctx, const double *partial, int n, int nblk, int width,
                           double *res) {
  k_reduce_rows<<<n * width, kThreads, 0, ctx->stream>>>(partial, nblk, res);
  LAUNCHCHK(ctx, "k_reduce_rows");
  return HISQ_OK;
}

int launch_dot_partials(hisq_ctx *ctx, int prec, int n, const void *a, const void *b,
                        double *partial, int *nblk_out) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = blas_nblk(ctx);
  dim3 grid(nblk, n);
  if (prec == HISQ_F64)
    k_dot_partials<double2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<const double2 *>(a), static_cast<const double2 *>(b), len, nblk, partial);
  else
    k_dot_partials<float2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<const float2 *>(a), static_cast<const float2 *>(b), len, nblk, partial);
  LAUNCHCHK(ctx, "k_dot_partials");
  *nblk_out = nblk;
  return HISQ_OK;
}

extern "C" int hisq_dot_mrhs(hisq_ctx *ctx, int prec, int n, const void *a, const void *b,
                             double *dots) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!a || !b || !dots) return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs: null pointer");
  if (!prec_valid(prec)) return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs: bad precision %d", prec);
  if (!elem_aligned(a, cplx_bytes(prec)) || !elem_aligned(b, cplx_bytes(prec)) || !elem_aligned(dots, sizeof(double)))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs: vectors must be aligned to %zu bytes, dots to 8",
                   cplx_bytes(prec));
  if (n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs: n = %d outside 1..%d", n, HISQ_MAX_RHS);
  const int nblk = blas_nblk(ctx);
  void *pp;
  RETCHK(ws_get(ctx, WS_PARTIAL, size_t(2 * n) * nblk * sizeof(double), &pp));
  double *partial = static_cast<double *>(pp);
  int nb;
  RETCHK(launch_dot_partials(ctx, prec, n, a, b, partial, &nb));
  return launch_reduce_partials(ctx, partial, n, nb, 2, dots);
}

// ---- allocation-free per-rhs inner products ----
//
// hisq_dot_mrhs_noalloc keeps its per-block partials in this file-scope device array instead of
// the context workspace: one copy per GPU, loaded with the library and held until the process
// ends.  Host code never passes `scratch` itself to a kernel (in host code the name stands for a
// host-side shadow, not a device address); scratch_lookup() asks the runtime for the array's
// device address once per device, with that device current, and every launch uses that address.
constexpr size_t kScratchDoubles = size_t(1) << 20;  // 8 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};
}  // namespace

int scratch_lookup(hisq_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_err(ctx, HISQ_ERR_ARG, "device index %d above the library's limit of %d", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[ctx->device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_err(ctx, HISQ_ERR_HIP, "hipGetSymbolAddress of the static scratch buffer failed: %s",
                     hipGetErrorString(e));
    }
    g_scratch_dev[ctx->device] = p;
  }
  ctx->scratch_dev = g_scratch_dev[ctx->device];
  return HISQ_OK;
}

extern "C" int hisq_dot_mrhs_noalloc(hisq_ctx *ctx, int prec, int n, const void *a, const void *b,
                                     double *dots) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!a || !b || !dots) return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs_noalloc: null pointer");
  if (!prec_valid(prec)) return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs_noalloc: bad precision %d", prec);
  if (!elem_aligned(a, cplx_bytes(prec)) || !elem_aligned(b, cplx_bytes(prec)) || !elem_aligned(dots, sizeof(double)))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs_noalloc: vectors must be aligned to %zu bytes, dots to 8",
                   cplx_bytes(prec));
  if (n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dot_mrhs_noalloc: n = %d outside 1..%d", n, HISQ_MAX_RHS);
  const int nblk = blas_nblk(ctx);
  const size_t need = size_t(2 * n) * nblk;
  if (need > kScratchDoubles)
    return set_err(ctx, HISQ_ERR_ARG,
                   "hisq_dot_mrhs_noalloc: %d rhs on %d sites per parity need %zu doubles of scratch, "
                   "above the static buffer's %zu (at most %zu rhs on this lattice)",
                   n, ctx->g.vh, need, kScratchDoubles, kScratchDoubles / (2 * size_t(nblk)));
  if (!ctx->scratch_dev)
    return set_err(ctx, HISQ_ERR_STATE, "hisq_dot_mrhs_noalloc: static scratch buffer not set up");
  double *partial = static_cast<double *>(ctx->scratch_dev);
  int nb;
  RETCHK(launch_dot_partials(ctx, prec, n, a, b, partial, &nb));
  return launch_reduce_partials(ctx, partial, n, nb, 2, dots);
}

// ---- CG building blocks used by cg.cpp ----

int cg_reduce_alpha(hisq_ctx *ctx, const double *partial, int nblk, CGState *S, int n) {
  k_reduce_alpha<<<n, kThreads, 0, ctx->stream>>>(partial, nblk, S);
  LAUNCHCHK(ctx, "k_reduce_alpha");
  return HISQ_OK;
}

// Workgroups of the unfused r and p/x passes take 256 elements each (one per thread) where the
// beta reduction is not folded into the p/x pass (large lattices): on MI355X a streaming pass
// over a few hundred MB runs ~10 % faster in workgroups of 256 elements than of 1024 (measured
// with 2-read 1-write and 3-read 2-write passes at 0.25 and 1.6 GB per operand).  Where it is
// folded, every workgroup re-reads all partials of its rhs, so the passes keep 1024 elements
// (and the env switch that unfolds the reductions keeps the same partials, so the same bits).
static bool fine_passes(const hisq_ctx *ctx) { return !cg_fuse_beta(ctx); }

int cg_pass_nblk(const hisq_ctx *ctx) {
  return fine_passes(ctx) ? (3 * ctx->g.vh + kThreads - 1) / kThreads : blas_nblk(ctx);
}

int cg_update_r(hisq_ctx *ctx, int body_prec, void *r, const void *q, CGState *S, int n, double *partial) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = cg_pass_nblk(ctx);
  dim3 grid(nblk, n);
  auto go = [&](auto *rr, auto *qq) {
    using C = std::remove_pointer_t<decltype(rr)>;
    if (fine_passes(ctx))
      k_update_r<1, C><<<grid, kThreads, 0, ctx->stream>>>(rr, qq, len, nblk, S, partial);
    else
      k_update_r<kItems, C><<<grid, kThreads, 0, ctx->stream>>>(rr, qq, len, nblk, S, partial);
  };
  if (body_prec == HISQ_F64)
    go(static_cast<double2 *>(r), static_cast<const double2 *>(q));
  else
    go(static_cast<float2 *>(r), static_cast<const float2 *>(q));
  LAUNCHCHK(ctx, "k_update_r");
  return HISQ_OK;
}

// Fold the alpha reduction into the r pass under the same rule: nblk workgroups x the Dslash's
// partials per rhs <= 2^20 (32^3 x 8: 384 x 2048).
bool cg_fuse_alpha(const hisq_ctx *ctx) {
  return (long long)blas_nblk(ctx) * dslash_partials(ctx->g) <= (1ll << 20);
}

size_t cg_partial_doubles(const hisq_ctx *ctx, int n) {
  return size_t(n) * (size_t(dslash_partials(ctx->g)) + size_t(std::max(blas_nblk(ctx), cg_pass_nblk(ctx))));
}

int cg_update_r_alpha(hisq_ctx *ctx, int body_prec, void *r, const void *q, CGState *S, int n,
                      const double *pq_partial, int nblk_pq, double *partial) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = blas_nblk(ctx);
  dim3 grid(nblk, n);
  if (body_prec == HISQ_F64)
    k_update_r_alpha<double2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<double2 *>(r), static_cast<const double2 *>(q), len, nblk, S, pq_partial, nblk_pq, partial);
  else
    k_update_r_alpha<float2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<float2 *>(r), static_cast<const float2 *>(q), len, nblk, S, pq_partial, nblk_pq, partial);
  LAUNCHCHK(ctx, "k_update_r_alpha");
  return HISQ_OK;
}

int cg_update_px(hisq_ctx *ctx, int body_prec, bool x64, void *x, const void *r, void *p, const CGState *S, int n) {
  const unsigned len = 3u * ctx->g.vh;
  dim3 grid(cg_pass_nblk(ctx), n);
  auto go = [&](auto *xx, auto *rr, auto *pp) {
    using CX = std::remove_pointer_t<decltype(xx)>;
    using C = std::remove_cv_t<std::remove_pointer_t<decltype(rr)>>;
    if (fine_passes(ctx))
      k_update_px<1, C, CX><<<grid, kThreads, 0, ctx->stream>>>(xx, rr, pp, len, S);
    else
      k_update_px<kItems, C, CX><<<grid, kThreads, 0, ctx->stream>>>(xx, rr, pp, len, S);
  };
  if (body_prec == HISQ_F64)
    go(static_cast<double2 *>(x), static_cast<const double2 *>(r), static_cast<double2 *>(p));
  else if (x64)
    go(static_cast<double2 *>(x), static_cast<const float2 *>(r), static_cast<float2 *>(p));
  else
    go(static_cast<float2 *>(x), static_cast<const float2 *>(r), static_cast<float2 *>(p));
  LAUNCHCHK(ctx, "k_update_px");
  return HISQ_OK;
}

// Fold the beta reduction into the p/x pass while every workgroup's share of redundant partial
// reads stays small: nblk workgroups x nblk partials per rhs <= 2^20 (lattices up to V/2 ~ 350 k
// sites; 32^3 x 8 has 384 of each).
bool cg_fuse_beta(const hisq_ctx *ctx) {
  const long long nb = blas_nblk(ctx);
  return nb * nb <= (1ll << 20);
}

int cg_update_px_beta(hisq_ctx *ctx, int body_prec, bool x64, void *x, const void *r, void *p, CGState *S, int n,
                      const double *partial, double tol2) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = blas_nblk(ctx);
  dim3 grid(nblk, n);
  if (body_prec == HISQ_F64)
    k_update_px_beta<double2, double2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<double2 *>(x), static_cast<const double2 *>(r), static_cast<double2 *>(p), len, S, partial,
        nblk, tol2);
  else if (x64)
    k_update_px_beta<float2, double2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<double2 *>(x), static_cast<const float2 *>(r), static_cast<float2 *>(p), len, S, partial,
        nblk, tol2);
  else
    k_update_px_beta<float2, float2><<<grid, kThreads, 0, ctx->stream>>>(
        static_cast<float2 *>(x), static_cast<const float2 *>(r), static_cast<float2 *>(p), len, S, partial,
        nblk, tol2);
  LAUNCHCHK(ctx, "k_update_px_beta");
  return HISQ_OK;
}

int cg_reduce_beta(hisq_ctx *ctx, const double *partial, int nblk, CGState *S, int n, double tol2) {
  k_reduce_beta<<<n, kThreads, 0, ctx->stream>>>(partial, nblk, S, tol2);
  LAUNCHCHK(ctx, "k_reduce_beta");
  return HISQ_OK;
}

int cg_select(hisq_ctx *ctx, CGState *S, int n, int all) {
  k_select<<<1, 64, 0, ctx->stream>>>(S, n, all);
  LAUNCHCHK(ctx, "k_select");
  return HISQ_OK;
}

int cg_accum_x(hisq_ctx *ctx, void *x64, void *xh32, const int *mask, int n) {
  dim3 grid(blas_nblk(ctx), n);
  k_accum_x<<<grid, kThreads, 0, ctx->stream>>>(static_cast<double2 *>(x64), static_cast<float2 *>(xh32),
                                                3u * ctx->g.vh, mask);
  LAUNCHCHK(ctx, "k_accum_x");
  return HISQ_OK;
}

int cg_replace_r(hisq_ctx *ctx, int body_prec, const void *b, const void *mx, void *r, void *p,
                 const CGState *S, const int *sel, int n, double *partial) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = blas_nblk(ctx);
  dim3 grid(nblk, n);
  const double2 *b2 = static_cast<const double2 *>(b), *m2 = static_cast<const double2 *>(mx);
  if (body_prec == HISQ_F64)
    k_replace_r<double2><<<grid, kThreads, 0, ctx->stream>>>(
        b2, m2, static_cast<double2 *>(r), static_cast<double2 *>(p), len, nblk, S, sel, partial);
  else
    k_replace_r<float2><<<grid, kThreads, 0, ctx->stream>>>(
        b2, m2, static_cast<float2 *>(r), static_cast<float2 *>(p), len, nblk, S, sel, partial);
  LAUNCHCHK(ctx, "k_replace_r");
  return HISQ_OK;
}

int cg_reduce_true(hisq_ctx *ctx, const double *partial, CGState *S, int n, double tol2, int final_only) {
  k_reduce_true<<<n, kThreads, 0, ctx->stream>>>(partial, blas_nblk(ctx), S, tol2, final_only);
  LAUNCHCHK(ctx, "k_reduce_true");
  return HISQ_OK;
}

int cg_init_state(hisq_ctx *ctx, const void *b, CGState *S, int n, double *partial) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = blas_nblk(ctx);
  dim3 grid(nblk, n);
  k_norm2_partials<double2><<<grid, kThreads, 0, ctx->stream>>>(static_cast<const double2 *>(b),
                                                                len, nblk, partial);
  LAUNCHCHK(ctx, "k_norm2_partials");
  k_init_state<<<n, kThreads, 0, ctx->stream>>>(partial, nblk, S, n);
  LAUNCHCHK(ctx, "k_init_state");
  return HISQ_OK;
}

int cg_set_rho(hisq_ctx *ctx, const double *partial, CGState *S, int n, double tol2) {
  k_set_rho<<<n, kThreads, 0, ctx->stream>>>(partial, blas_nblk(ctx), S, tol2);
  LAUNCHCHK(ctx, "k_set_rho");
  return HISQ_OK;
}

int cg_zero(hisq_ctx *ctx, int prec, void *v, const int *sel, int invert, int n) {
  const unsigned len = 3u * ctx->g.vh;
  dim3 grid(blas_nblk(ctx), n);
  if (prec == HISQ_F64)
    k_zero_sel<double2><<<grid, kThreads, 0, ctx->stream>>>(static_cast<double2 *>(v), len, sel, invert);
  else
    k_zero_sel<float2><<<grid, kThreads, 0, ctx->stream>>>(static_cast<float2 *>(v), len, sel, invert);
  LAUNCHCHK(ctx, "k_zero_sel");
  return HISQ_OK;
}

int fcg_alpha(hisq_ctx *ctx, const double *pq_partial, int nblk_pq, const double *pr_partial,
              int nblk_pr, CGState *S, int n) {
  k_fcg_alpha<<<n, kThreads, 0, ctx->stream>>>(pq_partial, nblk_pq, pr_partial, nblk_pr, S);
  LAUNCHCHK(ctx, "k_fcg_alpha");
  return HISQ_OK;
}

int fcg_update_xr(hisq_ctx *ctx, void *xh, void *r, const void *p, const void *q, CGState *S, int n,
                  double *partial) {
  const unsigned len = 3u * ctx->g.vh;
  const int nblk = blas_nblk(ctx);
  k_fcg_update_xr<<<dim3(nblk, n), kThreads, 0, ctx->stream>>>(
      static_cast<float2 *>(xh), static_cast<float2 *>(r), static_cast<const float2 *>(p),
      static_cast<const float2 *>(q), len, nblk, S, partial);
  LAUNCHCHK(ctx, "k_fcg_update_xr");
  return HISQ_OK;
}

int fcg_beta(hisq_ctx *ctx, const double *qz_partial, int nblk_qz, CGState *S, int n) {
  k_fcg_beta<<<n, kThreads, 0, ctx->stream>>>(qz_partial, nblk_qz, S);
  LAUNCHCHK(ctx, "k_fcg_beta");
  return HISQ_OK;
}

int fcg_update_p(hisq_ctx *ctx, const void *z, void *p, const CGState *S, int n) {
  const unsigned len = 3u * ctx->g.vh;
  k_fcg_update_p<<<dim3(blas_nblk(ctx), n), kThreads, 0, ctx->stream>>>(
      static_cast<const float2 *>(z), static_cast<float2 *>(p), len, S);
  LAUNCHCHK(ctx, "k_fcg_update_p");
  return HISQ_OK;
}

int cg_snapshot_pairs(hisq_ctx *ctx, const void *xstar, const void *xk, void *y, int n) {
  const size_t len = size_t(n) * 3 * ctx->g.vh;
  k_sub64<<<1024, kThreads, 0, ctx->stream>>>(static_cast<const double2 *>(xstar),
                                              static_cast<const double2 *>(xk),
                                              static_cast<double2 *>(y), len);
  LAUNCHCHK(ctx, "k_sub64");
  return HISQ_OK;
}
