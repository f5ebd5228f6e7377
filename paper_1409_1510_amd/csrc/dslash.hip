// Multi-rhs HISQ half Dslash for gfx950 (Section 1, Eq. 3 and Eq. 4).
//
// One thread owns one output site and a tile of RT right-hand sides (register blocking over
// rhs, Section 2): every link of the site is loaded once per tile and applied to the RT
// neighbour vectors, and tiles of the same sites run in neighbouring workgroups of the same XCD
// so that a second tile finds the links in that XCD's L2 (the 2-d site x rhs blocking of
// Section 2).  Hops are accumulated in a fixed order with explicit FMAs, so the result for a
// right-hand side does not depend on n or on the tile it is computed in.
//
// Layouts: links as packed by links.hip (planes of V/2 complex per matrix entry, per output
// parity); vectors [n][3][V/2] complex (colour-planar structure of arrays, Section 2).
#include "internal.hpp"

#include <cstdlib>

namespace {

template <typename Real> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

__device__ inline void ld_link(const double2 *p, double &re, double &im) {
  double2 v = *p;
  re = v.x;
  im = v.y;
}
__device__ inline void ld_link(const float2 *p, float &re, float &im) {
  float2 v = *p;
  re = v.x;
  im = v.y;
}
__device__ inline void ld_link(const __half2 *p, float &re, float &im) {
  float2 v = __half22float2(*p);
  re = v.x;
  im = v.y;
}

__device__ inline double fmaR(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float fmaR(float a, float b, float c) { return fmaf(a, b, c); }

template <typename Real> struct Lnk {
  Real re[3][3], im[3][3];
};

// Load the link of hop k at site s; a 14-real Naik link gets row 2 = z * conj(row0 x row1).
template <typename Real, typename LT, bool R14>
__device__ inline void load_link(const LT *__restrict__ links, int plane, unsigned vh, unsigned s,
                                 Lnk<Real> &L) {
  const LT *p = links + size_t(plane) * vh + s;
  constexpr int rows = R14 ? 2 : 3;
#pragma unroll
  for (int a = 0; a < rows; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ld_link(p + (a * 3 + b) * vh, L.re[a][b], L.im[a][b]);
  if constexpr (R14) {
    Real zr, zi;
    ld_link(p + 6 * vh, zr, zi);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
      // cross_b = r0[b1] r1[b2] - r0[b2] r1[b1]
      Real cr = (L.re[0][b1] * L.re[1][b2] - L.im[0][b1] * L.im[1][b2]) -
                (L.re[0][b2] * L.re[1][b1] - L.im[0][b2] * L.im[1][b1]);
      Real ci = (L.re[0][b1] * L.im[1][b2] + L.im[0][b1] * L.re[1][b2]) -
                (L.re[0][b2] * L.im[1][b1] + L.im[0][b2] * L.re[1][b1]);
      // row2_b = z * conj(cross_b)
      L.re[2][b] = zr * cr + zi * ci;
      L.im[2][b] = zi * cr - zr * ci;
    }
  }
}

// acc += s * L v for RT right-hand sides (s = +1 forward hop, -1 backward hop).
template <typename Real, int RT, bool NEG>
__device__ inline void apply_hop(const Lnk<Real> &L, const typename CT<Real>::T *__restrict__ in,
                                 unsigned vh, unsigned nbr, const bool *act,
                                 Real (&acc_re)[RT][3], Real (&acc_im)[RT][3]) {
  using C = typename CT<Real>::T;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    if (!act[r]) continue;
    C v[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) v[b] = in[(unsigned)(r * 3 + b) * vh + nbr];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const Real lr = NEG ? -L.re[a][b] : L.re[a][b];
        const Real li = NEG ? -L.im[a][b] : L.im[a][b];
        acc_re[r][a] = fmaR(lr, v[b].x, acc_re[r][a]);
        acc_re[r][a] = fmaR(-li, v[b].y, acc_re[r][a]);
        acc_im[r][a] = fmaR(lr, v[b].y, acc_im[r][a]);
        acc_im[r][a] = fmaR(li, v[b].x, acc_im[r][a]);
      }
    }
  }
}

template <typename Real, typename LT, int RT, bool R14, bool EPI>
__global__ void __launch_bounds__(256)
k_dslash(const LT *__restrict__ links, const typename CT<Real>::T *__restrict__ in_all,
         typename CT<Real>::T *__restrict__ out_all, Geometry g, int out_parity, int n, int ntiles,
         int nblk_sites, Real mass2, const typename CT<Real>::T *__restrict__ p_all,
         double *__restrict__ partial, const int *__restrict__ active) {
  using C = typename CT<Real>::T;
  // XCD-aware order: hardware deals workgroups round-robin to the 8 XCDs; give each XCD a
  // contiguous range of (site block, rhs tile) pairs so neighbour vectors and the links shared
  // by the rhs tiles of a site block stay in one L2.
  const int nb = nblk_sites * ntiles;
  const int chunk = gridDim.x >> 3;
  const int lb = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  if (lb >= nb) return;  // uniform for the whole workgroup
  const int sblk = lb / ntiles;
  const int tile = lb - sblk * ntiles;
  const int r0 = tile * RT;
  const unsigned vh = g.vh;
  const unsigned s = sblk * 256 + threadIdx.x;
  const bool valid = s < vh;
  const size_t tile_off = size_t(r0) * 3 * vh;
  const C *__restrict__ in = in_all + tile_off;
  C *__restrict__ out = out_all + tile_off;

  bool act[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) act[r] = (r0 + r < n) && (!active || active[r0 + r]);

  Real acc_re[RT][3], acc_im[RT][3];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc_re[r][a] = acc_im[r][a] = Real(0);

  if (valid) {
    const int xh = s % g.lxh;
    int rest = s / g.lxh;
    const int y = rest % g.ly;
    rest /= g.ly;
    const int z = rest % g.lz;
    const int t = rest / g.lz;
    const int x = 2 * xh + ((y + z + t + out_parity) & 1);
    const unsigned rowbase = s - xh;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      unsigned f1, b1, f3, b3;
      if (mu == 0) {
        int xf1 = x + 1 >= g.lx ? x + 1 - g.lx : x + 1;
        int xb1 = x - 1 < 0 ? x - 1 + g.lx : x - 1;
        int xf3 = x + 3 >= g.lx ? x + 3 - g.lx : x + 3;
        int xb3 = x - 3 < 0 ? x - 3 + g.lx : x - 3;
        f1 = rowbase + (xf1 >> 1);
        b1 = rowbase + (xb1 >> 1);
        f3 = rowbase + (xf3 >> 1);
        b3 = rowbase + (xb3 >> 1);
      } else {
        const int c = mu == 1 ? y : (mu == 2 ? z : t);
        const int L = mu == 1 ? g.ly : (mu == 2 ? g.lz : g.lt);
        const int S = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
        f1 = s + (c + 1 >= L ? 1 - L : 1) * S;
        b1 = s + (c - 1 < 0 ? L - 1 : -1) * S;
        f3 = s + (c + 3 >= L ? 3 - L : 3) * S;
        b3 = s + (c - 3 < 0 ? L - 3 : -3) * S;
      }
      Lnk<Real> L;
      load_link<Real, LT, false>(links, link_plane(mu, R14 ? 14 : 18), vh, s, L);
      apply_hop<Real, RT, false>(L, in, vh, f1, act, acc_re, acc_im);
      load_link<Real, LT, false>(links, link_plane(4 + mu, R14 ? 14 : 18), vh, s, L);
      apply_hop<Real, RT, true>(L, in, vh, b1, act, acc_re, acc_im);
      load_link<Real, LT, R14>(links, link_plane(8 + mu, R14 ? 14 : 18), vh, s, L);
      apply_hop<Real, RT, false>(L, in, vh, f3, act, acc_re, acc_im);
      load_link<Real, LT, R14>(links, link_plane(12 + mu, R14 ? 14 : 18), vh, s, L);
      apply_hop<Real, RT, true>(L, in, vh, b3, act, acc_re, acc_im);
    }
  }

  if constexpr (!EPI) {
    if (valid) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (!act[r]) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          C o;
          o.x = acc_re[r][a];
          o.y = acc_im[r][a];
          out[(unsigned)(r * 3 + a) * vh + s] = o;
        }
      }
    }
  } else {
    // q = m^2 p - D_eo t and the per-rhs FP64 partials of Re<p, q>
    const C *__restrict__ pv = p_all + tile_off;
    double dot[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      dot[r] = 0.0;
      if (!act[r] || !valid) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const C p = pv[(unsigned)(r * 3 + a) * vh + s];
        C o;
        o.x = fmaR(mass2, p.x, -acc_re[r][a]);
        o.y = fmaR(mass2, p.y, -acc_im[r][a]);
        out[(unsigned)(r * 3 + a) * vh + s] = o;
        dot[r] = fma(double(p.x), double(o.x), dot[r]);
        dot[r] = fma(double(p.y), double(o.y), dot[r]);
      }
    }
    if (partial) {
      __shared__ double red[RT][4];
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        double v = dot[r];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[r][wave] = v;
      }
      __syncthreads();
      if ((int)threadIdx.x < RT && r0 + (int)threadIdx.x < n) {
        const int r = threadIdx.x;
        partial[size_t(r0 + r) * nblk_sites + sblk] = ((red[r][0] + red[r][1]) + red[r][2]) + red[r][3];
      }
    }
  }
}

using DslashFn = void (*)(const void *, const void *, void *, Geometry, int, int, int, int, double,
                          const void *, double *, const int *, dim3, hipStream_t);

template <typename Real, typename LT, int RT, bool R14, bool EPI>
void launch_t(const void *links, const void *in, void *out, Geometry g, int out_parity, int n,
              int ntiles, int nblk_sites, double mass2, const void *p, double *partial,
              const int *active, dim3 grid, hipStream_t st) {
  using C = typename CT<Real>::T;
  k_dslash<Real, LT, RT, R14, EPI><<<grid, 256, 0, st>>>(
      static_cast<const LT *>(links), static_cast<const C *>(in), static_cast<C *>(out), g,
      out_parity, n, ntiles, nblk_sites, Real(mass2), static_cast<const C *>(p), partial, active);
}

template <typename Real, typename LT, bool R14, bool EPI> DslashFn pick_rt(int rt) {
  switch (rt) {
    case 1: return launch_t<Real, LT, 1, R14, EPI>;
    case 2: return launch_t<Real, LT, 2, R14, EPI>;
    case 4: return launch_t<Real, LT, 4, R14, EPI>;
    case 8: return launch_t<Real, LT, 8, R14, EPI>;
    default: return launch_t<Real, LT, 16, R14, EPI>;
  }
}

template <bool EPI> DslashFn pick(int prec, int recon, int rt) {
  if (prec == HISQ_F64) return pick_rt<double, double2, false, EPI>(rt);
  if (prec == HISQ_F32)
    return recon == 14 ? pick_rt<float, float2, true, EPI>(rt) : pick_rt<float, float2, false, EPI>(rt);
  return recon == 14 ? pick_rt<float, __half2, true, EPI>(rt) : pick_rt<float, __half2, false, EPI>(rt);
}

// Right-hand sides per thread.  Register budget (gfx950, 256-thread workgroups): FP64 tiles
// above 8 and epilogue tiles above 8 spill, so those are capped.
int default_rt(int prec, int n, bool epi) {
  static int forced = [] {
    const char *e = getenv("HISQ_DSLASH_RT");
    return e ? atoi(e) : 0;
  }();
  int cap = forced > 0 ? forced : (prec == HISQ_F64 ? 4 : 8);
  if (prec == HISQ_F64 || epi) cap = cap > 8 ? 8 : cap;
  int rt = 1;
  while (rt * 2 <= cap && rt * 2 <= n && rt < 16) rt *= 2;
  return rt;
}

}  // namespace

int launch_dslash(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in, void *out,
                  bool epi, double mass2, const void *pvec, double *partial, int *nblk_out,
                  const int *active) {
  const Geometry &g = ctx->g;
  const LinkCopy &l = ctx->links[prec];
  if (!l.base)
    return set_err(ctx, HISQ_ERR_STATE, "no %s link copy loaded (see hisq_load_links copies)",
                   prec == HISQ_F64 ? "FP64" : (prec == HISQ_F32 ? "FP32" : "FP16"));
  const int rt = default_rt(prec, n, epi);
  const int ntiles = (n + rt - 1) / rt;
  const int nblk_sites = (g.vh + 255) / 256;
  const int nb = nblk_sites * ntiles;
  const int grid = (nb + 7) / 8 * 8;
  DslashFn fn = epi ? pick<true>(prec, l.recon, rt) : pick<false>(prec, l.recon, rt);
  fn(l.par[out_parity], in, out, g, out_parity, n, ntiles, nblk_sites, mass2, pvec, partial, active,
     dim3(grid), ctx->stream);
  LAUNCHCHK(ctx, "k_dslash");
  if (nblk_out) *nblk_out = nblk_sites;
  return HISQ_OK;
}

extern "C" int hisq_dslash_mrhs(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in,
                                void *out) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!in || !out) return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: null vector pointer");
  if (in == out) return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: in and out alias");
  if (out_parity != 0 && out_parity != 1)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: out_parity must be 0 or 1");
  if (!prec_valid(prec)) return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: bad precision %d", prec);
  if (n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: n = %d outside 1..%d", n, HISQ_MAX_RHS);
  if (!ctx->links_loaded) return set_err(ctx, HISQ_ERR_STATE, "hisq_dslash_mrhs: no links loaded");
  return launch_dslash(ctx, out_parity, prec, n, in, out, false, 0.0, nullptr, nullptr, nullptr);
}

extern "C" int hisq_apply_m(hisq_ctx *ctx, int prec, double mass, int n, const void *in, void *out,
                            double *pq_out) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!in || !out) return set_err(ctx, HISQ_ERR_ARG, "hisq_apply_m: null vector pointer");
  if (in == out) return set_err(ctx, HISQ_ERR_ARG, "hisq_apply_m: in and out alias");
  if (!prec_valid(prec)) return set_err(ctx, HISQ_ERR_ARG, "hisq_apply_m: bad precision %d", prec);
  if (n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_apply_m: n = %d outside 1..%d", n, HISQ_MAX_RHS);
  if (!ctx->links_loaded) return set_err(ctx, HISQ_ERR_STATE, "hisq_apply_m: no links loaded");
  const Geometry &g = ctx->g;
  void *tmp;
  RETCHK(ws_get(ctx, WS_TMP_ODD, size_t(n) * 3 * g.vh * cplx_bytes(prec), &tmp));
  const int nblk = (g.vh + 255) / 256;
  double *partial = nullptr;
  if (pq_out) {
    void *pp;
    RETCHK(ws_get(ctx, WS_PARTIAL, size_t(n) * nblk * sizeof(double), &pp));
    partial = static_cast<double *>(pp);
  }
  RETCHK(launch_dslash(ctx, 1, prec, n, in, tmp, false, 0.0, nullptr, nullptr, nullptr));
  RETCHK(launch_dslash(ctx, 0, prec, n, tmp, out, true, mass * mass, in, partial, nullptr));
  if (pq_out) RETCHK(launch_reduce_partials(ctx, partial, n, nblk, 1, pq_out));
  return HISQ_OK;
}
