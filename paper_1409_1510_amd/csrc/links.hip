// Link packing (one-time): user FP64 [V][4][3][3] links -> per-output-parity planar arrays of
// the 16 hops of Eq. 3 (Section 1), in FP64, FP32 or FP16 storage, with the backward links
// stored already daggered so that every link an output site needs is indexed by that site.
// Optional compressed Naik storage (Sections 1 and 2 name 14- and 9/13-float reconstructions
// without a parametrisation; the readings taken):
//   14: rows 0 and 1 plus a complex scale z with row2 = z * conj(row0 x row1), exact for
//       N = c * U, U in U(3);
//   13: rows 0 and 1 plus a real z (the same with c real and U in SU(3): z = 1 / c);
//    9: N = c * U with c real and U in SU(3): u01, u02, u10, arg u00, arg u20 (the eight-real
//       parametrisation of SU(3) used for GPU lattice QCD by Clark et al. 2010) and c.
#include "internal.hpp"

namespace {

template <typename LT> __device__ inline LT to_link(double re, double im);
template <> __device__ inline double2 to_link<double2>(double re, double im) { return make_double2(re, im); }
template <> __device__ inline float2 to_link<float2>(double re, double im) {
  return make_float2(float(re), float(im));
}
// one correctly rounded double -> binary16 conversion per component
__device__ inline __half to_half(double v) {
  __half_raw h;
  h.data = static_cast<_Float16>(v);
  return __half(h);
}
template <> __device__ inline __half2 to_link<__half2>(double re, double im) {
  return __halves2half2(to_half(re), to_half(im));
}

struct M3 {
  double2 e[3][3];
};

__device__ inline M3 load_m3(const double2 *__restrict__ links, long long lex, int mu, bool dag) {
  const double2 *p = links + (lex * 4 + mu) * 9;
  M3 m;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double2 v = dag ? p[b * 3 + a] : p[a * 3 + b];
      m.e[a][b] = dag ? make_double2(v.x, -v.y) : v;
    }
  return m;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

template <typename LT>
__device__ inline void store_full(LT *__restrict__ dst, int vh, int s, int plane, const M3 &m) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dst[size_t(plane + a * 3 + b) * vh + s] = to_link<LT>(m.e[a][b].x, m.e[a][b].y);
}

// rows 0, 1 and z; returns the relative error of the reconstructed row 2 (FP64).
template <typename LT>
__device__ inline double store_r14(LT *__restrict__ dst, int vh, int s, int plane, const M3 &m) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dst[size_t(plane + a * 3 + b) * vh + s] = to_link<LT>(m.e[a][b].x, m.e[a][b].y);
  const double2 *r0 = m.e[0], *r1 = m.e[1], *r2 = m.e[2];
  double2 c[3];
  c[0] = cconj(csub(cmul(r0[1], r1[2]), cmul(r0[2], r1[1])));
  c[1] = cconj(csub(cmul(r0[2], r1[0]), cmul(r0[0], r1[2])));
  c[2] = cconj(csub(cmul(r0[0], r1[1]), cmul(r0[1], r1[0])));
  int j = 0;
  if (cabs2(c[1]) > cabs2(c[j])) j = 1;
  if (cabs2(c[2]) > cabs2(c[j])) j = 2;
  double den = cabs2(c[j]);
  double2 z = den > 0 ? cmul(r2[j], cconj(c[j])) : make_double2(0.0, 0.0);
  if (den > 0) {
    z.x /= den;
    z.y /= den;
  }
  dst[size_t(plane + 6) * vh + s] = to_link<LT>(z.x, z.y);
  double err = 0, nrm = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    double2 d = csub(cmul(z, c[b]), r2[b]);
    err = fmax(err, sqrt(cabs2(d)));
    nrm = fmax(nrm, sqrt(cabs2(r2[b])));
  }
  return nrm > 0 ? err / nrm : (den > 0 ? err : 1.0);
}

__device__ inline double2 cscale(double2 a, double f) { return make_double2(a.x * f, a.y * f); }

// Maximum entry error of a rebuilt Naik link against the given one, relative to its largest entry.
__device__ inline double rel_err(const M3 &rebuilt, const M3 &m) {
  double err = 0, nrm = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      err = fmax(err, sqrt(cabs2(csub(rebuilt.e[a][b], m.e[a][b]))));
      nrm = fmax(nrm, sqrt(cabs2(m.e[a][b])));
    }
  return nrm > 0 ? err / nrm : err;
}

// Row 2 of a 13-real link: z conj(row0 x row1) with the real z that fits the given row 2 best.
__device__ inline double fit_real_scale(const M3 &m, M3 &rebuilt) {
  const double2 *r0 = m.e[0], *r1 = m.e[1];
  double2 c[3];
  c[0] = cconj(csub(cmul(r0[1], r1[2]), cmul(r0[2], r1[1])));
  c[1] = cconj(csub(cmul(r0[2], r1[0]), cmul(r0[0], r1[2])));
  c[2] = cconj(csub(cmul(r0[0], r1[1]), cmul(r0[1], r1[0])));
  double num = 0, den = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    num += m.e[2][b].x * c[b].x + m.e[2][b].y * c[b].y;  // Re(row2 conj(c))
    den += cabs2(c[b]);
  }
  const double z = den > 0 ? num / den : 0.0;
  rebuilt = m;
#pragma unroll
  for (int b = 0; b < 3; ++b) rebuilt.e[2][b] = cscale(c[b], z);
  return z;
}

// Rows 0 and 1 into their planes; the real z is returned in *scale (the caller stores the 8 Naik
// scales of a site two per complex plane).  Returns the relative error of the reconstructed link
// (FP64).
template <typename LT>
__device__ inline double store_r13(LT *__restrict__ dst, int vh, int s, int plane, double *scale, const M3 &m) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      dst[size_t(plane + a * 3 + b) * vh + s] = to_link<LT>(m.e[a][b].x, m.e[a][b].y);
  M3 r;
  *scale = fit_real_scale(m, r);
  return rel_err(r, m);
}

// N = c U: c the real cube root of det N, then u01, u02, u10 and (arg u00, arg u20) of U = N / c.
// Returns the relative error of N rebuilt from these (FP64) as the kernels rebuild it.
template <typename LT>
__device__ inline double store_r9(LT *__restrict__ dst, int vh, int s, int plane, double *scale, const M3 &m) {
  const double2 d = csub(cmul(m.e[0][0], csub(cmul(m.e[1][1], m.e[2][2]), cmul(m.e[1][2], m.e[2][1]))),
                         csub(cmul(m.e[0][1], csub(cmul(m.e[1][0], m.e[2][2]), cmul(m.e[1][2], m.e[2][0]))),
                              cmul(m.e[0][2], csub(cmul(m.e[1][0], m.e[2][1]), cmul(m.e[1][1], m.e[2][0])))));
  const double c = cbrt(d.x);
  *scale = c;
  if (!(c != 0.0) || !isfinite(c)) return 1.0;
  M3 u;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) u.e[a][b] = cscale(m.e[a][b], 1.0 / c);
  const double th0 = atan2(u.e[0][0].y, u.e[0][0].x), th2 = atan2(u.e[2][0].y, u.e[2][0].x);
  dst[size_t(plane + 0) * vh + s] = to_link<LT>(u.e[0][1].x, u.e[0][1].y);
  dst[size_t(plane + 1) * vh + s] = to_link<LT>(u.e[0][2].x, u.e[0][2].y);
  dst[size_t(plane + 2) * vh + s] = to_link<LT>(u.e[1][0].x, u.e[1][0].y);
  dst[size_t(plane + 3) * vh + s] = to_link<LT>(th0, th2);
  // the reconstruction of the kernels, in FP64 from the exact parameters
  const double2 u01 = u.e[0][1], u02 = u.e[0][2], u10 = u.e[1][0];
  const double nn = cabs2(u01) + cabs2(u02);
  const double a0 = sqrt(fmax(0.0, 1.0 - nn)), b0 = sqrt(fmax(0.0, nn - cabs2(u10)));
  const double2 u00 = make_double2(a0 * cos(th0), a0 * sin(th0)), u20 = make_double2(b0 * cos(th2), b0 * sin(th2));
  const double inv = 1.0 / nn;
  const double2 p = cmul(u20, u02), q = cmul(u01, u10), t = cmul(u01, u20), v = cmul(u02, u10);
  M3 r;
  r.e[0][0] = u00; r.e[0][1] = u01; r.e[0][2] = u02;
  r.e[1][0] = u10;
  r.e[1][1] = cscale(make_double2(cconj(p).x + cmul(cconj(u00), q).x, cconj(p).y + cmul(cconj(u00), q).y), -inv);
  r.e[1][2] = cscale(csub(cconj(t), cmul(cconj(u00), v)), inv);
  r.e[2][0] = u20;
  r.e[2][1] = cscale(csub(cconj(v), cmul(cconj(u00), t)), inv);
  r.e[2][2] = cscale(make_double2(cconj(q).x + cmul(cconj(u00), p).x, cconj(q).y + cmul(cconj(u00), p).y), -inv);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) r.e[a][b] = cscale(r.e[a][b], c);
  return rel_err(r, m);
}

template <typename LT>
__global__ void __launch_bounds__(256)
k_pack_links(const double2 *__restrict__ fat, const double2 *__restrict__ naik, Geometry g,
             int parity, int recon, LT *__restrict__ dst, double *__restrict__ err_part) {
  __shared__ double red[256];
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  double err = 0.0;
  if (s < g.vh) {
    int xh = s % g.lxh;
    int rest = s / g.lxh;
    int y = rest % g.ly;
    rest /= g.ly;
    int z = rest % g.lz;
    int t = rest / g.lz;
    int x = 2 * xh + ((y + z + t + parity) & 1);
    int c[4] = {x, y, z, t};
    int ext[4] = {g.lx, g.ly, g.lz, g.lt};
    long long lex = x + (long long)g.lx * (y + (long long)g.ly * (z + (long long)g.lz * t));
    double scales[8] = {};  // real Naik scales of formats 13 and 9, hops 8..15
    for (int mu = 0; mu < 4; ++mu) {
      int cm1 = c[mu] - 1 < 0 ? c[mu] - 1 + ext[mu] : c[mu] - 1;
      int cm3 = c[mu] - 3 < 0 ? c[mu] - 3 + ext[mu] : c[mu] - 3;
      int cc[4] = {x, y, z, t};
      cc[mu] = cm1;
      long long lex1 = cc[0] + (long long)g.lx * (cc[1] + (long long)g.ly * (cc[2] + (long long)g.lz * cc[3]));
      cc[mu] = cm3;
      long long lex3 = cc[0] + (long long)g.lx * (cc[1] + (long long)g.ly * (cc[2] + (long long)g.lz * cc[3]));
      store_full(dst, g.vh, s, link_plane(mu, recon), load_m3(fat, lex, mu, false));
      store_full(dst, g.vh, s, link_plane(4 + mu, recon), load_m3(fat, lex1, mu, true));
      M3 nf = load_m3(naik, lex, mu, false);
      M3 nb = load_m3(naik, lex3, mu, true);
      if (recon == 14) {
        err = fmax(err, store_r14(dst, g.vh, s, link_plane(8 + mu, recon), nf));
        err = fmax(err, store_r14(dst, g.vh, s, link_plane(12 + mu, recon), nb));
      } else if (recon == 13) {
        err = fmax(err, store_r13(dst, g.vh, s, link_plane(8 + mu, recon), &scales[mu], nf));
        err = fmax(err, store_r13(dst, g.vh, s, link_plane(12 + mu, recon), &scales[4 + mu], nb));
      } else if (recon == 9) {
        err = fmax(err, store_r9(dst, g.vh, s, link_plane(8 + mu, recon), &scales[mu], nf));
        err = fmax(err, store_r9(dst, g.vh, s, link_plane(12 + mu, recon), &scales[4 + mu], nb));
      } else {
        store_full(dst, g.vh, s, link_plane(8 + mu, recon), nf);
        store_full(dst, g.vh, s, link_plane(12 + mu, recon), nb);
      }
    }
    if (recon == 13 || recon == 9)  // hops 8 + 2j and 9 + 2j share a scale plane
      for (int j = 0; j < 4; ++j)
        dst[size_t(naik_scale_plane(8 + 2 * j, recon)) * g.vh + s] = to_link<LT>(scales[2 * j], scales[2 * j + 1]);
    if (!(err <= 1.0)) err = 1.0;  // non-finite reconstruction
  }
  if (err_part) {
    red[threadIdx.x] = err;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) err_part[blockIdx.x] = red[0];
  }
}

}  // namespace

int launch_pack_links(hisq_ctx *ctx, const double *fat, const double *naik, int prec, int recon,
                      int parity, void *dst, double *max_recon_err_host) {
  const Geometry &g = ctx->g;
  int nblk = (g.vh + 255) / 256;
  double *err_part = nullptr;
  if (max_recon_err_host) {
    void *p;
    RETCHK(ws_get(ctx, WS_ERRPART, size_t(nblk) * sizeof(double), &p));
    err_part = static_cast<double *>(p);
  }
  const double2 *f2 = reinterpret_cast<const double2 *>(fat);
  const double2 *n2 = reinterpret_cast<const double2 *>(naik);
  if (prec == HISQ_F64)
    k_pack_links<double2><<<nblk, 256, 0, ctx->stream>>>(f2, n2, g, parity, recon,
                                                         static_cast<double2 *>(dst), err_part);
  else if (prec == HISQ_F32)
    k_pack_links<float2><<<nblk, 256, 0, ctx->stream>>>(f2, n2, g, parity, recon,
                                                        static_cast<float2 *>(dst), err_part);
  else
    k_pack_links<__half2><<<nblk, 256, 0, ctx->stream>>>(f2, n2, g, parity, recon,
                                                         static_cast<__half2 *>(dst), err_part);
  LAUNCHCHK(ctx, "k_pack_links");
  if (max_recon_err_host) {
    std::vector<double> h(nblk);
    HIPCHK(ctx, hipMemcpyAsync(h.data(), err_part, nblk * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double m = 0;
    for (double e : h) m = e > m || e != e ? e : m;
    *max_recon_err_host = m;
  }
  return HISQ_OK;
}
