// Multi-rhs HISQ half Dslash kernel template for gfx950 (Section 1, Eq. 3 and Eq. 4).
//
// One thread owns one output site and a tile of RT right-hand sides (register blocking over rhs,
// Section 2): each link of the site is loaded once per tile and applied to RT neighbour vectors.
// Several tiles of the same sites are kept close together, either as the 4 waves of one
// workgroup (SPB = 64 sites per workgroup: the waves read the same links through the CU's L1 --
// the 2-d site x rhs blocking of Section 2) or as neighbouring workgroups on one XCD (SPB = 256:
// the links are found in that XCD's L2).  Workgroups are remapped so that each XCD owns a
// contiguous range of site blocks.  Hops are accumulated in a fixed order with explicit FMAs, so
// the result for a rhs does not depend on n, on RT or on the workgroup shape.  Which shape is
// fastest depends on the GPU, the lattice and n; the launcher picks it by timing (Section 2,
// automatic tuning of the launch configuration).
//
// Layouts: links as packed by links.hip (planes of V/2 complex per matrix entry, per output
// parity); vectors [n][3][V/2] complex (colour-planar structure of arrays).
#pragma once

#include "internal.hpp"

namespace dslash {

template <typename Real> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

template <bool NT> __device__ inline void ld_link(const double2 *p, double &re, double &im) {
  if constexpr (NT) {
    d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    re = v.x;
    im = v.y;
  } else {
    double2 v = *p;
    re = v.x;
    im = v.y;
  }
}
template <bool NT> __device__ inline void ld_link(const float2 *p, float &re, float &im) {
  if constexpr (NT) {
    f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    re = v.x;
    im = v.y;
  } else {
    float2 v = *p;
    re = v.x;
    im = v.y;
  }
}
template <bool NT> __device__ inline void ld_link(const __half2 *p, float &re, float &im) {
  __half2 h;
  if constexpr (NT) {
    unsigned u = __builtin_nontemporal_load(reinterpret_cast<const unsigned *>(p));
    h = *reinterpret_cast<__half2 *>(&u);
  } else {
    h = *p;
  }
  float2 v = __half22float2(h);
  re = v.x;
  im = v.y;
}

__device__ inline double fmaR(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float fmaR(float a, float b, float c) { return fmaf(a, b, c); }

template <typename Real> struct Lnk {
  Real re[3][3], im[3][3];
};

// Row 2 of a 14-real Naik link from rows 0 and 1 and the stored scale z: z * conj(row0 x row1).
template <typename Real>
__device__ inline void naik_row2(Lnk<Real> &L, Real zr, Real zi) {
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

// Load the link of a hop at site s; a 14-real Naik link gets row 2 = z * conj(row0 x row1).
template <typename Real, typename LT, bool R14, bool NT>
__device__ inline void load_link(const LT *__restrict__ links, int plane, unsigned vh, unsigned s,
                                 Lnk<Real> &L) {
  const LT *p = links + size_t(plane) * vh + s;
  constexpr int rows = R14 ? 2 : 3;
#pragma unroll
  for (int a = 0; a < rows; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ld_link<NT>(p + (a * 3 + b) * vh, L.re[a][b], L.im[a][b]);
  if constexpr (R14) {
    Real zr, zi;
    ld_link<NT>(p + 6 * vh, zr, zi);
    naik_row2(L, zr, zi);
  }
}

// Row 2 of a 13-real Naik link from rows 0 and 1 and the real scale z: z * conj(row0 x row1).
template <typename Real>
__device__ inline void naik_row2_real(Lnk<Real> &L, Real z) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
    Real cr = (L.re[0][b1] * L.re[1][b2] - L.im[0][b1] * L.im[1][b2]) -
              (L.re[0][b2] * L.re[1][b1] - L.im[0][b2] * L.im[1][b1]);
    Real ci = (L.re[0][b1] * L.im[1][b2] + L.im[0][b1] * L.re[1][b2]) -
              (L.re[0][b2] * L.im[1][b1] + L.im[0][b2] * L.re[1][b1]);
    L.re[2][b] = z * cr;
    L.im[2][b] = -(z * ci);
  }
}

__device__ inline void sincos_r(float x, float &s, float &c) { sincosf(x, &s, &c); }
__device__ inline void sincos_r(double x, double &s, double &c) { sincos(x, &s, &c); }

// A 9-real Naik link N = c U with U in SU(3), from u01, u02, u10, the phases th0 = arg u00 and
// th2 = arg u20, and c: |u00| and |u20| follow from the unit norms of row 0 and column 0, and the
// four remaining entries from the orthogonality of rows 1 and 2 to row 0 and from
// row2 = conj(row0 x row1), row1 = conj(row2 x row0) (det U = 1); with n = 1 - |u00|^2:
//   u11 = -(conj(u20 u02) + conj(u00) u01 u10) / n    u12 = (conj(u01 u20) - conj(u00) u02 u10) / n
//   u21 = (conj(u10 u02) - conj(u00) u01 u20) / n     u22 = -(conj(u01 u10) + conj(u00) u02 u20) / n
template <typename Real>
__device__ inline void naik_from9(Lnk<Real> &L, Real u01r, Real u01i, Real u02r, Real u02i, Real u10r,
                                  Real u10i, Real th0, Real th2, Real c) {
  const Real nn = (u01r * u01r + u01i * u01i) + (u02r * u02r + u02i * u02i);
  const Real a2 = Real(1) - nn;
  const Real a0 = sqrt(a2 > Real(0) ? a2 : Real(0));
  const Real b2 = nn - (u10r * u10r + u10i * u10i);
  const Real b0 = sqrt(b2 > Real(0) ? b2 : Real(0));
  Real s0, c0, s2, c2;
  sincos_r(th0, s0, c0);
  sincos_r(th2, s2, c2);
  const Real u00r = a0 * c0, u00i = a0 * s0;
  const Real u20r = b0 * c2, u20i = b0 * s2;
  const Real inv = Real(1) / nn;
  const Real pr = u20r * u02r - u20i * u02i, pi = u20r * u02i + u20i * u02r;  // u20 u02
  const Real qr = u01r * u10r - u01i * u10i, qi = u01r * u10i + u01i * u10r;  // u01 u10
  const Real tr = u01r * u20r - u01i * u20i, ti = u01r * u20i + u01i * u20r;  // u01 u20
  const Real vr = u02r * u10r - u02i * u10i, vi = u02r * u10i + u02i * u10r;  // u02 u10
  const Real u11r = -(pr + (u00r * qr + u00i * qi)) * inv, u11i = -(-pi + (u00r * qi - u00i * qr)) * inv;
  const Real u12r = (tr - (u00r * vr + u00i * vi)) * inv, u12i = (-ti - (u00r * vi - u00i * vr)) * inv;
  const Real u21r = (vr - (u00r * tr + u00i * ti)) * inv, u21i = (-vi - (u00r * ti - u00i * tr)) * inv;
  const Real u22r = -(qr + (u00r * pr + u00i * pi)) * inv, u22i = -(-qi + (u00r * pi - u00i * pr)) * inv;
  L.re[0][0] = c * u00r; L.im[0][0] = c * u00i;
  L.re[0][1] = c * u01r; L.im[0][1] = c * u01i;
  L.re[0][2] = c * u02r; L.im[0][2] = c * u02i;
  L.re[1][0] = c * u10r; L.im[1][0] = c * u10i;
  L.re[1][1] = c * u11r; L.im[1][1] = c * u11i;
  L.re[1][2] = c * u12r; L.im[1][2] = c * u12i;
  L.re[2][0] = c * u20r; L.im[2][0] = c * u20i;
  L.re[2][1] = c * u21r; L.im[2][1] = c * u21i;
  L.re[2][2] = c * u22r; L.im[2][2] = c * u22i;
}

// Load Naik hop k (8..15) at site s of a link array with plane stride vh, rebuilding what the
// storage format NR (18, 14, 13 or 9, see link_plane) leaves out.
template <typename Real, typename LT, int NR, bool NT>
__device__ inline void load_naik(const LT *__restrict__ links, int k, unsigned vh, unsigned s, Lnk<Real> &L) {
  if constexpr (NR == 18 || NR == 14) {
    load_link<Real, LT, NR == 14, NT>(links, link_plane(k, NR), vh, s, L);
  } else if constexpr (NR == 13) {
    const LT *p = links + size_t(link_plane(k, NR)) * vh + s;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) ld_link<NT>(p + (a * 3 + b) * vh, L.re[a][b], L.im[a][b]);
    Real zr, zi;
    ld_link<NT>(links + size_t(naik_scale_plane(k, NR)) * vh + s, zr, zi);
    naik_row2_real(L, (k & 1) ? zi : zr);
  } else {
    static_assert(NR == 9, "Naik storage formats: 18, 14, 13, 9");
    const LT *p = links + size_t(link_plane(k, NR)) * vh + s;
    Real a1r, a1i, a2r, a2i, b0r, b0i, t0, t2, cr, ci;
    ld_link<NT>(p, a1r, a1i);
    ld_link<NT>(p + vh, a2r, a2i);
    ld_link<NT>(p + 2 * vh, b0r, b0i);
    ld_link<NT>(p + 3 * vh, t0, t2);
    ld_link<NT>(links + size_t(naik_scale_plane(k, NR)) * vh + s, cr, ci);
    naik_from9(L, a1r, a1i, a2r, a2i, b0r, b0i, t0, t2, (k & 1) ? ci : cr);
  }
}

// acc += sign * L v for the RT right-hand sides of the tile (sign -1 for backward hops).
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

// LDS forms: the same FMA sequence as apply_hop, but every lane computes every rhs of the tile
// (inactive lanes and rhs read clamped, in-range addresses; only active results are stored), so
// the hops are straight-line code the compiler can schedule across.  rr[r]: the rhs of the tile
// to read for r.  Per-lane offsets are 32-bit: a tile spans less than 4 GB (checked at launch).
template <typename Real, int RT, bool NEG>
__device__ inline void apply_hop_all(const Lnk<Real> &L, const typename CT<Real>::T *__restrict__ in,
                                     unsigned vh, unsigned nbr, const int (&rr)[RT],
                                     Real (&acc_re)[RT][3], Real (&acc_im)[RT][3]) {
  using C = typename CT<Real>::T;
  const char *base = reinterpret_cast<const char *>(in);
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    C v[3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
      v[b] = *reinterpret_cast<const C *>(base + (unsigned(rr[r] * 3 + b) * vh + nbr) * unsigned(sizeof(C)));
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

// apply_hop_all with the gathers as raw buffer loads: the tile's colour planes are one buffer
// (wave-uniform descriptor), the neighbour is a byte offset within a plane (the lane's only
// address operand) and the plane start a scalar offset, so a gather costs no vector address
// arithmetic.
typedef unsigned v2u_t __attribute__((__vector_size__(8)));
typedef unsigned v4u_t __attribute__((__vector_size__(16)));
__device__ inline void buf_load(__amdgpu_buffer_rsrc_t rs, unsigned off, unsigned soff, float2 &v) {
  const v2u_t u = __builtin_amdgcn_raw_buffer_load_b64(rs, off, soff, 0);
  v.x = __uint_as_float(u[0]);
  v.y = __uint_as_float(u[1]);
}
__device__ inline void buf_load(__amdgpu_buffer_rsrc_t rs, unsigned off, unsigned soff, double2 &v) {
  const v4u_t u = __builtin_amdgcn_raw_buffer_load_b128(rs, off, soff, 0);
  v.x = __hiloint2double(int(u[1]), int(u[0]));
  v.y = __hiloint2double(int(u[3]), int(u[2]));
}
template <typename Real, int RT, bool NEG>
__device__ inline void apply_hop_buf(const Lnk<Real> &L, __amdgpu_buffer_rsrc_t rs, unsigned plane_bytes,
                                     unsigned off, const int (&rr)[RT], Real (&acc_re)[RT][3],
                                     Real (&acc_im)[RT][3]) {
  using C = typename CT<Real>::T;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    C v[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) buf_load(rs, off, unsigned(rr[r] * 3 + b) * plane_bytes, v[b]);
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

// apply_hop_buf for the 32-site form: rhs r of a lane sits in the vector offset (off + r * 3
// planes) and the colour plane in the scalar offset, so that the buffer range check covers the
// rhs (a rhs past n reads 0 instead of memory past the vectors).
template <typename Real, int RT, bool NEG>
__device__ inline void apply_hop_buf32(const Lnk<Real> &L, __amdgpu_buffer_rsrc_t rs, unsigned plane_bytes,
                                       unsigned off, Real (&acc_re)[RT][3], Real (&acc_im)[RT][3]) {
  using C = typename CT<Real>::T;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    C v[3];
    const unsigned vo = off + unsigned(r * 3) * plane_bytes;
#pragma unroll
    for (int b = 0; b < 3; ++b) buf_load(rs, vo, unsigned(b) * plane_bytes, v[b]);
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

// Neighbour indices (within the input parity) of output site s at coordinates (x, y, z, t) for
// the four hops of direction mu: +1, -1, +3, -3.
__device__ inline void hop_sites(const Geometry &g, int mu, unsigned s, unsigned rowbase, int x, int y, int z, int t,
                                 unsigned &f1, unsigned &b1, unsigned &f3, unsigned &b3) {
  if (mu == 0) {
    const int xf1 = x + 1 >= g.lx ? x + 1 - g.lx : x + 1;
    const int xb1 = x - 1 < 0 ? x - 1 + g.lx : x - 1;
    const int xf3 = x + 3 >= g.lx ? x + 3 - g.lx : x + 3;
    const int xb3 = x - 3 < 0 ? x - 3 + g.lx : x - 3;
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
}

// Unsigned division by a run-time constant d with a multiply-high, two shifts and two adds
// (Granlund and Montgomery, "Division by invariant integers using multiplication", 1994, the
// unsigned round-up method): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, and
// q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) with t = mulhi(m, n), exact for every
// 32-bit n.  The lattice extents are divisors of this kind; the multipliers are set on the host.
struct FastDiv {
  unsigned m;
  int s1, s2;
};
inline FastDiv make_fastdiv(unsigned d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned long long m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return FastDiv{unsigned(m), l < 1 ? l : 1, l > 1 ? l - 1 : 0};
}
__device__ inline unsigned fast_div(unsigned n, const FastDiv &f) {
  const unsigned t = __umulhi(f.m, n);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Neighbour index (within the input parity) of output site s at (x, y, z, t) for the hop of
// direction mu by d = +1, -1, +3 or -3 (one periodic wrap: every extent is at least 4); the same
// values as hop_sites.
__device__ inline unsigned hop_site(const Geometry &g, int mu, int d, unsigned s, unsigned rowbase, int x, int y,
                                    int z, int t) {
  if (mu == 0) {
    const int xn = x + d;
    return rowbase + ((xn < 0 ? xn + g.lx : (xn >= g.lx ? xn - g.lx : xn)) >> 1);
  }
  const int c = mu == 1 ? y : (mu == 2 ? z : t);
  const int L = mu == 1 ? g.ly : (mu == 2 ? g.lz : g.lt);
  const int S = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
  const int cn = c + d;
  return s + (cn < 0 ? d + L : (cn >= L ? d - L : d)) * S;
}

// Rhs of tile r0 a wave computes: rr[r] (clamped to the last rhs), ract[r] (rhs active);
// returns whether any rhs of the tile is active.  All values are uniform across the wave.
struct Args {
  const void *links;
  const void *in;
  void *out;
  Geometry g;
  int out_parity;
  int n;
  int ntiles;   // ceil(n / RT)
  int ngroups;  // tile groups per site block
  int nsblk;    // site blocks
  double mass2;
  const void *pvec;       // epilogue: q = mass2 * pvec - D in
  double *partial;        // epilogue: Re<pvec, q> per rhs per 64-site wave, [n][ceil(V/2 / 64)]
  const int *active;      // per-rhs mask or null
  int xmap;               // LDS form, XCD map: 0 contiguous ranges, 1 z slabs, 2 y slabs
  int zmap_bps;           //   64-site blocks per (z, t) plane
  int zmap_zr;            //   z-slab map: z slices owned by each XCD (Lz / 8)
  FastDiv div_xh, div_y, div_z;  // division by Lx/2, Ly, Lz (site decoding of the LDS form)
};

template <int RT>
__device__ inline bool tile_rhs(const Args &a, int r0, int (&rr)[RT], bool (&ract)[RT]) {
  bool any = false;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int q = r0 + r;
    ract[r] = q < a.n && (!a.active || a.active[q]);
    rr[r] = q < a.n ? r : a.n - 1 - r0;
    any = any || ract[r];
  }
  return any;
}


// SPB: sites per 256-thread workgroup (256: one tile per workgroup; 64: 4 tiles, one per wave).
template <typename Real, typename LT, int RT, int NR, bool EPI, int SPB, bool NT>
__global__ void __launch_bounds__(256) k_dslash(Args a) {
  using C = typename CT<Real>::T;
  constexpr int TPB = 256 / SPB;  // tiles per workgroup
  const Geometry &g = a.g;
  // XCD-aware order: the hardware deals workgroups round-robin to the 8 XCDs; each XCD gets a
  // contiguous range of logical blocks (all rhs tiles of consecutive site blocks).
  const int nb = a.nsblk * a.ngroups;
  const int chunk = gridDim.x >> 3;
  const int lb = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
  if (lb >= nb) return;  // uniform for the whole workgroup
  const int sblk = lb / a.ngroups;
  const int grp = lb - sblk * a.ngroups;
  const int tile = grp * TPB + (TPB == 1 ? 0 : int(threadIdx.x) / SPB);
  const int r0 = tile * RT;
  const unsigned vh = g.vh;
  const unsigned s = sblk * SPB + (threadIdx.x % SPB);
  const bool valid = s < vh && tile < a.ntiles;
  const size_t tile_off = size_t(r0) * 3 * vh;
  const C *__restrict__ in = static_cast<const C *>(a.in) + tile_off;
  C *__restrict__ out = static_cast<C *>(a.out) + tile_off;
  const LT *__restrict__ links = static_cast<const LT *>(a.links);

  bool act[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) act[r] = valid && (r0 + r < a.n) && (!a.active || a.active[r0 + r]);

  Real acc_re[RT][3], acc_im[RT][3];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc_re[r][c] = acc_im[r][c] = Real(0);

  if (valid) {
    const int xh = s % g.lxh;
    int rest = s / g.lxh;
    const int y = rest % g.ly;
    rest /= g.ly;
    const int z = rest % g.lz;
    const int t = rest / g.lz;
    const int x = 2 * xh + ((y + z + t + a.out_parity) & 1);
    const unsigned rowbase = s - xh;
    constexpr int recon = NR;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      unsigned f1, b1, f3, b3;
      if (mu == 0) {
        const int xf1 = x + 1 >= g.lx ? x + 1 - g.lx : x + 1;
        const int xb1 = x - 1 < 0 ? x - 1 + g.lx : x - 1;
        const int xf3 = x + 3 >= g.lx ? x + 3 - g.lx : x + 3;
        const int xb3 = x - 3 < 0 ? x - 3 + g.lx : x - 3;
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
      Lnk<Real> Lk;
      load_link<Real, LT, false, NT>(links, link_plane(mu, recon), vh, s, Lk);
      apply_hop<Real, RT, false>(Lk, in, vh, f1, act, acc_re, acc_im);
      load_link<Real, LT, false, NT>(links, link_plane(4 + mu, recon), vh, s, Lk);
      apply_hop<Real, RT, true>(Lk, in, vh, b1, act, acc_re, acc_im);
      load_naik<Real, LT, NR, NT>(links, 8 + mu, vh, s, Lk);
      apply_hop<Real, RT, false>(Lk, in, vh, f3, act, acc_re, acc_im);
      load_naik<Real, LT, NR, NT>(links, 12 + mu, vh, s, Lk);
      apply_hop<Real, RT, true>(Lk, in, vh, b3, act, acc_re, acc_im);
    }
  }

  if constexpr (!EPI) {
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      if (!act[r]) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C o;
        o.x = acc_re[r][c];
        o.y = acc_im[r][c];
        out[(unsigned)(r * 3 + c) * vh + s] = o;
      }
    }
  } else {
    // q = m^2 p - D_eo t, and per-rhs FP64 partials of Re<p, q> per 64-site wave (the same
    // grouping for every workgroup shape, so the reduction is independent of the launch shape)
    const C *__restrict__ pv = static_cast<const C *>(a.pvec) + tile_off;
    const Real m2 = Real(a.mass2);
    double dot[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      dot[r] = 0.0;
      if (!act[r]) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const C p = pv[(unsigned)(r * 3 + c) * vh + s];
        C o;
        o.x = fmaR(m2, p.x, -acc_re[r][c]);
        o.y = fmaR(m2, p.y, -acc_im[r][c]);
        out[(unsigned)(r * 3 + c) * vh + s] = o;
        dot[r] = fma(double(p.x), double(o.x), dot[r]);
        dot[r] = fma(double(p.y), double(o.y), dot[r]);
      }
    }
    if (a.partial && tile < a.ntiles) {
      const int lane = threadIdx.x & 63;
      const unsigned wave_sites = s - lane;  // first site of this wave (SPB is a multiple of 64)
      const unsigned nw = (vh + 63) / 64;
      if (wave_sites < vh) {
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          double v = dot[r];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
          if (lane == 0 && r0 + r < a.n) a.partial[size_t(r0 + r) * nw + wave_sites / 64] = v;
        }
      }
    }
  }
}

// Word 3 of a raw buffer descriptor on CDNA (32-bit data format, no swizzle, no stride): a
// plain byte-addressed range checked against its size.
constexpr int kBufWord3 = 0x00020000;

// LDS of the whole-site form: the stored link planes of 64 sites, for 14-real Naik links the
// 8 x 3 rebuilt row-2 entries in the arithmetic type, then the neighbour table (16 byte
// offsets per site).
constexpr size_t kNbrTableBytes = size_t(16) * 64 * sizeof(unsigned);
// rebuilt Naik entries kept in LDS per site (arithmetic type): row 2 of the 8 Naik links for
// formats 14 and 13, all 9 entries for format 9
constexpr int lds_rebuilt_entries(int nr) { return (nr == 14 || nr == 13) ? 24 : (nr == 9 ? 72 : 0); }
// stored planes copied into LDS per site: all of them, except for format 9, whose Naik links are
// rebuilt straight from global memory (keeping their 36 stored planes in LDS as well would take
// a workgroup past half of a CU's LDS, one workgroup per CU instead of two)
constexpr int lds_staged_planes(int nr) { return nr == 9 ? 72 : link_planes_total(nr); }
template <typename Real, typename LT, int NR> constexpr size_t lds_nbr_offset() {
  return size_t(lds_staged_planes(NR)) * 64 * sizeof(LT) + size_t(lds_rebuilt_entries(NR)) * 64 * sizeof(typename CT<Real>::T);
}

// LDS of the 32-site form: the same pieces for 32 sites.
template <typename Real, typename LT, bool R14> constexpr size_t lds32_nbr_offset() {
  return size_t(R14 ? 128 : 144) * 32 * sizeof(LT) + (R14 ? size_t(24) * 32 * sizeof(typename CT<Real>::T) : 0);
}
constexpr size_t kNbrTable32Bytes = size_t(16) * 32 * sizeof(unsigned);

// 64-site block of LDS-form workgroup `bid` (of `nbid`, dealt round-robin to the 8 XCDs) under
// the XCD map of the launch (false: none).
__device__ inline bool lds_block_at(const Args &a, int bid, int nbid, int &sblk) {
  const Geometry &g = a.g;
  if (a.xmap == 2 || a.xmap == 3) {
    // XCD k owns the blocks [k, k+1) * bps/8 of every (z, t) plane (with Lx = 32: four y rows).
    // Map 2 walks the planes z-major (t fastest): the sites in flight on an XCD span a few z
    // slices of a thin slab whose t extent is the whole lattice, so the t and z neighbours they
    // gather (the Naik hops reach 3 slices away) are mostly still in that XCD's L2 while Lt is
    // small.  Map 3 walks z tiles of 4 slices, t within a tile and z fastest: a z neighbour is at
    // most 3 planes back in the walk inside a tile and a t neighbour 4 or 12, so on large
    // lattices (64^3 x 16: 4 blocks per plane and XCD, 16 planes in flight) the window that has
    // to stay in L2 no longer grows with Lt; hops that cross a tile boundary re-fetch.
    const int k = bid & 7, j = bid >> 3;
    const int bpx = a.zmap_bps >> 3;
    const int w = j / bpx;  // position of the (z, t) plane in the XCD's walk
    int z, t;
    if (a.xmap == 2) {
      z = w / g.lt;
      t = w - z * g.lt;
    } else {
      const int tile = w / (4 * g.lt), rem = w - tile * 4 * g.lt;
      t = rem >> 2;
      z = tile * 4 + (rem & 3);
    }
    if (z >= g.lz) return false;
    sblk = (t * g.lz + z) * a.zmap_bps + k * bpx + (j - w * bpx);
  } else if (a.xmap == 1) {
    // XCD k owns the z slices [k Lz/8, (k+1) Lz/8) for every t: the z and t neighbours of its
    // sites stay mostly in its own L2 (with contiguous chunks, Lt = 8 would give each XCD a single
    // t slice and send every t hop to another XCD's data)
    const int k = bid & 7, j = bid >> 3;
    const int per_t = a.zmap_zr * a.zmap_bps;
    const int t = j / per_t;
    if (t >= g.lt) return false;
    const int rem = j - t * per_t;
    const int zl = rem / a.zmap_bps;
    sblk = (t * g.lz + k * a.zmap_zr + zl) * a.zmap_bps + (rem - zl * a.zmap_bps);
  } else {
    const int chunk = nbid >> 3;
    sblk = (bid & 7) * chunk + (bid >> 3);
    if (sblk >= a.nsblk) return false;
  }
  return true;
}
__device__ inline bool lds_block(const Args &a, int &sblk) { return lds_block_at(a, blockIdx.x, gridDim.x, sblk); }

// Naik link k (0..7: hops 8 + k) of lane `lane` from the staged LDS copy: rows 0 and 1 from the
// stored planes and, for 14- and 13-real links, row 2 from the entries rebuilt once per site;
// 9-real links entirely from the rebuilt entries.  (SB: sites per LDS plane)
template <typename Real, typename LT, int NR, int SB = 64>
__device__ inline void load_naik_lds(const LT *__restrict__ sl, const typename CT<Real>::T *__restrict__ row2,
                                     int k, int lane, Lnk<Real> &L) {
  if constexpr (NR == 18) {
    load_link<Real, LT, false, false>(sl, link_plane(8 + k, NR), unsigned(SB), unsigned(lane), L);
  } else if constexpr (NR == 9) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const typename CT<Real>::T v = row2[(k * 9 + a * 3 + b) * SB + lane];
        L.re[a][b] = v.x;
        L.im[a][b] = v.y;
      }
  } else {
    const LT *p = sl + link_plane(8 + k, NR) * SB + lane;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) ld_link<false>(p + (a * 3 + b) * SB, L.re[a][b], L.im[a][b]);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const typename CT<Real>::T v = row2[(k * 3 + b) * SB + lane];
      L.re[2][b] = v.x;
      L.im[2][b] = v.y;
    }
  }
}

// Write one rhs tile of an LDS-form workgroup: w = acc, or for the fused M form
// q = m2 p - acc with the per-64-site FP64 partials of Re<p, q> (all 64 lanes of the wave take
// part in the reduction; the partial of block sblk is written by lane 0).
template <typename Real, int RT, bool EPI>
__device__ inline void store_tile(const Args &a, int r0, unsigned s, int lane, int sblk, const bool (&act)[RT],
                                  const Real (&acc_re)[RT][3], const Real (&acc_im)[RT][3]) {
  using C = typename CT<Real>::T;
  const unsigned vh = a.g.vh;
  const size_t tile_off = size_t(r0) * 3 * vh;
  C *__restrict__ out = static_cast<C *>(a.out) + tile_off;
  if constexpr (!EPI) {
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      if (!act[r]) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C o;
        o.x = acc_re[r][c];
        o.y = acc_im[r][c];
        out[(unsigned)(r * 3 + c) * vh + s] = o;
      }
    }
  } else {
    const C *__restrict__ pv = static_cast<const C *>(a.pvec) + tile_off;
    const Real m2 = Real(a.mass2);
    double dot[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      dot[r] = 0.0;
      if (!act[r]) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const C p = pv[(unsigned)(r * 3 + c) * vh + s];
        C o;
        o.x = fmaR(m2, p.x, -acc_re[r][c]);
        o.y = fmaR(m2, p.y, -acc_im[r][c]);
        out[(unsigned)(r * 3 + c) * vh + s] = o;
        dot[r] = fma(double(p.x), double(o.x), dot[r]);
        dot[r] = fma(double(p.y), double(o.y), dot[r]);
      }
    }
    if (a.partial) {
      const unsigned nw = (vh + 63) / 64;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        double v = dot[r];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0 && r0 + r < a.n) a.partial[size_t(r0 + r) * nw + sblk] = v;
      }
    }
  }
}

// raw link-entry load (optionally non-temporal) for LDS staging
template <bool NT> __device__ inline float2 ld_raw(const float2 *p) {
  if constexpr (NT) {
    const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
    return *reinterpret_cast<const float2 *>(&u);
  } else {
    return *p;
  }
}
template <bool NT> __device__ inline double2 ld_raw(const double2 *p) {
  if constexpr (NT) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    double2 o;
    o.x = v.x;
    o.y = v.y;
    return o;
  } else {
    return *p;
  }
}
template <bool NT> __device__ inline __half2 ld_raw(const __half2 *p) {
  if constexpr (NT) {
    const unsigned u = __builtin_nontemporal_load(reinterpret_cast<const unsigned *>(p));
    return *reinterpret_cast<const __half2 *>(&u);
  } else {
    return *p;
  }
}

// LDS-staged form: a workgroup of 64 sites x WPB waves first copies the links of its 64 sites
// (all 16 hops) into LDS, then the waves loop over the rhs tiles (wave w takes tiles w, w+WPB,
// ...), reading the links from LDS for every tile.  Only WPB*RT rhs of a site block are in
// flight at a time, so the neighbour vectors other workgroups gather are far more likely to be
// found in L2 than when every thread holds all n rhs; the links still come from HBM once.
// Same site order, hop order and FMA sequence per rhs as k_dslash (bit-identical output), and
// the same per-64-site grouping of the fused <p, Mp> partials.
// (the second launch bound is the waves per SIMD: two workgroups share a CU -- with 16 waves at
// most 64 VGPRs, with 8 at most 128 -- except with FP64 links, whose 147 KB take a CU's LDS alone)
template <typename Real, typename LT, int RT, int NR, bool EPI, int WPB, bool NT>
__global__ void __launch_bounds__(64 * WPB, WPB / 4 * (sizeof(LT) > 8 ? 1 : 2)) k_dslash_lds(Args a) {
  static_assert(WPB == 4 || WPB == 8 || WPB == 16, "4, 8 or 16 waves per workgroup");
  using C = typename CT<Real>::T;
  constexpr int recon = NR;
  constexpr int PL = lds_staged_planes(NR);  // stored planes per site staged in LDS
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LT *sl = reinterpret_cast<LT *>(smem_raw);
  const Geometry &g = a.g;
  int sblk;
  if (!lds_block(a, sblk)) return;  // uniform for the whole workgroup
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const unsigned vh = g.vh;
  const unsigned s = sblk * 64 + lane;
  const bool valid = s < vh;
  const LT *__restrict__ links = static_cast<const LT *>(a.links);
  // every lane computes: a lane past the last site works on site 0 (in-range addresses) and
  // stores nothing
  const unsigned sc = valid ? s : 0u;
  // stage the links of the 64 sites: plane-major, lane-minor (conflict-free LDS access); each
  // wave issues a batch of CH plane loads before it writes any of them, so their latencies
  // overlap.  With NT the global loads carry the non-temporal hint, so the streamed links do
  // not push the neighbour vectors out of L2.
  if constexpr (PL % WPB == 0 && (PL / WPB) % (PL / WPB % 9 == 0 ? 9 : 8) == 0) {
    constexpr int PPW = PL / WPB;
    constexpr int CH = PPW % 9 == 0 ? 9 : 8;
#pragma unroll 1
    for (int c0 = 0; c0 < PPW; c0 += CH) {
      LT v[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) v[i] = ld_raw<NT>(links + size_t(wave + (c0 + i) * WPB) * vh + sc);
#pragma unroll
      for (int i = 0; i < CH; ++i) sl[(wave + (c0 + i) * WPB) * 64 + lane] = v[i];
    }
  } else {  // plane counts that do not split into whole batches (Naik formats 13 and 9)
    constexpr int PPW = (PL + WPB - 1) / WPB;
    constexpr int CH = 8;
#pragma unroll 1
    for (int c0 = 0; c0 < PPW; c0 += CH) {
      LT v[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int pl = wave + (c0 + i) * WPB;
        if (pl < PL) v[i] = ld_raw<NT>(links + size_t(pl) * vh + sc);
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int pl = wave + (c0 + i) * WPB;
        if (pl < PL) sl[pl * 64 + lane] = v[i];
      }
    }
  }
  // 14-, 13- and 9-real Naik links: rebuild what the format leaves out once per site (not once
  // per rhs tile) into LDS entries of the arithmetic type after the staged planes, with the same
  // arithmetic as load_naik: the whole link for 9 here, from global memory; row 2 for 14 and 13
  // from the staged planes after the barrier below
  C *row2 = reinterpret_cast<C *>(sl + PL * 64);
  if constexpr (NR == 9) {
    for (int item = threadIdx.x; item < 8 * 64; item += 64 * WPB) {
      const int k = item >> 6, ln = item & 63;
      const unsigned site = sblk * 64 + ln;
      Lnk<Real> Lk;
      load_naik<Real, LT, NR, NT>(links, 8 + k, vh, site < vh ? site : 0u, Lk);
#pragma unroll
      for (int ra = 0; ra < 3; ++ra)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          C v;
          v.x = Lk.re[ra][b];
          v.y = Lk.im[ra][b];
          row2[(k * 9 + ra * 3 + b) * 64 + ln] = v;
        }
    }
  }
  // neighbour table: the byte offsets (within a colour plane) of the 16 neighbours of the 64
  // sites, [mu][site][+1, -1, +3, -3], built once per workgroup (one hop per wave and lane with
  // 16 waves) so the rhs-tile loop does no site arithmetic
  unsigned *nbt = reinterpret_cast<unsigned *>(smem_raw + lds_nbr_offset<Real, LT, NR>());
  {
    const unsigned q1 = fast_div(sc, a.div_xh);
    const unsigned q2 = fast_div(q1, a.div_y);
    const unsigned q3 = fast_div(q2, a.div_z);
    const int xh = int(sc - q1 * unsigned(g.lxh));
    const int y = int(q1 - q2 * unsigned(g.ly));
    const int z = int(q2 - q3 * unsigned(g.lz));
    const int t = int(q3);
    const int x = 2 * xh + ((y + z + t + a.out_parity) & 1);
    const unsigned rowbase = sc - unsigned(xh);
    for (int h = wave; h < 16; h += WPB) {
      const int mu = h >> 2, k = h & 3;
      const int d = k == 0 ? 1 : (k == 1 ? -1 : (k == 2 ? 3 : -3));
      nbt[(mu * 64 + lane) * 4 + k] = hop_site(g, mu, d, sc, rowbase, x, y, z, t) * unsigned(sizeof(C));
    }
  }
  __syncthreads();
  if constexpr (NR == 14 || NR == 13) {
    for (int item = threadIdx.x; item < 8 * 64; item += 64 * WPB) {
      const int k = item >> 6, ln = item & 63;
      Lnk<Real> Lk;
      load_naik<Real, LT, NR, false>(sl, 8 + k, 64u, unsigned(ln), Lk);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        C v;
        v.x = Lk.re[2][b];
        v.y = Lk.im[2][b];
        row2[(k * 3 + b) * 64 + ln] = v;
      }
    }
    __syncthreads();
  }
  // a tile spans RT * 3 colour planes of less than 4 GiB in all (checked at launch)
  const unsigned plane_bytes = vh * unsigned(sizeof(C));
  for (int tile = wave; tile < a.ntiles; tile += WPB) {
    const int r0 = tile * RT;
    int rr[RT];
    bool ract[RT];
    if (!tile_rhs<RT>(a, r0, rr, ract)) {  // the whole tile is inactive (uniform)
      if constexpr (EPI) {
        if (a.partial && lane == 0) {
          const unsigned nw = (vh + 63) / 64;
#pragma unroll
          for (int r = 0; r < RT; ++r)
            if (r0 + r < a.n) a.partial[size_t(r0 + r) * nw + sblk] = 0.0;
        }
      }
      continue;
    }
    const char *in = static_cast<const char *>(a.in) + size_t(r0) * 3 * plane_bytes;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(in), short(0), int(RT * 3 * plane_bytes), kBufWord3);
    Real acc_re[RT][3], acc_im[RT][3];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc_re[r][c] = acc_im[r][c] = Real(0);
    // hop order as in k_dslash: per mu, fat fwd, fat bwd, Naik fwd, Naik bwd
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const uint4 nb = reinterpret_cast<const uint4 *>(nbt)[mu * 64 + lane];
      Lnk<Real> Lk;
      load_link<Real, LT, false, false>(sl, link_plane(mu, recon), 64u, lane, Lk);
      apply_hop_buf<Real, RT, false>(Lk, rs, plane_bytes, nb.x, rr, acc_re, acc_im);
      load_link<Real, LT, false, false>(sl, link_plane(4 + mu, recon), 64u, lane, Lk);
      apply_hop_buf<Real, RT, true>(Lk, rs, plane_bytes, nb.y, rr, acc_re, acc_im);
      load_naik_lds<Real, LT, NR>(sl, row2, mu, lane, Lk);
      apply_hop_buf<Real, RT, false>(Lk, rs, plane_bytes, nb.z, rr, acc_re, acc_im);
      load_naik_lds<Real, LT, NR>(sl, row2, 4 + mu, lane, Lk);
      apply_hop_buf<Real, RT, true>(Lk, rs, plane_bytes, nb.w, rr, acc_re, acc_im);
    }
    bool act[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) act[r] = valid && ract[r];
    store_tile<Real, RT, EPI>(a, r0, s, lane, sblk, act, acc_re, acc_im);
  }
}

// 32-site LDS form (plain half Dslash): a workgroup of 32 sites x WPB waves stages half the links
// of the whole-site form, so that an FP64 workgroup (74 KB) shares a CU with another (and an
// FP32 or FP16 one with three).  The two 32-lane halves of a wave take different rhs: lane
// (site i, half h) computes rhs r0 + h RT + r of a tile of 2 RT rhs.  Workgroups 2j and 2j+1 of
// an XCD take the two halves of the 64-site block the XCD map gives for j.  The rhs offset of a
// lane goes into the buffer loads' vector offset, so a rhs past n reads past the buffer's range
// (returns 0) and is not stored.  Same hop order and FMA sequence per rhs as k_dslash
// (bit-identical output).  The second launch bound: FP64 two workgroups per CU, else four.
template <typename Real, typename LT, int RT, bool R14, int WPB, bool NT>
__global__ void __launch_bounds__(64 * WPB, WPB / 4 * (sizeof(LT) > 8 ? 2 : 4)) k_dslash_lds32(Args a) {
  static_assert(WPB == 4 || WPB == 8, "4 or 8 waves per workgroup");
  using C = typename CT<Real>::T;
  constexpr int recon = R14 ? 14 : 18;
  constexpr int PL = R14 ? 128 : 144;  // stored planes per site
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LT *sl = reinterpret_cast<LT *>(smem_raw);
  const Geometry &g = a.g;
  const int bx = blockIdx.x;
  int sblk;
  if (!lds_block_at(a, ((bx >> 3) >> 1) * 8 + (bx & 7), gridDim.x >> 1, sblk)) return;  // uniform
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int si = lane & 31, h = lane >> 5;
  const unsigned vh = g.vh;
  const unsigned s = sblk * 64 + ((bx >> 3) & 1) * 32 + si;
  const bool valid = s < vh;
  const unsigned sc = valid ? s : 0u;
  const LT *__restrict__ links = static_cast<const LT *>(a.links);
  // stage the links of the 32 sites, [plane][32]: a wave load covers planes 2 pp and 2 pp + 1
  {
    constexpr int PPW = PL / 2 / WPB;  // plane pairs per wave
    constexpr int CH = PPW % 9 == 0 ? 9 : 8;
    static_assert(PPW % CH == 0, "whole batches");
#pragma unroll 1
    for (int c0 = 0; c0 < PPW; c0 += CH) {
      LT v[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) v[i] = ld_raw<NT>(links + size_t(2 * (wave + (c0 + i) * WPB) + h) * vh + sc);
#pragma unroll
      for (int i = 0; i < CH; ++i) sl[(2 * (wave + (c0 + i) * WPB) + h) * 32 + si] = v[i];
    }
  }
  // neighbour table [mu][site][+1, -1, +3, -3] (byte offsets within a colour plane)
  unsigned *nbt = reinterpret_cast<unsigned *>(smem_raw + lds32_nbr_offset<Real, LT, R14>());
  {
    const unsigned q1 = fast_div(sc, a.div_xh);
    const unsigned q2 = fast_div(q1, a.div_y);
    const unsigned q3 = fast_div(q2, a.div_z);
    const int xh = int(sc - q1 * unsigned(g.lxh));
    const int y = int(q1 - q2 * unsigned(g.ly));
    const int z = int(q2 - q3 * unsigned(g.lz));
    const int t = int(q3);
    const int x = 2 * xh + ((y + z + t + a.out_parity) & 1);
    const unsigned rowbase = sc - unsigned(xh);
    for (int hp = 2 * wave + h; hp < 16; hp += 2 * WPB) {
      const int mu = hp >> 2, k = hp & 3;
      const int d = k == 0 ? 1 : (k == 1 ? -1 : (k == 2 ? 3 : -3));
      nbt[(mu * 32 + si) * 4 + k] = hop_site(g, mu, d, sc, rowbase, x, y, z, t) * unsigned(sizeof(C));
    }
  }
  __syncthreads();
  C *row2 = reinterpret_cast<C *>(sl + PL * 32);
  if constexpr (R14) {
    for (int item = threadIdx.x; item < 8 * 32; item += 64 * WPB) {
      const int k = item >> 5, ln = item & 31;
      Lnk<Real> Lk;
      load_link<Real, LT, true, false>(sl, link_plane(8 + k, recon), 32u, ln, Lk);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        C v;
        v.x = Lk.re[2][b];
        v.y = Lk.im[2][b];
        row2[(k * 3 + b) * 32 + ln] = v;
      }
    }
    __syncthreads();
  }

  const unsigned plane_bytes = vh * unsigned(sizeof(C));
  for (int tile = wave; tile < a.ntiles; tile += WPB) {
    const int r0 = tile * 2 * RT;
    const int q0 = r0 + h * RT;  // this lane's first rhs
    bool act[RT];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      act[r] = q0 + r < a.n && (!a.active || a.active[q0 + r]);
      any = any || act[r];
    }
    if (!__builtin_amdgcn_ballot_w64(any)) continue;  // the whole tile is inactive (uniform)
    const char *in = static_cast<const char *>(a.in) + size_t(r0) * 3 * plane_bytes;
    // the rhs of the tile that exist: a lane's gathers past them are out of range
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char *>(in), short(0), int(unsigned(min(2 * RT, a.n - r0)) * 3u * plane_bytes), kBufWord3);
    Real acc_re[RT][3], acc_im[RT][3];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc_re[r][c] = acc_im[r][c] = Real(0);
    const unsigned hoff = unsigned(h * RT * 3) * plane_bytes;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const uint4 nb = reinterpret_cast<const uint4 *>(nbt)[mu * 32 + si];
      Lnk<Real> Lk;
      load_link<Real, LT, false, false>(sl, link_plane(mu, recon), 32u, unsigned(si), Lk);
      apply_hop_buf32<Real, RT, false>(Lk, rs, plane_bytes, nb.x + hoff, acc_re, acc_im);
      load_link<Real, LT, false, false>(sl, link_plane(4 + mu, recon), 32u, unsigned(si), Lk);
      apply_hop_buf32<Real, RT, true>(Lk, rs, plane_bytes, nb.y + hoff, acc_re, acc_im);
      load_naik_lds<Real, LT, R14 ? 14 : 18, 32>(sl, row2, mu, si, Lk);
      apply_hop_buf32<Real, RT, false>(Lk, rs, plane_bytes, nb.z + hoff, acc_re, acc_im);
      load_naik_lds<Real, LT, R14 ? 14 : 18, 32>(sl, row2, 4 + mu, si, Lk);
      apply_hop_buf32<Real, RT, true>(Lk, rs, plane_bytes, nb.w + hoff, acc_re, acc_im);
    }
    C *__restrict__ out = static_cast<C *>(a.out) + size_t(r0) * 3 * vh;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      if (!(valid && act[r])) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C o;
        o.x = acc_re[r][c];
        o.y = acc_im[r][c];
        out[(unsigned)((h * RT + r) * 3 + c) * vh + s] = o;
      }
    }
  }
}

// Direction-pipelined LDS form: the workgroup (64 sites x WPB waves) stages the links of one
// direction mu at a time -- X(x,mu), X(x-mu,mu)^dag, N(x,mu), N(x-3mu,mu)^dag -- in one of two
// LDS buffers.  While the waves apply direction mu to their rhs tiles, the links of mu+1 are
// already being loaded into registers, so link streaming overlaps the neighbour gathers and
// the FMAs, and a workgroup needs a quarter of the LDS of the whole-site form.  Each wave keeps
// the accumulators of TPW rhs tiles across the four directions (ntiles <= TPW * WPB).  Same hop
// order and FMA sequence per rhs as k_dslash, same per-64-site partials.
// (16 waves x 1 tile: at most 64 VGPRs, so that two workgroups share a CU)
template <typename Real, typename LT, int RT, bool R14, bool EPI, int WPB, int TPW, bool NT>
__global__ void __launch_bounds__(64 * WPB, (WPB == 16 && TPW == 1) ? 8 : 1) k_dslash_mu(Args a) {
  using C = typename CT<Real>::T;
  constexpr int recon = R14 ? 14 : 18;
  constexpr int NS = R14 ? 7 : 9;            // stored planes of a Naik hop
  constexpr int PM = 18 + 2 * NS;            // stored planes of one direction
  constexpr int NPF = (PM + WPB - 1) / WPB;  // planes each wave stages
  constexpr int BUF = PM * 64;               // link entries per buffer
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LT *sl = reinterpret_cast<LT *>(smem_raw);          // two buffers of BUF entries
  C *row2 = reinterpret_cast<C *>(sl + 2 * BUF);      // 14-real Naik: two buffers of 2 x 3 x 64
  int sblk;
  if (!lds_block(a, sblk)) return;  // uniform for the whole workgroup
  const Geometry &g = a.g;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const unsigned vh = g.vh;
  const unsigned s = sblk * 64 + lane;
  const bool valid = s < vh;
  const LT *__restrict__ links = static_cast<const LT *>(a.links);

  LT pre[NPF];
  // issue the loads of direction mu's planes (local plane p -> stored plane)
  auto fetch = [&](int mu) {
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int p = wave + i * WPB;
      if (p < PM && valid) {
        int gp;
        if (p < 9) gp = link_plane(mu, recon) + p;
        else if (p < 18) gp = link_plane(4 + mu, recon) + p - 9;
        else if (p < 18 + NS) gp = link_plane(8 + mu, recon) + p - 18;
        else gp = link_plane(12 + mu, recon) + p - 18 - NS;
        pre[i] = ld_raw<NT>(links + size_t(gp) * vh + s);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int p = wave + i * WPB;
      if (p < PM && valid) sl[buf * BUF + p * 64 + lane] = pre[i];
    }
  };
  // 14-real Naik: row 2 of the two Naik hops of the buffer, once per site
  auto rebuild = [&](int buf) {
    if constexpr (R14) {
      for (int item = threadIdx.x; item < 2 * 64; item += 64 * WPB) {
        const int k = item >> 6, ln = item & 63;
        Lnk<Real> Lk;
        load_link<Real, LT, true, false>(sl + buf * BUF, 18 + k * NS, 64u, ln, Lk);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          C v;
          v.x = Lk.re[2][b];
          v.y = Lk.im[2][b];
          row2[(buf * 6 + k * 3 + b) * 64 + ln] = v;
        }
      }
      __syncthreads();
    }
  };

  // every lane computes: a lane past the last site works on site 0 and stores nothing
  const unsigned sc = valid ? s : 0u;
  int x, y, z, t;
  {
    const int xh = sc % g.lxh;
    int rest = sc / g.lxh;
    y = rest % g.ly;
    rest /= g.ly;
    z = rest % g.lz;
    t = rest / g.lz;
    x = 2 * xh + ((y + z + t + a.out_parity) & 1);
  }
  const unsigned rowbase = sc - (x >> 1);

  int rr[TPW][RT];
  bool ract[TPW][RT], tact[TPW];
  Real acc_re[TPW][RT][3], acc_im[TPW][RT][3];
#pragma unroll
  for (int tw = 0; tw < TPW; ++tw) {
    const int tile = wave + tw * WPB;
    tact[tw] = tile < a.ntiles && tile_rhs<RT>(a, tile * RT, rr[tw], ract[tw]);
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc_re[tw][r][c] = acc_im[tw][r][c] = Real(0);
  }

  fetch(0);
  stash(0);
  __syncthreads();
  rebuild(0);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    const int buf = mu & 1;
    if (mu < 3) fetch(mu + 1);
    unsigned f1, b1, f3, b3;
    hop_sites(g, mu, sc, rowbase, x, y, z, t, f1, b1, f3, b3);
    const LT *bl = sl + buf * BUF;
#pragma unroll
    for (int tw = 0; tw < TPW; ++tw) {
      if (!tact[tw]) continue;  // uniform
      const C *__restrict__ in = static_cast<const C *>(a.in) + size_t((wave + tw * WPB) * RT) * 3 * vh;
      Lnk<Real> Lk;
      load_link<Real, LT, false, false>(bl, 0, 64u, lane, Lk);
      apply_hop_all<Real, RT, false>(Lk, in, vh, f1, rr[tw], acc_re[tw], acc_im[tw]);
      load_link<Real, LT, false, false>(bl, 9, 64u, lane, Lk);
      apply_hop_all<Real, RT, true>(Lk, in, vh, b1, rr[tw], acc_re[tw], acc_im[tw]);
      if constexpr (!R14) {
        load_link<Real, LT, false, false>(bl, 18, 64u, lane, Lk);
      } else {
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
          for (int cb = 0; cb < 3; ++cb) ld_link<false>(bl + (18 + ra * 3 + cb) * 64 + lane, Lk.re[ra][cb], Lk.im[ra][cb]);
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
          const C v = row2[(buf * 6 + cb) * 64 + lane];
          Lk.re[2][cb] = v.x;
          Lk.im[2][cb] = v.y;
        }
      }
      apply_hop_all<Real, RT, false>(Lk, in, vh, f3, rr[tw], acc_re[tw], acc_im[tw]);
      if constexpr (!R14) {
        load_link<Real, LT, false, false>(bl, 27, 64u, lane, Lk);
      } else {
#pragma unroll
        for (int ra = 0; ra < 2; ++ra)
#pragma unroll
          for (int cb = 0; cb < 3; ++cb)
            ld_link<false>(bl + (18 + NS + ra * 3 + cb) * 64 + lane, Lk.re[ra][cb], Lk.im[ra][cb]);
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
          const C v = row2[(buf * 6 + 3 + cb) * 64 + lane];
          Lk.re[2][cb] = v.x;
          Lk.im[2][cb] = v.y;
        }
      }
      apply_hop_all<Real, RT, true>(Lk, in, vh, b3, rr[tw], acc_re[tw], acc_im[tw]);
    }
    if (mu < 3) {
      stash(buf ^ 1);
      __syncthreads();
      rebuild(buf ^ 1);
    }
  }
#pragma unroll
  for (int tw = 0; tw < TPW; ++tw) {
    const int tile = wave + tw * WPB;
    if (tile >= a.ntiles) continue;
    const int r0 = tile * RT;
    if (!tact[tw]) {  // inactive tile: zero partials, nothing stored
      if constexpr (EPI) {
        if (a.partial && lane == 0) {
          const unsigned nw = (vh + 63) / 64;
#pragma unroll
          for (int r = 0; r < RT; ++r)
            if (r0 + r < a.n) a.partial[size_t(r0 + r) * nw + sblk] = 0.0;
        }
      }
      continue;
    }
    bool act[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) act[r] = valid && ract[tw][r];
    store_tile<Real, RT, EPI>(a, r0, s, lane, sblk, act, acc_re[tw], acc_im[tw]);
  }
}

using DslashFn = void (*)(const Args &, dim3, hipStream_t);

template <typename Real, typename LT, int RT, int NR, bool EPI, int SPB, bool NT>
void launch_t(const Args &a, dim3 grid, hipStream_t st) {
  k_dslash<Real, LT, RT, NR, EPI, SPB, NT><<<grid, 256, 0, st>>>(a);
}

template <typename Real, typename LT, int RT, int NR, bool EPI, int WPB, bool NT>
void launch_lds(const Args &a, dim3 grid, hipStream_t st) {
  constexpr size_t lds = lds_nbr_offset<Real, LT, NR>() + kNbrTableBytes;
  k_dslash_lds<Real, LT, RT, NR, EPI, WPB, NT><<<grid, 64 * WPB, lds, st>>>(a);
}

template <typename Real, typename LT, int RT, bool R14, bool EPI, int WPB, int TPW, bool NT>
void launch_mu(const Args &a, dim3 grid, hipStream_t st) {
  constexpr size_t lds = 2 * size_t(R14 ? 32 : 36) * 64 * sizeof(LT) +
                         (R14 ? size_t(12) * 64 * sizeof(typename CT<Real>::T) : 0);
  k_dslash_mu<Real, LT, RT, R14, EPI, WPB, TPW, NT><<<grid, 64 * WPB, lds, st>>>(a);
}

// direction-pipelined forms: 4 = 16 waves x 1 tile each, 5 = 16 waves x 2 tiles, 6 = 8 waves x 2
template <typename Real, typename LT, bool R14, bool EPI, bool NT>
DslashFn pick_mu(int rt, int lds) {
  if (rt == 1) {
    if (lds == 4) return launch_mu<Real, LT, 1, R14, EPI, 16, 1, NT>;
    if (lds == 5) return launch_mu<Real, LT, 1, R14, EPI, 16, 2, NT>;
    if (lds == 6) return launch_mu<Real, LT, 1, R14, EPI, 8, 2, NT>;
  } else if (rt == 2) {
    if (lds == 4) return launch_mu<Real, LT, 2, R14, EPI, 16, 1, NT>;
    if (lds == 5) return launch_mu<Real, LT, 2, R14, EPI, 16, 2, NT>;
    if (lds == 6) return launch_mu<Real, LT, 2, R14, EPI, 8, 2, NT>;
  }
  return nullptr;
}

template <typename Real, typename LT, int NR, bool EPI, int WPB, bool NT>
DslashFn pick_lds_rt(int rt) {
  switch (rt) {
    case 1: return launch_lds<Real, LT, 1, NR, EPI, WPB, NT>;
    case 2: return launch_lds<Real, LT, 2, NR, EPI, WPB, NT>;
    case 4:
      if constexpr (WPB <= 8) return launch_lds<Real, LT, 4, NR, EPI, WPB, NT>;
      return nullptr;
    default: return nullptr;
  }
}

template <typename Real, typename LT, int RT, bool R14, int WPB, bool NT>
void launch_lds32(const Args &a, dim3 grid, hipStream_t st) {
  constexpr size_t lds = lds32_nbr_offset<Real, LT, R14>() + kNbrTable32Bytes;
  k_dslash_lds32<Real, LT, RT, R14, WPB, NT><<<grid, 64 * WPB, lds, st>>>(a);
}

// 32-site form: lds 1 = 4 waves, 2 = 8 waves; rhs_per_thread 1 or 2; plain half Dslash only
template <typename Real, typename LT, bool R14, bool NT>
DslashFn pick_lds32(int rt, int lds) {
  if (lds == 1) return rt == 1 ? launch_lds32<Real, LT, 1, R14, 4, NT> : (rt == 2 ? launch_lds32<Real, LT, 2, R14, 4, NT> : nullptr);
  if (lds == 2) return rt == 1 ? launch_lds32<Real, LT, 1, R14, 8, NT> : (rt == 2 ? launch_lds32<Real, LT, 2, R14, 8, NT> : nullptr);
  return nullptr;
}

// lds: 1 = 4 waves per 64-site workgroup, 2 = 8 waves, 3 = 16 waves; 4-6 the direction-pipelined
// forms (Naik formats 18 and 14 only)
template <typename Real, typename LT, int NR, bool EPI, bool NT>
DslashFn pick_lds(int rt, int lds) {
  if constexpr (sizeof(LT) > 8) {  // FP64: the whole-site forms only (one workgroup per CU)
    if (lds == 1) return pick_lds_rt<Real, LT, NR, EPI, 4, NT>(rt);
    if (lds == 2) return pick_lds_rt<Real, LT, NR, EPI, 8, NT>(rt);
    if (lds == 3) return pick_lds_rt<Real, LT, NR, EPI, 16, NT>(rt);
    return nullptr;
  } else {
    if (lds >= 4) {
      if constexpr (NR == 18 || NR == 14) return pick_mu<Real, LT, NR == 14, EPI, NT>(rt, lds);
      return nullptr;
    }
    if (lds == 1) return pick_lds_rt<Real, LT, NR, EPI, 4, NT>(rt);
    if (lds == 2) return pick_lds_rt<Real, LT, NR, EPI, 8, NT>(rt);
    if (lds == 3) return pick_lds_rt<Real, LT, NR, EPI, 16, NT>(rt);
    return nullptr;
  }
}

template <typename Real, typename LT, int NR, bool EPI, int SPB, bool NT>
DslashFn pick_rt(int rt) {
  switch (rt) {
    case 1: return launch_t<Real, LT, 1, NR, EPI, SPB, NT>;
    case 2: return launch_t<Real, LT, 2, NR, EPI, SPB, NT>;
    case 4: return launch_t<Real, LT, 4, NR, EPI, SPB, NT>;
    case 8: return launch_t<Real, LT, 8, NR, EPI, SPB, NT>;
    default:
      if constexpr (!EPI && sizeof(Real) == 4) return launch_t<Real, LT, 16, NR, EPI, SPB, NT>;
      return nullptr;
  }
}

// Every form for Naik storage format NR (the 32-site and direction-pipelined forms: 18 and 14).
template <typename Real, typename LT, int NR>
DslashFn pick_all(bool epi, int rt, int spb, bool nt, int lds) {
  if (lds) {
    if (spb == 32) {
      if constexpr (NR == 18 || NR == 14)
        return epi ? nullptr : (nt ? pick_lds32<Real, LT, NR == 14, true>(rt, lds) : pick_lds32<Real, LT, NR == 14, false>(rt, lds));
      return nullptr;
    }
    if (spb != 64) return nullptr;
    if (nt) return epi ? pick_lds<Real, LT, NR, true, true>(rt, lds) : pick_lds<Real, LT, NR, false, true>(rt, lds);
    return epi ? pick_lds<Real, LT, NR, true, false>(rt, lds) : pick_lds<Real, LT, NR, false, false>(rt, lds);
  }
  if (spb != 64 && spb != 256) return nullptr;
  if (epi) {
    if (spb == 64) return nt ? pick_rt<Real, LT, NR, true, 64, true>(rt) : pick_rt<Real, LT, NR, true, 64, false>(rt);
    return nt ? pick_rt<Real, LT, NR, true, 256, true>(rt) : pick_rt<Real, LT, NR, true, 256, false>(rt);
  }
  if (spb == 64) return nt ? pick_rt<Real, LT, NR, false, 64, true>(rt) : pick_rt<Real, LT, NR, false, 64, false>(rt);
  return nt ? pick_rt<Real, LT, NR, false, 256, true>(rt) : pick_rt<Real, LT, NR, false, 256, false>(rt);
}

}  // namespace dslash

// per-precision tables (dslash_f64.hip, dslash_f32.hip, dslash_f16.hip)
dslash::DslashFn dslash_fn_f64(bool epi, int rt, int spb, bool nt, int lds);
dslash::DslashFn dslash_fn_f32(bool epi, int recon, int rt, int spb, bool nt, int lds);
dslash::DslashFn dslash_fn_f16(bool epi, int recon, int rt, int spb, bool nt, int lds);
