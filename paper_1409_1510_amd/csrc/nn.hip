// Learned gauge-covariant preconditioner for the even-odd CG: a linear network of L layers,
// each a per-site channel mixing (C x C complex, C = 8; bf16 MFMA in the BF16 mode) followed by a
// per-channel gauge-covariant one-hop stencil over the fat links X of Eq. 3:
//
//   phi_1 = W_in (x) E(r);  psi_l = S(a_l, phi_l);  phi_l = W_l psi_{l-1} (l >= 2);
//   N r = sum_c W_out[c] psi_L[c] (full lattice);
//   direct form: z = R_even N r;  Gram form: z = N^dag N r (Hermitian positive semi-definite).
//   S(a, phi)_c(x) = a[0,c] phi_c(x) + sum_mu (a[1+mu,c] X(x,mu) phi_c(x+mu)
//                                            + a[5+mu,c] X(x-mu,mu)^dag phi_c(x-mu)).
//
// Forward and backward (adjoint network, Wirtinger weight gradients) are hand-written kernels;
// training uses Adam (Kingma and Ba 2014) on FP32 master weights.  Activations live on the full
// lattice in parity-split order (site index p * V/2 + cb) as [batch][colour][site][channel]
// complex, stored in FP32 or BF16 with FP32 arithmetic.
//
// Parameters (complex, canonical order): W_in[C]; for l = 1..L: (W_l[C][C] [out][in] if l >= 2),
// a_l[9][C]; W_out[C].  Hop h: 0 self, 1+mu forward, 5+mu backward.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <vector>

#include "cg_state.hpp"
#include "internal.hpp"

namespace {

constexpr int NC = 8;         // channels
constexpr int NR = 2 * NC;    // reals per (site, colour)
constexpr int kThreads = 256;

// ---- activation storage -------------------------------------------------------------------
using bf16 = unsigned short;

__device__ inline float bf2f(bf16 h) { return __uint_as_float(unsigned(h) << 16); }
__device__ inline bf16 f2bf(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return bf16(0x7fc0);
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16(u >> 16);
}

template <typename AT> struct Act;
template <> struct Act<float> {
  __device__ static void load(const float *p, float (&v)[NR]) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float4 t = q[k];
      v[4 * k] = t.x;
      v[4 * k + 1] = t.y;
      v[4 * k + 2] = t.z;
      v[4 * k + 3] = t.w;
    }
  }
  __device__ static void store(float *p, const float (&v)[NR]) {
    float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  }
};
template <> struct Act<bf16> {
  __device__ static void load(const bf16 *p, float (&v)[NR]) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      uint4 t = q[k];
      unsigned w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[8 * k + 2 * j] = __uint_as_float(w[j] << 16);
        v[8 * k + 2 * j + 1] = __uint_as_float(w[j] & 0xffff0000u);
      }
    }
  }
  __device__ static void store(bf16 *p, const float (&v)[NR]) {
    uint4 *q = reinterpret_cast<uint4 *>(p);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      unsigned w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        w[j] = unsigned(f2bf(v[8 * k + 2 * j])) | (unsigned(f2bf(v[8 * k + 2 * j + 1])) << 16);
      q[k] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
};

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

struct Site {
  unsigned p, s;      // parity, cb index
  int x, y, z, t;
};

__device__ inline Site decode(const Geometry &g, unsigned X) {
  Site o;
  o.p = X >= unsigned(g.vh);
  o.s = X - o.p * g.vh;
  const int xh = o.s % g.lxh;
  int rest = o.s / g.lxh;
  o.y = rest % g.ly;
  rest /= g.ly;
  o.z = rest % g.lz;
  o.t = rest / g.lz;
  o.x = 2 * xh + ((o.y + o.z + o.t + int(o.p)) & 1);
  return o;
}

// full-lattice index of the neighbour of site q along mu (dir = +1 or -1), 1 hop
__device__ inline unsigned nbr1(const Geometry &g, const Site &q, int mu, int dir) {
  unsigned cb;
  if (mu == 0) {
    int xn = q.x + dir;
    xn = xn >= g.lx ? xn - g.lx : (xn < 0 ? xn + g.lx : xn);
    cb = q.s - (q.x >> 1) + (xn >> 1);
  } else {
    const int c = mu == 1 ? q.y : (mu == 2 ? q.z : q.t);
    const int L = mu == 1 ? g.ly : (mu == 2 ? g.lz : g.lt);
    const int S = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
    int cn = c + dir;
    const int d = cn >= L ? dir - L : (cn < 0 ? dir + L : dir);
    cb = q.s + d * S;
  }
  return (1u - q.p) * g.vh + cb;
}

struct NNArgs {
  Geometry g;
  const void *links[2];   // per output parity, packed link planes (fat hops are planes 0..71)
  int batch;
  size_t sample_stride;   // elements of AT per sample = 3 * V * NR
};

__device__ inline float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// packed BF16 pairs (x = low half) and their FP32-accumulating dot product a.x b.x + a.y b.y + c
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline float dot2(unsigned a, unsigned b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), c, false);
}
__device__ inline unsigned pack_bf(float lo, float hi) {  // round to nearest even
  bf16x2 v;
  v.x = static_cast<__bf16>(lo);
  v.y = static_cast<__bf16>(hi);
  return __builtin_bit_cast(unsigned, v);
}

// stencil coefficient of hop h, channel c (the adjoint stencil uses conj(a[adj(h)]))
template <bool ADJ>
__device__ inline float2 coef(const float2 *__restrict__ a, int h, int c) {
  if (!ADJ) return a[h * NC + c];
  const int ha = h == 0 ? 0 : (h < 5 ? h + 4 : h - 4);
  float2 v = a[ha * NC + c];
  return make_float2(v.x, -v.y);
}

// out = S(a, in) (or S^dag(a, in)) on the full lattice for every sample.
template <typename AT, typename LT, bool ADJ>
__global__ void __launch_bounds__(kThreads)
k_nn_stencil(NNArgs A, const AT *__restrict__ in, AT *__restrict__ out, const float2 *__restrict__ a) {
  const Geometry &g = A.g;
  const unsigned X = (blockIdx.x / A.batch) * kThreads + threadIdx.x;  // samples fastest: the
  const unsigned V = 2u * g.vh;                                        // links are shared in L2
  if (X >= V) return;
  const size_t boff = size_t(blockIdx.x % A.batch) * A.sample_stride;
  const AT *__restrict__ ib = in + boff;
  AT *__restrict__ ob = out + boff;
  const Site q = decode(g, X);
  float acc[3][NR];
  {
    float v[NR];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      Act<AT>::load(ib + (size_t(col) * V + X) * NR, v);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float2 w = coef<ADJ>(a, 0, c);
        acc[col][2 * c] = w.x * v[2 * c] - w.y * v[2 * c + 1];
        acc[col][2 * c + 1] = w.x * v[2 * c + 1] + w.y * v[2 * c];
      }
    }
  }
  const LT *__restrict__ lk = static_cast<const LT *>(A.links[q.p]);
#pragma unroll 1
  for (int h = 1; h < 9; ++h) {
    const int mu = (h - 1) & 3;
    const bool fwd = h < 5;
    const unsigned nb = nbr1(g, q, mu, fwd ? 1 : -1);
    const int plane = link_plane(fwd ? mu : 4 + mu, 18);  // fat planes are the same for r14
    float lr[3][3], li[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ld_link(lk + size_t(plane + 3 * i + j) * g.vh + q.s, lr[i][j], li[i][j]);
    float v[3][NR];
#pragma unroll
    for (int col = 0; col < 3; ++col) Act<AT>::load(ib + (size_t(col) * V + nb) * NR, v[col]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float2 w = coef<ADJ>(a, h, c);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        float tr = 0.f, ti = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          tr = fmaf(lr[i][j], v[j][2 * c], tr);
          tr = fmaf(-li[i][j], v[j][2 * c + 1], tr);
          ti = fmaf(lr[i][j], v[j][2 * c + 1], ti);
          ti = fmaf(li[i][j], v[j][2 * c], ti);
        }
        acc[i][2 * c] = fmaf(w.x, tr, fmaf(-w.y, ti, acc[i][2 * c]));
        acc[i][2 * c + 1] = fmaf(w.x, ti, fmaf(w.y, tr, acc[i][2 * c + 1]));
      }
    }
  }
#pragma unroll
  for (int col = 0; col < 3; ++col) Act<AT>::store(ob + (size_t(col) * V + X) * NR, acc[col]);
}

// ---- fused inference layer -----------------------------------------------------------------
// One pass of the network for inference (no activations kept for a backward pass): the stencil
// S(a) (or S^dag(a)) of one layer followed in registers by what comes next, so that each layer
// reads and writes the activations once:
//   input  : an activation buffer, or (IN_VEC) a vector v [b][3][vin_sites] (vin_sites = V/2:
//            zero on odd sites) lifted to the channels with coefficients win (conjugated if
//            in_conj): phi_c = win[c] v, so every hop applies its link once for all channels;
//   output : (OUT_VEC) the readout z = sum_c wout[c] psi_c (conjugated if out_conj) on the first
//            out_sites sites ([b][3][out_sites]), or the activation mix W psi (W^dag if
//            mix_conjt) written to an activation buffer on the full lattice.
// The arithmetic is FP32; stored activations are AT.
struct FusedArgs {
  NNArgs A;
  const void *in;          // activation buffer or float2 vector
  void *out;               // activation buffer or float2 vector
  const float2 *a;         // stencil coefficients a[9][C]
  const float2 *w;         // post-mix matrix W[C][C] ([out][in])
  const float2 *win, *wout;
  unsigned vin_sites, out_sites;
  int in_conj, out_conj, mix_conjt;
};

// Grid: one workgroup per (256-site block, sample), samples fastest, so the workgroups that
// run together share their sites' links through L2.
template <typename AT, typename LT, bool ADJ, bool IN_VEC, bool OUT_VEC>
__global__ void __launch_bounds__(kThreads) k_nn_layer(FusedArgs F) {
  constexpr bool PK = std::is_same<AT, bf16>::value;  // BF16 storage: packed BF16 dot products
  const Geometry &g = F.A.g;
  const unsigned V = 2u * g.vh;
  const int b = blockIdx.x % F.A.batch;
  const unsigned X = (blockIdx.x / F.A.batch) * kThreads + threadIdx.x;
  // BF16 mix: the C x C complex matrix as packed pairs, (Re m, -Im m) and (Im m, Re m)
  __shared__ unsigned mixr[PK && !OUT_VEC ? NC * NC : 1], mixi[PK && !OUT_VEC ? NC * NC : 1];
  if constexpr (PK && !OUT_VEC) {
    if (threadIdx.x < NC * NC) {
      const int p = threadIdx.x / NC, c = threadIdx.x % NC;
      float2 m = F.mix_conjt ? F.w[c * NC + p] : F.w[p * NC + c];
      if (F.mix_conjt) m.y = -m.y;
      mixr[threadIdx.x] = pack_bf(m.x, -m.y);
      mixi[threadIdx.x] = pack_bf(m.y, m.x);
    }
    __syncthreads();
  }
  if (X >= F.out_sites) return;
  const Site q = decode(g, X);
  float acc[3][NR];
  float2 cin[NC];  // IN_VEC: a[h][c] * win[c] is formed per hop
  if constexpr (IN_VEC) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      cin[c] = F.win[c];
      if (F.in_conj) cin[c].y = -cin[c].y;
    }
  }
  const AT *ib = nullptr;
  const float2 *vb = nullptr;
  if constexpr (IN_VEC) vb = static_cast<const float2 *>(F.in) + size_t(b) * 3 * F.vin_sites;
  else ib = static_cast<const AT *>(F.in) + size_t(b) * F.A.sample_stride;
  // self term
  if constexpr (IN_VEC) {
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      const float2 v = X < F.vin_sites ? vb[size_t(col) * F.vin_sites + X] : make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float2 w = cmulf(coef<ADJ>(F.a, 0, c), cin[c]);
        acc[col][2 * c] = w.x * v.x - w.y * v.y;
        acc[col][2 * c + 1] = w.x * v.y + w.y * v.x;
      }
    }
  } else {
    float v[NR];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      Act<AT>::load(ib + (size_t(col) * V + X) * NR, v);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float2 w = coef<ADJ>(F.a, 0, c);
        acc[col][2 * c] = w.x * v[2 * c] - w.y * v[2 * c + 1];
        acc[col][2 * c + 1] = w.x * v[2 * c + 1] + w.y * v[2 * c];
      }
    }
  }
  // an even-site input vector has nothing on the neighbours of an even site
  const bool hops = !IN_VEC || F.vin_sites > unsigned(g.vh) || q.p == 1;
  const LT *__restrict__ lk = static_cast<const LT *>(F.A.links[q.p]);
  if (hops) {
#pragma unroll 1
    for (int h = 1; h < 9; ++h) {
      const int mu = (h - 1) & 3;
      const bool fwd = h < 5;
      const unsigned nb = nbr1(g, q, mu, fwd ? 1 : -1);
      const int plane = link_plane(fwd ? mu : 4 + mu, 18);
      float lr[3][3], li[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ld_link(lk + size_t(plane + 3 * i + j) * g.vh + q.s, lr[i][j], li[i][j]);
      if constexpr (IN_VEC) {
        if (nb >= F.vin_sites) continue;
        float2 v[3];
#pragma unroll
        for (int col = 0; col < 3; ++col) v[col] = vb[size_t(col) * F.vin_sites + nb];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          float tr = 0.f, ti = 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            tr = fmaf(lr[i][j], v[j].x, tr);
            tr = fmaf(-li[i][j], v[j].y, tr);
            ti = fmaf(lr[i][j], v[j].y, ti);
            ti = fmaf(li[i][j], v[j].x, ti);
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const float2 w = cmulf(coef<ADJ>(F.a, h, c), cin[c]);
            acc[i][2 * c] = fmaf(w.x, tr, fmaf(-w.y, ti, acc[i][2 * c]));
            acc[i][2 * c + 1] = fmaf(w.x, ti, fmaf(w.y, tr, acc[i][2 * c + 1]));
          }
        }
      } else if constexpr (PK) {
        // (U v)_i of channel c as packed BF16 dot products: Re = (Re u, -Im u).(Re v, Im v),
        // Im = (Im u, Re u).(Re v, Im v), accumulated in FP32
        unsigned ur[3][3], ui[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            ur[i][j] = pack_bf(lr[i][j], -li[i][j]);
            ui[i][j] = pack_bf(li[i][j], lr[i][j]);
          }
        unsigned vw[3][NC];
#pragma unroll
        for (int col = 0; col < 3; ++col) {
          const uint4 *q4 = reinterpret_cast<const uint4 *>(ib + (size_t(col) * V + nb) * NR);
          const uint4 t0 = q4[0], t1 = q4[1];
          vw[col][0] = t0.x; vw[col][1] = t0.y; vw[col][2] = t0.z; vw[col][3] = t0.w;
          vw[col][4] = t1.x; vw[col][5] = t1.y; vw[col][6] = t1.z; vw[col][7] = t1.w;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const float2 w = coef<ADJ>(F.a, h, c);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            float tr = 0.f, ti = 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              tr = dot2(ur[i][j], vw[j][c], tr);
              ti = dot2(ui[i][j], vw[j][c], ti);
            }
            acc[i][2 * c] = fmaf(w.x, tr, fmaf(-w.y, ti, acc[i][2 * c]));
            acc[i][2 * c + 1] = fmaf(w.x, ti, fmaf(w.y, tr, acc[i][2 * c + 1]));
          }
        }
      } else {
        float v[3][NR];
#pragma unroll
        for (int col = 0; col < 3; ++col) Act<AT>::load(ib + (size_t(col) * V + nb) * NR, v[col]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const float2 w = coef<ADJ>(F.a, h, c);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            float tr = 0.f, ti = 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              tr = fmaf(lr[i][j], v[j][2 * c], tr);
              tr = fmaf(-li[i][j], v[j][2 * c + 1], tr);
              ti = fmaf(lr[i][j], v[j][2 * c + 1], ti);
              ti = fmaf(li[i][j], v[j][2 * c], ti);
            }
            acc[i][2 * c] = fmaf(w.x, tr, fmaf(-w.y, ti, acc[i][2 * c]));
            acc[i][2 * c + 1] = fmaf(w.x, ti, fmaf(w.y, tr, acc[i][2 * c + 1]));
          }
        }
      }
    }
  }
  if constexpr (OUT_VEC) {
    float2 *zb = static_cast<float2 *>(F.out) + size_t(b) * 3 * F.out_sites;
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float wr = F.wout[c].x, wi = F.out_conj ? -F.wout[c].y : F.wout[c].y;
        re = fmaf(wr, acc[col][2 * c], fmaf(-wi, acc[col][2 * c + 1], re));
        im = fmaf(wr, acc[col][2 * c + 1], fmaf(wi, acc[col][2 * c], im));
      }
      zb[size_t(col) * F.out_sites + X] = make_float2(re, im);
    }
  } else if constexpr (PK) {
    // mix in packed BF16 (psi rounded to BF16, as the MFMA mixing of the training path does)
    AT *ob = static_cast<AT *>(F.out) + size_t(b) * F.A.sample_stride;
    unsigned pw[3][NC], ow[3][NC];
#pragma unroll
    for (int col = 0; col < 3; ++col)
#pragma unroll
      for (int c = 0; c < NC; ++c) pw[col][c] = pack_bf(acc[col][2 * c], acc[col][2 * c + 1]);
#pragma unroll 2
    for (int p = 0; p < NC; ++p) {  // one matrix row at a time from LDS (broadcast reads)
      unsigned mr[NC], mi[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        mr[c] = mixr[p * NC + c];
        mi[c] = mixi[p * NC + c];
      }
#pragma unroll
      for (int col = 0; col < 3; ++col) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          re = dot2(mr[c], pw[col][c], re);
          im = dot2(mi[c], pw[col][c], im);
        }
        ow[col][p] = pack_bf(re, im);
      }
    }
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      uint4 *q4 = reinterpret_cast<uint4 *>(ob + (size_t(col) * V + X) * NR);
      q4[0] = make_uint4(ow[col][0], ow[col][1], ow[col][2], ow[col][3]);
      q4[1] = make_uint4(ow[col][4], ow[col][5], ow[col][6], ow[col][7]);
    }
  } else {
    AT *ob = static_cast<AT *>(F.out) + size_t(b) * F.A.sample_stride;
#pragma unroll
    for (int col = 0; col < 3; ++col) {
      float o[NR];
#pragma unroll
      for (int p = 0; p < NC; ++p) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          float2 m = F.mix_conjt ? F.w[c * NC + p] : F.w[p * NC + c];
          if (F.mix_conjt) m.y = -m.y;
          re = fmaf(m.x, acc[col][2 * c], fmaf(-m.y, acc[col][2 * c + 1], re));
          im = fmaf(m.x, acc[col][2 * c + 1], fmaf(m.y, acc[col][2 * c], im));
        }
        o[2 * p] = re;
        o[2 * p + 1] = im;
      }
      Act<AT>::store(ob + (size_t(col) * V + X) * NR, o);
    }
  }
}

// Real 16 x 16 form of the complex channel mixing M (out = M in), interleaved (re, im) per
// channel: R[2o][2i] = Re M, R[2o][2i+1] = -Im M, R[2o+1][2i] = Im M, R[2o+1][2i+1] = Re M.
// CONJT: M = W^dag (M[o][i] = conj(W[i][o])).
template <bool CONJT>
__device__ inline float mix_real(const float2 *__restrict__ W, int row, int col) {
  const int o = row >> 1, i = col >> 1;
  float2 m = CONJT ? W[i * NC + o] : W[o * NC + i];
  if (CONJT) m.y = -m.y;
  const bool ro = row & 1, ci = col & 1;
  if (!ro && !ci) return m.x;
  if (!ro && ci) return -m.y;
  if (ro && !ci) return m.y;
  return m.x;
}

// out[col] = M in[col] for every (sample, colour, site) column, FP32 FMAs.
template <typename AT, bool CONJT>
__global__ void __launch_bounds__(kThreads)
k_nn_mix_fma(const AT *__restrict__ in, AT *__restrict__ out, size_t ncols, const float2 *__restrict__ W) {
  __shared__ float R[NR][NR];
  {
    const int r = threadIdx.x / NR, c = threadIdx.x % NR;
    R[r][c] = mix_real<CONJT>(W, r, c);
  }
  __syncthreads();
  const size_t col = size_t(blockIdx.x) * kThreads + threadIdx.x;
  if (col >= ncols) return;
  float v[NR], o[NR];
  Act<AT>::load(in + col * NR, v);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NR; ++c) s = fmaf(R[r][c], v[c], s);
    o[r] = s;
  }
  Act<AT>::store(out + col * NR, o);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// out[col] = M in[col] with v_mfma_f32_16x16x16_bf16: per instruction a wave multiplies the
// 16 x 16 real mixing matrix (A operand) by 16 columns (B operand).  Operand layout for wave64:
// lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16], and receives D[4(l/16)+j][l%16], j=0..3.
// Columns are contiguous 16-value records, so the B read and D write of a lane are 8 bytes.
template <bool CONJT>
__global__ void __launch_bounds__(kThreads)
k_nn_mix_mfma(const bf16 *__restrict__ in, bf16 *__restrict__ out, size_t ncols,
              const float2 *__restrict__ W) {
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
  bf16x4 a;
#pragma unroll
  for (int j = 0; j < 4; ++j) a[j] = short(f2bf(mix_real<CONJT>(W, m, 4 * kq + j)));
  const size_t wave = (size_t(blockIdx.x) * kThreads + threadIdx.x) >> 6;
  const size_t nwaves = (size_t(gridDim.x) * kThreads) >> 6;
  const size_t ngroups = ncols / 16;  // ncols is a multiple of 16 (3 * V, V even and >= 16)
  for (size_t grp = wave; grp < ngroups; grp += nwaves) {
    const size_t col = grp * 16 + m;
    const uint2 raw = *reinterpret_cast<const uint2 *>(in + col * NR + 4 * kq);
    bf16x4 b;
    b[0] = short(raw.x & 0xffffu);
    b[1] = short(raw.x >> 16);
    b[2] = short(raw.y & 0xffffu);
    b[3] = short(raw.y >> 16);
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d, 0, 0, 0);
    uint2 o;
    o.x = unsigned(f2bf(d[0])) | (unsigned(f2bf(d[1])) << 16);
    o.y = unsigned(f2bf(d[2])) | (unsigned(f2bf(d[3])) << 16);
    *reinterpret_cast<uint2 *>(out + col * NR + 4 * kq) = o;
  }
}

// out[b][col][X][c] = w[c] * (X < vs ? v[b][col][X] : 0); w = coefficients (conj if CONJW).
// vs = V/2 for an even-site vector (zero on odd sites), V for a full-lattice vector.
template <typename AT, bool CONJW>
__global__ void __launch_bounds__(kThreads)
k_nn_embed(const float2 *__restrict__ v, unsigned vs, AT *__restrict__ out, NNArgs A,
           const float2 *__restrict__ w) {
  const Geometry &g = A.g;
  const unsigned V = 2u * g.vh;
  const unsigned X = blockIdx.x * kThreads + threadIdx.x;
  if (X >= V) return;
  const int b = blockIdx.y;
  float o[NR];
#pragma unroll
  for (int col = 0; col < 3; ++col) {
    float2 r = make_float2(0.f, 0.f);
    if (X < vs) r = v[(size_t(b) * 3 + col) * vs + X];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      float2 wc = w[c];
      if (CONJW) wc.y = -wc.y;
      const float2 z = cmulf(wc, r);
      o[2 * c] = z.x;
      o[2 * c + 1] = z.y;
    }
    Act<AT>::store(out + size_t(b) * A.sample_stride + (size_t(col) * V + X) * NR, o);
  }
}

// z[b][col][s] = sum_c w[c] act[b][col][s][c] (conj(w[c]) if CONJW) for s < vs (V/2: even
// sites; V: the full lattice)
template <typename AT, bool CONJW>
__global__ void __launch_bounds__(kThreads)
k_nn_readout(const AT *__restrict__ act, float2 *__restrict__ z, unsigned vs, NNArgs A,
             const float2 *__restrict__ w) {
  const Geometry &g = A.g;
  const unsigned V = 2u * g.vh;
  const unsigned s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= vs) return;
  const int b = blockIdx.y;
#pragma unroll
  for (int col = 0; col < 3; ++col) {
    float v[NR];
    Act<AT>::load(act + size_t(b) * A.sample_stride + (size_t(col) * V + s) * NR, v);
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float wr = w[c].x, wi = CONJW ? -w[c].y : w[c].y;
      re = fmaf(wr, v[2 * c], fmaf(-wi, v[2 * c + 1], re));
      im = fmaf(wr, v[2 * c + 1], fmaf(wi, v[2 * c], im));
    }
    z[(size_t(b) * 3 + col) * vs + s] = make_float2(re, im);
  }
}

__device__ inline double block_sum_d(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// gz = 2 (z - y) / (||y||^2 * B) and per-block partials of sum_b ||z_b - y_b||^2 / ||y_b||^2 / B
__global__ void __launch_bounds__(kThreads)
k_nn_loss(const float2 *__restrict__ z, const float2 *__restrict__ y, const double *__restrict__ ynorm2,
          float2 *__restrict__ gz, unsigned len, int batch, double *__restrict__ partial) {
  __shared__ double red[4];
  const int b = blockIdx.y;
  const double inv = 1.0 / (ynorm2[b] * batch);
  double acc = 0.0;
  for (unsigned j = blockIdx.x * kThreads + threadIdx.x; j < len; j += gridDim.x * kThreads) {
    const size_t k = size_t(b) * len + j;
    const float2 d = make_float2(z[k].x - y[k].x, z[k].y - y[k].y);
    acc += (double(d.x) * d.x + double(d.y) * d.y) * inv;
    gz[k] = make_float2(float(2.0 * d.x * inv), float(2.0 * d.y * inv));
  }
  acc = block_sum_d(acc, red);
  if (threadIdx.x == 0) partial[size_t(b) * gridDim.x + blockIdx.x] = acc;
}

// per-block partials of G[c] = sum (CONJ_ACT ? conj(act_c) v : conj(v) act_c) over the first vs
// sites (V/2: even sites, V: full lattice), colours, samples; partial layout [blk][c][re, im]
template <typename AT, bool CONJ_ACT>
__global__ void __launch_bounds__(kThreads)
k_nn_chan_dot(const AT *__restrict__ act, const float2 *__restrict__ v, unsigned vs, NNArgs A,
              double *__restrict__ partial) {
  __shared__ double red[4];
  const Geometry &g = A.g;
  const unsigned V = 2u * g.vh;
  double acc[2 * NC];
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
  const size_t total = size_t(A.batch) * 3 * vs;
  for (size_t j = size_t(blockIdx.x) * kThreads + threadIdx.x; j < total; j += size_t(gridDim.x) * kThreads) {
    const size_t b = j / (3 * size_t(vs));
    const size_t rem = j - b * 3 * size_t(vs);
    const unsigned col = rem / vs, s = rem % vs;
    float a[NR];
    Act<AT>::load(act + b * A.sample_stride + (size_t(col) * V + s) * NR, a);
    const float2 w = v[j];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double ar = a[2 * c], ai = a[2 * c + 1];
      if (CONJ_ACT) {  // conj(a) w
        acc[2 * c] += ar * w.x + ai * w.y;
        acc[2 * c + 1] += ar * w.y - ai * w.x;
      } else {         // conj(w) a
        acc[2 * c] += w.x * ar + w.y * ai;
        acc[2 * c + 1] += w.x * ai - w.y * ar;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 2 * NC; ++k) {
    const double s = block_sum_d(acc[k], red);
    if (threadIdx.x == 0) partial[size_t(blockIdx.x) * 2 * NC + k] = s;
  }
}

// per-block partials of G_a[h][c] = sum conj((H_h phi_c)(x)) . g_c(x) over sites, colours,
// samples; partial layout [blk][h][c][re, im]
template <typename AT, typename LT>
__global__ void __launch_bounds__(kThreads)
k_nn_stencil_wgrad(NNArgs A, const AT *__restrict__ phi, const AT *__restrict__ gpsi,
                   double *__restrict__ partial) {
  __shared__ double red[4];
  const Geometry &g = A.g;
  const unsigned V = 2u * g.vh;
  const size_t total = size_t(A.batch) * V;
  for (int h = 0; h < 9; ++h) {
    double acc[2 * NC];
#pragma unroll
    for (int k = 0; k < 2 * NC; ++k) acc[k] = 0.0;
    for (size_t j = size_t(blockIdx.x) * kThreads + threadIdx.x; j < total;
         j += size_t(gridDim.x) * kThreads) {
      const size_t b = j / V;
      const unsigned X = j - b * V;
      const AT *ib = phi + b * A.sample_stride;
      const AT *gb = gpsi + b * A.sample_stride;
      float hv[3][NR];
      if (h == 0) {
#pragma unroll
        for (int col = 0; col < 3; ++col) Act<AT>::load(ib + (size_t(col) * V + X) * NR, hv[col]);
      } else {
        const Site q = decode(g, X);
        const int mu = (h - 1) & 3;
        const bool fwd = h < 5;
        const unsigned nb = nbr1(g, q, mu, fwd ? 1 : -1);
        const LT *lk = static_cast<const LT *>(A.links[q.p]);
        const int plane = link_plane(fwd ? mu : 4 + mu, 18);
        float lr[3][3], li[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int jj = 0; jj < 3; ++jj) ld_link(lk + size_t(plane + 3 * i + jj) * g.vh + q.s, lr[i][jj], li[i][jj]);
        float v[3][NR];
#pragma unroll
        for (int col = 0; col < 3; ++col) Act<AT>::load(ib + (size_t(col) * V + nb) * NR, v[col]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            float tr = 0.f, ti = 0.f;
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
              tr = fmaf(lr[i][jj], v[jj][2 * c], tr);
              tr = fmaf(-li[i][jj], v[jj][2 * c + 1], tr);
              ti = fmaf(lr[i][jj], v[jj][2 * c + 1], ti);
              ti = fmaf(li[i][jj], v[jj][2 * c], ti);
            }
            hv[i][2 * c] = tr;
            hv[i][2 * c + 1] = ti;
          }
      }
#pragma unroll
      for (int col = 0; col < 3; ++col) {
        float gv[NR];
        Act<AT>::load(gb + (size_t(col) * V + X) * NR, gv);
#pragma unroll
        for (int c = 0; c < NC; ++c) {  // conj(hv) g
          const double hr = hv[col][2 * c], hi = hv[col][2 * c + 1];
          acc[2 * c] += hr * gv[2 * c] + hi * gv[2 * c + 1];
          acc[2 * c + 1] += hr * gv[2 * c + 1] - hi * gv[2 * c];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 2 * NC; ++k) {
      const double s = block_sum_d(acc[k], red);
      if (threadIdx.x == 0) partial[(size_t(blockIdx.x) * 9 + h) * 2 * NC + k] = s;
    }
  }
}

// per-block partials of Q[p][q] = sum_cols gphi_real[p] psi_real[q] (16 x 16), for the mixing
// weight gradient; partial layout [blk][16][16]
template <typename AT>
__global__ void __launch_bounds__(kThreads)
k_nn_mix_wgrad(const AT *__restrict__ gphi, const AT *__restrict__ psi, size_t ncols,
               double *__restrict__ partial) {
  __shared__ float sg[kThreads][NR + 1];
  __shared__ float sp[kThreads][NR + 1];
  const int pr = threadIdx.x / NR, qr = threadIdx.x % NR;
  double acc = 0.0;
  for (size_t base = size_t(blockIdx.x) * kThreads; base < ncols; base += size_t(gridDim.x) * kThreads) {
    const size_t col = base + threadIdx.x;
    float a[NR], b[NR];
    if (col < ncols) {
      Act<AT>::load(gphi + col * NR, a);
      Act<AT>::load(psi + col * NR, b);
    } else {
#pragma unroll
      for (int k = 0; k < NR; ++k) a[k] = b[k] = 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      sg[threadIdx.x][k] = a[k];
      sp[threadIdx.x][k] = b[k];
    }
    __syncthreads();
    float s = 0.f;
    for (int k = 0; k < kThreads; ++k) s = fmaf(sg[k][pr], sp[k][qr], s);
    acc += s;
  }
  partial[size_t(blockIdx.x) * NR * NR + threadIdx.x] = acc;
}

// sum of partial rows: out[k] = sum_b partial[b * width + k] (added to out[k] if acc)
__global__ void k_nn_sum_partials(const double *__restrict__ partial, int nblk, int width,
                                  double *__restrict__ out, int acc) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) v += partial[size_t(b) * width + k];
  v = block_sum_d(v, red);
  if (threadIdx.x == 0) out[k] = acc ? out[k] + v : v;
}

// per-sample ||v_b||^2 partials: partial[b * gridDim.x + blk]
__global__ void __launch_bounds__(kThreads)
k_nn_norm2(const float2 *__restrict__ v, unsigned len, double *__restrict__ partial) {
  __shared__ double red[4];
  const int b = blockIdx.y;
  double acc = 0.0;
  for (unsigned j = blockIdx.x * kThreads + threadIdx.x; j < len; j += gridDim.x * kThreads) {
    const float2 x = v[size_t(b) * len + j];
    acc += double(x.x) * x.x + double(x.y) * x.y;
  }
  acc = block_sum_d(acc, red);
  if (threadIdx.x == 0) partial[size_t(b) * gridDim.x + blockIdx.x] = acc;
}

// out[row] = sum_b partial[row * nblk + b]
__global__ void k_nn_sum_rows(const double *__restrict__ partial, int nblk, double *__restrict__ out) {
  __shared__ double red[4];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) v += partial[size_t(blockIdx.x) * nblk + b];
  v = block_sum_d(v, red);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// Adam update of the FP32 master weights from the FP64 gradient (reals).
__global__ void k_adam(float *__restrict__ theta, const double *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int nreal, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nreal) return;
  const float gi = float(grad[i]);
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// complex128 -> complex64 copy, and ||y_b||^2 partials
__global__ void k_to_c64(const double2 *__restrict__ a, float2 *__restrict__ o, size_t len) {
  for (size_t j = size_t(blockIdx.x) * kThreads + threadIdx.x; j < len; j += size_t(gridDim.x) * kThreads)
    o[j] = make_float2(float(a[j].x), float(a[j].y));
}
__global__ void k_to_c128(const float2 *__restrict__ a, double2 *__restrict__ o, size_t len) {
  for (size_t j = size_t(blockIdx.x) * kThreads + threadIdx.x; j < len; j += size_t(gridDim.x) * kThreads)
    o[j] = make_double2(a[j].x, a[j].y);
}

}  // namespace

// ============================================================================================
// host side

struct NNState {
  int layers = 0;
  int nparam = 0;                // complex parameters
  std::vector<int> off_w, off_a;  // complex offsets of W_l (l >= 1) and a_l
  int off_out = 0;
  float2 *theta = nullptr;       // FP32 master weights
  float *adam_m = nullptr, *adam_v = nullptr;
  int adam_step = 0;
  double *grad = nullptr;        // FP64 gradient (2 * nparam reals)
  bool bf16 = true;              // activation storage
  int loss_kind = HISQ_NN_LOSS_SOLUTION;
  int form = HISQ_NN_FORM_DIRECT;
  double loss_mass = 0.0;        // mass of M for the residual-norm loss
  // activation buffers (grow-only)
  void *act = nullptr;
  size_t act_bytes = 0;
  void *scratch = nullptr;       // partials, per-sample norms, input/output conversions
  size_t scratch_bytes = 0;
};

void nn_free_state(hisq_ctx *ctx) {
  NNState *s = ctx->nn;
  if (!s) return;
  const size_t nreal = size_t(2) * s->nparam;
  dev_free(ctx, s->theta, nreal * sizeof(float));
  dev_free(ctx, s->adam_m, nreal * sizeof(float));
  dev_free(ctx, s->adam_v, nreal * sizeof(float));
  dev_free(ctx, s->grad, nreal * sizeof(double));
  dev_free(ctx, s->act, s->act_bytes);
  dev_free(ctx, s->scratch, s->scratch_bytes);
  delete s;
  ctx->nn = nullptr;
}

namespace {

int nn_params_count(int layers) { return NC + layers * 9 * NC + (layers - 1) * NC * NC + NC; }

int grow(hisq_ctx *ctx, void **p, size_t *cur, size_t bytes) {
  if (*cur >= bytes) return HISQ_OK;
  if (*p) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx, *p, *cur);
    *p = nullptr;
    *cur = 0;
  }
  bytes = (bytes + 4095) & ~size_t(4095);
  RETCHK(dev_alloc(ctx, p, bytes, "network workspace"));
  *cur = bytes;
  return HISQ_OK;
}

// Link copy the network reads: FP16 with BF16 activations (its rounding, 4.9e-4, is below
// BF16's 3.9e-3, and it halves the link bytes), else FP32, else FP16.
bool nn_links(hisq_ctx *ctx, int *prec) {
  if (ctx->nn && ctx->nn->bf16 && ctx->links[HISQ_F16].base) {
    *prec = HISQ_F16;
    return true;
  }
  if (ctx->links[HISQ_F32].base) {
    *prec = HISQ_F32;
    return true;
  }
  if (ctx->links[HISQ_F16].base) {
    *prec = HISQ_F16;
    return true;
  }
  return false;
}

NNArgs nn_args(hisq_ctx *ctx, int batch, int prec) {
  NNArgs A;
  A.g = ctx->g;
  A.links[0] = ctx->links[prec].par[0];
  A.links[1] = ctx->links[prec].par[1];
  A.batch = batch;
  A.sample_stride = size_t(3) * 2 * ctx->g.vh * NR;
  return A;
}

size_t act_elem(const NNState *s) { return s->bf16 ? 2 : 4; }

int check_nn(hisq_ctx *ctx, const char *fn) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "%s: no network (call hisq_nn_init)", fn);
  int prec;
  if (!ctx->links_loaded || !nn_links(ctx, &prec))
    return set_err(ctx, HISQ_ERR_STATE, "%s: the network needs the FP32 or FP16 link copy", fn);
  return HISQ_OK;
}

// ---- kernel launch helpers ----

template <typename AT>
int launch_stencil(hisq_ctx *ctx, const NNArgs &A, int prec, const void *in, void *out,
                   const float2 *a, bool adj) {
  const unsigned V = 2u * ctx->g.vh;
  dim3 grid((V + kThreads - 1) / kThreads * A.batch);
  const AT *i = static_cast<const AT *>(in);
  AT *o = static_cast<AT *>(out);
  if (prec == HISQ_F32) {
    if (adj) k_nn_stencil<AT, float2, true><<<grid, kThreads, 0, ctx->stream>>>(A, i, o, a);
    else k_nn_stencil<AT, float2, false><<<grid, kThreads, 0, ctx->stream>>>(A, i, o, a);
  } else {
    if (adj) k_nn_stencil<AT, __half2, true><<<grid, kThreads, 0, ctx->stream>>>(A, i, o, a);
    else k_nn_stencil<AT, __half2, false><<<grid, kThreads, 0, ctx->stream>>>(A, i, o, a);
  }
  LAUNCHCHK(ctx, "k_nn_stencil");
  return HISQ_OK;
}

int launch_mix(hisq_ctx *ctx, const NNState *s, const void *in, void *out, size_t ncols,
               const float2 *W, bool conjt) {
  if (s->bf16) {
    const bf16 *i = static_cast<const bf16 *>(in);
    bf16 *o = static_cast<bf16 *>(out);
    size_t groups = ncols / 16;
    int blocks = int(std::min<size_t>((groups + 3) / 4, 8192));
    if (conjt) k_nn_mix_mfma<true><<<blocks, kThreads, 0, ctx->stream>>>(i, o, ncols, W);
    else k_nn_mix_mfma<false><<<blocks, kThreads, 0, ctx->stream>>>(i, o, ncols, W);
  } else {
    const float *i = static_cast<const float *>(in);
    float *o = static_cast<float *>(out);
    int blocks = int((ncols + kThreads - 1) / kThreads);
    if (conjt) k_nn_mix_fma<float, true><<<blocks, kThreads, 0, ctx->stream>>>(i, o, ncols, W);
    else k_nn_mix_fma<float, false><<<blocks, kThreads, 0, ctx->stream>>>(i, o, ncols, W);
  }
  LAUNCHCHK(ctx, "k_nn_mix");
  return HISQ_OK;
}

// Buffers: forward keeps phi_l and psi_l for every layer (2L activations) plus two gradient
// buffers for the backward pass.
struct ActBufs {
  std::vector<void *> phi, psi;
  void *g0 = nullptr, *g1 = nullptr;
};

int act_bufs(hisq_ctx *ctx, int batch, bool train, ActBufs *b) {
  NNState *s = ctx->nn;
  const size_t one = size_t(batch) * 3 * 2 * ctx->g.vh * NR * act_elem(s);
  const int count = train ? 2 * s->layers + 2 : 2;
  RETCHK(grow(ctx, &s->act, &s->act_bytes, one * count));
  char *base = static_cast<char *>(s->act);
  b->phi.resize(s->layers);
  b->psi.resize(s->layers);
  if (train) {
    for (int l = 0; l < s->layers; ++l) {
      b->phi[l] = base + one * (2 * l);
      b->psi[l] = base + one * (2 * l + 1);
    }
    b->g0 = base + one * (2 * s->layers);
    b->g1 = base + one * (2 * s->layers + 1);
  } else {  // ping-pong
    for (int l = 0; l < s->layers; ++l) {
      b->phi[l] = base;
      b->psi[l] = base + one;
    }
  }
  return HISQ_OK;
}

// N r for even-site vectors r32 ([b][3][V/2]); the readout goes to z32 on the even sites
// ([b][3][V/2], the direct form) or on the full lattice ([b][3][V], full_out).
template <typename AT>
int forward_t(hisq_ctx *ctx, int batch, const float2 *r32, float2 *z32, bool full_out, const ActBufs &b) {
  NNState *s = ctx->nn;
  int prec;
  nn_links(ctx, &prec);
  const NNArgs A = nn_args(ctx, batch, prec);
  const unsigned V = 2u * ctx->g.vh;
  const size_t ncols = size_t(batch) * 3 * V;
  dim3 gv((V + kThreads - 1) / kThreads, batch);
  k_nn_embed<AT, false><<<gv, kThreads, 0, ctx->stream>>>(r32, unsigned(ctx->g.vh), static_cast<AT *>(b.phi[0]),
                                                          A, s->theta);
  LAUNCHCHK(ctx, "k_nn_embed");
  for (int l = 0; l < s->layers; ++l) {
    if (l >= 1) RETCHK(launch_mix(ctx, s, b.psi[l - 1], b.phi[l], ncols, s->theta + s->off_w[l], false));
    RETCHK(launch_stencil<AT>(ctx, A, prec, b.phi[l], b.psi[l], s->theta + s->off_a[l], false));
  }
  const unsigned vs = full_out ? V : unsigned(ctx->g.vh);
  dim3 ge((vs + kThreads - 1) / kThreads, batch);
  k_nn_readout<AT, false><<<ge, kThreads, 0, ctx->stream>>>(static_cast<const AT *>(b.psi[s->layers - 1]), z32, vs,
                                                           A, s->theta + s->off_out);
  LAUNCHCHK(ctx, "k_nn_readout");
  return HISQ_OK;
}

int forward(hisq_ctx *ctx, int batch, const float2 *r32, float2 *z32, bool full_out, const ActBufs &b) {
  return ctx->nn->bf16 ? forward_t<bf16>(ctx, batch, r32, z32, full_out, b)
                       : forward_t<float>(ctx, batch, r32, z32, full_out, b);
}

// N^dag u for full-lattice vectors u32 ([b][3][V]) into even-site vectors z32 ([b][3][V/2]): the
// layers in reverse order with conjugated readout, adjoint stencils and W_l^dag mixings, ending
// with the conjugated input weights.  t0 and t1 are two activation buffers.
template <typename AT>
int adjoint_t(hisq_ctx *ctx, int batch, const float2 *u32, float2 *z32, void *t0, void *t1) {
  NNState *s = ctx->nn;
  int prec;
  nn_links(ctx, &prec);
  const NNArgs A = nn_args(ctx, batch, prec);
  const unsigned V = 2u * ctx->g.vh;
  const size_t ncols = size_t(batch) * 3 * V;
  dim3 gv((V + kThreads - 1) / kThreads, batch);
  k_nn_embed<AT, true><<<gv, kThreads, 0, ctx->stream>>>(u32, V, static_cast<AT *>(t0), A, s->theta + s->off_out);
  LAUNCHCHK(ctx, "k_nn_embed");
  for (int l = s->layers - 1; l >= 0; --l) {
    RETCHK(launch_stencil<AT>(ctx, A, prec, t0, t1, s->theta + s->off_a[l], true));
    if (l >= 1) RETCHK(launch_mix(ctx, s, t1, t0, ncols, s->theta + s->off_w[l], true));
  }
  dim3 ge((ctx->g.vh + kThreads - 1) / kThreads, batch);
  k_nn_readout<AT, true><<<ge, kThreads, 0, ctx->stream>>>(static_cast<const AT *>(t1), z32, unsigned(ctx->g.vh),
                                                          A, s->theta);
  LAUNCHCHK(ctx, "k_nn_readout");
  return HISQ_OK;
}

int adjoint(hisq_ctx *ctx, int batch, const float2 *u32, float2 *z32, void *t0, void *t1) {
  return ctx->nn->bf16 ? adjoint_t<bf16>(ctx, batch, u32, z32, t0, t1)
                       : adjoint_t<float>(ctx, batch, u32, z32, t0, t1);
}

// complex G_W[o][i] += (Q[2o][2i] + Q[2o+1][2i+1]) + i (Q[2o+1][2i] - Q[2o][2i+1])
__global__ void k_nn_assemble_w(const double *__restrict__ Q, double *__restrict__ gw) {
  const int t = threadIdx.x;
  if (t >= NC * NC) return;
  const int o = t / NC, i = t % NC;
  gw[2 * t] += Q[(2 * o) * NR + 2 * i] + Q[(2 * o + 1) * NR + 2 * i + 1];
  gw[2 * t + 1] += Q[(2 * o + 1) * NR + 2 * i] - Q[(2 * o) * NR + 2 * i + 1];
}

// Backward pass after forward_t with the train buffers on the input x32: adds to s->grad the
// Wirtinger gradient of Re<gz, N x>, with gz the output gradient on the even sites ([b][3][V/2],
// gvs = V/2; the direct form) or on the full lattice ([b][3][V], gvs = V).
template <typename AT>
int backward_t(hisq_ctx *ctx, int batch, const float2 *x32, const float2 *gz, unsigned gvs, const ActBufs &b,
               double *partial, size_t partial_cap, double *red) {
  NNState *s = ctx->nn;
  int prec;
  nn_links(ctx, &prec);
  const NNArgs A = nn_args(ctx, batch, prec);
  const unsigned V = 2u * ctx->g.vh;
  const size_t ncols = size_t(batch) * 3 * V;
  const int nblk = 1024;
  if (size_t(nblk) * 9 * 2 * NC > partial_cap || size_t(nblk) * NR * NR > partial_cap)
    return set_err(ctx, HISQ_ERR_STATE, "network partial buffer too small");
  // W_out: G[c] = sum conj(psi_L[c]) gz
  k_nn_chan_dot<AT, true><<<nblk, kThreads, 0, ctx->stream>>>(static_cast<const AT *>(b.psi[s->layers - 1]), gz,
                                                             gvs, A, partial);
  LAUNCHCHK(ctx, "k_nn_chan_dot");
  k_nn_sum_partials<<<2 * NC, kThreads, 0, ctx->stream>>>(partial, nblk, 2 * NC, s->grad + 2 * s->off_out, 1);
  LAUNCHCHK(ctx, "k_nn_sum_partials");
  // g_psi_L = conj(W_out) (x) gz
  dim3 gv((V + kThreads - 1) / kThreads, batch);
  void *gpsi = b.g0, *gphi = b.g1;
  k_nn_embed<AT, true><<<gv, kThreads, 0, ctx->stream>>>(gz, gvs, static_cast<AT *>(gpsi), A, s->theta + s->off_out);
  LAUNCHCHK(ctx, "k_nn_embed");
  for (int l = s->layers - 1; l >= 0; --l) {
    // stencil weights
    if (prec == HISQ_F32)
      k_nn_stencil_wgrad<AT, float2><<<nblk, kThreads, 0, ctx->stream>>>(
          A, static_cast<const AT *>(b.phi[l]), static_cast<const AT *>(gpsi), partial);
    else
      k_nn_stencil_wgrad<AT, __half2><<<nblk, kThreads, 0, ctx->stream>>>(
          A, static_cast<const AT *>(b.phi[l]), static_cast<const AT *>(gpsi), partial);
    LAUNCHCHK(ctx, "k_nn_stencil_wgrad");
    k_nn_sum_partials<<<9 * 2 * NC, kThreads, 0, ctx->stream>>>(partial, nblk, 9 * 2 * NC,
                                                               s->grad + 2 * s->off_a[l], 1);
    LAUNCHCHK(ctx, "k_nn_sum_partials");
    // g_phi = S^dag g_psi
    RETCHK(launch_stencil<AT>(ctx, A, prec, gpsi, gphi, s->theta + s->off_a[l], true));
    if (l >= 1) {
      // W_l: Q = sum g_phi_real psi_{l-1}_real^T, assembled into the complex gradient
      k_nn_mix_wgrad<AT><<<nblk, kThreads, 0, ctx->stream>>>(static_cast<const AT *>(gphi),
                                                             static_cast<const AT *>(b.psi[l - 1]), ncols, partial);
      LAUNCHCHK(ctx, "k_nn_mix_wgrad");
      k_nn_sum_partials<<<NR * NR, kThreads, 0, ctx->stream>>>(partial, nblk, NR * NR, red, 0);
      LAUNCHCHK(ctx, "k_nn_sum_partials");
      k_nn_assemble_w<<<1, 64, 0, ctx->stream>>>(red, s->grad + 2 * s->off_w[l]);
      LAUNCHCHK(ctx, "k_nn_assemble_w");
      // g_psi_{l-1} = W_l^dag g_phi
      RETCHK(launch_mix(ctx, s, gphi, gpsi, ncols, s->theta + s->off_w[l], true));
    } else {
      // W_in: G[c] = sum conj(x) g_phi_1[c] over the even sites
      k_nn_chan_dot<AT, false><<<nblk, kThreads, 0, ctx->stream>>>(static_cast<const AT *>(gphi), x32,
                                                                  unsigned(ctx->g.vh), A, partial);
      LAUNCHCHK(ctx, "k_nn_chan_dot");
      k_nn_sum_partials<<<2 * NC, kThreads, 0, ctx->stream>>>(partial, nblk, 2 * NC, s->grad, 1);
      LAUNCHCHK(ctx, "k_nn_sum_partials");
    }
  }
  return HISQ_OK;
}

int backward(hisq_ctx *ctx, int batch, const float2 *x32, const float2 *gz, unsigned gvs, const ActBufs &b,
             double *partial, size_t partial_cap, double *red) {
  return ctx->nn->bf16 ? backward_t<bf16>(ctx, batch, x32, gz, gvs, b, partial, partial_cap, red)
                       : backward_t<float>(ctx, batch, x32, gz, gvs, b, partial, partial_cap, red);
}

struct Scratch {
  float2 *r32, *y32, *z32, *gz, *w32, *t32, *gw;
  float2 *u, *ng;   // full-lattice N r and N G of the Gram form ([b][3][V])
  double *ynorm2, *partial, *red, *loss;
  size_t partial_cap;
};

int scratch(hisq_ctx *ctx, int batch, Scratch *sc) {
  NNState *s = ctx->nn;
  const size_t vec = size_t(batch) * 3 * ctx->g.vh * sizeof(float2);
  const size_t partial_cap = 1024 * NR * NR;  // doubles: >= 1024 * 9 * 2C, 1024 * 256, 256 * batch
  const size_t bytes = 11 * vec + (batch + partial_cap + NR * NR + 64) * sizeof(double) + 4096;
  RETCHK(grow(ctx, &s->scratch, &s->scratch_bytes, bytes));
  char *p = static_cast<char *>(s->scratch);
  float2 *v[7];
  for (int i = 0; i < 7; ++i) v[i] = reinterpret_cast<float2 *>(p + i * vec);
  sc->r32 = v[0];
  sc->y32 = v[1];
  sc->z32 = v[2];
  sc->gz = v[3];
  sc->w32 = v[4];
  sc->t32 = v[5];
  sc->gw = v[6];
  sc->u = reinterpret_cast<float2 *>(p + 7 * vec);
  sc->ng = reinterpret_cast<float2 *>(p + 9 * vec);
  double *d = reinterpret_cast<double *>(p + 11 * vec);
  sc->ynorm2 = d;
  sc->partial = d + batch;
  sc->partial_cap = partial_cap;
  sc->red = sc->partial + partial_cap;
  sc->loss = sc->red + NR * NR;
  return HISQ_OK;
}

// Loss and gradient of one minibatch.  Direct form: z = R_even N r, one forward and one backward
// pass.  Gram form: u = N r, z = N^dag u; with G the loss gradient with respect to z,
// dL = Re<u, dN G> + Re<N G, dN r>, i.e. two backward passes (input G with output gradient u,
// input r with output gradient N G).
int nn_batch_grad(hisq_ctx *ctx, int batch, const void *r, const void *y, bool f64_io, double *loss_dev) {
  NNState *s = ctx->nn;
  Scratch sc;
  RETCHK(scratch(ctx, batch, &sc));
  ActBufs b;
  RETCHK(act_bufs(ctx, batch, true, &b));
  const size_t len = size_t(batch) * 3 * ctx->g.vh;
  const unsigned V = 2u * ctx->g.vh;
  const float2 *r32 = static_cast<const float2 *>(r), *y32 = static_cast<const float2 *>(y);
  if (f64_io) {
    k_to_c64<<<1024, kThreads, 0, ctx->stream>>>(static_cast<const double2 *>(r), sc.r32, len);
    k_to_c64<<<1024, kThreads, 0, ctx->stream>>>(static_cast<const double2 *>(y), sc.y32, len);
    LAUNCHCHK(ctx, "k_to_c64");
    r32 = sc.r32;
    y32 = sc.y32;
  }
  const bool resid = s->loss_kind == HISQ_NN_LOSS_RESIDUAL;
  const bool gram = s->form == HISQ_NN_FORM_GRAM;
  // ||t_b||^2 in FP64 of the FP32 vector the loss compares against (y, or r for the residual loss)
  const float2 *target = resid ? r32 : y32;
  {
    const int nblk = 256;
    k_nn_norm2<<<dim3(nblk, batch), kThreads, 0, ctx->stream>>>(target, unsigned(3 * ctx->g.vh), sc.partial);
    LAUNCHCHK(ctx, "k_nn_norm2");
    k_nn_sum_rows<<<batch, kThreads, 0, ctx->stream>>>(sc.partial, nblk, sc.ynorm2);
    LAUNCHCHK(ctx, "k_nn_sum_rows");
  }
  if (gram) {
    RETCHK(forward(ctx, batch, r32, sc.u, true, b));
    RETCHK(adjoint(ctx, batch, sc.u, sc.z32, b.g0, b.g1));
  } else {
    RETCHK(forward(ctx, batch, r32, sc.z32, false, b));
  }
  const int lblk = 256;
  dim3 gl(lblk, batch);
  if (resid) {  // w = M z; gradient w.r.t. w, then g_z = M g_w (M is Hermitian)
    const int mprec = ctx->links[HISQ_F32].base ? HISQ_F32 : HISQ_F16;
    const double m2 = s->loss_mass * s->loss_mass;
    RETCHK(launch_dslash(ctx, 1, mprec, batch, sc.z32, sc.t32, false, 0.0, nullptr, nullptr, nullptr));
    RETCHK(launch_dslash(ctx, 0, mprec, batch, sc.t32, sc.w32, true, m2, sc.z32, nullptr, nullptr));
    k_nn_loss<<<gl, kThreads, 0, ctx->stream>>>(sc.w32, r32, sc.ynorm2, sc.gw, unsigned(3 * ctx->g.vh), batch, sc.partial);
    LAUNCHCHK(ctx, "k_nn_loss");
    RETCHK(launch_dslash(ctx, 1, mprec, batch, sc.gw, sc.t32, false, 0.0, nullptr, nullptr, nullptr));
    RETCHK(launch_dslash(ctx, 0, mprec, batch, sc.t32, sc.gz, true, m2, sc.gw, nullptr, nullptr));
  } else {
    k_nn_loss<<<gl, kThreads, 0, ctx->stream>>>(sc.z32, y32, sc.ynorm2, sc.gz, unsigned(3 * ctx->g.vh), batch, sc.partial);
    LAUNCHCHK(ctx, "k_nn_loss");
  }
  k_nn_sum_partials<<<1, kThreads, 0, ctx->stream>>>(sc.partial, lblk * batch, 1, loss_dev, 0);
  LAUNCHCHK(ctx, "k_nn_sum_partials");
  HIPCHK(ctx, hipMemsetAsync(s->grad, 0, size_t(2) * s->nparam * sizeof(double), ctx->stream));
  if (gram) {
    RETCHK(forward(ctx, batch, sc.gz, sc.ng, true, b));
    RETCHK(backward(ctx, batch, sc.gz, sc.u, V, b, sc.partial, sc.partial_cap, sc.red));
    RETCHK(forward(ctx, batch, r32, sc.u, true, b));  // caches for input r (u is no longer needed)
    RETCHK(backward(ctx, batch, r32, sc.ng, V, b, sc.partial, sc.partial_cap, sc.red));
  } else {
    RETCHK(backward(ctx, batch, r32, sc.gz, unsigned(ctx->g.vh), b, sc.partial, sc.partial_cap, sc.red));
  }
  return HISQ_OK;
}

// deterministic host-side initial weights: near identity plus small SplitMix64/Box-Muller noise
void init_weights(std::vector<float> &w, const NNState *s, unsigned long long seed, float scale) {
  unsigned long long st = seed;
  auto next = [&]() {
    unsigned long long z = (st += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  };
  auto unif = [&]() { return (double(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  for (size_t i = 0; i < w.size(); i += 2) {
    const double u1 = unif(), u2 = unif();
    const double rad = std::sqrt(-2.0 * std::log(u1)) * std::sqrt(0.5);
    w[i] = float(scale * rad * std::cos(2 * M_PI * u2));
    w[i + 1] = float(scale * rad * std::sin(2 * M_PI * u2));
  }
  w[0] += 1.f;                                 // W_in[0]
  w[2 * s->off_out] += 1.f;                    // W_out[0]
  for (int l = 0; l < s->layers; ++l) {
    w[2 * s->off_a[l]] += 1.f;                 // a_l[0][0]
    if (l >= 1) w[2 * s->off_w[l]] += 1.f;     // W_l[0][0]
  }
}

}  // namespace

// ---- C ABI ----------------------------------------------------------------------------------

extern "C" int hisq_nn_init(hisq_ctx *ctx, int layers, int channels, unsigned long long seed) {
  if (!ctx) return HISQ_ERR_ARG;
  if (channels != NC || layers < 1 || layers > 8)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_init: need channels == %d and 1 <= layers <= 8", NC);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  nn_free_state(ctx);
  NNState *s = new NNState();
  ctx->nn = s;
  s->layers = layers;
  s->nparam = nn_params_count(layers);
  s->off_w.assign(layers, -1);
  s->off_a.assign(layers, -1);
  int k = NC;
  for (int l = 0; l < layers; ++l) {
    if (l >= 1) {
      s->off_w[l] = k;
      k += NC * NC;
    }
    s->off_a[l] = k;
    k += 9 * NC;
  }
  s->off_out = k;
  const size_t nreal = size_t(2) * s->nparam;
  void *p;
  if (dev_alloc(ctx, &p, nreal * sizeof(float), "hisq_nn_init") != HISQ_OK) goto oom;
  s->theta = static_cast<float2 *>(p);
  if (dev_alloc(ctx, &p, nreal * sizeof(float), "hisq_nn_init") != HISQ_OK) goto oom;
  s->adam_m = static_cast<float *>(p);
  if (dev_alloc(ctx, &p, nreal * sizeof(float), "hisq_nn_init") != HISQ_OK) goto oom;
  s->adam_v = static_cast<float *>(p);
  if (dev_alloc(ctx, &p, nreal * sizeof(double), "hisq_nn_init") != HISQ_OK) goto oom;
  s->grad = static_cast<double *>(p);
  {
    std::vector<float> w(nreal);
    init_weights(w, s, seed, 0.05f);
    HIPCHK(ctx, hipMemcpy(s->theta, w.data(), nreal * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(s->adam_m, 0, nreal * sizeof(float)));
    HIPCHK(ctx, hipMemset(s->adam_v, 0, nreal * sizeof(float)));
  }
  return HISQ_OK;
oom:
  nn_free_state(ctx);
  return HISQ_ERR_OOM;
}

extern "C" int hisq_nn_num_params(hisq_ctx *ctx) {
  if (!ctx || !ctx->nn) return ctx ? set_err(ctx, HISQ_ERR_STATE, "no network") : HISQ_ERR_ARG;
  return ctx->nn->nparam;
}

extern "C" int hisq_nn_get_params(hisq_ctx *ctx, double *out, int n_reals) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_get_params: no network");
  if (!out || n_reals != 2 * ctx->nn->nparam)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_get_params: need %d reals", 2 * ctx->nn->nparam);
  std::vector<float> w(n_reals);
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(w.data(), ctx->nn->theta, n_reals * sizeof(float), hipMemcpyDeviceToHost));
  for (int i = 0; i < n_reals; ++i) out[i] = w[i];
  return HISQ_OK;
}

extern "C" int hisq_nn_set_params(hisq_ctx *ctx, const double *in, int n_reals) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_set_params: no network");
  if (!in || n_reals != 2 * ctx->nn->nparam)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_set_params: need %d reals", 2 * ctx->nn->nparam);
  std::vector<float> w(n_reals);
  for (int i = 0; i < n_reals; ++i) {
    if (!std::isfinite(in[i])) return set_err(ctx, HISQ_ERR_NONFINITE, "hisq_nn_set_params: non-finite weight");
    w[i] = float(in[i]);
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(ctx->nn->theta, w.data(), n_reals * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemset(ctx->nn->adam_m, 0, n_reals * sizeof(float)));
  HIPCHK(ctx, hipMemset(ctx->nn->adam_v, 0, n_reals * sizeof(float)));
  ctx->nn->adam_step = 0;
  return HISQ_OK;
}

extern "C" int hisq_nn_set_loss(hisq_ctx *ctx, int kind, double mass) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_set_loss: no network");
  if ((kind != HISQ_NN_LOSS_SOLUTION && kind != HISQ_NN_LOSS_RESIDUAL) || !std::isfinite(mass))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_set_loss: bad loss kind or mass");
  ctx->nn->loss_kind = kind;
  ctx->nn->loss_mass = mass;
  return HISQ_OK;
}

extern "C" int hisq_nn_set_form(hisq_ctx *ctx, int form) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_set_form: no network");
  if (form != HISQ_NN_FORM_DIRECT && form != HISQ_NN_FORM_GRAM)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_set_form: bad form %d", form);
  ctx->nn->form = form;
  return HISQ_OK;
}

extern "C" int hisq_nn_set_precision(hisq_ctx *ctx, int bf16_storage) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_set_precision: no network");
  ctx->nn->bf16 = bf16_storage != 0;
  return HISQ_OK;
}

// ---- fused inference ----
template <typename AT, typename LT>
int launch_layer_t(hisq_ctx *ctx, const FusedArgs &F, bool adj, bool in_vec, bool out_vec, int batch) {
  dim3 grid((F.out_sites + kThreads - 1) / kThreads * batch);
  const int key = (adj ? 4 : 0) | (in_vec ? 2 : 0) | (out_vec ? 1 : 0);
  switch (key) {
    case 0: k_nn_layer<AT, LT, false, false, false><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    case 1: k_nn_layer<AT, LT, false, false, true><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    case 2: k_nn_layer<AT, LT, false, true, false><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    case 3: k_nn_layer<AT, LT, false, true, true><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    case 4: k_nn_layer<AT, LT, true, false, false><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    case 5: k_nn_layer<AT, LT, true, false, true><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    case 6: k_nn_layer<AT, LT, true, true, false><<<grid, kThreads, 0, ctx->stream>>>(F); break;
    default: k_nn_layer<AT, LT, true, true, true><<<grid, kThreads, 0, ctx->stream>>>(F); break;
  }
  LAUNCHCHK(ctx, "k_nn_layer");
  return HISQ_OK;
}

int launch_layer(hisq_ctx *ctx, const FusedArgs &F, bool adj, bool in_vec, bool out_vec, int batch,
                 int prec) {
  if (ctx->nn->bf16)
    return prec == HISQ_F32 ? launch_layer_t<bf16, float2>(ctx, F, adj, in_vec, out_vec, batch)
                            : launch_layer_t<bf16, __half2>(ctx, F, adj, in_vec, out_vec, batch);
  return prec == HISQ_F32 ? launch_layer_t<float, float2>(ctx, F, adj, in_vec, out_vec, batch)
                          : launch_layer_t<float, __half2>(ctx, F, adj, in_vec, out_vec, batch);
}

// N r (forward) for even-site r32 into out32: on the even sites ([b][3][V/2]) or the full lattice
// ([b][3][V], full_out).  One fused layer kernel per layer; t0, t1: two activation buffers.
int forward_infer(hisq_ctx *ctx, int batch, const float2 *r32, float2 *out32, bool full_out, void *t0, void *t1) {
  NNState *s = ctx->nn;
  int prec;
  nn_links(ctx, &prec);
  const unsigned V = 2u * ctx->g.vh;
  void *buf[2] = {t0, t1};
  for (int l = 0; l < s->layers; ++l) {
    FusedArgs F{};
    F.A = nn_args(ctx, batch, prec);
    const bool in_vec = l == 0, out_vec = l == s->layers - 1;
    F.in = in_vec ? static_cast<const void *>(r32) : buf[(l - 1) & 1];
    F.out = out_vec ? static_cast<void *>(out32) : buf[l & 1];
    F.a = s->theta + s->off_a[l];
    F.w = out_vec ? nullptr : s->theta + s->off_w[l + 1];
    F.win = s->theta;
    F.wout = s->theta + s->off_out;
    F.vin_sites = unsigned(ctx->g.vh);
    F.out_sites = out_vec && !full_out ? unsigned(ctx->g.vh) : V;
    RETCHK(launch_layer(ctx, F, false, in_vec, out_vec, batch, prec));
  }
  return HISQ_OK;
}

// N^dag u for full-lattice u32 ([b][3][V]) into even-site z32 ([b][3][V/2]).
int adjoint_infer(hisq_ctx *ctx, int batch, const float2 *u32, float2 *z32, void *t0, void *t1) {
  NNState *s = ctx->nn;
  int prec;
  nn_links(ctx, &prec);
  const unsigned V = 2u * ctx->g.vh;
  void *buf[2] = {t0, t1};
  int k = 0;
  for (int l = s->layers - 1; l >= 0; --l, ++k) {
    FusedArgs F{};
    F.A = nn_args(ctx, batch, prec);
    const bool in_vec = l == s->layers - 1, out_vec = l == 0;
    F.in = in_vec ? static_cast<const void *>(u32) : buf[(k - 1) & 1];
    F.out = out_vec ? static_cast<void *>(z32) : buf[k & 1];
    F.a = s->theta + s->off_a[l];
    F.w = out_vec ? nullptr : s->theta + s->off_w[l];
    F.mix_conjt = 1;
    F.win = s->theta + s->off_out;
    F.in_conj = 1;
    F.wout = s->theta;
    F.out_conj = 1;
    F.vin_sites = V;
    F.out_sites = out_vec ? unsigned(ctx->g.vh) : V;
    RETCHK(launch_layer(ctx, F, true, in_vec, out_vec, batch, prec));
  }
  return HISQ_OK;
}

// z = P r for n vectors in FP32 (direct: R_even N r; Gram: N^dag N r)
int nn_apply_internal(hisq_ctx *ctx, int n, const float2 *r32, float2 *z32) {
  ActBufs b;
  RETCHK(act_bufs(ctx, n, false, &b));
  if (ctx->nn->form != HISQ_NN_FORM_GRAM) return forward_infer(ctx, n, r32, z32, false, b.phi[0], b.psi[0]);
  Scratch sc;
  RETCHK(scratch(ctx, n, &sc));
  RETCHK(forward_infer(ctx, n, r32, sc.u, true, b.phi[0], b.psi[0]));
  return adjoint_infer(ctx, n, sc.u, z32, b.phi[0], b.psi[0]);
}

extern "C" int hisq_nn_apply(hisq_ctx *ctx, int n, int prec_io, const void *r, void *z) {
  RETCHK(check_nn(ctx, "hisq_nn_apply"));
  if (!r || !z || n < 1 || n > HISQ_MAX_RHS || (prec_io != HISQ_F64 && prec_io != HISQ_F32))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_apply: bad argument");
  if (!elem_aligned(r, cplx_bytes(prec_io)) || !elem_aligned(z, cplx_bytes(prec_io)))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_apply: r and z must be aligned to %zu bytes", cplx_bytes(prec_io));
  if (prec_io == HISQ_F32) return nn_apply_internal(ctx, n, static_cast<const float2 *>(r), static_cast<float2 *>(z));
  Scratch sc;
  RETCHK(scratch(ctx, n, &sc));
  const size_t len = size_t(n) * 3 * ctx->g.vh;
  k_to_c64<<<1024, kThreads, 0, ctx->stream>>>(static_cast<const double2 *>(r), sc.r32, len);
  LAUNCHCHK(ctx, "k_to_c64");
  RETCHK(nn_apply_internal(ctx, n, sc.r32, sc.z32));
  k_to_c128<<<1024, kThreads, 0, ctx->stream>>>(sc.z32, static_cast<double2 *>(z), len);
  LAUNCHCHK(ctx, "k_to_c128");
  return HISQ_OK;
}

extern "C" int hisq_nn_loss_grad(hisq_ctx *ctx, int n, const void *r, const void *y, double *loss,
                                 double *grad) {
  RETCHK(check_nn(ctx, "hisq_nn_loss_grad"));
  if (!r || !y || n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_loss_grad: bad argument");
  if (!elem_aligned(r, 16) || !elem_aligned(y, 16))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_loss_grad: r and y must be aligned to 16 bytes");
  Scratch sc;
  RETCHK(scratch(ctx, n, &sc));
  RETCHK(nn_batch_grad(ctx, n, r, y, true, sc.loss));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (loss) HIPCHK(ctx, hipMemcpy(loss, sc.loss, sizeof(double), hipMemcpyDeviceToHost));
  if (grad)
    HIPCHK(ctx, hipMemcpy(grad, ctx->nn->grad, size_t(2) * ctx->nn->nparam * sizeof(double), hipMemcpyDeviceToHost));
  return HISQ_OK;
}

extern "C" int hisq_nn_train(hisq_ctx *ctx, int n_pairs, const void *r, const void *y, int epochs,
                             int batch, double lr, unsigned long long seed, double *loss_history) {
  RETCHK(check_nn(ctx, "hisq_nn_train"));
  if (!r || !y || n_pairs < 1 || epochs < 1 || batch < 1 || batch > HISQ_MAX_RHS || !(lr > 0))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_train: bad argument");
  if (!elem_aligned(r, 16) || !elem_aligned(y, 16))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_train: r and y must be aligned to 16 bytes");
  NNState *s = ctx->nn;
  const size_t vlen = size_t(3) * ctx->g.vh;
  const int nbatches = n_pairs / batch;
  if (nbatches < 1) return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_train: fewer pairs than one batch");
  Scratch sc;
  RETCHK(scratch(ctx, batch, &sc));
  double *loss_acc = sc.loss + 1;  // per-batch losses summed on the host
  std::vector<int> order(nbatches);
  for (int i = 0; i < nbatches; ++i) order[i] = i;
  unsigned long long st = seed ? seed : 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int nreal = 2 * s->nparam;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int i = nbatches - 1; i > 0; --i) {  // Fisher-Yates with a SplitMix64 stream
      unsigned long long z = (st += 0x9e3779b97f4a7c15ULL);
      z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
      z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
      z ^= z >> 31;
      std::swap(order[i], order[z % (i + 1)]);
    }
    double ep_loss = 0.0;
    for (int bi = 0; bi < nbatches; ++bi) {
      const size_t off = size_t(order[bi]) * batch * vlen;
      RETCHK(nn_batch_grad(ctx, batch, static_cast<const double2 *>(r) + off,
                           static_cast<const double2 *>(y) + off, true, loss_acc));
      s->adam_step += 1;
      const float c1 = 1.f - std::pow(b1, float(s->adam_step));
      const float c2 = 1.f - std::pow(b2, float(s->adam_step));
      k_adam<<<(nreal + 255) / 256, 256, 0, ctx->stream>>>(reinterpret_cast<float *>(s->theta), s->grad,
                                                           s->adam_m, s->adam_v, nreal, float(lr), b1, b2,
                                                           eps, c1, c2);
      LAUNCHCHK(ctx, "k_adam");
      double lb = 0.0;
      HIPCHK(ctx, hipMemcpyAsync(&lb, loss_acc, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      if (!std::isfinite(lb)) return set_err(ctx, HISQ_ERR_NONFINITE, "hisq_nn_train: non-finite loss");
      ep_loss += lb;
    }
    if (loss_history) loss_history[ep] = ep_loss / nbatches;
  }
  return HISQ_OK;
}

extern "C" int hisq_nn_save(hisq_ctx *ctx, const char *path) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!ctx->nn) return set_err(ctx, HISQ_ERR_STATE, "hisq_nn_save: no network");
  if (!path) return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_save: null path");
  const int nreal = 2 * ctx->nn->nparam;
  std::vector<double> w(nreal);
  RETCHK(hisq_nn_get_params(ctx, w.data(), nreal));
  FILE *f = fopen(path, "wb");
  if (!f) return set_err(ctx, HISQ_ERR_IO, "hisq_nn_save: cannot open %s", path);
  const int hdr[5] = {0x51534948 /* "HISQ" */, 2, ctx->nn->layers, NC, ctx->nn->form};
  bool ok = fwrite(hdr, sizeof hdr, 1, f) == 1 && fwrite(w.data(), sizeof(double), nreal, f) == size_t(nreal);
  ok = (fclose(f) == 0) && ok;
  return ok ? HISQ_OK : set_err(ctx, HISQ_ERR_IO, "hisq_nn_save: write failed");
}

extern "C" int hisq_nn_load(hisq_ctx *ctx, const char *path) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!path) return set_err(ctx, HISQ_ERR_ARG, "hisq_nn_load: null path");
  FILE *f = fopen(path, "rb");
  if (!f) return set_err(ctx, HISQ_ERR_IO, "hisq_nn_load: cannot open %s", path);
  int hdr[5] = {0, 0, 0, 0, HISQ_NN_FORM_DIRECT};  // version 1 files have no form field
  bool hdr_ok = fread(hdr, sizeof(int), 4, f) == 4 && hdr[0] == 0x51534948 && (hdr[1] == 1 || hdr[1] == 2) &&
                hdr[3] == NC && hdr[2] >= 1 && hdr[2] <= 8;
  if (hdr_ok && hdr[1] == 2)
    hdr_ok = fread(hdr + 4, sizeof(int), 1, f) == 1 && (hdr[4] == HISQ_NN_FORM_DIRECT || hdr[4] == HISQ_NN_FORM_GRAM);
  if (!hdr_ok) {
    fclose(f);
    return set_err(ctx, HISQ_ERR_IO, "hisq_nn_load: %s is not a network file", path);
  }
  const int nreal = 2 * nn_params_count(hdr[2]);
  std::vector<double> w(nreal);
  const bool ok = fread(w.data(), sizeof(double), nreal, f) == size_t(nreal);
  fclose(f);
  if (!ok) return set_err(ctx, HISQ_ERR_IO, "hisq_nn_load: %s is truncated", path);
  if (!ctx->nn || ctx->nn->layers != hdr[2]) RETCHK(hisq_nn_init(ctx, hdr[2], NC, 1));
  ctx->nn->form = hdr[4];
  return hisq_nn_set_params(ctx, w.data(), nreal);
}

// Flexible CG preconditioned by the network (Notay 2000, truncation 1), per rhs, with complex
// step sizes (the network is not Hermitian): q = M p; alpha = <p, r>/<p, q>; xh += alpha p;
// r -= alpha q; z = P r; beta = -<q, z>/<p, q>; p = z + beta p.  FP32 body (FP32 or FP16 link
// storage), FP64 solution and reductions, FP64 reliable updates as in the mixed solver.  A rhs
// whose step breaks down (<p, Mp> <= 0, non-finite) or stagnates falls back to the mixed-precision
// CG started from its current x.
int fcg_nn_solve(hisq_ctx *ctx, double mass, int n, const void *b, void *x,
                 const hisq_cg_params *prm, hisq_cg_stats *st, CGState *S, CGState *hS,
                 double *partial) {
  RETCHK(check_nn(ctx, "hisq_cg_mrhs(HISQ_FCG_NN)"));
  const Geometry &g = ctx->g;
  const int op_prec = prm->link_prec;
  const size_t vb = size_t(n) * 3 * g.vh * sizeof(float2);
  const double tol2 = prm->tol * prm->tol;
  const int check_every = prm->check_every > 0 ? prm->check_every : 8;
  const int reliable_every = prm->reliable_every > 0 ? prm->reliable_every : 50;
  void *r, *p, *q, *t, *xh, *z, *mx64, *t64, *p2;
  RETCHK(ws_get(ctx, WS_CG0, vb, &r));
  RETCHK(ws_get(ctx, WS_CG1, vb, &p));
  RETCHK(ws_get(ctx, WS_CG2, vb, &q));
  RETCHK(ws_get(ctx, WS_CG3, vb, &t));
  RETCHK(ws_get(ctx, WS_CG4, vb, &xh));
  RETCHK(ws_get(ctx, WS_CG5, size_t(n) * 3 * g.vh * 16, &mx64));
  RETCHK(ws_get(ctx, WS_CG6, size_t(n) * 3 * g.vh * 16, &t64));
  RETCHK(ws_get(ctx, WS_CG7, vb, &z));
  RETCHK(ws_get(ctx, WS_NN0, size_t(2 * n) * blas_nblk(ctx) * sizeof(double), &p2));
  double *partial2 = static_cast<double *>(p2);

  // initial residual, as in the mixed solver
  RETCHK(cg_init_state(ctx, b, S, n, partial));
  RETCHK(cg_select(ctx, S, n, 1));
  RETCHK(cg_zero(ctx, HISQ_F64, x, S->sel, 1, n));
  if (prm->use_x0) {
    RETCHK(apply_m64(ctx, mass, n, x, t64, mx64, S->sel));
  } else {
    RETCHK(cg_zero(ctx, HISQ_F64, x, nullptr, 0, n));
    RETCHK(cg_zero(ctx, HISQ_F64, mx64, nullptr, 0, n));
  }
  RETCHK(cg_replace_r(ctx, HISQ_F32, b, mx64, r, nullptr, S, S->sel, n, partial));
  RETCHK(cg_set_rho(ctx, partial, S, n, tol2));
  RETCHK(cg_zero(ctx, HISQ_F32, xh, nullptr, 0, n));
  RETCHK(cg_poll(ctx, S, hS));
  for (int i = 0; i < n; ++i)
    if (hS->status[i] == CG_NONFINITE)
      return set_err(ctx, HISQ_ERR_NONFINITE, "hisq_cg_mrhs: non-finite source %d", i);
  RETCHK(nn_apply_internal(ctx, n, static_cast<const float2 *>(r), static_cast<float2 *>(z)));
  HIPCHK(ctx, hipMemcpyAsync(p, z, vb, hipMemcpyDeviceToDevice, ctx->stream));

  auto reliable = [&](int all) -> int {
    RETCHK(cg_select(ctx, S, n, all));
    RETCHK(cg_accum_x(ctx, x, xh, S->sel, n));
    RETCHK(apply_m64(ctx, mass, n, x, t64, mx64, S->sel));
    RETCHK(cg_replace_r(ctx, HISQ_F32, b, mx64, r, nullptr, S, S->sel, n, partial));
    RETCHK(cg_reduce_true(ctx, partial, S, n, tol2, 0));
    return HISQ_OK;
  };

  double best[HISQ_MAX_RHS];
  int stale[HISQ_MAX_RHS], last_rep[HISQ_MAX_RHS], fell[HISQ_MAX_RHS];
  for (int i = 0; i < n; ++i) {
    best[i] = hS->rr_true[i];
    stale[i] = last_rep[i] = fell[i] = 0;
  }
  int it = 0, reps = 0, nactive = 0;
  for (int i = 0; i < n; ++i) nactive += hS->active[i];
  while (nactive > 0 && it < prm->max_iter) {
    int nblk_d = 0, nb2 = 0;
    RETCHK(cg_apply_op(ctx, op_prec, mass, n, p, t, q, partial, &nblk_d, S->active));
    RETCHK(launch_dot_partials(ctx, HISQ_F32, n, p, r, partial2, &nb2));
    RETCHK(fcg_alpha(ctx, partial, nblk_d, partial2, nb2, S, n));
    RETCHK(fcg_update_xr(ctx, xh, r, p, q, S, n, partial));
    RETCHK(cg_reduce_beta(ctx, partial, blas_nblk(ctx), S, n, tol2));
    RETCHK(nn_apply_internal(ctx, n, static_cast<const float2 *>(r), static_cast<float2 *>(z)));
    RETCHK(launch_dot_partials(ctx, HISQ_F32, n, q, z, partial2, &nb2));
    RETCHK(fcg_beta(ctx, partial2, nb2, S, n));
    RETCHK(fcg_update_p(ctx, z, p, S, n));
    ++it;
    if (it % reliable_every == 0) {
      RETCHK(reliable(1));
      ++reps;
    }
    if (it % check_every == 0 || it == prm->max_iter) {
      RETCHK(cg_poll(ctx, S, hS));
      bool any_hit = false;
      for (int i = 0; i < n; ++i) any_hit = any_hit || (hS->active[i] && hS->hit[i]);
      if (any_hit) {
        RETCHK(reliable(0));
        ++reps;
        RETCHK(cg_poll(ctx, S, hS));
      }
      nactive = 0;
      for (int i = 0; i < n; ++i) {
        if (hS->active[i] && hS->replacements[i] != last_rep[i]) {
          last_rep[i] = hS->replacements[i];
          if (hS->rr_true[i] < kStallDrop * best[i]) {
            best[i] = hS->rr_true[i];
            stale[i] = 0;
          } else if (++stale[i] >= kStallUpdates) {
            fell[i] = 1;  // stagnation: hand this rhs to the mixed solver
          }
        }
        if (hS->status[i] == CG_BREAKDOWN) fell[i] = 1;
        nactive += hS->active[i] && !fell[i];
      }
    }
  }
  RETCHK(cg_accum_x(ctx, x, xh, S->fin, n));
  bool ok = false;
  RETCHK(cg_finish(ctx, mass, n, b, x, prm->tol, S, hS, partial, st, &ok));
  int fcg_iters[HISQ_MAX_RHS];
  for (int i = 0; i < n; ++i) fcg_iters[i] = hS->iters[i];
  const long long fcg_site_rhs = st ? st->dslash_site_rhs : 0;
  bool need = false;
  for (int i = 0; i < n; ++i) {
    const double res = hS->bnorm2[i] > 0 ? std::sqrt(hS->rr_true[i] / hS->bnorm2[i]) : 0.0;
    if (!(res <= prm->tol)) {
      fell[i] = 1;
      need = true;
    } else {
      fell[i] = 0;
    }
  }
  int total = it;
  if (need) {  // fallback: mixed-precision CG from the current x (converged rhs stop at once)
    hisq_cg_params mp = *prm;
    mp.kind = HISQ_CG_MIXED;
    mp.use_x0 = 1;
    mp.max_iter = std::max(1, prm->max_iter - it);
    int rc = cg_solve(ctx, mass, n, b, x, &mp, st, S, hS, partial, nullptr, 0, 0, nullptr);
    if (rc != HISQ_OK && rc != HISQ_ERR_NOCONV) return rc;
    ok = rc == HISQ_OK;
    if (st) total += st->total_iters;
  }
  if (st) {
    if (st->iters)
      for (int i = 0; i < n; ++i) st->iters[i] = fcg_iters[i] + (need ? st->iters[i] : 0);
    if (st->fell_back)
      for (int i = 0; i < n; ++i) st->fell_back[i] = fell[i];
    st->total_iters = total;
    st->reliable_updates = reps + (need ? st->reliable_updates : 0);
    if (need) st->dslash_site_rhs += fcg_site_rhs;
  }
  if (!ok) return set_err(ctx, HISQ_ERR_NOCONV, "hisq_cg_mrhs: some rhs missed tol %.3g", prm->tol);
  return HISQ_OK;
}
