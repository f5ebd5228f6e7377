// Stochastic trace of M^-1 on the even sites (Section 1, Eq. 2: the observables are traces
// estimated with many random vectors, which is what the multi-rhs solver is for):
//   Tr M^-1 ~ (1/N) sum_k eta_k^dag M^-1 eta_k,
// Z2 noise eta_k (each colour component of each even site +1 or -1, real), solved in bundles by
// the multi-rhs CG.  The noise is counter based: component c = (k*3 + colour)*V/2 + site of the
// stream takes the sign of the top bit of the c-th SplitMix64 output for the seed (Steele, Lea
// and Flood 2014: output c is mix(seed + (c+1)*0x9E3779B97F4A7C15)), so any vector of the
// stream can be drawn on its own, in any bundle.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace {

constexpr int kThreads = 256;

__device__ inline unsigned long long splitmix64_at(unsigned long long seed, unsigned long long c) {
  unsigned long long z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// eta[j] for the components j of vectors k0 .. k0+n-1 ([n][3][V/2] complex128, j < len)
__global__ void __launch_bounds__(kThreads)
k_z2_noise(double2 *__restrict__ eta, size_t len, unsigned long long seed, unsigned long long c0) {
  for (size_t j = size_t(blockIdx.x) * kThreads + threadIdx.x; j < len; j += size_t(gridDim.x) * kThreads) {
    const unsigned long long top = splitmix64_at(seed, c0 + j) >> 63;
    eta[j] = make_double2(top ? -1.0 : 1.0, 0.0);
  }
}

int launch_noise(hisq_ctx *ctx, unsigned long long seed, long long k0, int n, void *out) {
  const size_t comp = size_t(3) * ctx->g.vh;
  const size_t len = size_t(n) * comp;
  const int blocks = int(std::min<size_t>((len + kThreads - 1) / kThreads, 4096));
  k_z2_noise<<<blocks, kThreads, 0, ctx->stream>>>(static_cast<double2 *>(out), len, seed,
                                                   (unsigned long long)k0 * comp);
  LAUNCHCHK(ctx, "k_z2_noise");
  return HISQ_OK;
}

}  // namespace

extern "C" int hisq_z2_noise(hisq_ctx *ctx, unsigned long long seed, long long k0, int n, void *out) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!out || n < 1 || n > HISQ_MAX_RHS || k0 < 0)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_z2_noise: need out, 1 <= n <= %d, k0 >= 0", HISQ_MAX_RHS);
  if (!elem_aligned(out, 16)) return set_err(ctx, HISQ_ERR_ARG, "hisq_z2_noise: out must be aligned to 16 bytes");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  return launch_noise(ctx, seed, k0, n, out);
}

extern "C" int hisq_trace_minv(hisq_ctx *ctx, double mass, int n_vec, int bundle, unsigned long long seed,
                               const hisq_cg_params *p, double *samples, double *estimate, double *std_error) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!p || !estimate || n_vec < 1 || bundle < 1 || bundle > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_trace_minv: need params, estimate, n_vec >= 1, 1 <= bundle <= %d",
                   HISQ_MAX_RHS);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const size_t vbytes = size_t(bundle) * 3 * ctx->g.vh * sizeof(double2);
  void *eta, *x, *dots;
  RETCHK(ws_get(ctx, WS_TR0, vbytes, &eta));
  RETCHK(ws_get(ctx, WS_TR1, vbytes, &x));
  RETCHK(ws_get(ctx, WS_TR2, size_t(2) * bundle * sizeof(double), &dots));
  std::vector<double> s(n_vec), d(2 * bundle);
  int rc_all = HISQ_OK;
  for (int k0 = 0; k0 < n_vec; k0 += bundle) {
    const int nb = std::min(bundle, n_vec - k0);
    RETCHK(launch_noise(ctx, seed, k0, nb, eta));
    hisq_cg_params q = *p;
    q.use_x0 = 0;
    const int rc = hisq_cg_mrhs(ctx, mass, nb, eta, x, &q, nullptr);
    if (rc != HISQ_OK && rc != HISQ_ERR_NOCONV) return rc;
    if (rc == HISQ_ERR_NOCONV) rc_all = rc;
    RETCHK(hisq_dot_mrhs(ctx, HISQ_F64, nb, eta, x, static_cast<double *>(dots)));
    HIPCHK(ctx, hipMemcpyAsync(d.data(), dots, size_t(2) * nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < nb; ++i) s[k0 + i] = d[2 * i];  // M is Hermitian: the imaginary part is rounding
  }
  double mean = 0.0;
  for (double v : s) mean += v;
  mean /= n_vec;
  double var = 0.0;
  for (double v : s) var += (v - mean) * (v - mean);
  var = n_vec > 1 ? var / (n_vec - 1) : 0.0;
  *estimate = mean;
  if (std_error) *std_error = std::sqrt(var / n_vec);
  if (samples)
    for (int i = 0; i < n_vec; ++i) samples[i] = s[i];
  if (rc_all != HISQ_OK) return set_err(ctx, rc_all, "hisq_trace_minv: some solves missed tol %.3g", p->tol);
  return HISQ_OK;
}

extern "C" int hisq_chiral_condensate(hisq_ctx *ctx, double mass, int n_vec, int bundle, unsigned long long seed,
                                      const hisq_cg_params *p, double *estimate, double *std_error) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!estimate) return set_err(ctx, HISQ_ERR_ARG, "hisq_chiral_condensate: estimate is required");
  double t = 0.0, e = 0.0;
  const int rc = hisq_trace_minv(ctx, mass, n_vec, bundle, seed, p, nullptr, &t, &e);
  if (rc != HISQ_OK && rc != HISQ_ERR_NOCONV) return rc;
  // (1/V) Tr (m + D)^-1 = (2 m / V) Tr M_ee^-1 (V = 2 * V/2 sites)
  const double scale = 2.0 * mass / (2.0 * double(ctx->g.vh));
  *estimate = scale * t;
  if (std_error) *std_error = std::fabs(scale) * e;
  return rc;
}

