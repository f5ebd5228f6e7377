// Internal declarations shared by the HIP sources of libhisq (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdarg>
#include <cstddef>
#include <string>
#include <vector>

#include "hisq.h"

// Lattice geometry in the single-parity ("checkerboard") index used on the device:
// cb = lex >> 1 with lex = x + Lx*(y + Ly*(z + Lz*t)), so cb = (x>>1) + lxh*(y + ly*(z + lz*t)).
struct Geometry {
  int lx, ly, lz, lt;
  int lxh;      // lx / 2
  int vh;       // sites of one parity
  int sy;       // cb stride of y  = lxh
  int sz;       // cb stride of z  = lxh * ly
  int st;       // cb stride of t  = lxh * ly * lz
};

// Planes of one output parity's link array.  The 16 hops of an output site x are, for
// mu = 0..3: k = mu       fat forward   X(x, mu)
//            k = 4 + mu   fat backward  X(x - mu, mu)^dag      (stored already daggered)
//            k = 8 + mu   Naik forward  N(x, mu)
//            k = 12 + mu  Naik backward N(x - 3mu, mu)^dag     (stored already daggered)
// Each hop is stored as planes of V/2 complex numbers (one plane per stored complex entry).  Fat
// links: 9 planes.  Naik links by storage format (recon):
//   18: the 9 entries;
//   14: rows 0 and 1, then the complex scale z (row 2 = z conj(row0 x row1));
//   13: rows 0 and 1; the real scale z of hops 8 + 2j and 9 + 2j shares one plane (re, im);
//    9: N = c U, U in SU(3): u01, u02, u10 and the plane (arg u00, arg u20); the real c of hops
//       8 + 2j and 9 + 2j shares one plane.
__host__ __device__ constexpr int naik_planes(int recon) {
  return recon == 18 ? 9 : (recon == 14 ? 7 : (recon == 13 ? 6 : 4));
}
__host__ __device__ constexpr int link_plane(int k, int recon) {
  return k < 8 ? 9 * k : 72 + (k - 8) * naik_planes(recon);
}
// plane of the real scale of Naik hop k (formats 13 and 9; the re part for even k, im for odd)
__host__ __device__ constexpr int naik_scale_plane(int k, int recon) {
  return 72 + 8 * naik_planes(recon) + (k - 8) / 2;
}
__host__ __device__ constexpr int link_planes_total(int recon) {
  return 72 + 8 * naik_planes(recon) + ((recon == 13 || recon == 9) ? 4 : 0);
}
__host__ __device__ constexpr bool naik_recon_valid(int recon) {
  return recon == 18 || recon == 14 || recon == 13 || recon == 9;
}

struct LinkCopy {
  void *base = nullptr;              // one allocation holding both parities
  void *par[2] = {nullptr, nullptr}; // per output parity
  size_t bytes = 0;
  int recon = 18;
};

enum WsSlot {
  WS_PARTIAL = 0,   // per-block FP64 partial sums
  WS_SCAL,          // per-rhs FP64 scalars of the solvers
  WS_TMP_ODD,       // odd-parity temporary of the M operator
  WS_DOTS,          // per-rhs dot results
  WS_LINKSTAGE,     // host links staged on the device during hisq_load_links
  WS_ERRPART,       // per-block reconstruction errors of hisq_load_links
  WS_CG0, WS_CG1, WS_CG2, WS_CG3, WS_CG4, WS_CG5, WS_CG6, WS_CG7,
  WS_NN0, WS_NN1, WS_NN2, WS_NN3, WS_NN4, WS_NN5, WS_NN6, WS_NN7,
  WS_TUNE0, WS_TUNE1, WS_TUNE2,  // launch-configuration tuning scratch (freed after tuning)
  WS_TR0, WS_TR1, WS_TR2,        // trace estimator: noise bundle, solutions, dot results
  WS_CMPX, WS_CMPB,              // slot-ordered solution and source of a compacted CG bundle
  WS_COUNT
};

// Launch configuration of the Dslash for one (precision, n, plain/fused-M) key.
struct TuneEntry {
  enum State { NONE = 0, HEURISTIC, TUNED, FORCED };
  hisq_launch cfg{};
  State state = NONE;
  float ms = 0.f;
};

struct NNState;

struct hisq_ctx {
  Geometry g{};
  int device = 0;
  size_t lds_max = 65536;            // dynamic LDS bytes a workgroup may use on this device
  hipStream_t stream = nullptr;
  std::string err;
  bool links_loaded = false;
  int naik_recon = 18;
  LinkCopy links[3];                 // indexed by HISQ_F64 / HISQ_F32 / HISQ_F16
  void *ws[WS_COUNT] = {};
  size_t ws_bytes[WS_COUNT] = {};
  TuneEntry tune[3][HISQ_MAX_RHS + 1][2];
  void *pinned = nullptr;            // pinned host mirror of per-rhs residuals
  size_t pinned_bytes = 0;
  NNState *nn = nullptr;
  void *scratch_dev = nullptr;       // device address of the library's static scratch array
  size_t dev_bytes = 0;              // device memory the context holds now (dev_alloc / dev_free)
  size_t dev_peak = 0;               // largest dev_bytes since the last reset (a solve resets it)
};

int set_err(hisq_ctx *ctx, int code, const char *fmt, ...);

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return set_err((ctx), HISQ_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
  } while (0)

#define LAUNCHCHK(ctx, what)                                                                  \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess)                                                                     \
      return set_err((ctx), HISQ_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

#define RETCHK(expr)                                                                          \
  do {                                                                                        \
    int rc_ = (expr);                                                                         \
    if (rc_ != HISQ_OK) return rc_;                                                           \
  } while (0)

// Every device allocation of the context goes through these two, which keep dev_bytes and its
// running peak dev_peak (links, workspace slots, tuning scratch, network state).
int dev_alloc(hisq_ctx *ctx, void **p, size_t bytes, const char *what);
void dev_free(hisq_ctx *ctx, void *p, size_t bytes);

// Look up (once per device, device current) the static scratch array of the allocation-free
// entry point and store its device address in ctx->scratch_dev.
int scratch_lookup(hisq_ctx *ctx);

// Grow-only device workspace slot.
int ws_get(hisq_ctx *ctx, int slot, size_t bytes, void **out);
// Release a workspace slot (tuning scratch, link staging).
void ws_release(hisq_ctx *ctx, int slot);
int pinned_get(hisq_ctx *ctx, size_t bytes, void **out);

// ---- kernels' host launchers (each enqueues on ctx->stream and checks the launch) ----

// Fill one parity's link array of the given precision from device FP64 [V][4][3][3] links.
int launch_pack_links(hisq_ctx *ctx, const double *fat, const double *naik, int prec, int recon,
                      int parity, void *dst, double *max_recon_err_host);

// out = D_{out_parity,1-out_parity} in  (epi = false), or for out_parity = 0 with epi = true:
// out = mass2 * pvec - D_eo in and, if partial != nullptr, per-64-site partials of
// Re<pvec, out> written to partial[r * nblk + b], nblk (= dslash_partials) in *nblk_out.
// active: per-rhs mask (rhs with active[r] == 0 are neither read nor written), or null.
int launch_dslash(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in, void *out,
                  bool epi, double mass2, const void *pvec, double *partial, int *nblk_out,
                  const int *active = nullptr);

// Number of per-rhs partials the fused-M Dslash writes (one per 64-site wave).
int dslash_partials(const Geometry &g);

// Sum partial[r * nblk + b] over b for r < n in a fixed order into res[r] (device).
int launch_reduce_partials(hisq_ctx *ctx, const double *partial, int n, int nblk, int width,
                           double *res);

// Per-block partial sums of <a_r, b_r> (re and im, FP64) for r < n: partial[(2r+c)*nblk + b].
int launch_dot_partials(hisq_ctx *ctx, int prec, int n, const void *a, const void *b,
                        double *partial, int *nblk_out);

bool prec_valid(int prec);
size_t cplx_bytes(int prec);
// vector arguments are arrays of complex elements: their addresses must be multiples of the
// element size (8 bytes complex64, 16 bytes complex128); nullptr counts as aligned
inline bool elem_aligned(const void *p, size_t elem) { return reinterpret_cast<size_t>(p) % elem == 0; }
