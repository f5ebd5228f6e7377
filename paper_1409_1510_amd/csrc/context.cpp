// Context lifecycle, errors, workspace and link loading of libhisq.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.hpp"

static thread_local std::string g_create_err;

int set_err(hisq_ctx *ctx, int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_create_err = buf;
  return code;
}

bool prec_valid(int prec) { return prec == HISQ_F64 || prec == HISQ_F32 || prec == HISQ_F16; }
size_t cplx_bytes(int prec) { return prec == HISQ_F64 ? 16 : 8; }

int dev_alloc(hisq_ctx *ctx, void **p, size_t bytes, const char *what) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_err(ctx, HISQ_ERR_OOM, "%s: device allocation of %zu bytes failed: %s", what, bytes,
                   hipGetErrorString(e));
  }
  ctx->dev_bytes += bytes;
  if (ctx->dev_bytes > ctx->dev_peak) ctx->dev_peak = ctx->dev_bytes;
  return HISQ_OK;
}

void dev_free(hisq_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->dev_bytes -= std::min(bytes, ctx->dev_bytes);
}

int ws_get(hisq_ctx *ctx, int slot, size_t bytes, void **out) {
  if (bytes == 0) bytes = 256;
  if (ctx->ws_bytes[slot] < bytes) {
    if (ctx->ws[slot]) {
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      ws_release(ctx, slot);
    }
    size_t want = (bytes + 4095) & ~size_t(4095);
    RETCHK(dev_alloc(ctx, &ctx->ws[slot], want, "workspace"));
    ctx->ws_bytes[slot] = want;
  }
  *out = ctx->ws[slot];
  return HISQ_OK;
}

void ws_release(hisq_ctx *ctx, int slot) {
  dev_free(ctx, ctx->ws[slot], ctx->ws_bytes[slot]);
  ctx->ws[slot] = nullptr;
  ctx->ws_bytes[slot] = 0;
}

int pinned_get(hisq_ctx *ctx, size_t bytes, void **out) {
  if (ctx->pinned_bytes < bytes) {
    if (ctx->pinned) {
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      HIPCHK(ctx, hipHostFree(ctx->pinned));
      ctx->pinned = nullptr;
      ctx->pinned_bytes = 0;
    }
    HIPCHK(ctx, hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
    ctx->pinned_bytes = bytes;
  }
  *out = ctx->pinned;
  return HISQ_OK;
}

static void free_links(hisq_ctx *ctx) {
  for (auto &l : ctx->links) {
    dev_free(ctx, l.base, l.bytes);
    l = LinkCopy{};
  }
  ctx->links_loaded = false;
}

void nn_free_state(hisq_ctx *ctx);

extern "C" {

const char *hisq_last_error(const hisq_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int hisq_create(hisq_ctx **out, const int dims[4], int device, void *stream) {
  if (!out || !dims) return set_err(nullptr, HISQ_ERR_ARG, "hisq_create: null argument");
  *out = nullptr;
  for (int i = 0; i < 4; ++i)
    if (dims[i] < 4 || dims[i] % 2)
      return set_err(nullptr, HISQ_ERR_ARG,
                     "hisq_create: extent %d of direction %d must be even and >= 4", dims[i], i);
  long long v = 1LL * dims[0] * dims[1] * dims[2] * dims[3];
  if (v / 2 > (1LL << 30))
    return set_err(nullptr, HISQ_ERR_ARG, "hisq_create: lattice too large (%lld sites)", v);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev)
    return set_err(nullptr, HISQ_ERR_HIP, "hisq_create: device %d not available (%d devices, %s)",
                   device, ndev, hipGetErrorString(e));
  e = hipSetDevice(device);
  if (e != hipSuccess)
    return set_err(nullptr, HISQ_ERR_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
  hisq_ctx *ctx = new hisq_ctx();
  Geometry &g = ctx->g;
  g.lx = dims[0];
  g.ly = dims[1];
  g.lz = dims[2];
  g.lt = dims[3];
  g.lxh = g.lx / 2;
  g.vh = int(v / 2);
  g.sy = g.lxh;
  g.sz = g.lxh * g.ly;
  g.st = g.lxh * g.ly * g.lz;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
      lds > 0)
    ctx->lds_max = size_t(lds);
  if (scratch_lookup(ctx) != HISQ_OK) {
    set_err(nullptr, HISQ_ERR_HIP, "hisq_create: %s", ctx->err.c_str());
    delete ctx;
    return HISQ_ERR_HIP;
  }
  *out = ctx;
  return HISQ_OK;
}

int hisq_destroy(hisq_ctx *ctx) {
  if (!ctx) return HISQ_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_links(ctx);
  for (int i = 0; i < WS_COUNT; ++i) ws_release(ctx, i);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  nn_free_state(ctx);
  delete ctx;
  return HISQ_OK;
}

int hisq_set_stream(hisq_ctx *ctx, void *stream) {
  if (!ctx) return HISQ_ERR_ARG;
  ctx->stream = static_cast<hipStream_t>(stream);
  return HISQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Link loading

__global__ void k_count_nonfinite(const double *__restrict__ p, size_t count, int *__restrict__ bad) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  int local = 0;
  for (; i < count; i += stride) local |= !isfinite(p[i]);
  if (local) atomicOr(bad, 1);
}

static bool is_device_ptr(const void *p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

static size_t link_elem_bytes(int prec) { return prec == HISQ_F64 ? 16 : (prec == HISQ_F32 ? 8 : 4); }

extern "C" int hisq_load_links(hisq_ctx *ctx, const double *fat, const double *naik, int copies,
                               int naik_recon) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!fat || !naik) return set_err(ctx, HISQ_ERR_ARG, "hisq_load_links: null link pointer");
  if (copies <= 0 || copies > HISQ_LINKS_ALL)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_load_links: bad copies mask %d", copies);
  if (!naik_recon_valid(naik_recon))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_load_links: naik_recon must be 18, 14, 13 or 9, got %d",
                   naik_recon);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const Geometry &g = ctx->g;
  const size_t nreal = size_t(g.vh) * 2 * 4 * 18;  // doubles per link field
  const double *dfat = fat, *dnaik = naik;
  if (!is_device_ptr(fat) || !is_device_ptr(naik)) {
    void *stage;
    RETCHK(ws_get(ctx, WS_LINKSTAGE, 2 * nreal * sizeof(double), &stage));
    double *s = static_cast<double *>(stage);
    HIPCHK(ctx, hipMemcpyAsync(s, fat, nreal * sizeof(double), hipMemcpyDefault, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(s + nreal, naik, nreal * sizeof(double), hipMemcpyDefault, ctx->stream));
    dfat = s;
    dnaik = s + nreal;
  }
  void *flagp;
  RETCHK(ws_get(ctx, WS_SCAL, 256, &flagp));
  int *flag = static_cast<int *>(flagp);
  HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
  k_count_nonfinite<<<1024, 256, 0, ctx->stream>>>(dfat, nreal, flag);
  k_count_nonfinite<<<1024, 256, 0, ctx->stream>>>(dnaik, nreal, flag);
  LAUNCHCHK(ctx, "k_count_nonfinite");
  int bad = 0;
  HIPCHK(ctx, hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (bad) return set_err(ctx, HISQ_ERR_NONFINITE, "hisq_load_links: non-finite link entries");

  free_links(ctx);
  for (auto &per_prec : ctx->tune)  // launch choices depend on the link format: tune again
    for (auto &per_n : per_prec)
      for (auto &t : per_n)
        if (t.state != TuneEntry::FORCED) t = TuneEntry{};
  for (int prec = 0; prec < 3; ++prec) {
    if (!(copies & (1 << prec))) continue;
    int recon = prec == HISQ_F64 ? 18 : naik_recon;
    size_t per_par = size_t(link_planes_total(recon)) * g.vh * link_elem_bytes(prec);
    LinkCopy &l = ctx->links[prec];
    int rc_alloc = dev_alloc(ctx, &l.base, 2 * per_par, "hisq_load_links");
    if (rc_alloc != HISQ_OK) {
      free_links(ctx);
      return rc_alloc;
    }
    l.bytes = 2 * per_par;
    l.recon = recon;
    l.par[0] = l.base;
    l.par[1] = static_cast<char *>(l.base) + per_par;
    for (int par = 0; par < 2; ++par) {
      double err = 0.0;
      int rc = launch_pack_links(ctx, dfat, dnaik, prec, recon, par, l.par[par],
                                 recon != 18 ? &err : nullptr);
      if (rc != HISQ_OK) {
        free_links(ctx);
        return rc;
      }
      if (recon != 18 && !(err <= 1e-10)) {
        free_links(ctx);
        return set_err(ctx, HISQ_ERR_ARG,
                       "hisq_load_links: Naik links are not of the form the %d-real storage needs "
                       "(14: a multiple of a U(3) matrix; 13 and 9: a real multiple of an SU(3) "
                       "matrix; reconstruction error %.3g); use naik_recon = 18",
                       recon, err);
      }
    }
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ws_release(ctx, WS_LINKSTAGE);  // the staging copy is only needed while packing
  ctx->naik_recon = naik_recon;
  ctx->links_loaded = true;
  return HISQ_OK;
}
