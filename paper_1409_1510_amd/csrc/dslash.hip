// Multi-rhs HISQ half Dslash: launch-configuration choice (automatic tuning, Section 2), the
// C ABI entry points hisq_dslash_mrhs / hisq_apply_m and the tuning controls.  The kernel
// itself is in dslash_kernel.hpp, instantiated per precision in dslash_f64/f32/f16.hip.
#include "dslash_kernel.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <utility>
#include <vector>

using dslash::Args;
using dslash::DslashFn;

namespace {

DslashFn lookup(int prec, int recon, bool epi, const hisq_launch &c) {
  const int lds = c.lds_links;
  if (prec == HISQ_F64)
    return dslash_fn_f64(epi, c.rhs_per_thread, c.sites_per_block, c.nontemporal_links, lds);
  if (prec == HISQ_F32)
    return dslash_fn_f32(epi, recon, c.rhs_per_thread, c.sites_per_block, c.nontemporal_links, lds);
  return dslash_fn_f16(epi, recon, c.rhs_per_thread, c.sites_per_block, c.nontemporal_links, lds);
}

size_t lds_bytes(int prec, int recon, const hisq_launch &c) {
  if (!c.lds_links) return 0;
  const size_t elem = prec == HISQ_F64 ? 16 : (prec == HISQ_F32 ? 8 : 4);
  if (prec == HISQ_F64) recon = 18;
  const bool r14 = recon == 14;
  if (c.sites_per_block == 32)  // 32-site form: half of the whole-site form's pieces (18 and 14)
    return size_t(link_planes_total(recon)) * 32 * elem + (r14 ? size_t(24) * 32 * 8 : 0) +
           dslash::kNbrTable32Bytes;
  if (c.lds_links >= 4)  // two buffers of one direction's planes (+ rebuilt Naik rows; 18 and 14)
    return 2 * size_t(r14 ? 32 : 36) * 64 * elem + (r14 ? size_t(12) * 64 * 8 : 0);
  // staged planes, rebuilt Naik entries (arithmetic type: 8 bytes), neighbour table
  return size_t(dslash::lds_staged_planes(recon)) * 64 * elem + size_t(dslash::lds_rebuilt_entries(recon)) * 64 * 8 +
         dslash::kNbrTableBytes;
}

bool config_valid(int prec, bool epi, const hisq_launch &c, int recon = 18, size_t lds_max = 0) {
  if (c.lds_links && lds_max && lds_bytes(prec, recon, c) > lds_max) return false;
  const int rt = c.rhs_per_thread;
  if (rt != 1 && rt != 2 && rt != 4 && rt != 8 && rt != 16) return false;
  if (c.sites_per_block != 32 && c.sites_per_block != 64 && c.sites_per_block != 256) return false;
  if (c.nontemporal_links != 0 && c.nontemporal_links != 1) return false;
  if (c.lds_links < 0 || c.lds_links > 6) return false;
  if (c.xcd_map < 0 || c.xcd_map > 3 || (c.xcd_map != 0 && !c.lds_links)) return false;
  return lookup(prec, prec == HISQ_F64 ? 18 : recon, epi, c) != nullptr;
}

// rhs tiles a workgroup of the direction-pipelined forms can hold (their waves keep every tile's
// accumulators across the four directions)
int max_tiles(const hisq_launch &c) {
  if (c.lds_links == 4) return 16;
  if (c.lds_links == 5) return 32;
  if (c.lds_links == 6) return 16;
  return 1 << 30;
}
bool fits_n(const hisq_launch &c, int n) {
  return (n + c.rhs_per_thread - 1) / c.rhs_per_thread <= max_tiles(c);
}
// every form addresses a rhs tile with 32-bit offsets: the LDS forms in bytes (a tile of
// rhs_per_thread rhs, 2 rhs_per_thread in the 32-site form), the register-tile form in complex
// elements
bool fits_lattice(const hisq_launch &c, const Geometry &g, int prec) {
  const size_t elem = prec == HISQ_F64 ? 16 : 8;
  const size_t tile = size_t(c.rhs_per_thread) * (c.sites_per_block == 32 ? 2 : 1);
  const size_t span = tile * 3 * size_t(g.vh) * (c.lds_links ? elem : 1);
  return span < (size_t(1) << 32);
}

int next_pow2(int n) {
  int p = 1;
  while (p < n) p *= 2;
  return p;
}

// Heuristic used until a configuration is tuned or forced (the largest register tile up to 4 or
// 8 rhs whose offsets fit in 32 bits on this lattice).
hisq_launch heuristic(const Geometry &g, int prec, int n, bool epi) {
  int cap = (prec == HISQ_F64 || epi) ? 4 : 8;
  int rt = 1;
  while (rt * 2 <= cap && rt * 2 <= n) rt *= 2;
  hisq_launch c{rt, 256, 0, 0, 0};
  while (c.rhs_per_thread > 1 && !fits_lattice(c, g, prec)) c.rhs_per_thread /= 2;
  return c;
}

struct Geo {
  int ntiles, ngroups, nsblk, grid, xmap, zmap_bps, zmap_zr;
};

// XCD maps: all need whole 64-site blocks per (z, t) plane; the z-slab map (1) needs Lz
// divisible by 8, the y-slab maps (2, 3) a multiple of 8 blocks per plane, and the z-tiled walk
// of map 3 Lz divisible by 4
bool map_possible(const Geometry &g, int xm) {
  if (xm == 0) return true;
  if ((g.lxh * g.ly) % 64 != 0) return false;
  if (xm == 1) return g.lz % 8 == 0;
  if (xm == 2) return (g.lxh * g.ly / 64) % 8 == 0;
  if (xm == 3) return (g.lxh * g.ly / 64) % 8 == 0 && g.lz % 4 == 0;
  return false;
}
const char *map_requirement(int xm) {
  return xm == 1 ? "the z-slab XCD map needs (Lx/2)*Ly % 64 == 0 and Lz % 8 == 0"
       : xm == 2 ? "the y-slab XCD map needs (Lx/2)*Ly % 512 == 0"
                 : "the z-tiled y-slab XCD map needs (Lx/2)*Ly % 512 == 0 and Lz % 4 == 0";
}

Geo geometry(const Geometry &g, int n, const hisq_launch &c) {
  Geo o;
  o.xmap = 0;
  o.zmap_bps = 0;
  o.zmap_zr = 0;
  const bool half = c.sites_per_block == 32;  // 32-site LDS form: tiles of 2 rt rhs
  const int tw = c.rhs_per_thread * (half ? 2 : 1);
  o.ntiles = (n + tw - 1) / tw;
  const int tpb = 256 / c.sites_per_block;
  o.ngroups = c.lds_links ? 1 : (o.ntiles + tpb - 1) / tpb;  // the LDS form loops over the tiles
  const int spb = half ? 64 : c.sites_per_block;              // the XCD maps deal 64-site blocks
  o.nsblk = (g.vh + spb - 1) / spb;
  const int nb = o.nsblk * o.ngroups;
  o.grid = (nb + 7) / 8 * 8;
  if (c.lds_links && c.xcd_map && map_possible(g, c.xcd_map)) {
    o.xmap = c.xcd_map;
    o.zmap_bps = g.lxh * g.ly / 64;
    o.zmap_zr = g.lz / 8;
    o.grid = o.nsblk;  // 8 * Lt * (Lz/8) * bps (z slabs) or 8 * Lz * Lt * (bps/8) (y slabs)
  }
  if (half) o.grid *= 2;  // two workgroups per 64-site block
  return o;
}

int run(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in, void *out, bool epi,
        double mass2, const void *pvec, double *partial, const int *active, const hisq_launch &c) {
  const LinkCopy &l = ctx->links[prec];
  DslashFn fn = lookup(prec, l.recon, epi, c);
  if (!fn) return set_err(ctx, HISQ_ERR_ARG, "invalid Dslash launch configuration");
  if (lds_bytes(prec, l.recon, c) > ctx->lds_max)
    return set_err(ctx, HISQ_ERR_ARG, "Dslash launch configuration needs %zu bytes of LDS (%zu available)",
                   lds_bytes(prec, l.recon, c), ctx->lds_max);
  const Geo geo = geometry(ctx->g, n, c);
  if (!fits_n(c, n))
    return set_err(ctx, HISQ_ERR_ARG, "this Dslash form holds at most %d rhs tiles (n = %d)", max_tiles(c), n);
  if (!fits_lattice(c, ctx->g, prec))
    return set_err(ctx, HISQ_ERR_ARG, "rhs_per_thread too large for this lattice: a rhs tile must span less "
                   "than 2^32 bytes (LDS forms) or complex elements (register-tile form)");
  if (c.xcd_map && geo.xmap != c.xcd_map) return set_err(ctx, HISQ_ERR_ARG, "%s", map_requirement(c.xcd_map));
  Args a{l.par[out_parity], in, out, ctx->g, out_parity, n, geo.ntiles, geo.ngroups, geo.nsblk,
         mass2, pvec, partial, active, geo.xmap, geo.zmap_bps, geo.zmap_zr,
         dslash::make_fastdiv(unsigned(ctx->g.lxh)), dslash::make_fastdiv(unsigned(ctx->g.ly)),
         dslash::make_fastdiv(unsigned(ctx->g.lz))};
  fn(a, dim3(geo.grid), ctx->stream);
  LAUNCHCHK(ctx, "k_dslash");
  return HISQ_OK;
}

bool autotune_enabled() {
  static int on = [] {
    const char *e = getenv("HISQ_AUTOTUNE");
    return e ? atoi(e) : 1;
  }();
  return on != 0;
}

}  // namespace

int dslash_partials(const Geometry &g) { return (g.vh + 63) / 64; }

int tune(hisq_ctx *ctx, int prec, int n, bool epi, hisq_launch *best_out, double *ms_out) {
  const Geometry &g = ctx->g;
  const size_t bytes = size_t(n) * 3 * g.vh * cplx_bytes(prec);
  void *a, *b, *pp;
  RETCHK(ws_get(ctx, WS_TUNE0, bytes, &a));
  RETCHK(ws_get(ctx, WS_TUNE1, bytes, &b));
  RETCHK(ws_get(ctx, WS_TUNE2, size_t(n) * dslash_partials(g) * sizeof(double), &pp));
  HIPCHK(ctx, hipMemsetAsync(a, 0, bytes, ctx->stream));
  HIPCHK(ctx, hipMemsetAsync(b, 0, bytes, ctx->stream));
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  hisq_launch best = heuristic(g, prec, n, epi);
  float best_ms = 1e30f;
  const int rts[] = {1, 2, 4, 8, 16};
  int rc = HISQ_OK;
  std::vector<std::pair<float, hisq_launch>> timed;
  // launches alternate between the two output parities (a -> b, b -> a), as in D = D_oe + D_eo
  // and in the solvers: repeating one parity would let the 256 MB last-level cache keep that
  // parity's links and time a cache-resident case
  auto time_cfg = [&](const hisq_launch &c, int reps, float *ms_out) -> int {
    for (int k = 0; k <= 2 * reps; ++k) {
      if (k == 1) (void)hipEventRecord(e0, ctx->stream);
      const bool odd = k & 1;
      RETCHK(run(ctx, odd ? 0 : 1, prec, n, odd ? b : a, odd ? a : b, epi, 0.01, odd ? b : a,
                 static_cast<double *>(pp), nullptr, c));
    }
    (void)hipEventRecord(e1, ctx->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms / (2 * reps);
    return HISQ_OK;
  };
  for (int rt : rts) {
    if (rt > next_pow2(n)) break;
    for (int spb : {256, 64, 32})
      for (int nt : {0, 1})
        for (int lds = 0; lds <= 6; ++lds)
          for (int xm : {0, 1, 2, 3}) {
            hisq_launch c{rt, spb, nt, lds, xm};
            if (!config_valid(prec, epi, c, ctx->links[prec].recon, ctx->lds_max)) continue;
            if (!map_possible(g, xm) || !fits_n(c, n) || !fits_lattice(c, g, prec)) continue;
            float ms;
            rc = time_cfg(c, 3, &ms);
            if (rc != HISQ_OK) break;
            timed.push_back({ms, c});
          }
  }
  if (rc == HISQ_OK && !timed.empty()) {  // re-time the three fastest with more repetitions
    std::sort(timed.begin(), timed.end(), [](const auto &u, const auto &v) { return u.first < v.first; });
    for (size_t i = 0; i < timed.size() && i < 3 && rc == HISQ_OK; ++i) {
      float ms;
      rc = time_cfg(timed[i].second, 12, &ms);
      if (rc == HISQ_OK && ms < best_ms) {
        best_ms = ms;
        best = timed[i].second;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int slot : {WS_TUNE0, WS_TUNE1, WS_TUNE2}) ws_release(ctx, slot);  // tuning scratch is not kept
  if (rc != HISQ_OK) return rc;
  TuneEntry &t = ctx->tune[prec][n][epi ? 1 : 0];
  t.cfg = best;
  t.state = TuneEntry::TUNED;
  t.ms = best_ms;
  if (best_out) *best_out = best;
  if (ms_out) *ms_out = best_ms;
  return HISQ_OK;
}

int config_for(hisq_ctx *ctx, int prec, int n, bool epi, hisq_launch *c) {
  TuneEntry &t = ctx->tune[prec][n][epi ? 1 : 0];
  if (t.state == TuneEntry::NONE) {
    if (autotune_enabled()) {
      RETCHK(tune(ctx, prec, n, epi, nullptr, nullptr));
    } else {
      t.cfg = heuristic(ctx->g, prec, n, epi);
      t.state = TuneEntry::HEURISTIC;
    }
  }
  *c = t.cfg;
  return HISQ_OK;
}

int launch_dslash(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in, void *out,
                  bool epi, double mass2, const void *pvec, double *partial, int *nblk_out,
                  const int *active) {
  if (!ctx->links[prec].base)
    return set_err(ctx, HISQ_ERR_STATE, "no %s link copy loaded (see hisq_load_links copies)",
                   prec == HISQ_F64 ? "FP64" : (prec == HISQ_F32 ? "FP32" : "FP16"));
  hisq_launch c;
  RETCHK(config_for(ctx, prec, n, epi, &c));
  RETCHK(run(ctx, out_parity, prec, n, in, out, epi, mass2, pvec, partial, active, c));
  if (nblk_out) *nblk_out = dslash_partials(ctx->g);
  return HISQ_OK;
}

extern "C" int hisq_set_launch(hisq_ctx *ctx, int prec, int n, const hisq_launch *cfg) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!prec_valid(prec) || n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_set_launch: bad precision or n");
  for (int epi = 0; epi < 2; ++epi) {
    TuneEntry &t = ctx->tune[prec][n][epi];
    if (!cfg) {
      t = TuneEntry{};
      continue;
    }
    hisq_launch c = *cfg;
    // the 32-site form exists for the plain half Dslash only: the fused M form keeps its own
    // (tuned or heuristic) configuration
    if (epi && c.sites_per_block == 32 && c.lds_links) continue;
    const int recon = ctx->links[prec].base ? ctx->links[prec].recon : 18;
    if (c.xcd_map >= 1 && c.xcd_map <= 3 && !map_possible(ctx->g, c.xcd_map))
      return set_err(ctx, HISQ_ERR_ARG, "%s", map_requirement(c.xcd_map));
    if (!config_valid(prec, epi, c, recon, ctx->lds_max)) {
      if (epi) {  // the fused-M form caps the register tile: use the largest valid one
        while (c.rhs_per_thread > 1 && !config_valid(prec, true, c, recon, ctx->lds_max))
          c.rhs_per_thread /= 2;
      }
      if (!config_valid(prec, epi, c, recon, ctx->lds_max))
        return set_err(ctx, HISQ_ERR_ARG, "hisq_set_launch: invalid configuration (rt %d, spb %d, nt %d)",
                       cfg->rhs_per_thread, cfg->sites_per_block, cfg->nontemporal_links);
    }
    if (!fits_n(c, n))
      return set_err(ctx, HISQ_ERR_ARG, "hisq_set_launch: this form holds at most %d rhs tiles (n = %d)",
                     max_tiles(c), n);
    if (!fits_lattice(c, ctx->g, prec))
      return set_err(ctx, HISQ_ERR_ARG,
                     "hisq_set_launch: rhs_per_thread too large for this lattice (a rhs tile must span less "
                     "than 2^32 bytes in the LDS forms, 2^32 complex elements in the register-tile form)");
    t.cfg = c;
    t.state = TuneEntry::FORCED;
  }
  return HISQ_OK;
}

extern "C" int hisq_get_launch(hisq_ctx *ctx, int prec, int n, int fused_m, hisq_launch *cfg) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!cfg || !prec_valid(prec) || n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_get_launch: bad argument");
  const TuneEntry &t = ctx->tune[prec][n][fused_m ? 1 : 0];
  *cfg = t.state == TuneEntry::NONE ? heuristic(ctx->g, prec, n, fused_m != 0) : t.cfg;
  return HISQ_OK;
}

// ---- persistent tuning table ----------------------------------------------------------------
// text lines: lx ly lz lt prec recon n fused rt spb nt lds xm ms

extern "C" int hisq_save_tuning(hisq_ctx *ctx, const char *path) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!path) return set_err(ctx, HISQ_ERR_ARG, "hisq_save_tuning: null path");
  const Geometry &g = ctx->g;
  std::vector<std::string> keep;
  if (FILE *f = fopen(path, "r")) {  // keep entries of other lattices / link formats
    char line[512];
    while (fgets(line, sizeof line, f)) {
      int d[4], prec, recon;
      if (line[0] == '#' || sscanf(line, "%d %d %d %d %d %d", &d[0], &d[1], &d[2], &d[3], &prec, &recon) != 6)
        continue;
      const bool mine = d[0] == g.lx && d[1] == g.ly && d[2] == g.lz && d[3] == g.lt && prec >= 0 && prec < 3 &&
                        ctx->links[prec].base && recon == ctx->links[prec].recon;
      if (!mine) keep.push_back(line);
    }
    fclose(f);
  }
  FILE *f = fopen(path, "w");
  if (!f) return set_err(ctx, HISQ_ERR_IO, "hisq_save_tuning: cannot write %s", path);
  fprintf(f, "# lx ly lz lt prec recon n fused rt spb nt lds xm ms\n");
  for (const auto &l : keep) fputs(l.c_str(), f);
  for (int prec = 0; prec < 3; ++prec) {
    if (!ctx->links[prec].base) continue;
    for (int n = 1; n <= HISQ_MAX_RHS; ++n)
      for (int e = 0; e < 2; ++e) {
        const TuneEntry &t = ctx->tune[prec][n][e];
        if (t.state != TuneEntry::TUNED) continue;
        fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d %.5f\n", g.lx, g.ly, g.lz, g.lt, prec,
                ctx->links[prec].recon, n, e, t.cfg.rhs_per_thread, t.cfg.sites_per_block,
                t.cfg.nontemporal_links, t.cfg.lds_links, t.cfg.xcd_map, t.ms);
      }
  }
  return fclose(f) == 0 ? HISQ_OK : set_err(ctx, HISQ_ERR_IO, "hisq_save_tuning: write failed");
}

extern "C" int hisq_load_tuning(hisq_ctx *ctx, const char *path, int *n_loaded) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!path) return set_err(ctx, HISQ_ERR_ARG, "hisq_load_tuning: null path");
  if (!ctx->links_loaded) return set_err(ctx, HISQ_ERR_STATE, "hisq_load_tuning: load the links first");
  FILE *f = fopen(path, "r");
  if (!f) return set_err(ctx, HISQ_ERR_IO, "hisq_load_tuning: cannot read %s", path);
  const Geometry &g = ctx->g;
  char line[512];
  int count = 0;
  while (fgets(line, sizeof line, f)) {
    int d[4], prec, recon, n, e;
    hisq_launch c;
    float ms;
    if (line[0] == '#' ||
        sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %d %f", &d[0], &d[1], &d[2], &d[3], &prec, &recon,
               &n, &e, &c.rhs_per_thread, &c.sites_per_block, &c.nontemporal_links, &c.lds_links, &c.xcd_map,
               &ms) != 14)
      continue;
    if (d[0] != g.lx || d[1] != g.ly || d[2] != g.lz || d[3] != g.lt) continue;
    if (prec < 0 || prec > 2 || n < 1 || n > HISQ_MAX_RHS || (e != 0 && e != 1)) continue;
    if (!ctx->links[prec].base || ctx->links[prec].recon != recon) continue;
    if (!config_valid(prec, e != 0, c, recon, ctx->lds_max)) continue;
    if (!map_possible(g, c.xcd_map) || !fits_n(c, n) || !fits_lattice(c, g, prec)) continue;
    TuneEntry &t = ctx->tune[prec][n][e];
    t.cfg = c;
    t.state = TuneEntry::TUNED;
    t.ms = ms;
    ++count;
  }
  fclose(f);
  if (n_loaded) *n_loaded = count;
  return HISQ_OK;
}

extern "C" int hisq_autotune(hisq_ctx *ctx, int prec, int n, int fused_m, hisq_launch *best,
                             double *ms_out) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!prec_valid(prec) || n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_autotune: bad precision or n");
  if (!ctx->links_loaded || !ctx->links[prec].base)
    return set_err(ctx, HISQ_ERR_STATE, "hisq_autotune: link copy of this precision not loaded");
  return tune(ctx, prec, n, fused_m != 0, best, ms_out);
}

extern "C" int hisq_dslash_mrhs(hisq_ctx *ctx, int out_parity, int prec, int n, const void *in,
                                void *out) {
  if (!ctx) return HISQ_ERR_ARG;
  if (!in || !out) return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: null vector pointer");
  if (in == out) return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: in and out alias");
  if (out_parity != 0 && out_parity != 1)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: out_parity must be 0 or 1");
  if (!prec_valid(prec)) return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: bad precision %d", prec);
  if (!elem_aligned(in, cplx_bytes(prec)) || !elem_aligned(out, cplx_bytes(prec)))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_dslash_mrhs: vectors must be aligned to %zu bytes", cplx_bytes(prec));
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
  if (!elem_aligned(in, cplx_bytes(prec)) || !elem_aligned(out, cplx_bytes(prec)) ||
      !elem_aligned(pq_out, sizeof(double)))
    return set_err(ctx, HISQ_ERR_ARG, "hisq_apply_m: vectors must be aligned to %zu bytes, pq_out to 8",
                   cplx_bytes(prec));
  if (n < 1 || n > HISQ_MAX_RHS)
    return set_err(ctx, HISQ_ERR_ARG, "hisq_apply_m: n = %d outside 1..%d", n, HISQ_MAX_RHS);
  if (!ctx->links_loaded) return set_err(ctx, HISQ_ERR_STATE, "hisq_apply_m: no links loaded");
  const Geometry &g = ctx->g;
  void *tmp;
  RETCHK(ws_get(ctx, WS_TMP_ODD, size_t(n) * 3 * g.vh * cplx_bytes(prec), &tmp));
  const int nblk = dslash_partials(g);
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
