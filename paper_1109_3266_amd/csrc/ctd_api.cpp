// C ABI of the MI355X imaging-dose transport library: handles, input
// validation, device buffers, batch driver (Jia et al., Sec. 2.2.1: histories
// split into N_b batches, one transport launch per batch, per-voxel mean and
// uncertainty from the batches), run-to-sigma controller, batched engine,
// readout and the launch-configuration tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctd_api_internal.h"
#include "ctd_bound.h"
#include "ctd_headroom.h"
#include "ctd_tables.h"

using namespace ctd;

// ------------------------------------------------------------ error helpers

int ctd::set_err(ctd_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int ctd::hip_err(ctd_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return CTD_OK;
  if (e == hipErrorOutOfMemory)
    return set_err(ctx, CTD_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_err(ctx, CTD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                        \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return ctd::hip_err((ctx), e_, #call); \
  } while (0)

#define NEED(ctx, cond, ...)                                   \
  do {                                                         \
    if (!(cond)) return ctd::set_err((ctx), CTD_EINVAL, __VA_ARGS__); \
  } while (0)

// A case whose last run call failed part-way (ctd_case::failed) is refused
// by the calls that run or read it until ctd_case_reset.
#define NEED_INTACT(ctx, cs)                                                                \
  NEED(ctx, !(cs)->failed,                                                                  \
       "a run call on this case failed after enqueueing part of its work; its sums are "    \
       "undefined until ctd_case_reset")

static void dfree(void *p) {
  if (p) (void)hipFree(p);
}

// --------------------------------------------------------------- context

extern "C" int32_t ctd_create(ctd_ctx **out, int32_t device) {
  if (!out) return CTD_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return CTD_EDEVICE;
  }
  ctd_ctx *ctx = new (std::nothrow) ctd_ctx();
  if (!ctx) return CTD_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return CTD_EDEVICE;
  }
  ctx->stream = ctx->own;
  ctx->n_cu = device_cu_count(device);
  if (ctx->n_cu <= 0) ctx->n_cu = 256;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) ==
          hipSuccess && v > 0)
    ctx->lds_per_cu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
          hipSuccess && v > 0)
    ctx->lds_per_block = v;
  (void)hipGetLastError();
  ctx->slots.resize(64);
  if (hipMalloc(&ctx->sigma_scratch, sizeof(double) * (3 * kSigmaBlocks + 4)) != hipSuccess ||
      hipMalloc(&ctx->pack_stats, sizeof(unsigned int) * kPackStats) != hipSuccess ||
      hipHostMalloc(&ctx->sigma_host, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess) {
    ctd_destroy(ctx);
    return CTD_ENOMEM;
  }
  // per-XCD tallies need every XCC id to index one of kTallyCopies copies
  unsigned int *probe = nullptr;
  unsigned int mx = ~0u;
  if (hipMalloc(&probe, 4) == hipSuccess && hipMemsetAsync(probe, 0, 4, ctx->stream) == hipSuccess &&
      launch_xcc_probe(probe, 16 * ctx->n_cu, ctx->stream) == 0 &&
      hipMemcpyAsync(&mx, probe, 4, hipMemcpyDeviceToHost, ctx->stream) == hipSuccess &&
      hipStreamSynchronize(ctx->stream) == hipSuccess) {
    ctx->max_xcc = mx;
    ctx->xcd_tally_ok = mx < (unsigned)kTallyCopies;
  }
  dfree(probe);
  // the static round table of ctd_run_batches_static: each device holds its
  // own copy of the array, at the address this lookup returns (never the
  // host-side name)
  if (static_scratch_address(&ctx->static_table) != 0) {
    (void)hipGetLastError();
    ctx->static_table = nullptr;
  }
  *out = ctx;
  return CTD_OK;
}

extern "C" int32_t ctd_destroy(ctd_ctx *ctx) {
  if (!ctx) return CTD_EINVAL;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->own) (void)hipStreamSynchronize(ctx->own);
  for (auto &s : ctx->slots) {
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.host) (void)hipHostFree(s.host);
    dfree(s.dev);
  }
  dfree(ctx->sigma_scratch);
  dfree(ctx->pack_stats);
  if (ctx->sigma_host) (void)hipHostFree(ctx->sigma_host);
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  delete ctx;
  return CTD_OK;
}

extern "C" const char *ctd_last_error(const ctd_ctx *ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

extern "C" int32_t ctd_set_stream(ctd_ctx *ctx, void *hip_stream) {
  if (!ctx) return CTD_EINVAL;
  // work already enqueued finishes before anything goes to the new stream
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->own;
  return CTD_OK;
}

// --------------------------------------------------------------- phantom

// Piecewise-constant phantoms (at most 256 distinct (rho, material) records)
// also get a 1-byte-per-voxel index into a 256-entry table: an 8x smaller
// gather footprint for the same numbers.  Scanned in slices so a phantom
// with many distinct densities is rejected after a few thousand voxels.
static int build_palette(ctd_ctx *ctx, ctd_phantom *ph) {
  const int64_t V = ph->V;
  const int64_t slice = (int64_t)1 << 20;
  std::vector<uint2> rec((size_t)std::min<int64_t>(V, slice));
  std::vector<uint8_t> idx((size_t)V);
  uint64_t keys[256];
  int n = 0;
  for (int64_t b = 0; b < V; b += slice) {
    const int64_t m = std::min<int64_t>(slice, V - b);
    HIPCHK(ctx, hipMemcpy(rec.data(), ph->vox + b, sizeof(uint2) * m, hipMemcpyDeviceToHost));
    uint64_t last = ~0ull;
    int last_i = -1;
    for (int64_t i = 0; i < m; ++i) {
      const uint64_t key = ((uint64_t)rec[i].y << 32) | rec[i].x;
      int k = -1;
      if (key == last) {
        k = last_i;
      } else {
        for (int j = 0; j < n; ++j)
          if (keys[j] == key) { k = j; break; }
        if (k < 0) {
          if (n == 256) return CTD_OK;  // too many distinct records: keep 8-byte layout
          keys[n] = key;
          k = n++;
        }
        last = key;
        last_i = k;
      }
      idx[(size_t)(b + i)] = (uint8_t)k;
    }
  }
  std::vector<uint2> pal(256, make_uint2(0u, 0u));
  for (int j = 0; j < n; ++j) pal[j] = make_uint2((uint32_t)keys[j], (uint32_t)(keys[j] >> 32));
  HIPCHK(ctx, hipMalloc(&ph->vox8, (size_t)V));
  HIPCHK(ctx, hipMalloc(&ph->palette, sizeof(uint2) * 256));
  HIPCHK(ctx, hipMemcpy(ph->vox8, idx.data(), (size_t)V, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ph->palette, pal.data(), sizeof(uint2) * 256, hipMemcpyHostToDevice));
  ph->npal = n;
  return CTD_OK;
}

// Bound grids of a record-layout phantom: for each material present, K
// density levels spaced evenly over (rho_min, rho_max], rounded up to float,
// the last exactly rho_max (K = 254 / materials present, at most 32); then
// every block of 1, 2 and 4 voxels per edge is classified by its material
// and the first level at or above its largest density (k_block_class).
static int build_bound_grids(ctd_ctx *ctx, ctd_phantom *ph) {
  int n_present = 0;
  for (int m = 0; m < 256; ++m) n_present += ph->present[m] ? 1 : 0;
  if (n_present == 0 || n_present > 254) return CTD_OK;  // no classes: no early rejection
  const int K = std::min(32, 254 / n_present);
  std::vector<uint2> cls(256, make_uint2(0u, 0u));
  std::vector<int2> range(256, make_int2(0, 0));
  int c = 0;
  for (int m = 0; m < 256; ++m) {
    if (!ph->present[m]) continue;
    const double lo = ph->rho_min[m], hi = ph->rho_max[m];
    const float top = (float)hi;  // rho_max came from float bits: exact
    range[m] = make_int2(c, K);
    for (int l = 0; l < K; ++l) {
      float f = l == K - 1 ? top : std::min(round_up_to_float(lo + (hi - lo) * (l + 1) / K), top);
      uint32_t bits;
      std::memcpy(&bits, &f, 4);
      cls[c++] = make_uint2(bits, (uint32_t)m);
    }
  }
  const ctd_grid &g = ph->g;
  HIPCHK(ctx, hipMalloc(&ph->bclass, sizeof(uint2) * 256));
  HIPCHK(ctx, hipMalloc(&ph->bclass_range, sizeof(int2) * 256));
  HIPCHK(ctx, hipMemcpy(ph->bclass, cls.data(), sizeof(uint2) * 256, hipMemcpyHostToDevice));
  HIPCHK(ctx, hipMemcpy(ph->bclass_range, range.data(), sizeof(int2) * 256,
                        hipMemcpyHostToDevice));
  for (int s = 0; s < 3; ++s) {
    const int e = (1 << s) - 1;
    const size_t nb = (size_t)((g.nx + e) >> s) * (size_t)((g.ny + e) >> s) *
                      (size_t)((g.nz + e) >> s);
    HIPCHK(ctx, hipMalloc(&ph->bgrid[s], nb));
    if (launch_block_class(ph->vox, g.nx, g.ny, g.nz, s, ph->bclass, ph->bclass_range,
                           ph->bgrid[s], ctx->stream) != 0)
      return hip_err(ctx, hipGetLastError(), "bound grid kernel");
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ph->nclass = c;
  ph->bclass_host.assign(cls.begin(), cls.begin() + c);
  return CTD_OK;
}

static void free_phantom_buffers(ctd_phantom *ph) {
  dfree(ph->vox);
  dfree(ph->vox8);
  dfree(ph->palette);
  for (auto &b : ph->bgrid) dfree(b);
  dfree(ph->bclass);
  dfree(ph->bclass_range);
}

extern "C" int32_t ctd_phantom_load(ctd_ctx *ctx, const ctd_grid *g, const uint8_t *mat,
                                    const float *rho, int32_t mem, ctd_phantom **out) {
  if (!ctx || !out) return CTD_EINVAL;
  *out = nullptr;
  NEED(ctx, g && mat && rho, "null argument");
  NEED(ctx, g->nx > 0 && g->ny > 0 && g->nz > 0, "grid dimensions must be positive");
  NEED(ctx, g->dx > 0 && g->dy > 0 && g->dz > 0, "voxel spacing must be positive");
  NEED(ctx, mem == CTD_MEM_HOST || mem == CTD_MEM_DEVICE, "mem must be HOST or DEVICE");
  const int64_t V = (int64_t)g->nx * g->ny * g->nz;
  NEED(ctx, V < ((int64_t)1 << 31), "at most 2^31 - 1 voxels");
  NEED(ctx, g->nx < (1 << 24) && g->ny < (1 << 24) && g->nz < (1 << 24), "axis too long");
  // the transport forms voxel indices with 24-bit multiplies: (z ny + y) nx + x
  NEED(ctx, (int64_t)g->ny * g->nz <= ((int64_t)1 << 24), "ny * nz must be at most 2^24");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctd_phantom *ph = new (std::nothrow) ctd_phantom();
  if (!ph) return CTD_ENOMEM;
  ph->device = ctx->device;
  ph->g = *g;
  ph->V = V;
  uint8_t *dmat = nullptr;
  float *drho = nullptr;
  // the context's statistics buffer: a device-memory input is packed with no
  // allocation freed on the way (a free waits for the whole device)
  unsigned int *dstat = ctx->pack_stats;
  int rc = CTD_OK;
  auto fail = [&](int code) {
    dfree(dmat);
    dfree(drho);
    free_phantom_buffers(ph);
    delete ph;
    return code;
  };
  hipError_t e = hipMalloc(&ph->vox, sizeof(uint2) * V);
  if (e != hipSuccess) return fail(hip_err(ctx, e, "phantom alloc"));
  const uint8_t *pm = mat;
  const float *pr = rho;
  if (mem == CTD_MEM_HOST) {
    if ((e = hipMalloc(&dmat, V)) != hipSuccess || (e = hipMalloc(&drho, 4 * V)) != hipSuccess)
      return fail(hip_err(ctx, e, "phantom staging alloc"));
    if ((e = hipMemcpyAsync(dmat, mat, V, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(drho, rho, 4 * V, hipMemcpyHostToDevice, ctx->stream)) != hipSuccess)
      return fail(hip_err(ctx, e, "phantom upload"));
    pm = dmat;
    pr = drho;
  }
  if ((e = hipMemsetAsync(dstat, 0, sizeof(unsigned int) * kPackStats, ctx->stream)) != hipSuccess)
    return fail(hip_err(ctx, e, "phantom stats clear"));
  if (launch_pack(pm, pr, ph->vox, V, dstat, ctx->stream) != 0)
    return fail(hip_err(ctx, hipGetLastError(), "pack kernel"));
  unsigned int hstat[kPackStats];
  if ((e = hipMemcpyAsync(hstat, dstat, sizeof hstat, hipMemcpyDeviceToHost, ctx->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
    return fail(hip_err(ctx, e, "phantom stats readback"));
  if (hstat[513] != 0) {
    rc = set_err(ctx, CTD_EINVAL, "%u voxels with a negative or non-finite density", hstat[513]);
    return fail(rc);
  }
  ph->max_mat = (int)hstat[512];
  for (int m = 0; m < 256; ++m) {
    float f;
    std::memcpy(&f, &hstat[m], 4);
    ph->rho_max[m] = (double)f;
    const unsigned int mn = ~hstat[514 + m];
    std::memcpy(&f, &mn, 4);
    ph->rho_min[m] = hstat[256 + m] ? (double)f : 0.0;
    ph->present[m] = hstat[256 + m] != 0;
    ph->count[m] = hstat[256 + m];
  }
  dfree(dmat);
  dfree(drho);
  dmat = nullptr;
  drho = nullptr;
  if ((rc = build_palette(ctx, ph)) != CTD_OK) return fail(rc);
  if (ph->npal == 0 && (rc = build_bound_grids(ctx, ph)) != CTD_OK) return fail(rc);
  *out = ph;
  return CTD_OK;
}

extern "C" int32_t ctd_phantom_release(ctd_ctx *ctx, ctd_phantom *ph) {
  if (!ctx || !ph) return CTD_EINVAL;
  if (ph->refs > 0) return set_err(ctx, CTD_EBUSY, "phantom is used by %d case(s)", ph->refs.load());
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_phantom_buffers(ph);
  delete ph;
  return CTD_OK;
}

// ------------------------------------------------------------- materials

static int upload(ctd_ctx *ctx, void **dst, const void *src, size_t bytes) {
  HIPCHK(ctx, hipMalloc(dst, bytes));
  HIPCHK(ctx, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return CTD_OK;
}

static bool surface_ok(const float *S, int ne, int nz) {
  for (int j = 0; j < ne; ++j) {
    const float *r = S + (size_t)j * nz;
    for (int i = 0; i < nz; ++i) {
      if (!(r[i] >= -1.0f && r[i] <= 1.0f)) return false;
      if (i > 0 && r[i] < r[i - 1]) return false;
    }
  }
  return true;
}

// [ns][ne][nz] rows -> [ns][ne-1][nz-1] bilinear cells
static std::vector<float4> quad_cells(const float *S, int ns, int ne, int nz) {
  std::vector<float4> q((size_t)ns * (ne - 1) * (nz - 1));
  for (int s = 0; s < ns; ++s)
    for (int j = 0; j + 1 < ne; ++j) {
      const float *r0 = S + ((size_t)s * ne + j) * nz;
      const float *r1 = r0 + nz;
      for (int i = 0; i + 1 < nz; ++i)
        q[((size_t)s * (ne - 1) + j) * (nz - 1) + i] =
            make_float4(r0[i], r0[i + 1], r1[i], r1[i + 1]);
    }
  return q;
}

extern "C" int32_t ctd_materials_load(ctd_ctx *ctx, const ctd_egrid *eg, int32_t M,
                                      const float *mu_rho, const float *comp,
                                      int32_t comp_per_mat, int32_t n_zeta_c, const float *rayl,
                                      int32_t n_zeta_r, ctd_matset **out) {
  if (!ctx || !out) return CTD_EINVAL;
  *out = nullptr;
  NEED(ctx, eg && mu_rho && comp, "null argument");
  NEED(ctx, M >= 1 && M <= 255, "1 <= M <= 255 materials");
  NEED(ctx, eg->ne >= 2 && eg->de > 0 && std::isfinite(eg->e0), "bad energy grid");
  NEED(ctx, n_zeta_c >= 2 && (!rayl || n_zeta_r >= 2), "surfaces need >= 2 zeta nodes");
  const int ne = eg->ne;
  for (size_t i = 0; i < (size_t)M * ne * 3; ++i)
    NEED(ctx, mu_rho[i] >= 0.0f && std::isfinite(mu_rho[i]),
         "attenuation coefficient %zu is negative or not finite", i);
  const int ncomp = comp_per_mat ? M : 1;
  NEED(ctx, surface_ok(comp, ncomp * ne, n_zeta_c),
       "Compton surface leaves [-1,1] or decreases in zeta");
  if (rayl)
    NEED(ctx, surface_ok(rayl, M * ne, n_zeta_r),
         "Rayleigh surface leaves [-1,1] or decreases in zeta");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctd_matset *ms = new (std::nothrow) ctd_matset();
  if (!ms) return CTD_ENOMEM;
  ms->device = ctx->device;
  ms->eg = *eg;
  ms->M = M;
  ms->ncomp = ncomp;
  ms->nzc = n_zeta_c;
  ms->nzr = rayl ? n_zeta_r : 0;
  ms->mu_rho.assign(mu_rho, mu_rho + (size_t)M * ne * 3);
  std::vector<float4> mu4((size_t)M * ne);
  for (size_t i = 0; i < mu4.size(); ++i)
    mu4[i] = make_float4(mu_rho[3 * i], mu_rho[3 * i + 1], mu_rho[3 * i + 2], 0.0f);
  int rc = upload(ctx, (void **)&ms->d_mu, mu4.data(), sizeof(float4) * mu4.size());
  if (rc == CTD_OK) {
    auto q = quad_cells(comp, ncomp, ne, n_zeta_c);
    rc = upload(ctx, (void **)&ms->d_comp, q.data(), sizeof(float4) * q.size());
  }
  if (rc == CTD_OK && rayl) {
    auto q = quad_cells(rayl, M, ne, n_zeta_r);
    rc = upload(ctx, (void **)&ms->d_rayl, q.data(), sizeof(float4) * q.size());
  }
  if (rc != CTD_OK) {
    dfree(ms->d_mu);
    dfree(ms->d_comp);
    dfree(ms->d_rayl);
    delete ms;
    return rc;
  }
  *out = ms;
  return CTD_OK;
}

extern "C" int32_t ctd_materials_release(ctd_ctx *ctx, ctd_matset *ms) {
  if (!ctx || !ms) return CTD_EINVAL;
  if (ms->refs > 0) return set_err(ctx, CTD_EBUSY, "material set is used by %d case(s)", ms->refs.load());
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  dfree(ms->d_mu);
  dfree(ms->d_comp);
  dfree(ms->d_rayl);
  delete ms;
  return CTD_OK;
}

// ------------------------------------------------------ spectrum, geometry

extern "C" int32_t ctd_spectrum_set(ctd_ctx *ctx, int32_t nbins, const double *e_lo, double width,
                                    const double *weight, ctd_spectrum **out) {
  if (!ctx || !out) return CTD_EINVAL;
  *out = nullptr;
  NEED(ctx, nbins >= 1 && nbins <= 4096 && e_lo && weight, "1..4096 bins required");
  NEED(ctx, width >= 0.0 && std::isfinite(width), "bin width must be >= 0");
  double W = 0.0;
  for (int j = 0; j < nbins; ++j) {
    NEED(ctx, weight[j] >= 0.0 && std::isfinite(weight[j]), "weight %d is negative", j);
    NEED(ctx, e_lo[j] > 0.0 && std::isfinite(e_lo[j]), "bin energy %d must be positive", j);
    W += weight[j];
  }
  NEED(ctx, W > 0.0, "spectrum weights sum to zero");
  ctd_spectrum *sp = new (std::nothrow) ctd_spectrum();
  if (!sp) return CTD_ENOMEM;
  sp->lo.assign(e_lo, e_lo + nbins);
  sp->w.assign(weight, weight + nbins);
  sp->width = width;
  *out = sp;
  return CTD_OK;
}

extern "C" int32_t ctd_spectrum_release(ctd_ctx *ctx, ctd_spectrum *sp) {
  if (!ctx || !sp) return CTD_EINVAL;
  if (sp->refs > 0) return set_err(ctx, CTD_EBUSY, "spectrum is used by %d case(s)", sp->refs.load());
  delete sp;
  return CTD_OK;
}

extern "C" int32_t ctd_geometry_set(ctd_ctx *ctx, const ctd_geom *g, ctd_geometry **out) {
  if (!ctx || !out) return CTD_EINVAL;
  *out = nullptr;
  NEED(ctx, g, "null geometry");
  NEED(ctx, g->kind == CTD_GEOM_PENCIL || g->kind == CTD_GEOM_CONE, "unknown geometry kind");
  if (g->kind == CTD_GEOM_PENCIL) {
    const double n = std::sqrt(g->dir[0] * g->dir[0] + g->dir[1] * g->dir[1] +
                               g->dir[2] * g->dir[2]);
    NEED(ctx, n > 0 && std::isfinite(n), "pencil direction is zero");
  } else {
    NEED(ctx, g->sad > 0 && std::isfinite(g->sad), "sad must be positive");
    NEED(ctx, g->a1 > g->a0 && g->b1 > g->b0, "empty field rectangle");
    NEED(ctx, g->n_proj >= 0 && g->n_proj <= (1 << 20), "0 <= n_proj <= 2^20");
    NEED(ctx, std::isfinite(g->z_feed) && std::isfinite(g->arc_deg) &&
                  std::isfinite(g->phi0_deg), "non-finite trajectory parameter");
  }
  NEED(ctx, g->kind == CTD_GEOM_CONE || g->fluence == nullptr,
       "a fluence map needs the cone source");
  const bool has_map = g->fluence != nullptr;
  if (has_map) {
    NEED(ctx, g->fluence_na > 0 && g->fluence_nb > 0 &&
                  (int64_t)g->fluence_na * g->fluence_nb <= (1 << 24),
         "fluence map needs 1 <= na*nb <= 2^24 beamlets");
    NEED(ctx, g->fluence_chains >= 0 && g->fluence_chains <= (1 << 24),
         "0 <= fluence_chains <= 2^24");
  } else {
    NEED(ctx, g->fluence_chains == 0, "fluence_chains without a fluence map");
  }
  std::vector<double> cdf;
  if (has_map) {
    // running sums in beamlet order, FP64 (Sec. 2.2.4: P(I) = f_I / sum f)
    const int64_t n = (int64_t)g->fluence_na * g->fluence_nb;
    cdf.resize((size_t)n);
    double run = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const float f = g->fluence[i];
      NEED(ctx, std::isfinite(f) && f >= 0.0f, "fluence[%lld] = %g is not a finite value >= 0",
           (long long)i, (double)f);
      NEED(ctx, g->fluence_chains == 0 || f > 0.0f,
           "Metropolis-Hastings sampling needs f_I > 0 (fluence[%lld] = 0)", (long long)i);
      run += (double)f;
      cdf[(size_t)i] = run;
    }
    NEED(ctx, run > 0.0, "fluence map sums to zero");
  }
  ctd_geometry *geo = new (std::nothrow) ctd_geometry();
  if (!geo) return CTD_ENOMEM;
  geo->g = *g;
  geo->g.fluence = nullptr;   // the caller's buffer is not kept
  if (has_map) {
    // guide table over 2^gbits >= N equal slices of [0, F): entry k is the
    // first beamlet whose running sum exceeds (k / 2^gbits) F, a lower bound
    // of the answer for every u in slice k since k / 2^gbits <= u exactly.
    const int64_t n = (int64_t)cdf.size();
    int gbits = 0;
    while ((int64_t(1) << gbits) < n) ++gbits;
    const int64_t G = int64_t(1) << gbits;
    const double F = cdf.back();
    geo->fl_guide.resize((size_t)G);
    int64_t I = 0;
    for (int64_t k = 0; k < G; ++k) {
      const double t = ((double)k / (double)G) * F;
      while (I < n - 1 && cdf[(size_t)I] <= t) ++I;
      geo->fl_guide[(size_t)k] = (int32_t)I;
    }
    geo->fl_gbits = gbits;
    geo->fl_cdf = std::move(cdf);
    if (g->fluence_chains > 0) geo->fl_f.assign(g->fluence, g->fluence + n);
  }
  if (g->kind == CTD_GEOM_CONE && g->n_proj > 0) {
    geo->proj_sc.resize((size_t)g->n_proj);
    const double d2r = 0.017453292519943295769236907684886;
    for (int p = 0; p < g->n_proj; ++p) {
      const double turn_deg = (double)p * g->arc_deg / (double)g->n_proj;
      const double phi = (g->phi0_deg + turn_deg) * d2r;
      geo->proj_sc[p] = make_float4((float)std::sin(phi), (float)std::cos(phi),
                                    (float)(g->z_feed * turn_deg / 360.0), 0.0f);
    }
  }
  *out = geo;
  return CTD_OK;
}

extern "C" int32_t ctd_geometry_release(ctd_ctx *ctx, ctd_geometry *geo) {
  if (!ctx || !geo) return CTD_EINVAL;
  if (geo->refs > 0) return set_err(ctx, CTD_EBUSY, "geometry is used by %d case(s)", geo->refs.load());
  delete geo;
  return CTD_OK;
}

// ------------------------------------------------------------------ cases

static double e_max_of(const ctd_spectrum *sp) {
  double m = 0.0;
  for (double lo : sp->lo) m = std::max(m, lo + sp->width);
  return m;
}

// CTD_TRACK_AUTO: macro-cell majorants pay where one material's attenuation
// sets the global majorant well above that of the material filling most of
// the phantom (bone in tissue): at the spectrum's mean energy, the largest
// rho_max * mu/rho over the present materials against that of the most
// frequent material denser than 0.05 g/cm^3; MACRO above 1.5.  Depends on
// the inputs only, so a case's histories do not depend on the machine.
int ctd::auto_tracking(const ctd_phantom *ph, const ctd_matset *ms, const ctd_spectrum *sp,
                       bool rayleigh) {
  double wsum = 0.0, emean = 0.0;
  for (size_t i = 0; i < sp->lo.size(); ++i) {
    wsum += sp->w[i];
    emean += sp->w[i] * (sp->lo[i] + 0.5 * sp->width);
  }
  emean /= wsum;
  const ctd_egrid &eg = ms->eg;
  const int j = std::min(std::max((int)std::lround((emean - eg.e0) / eg.de), 0), eg.ne - 1);
  double top = 0.0, bulk = 0.0;
  uint32_t bulk_n = 0;
  for (int m = 0; m < ms->M; ++m) {
    if (!ph->present[m]) continue;
    const float *r = ms->mu_rho.data() + ((size_t)m * eg.ne + j) * 3;
    const double mu = ph->rho_max[m] * ((double)r[0] + r[1] + (rayleigh ? r[2] : 0.0f));
    top = std::max(top, mu);
    if (ph->rho_max[m] > 0.05 && ph->count[m] > bulk_n) {
      bulk_n = ph->count[m];
      bulk = mu;
    }
  }
  return bulk > 0.0 && top > 1.5 * bulk ? CTD_TRACK_MACRO : CTD_TRACK_GLOBAL;
}

int ctd::upload_desc(ctd_ctx *ctx, ctd_case *cs) {
  HIPCHK(ctx, hipMemcpyAsync(cs->d_desc, &cs->desc, sizeof(CaseDev), hipMemcpyHostToDevice,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return CTD_OK;
}

// Bound-test sums (CaseDev::bnd; ctd_bound.h).
static std::vector<float> bound_sums(const ctd_matset *ms, bool rayleigh) {
  std::vector<float> out((size_t)ms->M * (size_t)(ms->eg.ne - 1));
  ctd::bound_sums(ms->mu_rho.data(), ms->M, ms->eg.ne, rayleigh, out.data());
  return out;
}

// The bound test of a case is exact while every class level times its
// material's bound-test sum stays a normal float: only absurdly small
// densities and cross sections would leave that range.
static bool bound_test_in_range(const ctd_phantom *ph, const std::vector<float> &bnd, int ne) {
  for (const uint2 &c : ph->bclass_host) {
    float rho;
    std::memcpy(&rho, &c.x, 4);
    if (rho == 0.0f) continue;
    for (int j = 0; j + 1 < ne; ++j) {
      const double v = (double)rho * bnd[(size_t)c.y * (ne - 1) + j];
      if (v != 0.0 && v < 0x1p-100) return false;
    }
  }
  return true;
}

extern "C" int32_t ctd_case_create(ctd_ctx *ctx, ctd_phantom *ph, ctd_matset *ms,
                                   ctd_spectrum *sp, ctd_geometry *geo, const ctd_params *p,
                                   ctd_case **out) {
  if (!ctx || !out) return CTD_EINVAL;
  *out = nullptr;
  NEED(ctx, ph && ms && sp && geo && p, "null argument");
  NEED(ctx, p->n_batches >= 2, "n_batches must be >= 2");
  NEED(ctx, ph->device == ctx->device && ms->device == ctx->device,
       "phantom (device %d) and material set (device %d) must be on the context's device %d",
       ph->device, ms->device, ctx->device);
  NEED(ctx, ph->max_mat < ms->M, "phantom uses material %d but only %d are loaded", ph->max_mat,
       ms->M);
  const double emax = e_max_of(sp);
  const ctd_egrid &eg = ms->eg;
  const double etop = eg.e0 + (eg.ne - 1) * eg.de;
  NEED(ctx, p->e_cut_kev >= eg.e0 && p->e_cut_kev > 0.0, "e_cut %.6g below the energy grid",
       p->e_cut_kev);
  // Exact fixed point: a float32 energy >= 0.5 keV is a multiple of q =
  // 2^-24 keV.  Sources start at >= 1 keV and a Compton scatter keeps
  // E' > E/2, so a photon that scatters on (E' >= e_cut >= 1 keV) or is cut
  // off (E' > E/2 >= 0.5 keV) never carries a non-multiple of q.
  NEED(ctx, p->e_cut_kev >= 1.0, "e_cut %.6g keV: must be >= 1 keV (exact q = 2^-24 keV tally)",
       p->e_cut_kev);
  double emin = INFINITY;
  for (double lo : sp->lo) emin = std::min(emin, lo);
  NEED(ctx, emin >= 1.0,
       "spectrum starts at %.6g keV: every bin must start at >= 1 keV (exact q = 2^-24 keV "
       "tally)", emin);
  NEED(ctx, emax <= etop, "spectrum reaches %.6g keV beyond the energy grid (%.6g)", emax, etop);
  NEED(ctx, emax < 255.0, "spectrum energies must stay below 255 keV");
  NEED(ctx, !p->rayleigh || ms->d_rayl, "Rayleigh on but no Rayleigh surfaces loaded");
  NEED(ctx, p->tracking == CTD_TRACK_GLOBAL || p->tracking == CTD_TRACK_MACRO ||
                p->tracking == CTD_TRACK_AUTO,
       "unknown tracking mode %d", p->tracking);
  NEED(ctx, p->macro_cell >= 0 && p->macro_cell <= 64, "macro_cell must be 0..64");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  ctd_case *cs = new (std::nothrow) ctd_case();
  if (!cs) return CTD_ENOMEM;
  cs->ctx = ctx;
  cs->ph = ph;
  cs->ms = ms;
  cs->sp = sp;
  cs->geo = geo;
  cs->p = *p;
  if (p->tracking == CTD_TRACK_AUTO) cs->p.tracking = auto_tracking(ph, ms, sp, p->rayleigh != 0);
  cs->e_max = emax;
  cs->tune = default_tuning(ctx);
  // majorant from per-material maximum density (Sec. 2.1)
  std::vector<double> rmax((size_t)ms->M, 0.0);
  bool pres[256];
  for (int m = 0; m < ms->M; ++m) {
    rmax[m] = ph->rho_max[m];
    pres[m] = ph->present[m];
  }
  int rc = CTD_OK;
  cs->mu_max.resize((size_t)eg.ne);
  majorant_fp64(eg.ne, ms->M, ms->mu_rho.data(), rmax.data(), pres, p->rayleigh != 0,
                cs->mu_max.data());
  bool any = false;
  for (float v : cs->mu_max) any |= v > 0.0f;
  if (!any) {
    delete cs;
    return set_err(ctx, CTD_EINVAL, "majorant is zero: empty phantom");
  }
  const int64_t V = ph->V;
  auto cleanup = [&](int code) {
    free_case_buffers(cs);
    delete cs;
    return code;
  };
  hipError_t e;
  std::vector<float> blo(sp->lo.begin(), sp->lo.end());
  if ((e = hipMalloc(&cs->d_tally, 8 * V)) != hipSuccess ||
      (e = hipMalloc(&cs->d_s1, 8 * V)) != hipSuccess ||
      (e = hipMalloc(&cs->d_s2, 16 * V)) != hipSuccess ||
      (e = hipMalloc(&cs->d_acc, 8 * kAccWords)) != hipSuccess ||
      (e = hipMalloc(&cs->d_desc, sizeof(CaseDev))) != hipSuccess ||
      (e = hipMalloc(&cs->d_mu_max, 4 * eg.ne)) != hipSuccess ||
      (e = hipMalloc(&cs->d_bin_lo, 4 * blo.size())) != hipSuccess)
    return cleanup(hip_err(ctx, e, "case alloc"));
  {
    const std::vector<float> bnd = bound_sums(ms, p->rayleigh != 0);
    cs->use_bound_grid = ph->nclass > 0 && bound_test_in_range(ph, bnd, eg.ne);
    if ((e = hipMalloc(&cs->d_bnd, 4 * bnd.size())) != hipSuccess ||
        (e = hipMemcpy(cs->d_bnd, bnd.data(), 4 * bnd.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
      return cleanup(hip_err(ctx, e, "bound-test sums"));
  }
  if (!geo->proj_sc.empty() &&
      (e = hipMalloc(&cs->d_proj, sizeof(float4) * geo->proj_sc.size())) != hipSuccess)
    return cleanup(hip_err(ctx, e, "case alloc"));
  if (!geo->fl_cdf.empty() &&
      ((e = hipMalloc(&cs->d_fl_cdf, sizeof(double) * geo->fl_cdf.size())) != hipSuccess ||
       (e = hipMalloc(&cs->d_fl_guide, sizeof(int32_t) * geo->fl_guide.size())) != hipSuccess ||
       (e = hipMemcpy(cs->d_fl_cdf, geo->fl_cdf.data(), sizeof(double) * geo->fl_cdf.size(),
                      hipMemcpyHostToDevice)) != hipSuccess ||
       (e = hipMemcpy(cs->d_fl_guide, geo->fl_guide.data(),
                      sizeof(int32_t) * geo->fl_guide.size(), hipMemcpyHostToDevice)) !=
           hipSuccess))
    return cleanup(hip_err(ctx, e, "fluence map upload"));
  if (!geo->fl_f.empty() &&
      ((e = hipMalloc(&cs->d_fl_f, sizeof(float) * geo->fl_f.size())) != hipSuccess ||
       (e = hipMalloc(&cs->d_mh_state, sizeof(int32_t) * (size_t)geo->g.fluence_chains)) !=
           hipSuccess ||
       (e = hipMemcpy(cs->d_fl_f, geo->fl_f.data(), sizeof(float) * geo->fl_f.size(),
                      hipMemcpyHostToDevice)) != hipSuccess))
    return cleanup(hip_err(ctx, e, "fluence chain upload"));
  if ((e = hipMemcpy(cs->d_mu_max, cs->mu_max.data(), 4 * eg.ne, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(cs->d_bin_lo, blo.data(), 4 * blo.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (cs->d_proj && (e = hipMemcpy(cs->d_proj, geo->proj_sc.data(),
                                    sizeof(float4) * geo->proj_sc.size(),
                                    hipMemcpyHostToDevice)) != hipSuccess))
    return cleanup(hip_err(ctx, e, "case upload"));
  if (cs->p.tracking == CTD_TRACK_MACRO && (rc = build_macro(ctx, cs)) != CTD_OK)
    return cleanup(rc);
  if (launch_zero(cs->d_tally, 8 * V, ctx->stream) || launch_zero(cs->d_s1, 8 * V, ctx->stream) ||
      launch_zero(cs->d_s2, 16 * V, ctx->stream) ||
      launch_zero(cs->d_acc, 8 * kAccWords, ctx->stream))
    return cleanup(hip_err(ctx, hipGetLastError(), "case clear"));
  fill_desc(cs);
  if ((rc = upload_desc(ctx, cs)) != CTD_OK) return cleanup(rc);
  ph->refs++;
  ms->refs++;
  sp->refs++;
  geo->refs++;
  *out = cs;
  return CTD_OK;
}

void ctd::fill_desc(ctd_case *cs) {
  CaseDev &d = cs->desc;
  std::memset(&d, 0, sizeof d);
  const ctd_grid &g = cs->ph->g;
  d.nx = g.nx;
  d.ny = g.ny;
  d.nz = g.nz;
  d.nmat = cs->ms->M;
  d.fnx = (float)g.nx;
  d.fny = (float)g.ny;
  d.fnz = (float)g.nz;
  d.inv_dx = (float)(1.0 / g.dx);
  d.inv_dy = (float)(1.0 / g.dy);
  d.inv_dz = (float)(1.0 / g.dz);
  d.ox = (float)g.origin[0];
  d.oy = (float)g.origin[1];
  d.oz = (float)g.origin[2];
  d.vox = cs->ph->vox;
  d.V = cs->ph->V;
  d.vox8 = cs->ph->vox8;
  d.palette = cs->ph->palette;
  d.npal = cs->ph->npal;
  for (int s = 0; s < 3; ++s) d.bgrid[s] = cs->ph->bgrid[s];
  d.bclass = cs->use_bound_grid ? cs->ph->bclass : nullptr;
  d.bnd = cs->d_bnd;
  const ctd_matset *ms = cs->ms;
  d.ne = ms->eg.ne;
  d.nzc = ms->nzc;
  d.nzr = ms->nzr;
  d.rayleigh = cs->p.rayleigh ? 1 : 0;
  d.e0 = (float)ms->eg.e0;
  d.inv_de = (float)(1.0 / ms->eg.de);
  d.e_cut = (float)cs->p.e_cut_kev;
  d.mu_rho = ms->d_mu;
  d.mu_max = cs->d_mu_max;
  d.comp_quad = ms->d_comp;
  d.rayl_quad = ms->d_rayl;
  d.comp_per_mat = ms->ncomp > 1 ? 1 : 0;
  d.nbins = (int)cs->sp->lo.size();
  d.bin_width = (float)cs->sp->width;
  d.bin_lo = cs->d_bin_lo;
  const ctd_geom &G = cs->geo->g;
  d.kind = G.kind;
  d.nproj = G.kind == CTD_GEOM_CONE ? G.n_proj : 0;
  d.sad = (float)G.sad;
  if (G.kind == CTD_GEOM_PENCIL) {
    const double n = std::sqrt(G.dir[0] * G.dir[0] + G.dir[1] * G.dir[1] + G.dir[2] * G.dir[2]);
    for (int a = 0; a < 3; ++a) {
      d.src[a] = (float)G.src[a];
      d.dir[a] = (float)(G.dir[a] / n);
    }
  }
  for (int a = 0; a < 3; ++a) d.iso[a] = (float)G.iso[a];
  d.a0 = (float)G.a0;
  d.a1 = (float)G.a1;
  d.b0 = (float)G.b0;
  d.b1 = (float)G.b1;
  d.phi0_turns = (float)(G.phi0_deg / 360.0);
  d.arc_turns = (float)(G.arc_deg / 360.0);
  d.z_feed = (float)G.z_feed;
  d.proj_sc = cs->d_proj;
  const ctd_geometry *geo = cs->geo;
  d.fl_n = (int32_t)geo->fl_cdf.size();
  if (d.fl_n > 0) {
    d.fl_na = G.fluence_na;
    d.fl_gbits = geo->fl_gbits;
    d.fl_da = (float)((G.a1 - G.a0) / G.fluence_na);
    d.fl_db = (float)((G.b1 - G.b0) / G.fluence_nb);
    d.fl_total = geo->fl_cdf.back();
  }
  d.fl_cdf = cs->d_fl_cdf;
  d.fl_guide = cs->d_fl_guide;
  d.fl_chains = geo->fl_f.empty() ? 0 : G.fluence_chains;
  d.mc_cs = cs->mc_cs;
  d.mc_nx = cs->mc_n[0];
  d.mc_ny = cs->mc_n[1];
  d.mc_nz = cs->mc_n[2];
  d.mc_fcs = (float)cs->mc_cs;
  d.mc_inv_cs = cs->mc_cs ? 1.0f / (float)cs->mc_cs : 0.0f;
  d.mc_shift = cs->mc_shift;
  d.mc_ncell = cs->mc_n[0] * cs->mc_n[1] * cs->mc_n[2];
  d.mc_f = cs->d_mc_f;
  d.key0 = (uint32_t)cs->p.seed;
  d.key1 = (uint32_t)(cs->p.seed >> 32);
  d.tally = cs->d_tally;
  d.s1 = cs->d_s1;
  d.s2 = cs->d_s2;
  d.acc = cs->d_acc;
  d.log = cs->d_log;
  d.log_n = cs->d_log_n;
  d.log_h0 = cs->log_h0;
  d.log_h1 = cs->log_h1;
  d.log_cap = cs->log_cap;
}

void ctd::free_case_buffers(ctd_case *cs) {
  dfree(cs->d_tally);
  dfree(cs->d_s1);
  dfree(cs->d_s2);
  dfree(cs->d_acc);
  dfree(cs->d_desc);
  dfree(cs->d_mu_max);
  dfree(cs->d_bin_lo);
  dfree(cs->d_proj);
  dfree(cs->d_fl_cdf);
  dfree(cs->d_fl_guide);
  dfree(cs->d_fl_f);
  dfree(cs->d_mh_state);
  dfree(cs->d_mh_beam);
  dfree(cs->d_mc_f);
  dfree(cs->d_bnd);
  dfree(cs->d_log);
  dfree(cs->d_log_n);
  for (auto &t : cs->timing) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
    (void)hipEventDestroy(t.c);
  }
  cs->timing.clear();
}

extern "C" int32_t ctd_case_destroy(ctd_ctx *ctx, ctd_case *cs) {
  if (!ctx || !cs) return CTD_EINVAL;
  if (cs->in_server) return set_err(ctx, CTD_EBUSY, "case is queued in a server");
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_case_buffers(cs);
  cs->ph->refs--;
  cs->ms->refs--;
  cs->sp->refs--;
  cs->geo->refs--;
  delete cs;
  return CTD_OK;
}

extern "C" int32_t ctd_case_reset(ctd_ctx *ctx, ctd_case *cs) {
  if (!ctx || !cs) return CTD_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int64_t V = cs->ph->V;
  if (launch_zero(cs->d_tally, 8 * V * cs->tally_copies, ctx->stream) ||
      launch_zero(cs->d_s1, 8 * V, ctx->stream) || launch_zero(cs->d_s2, 16 * V, ctx->stream) ||
      launch_zero(cs->d_acc, 8 * kAccWords, ctx->stream))
    return hip_err(ctx, hipGetLastError(), "case reset");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  cs->h_next = 0;
  cs->batches = 0;
  cs->batch_min = UINT64_MAX;
  cs->batch_max = 0;
  cs->s1_bound = cs->s2_bound = 0.0;
  cs->sigma_local = cs->sigma_paper = NAN;
  for (auto &t : cs->timing) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
    (void)hipEventDestroy(t.c);
  }
  cs->timing.clear();
  cs->transport_ms = cs->fold_ms = 0.0;
  cs->failed = false;
  return CTD_OK;
}

ctd_tuning ctd::default_tuning(const ctd_ctx *ctx) {
  ctd_tuning t;
  t.block = 256;
  t.waves_per_simd = 5;  // the resident waves per SIMD of the 96-VGPR kernel
  t.refill_min = 16;
  t.chunk = 1024;
  t.tally_mode = 0;  // per-XCD copies measured no faster on MI355X; 8x the fold traffic
  t.bound_block = 2;
  t.defer_min = 16;
  (void)ctx;
  return t;
}

int ctd::step_kind(const ctd_case *cs, const ctd_tuning &t) {
  if (cs->mc_cs > 0) return kStepMacro;
  return cs->use_bound_grid && t.bound_block != 0 ? kStepDeferred : kStepPlain;
}

static bool tuning_ok(const ctd_tuning &t) {
  return (t.block == 64 || t.block == 128 || t.block == 256 || t.block == 512) &&
         t.waves_per_simd >= 1 && t.waves_per_simd <= 8 && t.refill_min >= 1 &&
         t.refill_min <= 64 && t.chunk >= 64 && t.chunk <= 65536 &&
         t.tally_mode >= 0 && t.tally_mode <= 2 &&
         (t.bound_block == 0 || t.bound_block == 1 || t.bound_block == 2 || t.bound_block == 4) &&
         t.defer_min >= 0 && t.defer_min <= 64;
}

int ctd::ensure_tally_copies(ctd_ctx *ctx, ctd_case *cs, int copies) {
  if (cs->tally_copies >= copies) return CTD_OK;
  const int64_t V = cs->ph->V;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  unsigned long long *t = nullptr;
  HIPCHK(ctx, hipMalloc(&t, 8 * V * copies));
  // batch tallies are zero between rounds: a fresh zeroed array replaces them
  if (launch_zero(t, 8 * V * copies, ctx->stream) != 0) {
    dfree(t);
    return hip_err(ctx, hipGetLastError(), "tally clear");
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  dfree(cs->d_tally);
  cs->d_tally = t;
  cs->tally_copies = copies;
  fill_desc(cs);
  return upload_desc(ctx, cs);
}

int ctd::ensure_mh_buffer(ctd_ctx *ctx, ctd_case *cs, uint64_t n) {
  if (cs->mh_cap >= n) return CTD_OK;
  // the buffer may still be read by an earlier round on the stream
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  dfree(cs->d_mh_beam);
  cs->d_mh_beam = nullptr;
  cs->mh_cap = 0;
  HIPCHK(ctx, hipMalloc(&cs->d_mh_beam, sizeof(int32_t) * n));
  cs->mh_cap = n;
  return CTD_OK;
}

uint64_t ctd::case_footprint(const ctd_grid &g, const ctd_geometry *geo, const ctd_params &p,
                             int ne, int tally_copies, uint64_t round_histories) {
  const uint64_t V = (uint64_t)g.nx * g.ny * g.nz;
  uint64_t b = V * (24 + 8 * (uint64_t)tally_copies) + 8 * kAccWords + sizeof(CaseDev) +
               sizeof(float4) * geo->proj_sc.size() + 65536 + 4 * 256 * (uint64_t)ne;
  if (p.tracking != CTD_TRACK_GLOBAL) {  // MACRO, or AUTO that may choose it
    int n[3];
    const uint64_t cells = (uint64_t)macro_cells(g, macro_edge(g, p.macro_cell), n);
    b += 4 * (uint64_t)kMacroBands * cells;
    (void)ne;
  }
  b += 8 * geo->fl_cdf.size() + 4 * geo->fl_guide.size();
  if (!geo->fl_f.empty())
    b += 4 * geo->fl_f.size() + 4 * (uint64_t)geo->g.fluence_chains + 4 * round_histories;
  return b;
}

extern "C" int32_t ctd_set_tuning(ctd_ctx *ctx, ctd_case *cs, const ctd_tuning *t) {
  if (!ctx || !cs || !t) return CTD_EINVAL;
  NEED(ctx, tuning_ok(*t), "tuning out of range");
  NEED(ctx, t->tally_mode == 0 || ctx->xcd_tally_ok,
       "per-XCD tallies unavailable: XCC id %u >= %d", ctx->max_xcc, kTallyCopies);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  NEED(ctx, transport_lds_fits(t->block, t->tally_mode, ctx->device),
       "tally_mode %d with %d-thread workgroups exceeds the LDS limit", t->tally_mode, t->block);
  if (t->tally_mode != 0) {
    int rc = ensure_tally_copies(ctx, cs, kTallyCopies);
    if (rc != CTD_OK) return rc;
  }
  cs->tune = *t;
  return CTD_OK;
}

extern "C" int32_t ctd_get_tuning(ctd_ctx *ctx, const ctd_case *cs, ctd_tuning *t) {
  if (!ctx || !cs || !t) return CTD_EINVAL;
  *t = cs->tune;
  return CTD_OK;
}

// ------------------------------------------------------------- launching

// Grid of the persistent transport kernel: waves_per_simd resident waves on
// each of the 4 SIMDs of every CU.
static LaunchCfg launch_cfg(const ctd_ctx *ctx, const ctd_tuning &t) {
  LaunchCfg cfg;
  cfg.block = t.block;
  cfg.grid = std::max(1, ctx->n_cu * 4 * t.waves_per_simd / (t.block / 64));
  cfg.refill_min = t.refill_min;
  cfg.chunk = t.chunk;
  cfg.tally_mode = t.tally_mode;
  cfg.bound_shift = t.bound_block == 1 ? 0 : t.bound_block == 2 ? 1 : t.bound_block == 4 ? 2 : -1;
  cfg.defer_min = t.defer_min;
  cfg.tab_n = 0;
  cfg.tab_ne = 0;
  // LDS per workgroup that keeps 4 x waves_per_simd waves resident per CU
  const int wgs_per_cu = std::max(1, 4 * t.waves_per_simd / (t.block / 64));
  cfg.lds_budget = (size_t)std::min(ctx->lds_per_block, ctx->lds_per_cu / wgs_per_cu);
  return cfg;
}

// Stage one round (RoundCase table, bin prefixes, chunk counter) through a
// pinned slot and launch the transport kernel on the ctx stream.
int ctd::submit_round(ctd_ctx *ctx, const std::vector<RoundItem> &items, const ctd_tuning &t,
                      bool with_log) {
  const int nrc = (int)items.size();
  if (nrc == 0) return CTD_OK;
  const int kind = items[0].step_kind;
  size_t bytes = sizeof(RoundCase) * nrc;
  std::vector<size_t> poff((size_t)nrc);
  for (int i = 0; i < nrc; ++i) {
    poff[i] = bytes;
    bytes += 8 * (items[i].prefix.size());
  }
  // one chunk counter per case
  const size_t ctr_off = (bytes + 255) & ~(size_t)255;
  const size_t ctr_bytes = (8 * (size_t)nrc + 255) & ~(size_t)255;
  bytes = ctr_off + ctr_bytes;
  ctd_ctx::Slot &s = ctx->slots[ctx->next_slot];
  ctx->next_slot = (ctx->next_slot + 1) % ctx->slots.size();
  if (s.ev) HIPCHK(ctx, hipEventSynchronize(s.ev));
  else HIPCHK(ctx, hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
  if (s.cap < bytes) {
    if (s.host) (void)hipHostFree(s.host);
    dfree(s.dev);
    s.host = nullptr;
    s.dev = nullptr;
    s.cap = 0;
    const size_t cap = std::max(bytes * 2, (size_t)65536);
    HIPCHK(ctx, hipHostMalloc(&s.host, cap, hipHostMallocDefault));
    HIPCHK(ctx, hipMalloc(&s.dev, cap));
    s.cap = cap;
  }
  char *h = (char *)s.host;
  char *d = (char *)s.dev;
  RoundCase *rc = (RoundCase *)h;
  LaunchCfg cfg = launch_cfg(ctx, t);
  uint64_t chunks = 0;
  for (int i = 0; i < nrc; ++i) {
    rc[i].cd = items[i].cd;
    rc[i].prefix = (const unsigned long long *)(d + poff[i]);
    rc[i].h_begin = items[i].h_begin;
    rc[i].n = items[i].n;
    rc[i].chunk_begin = chunks;
    rc[i].beamlets = items[i].beamlets;
    chunks += (items[i].n + (uint64_t)t.chunk - 1) / (uint64_t)t.chunk;
    std::memcpy(h + poff[i], items[i].prefix.data(), 8 * items[i].prefix.size());
  }
  home_round_cases(rc, nrc, cfg.grid, cfg.block / 64);
  std::memset(h + ctr_off, 0, ctr_bytes);
  HIPCHK(ctx, hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, ctx->stream));
  // LDS room for the largest case's tables: each workgroup stages the
  // tables of the case it works on
  for (const RoundItem &it : items) {
    cfg.tab_n = std::max(cfg.tab_n, it.tab_n);
    cfg.tab_ne = std::max(cfg.tab_ne, it.tab_ne);
  }
  if (chunks > 0 &&
      launch_transport((const RoundCase *)d, nrc, chunks, (unsigned long long *)(d + ctr_off),
                       cfg, with_log, kind, ctx->stream) != 0)
    return hip_err(ctx, hipGetLastError(), "transport launch");
  HIPCHK(ctx, hipEventRecord(s.ev, ctx->stream));
  return CTD_OK;
}

int ctd::batch_prefix(ctd_ctx *ctx, const ctd_case *cs, uint64_t n,
                      std::vector<unsigned long long> &prefix) {
  const int nb = (int)cs->sp->w.size();
  std::vector<uint64_t> cnt((size_t)nb);
  if (alloc_bins(n, nb, cs->sp->w.data(), cnt.data()) != CTD_OK)
    return set_err(ctx, CTD_EINVAL, "bin allocation failed");
  prefix.resize((size_t)nb + 1);
  prefix[0] = 0;
  for (int j = 0; j < nb; ++j) prefix[j + 1] = prefix[j] + cnt[j];
  return CTD_OK;
}

// Fixed-point headroom before a batch of n histories (ctd_headroom.h): the
// pessimistic bounds first, the exact maxima the folds recorded when those
// bounds get close to the int64 / 128-bit limits.
static int check_headroom(ctd_ctx *ctx, ctd_case *cs, uint64_t n) {
  double s1 = 0.0, s2 = 0.0;
  int v = headroom_bounds((double)n, cs->e_max, cs->s1_bound, cs->s2_bound, &s1, &s2);
  if (v == kHeadroomBatch)
    return set_err(ctx, CTD_EOVERFLOW, "a batch of %.3g histories at %.4g keV exceeds 2^62 q",
                   (double)n, cs->e_max);
  if (v == kHeadroomNeedExact) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long m[2];
    HIPCHK(ctx, hipMemcpy(m, cs->d_acc + kAccMaxS1, sizeof m, hipMemcpyDeviceToHost));
    if (headroom_exact((double)n, cs->e_max, m[0], m[1], &s1, &s2) != kHeadroomOk)
      return set_err(ctx, CTD_EOVERFLOW, "a voxel's fixed-point sums would overflow");
  }
  cs->s1_bound = s1;
  cs->s2_bound = s2;
  return CTD_OK;
}

// Add the elapsed times of a case's completed rounds to its totals and free
// their events; rounds still in flight stay queued.
static void harvest_timing(ctd_case *cs) {
  size_t done = 0;
  for (auto &t : cs->timing) {
    if (hipEventQuery(t.c) != hipSuccess) break;  // rounds complete in order
    float ms1 = 0.f, ms2 = 0.f;
    if (hipEventElapsedTime(&ms1, t.a, t.b) == hipSuccess) cs->transport_ms += ms1;
    if (hipEventElapsedTime(&ms2, t.b, t.c) == hipSuccess) cs->fold_ms += ms2;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
    (void)hipEventDestroy(t.c);
    ++done;
  }
  cs->timing.erase(cs->timing.begin(), cs->timing.begin() + (long)done);
}

// Enqueue one round over several cases (each with its own batch size), then
// fold every participating case.
int ctd::run_round(ctd_ctx *ctx, std::vector<ctd_case *> &cases, const std::vector<uint64_t> &n,
                   const ctd_tuning &t) {
  std::vector<RoundItem> items;
  bool with_log = false;
  for (size_t i = 0; i < cases.size(); ++i)
    if (n[i]) NEED_INTACT(ctx, cases[i]);
  for (size_t i = 0; i < cases.size(); ++i) {
    if (n[i] == 0) continue;
    int rc0 = check_headroom(ctx, cases[i], n[i]);
    if (rc0 != CTD_OK) return rc0;
    if (t.tally_mode != 0 && cases[i]->tally_copies < kTallyCopies) {
      rc0 = ensure_tally_copies(ctx, cases[i], kTallyCopies);
      if (rc0 != CTD_OK) return rc0;
    }
    RoundItem it;
    it.cd = cases[i]->d_desc;
    it.h_begin = cases[i]->h_next;
    it.n = n[i];
    it.step_kind = step_kind(cases[i], t);
    it.tab_n = cases[i]->ms->M * cases[i]->ms->eg.ne;
    it.tab_ne = cases[i]->ms->eg.ne;
    if (cases[i]->d_mh_state) {
      rc0 = ensure_mh_buffer(ctx, cases[i], n[i]);
      if (rc0 != CTD_OK) return rc0;
      it.beamlets = cases[i]->d_mh_beam;
    }
    int rc = batch_prefix(ctx, cases[i], n[i], it.prefix);
    if (rc != CTD_OK) return rc;
    items.push_back(std::move(it));
    with_log |= cases[i]->log_cap > 0;
  }
  if (items.empty()) return CTD_OK;
  ctd_case *first = cases[0];
  // the round's timing events; destroyed here unless the round completes
  struct TimingGuard {
    ctd_case::Timing tm{};
    bool keep = false;
    ~TimingGuard() {
      if (keep) return;
      for (hipEvent_t e : {tm.a, tm.b, tm.c})
        if (e) (void)hipEventDestroy(e);
    }
  } guard;
  ctd_case::Timing &tm = guard.tm;
  // from the first enqueue that changes a case on, a failure leaves the
  // round's cases part-way through it
  struct FailMark {
    const std::vector<ctd_case *> &cases;
    const std::vector<uint64_t> &n;
    bool armed = false;
    ~FailMark() {
      if (!armed) return;
      for (size_t i = 0; i < cases.size(); ++i)
        if (n[i]) cases[i]->failed = true;
    }
  } mark{cases, n};
  const bool timed = cases.size() == 1;
  if (timed) {
    HIPCHK(ctx, hipEventCreate(&tm.a));
    HIPCHK(ctx, hipEventCreate(&tm.b));
    HIPCHK(ctx, hipEventCreate(&tm.c));
    HIPCHK(ctx, hipEventRecord(tm.a, ctx->stream));
  }
  mark.armed = true;
  // Alg. A1 chains of this round's histories (same stream: ordered before the
  // transport that reads them and after the previous round's)
  for (size_t i = 0, k = 0; i < cases.size(); ++i) {
    if (n[i] == 0) continue;
    ctd_case *cs = cases[i];
    const RoundItem &it = items[k++];
    if (!it.beamlets) continue;
    if (launch_mh_fill(cs->d_fl_f, (int)cs->geo->fl_f.size(), cs->geo->g.fluence_chains,
                       it.h_begin, it.n, cs->desc.key0, cs->desc.key1, cs->d_mh_state,
                       cs->d_mh_beam, ctx->stream) != 0)
      return hip_err(ctx, hipGetLastError(), "Metropolis-Hastings fill launch");
  }
  int rc = CTD_OK;
  std::vector<RoundItem> group[3];
  for (auto &it : items) group[it.step_kind].push_back(std::move(it));
  for (int gi = 0; gi < 3 && rc == CTD_OK; ++gi) {
    if (group[gi].empty()) continue;
    rc = submit_round(ctx, group[gi], t, with_log);
    if (rc == CTD_OK && ctx->fail_next_round) {
      ctx->fail_next_round = false;
      rc = set_err(ctx, CTD_EDEVICE, "failure injected after a transport launch");
    }
  }
  if (rc != CTD_OK) return rc;
  if (timed) HIPCHK(ctx, hipEventRecord(tm.b, ctx->stream));
  for (size_t i = 0; i < cases.size(); ++i) {
    if (n[i] == 0) continue;
    ctd_case *cs = cases[i];
    if (launch_fold(cs->d_tally, t.tally_mode ? kTallyCopies : 1, cs->d_s1, cs->d_s2, cs->ph->V,
                    cs->d_acc, ctx->stream) != 0)
      return hip_err(ctx, hipGetLastError(), "fold launch");
    cs->h_next += n[i];
    cs->batches += 1;
    cs->batch_min = std::min(cs->batch_min, n[i]);
    cs->batch_max = std::max(cs->batch_max, n[i]);
  }
  if (timed) {
    HIPCHK(ctx, hipEventRecord(tm.c, ctx->stream));
    // a long run without a stats read keeps only the rounds still in flight
    if (first->timing.size() >= 64) harvest_timing(first);
    first->timing.push_back(tm);
    guard.keep = true;
  }
  mark.armed = false;
  return CTD_OK;
}

std::vector<uint64_t> ctd::split_batches(uint64_t n, int nb) {
  std::vector<uint64_t> v((size_t)nb, n / (uint64_t)nb);
  for (uint64_t b = 0; b < n % (uint64_t)nb; ++b) v[b] += 1;
  return v;
}

extern "C" int32_t ctd_run(ctd_ctx *ctx, ctd_case *cs, uint64_t n_histories) {
  if (!ctx || !cs) return CTD_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (n_histories == 0) return CTD_OK;
  const auto sizes = split_batches(n_histories, cs->p.n_batches);
  std::vector<ctd_case *> one{cs};
  int rc = CTD_OK;
  for (uint64_t nb : sizes) {
    if (nb == 0) continue;
    rc = run_round(ctx, one, std::vector<uint64_t>{nb}, cs->tune);
    if (rc != CTD_OK) return rc;
  }
  return CTD_OK;
}

extern "C" int32_t ctd_run_many(ctd_ctx *ctx, ctd_case *const *cs, const uint64_t *n,
                                int32_t count) {
  if (!ctx || !cs || !n || count < 1) return CTD_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<std::vector<uint64_t>> sizes((size_t)count);
  size_t rounds = 0;
  for (int i = 0; i < count; ++i) {
    NEED(ctx, cs[i], "null case %d", i);
    for (int j = 0; j < i; ++j) NEED(ctx, cs[j] != cs[i], "case %d listed twice", i);
    if (n[i]) sizes[i] = split_batches(n[i], cs[i]->p.n_batches);
    rounds = std::max(rounds, sizes[i].size());
  }
  const ctd_tuning t = cs[0]->tune;
  std::vector<ctd_case *> cases(cs, cs + count);
  for (size_t r = 0; r < rounds; ++r) {
    std::vector<uint64_t> nr((size_t)count, 0);
    for (int i = 0; i < count; ++i)
      if (r < sizes[i].size()) nr[i] = sizes[i][r];
    int rc = run_round(ctx, cases, nr, t);
    if (rc != CTD_OK) return rc;
  }
  return CTD_OK;
}

extern "C" int32_t ctd_sync(ctd_ctx *ctx, ctd_case *cs) {
  (void)cs;
  if (!ctx) return CTD_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return CTD_OK;
}

int ctd::check_batch_sizes(ctd_ctx *ctx, const ctd_case *cs, uint64_t next_size) {
  uint64_t lo = cs->batch_min, hi = cs->batch_max;
  if (next_size) {
    lo = std::min(lo, next_size);
    hi = std::max(hi, next_size);
  }
  if (hi > lo + 1)
    return set_err(ctx, CTD_EINVAL,
                   "batch statistics need equal batches: sizes %llu .. %llu histories",
                   (unsigned long long)lo, (unsigned long long)hi);
  return CTD_OK;
}

int ctd::sigma_async(ctd_ctx *ctx, ctd_case *cs, int kind, double frac, double *host_out) {
  NEED_INTACT(ctx, cs);
  if (cs->batches < 2) return set_err(ctx, CTD_EINVAL, "sigma needs >= 2 folded batches");
  int rc = check_batch_sizes(ctx, cs, 0);
  if (rc != CTD_OK) return rc;
  double rho_min = cs->p.sigma_rho_min;
  // the scratch is reused by the next reduction on the stream, which starts
  // after this one's results have been copied out
  double *out_dev = ctx->sigma_scratch + 3 * kSigmaBlocks;
  if (launch_sigma(cs->d_s1, cs->d_s2, cs->ph->vox, cs->ph->V, cs->batches, rho_min, frac, kind,
                   ctx->sigma_scratch, kSigmaBlocks, out_dev, ctx->stream) != 0)
    return hip_err(ctx, hipGetLastError(), "sigma launch");
  HIPCHK(ctx, hipMemcpyAsync(host_out, out_dev, 3 * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  return CTD_OK;
}

int ctd::sigma_now(ctd_ctx *ctx, ctd_case *cs, int kind, double frac, double *out) {
  int rc = sigma_async(ctx, cs, kind, frac, ctx->sigma_host);
  if (rc != CTD_OK) return rc;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *out = ctx->sigma_host[0];
  return CTD_OK;
}

extern "C" int32_t ctd_sigma(ctd_ctx *ctx, ctd_case *cs, int32_t sigma_kind, double dose_frac,
                             double *out) {
  if (!ctx || !cs || !out) return CTD_EINVAL;
  NEED(ctx, sigma_kind == CTD_SIGMA_LOCAL || sigma_kind == CTD_SIGMA_PAPER, "bad sigma kind");
  NEED(ctx, dose_frac >= 0.0 && dose_frac < 1.0, "dose_frac must be in [0,1)");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  return sigma_now(ctx, cs, sigma_kind, dose_frac, out);
}

// sigma ~ batches^-1/2 at a fixed batch size: aim 2 % past the target.  No
// dose in the region yet (sigma-bar infinite): run to the cap.
uint64_t ctd::sigma_plan(uint64_t have, double sig, double target, uint64_t max_batches) {
  if (sig <= target || have >= max_batches) return 0;
  const uint64_t room = max_batches - have;
  if (!(sig < INFINITY)) return room;
  const double want = std::ceil((double)have * (sig / target) * (sig / target) * 1.02);
  const double more = std::min(std::max(1.0, want - (double)have), (double)room);
  return (uint64_t)more;
}

int ctd::run_batches(ctd_ctx *ctx, ctd_case *cs, uint64_t batch, uint64_t count) {
  int rc = CTD_OK;
  std::vector<ctd_case *> one{cs};
  for (uint64_t b = 0; b < count; ++b) {
    rc = run_round(ctx, one, std::vector<uint64_t>{batch}, cs->tune);
    if (rc != CTD_OK) return rc;
  }
  return CTD_OK;
}

extern "C" int32_t ctd_run_batches(ctd_ctx *ctx, ctd_case *cs, uint64_t batch_histories,
                                   uint64_t count) {
  if (!ctx || !cs) return CTD_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (batch_histories == 0 || count == 0) return CTD_OK;
  return run_batches(ctx, cs, batch_histories, count);
}

extern "C" int32_t ctd_run_batches_static(ctd_ctx *ctx, ctd_case *cs, uint64_t batch_histories,
                                          uint64_t count) {
  if (!ctx || !cs) return CTD_EINVAL;
  NEED(ctx, ctx->static_table, "no static round table on device %d", ctx->device);
  const int nb = (int)cs->sp->w.size();
  NEED(ctx, nb <= kStaticMaxBins, "%d spectrum bins: the static round table holds at most %d",
       nb, kStaticMaxBins);
  const ctd_tuning &t = cs->tune;
  NEED(ctx, t.tally_mode == 0 || cs->tally_copies >= kTallyCopies,
       "tally mode %d without per-XCD tallies", t.tally_mode);
  NEED(ctx, !cs->d_mh_state || cs->mh_cap >= batch_histories,
       "Metropolis-Hastings beamlets for %llu histories; run ctd_run_batches once with batches "
       "of %llu histories first", (unsigned long long)cs->mh_cap,
       (unsigned long long)batch_histories);
  NEED_INTACT(ctx, cs);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (batch_histories == 0 || count == 0) return CTD_OK;
  StaticRoundArgs a;
  std::memset(&a, 0, sizeof a);
  a.cd = cs->d_desc;
  a.beamlets = cs->d_mh_state ? cs->d_mh_beam : nullptr;
  a.nbins = nb;
  uint64_t cnt[kStaticMaxBins];
  if (alloc_bins(batch_histories, nb, cs->sp->w.data(), cnt) != CTD_OK)
    return set_err(ctx, CTD_EINVAL, "bin allocation failed");
  for (int j = 0; j < nb; ++j) a.prefix[j + 1] = a.prefix[j] + cnt[j];
  LaunchCfg cfg = launch_cfg(ctx, t);
  cfg.tab_n = cs->ms->M * cs->ms->eg.ne;
  cfg.tab_ne = cs->ms->eg.ne;
  a.home_waves = (uint32_t)cfg.grid * (uint32_t)(cfg.block / 64);
  const uint64_t chunks = (batch_histories + (uint64_t)t.chunk - 1) / (uint64_t)t.chunk;
  unsigned char *table = (unsigned char *)ctx->static_table;
  const bool with_log = cs->log_cap > 0;
  for (uint64_t b = 0; b < count; ++b) {
    double s1 = 0.0, s2 = 0.0;
    const int v = headroom_bounds((double)batch_histories, cs->e_max, cs->s1_bound,
                                  cs->s2_bound, &s1, &s2);
    if (v != kHeadroomOk)
      return set_err(ctx, CTD_EOVERFLOW,
                     v == kHeadroomBatch
                         ? "a batch of %.3g histories exceeds 2^62 q"
                         : "the fixed-point bounds after %.3g more histories need the exact "
                           "maxima, which only ctd_run_batches reads back",
                     (double)batch_histories);
    a.h_begin = cs->h_next;
    a.n = batch_histories;
    // from here on a failure leaves the case part-way through a batch
    cs->failed = true;
    if (a.beamlets &&
        launch_mh_fill(cs->d_fl_f, (int)cs->geo->fl_f.size(), cs->geo->g.fluence_chains,
                       a.h_begin, a.n, cs->desc.key0, cs->desc.key1, cs->d_mh_state,
                       cs->d_mh_beam, ctx->stream) != 0)
      return hip_err(ctx, hipGetLastError(), "Metropolis-Hastings fill launch");
    if (launch_static_round_setup(table, a, ctx->stream) != 0 ||
        launch_transport((const RoundCase *)table, 1, chunks,
                         (unsigned long long *)(table + kStaticCounterOff), cfg, with_log,
                         step_kind(cs, t), ctx->stream) != 0 ||
        launch_fold(cs->d_tally, t.tally_mode ? kTallyCopies : 1, cs->d_s1, cs->d_s2,
                    cs->ph->V, cs->d_acc, ctx->stream) != 0)
      return hip_err(ctx, hipGetLastError(), "static round launch");
    cs->failed = false;
    cs->s1_bound = s1;
    cs->s2_bound = s2;
    cs->h_next += batch_histories;
    cs->batches += 1;
    cs->batch_min = std::min(cs->batch_min, batch_histories);
    cs->batch_max = std::max(cs->batch_max, batch_histories);
  }
  return CTD_OK;
}

extern "C" int32_t ctd_run_to_sigma(ctd_ctx *ctx, ctd_case *cs, double target, double dose_frac,
                                    int32_t sigma_kind, uint64_t batch_histories,
                                    uint64_t max_histories, double *achieved) {
  if (!ctx || !cs) return CTD_EINVAL;
  NEED(ctx, target > 0.0, "target must be positive");
  NEED(ctx, batch_histories > 0, "batch_histories must be positive");
  NEED(ctx, sigma_kind == CTD_SIGMA_LOCAL || sigma_kind == CTD_SIGMA_PAPER, "bad sigma kind");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int rc = check_batch_sizes(ctx, cs, batch_histories);
  if (rc != CTD_OK) return rc;
  const uint64_t max_b = std::max<uint64_t>(max_histories / batch_histories, 2);
  uint64_t have = cs->batches;
  const uint64_t pilot = (uint64_t)cs->p.n_batches;
  if (have < pilot) {
    rc = run_batches(ctx, cs, batch_histories, std::min(pilot - have, max_b - std::min(max_b, have)));
    if (rc != CTD_OK) return rc;
  }
  double sig = INFINITY;
  for (;;) {
    rc = sigma_now(ctx, cs, sigma_kind, dose_frac, &sig);
    if (rc != CTD_OK) return rc;
    const uint64_t more = sigma_plan(cs->batches, sig, target, max_b);
    if (more == 0) break;
    rc = run_batches(ctx, cs, batch_histories, more);
    if (rc != CTD_OK) return rc;
  }
  if (sigma_kind == CTD_SIGMA_LOCAL) cs->sigma_local = sig; else cs->sigma_paper = sig;
  if (achieved) *achieved = sig;
  return CTD_OK;
}

// ---------------------------------------------------------------- readout

extern "C" int32_t ctd_tally_device(ctd_ctx *ctx, ctd_case *cs, void **s1, void **s2) {
  if (!ctx || !cs) return CTD_EINVAL;
  NEED_INTACT(ctx, cs);
  if (s1) *s1 = cs->d_s1;
  if (s2) *s2 = cs->d_s2;
  return CTD_OK;
}

extern "C" int32_t ctd_read_tally(ctd_ctx *ctx, ctd_case *cs, int64_t *s1, uint64_t *s2_hi,
                                  uint64_t *s2_lo, uint32_t *n_batches) {
  if (!ctx || !cs) return CTD_EINVAL;
  NEED_INTACT(ctx, cs);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t V = cs->ph->V;
  if (s1) HIPCHK(ctx, hipMemcpy(s1, cs->d_s1, 8 * V, hipMemcpyDeviceToHost));
  if (s2_hi || s2_lo) {
    std::vector<uint64_t> s2((size_t)V * 2);
    HIPCHK(ctx, hipMemcpy(s2.data(), cs->d_s2, 16 * V, hipMemcpyDeviceToHost));
    for (int64_t v = 0; v < V; ++v) {
      if (s2_lo) s2_lo[v] = s2[2 * v];
      if (s2_hi) s2_hi[v] = s2[2 * v + 1];
    }
  }
  if (n_batches) *n_batches = cs->batches;
  return CTD_OK;
}

// (nb*S2 - S1^2) exactly in 192-bit unsigned arithmetic, returned as double.
static double var_numerator(int64_t s1, uint64_t hi, uint64_t lo, uint32_t nb) {
  const unsigned __int128 plo = (unsigned __int128)lo * nb;
  const unsigned __int128 pmid = (unsigned __int128)hi * nb + (uint64_t)(plo >> 64);
  const uint64_t a0 = (uint64_t)plo, a1 = (uint64_t)pmid, a2 = (uint64_t)(pmid >> 64);
  const unsigned __int128 B = (unsigned __int128)(uint64_t)s1 * (uint64_t)s1;
  const uint64_t b0 = (uint64_t)B, b1 = (uint64_t)(B >> 64);
  const uint64_t r0 = a0 - b0;
  const uint64_t br0 = a0 < b0 ? 1 : 0;
  const uint64_t r1 = a1 - b1 - br0;
  const uint64_t br1 = (a1 < b1 || (a1 - b1) < br0) ? 1 : 0;
  if (a2 < br1) return 0.0;  // cannot happen for consistent sums
  const uint64_t r2 = a2 - br1;
  return (double)r2 * 0x1p128 + (double)r1 * 0x1p64 + (double)r0;
}

extern "C" int32_t ctd_read_dose(ctd_ctx *ctx, ctd_case *cs, double *dose, double *var_of_mean) {
  if (!ctx || !cs) return CTD_EINVAL;
  NEED(ctx, cs->batches >= 2, "dose needs >= 2 folded batches");
  if (int rc0 = check_batch_sizes(ctx, cs, 0); rc0 != CTD_OK) return rc0;
  const int64_t V = cs->ph->V;
  std::vector<int64_t> s1((size_t)V);
  std::vector<uint64_t> hi((size_t)V), lo((size_t)V);
  uint32_t nb = 0;
  int rc = ctd_read_tally(ctx, cs, s1.data(), hi.data(), lo.data(), &nb);
  if (rc != CTD_OK) return rc;
  std::vector<uint2> rec((size_t)V);
  HIPCHK(ctx, hipMemcpy(rec.data(), cs->ph->vox, 8 * V, hipMemcpyDeviceToHost));
  const ctd_grid &g = cs->ph->g;
  const double vol = g.dx * g.dy * g.dz;
  const double N = (double)cs->h_next;
  const double per_batch = N / (double)nb;
  for (int64_t v = 0; v < V; ++v) {
    float r;
    std::memcpy(&r, &rec[v].x, 4);
    const double mass_kg = (double)r * vol * 1e-3;
    if (!(mass_kg > 0.0)) {
      if (dose) dose[v] = 0.0;
      if (var_of_mean) var_of_mean[v] = 0.0;
      continue;
    }
    const double conv = 1.602176634e-16 / (16777216.0 * mass_kg);  // q -> Gy
    if (dose) dose[v] = (double)s1[v] / N * conv;
    if (var_of_mean) {
      const double num = var_numerator(s1[v], hi[v], lo[v], nb);
      const double var_t = num / ((double)nb * nb * (double)(nb - 1));
      var_of_mean[v] = var_t / (per_batch * per_batch) * conv * conv;
    }
  }
  return CTD_OK;
}

extern "C" int32_t ctd_read_balance(ctd_ctx *ctx, ctd_case *cs, ctd_balance *out) {
  if (!ctx || !cs || !out) return CTD_EINVAL;
  NEED_INTACT(ctx, cs);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  uint64_t w[kAccWords];
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(w, cs->d_acc, sizeof w, hipMemcpyDeviceToHost));
  uint64_t a[ACC_COUNT];
  for (int i = 0; i < ACC_COUNT; ++i) a[i] = w[kAccTotal + 2 * i];
  out->q_incident = a[ACC_Q_INC];
  out->q_deposited = a[ACC_Q_DEP];
  out->q_escaped = a[ACC_Q_ESC];
  out->q_incident_hi = w[kAccTotal + 2 * ACC_Q_INC + 1];
  out->q_deposited_hi = w[kAccTotal + 2 * ACC_Q_DEP + 1];
  out->q_escaped_hi = w[kAccTotal + 2 * ACC_Q_ESC + 1];
  out->n_histories = a[ACC_N_HIST];
  out->n_missed = a[ACC_N_MISS];
  out->n_unscattered = a[ACC_N_UNSCATTERED];
  out->n_cutoff = a[ACC_N_CUTOFF];
  if (a[ACC_STEP_GUARD])
    return set_err(ctx, CTD_ESTEPS, "%llu histories hit the step guard",
                   (unsigned long long)a[ACC_STEP_GUARD]);
  return CTD_OK;
}

extern "C" int32_t ctd_read_stats(ctd_ctx *ctx, ctd_case *cs, ctd_stats *out) {
  if (!ctx || !cs || !out) return CTD_EINVAL;
  NEED_INTACT(ctx, cs);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  uint64_t w[kAccWords];
  HIPCHK(ctx, hipMemcpy(w, cs->d_acc, sizeof w, hipMemcpyDeviceToHost));
  uint64_t a[ACC_COUNT];
  for (int i = 0; i < ACC_COUNT; ++i) a[i] = w[kAccTotal + 2 * i];
  harvest_timing(cs);
  if (cs->batches >= 2) {
    double s;
    if (sigma_now(ctx, cs, CTD_SIGMA_LOCAL, 0.5, &s) == CTD_OK) cs->sigma_local = s;
    if (sigma_now(ctx, cs, CTD_SIGMA_PAPER, 0.2, &s) == CTD_OK) cs->sigma_paper = s;
  }
  out->sigma_local = cs->sigma_local;
  out->sigma_paper = cs->sigma_paper;
  // the step counter holds, per finished history, the random pairs it took
  // (global majorant: one per step and one per scatter) or its flights (MACRO)
  out->n_steps = cs->mc_cs > 0 ? a[ACC_N_STEPS]
                               : a[ACC_N_STEPS] - a[ACC_N_COMPTON] - a[ACC_N_RAYLEIGH];
  out->n_photo = a[ACC_N_PHOTO];
  out->n_compton = a[ACC_N_COMPTON];
  out->n_rayleigh = a[ACC_N_RAYLEIGH];
  out->n_real = a[ACC_N_PHOTO] + a[ACC_N_COMPTON] + a[ACC_N_RAYLEIGH];
  out->n_deposits = a[ACC_N_DEPOSITS];
  out->n_escapes = a[ACC_N_ESCAPES];
  out->n_refills = a[ACC_N_REFILLS];
  out->transport_ms = cs->transport_ms;
  out->fold_ms = cs->fold_ms;
  out->n_batches = cs->batches;
  out->tracking = cs->mc_cs > 0 ? CTD_TRACK_MACRO : CTD_TRACK_GLOBAL;
  out->n_histories = cs->h_next;
  out->n_crossings = a[ACC_N_CROSS];
  out->max_s1 = w[kAccMaxS1];
  out->max_s2_hi = w[kAccMaxS2Hi];
  return CTD_OK;
}

extern "C" int32_t ctd_read_majorant(ctd_ctx *ctx, ctd_case *cs, float *out) {
  if (!ctx || !cs || !out) return CTD_EINVAL;
  std::memcpy(out, cs->mu_max.data(), 4 * cs->mu_max.size());
  return CTD_OK;
}

// -------------------------------------------------------------- debug log

extern "C" int32_t ctd_debug_deposit_log(ctd_ctx *ctx, ctd_case *cs, uint64_t h0, uint64_t nh,
                                         uint64_t capacity) {
  if (!ctx || !cs) return CTD_EINVAL;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  dfree(cs->d_log);
  dfree(cs->d_log_n);
  cs->d_log = nullptr;
  cs->d_log_n = nullptr;
  cs->log_cap = 0;
  cs->log_h0 = cs->log_h1 = 0;
  if (capacity > 0 && nh > 0) {
    HIPCHK(ctx, hipMalloc(&cs->d_log, sizeof(ctd_event) * capacity));
    HIPCHK(ctx, hipMalloc(&cs->d_log_n, 256));
    HIPCHK(ctx, hipMemset(cs->d_log_n, 0, 256));
    cs->log_cap = capacity;
    cs->log_h0 = h0;
    cs->log_h1 = h0 + nh;
  }
  fill_desc(cs);
  return upload_desc(ctx, cs);
}

extern "C" int32_t ctd_debug_fail_next_round(ctd_ctx *ctx) {
  if (!ctx) return CTD_EINVAL;
  ctx->fail_next_round = true;
  return CTD_OK;
}

extern "C" int32_t ctd_read_event_log(ctd_ctx *ctx, ctd_case *cs, ctd_event *out,
                                      uint64_t capacity, uint64_t *n) {
  if (!ctx || !cs || !n) return CTD_EINVAL;
  NEED_INTACT(ctx, cs);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *n = 0;
  if (!cs->d_log_n) return CTD_OK;
  unsigned long long cnt = 0;
  HIPCHK(ctx, hipMemcpy(&cnt, cs->d_log_n, 8, hipMemcpyDeviceToHost));
  *n = cnt;
  const uint64_t k = std::min<uint64_t>({cnt, capacity, cs->log_cap});
  if (k && out) HIPCHK(ctx, hipMemcpy(out, cs->d_log, sizeof(ctd_event) * k, hipMemcpyDeviceToHost));
  return CTD_OK;
}

// ------------------------------------------------------------------ tuner

extern "C" int32_t ctd_autotune(ctd_ctx *ctx, ctd_case *cs, uint64_t trial_histories,
                                ctd_tuning *best) {
  if (!ctx || !cs) return CTD_EINVAL;
  NEED(ctx, trial_histories > 0, "trial_histories must be positive");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  // scratch twin of the case: same inputs, private tallies
  ctd_case tw = *cs;
  tw.timing.clear();
  tw.d_tally = nullptr;
  tw.d_s1 = nullptr;
  tw.d_s2 = nullptr;
  tw.d_acc = nullptr;
  tw.d_desc = nullptr;
  tw.d_log = nullptr;
  tw.d_log_n = nullptr;
  tw.log_cap = 0;
  // the twin starts at history 0 with chains and buffers of its own (the
  // case's Metropolis-Hastings chains must only advance with its own runs)
  tw.h_next = 0;
  tw.batches = 0;
  tw.batch_min = UINT64_MAX;
  tw.batch_max = 0;
  tw.d_mh_state = nullptr;
  tw.d_mh_beam = nullptr;
  tw.mh_cap = 0;
  tw.failed = false;
  const int64_t V = cs->ph->V;
  auto release = [&]() {
    dfree(tw.d_tally);
    dfree(tw.d_s1);
    dfree(tw.d_s2);
    dfree(tw.d_acc);
    dfree(tw.d_desc);
    dfree(tw.d_mh_state);
    dfree(tw.d_mh_beam);
  };
  hipError_t e;
  tw.tally_copies = kTallyCopies;
  if (cs->d_mh_state &&
      (e = hipMalloc(&tw.d_mh_state, sizeof(int32_t) * (size_t)cs->geo->g.fluence_chains)) !=
          hipSuccess) {
    release();
    return hip_err(ctx, e, "autotune alloc");
  }
  if ((e = hipMalloc(&tw.d_tally, 8 * V * kTallyCopies)) != hipSuccess ||
      (e = hipMalloc(&tw.d_s1, 8 * V)) != hipSuccess ||
      (e = hipMalloc(&tw.d_s2, 16 * V)) != hipSuccess ||
      (e = hipMalloc(&tw.d_acc, 8 * kAccWords)) != hipSuccess ||
      (e = hipMalloc(&tw.d_desc, sizeof(CaseDev))) != hipSuccess) {
    release();
    return hip_err(ctx, e, "autotune alloc");
  }
  launch_zero(tw.d_tally, 8 * V * kTallyCopies, ctx->stream);
  launch_zero(tw.d_s1, 8 * V, ctx->stream);
  launch_zero(tw.d_s2, 16 * V, ctx->stream);
  launch_zero(tw.d_acc, 8 * kAccWords, ctx->stream);
  tw.s1_bound = tw.s2_bound = 0.0;
  fill_desc(&tw);
  int rc = upload_desc(ctx, &tw);
  if (rc != CTD_OK) {
    release();
    return rc;
  }
  // stage 1: launch shape and tally mode with the default bound grid; stage
  // 2 (below): the bound grid's block size for the best of stage 1
  const bool bounded = cs->ph->nclass > 0 && cs->mc_cs == 0;
  const int bb0 = bounded ? default_tuning(ctx).bound_block : 0;
  const int dm0 = default_tuning(ctx).defer_min;
  std::vector<ctd_tuning> cand;
  for (int tm = ctx->xcd_tally_ok ? 2 : 0; tm >= 0; --tm) {
    if (!transport_lds_fits(256, tm, ctx->device)) continue;
    for (int wps : {2, 4, 5, 8})  // 5: the resident waves per SIMD
      for (int rm : {8, 16, 32})
        for (int ch : {256, 1024}) {
          ctd_tuning t;
          t.block = 256;
          t.waves_per_simd = wps;
          t.refill_min = rm;
          t.chunk = ch;
          t.tally_mode = tm;
          t.bound_block = bb0;
          t.defer_min = dm0;
          cand.push_back(t);
        }
  }
  const size_t stage1 = cand.size();
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  double best_ms = INFINITY;
  ctd_tuning best_t = cs->tune;
  std::vector<ctd_case *> one{&tw};
  for (size_t i = 0;; ++i) {
    // stage 2: the bound grid's block size, then the collision deferral, each
    // varied around the best so far
    if (i == stage1 + 1 && bounded) {
      for (int bb : {0, 1, 2, 4}) {
        if (bb == best_t.bound_block) continue;
        ctd_tuning t = best_t;
        t.bound_block = bb;
        cand.push_back(t);
      }
    }
    if (i == stage1 + 4 && bounded && best_t.bound_block > 0) {
      for (int dm : {0, 8, 16, 32}) {
        if (dm == best_t.defer_min) continue;
        ctd_tuning t = best_t;
        t.defer_min = dm;
        cand.push_back(t);
      }
    }
    if (i > cand.size()) break;
    const ctd_tuning t = i == 0 ? cand[0] : cand[i - 1];  // first run warms up
    (void)hipEventRecord(a, ctx->stream);
    rc = run_round(ctx, one, std::vector<uint64_t>{trial_histories}, t);
    if (rc != CTD_OK) break;
    (void)hipEventRecord(b, ctx->stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (i > 0 && ms < best_ms) {
      best_ms = ms;
      best_t = t;
    }
  }
  for (auto &t : tw.timing) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
    (void)hipEventDestroy(t.c);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(ctx->stream);
  release();
  if (rc != CTD_OK) return rc;
  if (best_t.tally_mode != 0 && (rc = ensure_tally_copies(ctx, cs, kTallyCopies)) != CTD_OK)
    return rc;
  cs->tune = best_t;
  if (best) *best = best_t;
  return CTD_OK;
}

// -------------------------------------------------------- microbenchmarks

extern "C" int32_t ctd_microbench(ctd_ctx *ctx, int32_t kind, uint64_t bytes, uint64_t ops,
                                  double *rate, double *ms) {
  if (!ctx || !rate) return CTD_EINVAL;
  NEED(ctx, kind >= 0 && kind <= 3, "kind must be 0..3");
  NEED(ctx, bytes >= 4096 && bytes <= ((uint64_t)1 << 36) && bytes % 16 == 0,
       "bytes must be a multiple of 16 in [4 KiB, 64 GiB]");
  NEED(ctx, kind == 0 || (ops > 0 && bytes / 8 <= 0xFFFFFFFFull), "bad ops or size");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  void *a = nullptr, *b = nullptr;
  HIPCHK(ctx, hipMalloc(&a, bytes));
  hipError_t e = hipMalloc(&b, kind == 0 ? bytes : 256);
  if (e != hipSuccess) {
    dfree(a);
    return hip_err(ctx, e, "microbench alloc");
  }
  launch_zero(a, bytes, ctx->stream);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int grid = ctx->n_cu * 8;
  int rc = CTD_OK;
  float best = INFINITY;
  for (int rep = 0; rep < 4 && rc == CTD_OK; ++rep) {  // first pass warms up
    (void)hipEventRecord(e0, ctx->stream);
    if (launch_microbench(kind, a, b, (int64_t)bytes, (int64_t)ops, grid, ctx->stream) != 0)
      rc = hip_err(ctx, hipGetLastError(), "microbench launch");
    (void)hipEventRecord(e1, ctx->stream);
    (void)hipEventSynchronize(e1);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    if (rep > 0) best = std::min(best, t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);
  dfree(a);
  dfree(b);
  if (rc != CTD_OK) return rc;
  const double sec = (double)best * 1e-3;
  *rate = kind == 0 ? 2.0 * (double)bytes / sec / 1e9 : (double)ops / sec;
  if (ms) *ms = best;
  return CTD_OK;
}
