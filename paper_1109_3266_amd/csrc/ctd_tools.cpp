// Dose comparison tools behind the C ABI: the gamma-index agreement test of
// Sec. 3.1 (kernel in ctd_gamma.hip).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ctd.h"
#include "ctd_api_internal.h"

using namespace ctd;

namespace {

constexpr int kMaxOffsets = 1 << 22;

struct Dev {
  void *p = nullptr;
  ~Dev() {
    if (p) (void)hipFree(p);
  }
};

// One search offset, laid out as the kernel's double4 (four doubles) but
// with the alignment of a double: std::stable_sort's temporary buffer is not
// aligned for the 32-byte HIP vector type.
struct Offset {
  double x, y, z, r2;
};
static_assert(sizeof(Offset) == sizeof(double4), "Offset must match double4");

// Lattice offsets h*(i,j,k), h = dta/substeps, with |offset| <= cap*dta, as
// (voxel-unit x, y, z, |offset|^2/dta^2), ascending in distance.
std::vector<Offset> gamma_offsets(const ctd_grid &g, const ctd_gamma_params &p) {
  const int s = p.substeps;
  const double rmax = p.gamma_cap * s;          // radius in lattice steps
  const int L = (int)std::ceil(rmax);
  const double h = p.dta_cm / s;
  std::vector<Offset> out;
  for (int k = -L; k <= L; ++k)
    for (int j = -L; j <= L; ++j)
      for (int i = -L; i <= L; ++i) {
        const double r2 = (double)(i * i + j * j + k * k);
        if (r2 > rmax * rmax) continue;
        out.push_back(Offset{i * h / g.dx, j * h / g.dy, k * h / g.dz, r2 / ((double)s * s)});
      }
  std::stable_sort(out.begin(), out.end(),
                   [](const Offset &a, const Offset &b) { return a.r2 < b.r2; });
  return out;
}

}  // namespace

extern "C" int32_t ctd_gamma(ctd_ctx *ctx, const ctd_grid *g, const float *ref, const float *ev,
                             int32_t mem, const ctd_gamma_params *p, float *gamma,
                             uint64_t *n_region, uint64_t *n_pass) {
  if (!ctx) return CTD_EINVAL;
  if (!g || !ref || !ev || !p) return set_err(ctx, CTD_EINVAL, "null argument");
  if (mem != CTD_MEM_HOST && mem != CTD_MEM_DEVICE)
    return set_err(ctx, CTD_EINVAL, "mem must be HOST or DEVICE");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) ||
      !std::isfinite(g->dx) || !std::isfinite(g->dy) || !std::isfinite(g->dz))
    return set_err(ctx, CTD_EINVAL, "bad grid");
  if (!(p->dose_tol > 0) || !std::isfinite(p->dose_tol) || !(p->dta_cm > 0) ||
      !std::isfinite(p->dta_cm) || !std::isfinite(p->region_min))
    return set_err(ctx, CTD_EINVAL, "dose_tol and dta_cm must be > 0, region_min finite");
  if (!(p->gamma_cap >= 1.0 && p->gamma_cap <= 4.0) || p->substeps < 1 || p->substeps > 20)
    return set_err(ctx, CTD_EINVAL, "need 1 <= gamma_cap <= 4 and 1 <= substeps <= 20");
  const std::vector<Offset> offs = gamma_offsets(*g, *p);
  if ((int64_t)offs.size() > kMaxOffsets)
    return set_err(ctx, CTD_EINVAL, "%zu search offsets exceed %d", offs.size(), kMaxOffsets);
  const int64_t V = (int64_t)g->nx * g->ny * g->nz;
  const hipStream_t st = ctx->stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, CTD_EDEVICE, "hipSetDevice");
  Dev d_offs, d_cnt, d_ref, d_ev, d_gam;
  hipError_t e;
  if ((e = hipMalloc(&d_offs.p, sizeof(Offset) * offs.size())) != hipSuccess ||
      (e = hipMalloc(&d_cnt.p, 2 * sizeof(unsigned long long))) != hipSuccess)
    return hip_err(ctx, e, "gamma alloc");
  const float *r = ref, *v = ev;
  float *gout = mem == CTD_MEM_DEVICE ? gamma : nullptr;
  if (mem == CTD_MEM_HOST) {
    if ((e = hipMalloc(&d_ref.p, 4 * V)) != hipSuccess ||
        (e = hipMalloc(&d_ev.p, 4 * V)) != hipSuccess ||
        (gamma && (e = hipMalloc(&d_gam.p, 4 * V)) != hipSuccess))
      return hip_err(ctx, e, "gamma alloc");
    if ((e = hipMemcpyAsync(d_ref.p, ref, 4 * V, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(d_ev.p, ev, 4 * V, hipMemcpyHostToDevice, st)) != hipSuccess)
      return hip_err(ctx, e, "gamma upload");
    r = (const float *)d_ref.p;
    v = (const float *)d_ev.p;
    gout = (float *)d_gam.p;
  }
  if ((e = hipMemcpyAsync(d_offs.p, offs.data(), sizeof(Offset) * offs.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_err(ctx, e, "gamma upload");
  if (launch_zero(d_cnt.p, 2 * sizeof(unsigned long long), st) != 0 ||
      launch_gamma(r, v, g->nx, g->ny, g->nz, d_offs.p, (int)offs.size(),
                   1.0 / (p->dose_tol * p->dose_tol), p->region_min,
                   p->gamma_cap * p->gamma_cap, gout, (unsigned long long *)d_cnt.p, st) != 0)
    return hip_err(ctx, hipGetLastError(), "gamma launch");
  unsigned long long cnt[2];
  if ((e = hipMemcpyAsync(cnt, d_cnt.p, sizeof cnt, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (mem == CTD_MEM_HOST && gamma &&
       (e = hipMemcpyAsync(gamma, d_gam.p, 4 * V, hipMemcpyDeviceToHost, st)) != hipSuccess) ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hip_err(ctx, e, "gamma readback");
  if (n_region) *n_region = cnt[0];
  if (n_pass) *n_pass = cnt[1];
  return CTD_OK;
}
