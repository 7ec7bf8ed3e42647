// Macro-cell majorants for MACRO tracking (a space-dependent majorant for the
// Woodcock tracking of Sec. 2.1).
//
// The phantom is cut into cubic cells of cs^3 voxels.  For each cell and
// material the largest density present is found on the device; on the host
// it is rounded up to 10 significant mantissa bits (so that cells group into
// classes), and each distinct vector of rounded densities becomes a class
// whose majorant at every energy node is formed exactly like the global one
// (largest rho * (mu_pe + mu_C [+ mu_R]) / rho over the materials, FP64,
// 2^-20 margin, rounded up to float).  The transport reads one number per
// cell crossing: the energy grid is cut into at most 16 bands of 2^shift grid
// cells, and per band and cell it stores the factor f with f * mu_max >= the
// class majorant at every node the band's grid cells interpolate between
// (largest ratio, widened by 2^-18 for the float lerps and the product,
// rounded up, at most 1).  Both majorants are linear between nodes, so
// f * mu_max(E) bounds every voxel of the cell at every energy of the band,
// and f = 1 gives the global majorant, which bounds every voxel anywhere.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "ctd.h"
#include "ctd_api_internal.h"
#include "ctd_tables.h"

using namespace ctd;

namespace {

// Round a non-negative float up to 10 significant mantissa bits.
float round_up_10bits(float v) {
  uint32_t b;
  std::memcpy(&b, &v, 4);
  const uint32_t low = (1u << 13) - 1u;
  if (b & low) b = (b | low) + 1u;
  float r;
  std::memcpy(&r, &b, 4);
  return r;
}

}  // namespace

int ctd::macro_edge(const ctd_grid &g, int requested) {
  if (requested > 0) return requested;
  // about 1.6 cm: long enough that a crossing is rarer than a fictitious
  // step would be, short enough to separate bone from soft tissue
  const double h = std::min(g.dx, std::min(g.dy, g.dz));
  return std::max(1, (int)std::lround(std::min(1.6 / h, 64.0)));
}

int ctd::macro_cells(const ctd_grid &g, int cs, int n[3]) {
  n[0] = (g.nx + cs - 1) / cs;
  n[1] = (g.ny + cs - 1) / cs;
  n[2] = (g.nz + cs - 1) / cs;
  return n[0] * n[1] * n[2];
}

int ctd::build_macro(ctd_ctx *ctx, ctd_case *cs) {
  const int cell = macro_edge(cs->ph->g, cs->p.macro_cell);
  const ctd_grid &g = cs->ph->g;
  int n[3];
  const int64_t cells = macro_cells(g, cell, n);
  const int M = cs->ms->M;
  // the transport packs a cell index as x | y << 10 | z << 20
  if (n[0] > 1023 || n[1] > 1023 || n[2] > 4095 || cells * M > ((int64_t)1 << 31))
    return set_err(ctx, CTD_EINVAL, "too many macro cells (%d x %d x %d): raise macro_cell",
                   n[0], n[1], n[2]);
  unsigned int *d_max = nullptr;
  // whole 8-byte words, so the clearing kernel covers every entry
  const size_t bytes = (sizeof(unsigned int) * (size_t)(cells * M) + 7) & ~(size_t)7;
  hipError_t e = hipMalloc(&d_max, bytes);
  if (e != hipSuccess) return hip_err(ctx, e, "macro-cell scratch");
  std::vector<unsigned int> hmax((size_t)(cells * M));
  int rc = CTD_OK;
  if (launch_zero(d_max, bytes, ctx->stream) != 0 ||
      launch_cell_max(cs->ph->vox, g.nx, g.ny, g.nz, cell, n[0], n[1], M, d_max, ctx->stream) !=
          0) {
    rc = hip_err(ctx, hipGetLastError(), "macro-cell kernel");
  } else if ((e = hipMemcpyAsync(hmax.data(), d_max, sizeof(unsigned int) * hmax.size(),
                                 hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess ||
             (e = hipStreamSynchronize(ctx->stream)) != hipSuccess) {
    rc = hip_err(ctx, e, "macro-cell readback");
  }
  (void)hipFree(d_max);
  if (rc != CTD_OK) return rc;

  const int ne = cs->ms->eg.ne;
  std::map<std::vector<uint32_t>, int> classes;
  std::vector<int32_t> cls((size_t)cells);
  std::vector<float> tab;
  std::vector<double> rmax((size_t)M);
  bool pres[256];
  std::vector<uint32_t> key((size_t)M);
  for (int64_t c = 0; c < cells; ++c) {
    for (int m = 0; m < M; ++m) {
      float v;
      std::memcpy(&v, &hmax[(size_t)(c * M + m)], 4);
      v = round_up_10bits(v);
      std::memcpy(&key[(size_t)m], &v, 4);
    }
    auto it = classes.find(key);
    if (it == classes.end()) {
      const int id = (int)classes.size();
      it = classes.emplace(key, id).first;
      for (int m = 0; m < M; ++m) {
        float v;
        std::memcpy(&v, &key[(size_t)m], 4);
        rmax[(size_t)m] = (double)v;
        pres[m] = v > 0.0f;
      }
      tab.resize(tab.size() + (size_t)ne);
      majorant_fp64(ne, M, cs->ms->mu_rho.data(), rmax.data(), pres, cs->p.rayleigh != 0,
                    tab.data() + (size_t)id * ne);
    }
    cls[(size_t)c] = it->second;
  }
  // energy bands: grid cell j (nodes j, j + 1) lies in band j >> shift
  int shift = 0;
  while (((ne - 2) >> shift) >= kMacroBands) ++shift;
  const int nb = ((ne - 2) >> shift) + 1;
  const int ncls = (int)classes.size();
  const std::vector<float> &gmaj = cs->mu_max;  // the case's global majorant
  std::vector<float> fcls((size_t)ncls * nb);
  for (int k = 0; k < ncls; ++k)
    for (int b = 0; b < nb; ++b) {
      const int j0 = b << shift, j1 = std::min((b + 1) << shift, ne - 1);
      double r = 0.0;
      for (int j = j0; j <= j1; ++j) {
        const double c = (double)tab[(size_t)k * ne + j];
        if (c > 0.0) r = std::max(r, gmaj[j] > 0.0f ? c / (double)gmaj[j] : INFINITY);
      }
      r *= 1.0 + 0x1p-18;
      float f = (float)r;
      if ((double)f < r) f = std::nextafter(f, INFINITY);
      // mu_max itself bounds every voxel: a cell never needs more
      fcls[(size_t)k * nb + b] = std::min(f, 1.0f);
    }
  std::vector<float> fac((size_t)nb * cells);
  for (int b = 0; b < nb; ++b)
    for (int64_t c = 0; c < cells; ++c)
      fac[(size_t)b * cells + c] = fcls[(size_t)cls[(size_t)c] * nb + b];
  if ((e = hipMalloc(&cs->d_mc_f, sizeof(float) * fac.size())) != hipSuccess ||
      (e = hipMemcpy(cs->d_mc_f, fac.data(), sizeof(float) * fac.size(),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return hip_err(ctx, e, "macro-cell upload");
  cs->mc_shift = shift;
  cs->mc_bands = nb;
  cs->mc_cs = cell;
  for (int a = 0; a < 3; ++a) cs->mc_n[a] = n[a];
  cs->mc_classes = (int)classes.size();
  return CTD_OK;
}
