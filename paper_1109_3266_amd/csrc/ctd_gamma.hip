// Gamma-index evaluation (the dose agreement test of Sec. 3.1, after Low et
// al. 1998): gamma(r) = min over r' of sqrt((D_ref(r) - D_eval(r'))^2 / dD^2 +
// |r - r'|^2 / dr^2), with r' on a lattice of step dr / substeps around the
// voxel centre r and D_eval trilinearly interpolated between voxel centres
// (clamped at the grid's outer centres).
//
// One lane per reference voxel.  The candidate offsets come sorted by
// distance, so a lane is finished once the distance term alone reaches its
// best value; the offset index is wave-uniform (the table is read through
// the scalar path) and the loop ends when no lane of the wave still needs a
// candidate.  All arithmetic is FP64: the pass decision gamma < 1 is taken on
// gamma^2 < 1 in double.
#include <hip/hip_runtime.h>

#include "ctd_internal.h"

namespace ctd {

namespace {

// Clamp a voxel-centre coordinate to [0, n-1] and split it into the lower
// node, the upper node and the weight of the upper node.
__device__ __forceinline__ void axis(double u, int n, int &i0, int &i1, double &f) {
  u = fmin(fmax(u, 0.0), (double)(n - 1));
  i0 = (int)u;
  if (i0 > n - 2) i0 = n > 1 ? n - 2 : 0;
  f = u - (double)i0;
  i1 = i0 + 1 < n ? i0 + 1 : n - 1;
}

__device__ __forceinline__ double lerp(double a, double b, double f) { return a + f * (b - a); }

__device__ double interp(const float *__restrict__ D, int nx, int ny, int nz, double x, double y,
                         double z) {
  int x0, x1, y0, y1, z0, z1;
  double fx, fy, fz;
  axis(x, nx, x0, x1, fx);
  axis(y, ny, y0, y1, fy);
  axis(z, nz, z0, z1, fz);
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  const float *p00 = D + z0 * sz + y0 * sy, *p01 = D + z0 * sz + y1 * sy;
  const float *p10 = D + z1 * sz + y0 * sy, *p11 = D + z1 * sz + y1 * sy;
  const double c00 = lerp((double)p00[x0], (double)p00[x1], fx);
  const double c01 = lerp((double)p01[x0], (double)p01[x1], fx);
  const double c10 = lerp((double)p10[x0], (double)p10[x1], fx);
  const double c11 = lerp((double)p11[x0], (double)p11[x1], fx);
  return lerp(lerp(c00, c01, fy), lerp(c10, c11, fy), fz);
}

}  // namespace

// offs[k] = (dx, dy, dz in voxel units, |offset|^2 / dr^2), ascending in .w.
// counts[0] += voxels with D_ref > region, counts[1] += those with gamma < 1.
__global__ void __launch_bounds__(256) k_gamma(const float *__restrict__ ref,
                                               const float *__restrict__ ev, int nx, int ny,
                                               int nz, const double4 *__restrict__ offs,
                                               int n_off, double inv_dd2, double region,
                                               double cap2, float *__restrict__ gamma,
                                               unsigned long long *__restrict__ counts) {
  const int64_t V = (int64_t)nx * ny * nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool active = false;
  double dr = 0.0, best = cap2;
  int ix = 0, iy = 0, iz = 0;
  if (v < V) {
    dr = (double)ref[v];
    active = dr > region;
    ix = (int)(v % nx);
    const int64_t t = v / nx;
    iy = (int)(t % ny);
    iz = (int)(t / ny);
  }
  for (int k = 0; k < n_off; ++k) {
    const double4 o = offs[k];
    const bool want = active && o.w < best;
    if (!__any(want)) break;
    if (want) {
      const double d = dr - interp(ev, nx, ny, nz, ix + o.x, iy + o.y, iz + o.z);
      best = fmin(best, o.w + d * d * inv_dd2);
    }
  }
  if (gamma && v < V) gamma[v] = active ? (float)sqrt(best) : -1.0f;
  const unsigned long long m_reg = __ballot(active);
  const unsigned long long m_pass = __ballot(active && best < 1.0);
  if ((threadIdx.x & 63) == 0 && m_reg) {
    atomicAdd(&counts[0], (unsigned long long)__popcll(m_reg));
    if (m_pass) atomicAdd(&counts[1], (unsigned long long)__popcll(m_pass));
  }
}

int launch_gamma(const float *ref, const float *ev, int nx, int ny, int nz, const void *offs,
                 int n_off, double inv_dd2, double region, double cap2, float *gamma,
                 unsigned long long *counts, void *stream) {
  const int64_t V = (int64_t)nx * ny * nz;
  if (V <= 0) return 0;
  const int64_t blocks = (V + 255) / 256;
  if (blocks > 0x7fffffff) return -1;
  hipLaunchKernelGGL(k_gamma, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, ref, ev,
                     nx, ny, nz, (const double4 *)offs, n_off, inv_dd2, region, cap2, gamma,
                     counts);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ctd
