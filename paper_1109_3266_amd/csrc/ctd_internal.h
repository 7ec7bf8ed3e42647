// Plain-old-data structures shared by the host runtime (ctd_api.cpp) and the
// HIP kernels (ctd_kernels.hip).  Everything a kernel reads about a case lives
// in one CaseDev record in device memory; a launch covers one "round": for
// each participating case, one batch of histories, consumed in chunks.
#pragma once

#include <algorithm>
#include <vector>

#include <stddef.h>
#include <stdint.h>

#include "ctd.h"
#include "ctd_schedule.h"

namespace ctd {

// Per-case accumulators (device, uint64 each).
enum Acc : int {
  ACC_Q_INC = 0,     // incident energy, q units
  ACC_Q_DEP,         // deposited energy, q units
  ACC_Q_ESC,         // escaped energy (including misses), q units
  ACC_N_HIST,
  ACC_N_STEPS,
  ACC_N_REAL,
  ACC_N_PHOTO,
  ACC_N_COMPTON,
  ACC_N_RAYLEIGH,
  ACC_N_DEPOSITS,
  ACC_N_ESCAPES,
  ACC_N_MISS,
  ACC_N_UNSCATTERED,
  ACC_N_CUTOFF,
  ACC_N_REFILLS,
  ACC_STEP_GUARD,    // histories killed by the step guard (must stay 0)
  ACC_N_CROSS,       // macro-cell boundary crossings (MACRO tracking)
  ACC_COUNT
};

// Layout of a case's counter block (uint64 words): [0, ACC_COUNT) counters of
// the current batch (kernel atomics), [ACC_COUNT, 3 ACC_COUNT) exact 128-bit
// totals as (lo, hi) pairs, folded after every batch, then the per-voxel
// maxima seen by the folds: max S1, max high word of S2.
constexpr int kAccTotal = ACC_COUNT;
constexpr int kAccMaxS1 = 3 * ACC_COUNT;
constexpr int kAccMaxS2Hi = 3 * ACC_COUNT + 1;
constexpr int kAccWords = 3 * ACC_COUNT + 4;

constexpr float kQScale = 16777216.0f;  // 2^24: tally unit q = 2^-24 keV
constexpr int kTallyCopies = 8;         // one batch tally per XCD of an MI355X
constexpr int kMacroBands = 16;         // MACRO tracking: most energy bands
constexpr int kPackStats = 770;         // words of k_pack's statistics
constexpr uint32_t kMixedClass = 255;   // bound grid: a block of several materials
constexpr uint32_t kStepGuard = 1000000u;  // random pairs (MACRO: flights) a history may take
constexpr float kInvMeC2 = (float)(1.0 / 510.99895);

struct CaseDev {
  // voxel grid; positions are tracked in voxel units
  int32_t nx, ny, nz, nmat;
  float fnx, fny, fnz, pad0;
  float inv_dx, inv_dy, inv_dz, pad1;
  float ox, oy, oz, pad2;
  const uint2 *vox;            // [V] (float bits of rho, material id)
  int64_t V;
  // palette layout (phantoms with <= 256 distinct (rho, material) pairs):
  // vox8[V] indexes palette[256]; npal = 0 when not used
  const uint8_t *vox8;
  const uint2 *palette;
  int32_t npal, pad9;
  // energy grid and tables
  int32_t ne, nzc, nzr, rayleigh;
  float e0, inv_de, e_cut, pad3;
  const float4 *mu_rho;        // [nmat][ne] (pe, Compton, Rayleigh, 0) cm^2/g
  const float *mu_max;         // [ne] cm^-1
  const float4 *comp_quad;     // [ncomp][ne-1][nzc-1] bilinear cells
  const float4 *rayl_quad;     // [nmat][ne-1][nzr-1] or null
  int32_t comp_per_mat, nbins;
  float bin_width, pad4;
  const float *bin_lo;         // [nbins]
  // geometry
  int32_t kind, nproj;
  float sad, pad5;
  float src[3], dir[3];
  float iso[3], pad6;
  float a0, a1, b0, b1;
  float phi0_turns, arc_turns, z_feed, pad8;   // z_feed: cm per turn
  const float4 *proj_sc;       // [nproj] (sin phi_p, cos phi_p, z offset of p, 0)
  // fluence map: fl_n beamlets (0 = uniform field), fl_na along a
  int32_t fl_n, fl_na, fl_gbits, fl_chains;   // fl_chains > 0: Alg. A1 beamlets
  float fl_da, fl_db;          // beamlet size at the isocentre (cm)
  double fl_total;             // F = C_{n-1}
  const double *fl_cdf;        // [fl_n] running sums of f
  const int32_t *fl_guide;     // [2^fl_gbits]
  // MACRO tracking: cells of mc_cs^3 voxels, mc_n[3] per axis (mc_cs = 0:
  // GLOBAL).  Energy-grid cell j lies in band j >> mc_shift; the majorant of
  // a cell in band b is mc_f[b * mc_ncell + cell] * mu_max(E).
  int32_t mc_cs, mc_nx, mc_ny, mc_nz;
  float mc_fcs, mc_inv_cs;
  int32_t mc_shift, mc_ncell;
  const float *mc_f;
  // Bound grid (8-byte record layout only): the class of every block of
  // 2^s x 2^s x 2^s voxels, s = 0, 1, 2 (blocks per axis ceil(n / 2^s), x
  // fastest; kMixedClass where the block holds more than one material), and
  // the class table bclass[256] = (float bits of a density level, material):
  // every voxel of a block of class c has material bclass[c].y and a density
  // <= the level, so the Woodcock selection evaluated at the level bounds the
  // voxel's own (float rounding is monotone).  Null where not built.
  const uint8_t *bgrid[3];
  const uint2 *bclass;
  // per material and energy cell j ([E_j, E_j+1]): a float at or above the
  // interaction sum (photoelectric + Compton, + Rayleigh when on) that the
  // selection forms anywhere in the cell, so rho_c * bnd bounds the selection
  // at class level rho_c without the table rows  [nmat][ne - 1]
  const float *bnd;
  // random stream key
  uint32_t key0, key1;
  // tallies
  unsigned long long *tally;   // T_b [kTallyCopies][V]
  long long *s1;               // [V]
  unsigned long long *s2;      // [V][2] (lo, hi)
  unsigned long long *acc;     // [ACC_COUNT]
  // event log (debug)
  ctd_event *log;
  unsigned long long *log_n;
  uint64_t log_h0, log_h1, log_cap;
};

// One case's share of a launch: batch histories [h_begin, h_begin + n) laid
// out bin-major by prefix[0..nbins]; chunks [chunk_begin, chunk_begin +
// ceil(n/chunk)) of the launch-wide chunk counter belong to it.
struct RoundCase {
  const CaseDev *cd;
  const unsigned long long *prefix;
  uint64_t h_begin, n, chunk_begin;
  const int32_t *beamlets;     // [n] Alg. A1 beamlet per history, or null
  // the case's home workgroups [wg_lo, next case's wg_lo) of the launch's
  // grid (home_round_cases); home_waves = their waves, which take the case's
  // first chunks by rank
  uint32_t wg_lo, home_waves;
};

// Fill wg_lo and home_waves of a round's cases (chunk_begin already set) for
// a grid of `grid` workgroups of `waves` waves (ctd_schedule.h).
inline void home_round_cases(RoundCase *rc, int nrc, int grid, int waves) {
  std::vector<uint64_t> begin((size_t)nrc);
  std::vector<uint32_t> lo((size_t)nrc), hw((size_t)nrc);
  for (int i = 0; i < nrc; ++i) begin[i] = rc[i].chunk_begin;
  home_workgroups(begin.data(), nrc, grid, waves, lo.data(), hw.data());
  for (int i = 0; i < nrc; ++i) {
    rc[i].wg_lo = lo[i];
    rc[i].home_waves = hw[i];
  }
}

// Entry point that allocates nothing (ctd_run_batches_static): the launch
// table of one single-case round -- the RoundCase, the spectrum's bin prefix
// sums and the chunk counter -- lives in a file-scope device array of
// kStaticScratchBytes, written by a one-block set-up kernel from its
// arguments (no copy, no memset).  Byte offsets inside the array:
constexpr int kStaticMaxBins = 256;
constexpr size_t kStaticPrefixOff = 256;                          // after the RoundCase
constexpr size_t kStaticCounterOff = 2560;                        // 256-aligned, past the prefix
constexpr size_t kStaticScratchBytes = kStaticCounterOff + 256;   // 2816 B
static_assert(kStaticPrefixOff + 8 * (kStaticMaxBins + 1) <= kStaticCounterOff,
              "static round table layout");

// The round a set-up kernel writes (passed by value: 2.1 KB of arguments).
struct StaticRoundArgs {
  const CaseDev *cd;
  uint64_t h_begin, n;
  const int32_t *beamlets;
  int32_t nbins;
  uint32_t home_waves;   // every wave of the grid: the one case is everyone's home
  unsigned long long prefix[kStaticMaxBins + 1];
};

struct LaunchCfg {
  int block;
  int grid;
  int refill_min;
  int chunk;
  int tally_mode;
  int bound_shift;   // bound grid of 2^s-voxel blocks, or -1 (no early rejection)
  int defer_min;     // with a bound grid: collision pass once this many wait (0: at once)
  int tab_n, tab_ne; // the round's largest case: mu/rho rows and energy nodes to stage in LDS
  size_t lds_budget; // LDS a workgroup may take without lowering the residency
};

// Step of a transport launch, the same for every case of it: kStepPlain
// (GLOBAL tracking, every tentative collision read from its voxel),
// kStepDeferred (GLOBAL tracking with the bound grid's early rejection and
// collision passes: every case has a bound grid in use),
// kStepMacro (MACRO tracking).  A round whose cases need different steps is
// split into one launch per step.
constexpr int kStepPlain = 0, kStepDeferred = 1, kStepMacro = 2;

// Kernel launchers (ctd_kernels.hip).  All enqueue on `stream`.
int launch_transport(const RoundCase *rc_dev, int nrc, uint64_t total_chunks,
                     unsigned long long *chunk_ctr, const LaunchCfg &cfg, bool with_log,
                     int step_kind, void *stream);
// Whether a transport workgroup of `block` threads in tally_mode fits the
// device's LDS limit (mode 2 adds a sub-tally per wave).
bool transport_lds_fits(int block, int tally_mode, int device);
// Dynamic LDS of a transport workgroup: its header, case descriptor and
// class table, per-wave counters, the tally-mode-2 sub-tallies, and room for
// tab_n mu/rho rows, tab_ne majorant nodes and tab_n bound-test sums (0:
// none), and a source stash of stash_cap records per wave.
size_t transport_lds_bytes(int block, int tally_mode, int tab_n, int tab_ne, int stash_cap);
// Fold ncopies batch tallies [ncopies][V]: S1 += sum, S2 += sum^2, zero them;
// fold the batch counters of acc into its 128-bit totals and record the
// per-voxel maxima of S1 and of S2's high word.
int launch_fold(unsigned long long *tally, int ncopies, long long *s1, unsigned long long *s2,
                int64_t V, unsigned long long *acc, void *stream);
// Largest XCC id seen by `blocks` workgroups (written to *out, device).
int launch_xcc_probe(unsigned int *out, int blocks, void *stream);
// stats[kPackStats]: [0,256) max density bits per material, [256,512) voxel
// count per material, [512] largest material id, [513] voxels with a bad
// density, [514,770) complemented min density bits per material.
int launch_pack(const uint8_t *mat, const float *rho, uint2 *vox, int64_t V, unsigned int *stats,
                void *stream);
int launch_zero(void *ptr, size_t bytes, void *stream);
// Device address of this device's static round table (hipGetSymbolAddress
// with the device current); 0 on success.
int static_scratch_address(void **out);
// Write one round's table into the static array at `table` (its device
// address) and clear its chunk counter; then the transport may run on it.
int launch_static_round_setup(void *table, const StaticRoundArgs &args, void *stream);
// sigma-bar over one case: out[0] = sigma, out[1] = voxel count, out[2] =
// max dose (S1/rho); scratch holds 3 * nblocks doubles.
int launch_sigma(const long long *s1, const unsigned long long *s2, const uint2 *vox, int64_t V,
                 uint32_t nb, double rho_min, double frac, int kind, double *scratch,
                 int nblocks, double *out, void *stream);
// kind 0 copy (n bytes), 1 random atomics / 2 hot-spot atomics (ops on an
// n-byte uint64 array), 3 random 8-byte gathers (ops over n bytes).
int launch_microbench(int kind, void *buf_a, void *buf_b, int64_t n, int64_t ops, int grid,
                      void *stream);
int device_cu_count(int device);
// Alg. A1: advance C logical chains (chain = h mod C) over histories
// [h_begin, h_begin + n): state[C] in/out, out[n] the beamlet of each history.
// MACRO tracking: out[cell * M + m] = max float bits of the density of
// material m over the voxels of each cell of cs^3 voxels (out zeroed).
int launch_cell_max(const uint2 *vox, int nx, int ny, int nz, int cs, int ncx, int ncy, int M,
                    unsigned int *out, void *stream);
// Bound grid of blocks of 2^shift voxels per edge: out[block] = the class
// (index into cls) of the smallest density level of the block's material at
// or above the block's largest density, or kMixedClass.  range[m] = (first
// class of material m, level count), levels ascending within a material.
int launch_block_class(const uint2 *vox, int nx, int ny, int nz, int shift, const uint2 *cls,
                       const int2 *range, uint8_t *out, void *stream);
int launch_mh_fill(const float *f, int n_f, int C, uint64_t h_begin, uint64_t n, uint32_t key0,
                   uint32_t key1, int32_t *state, int32_t *out, void *stream);
// Gamma index of ev against ref on an nx*ny*nz grid (ctd_gamma.hip); offs is
// a device double4 table sorted by distance; gamma may be null; counts[2]
// (region voxels, passing voxels) are accumulated, not cleared.
int launch_gamma(const float *ref, const float *ev, int nx, int ny, int nz, const void *offs,
                 int n_off, double inv_dd2, double region, double cap2, float *gamma,
                 unsigned long long *counts, void *stream);

}  // namespace ctd
