// HIP kernels for gfx950 (MI355X): Woodcock photon transport (Jia et al.,
// arXiv 1109.3266, Sec. 2.1-2.2), batch fold and sigma-bar reduction,
// Metropolis-Hastings beamlet chains (Alg. A1), macro-cell set-up and
// microbenchmarks.
//
// Execution model.  One persistent launch per round (per tracking mode: the
// global-majorant and macro-cell steps are separate instantiations).  A round is, for each
// participating case, one batch of histories laid out bin-major over the
// spectrum (Sec. 2.2.5), split into chunks of consecutive history ids.  Each
// 64-lane wave owns one case at a time and a pool of history ids claimed one
// chunk per atomic; lanes are one photon each (Sec. 2.2, one thread per
// photon).  When at least `refill_min` lanes of a wave are idle the wave
// refills them in one step from its source stash in LDS, which the whole wave
// fills by sampling the sources of its pool's next ids at once, so a wave
// keeps ~all lanes busy without sampling on a few lanes at a time, and its
// lanes hold photons of neighbouring ids, i.e. similar energies.  A wave
// that claims a chunk of a different case finishes its live photons first.
//
// Numerics.  Transport is float32.  Every deposit (E - E' of a Compton event,
// E of a photoelectric or cutoff event) and every escape is an exact
// multiple of q = 2^-24 keV for E < 256 keV, so deposits enter the int64 tally
// exactly and incident = deposited + escaped holds exactly in q units.
// Random numbers: Philox4x32-10 keyed by the case seed, counter (k,
// history id lo, hi, 0); k = 0 draws the source.  With the global majorant
// blocks k >= 1 are read two words (a pair) at a time: a Woodcock step takes
// a pair (free path, interaction type), a Compton or Rayleigh scatter the
// pair after its step (polar zeta, azimuth); with MACRO tracking flight k
// takes block k (optical depth, interaction type, zeta, azimuth).  Two more
// streams use
// the fourth counter word: (0, h lo, h hi, 1) the fluence-map beamlet of
// history h (inverse CDF, or trial and acceptance of Alg. A1), and
// (0, c, 0, 2) the starting beamlet of Metropolis-Hastings chain c.
#include <hip/hip_runtime.h>

#include "ctd_internal.h"

namespace ctd {

// Pointers the step loop dereferences are tagged with the global address
// space so they compile to global_* (not flat_*) memory instructions (the
// tag only exists in the device compilation pass).
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#define LOCAL __attribute__((address_space(3)))
#else
#define GLOBAL
#define LOCAL
#endif

// ---------------------------------------------------------------- helpers

// Tally mode 2: per-wave LDS sub-tally of 2^kCacheBits slots (int32 key +
// uint64 value each, 6 KB per wave), in dynamic shared memory.
constexpr int kCacheBits = 9;
constexpr int kCacheSlots = 1 << kCacheBits;
constexpr int kCacheBytesPerWave = kCacheSlots * (8 + 4);

// Dynamic LDS of a transport workgroup, in this order: a 16-byte header
// (the workgroup's next case); the descriptor of the case the workgroup works
// on and its 256-entry palette or bound-class table (every wave of a
// workgroup works on the same case); per wave, its event counters and an
// 8-byte word per lane (what a lane's waiting collision or scatter needs
// later); in tally mode 2, each wave's sub-tally; per wave, its source
// stash of stash_cap records (stash_cap entry points and energies as float4,
// then stash_cap directions as float4, w = the record's history offset);
// where the tables fit, the case's majorant nodes (padded to 16 B) and mu/rho
// rows.
constexpr int kWaveAccBytes = (ACC_COUNT * 8 + 15) & ~15;
constexpr int kStashRecBytes = 32;
constexpr int kWaveSlotBytes = kWaveAccBytes + 64 * 8;
constexpr int kWaveCaseBytes = ((int)sizeof(CaseDev) + 15) & ~15;
constexpr int kWgHeaderBytes = 16;
constexpr int kWgCaseOff = kWgHeaderBytes;
constexpr int kWgPalOff = kWgCaseOff + kWaveCaseBytes;
constexpr int kWgSlotsOff = kWgPalOff + 256 * 8;

// a ^ b ^ c in one instruction (gfx950 three-input bitwise op, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t y0 = xor3((uint32_t)(p1 >> 32), x1, k0);
    const uint32_t y2 = xor3((uint32_t)(p0 >> 32), x3, k1);
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(x0, x1, x2, x3);
}

// (2 (r >> 9) + 1) 2^-24 exactly: [1,2) mantissa trick minus (1 - 2^-24).
// The float 1.m with m = r >> 9 is bits [40:9] of the 64-bit {0x7F, r}: one
// v_alignbit_b32 instead of a shift and an or.
__device__ __forceinline__ float unif(uint32_t r) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9u)) - 0x1.fffffep-1f;
}

__device__ __forceinline__ float lerpf(float a, float b, float w) { return fmaf(w, b - a, a); }

// sin / cos of a phase given in turns (revolutions), hardware transcendental.
__device__ __forceinline__ float sin_turns(float t) { return __builtin_amdgcn_sinf(t); }
__device__ __forceinline__ float cos_turns(float t) { return __builtin_amdgcn_cosf(t); }

// Inverse-CDF surface mu(zeta, E): one 16-byte cell gives both zeta
// neighbours at both energy neighbours; bilinear, clamped to [-1, 1].
__device__ __forceinline__ float surface(const GLOBAL float4 *__restrict__ Q, int nz, int je,
                                         float we,
                                         float zeta) {
  const float f = zeta * (float)(nz - 1);
  const int i = min((int)f, nz - 2);
  const float wz = f - (float)i;
  const float4 q = Q[(size_t)je * (size_t)(nz - 1) + (size_t)i];
  const float s0 = lerpf(q.x, q.y, wz);
  const float s1 = lerpf(q.z, q.w, wz);
  return fminf(fmaxf(lerpf(s0, s1, we), -1.0f), 1.0f);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void atomic_add_u64(unsigned long long *p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The fields the step loop reads, as one wave-uniform record.  It is filled
// with readfirstlane when a wave takes its first chunk of a case, so the
// compiler keeps it in scalar registers; everything else about a case (source
// geometry, the angular surfaces and cutoff used at real scatters, counters,
// log) is read from the workgroup's LDS copy of the full descriptor.
struct StepCase {
  const GLOBAL uint2 *vox;
  const GLOBAL uint8_t *vox8;
  const GLOBAL float4 *mu_rho;
  const GLOBAL float *mu_max;
  // the workgroup's LDS copies of mu_rho and mu_max, or null (read mu_rho,
  // mu_max through the caches)
  const LOCAL float4 *tab;
  const LOCAL float *tabmax;
  const LOCAL float *tabbnd;
  // bound-test sums per material and energy cell (CaseDev::bnd)
  const GLOBAL float *bnd;
  GLOBAL unsigned long long *tally;
  float fnx, fny, fnz, inv_dx, inv_dy, inv_dz, e0, inv_de;
  int32_t nx, ny, ne, rayleigh, npal;
  // tally mode 2: the wave's LDS sub-tally (slot keys = voxel or -1, values);
  // null in modes 0 and 1
  LOCAL int32_t *ckeys;
  LOCAL unsigned long long *cvals;
  // bound grid of blocks of 2^bshift voxels per edge (ceil(n / 2^bshift)
  // blocks per axis); null: every tentative collision reads its voxel
  const GLOBAL uint8_t *bgrid;
  int32_t bshift;
  uint32_t key0, key1;
};

// Id of the XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ uint32_t xcc_id() {
  // hwreg(HW_REG_XCC_ID, 0, 16): read-only hardware register
  return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((16 - 1) << 11)) & 0xFu;
}

template <typename T>
__device__ __forceinline__ GLOBAL T *uniform_ptr(T *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (GLOBAL T *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int32_t uniform_i(int32_t x) {
  return __builtin_amdgcn_readfirstlane(x);
}

// tally_mode 0: the case's tally; 1, 2: this XCD's copy of it; cache: the
// wave's LDS sub-tally (mode 2) or null; bound_shift: the bound grid used
// (-1: none).
__device__ __forceinline__ StepCase make_step_case(const CaseDev &c, int tally_mode,
                                                   int bound_shift,
                                                   LOCAL unsigned char *cache) {
  StepCase s;
  s.bgrid = nullptr;
  s.bshift = 0;
  if (bound_shift >= 0 && c.bclass) {
    s.bgrid = uniform_ptr(c.bgrid[bound_shift]);
    s.bshift = bound_shift;
  }
  s.vox = uniform_ptr(c.vox);
  s.vox8 = uniform_ptr(c.vox8);
  s.npal = uniform_i(c.npal);
  s.mu_rho = uniform_ptr(c.mu_rho);
  s.tab = nullptr;
  s.tabmax = nullptr;
  s.tabbnd = nullptr;
  s.bnd = uniform_ptr(c.bnd);
  s.mu_max = uniform_ptr(c.mu_max);
  s.tally = uniform_ptr(c.tally);
  if (tally_mode) s.tally += (size_t)xcc_id() * (size_t)uniform_i((int32_t)c.V);
  s.cvals = (LOCAL unsigned long long *)cache;
  s.ckeys = cache ? (LOCAL int32_t *)(cache + kCacheSlots * 8) : nullptr;
  s.fnx = uniform_f(c.fnx);
  s.fny = uniform_f(c.fny);
  s.fnz = uniform_f(c.fnz);
  s.inv_dx = uniform_f(c.inv_dx);
  s.inv_dy = uniform_f(c.inv_dy);
  s.inv_dz = uniform_f(c.inv_dz);
  s.e0 = uniform_f(c.e0);
  s.inv_de = uniform_f(c.inv_de);
  s.nx = uniform_i(c.nx);
  s.ny = uniform_i(c.ny);
  s.ne = uniform_i(c.ne);
  s.rayleigh = uniform_i(c.rayleigh);
  s.key0 = (uint32_t)uniform_i((int32_t)c.key0);
  s.key1 = (uint32_t)uniform_i((int32_t)c.key1);
  return s;
}

__device__ __forceinline__ uint64_t lane0_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 0);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 0);
  return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------ lane state

// Per-wave event counters in LDS (one slot of ACC_COUNT words per wave),
// bumped with LDS atomics when an event happens and added to the case's
// device counters when the wave switches case or exits.  Keeping them out of
// registers leaves room for more resident waves.
struct Counters {
  unsigned long long *s;
  __device__ __forceinline__ void add(int i, unsigned long long v) { atomicAdd(s + i, v); }
};

__device__ void flush(Counters &c, unsigned long long *acc, int lane, uint32_t refills) {
  if (lane == 0 && refills) c.add(ACC_N_REFILLS, refills);
  if (lane < ACC_COUNT) {
    const unsigned long long v = atomicExch(c.s + lane, 0ull);
    if (v) atomic_add_u64(acc + lane, v);
  }
}

// Device scope in every tally mode: a per-XCD copy is only updated by waves of
// its XCD, but those belong to many workgroups (on gfx950 both scopes give the
// same atomic instruction, performed at the memory side).
__device__ __forceinline__ void tally_add(const StepCase &S, int32_t vox, unsigned long long q) {
  __hip_atomic_fetch_add(S.tally + vox, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tally mode 2: add the wave's LDS sub-tally to the case's tally and empty it
// (called by the whole wave, before it changes case and at exit).
__device__ void flush_cache(const StepCase &S, int lane) {
  if (!S.ckeys) return;
  for (int i = lane; i < kCacheSlots; i += 64) {
    const int32_t key = S.ckeys[i];
    if (key >= 0) {
      const unsigned long long v = S.cvals[i];
      if (v) tally_add(S, key, v);
      S.ckeys[i] = -1;
      S.cvals[i] = 0ull;
    }
  }
  // the wave's later deposits (any lane) must see the emptied slots
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ void clear_cache(LOCAL unsigned char *cache, int lane) {
  LOCAL unsigned long long *v = (LOCAL unsigned long long *)cache;
  LOCAL int32_t *k = (LOCAL int32_t *)(cache + kCacheSlots * 8);
  for (int i = lane; i < kCacheSlots; i += 64) {
    v[i] = 0ull;
    k[i] = -1;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

struct Photon {
  float px, py, pz;   // position, voxel units
  float ux, uy, uz;   // unit direction
  float E;            // keV
  float mumax;        // majorant at E, cm^-1
  float sc;           // ln2 / mumax
  float we;           // energy-grid weight
  int je;             // energy-grid cell
  uint32_t hlo, hhi;  // history id
  uint32_t k;         // random pairs taken (MACRO tracking: flights), flag bits
  uint32_t seq;       // event sequence (debug log only)
  uint32_t ks;        // Woodcock steps taken (debug log only)
  // MACRO tracking: a flight (optical depth tau to spend) may span several
  // calls; its random words for the collision and its current cell persist
  float tau;            // < 0: no flight in progress
  uint32_t ry, rz, rw;
  uint32_t cell;        // x | y << 10 | z << 20; all ones: take it from the position
};

// Photon.k: in the low bits the random pairs the photon has taken (global
// majorant) or its flights (MACRO tracking), kScatBit once the photon has
// scattered, kGoneBit while an escaped photon's counters wait for the wave's
// next refill step (deferred collisions), kDueBit while a scatter selected
// at a block's second pair waits for the next block (plain steps; the
// voxel, material and process wait in the lane's LDS slot).
constexpr uint32_t kScatBit = 0x80000000u;
constexpr uint32_t kGoneBit = 0x40000000u;
constexpr uint32_t kDueBit = 0x20000000u;
constexpr uint32_t kStepMask = 0x1FFFFFFFu;

// mu/rho rows ti and ti + 1 (energy nodes je, je + 1 of one material): from
// the workgroup's LDS copy (TAB) or through the caches.
template <bool TAB>
__device__ __forceinline__ void table_rows(const StepCase &S, uint32_t ti, float4 &t0, float4 &t1) {
  if constexpr (TAB) {
    t0 = S.tab[ti];
    t1 = S.tab[ti + 1];
  } else {
    t0 = S.mu_rho[ti];
    t1 = S.mu_rho[ti + 1];
  }
}

// Bound-test sum of material m in energy cell j (CaseDev::bnd).
template <bool TAB>
__device__ __forceinline__ float bound_sum(const StepCase &S, uint32_t m, int j) {
  const uint32_t i = __umul24(m, (uint32_t)(S.ne - 1)) + (uint32_t)j;
  if constexpr (TAB) return S.tabbnd[i];
  else return S.bnd[i];
}

template <bool TAB>
__device__ __forceinline__ void set_energy(Photon &p, const StepCase &S, float E) {
  p.E = E;
  const float f = (E - S.e0) * S.inv_de;
  const int j = min(max((int)f, 0), S.ne - 2);
  p.je = j;
  p.we = f - (float)j;
  if constexpr (TAB)
    p.mumax = lerpf(S.tabmax[j], S.tabmax[j + 1], p.we);
  else
    p.mumax = lerpf(S.mu_max[j], S.mu_max[j + 1], p.we);
  p.sc = 0.69314718055994531f * __builtin_amdgcn_rcpf(p.mumax);
}

// Direction after deflection cos(theta) = mu and azimuth 2 pi t (t in turns).
__device__ __forceinline__ void rotate(Photon &p, float mu, float t) {
  const float st = __builtin_amdgcn_sqrtf(fmaxf(0.0f, (1.0f - mu) * (1.0f + mu)));
  const float sp = sin_turns(t), cp = cos_turns(t);
  const float u = p.ux, v = p.uy, w = p.uz;
  float nu, nv, nw;
  if (fabsf(w) < 1.0f - 1e-5f) {
    const float r = __builtin_amdgcn_sqrtf((1.0f - w) * (1.0f + w));
    const float g = st * __builtin_amdgcn_rcpf(r);
    nu = fmaf(u, mu, g * (u * w * cp - v * sp));
    nv = fmaf(v, mu, g * (v * w * cp + u * sp));
    nw = fmaf(w, mu, -st * cp * r);
  } else {
    nu = st * cp;
    nv = st * sp;
    nw = w >= 0.0f ? mu : -mu;
  }
  const float n = rsqrtf(nu * nu + nv * nv + nw * nw);
  p.ux = nu * n;
  p.uy = nv * n;
  p.uz = nw * n;
}

template <bool LOG>
__device__ __forceinline__ void log_event(const CaseDev &G, Photon &p, int type, int64_t vox,
                                          float e, float Eafter) {
  if (!LOG) return;
  const uint64_t h = ((uint64_t)p.hhi << 32) | p.hlo;
  if (h < G.log_h0 || h >= G.log_h1) return;
  const unsigned long long idx = atomicAdd(G.log_n, 1ull);
  if (idx < G.log_cap) {
    ctd_event ev;
    ev.h = h;
    ev.seq = p.seq;
    ev.k = p.ks;
    ev.type = type;
    ev.reserved = 0;
    ev.vox = vox;
    ev.e = e;
    ev.E = Eafter;
    G.log[idx] = ev;
  }
  p.seq += 1;
}

// Exact tally update: e is a multiple of 2^-24 keV, so q = e * 2^24 is an
// integer (< 2^32 for e < 256 keV) and the int64 sum is exact in any order.
template <bool LOG>
__device__ __forceinline__ void deposit(const StepCase &S, const CaseDev &G, Photon &p,
                                        Counters &c, int32_t vox, float e, int type,
                                        float Eafter) {
  const uint32_t q = (uint32_t)(e * kQScale);
  if (q) {
    bool cached = false;
    if (S.ckeys) {
      // LDS sub-tally: the slot of vox belongs to the first voxel that took
      // it during this wave's case; other voxels go straight to the tally
      const uint32_t slot = ((uint32_t)vox * 2654435761u) >> (32 - kCacheBits);
      int32_t owner = S.ckeys[slot];
      if (owner == -1) {
        int32_t expected = -1;
        __hip_atomic_compare_exchange_strong(S.ckeys + slot, &expected, vox, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        owner = expected == -1 ? vox : expected;
      }
      if (owner == vox) {
        __hip_atomic_fetch_add(S.cvals + slot, (unsigned long long)q, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
        cached = true;
      }
    }
    if (!cached) tally_add(S, vox, q);
    c.add(ACC_Q_DEP, q);
  }
  c.add(ACC_N_DEPOSITS, 1);
  log_event<LOG>(G, p, type, vox, e, Eafter);
}

// Source photon of history h from spectrum bin j (Sec. 2.2.5-2.2.6): its
// entry point into the voxel box (voxel units) and energy in pe, its unit
// direction in dir.xyz; returns false when the ray misses the box (the photon
// escapes at once).  Its start event is logged here (event 0 of the history).
template <bool LOG>
__device__ bool source(const StepCase &S, const CaseDev &G, uint64_t h, int j,
                       const int32_t *__restrict__ mh_beam, uint64_t local, Counters &c,
                       float4 &pe, float4 &dir) {
  Photon p;   // only the history id and log fields are used here
  p.hlo = (uint32_t)h;
  p.hhi = (uint32_t)(h >> 32);
  p.seq = 0;
  p.ks = 0;
  const uint4 r = philox10(0u, p.hlo, p.hhi, 0u, S.key0, S.key1);
  const float E = fmaf(unif(r.x), G.bin_width, G.bin_lo[j]);
  float sx, sy, sz, dx, dy, dz;
  int beamlet = -1;
  if (G.kind == CTD_GEOM_PENCIL) {
    sx = G.src[0]; sy = G.src[1]; sz = G.src[2];
    dx = G.dir[0]; dy = G.dir[1]; dz = G.dir[2];
  } else {
    float sp, cp, zoff;
    if (G.nproj > 0) {
      // exact in double: 24-bit uniform times an integer < 2^31
      int pi = (int)((double)unif(r.y) * (double)G.nproj);
      pi = min(pi, G.nproj - 1);
      const float4 sc = G.proj_sc[pi];
      sp = sc.x;
      cp = sc.y;
      zoff = sc.z;
    } else {
      const float rel = unif(r.y) * G.arc_turns;     // turns since phi0
      const float t = rel + G.phi0_turns;
      sp = sin_turns(t);
      cp = cos_turns(t);
      zoff = G.z_feed * rel;
    }
    sx = fmaf(G.sad, sp, G.iso[0]);
    sy = fmaf(G.sad, cp, G.iso[1]);
    sz = G.iso[2] + zoff;
    float a, b;
    if (G.fl_n > 0) {
      int I;
      if (G.fl_chains > 0) {
        I = mh_beam[local];               // Alg. A1 chain step of this history
      } else {
        // beamlet I = min{I : C_I > u F}, decided in FP64 (exact inputs: u has
        // 24 bits, k / 2^gbits <= u exactly, so the guide entry is a lower bound)
        const uint4 r2 = philox10(0u, p.hlo, p.hhi, 1u, S.key0, S.key1);
        const double u = (double)unif(r2.x);
        const double x = u * G.fl_total;
        I = G.fl_guide[(int)(u * (double)(1 << G.fl_gbits))];
        while (I < G.fl_n - 1 && G.fl_cdf[I] <= x) ++I;
      }
      const int ib = I / G.fl_na;
      const int ia = I - ib * G.fl_na;
      a = fmaf((float)ia + unif(r.z), G.fl_da, G.a0);
      b = fmaf((float)ib + unif(r.w), G.fl_db, G.b0);
      beamlet = I;
    } else {
      a = fmaf(unif(r.z), G.a1 - G.a0, G.a0);
      b = fmaf(unif(r.w), G.b1 - G.b0, G.b0);
    }
    const float Px = fmaf(a, cp, G.iso[0]);
    const float Py = fmaf(-a, sp, G.iso[1]);
    const float Pz = sz + b;
    const float vx = Px - sx, vy = Py - sy, vz = Pz - sz;
    const float inv = rsqrtf(vx * vx + vy * vy + vz * vz);
    dx = vx * inv; dy = vy * inv; dz = vz * inv;
  }
  c.add(ACC_N_HIST, 1);
  c.add(ACC_Q_INC, (uint32_t)(E * kQScale));
  log_event<LOG>(G, p, 0, beamlet, E, E);
  // slab entry into the box [0, n) in voxel units
  const float Sv[3] = {(sx - G.ox) * S.inv_dx, (sy - G.oy) * S.inv_dy, (sz - G.oz) * S.inv_dz};
  const float D[3] = {dx * S.inv_dx, dy * S.inv_dy, dz * S.inv_dz};
  const float N[3] = {S.fnx, S.fny, S.fnz};
  float tn = -INFINITY, tf = INFINITY;
  bool miss = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (D[a] == 0.0f) {
      miss |= (Sv[a] < 0.0f) | (Sv[a] > N[a]);
    } else {
      const float inv = __builtin_amdgcn_rcpf(D[a]);
      const float t1 = (0.0f - Sv[a]) * inv, t2 = (N[a] - Sv[a]) * inv;
      tn = fmaxf(tn, fminf(t1, t2));
      tf = fminf(tf, fmaxf(t1, t2));
    }
  }
  const float tin = fmaxf(tn, 0.0f);
  if (miss || !(tin < tf)) {
    c.add(ACC_N_MISS, 1);
    c.add(ACC_Q_ESC, (uint32_t)(E * kQScale));
    log_event<LOG>(G, p, 6, -1, E, E);
    return false;
  }
  // entry point, kept inside [0, n) against rounding
  // (+ 0.0f turns a -0 into +0 and leaves every other value as it is; a
  // step's fma from a position that is not -0 never gives -0, so positions
  // are never -0: see inside_box)
  pe.x = fminf(fmaxf(fmaf(tin, D[0], Sv[0]), 0.0f), __int_as_float(__float_as_int(N[0]) - 1)) + 0.0f;
  pe.y = fminf(fmaxf(fmaf(tin, D[1], Sv[1]), 0.0f), __int_as_float(__float_as_int(N[1]) - 1)) + 0.0f;
  pe.z = fminf(fmaxf(fmaf(tin, D[2], Sv[2]), 0.0f), __int_as_float(__float_as_int(N[2]) - 1)) + 0.0f;
  pe.w = E;
  dir.x = dx; dir.y = dy; dir.z = dz;
  return true;
}

// The photon leaves the voxel box with its energy.
template <bool LOG>
__device__ __forceinline__ bool escape(Photon &p, const CaseDev &G, Counters &c, uint32_t k) {
  c.add(ACC_N_STEPS, k);
  c.add(ACC_N_ESCAPES, 1);
  if (!(p.k & kScatBit)) c.add(ACC_N_UNSCATTERED, 1);
  c.add(ACC_Q_ESC, (uint32_t)(p.E * kQScale));
  log_event<LOG>(G, p, 5, -1, p.E, p.E);
  return false;
}

// Outcome of the selection at a tentative collision; kSelPhoto and kSelDone
// end the photon.
constexpr int kSelFict = 0, kSelCompton = 1, kSelRayleigh = 2, kSelPhoto = 3, kSelDone = 4;

// Selection at a tentative collision (Sec. 2.1) in voxel vox of density rho,
// given the mass attenuation coefficients (a, b, cr) = (photoelectric,
// Compton, Rayleigh) interpolated at E and xi = u1 * the majorant:
// photoelectric, Compton, Rayleigh or fictitious by comparing xi with the
// cumulative sums in that order.  A photoelectric absorption deposits E
// locally here; nsteps is what the photon adds to the step counter when it
// ends.
template <bool LOG>
__device__ __forceinline__ int select_process(Photon &p, const StepCase &S, const CaseDev &G,
                                              Counters &c, int32_t vox, float rho, float a,
                                              float b, float cr, float xi, uint32_t nsteps) {
  const float mpe = rho * a;
  const float c1 = mpe + rho * b;
  if (xi < mpe) {  // photoelectric: absorb, deposit E locally
    c.add(ACC_N_STEPS, nsteps);
    c.add(ACC_N_PHOTO, 1);
    deposit<LOG>(S, G, p, c, vox, p.E, 1, 0.0f);
    return kSelPhoto;
  }
  if (xi < c1) return kSelCompton;
  if (S.rayleigh) {
    const float c2 = c1 + rho * cr;
    if (xi < c2) return kSelRayleigh;
  }
  return kSelFict;
}

// Tentative collision at voxel vox against majorant mumax with selection
// word ry: read the voxel (1-byte palette index or 8-byte record) and its
// table rows, then select; m receives the voxel's material.
template <bool LOG, bool TAB>
__device__ __forceinline__ int select_at(Photon &p, const StepCase &S, const CaseDev &G,
                                         const LOCAL uint2 *pal, Counters &c, int32_t vox,
                                         uint32_t ry, float mumax, uint32_t nsteps,
                                         uint32_t &m) {
  uint32_t rbits;
  if (S.npal) {  // 1-byte index into the workgroup's LDS palette
    const uint32_t i8 = S.vox8[vox];
    rbits = pal[i8].x;
    m = pal[i8].y;
  } else {
    const uint2 rec = S.vox[vox];
    rbits = rec.x;
    m = rec.y;
  }
  const uint32_t ti = __umul24(m, (uint32_t)S.ne) + (uint32_t)p.je;
  float4 t0, t1;
  table_rows<TAB>(S, ti, t0, t1);
  const float a = lerpf(t0.x, t1.x, p.we), b = lerpf(t0.y, t1.y, p.we);
  const float cr = S.rayleigh ? lerpf(t0.z, t1.z, p.we) : 0.0f;
  return select_process<LOG>(p, S, G, c, vox, __uint_as_float(rbits), a, b, cr,
                             unif(ry) * mumax, nsteps);
}

// Compton (sel = kSelCompton, Sec. 2.2.3) or Rayleigh (Sec. 2.2.2) scatter in
// voxel vox of material m: the polar angle from the process's surface at
// uniform w0, the azimuth from w1; returns false when the photon is done
// (Compton below the cutoff).  nsteps as in select_process.
template <bool LOG, bool TAB>
__device__ __forceinline__ bool scatter(Photon &p, const StepCase &S, const CaseDev &G,
                                        Counters &c, int sel, int32_t vox, uint32_t m,
                                        uint32_t w0, uint32_t w1, uint32_t nsteps) {
  p.k |= kScatBit;
  if (sel == kSelCompton) {
    c.add(ACC_N_COMPTON, 1);
    // surface fields from the workgroup's LDS copy of the case (read only here)
    const int nzc = G.nzc;
    const GLOBAL float4 *Q = (const GLOBAL float4 *)G.comp_quad;
    if (G.comp_per_mat) Q += (size_t)m * (size_t)(S.ne - 1) * (size_t)(nzc - 1);
    const float mu = surface(Q, nzc, p.je, p.we, unif(w0));
    const float E = p.E;
    const float Ep = E * __builtin_amdgcn_rcpf(fmaf(E * kInvMeC2, 1.0f - mu, 1.0f));
    deposit<LOG>(S, G, p, c, vox, E - Ep, 2, Ep);  // exact: Ep > E/2 (Sterbenz)
    rotate(p, mu, unif(w1));
    set_energy<TAB>(p, S, Ep);
    if (Ep < G.e_cut) {
      c.add(ACC_N_STEPS, nsteps);
      c.add(ACC_N_CUTOFF, 1);
      deposit<LOG>(S, G, p, c, vox, Ep, 4, 0.0f);
      return false;
    }
    return true;
  }
  c.add(ACC_N_RAYLEIGH, 1);
  const int nzr = G.nzr;
  const GLOBAL float4 *Q =
      (const GLOBAL float4 *)G.rayl_quad + (size_t)m * (size_t)(S.ne - 1) * (size_t)(nzr - 1);
  const float mu = surface(Q, nzr, p.je, p.we, unif(w0));
  rotate(p, mu, unif(w1));
  log_event<LOG>(G, p, 3, vox, 0.0f, p.E);
  return true;
}

// 0 <= position < n on each axis, as one unsigned compare of the float bits.
// Positions are never -0 (the entry point is made +0, and a step's fma
// x + s d from an x that is not -0 cannot give -0); for the other floats the
// bits of non-negative values order like the values, while negative values,
// infinities and NaNs (sign bit set, or exponent all ones) compare above
// every finite positive bound -- outside, as the two float compares say.
__device__ __forceinline__ bool inside_box(const Photon &p, const StepCase &S) {
  return (__float_as_uint(p.px) < __float_as_uint(S.fnx)) &
         (__float_as_uint(p.py) < __float_as_uint(S.fny)) &
         (__float_as_uint(p.pz) < __float_as_uint(S.fnz));
}

// Step guard of the global-majorant steps, checked once per block: a photon
// that has taken kStepGuard pairs stops (a runaway history, which
// ctd_read_balance reports as an error); returns false then.
__device__ __forceinline__ bool guard_ok(const Photon &p, Counters &c) {
  const uint32_t P = p.k & kStepMask;
  if (P < kStepGuard) return true;
  c.add(ACC_STEP_GUARD, 1);
  c.add(ACC_N_STEPS, P);
  return false;
}

// Random words of the global-majorant steps: the history's transport blocks
// are read two words (a pair) at a time in order; pair P (the low bits of
// Photon.k count the pairs taken) is words 2 (P mod 2), 2 (P mod 2) + 1 of
// block P / 2 + 1.  A step takes a pair (free path, selection), a Compton or
// Rayleigh scatter the pair after its step (polar angle, azimuth).
__device__ __forceinline__ uint4 pair_block(const Photon &p, const StepCase &S, uint32_t P) {
  return philox10((P >> 1) + 1u, p.hlo, p.hhi, 0u, S.key0, S.key1);
}

// One Woodcock step (Sec. 2.1) against the global majorant with words w0
// (free path) and w1 (selection), the tentative collision read from its voxel
// (cases with a bound grid take step_fast and the collision passes instead).
// Returns the selection; a Compton or Rayleigh scatter is left to the
// caller, with the voxel and its material in vox and m.  The caller applies
// the step guard, once per block.
template <bool LOG, bool TAB>
__device__ __forceinline__ int step(Photon &p, const StepCase &S, const CaseDev &G,
                                    const LOCAL uint2 *pal, Counters &c, uint32_t w0,
                                    uint32_t w1, int32_t &vox, uint32_t &m) {
  const uint32_t P = p.k & kStepMask;
  p.k += 1;
  if (LOG) p.ks += 1;
  const float s = -__log2f(unif(w0)) * p.sc;  // -ln(u) / mu_max
  p.px = fmaf(s, p.ux * S.inv_dx, p.px);
  p.py = fmaf(s, p.uy * S.inv_dy, p.py);
  p.pz = fmaf(s, p.uz * S.inv_dz, p.pz);
  const bool inside = inside_box(p, S);
  if (!inside) {
    escape<LOG>(p, G, c, P + 1u);
    return kSelDone;
  }
  const uint32_t ix = (uint32_t)p.px, iy = (uint32_t)p.py, iz = (uint32_t)p.pz;
  vox = (int32_t)__umul24(__umul24(iz, (uint32_t)S.ny) + iy, (uint32_t)S.nx) + (int32_t)ix;
  return select_at<LOG, TAB>(p, S, G, pal, c, vox, w1, p.mumax, P + 1u, m);
}

// One Woodcock step with deferred collisions (bound grid present), words w0
// (free path) and w1 (selection): the fast part of step() -- free path,
// move, exit test and the bound-grid rejection of fictitious collisions --
// for every live lane of the wave, leaving the rest to the wave's next
// collision pass.  Returns kStepOn (fictitious, decided by the bound),
// kStepPending (a tentative collision at *pvox that needs the voxel; w1 is
// kept in the lane's LDS word *u1 for the pass, which reads the voxel and
// selects as step() does) or kStepGone (left the box: kGoneBit set, its
// counters added at the next refill step).  The caller applies the step
// guard, once per block.
constexpr int kStepOn = 0, kStepPending = 1, kStepGone = 2;

template <bool LOG, bool TAB>
__device__ __forceinline__ int step_fast(Photon &p, const StepCase &S, const LOCAL uint2 *cls_tab,
                                         const GLOBAL uint8_t *bgrid, int32_t &pvox,
                                         LOCAL uint32_t *u1, uint32_t w0, uint32_t w1) {
  p.k += 1;
  if (LOG) p.ks += 1;
  const float s = -__log2f(unif(w0)) * p.sc;  // -ln(u) / mu_max
  p.px = fmaf(s, p.ux * S.inv_dx, p.px);
  p.py = fmaf(s, p.uy * S.inv_dy, p.py);
  p.pz = fmaf(s, p.uz * S.inv_dz, p.pz);
  const bool inside = inside_box(p, S);
  if (!inside) {
    p.k |= kGoneBit;
    return kStepGone;
  }
  const uint32_t ix = (uint32_t)p.px, iy = (uint32_t)p.py, iz = (uint32_t)p.pz;
  const int32_t vox = (int32_t)__umul24(__umul24(iz, (uint32_t)S.ny) + iy, (uint32_t)S.nx) +
                      (int32_t)ix;
  const uint32_t e = (1u << S.bshift) - 1u;
  const uint32_t bgx = ((uint32_t)S.nx + e) >> S.bshift, bgy = ((uint32_t)S.ny + e) >> S.bshift;
  const uint32_t blk = __umul24(__umul24(iz >> S.bshift, bgy) + (iy >> S.bshift), bgx) +
                       (ix >> S.bshift);
  const uint32_t cls = bgrid[blk];
  if (cls != kMixedClass) {
    const uint2 ce = cls_tab[cls];
    const float rho_c = __uint_as_float(ce.x);
    if (unif(w1) * p.mumax >= rho_c * bound_sum<TAB>(S, ce.y, p.je)) return kStepOn;
  }
  pvox = vox;
  *u1 = w1;
  return kStepPending;
}

// Woodcock tracking with the macro-cell majorant (MACRO tracking).  A flight
// draws its random block (step k) and spends the optical depth tau = -ln(u0)
// cell by cell along the ray; a boundary crossing draws no random number.  A
// call takes at most kMacroCrossings cells and then hands the flight on to
// the next call (tau, the block's remaining words and the cell are kept in
// the photon), so the lanes of a wave advance in similar strides instead of
// all waiting for the longest flight.  Termination: a flight's cell index
// moves one cell per crossing along the direction of travel, so it leaves the
// grid or collides within the cells per axis summed; every call takes at
// least one crossing or ends the flight.
constexpr int kMacroCrossings = 4;

template <bool LOG, bool TAB>
__device__ __forceinline__ bool step_macro(Photon &p, const StepCase &S, const CaseDev &G,
                                           const LOCAL uint2 *pal, Counters &c) {
  if (p.tau < 0.0f) {  // a new flight
    p.k += 1;
    if (LOG) p.ks += 1;
    const uint32_t k0 = p.k & kStepMask;
    if (k0 > kStepGuard) {
      c.add(ACC_STEP_GUARD, 1);
      c.add(ACC_N_STEPS, k0);
      return false;
    }
    const uint4 r = philox10(k0, p.hlo, p.hhi, 0u, S.key0, S.key1);
    p.tau = -__log2f(unif(r.x)) * 0.69314718055994531f;
    p.ry = r.y;
    p.rz = r.z;
    p.rw = r.w;
    p.cell = 0xFFFFFFFFu;
  }
  const uint32_t k = p.k & kStepMask;
  float tau = p.tau;
  const int ncx = G.mc_nx, ncy = G.mc_ny, ncz = G.mc_nz;
  const float fcs = G.mc_fcs;
  const float Dx = p.ux * S.inv_dx, Dy = p.uy * S.inv_dy, Dz = p.uz * S.inv_dz;
  int cx, cy, cz;
  if (p.cell == 0xFFFFFFFFu) {
    cx = min(max((int)(p.px * G.mc_inv_cs), 0), ncx - 1);
    cy = min(max((int)(p.py * G.mc_inv_cs), 0), ncy - 1);
    cz = min(max((int)(p.pz * G.mc_inv_cs), 0), ncz - 1);
  } else {
    cx = (int)(p.cell & 1023u);
    cy = (int)((p.cell >> 10) & 1023u);
    cz = (int)(p.cell >> 20);
  }
  // the cell majorant factors of the photon's energy band
  const GLOBAL float *fband =
      (const GLOBAL float *)G.mc_f + (size_t)(p.je >> G.mc_shift) * (size_t)G.mc_ncell;
  // per axis, fixed for the call: the face the ray leaves a cell by, the
  // index step, 1/D, and whether the ray moves along the axis at all
  const bool fx = Dx > 0.0f, fy = Dy > 0.0f, fz = Dz > 0.0f;
  const bool mx = Dx != 0.0f, my = Dy != 0.0f, mz = Dz != 0.0f;
  const float rx = __builtin_amdgcn_rcpf(Dx), ry = __builtin_amdgcn_rcpf(Dy),
              rz = __builtin_amdgcn_rcpf(Dz);
  uint32_t crossings = 0;
  float mu_c = 0.0f;
  bool hit = false, out = false;
#pragma unroll
  for (int it = 0; it < kMacroCrossings; ++it) {
    mu_c = fband[(cz * ncy + cy) * ncx + cx] * p.mumax;
    const float x0 = (float)cx * fcs, y0 = (float)cy * fcs, z0 = (float)cz * fcs;
    const float bx = fx ? fminf(x0 + fcs, S.fnx) : x0;
    const float by = fy ? fminf(y0 + fcs, S.fny) : y0;
    const float bz = fz ? fminf(z0 + fcs, S.fnz) : z0;
    const float tx = mx ? fmaxf((bx - p.px) * rx, 0.0f) : INFINITY;
    const float ty = my ? fmaxf((by - p.py) * ry, 0.0f) : INFINITY;
    const float tz = mz ? fmaxf((bz - p.pz) * rz, 0.0f) : INFINITY;
    const float d = fminf(tx, fminf(ty, tz));
    if (tau < mu_c * d) {  // tentative collision inside this cell
      hit = true;
      break;
    }
    tau -= mu_c * d;
    p.px = fmaf(d, Dx, p.px);
    p.py = fmaf(d, Dy, p.py);
    p.pz = fmaf(d, Dz, p.pz);
    ++crossings;
    // the nearest face, ties to x then y (no branches: one index moves)
    const bool ax = tx <= ty && tx <= tz;
    const bool ay = !ax && ty <= tz;
    cx += ax ? (fx ? 1 : -1) : 0;
    cy += ay ? (fy ? 1 : -1) : 0;
    cz += (!ax && !ay) ? (fz ? 1 : -1) : 0;
    out = (unsigned)cx >= (unsigned)ncx || (unsigned)cy >= (unsigned)ncy ||
          (unsigned)cz >= (unsigned)ncz;
    if (out) break;
  }
  if (crossings) c.add(ACC_N_CROSS, crossings);
  if (out) {
    p.tau = -1.0f;
    return escape<LOG>(p, G, c, k);
  }
  if (!hit) {  // the flight goes on in the next call, from this cell
    p.tau = tau;
    p.cell = (uint32_t)cx | ((uint32_t)cy << 10) | ((uint32_t)cz << 20);
    return true;
  }
  p.tau = -1.0f;
  const float s = tau * __builtin_amdgcn_rcpf(mu_c);
  p.px = fmaf(s, Dx, p.px);
  p.py = fmaf(s, Dy, p.py);
  p.pz = fmaf(s, Dz, p.pz);
  // the voxel is taken inside the current cell, whose majorant bounds it
  const int cs = G.mc_cs;
  const int ix = min(max((int)p.px, cx * cs), min(cx * cs + cs, S.nx) - 1);
  const int iy = min(max((int)p.py, cy * cs), min(cy * cs + cs, S.ny) - 1);
  const int iz = min(max((int)p.pz, cz * cs), min(cz * cs + cs, (int)S.fnz) - 1);
  const int32_t vox = (int32_t)__umul24(__umul24((uint32_t)iz, (uint32_t)S.ny) + (uint32_t)iy,
                                         (uint32_t)S.nx) + ix;
  uint32_t m;
  const int sel = select_at<LOG, TAB>(p, S, G, pal, c, vox, p.ry, mu_c, k, m);
  if (sel == kSelFict) return true;
  if (sel == kSelPhoto) return false;
  return scatter<LOG, TAB>(p, S, G, c, sel, vox, m, p.rz, p.rw, k);
}

// ------------------------------------------------------- transport kernel

__device__ __forceinline__ int find_bin(const unsigned long long *__restrict__ prefix, int nbins,
                                        uint64_t local) {
  int lo = 0, hi = nbins - 1;
  while (lo < hi) {  // last bin with prefix[bin] <= local
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= local) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Chunks of round case c, reloaded from the launch table where needed
// rather than kept live across the step loop.
__device__ __forceinline__ uint64_t case_chunk_count(const RoundCase *__restrict__ rcs, int nrc,
                                                     uint64_t total_chunks, int c) {
  return (c + 1 < nrc ? rcs[c + 1].chunk_begin : total_chunks) - rcs[c].chunk_begin;
}

// The home case of workgroup g: the last case whose home workgroups start
// at or before g.
__device__ __forceinline__ int home_case(const RoundCase *__restrict__ rcs, int nrc, uint32_t g) {
  int lo = 0, hi = nrc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rcs[mid].wg_lo <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static_assert(sizeof(CaseDev) % 4 == 0 && sizeof(CaseDev) <= 512, "CaseDev copy size");

// Copy a case descriptor (and its voxel palette, or else its bound-grid class
// table, if any) into the workgroup's LDS (threads copy words; the caller's
// barrier publishes them).
__device__ __forceinline__ void stage_case(CaseDev *dst, uint2 *pal, const CaseDev *src) {
  const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
  uint32_t *d = reinterpret_cast<uint32_t *>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(CaseDev) / 4); i += blockDim.x) d[i] = s[i];
  const uint2 *sp = src->palette;
  const uint2 *sc = src->bclass;
  if (__builtin_amdgcn_readfirstlane(src->npal) > 0)
    for (int i = threadIdx.x; i < 256; i += blockDim.x) pal[i] = sp[i];
  else if (sc)
    for (int i = threadIdx.x; i < 256; i += blockDim.x) pal[i] = sc[i];
}

// KIND selects the step for every case of the launch (kStepPlain,
// kStepDeferred, kStepMacro; a round whose cases need different steps is
// split into one launch per step), so each instance carries only its own
// step's registers and a tight loop of its steps between refills.  Every
// instance is held to 96 VGPRs (5 waves per SIMD): the global steps fit
// without spilling, the macro-cell step spills a few words outside its cell
// walk and gains more from the fifth wave hiding its dependent cell/majorant
// loads than the spills cost.
template <bool LOG, int KIND, bool TAB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(5))) k_transport(const RoundCase *__restrict__ rcs, int nrc,
                                                   uint64_t total_chunks,
                                                   unsigned long long *chunk_ctr, int refill_min,
                                                   int chunk, int tally_mode, int bound_shift,
                                                   int defer_min, int tab_n, int tab_ne,
                                                   int stash_cap) {
  extern __shared__ unsigned long long dyn_lds[];   // layout: see kWgSlotsOff
  const int lane = __lane_id();
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned char *base = (unsigned char *)dyn_lds;
  int *wg_next = (int *)base;   // the workgroup's next case (header word)
  CaseDev &G = *(CaseDev *)(base + kWgCaseOff);
  uint2 *pal = (uint2 *)(base + kWgPalOff);
  const LOCAL uint2 *pal_lds = (const LOCAL uint2 *)pal;
  unsigned char *slot = base + kWgSlotsOff + w * kWaveSlotBytes;
  unsigned char *after_slots = base + kWgSlotsOff + nw * kWaveSlotBytes;
  LOCAL uint2 *lane_word = (LOCAL uint2 *)(slot + kWaveAccBytes) + lane;
  // staged tables: the majorant nodes and mu/rho rows of the workgroup's
  // current case and its bound-test sums, shared by its waves (room for the
// round's largest case)
  LOCAL float *tabmax = nullptr;
  LOCAL float4 *tab = nullptr;
  LOCAL float *tabbnd = nullptr;
  unsigned char *after_cache = after_slots + (tally_mode == 2 ? nw * kCacheBytesPerWave : 0);
  LOCAL float4 *st_a = (LOCAL float4 *)(after_cache + w * stash_cap * kStashRecBytes);
  LOCAL float4 *st_b = st_a + stash_cap;
  if (TAB) {
    tabmax = (LOCAL float *)(after_cache + nw * stash_cap * kStashRecBytes);
    tab = (LOCAL float4 *)(tabmax + ((tab_ne + 3) & ~3));
    tabbnd = (LOCAL float *)(tab + tab_n);
  }

  Counters cnt;
  cnt.s = (unsigned long long *)slot;
  if (lane < ACC_COUNT) cnt.s[lane] = 0ull;
  LOCAL unsigned char *cache =
      tally_mode == 2 ? (LOCAL unsigned char *)after_slots + w * kCacheBytesPerWave : nullptr;
  if (cache) clear_cache(cache, lane);

  // Workgroup g starts on its home case (RoundCase::wg_lo: the case holding
  // chunk g * waves of the round).  The home waves of a case take its first
  // chunks by rank, with no atomic (the launch does not start with every
  // wave queueing on one address); every later claim of case c is
  // home_waves(c) + atomicAdd(counter c).  When a case has no chunk left,
  // the workgroup's waves drain, and the workgroup moves on together to the
  // next case (cyclically) that still has chunks, restaging its tables; it
  // exits when none has.  Results do not depend on this order: each history
  // is a function of its id, and the tallies are exact integer sums.
  int c = home_case(rcs, nrc, blockIdx.x);
  bool home = true;
  StepCase S;
  uint64_t pool_next = 0, pool_end = 0;  // local history indices of case c
  int wbin = 0;                          // bin of pool_next
  // the stash: records [st_pos, st_n) are sources not yet handed out, of the
  // histories st_base + their offsets
  uint64_t st_base = 0;
  uint32_t st_pos = 0, st_n = 0;
  bool first = true, claims_done = false;
  uint32_t refills = 0;
  Photon p;
  p.k = 0;
  bool alive = false;
  int32_t pvox = -1;   // deferred collisions: voxel of the lane's pending collision
  for (;;) {
    if (TAB) {
      const CaseDev *cd = rcs[c].cd;
      const int n_rows = cd->nmat * cd->ne, n_e = cd->ne;
      const float4 *src = cd->mu_rho;
      const float *srcm = cd->mu_max;
      for (int i = threadIdx.x; i < n_rows; i += blockDim.x) tab[i] = src[i];
      for (int i = threadIdx.x; i < n_e; i += blockDim.x) tabmax[i] = srcm[i];
      const float *srcb = cd->bnd;
      const int n_b = cd->nmat * (n_e - 1);
      for (int i = threadIdx.x; i < n_b; i += blockDim.x) tabbnd[i] = srcb[i];
    }
    stage_case(&G, pal, rcs[c].cd);
    __syncthreads();   // case and tables staged before any wave steps
    pool_next = pool_end = 0;
    wbin = 0;
    st_pos = st_n = 0;
    first = true;
    claims_done = false;
    refills = 0;

    for (;;) {
      const unsigned long long dead = __ballot(!alive);
      const int ndead = __popcll(dead);
      if (ndead == 64 || ndead >= refill_min) {
        // counters of photons that left the box since the last refill step
        if (!alive && (p.k & kGoneBit)) {
          p.k &= ~kGoneBit;
          escape<LOG>(p, G, cnt, p.k & kStepMask);
        }
        // idle lanes take the stash's records in order, lowest lanes first;
        // an empty stash is refilled from the pool (a chunk of case c is
        // claimed when the pool is empty) with the sources of the pool's
        // next stash_cap ids, sampled by the whole wave at once
        const bool want = !alive;
        const uint32_t rank = (uint32_t)__popcll(dead & lt_mask);
        uint32_t filled = 0;
        for (;;) {
          if (st_pos < st_n) {
            const uint32_t take = min((uint32_t)ndead - filled, st_n - st_pos);
            if (want && rank >= filled && rank < filled + take) {
              const uint32_t i = st_pos + (rank - filled);
              const float4 a = st_a[i], b = st_b[i];
              const uint64_t h = rcs[c].h_begin + st_base + __float_as_uint(b.w);
              p.hlo = (uint32_t)h;
              p.hhi = (uint32_t)(h >> 32);
              p.k = 0;
              p.seq = LOG ? 1u : 0u;   // event 0 (the start) was logged at sampling
              p.ks = 0;
              p.tau = -1.0f;
              p.px = a.x; p.py = a.y; p.pz = a.z;
              p.ux = b.x; p.uy = b.y; p.uz = b.z;
              set_energy<TAB>(p, S, a.w);
              alive = true;
            }
            st_pos += take;
            filled += take;
            if (filled == (uint32_t)ndead) break;
          }
          while (pool_next >= pool_end && !claims_done) {
            uint64_t t;
            if (home && first) {
              t = (uint64_t)__builtin_amdgcn_readfirstlane(
                  (blockIdx.x - rcs[c].wg_lo) * (uint32_t)nw + (uint32_t)w);
            } else {
              unsigned long long a = 0;
              if (lane == 0) a = atomicAdd(chunk_ctr + c, 1ull);
              t = rcs[c].home_waves + lane0_u64(a);
            }
            if (t >= case_chunk_count(rcs, nrc, total_chunks, c)) {
              claims_done = true;
              break;
            }
            const uint64_t lo = t * (uint64_t)chunk;
            const uint64_t hi = min(lo + (uint64_t)chunk, rcs[c].n);
            // the wave's step constants at its first chunk; a wave's claims
            // of one case increase, so later bin searches start from the last
            if (first) {
              S = make_step_case(G, tally_mode, bound_shift, cache);
              S.tab = tab;
              S.tabmax = tabmax;
              S.tabbnd = tabbnd;
              wbin = find_bin(rcs[c].prefix, G.nbins, lo);
            }
            first = false;
            pool_next = lo;
            pool_end = hi;
          }
          if (pool_next >= pool_end) break;   // nothing left to hand out
          // sample: lane l takes pool id pool_next + l; the records of the
          // photons that enter the box are stored compacted, in id order
          const RoundCase &R = rcs[c];
          const uint32_t ng = (uint32_t)min((uint64_t)stash_cap, pool_end - pool_next);
          const uint64_t local = pool_next + (uint64_t)lane;
          bool ok = false;
          float4 pe, dir;
          if ((uint32_t)lane < ng) {
            int j = wbin;
            while (j + 1 < G.nbins && local >= R.prefix[j + 1]) ++j;
            ok = source<LOG>(S, G, R.h_begin + local, j, R.beamlets, local, cnt, pe, dir);
          }
          const unsigned long long okm = __ballot(ok);
          __builtin_amdgcn_wave_barrier();   // the last records were read
          if (ok) {
            const uint32_t i = (uint32_t)__popcll(okm & lt_mask);
            dir.w = __uint_as_float((uint32_t)lane);
            st_a[i] = pe;
            st_b[i] = dir;
          }
          __builtin_amdgcn_wave_barrier();   // records written before any lane reads them
          st_base = pool_next;
          st_pos = 0;
          st_n = (uint32_t)__popcll(okm);
          pool_next += ng;
          if (pool_next < pool_end) {
            while (wbin + 1 < G.nbins && pool_next >= R.prefix[wbin + 1]) ++wbin;
          }
        }
        if (filled > 0) refills += 1;
      }
      if (__ballot(alive) == 0ull) {
        // case c done for this wave
        if (claims_done && pool_next >= pool_end && st_pos >= st_n) break;
        continue;
      }
      if constexpr (KIND == kStepMacro) {
        // one call per pass of the loop: a tight loop of macro-cell calls
        // spills more than it saves
        if (alive) alive = step_macro<LOG, TAB>(p, S, G, pal_lds, cnt);
      } else if constexpr (KIND == kStepDeferred) {
        // collision pass: the pending tentative collisions of the wave, once
        // defer_min of them have gathered (or every live lane waits on one)
        const unsigned long long pm = __ballot(alive && pvox >= 0);
        if (pm && (__popcll(pm) >= defer_min || pm == __ballot(alive))) {
          if (alive && pvox >= 0) {
            // the step's selection word waited in the lane's LDS word
            const uint32_t P = p.k & kStepMask;
            uint32_t m;
            const int sel =
                select_at<LOG, TAB>(p, S, G, pal_lds, cnt, pvox, lane_word->y, p.mumax, P, m);
            if (sel == kSelPhoto) {
              alive = false;
            } else if (sel != kSelFict) {   // the scatter takes the next pair
              const uint4 q = pair_block(p, S, P);
              const bool odd = (P & 1u) != 0u;
              p.k += 1;
              alive = scatter<LOG, TAB>(p, S, G, cnt, sel, pvox, m, odd ? q.z : q.x,
                                        odd ? q.w : q.y, P + 1u);
            }
            pvox = -1;
          }
        }
        // fast steps until a refill or a collision pass is due: a tight
        // loop in which a photon's direction, energy and tables stay put;
        // one block serves two steps (a photon at an odd pair takes one)
        for (;;) {
          if (alive && pvox < 0 && (alive = guard_ok(p, cnt))) {
            const uint32_t P = p.k & kStepMask;
            const uint4 r = pair_block(p, S, P);
            LOCAL uint32_t *u1 = &lane_word->y;
            // the bound grid's address into scalar registers once per block
            // (held in vector registers, it was re-read before every step)
            const GLOBAL uint8_t *bg = uniform_ptr(S.bgrid);
            int st = kStepOn;
            if ((P & 1u) == 0u) st = step_fast<LOG, TAB>(p, S, pal_lds, bg, pvox, u1, r.x, r.y);
            if (st == kStepOn) st = step_fast<LOG, TAB>(p, S, pal_lds, bg, pvox, u1, r.z, r.w);
            alive = st <= kStepPending;
          }
          const unsigned long long al = __ballot(alive);
          if (64 - __popcll(al) >= refill_min) break;
          const unsigned long long pw = __ballot(alive && pvox >= 0);
          if (pw && (__popcll(pw) >= defer_min || pw == al)) break;
        }
      } else {
        // steps until a refill is due, one block per pass of the loop: its
        // first pair takes a step (and its second pair that step's scatter)
        // or the scatter a photon left waiting; its second pair takes the
        // next step, whose scatter then waits for the next block.  A photon
        // starts every pass at an even pair.
        for (;;) {
          if (alive && (alive = guard_ok(p, cnt))) {
            const uint4 r = pair_block(p, S, p.k & kStepMask);
            int sel;
            int32_t vox = 0;
            uint32_t m = 0, w0 = r.z, w1 = r.w;
            if (p.k & kDueBit) {   // the waiting scatter takes the first pair
              const uint2 lw = *lane_word;
              vox = (int32_t)lw.x;
              m = lw.y & 0xFFFFu;
              sel = (int)(lw.y >> 16);
              p.k &= ~kDueBit;
              w0 = r.x;
              w1 = r.y;
            } else {
              sel = step<LOG, TAB>(p, S, G, pal_lds, cnt, r.x, r.y, vox, m);
            }
            if (sel == kSelCompton || sel == kSelRayleigh) {
              p.k += 1;
              alive = scatter<LOG, TAB>(p, S, G, cnt, sel, vox, m, w0, w1, p.k & kStepMask);
            } else if (sel >= kSelPhoto) {
              alive = false;
            }
            if (alive && (p.k & 1u)) {   // the block's second pair: a step
              sel = step<LOG, TAB>(p, S, G, pal_lds, cnt, r.z, r.w, vox, m);
              if (sel == kSelCompton || sel == kSelRayleigh) {
                *lane_word = make_uint2((uint32_t)vox, m | ((uint32_t)sel << 16));
                p.k |= kDueBit;
              } else if (sel >= kSelPhoto) {
                alive = false;
              }
            }
          }
          if (64 - __popcll(__ballot(alive)) >= refill_min) break;
        }
      }
    }
    if (!first) {   // the wave ran histories of case c
      flush(cnt, G.acc, lane, refills);
      flush_cache(S, lane);
    }
    // every wave of the workgroup has drained case c: pick the next case
    // with chunks left, scanning cyclically from c + 1 (c itself last)
    __syncthreads();
    if (threadIdx.x == 0) {
      int nxt = -1;
      for (int i = 1; i <= nrc && nxt < 0; ++i) {
        const int d = c + i < nrc ? c + i : c + i - nrc;
        const uint64_t taken =
            rcs[d].home_waves +
            __hip_atomic_load(chunk_ctr + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (taken < case_chunk_count(rcs, nrc, total_chunks, d)) nxt = d;
      }
      *wg_next = nxt;
    }
    __syncthreads();
    c = __builtin_amdgcn_readfirstlane(*wg_next);   // uniform: scalar from here on
    home = false;
    if (c < 0) break;
  }
}

// MACRO tracking set-up: per cell of cs^3 voxels and material, the largest
// density (float bits; densities are >= 0 so their bits order like values).
__global__ void __launch_bounds__(256) k_cell_max(const uint2 *__restrict__ vox, int nx, int ny,
                                                  int64_t V, int cs, int ncx, int ncy, int M,
                                                  unsigned int *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
    const uint2 rec = vox[v];
    if (rec.x == 0u || (int)rec.y >= M) continue;
    const int x = (int)(v % nx);
    const int64_t t = v / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
    const int64_t cell = ((int64_t)(z / cs) * ncy + y / cs) * ncx + x / cs;
    atomicMax(out + cell * M + rec.y, rec.x);
  }
}

// Bound grid: one lane per block of 2^shift voxels per edge.  A block whose
// voxels share one material m gets the first of m's density levels (ascending
// in cls[range[m].x ...]) that is at or above the block's largest density;
// the last level is m's largest density over the phantom, so one exists.
// Densities are >= 0 and sign-clear, so their bits order like their values.
__global__ void __launch_bounds__(256) k_block_class(const uint2 *__restrict__ vox, int nx, int ny,
                                                     int nz, int shift, int bx, int by,
                                                     int64_t nblocks,
                                                     const uint2 *__restrict__ cls,
                                                     const int2 *__restrict__ range,
                                                     uint8_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int B = 1 << shift;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblocks; b += stride) {
    const int x0 = (int)(b % bx) * B;
    const int64_t t = b / bx;
    const int y0 = (int)(t % by) * B, z0 = (int)(t / by) * B;
    const int x1 = min(x0 + B, nx), y1 = min(y0 + B, ny), z1 = min(z0 + B, nz);
    uint32_t m = vox[((int64_t)z0 * ny + y0) * nx + x0].y, rmax = 0u;
    bool mixed = false;
    for (int z = z0; z < z1; ++z)
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
          const uint2 r = vox[((int64_t)z * ny + y) * nx + x];
          mixed |= r.y != m;
          rmax = max(rmax, r.x);
        }
    uint32_t c = kMixedClass;
    if (!mixed) {
      const int2 rg = range[m];
      c = (uint32_t)(rg.x + rg.y - 1);
      for (int l = 0; l < rg.y; ++l)
        if (cls[rg.x + l].x >= rmax) {
          c = (uint32_t)(rg.x + l);
          break;
        }
    }
    out[b] = (uint8_t)c;
  }
}

// Alg. A1 (Metropolis-Hastings) on logical chains: lane c advances chain c
// over its histories h = c (mod C) of [h_begin, h_begin + n) in increasing h.
// Step of history h: trial J = floor(u0 N_f) and zeta = u1 from the second
// source block; move to J when zeta f_I < f_J (exact in FP64: 24-bit
// operands).  A chain's first history (h = c) starts from a beamlet drawn
// from the counter (0, c_lo, c_hi, 2).
__global__ void __launch_bounds__(256) k_mh_fill(const float *__restrict__ f, int n_f, int C,
                                                 uint64_t h_begin, uint64_t n, uint32_t key0,
                                                 uint32_t key1, int32_t *__restrict__ state,
                                                 int32_t *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const uint64_t Cu = (uint64_t)C;
  const uint64_t r = h_begin % Cu;
  uint64_t h = h_begin + (((uint64_t)c + Cu - r) % Cu);
  const uint64_t end = h_begin + n;
  if (h >= end) return;
  int I;
  if (h < Cu) {
    const uint4 r0 = philox10(0u, (uint32_t)c, 0u, 2u, key0, key1);
    I = min((int)((double)unif(r0.x) * (double)n_f), n_f - 1);
  } else {
    I = state[c];
  }
  double fI = (double)f[I];
  for (; h < end; h += Cu) {
    const uint4 r2 = philox10(0u, (uint32_t)h, (uint32_t)(h >> 32), 1u, key0, key1);
    const int J = min((int)((double)unif(r2.x) * (double)n_f), n_f - 1);
    const double fJ = (double)f[J];
    if ((double)unif(r2.y) * fI < fJ) {
      I = J;
      fI = fJ;
    }
    out[h - h_begin] = I;
  }
  state[c] = I;
}

// --------------------------------------------------------------- fold etc.

// S1 += T_b, S2 += T_b^2 (128-bit), T_b = 0 (Sec. 2.2.1 batch statistics);
// T_b is the exact sum of the ncopies per-XCD batch tallies.  Block 0 also
// folds the batch counters into their 128-bit totals; every block records
// the largest S1 and S2 high word it produced (overflow headroom).
__global__ void __launch_bounds__(256) k_fold(unsigned long long *__restrict__ T, int ncopies,
                                              long long *__restrict__ S1,
                                              unsigned long long *__restrict__ S2, int64_t V,
                                              unsigned long long *__restrict__ acc) {
  __shared__ unsigned long long m1[256], m2[256];
  if (blockIdx.x == 0 && threadIdx.x < ACC_COUNT) {
    const unsigned long long v = acc[threadIdx.x];
    if (v) {
      unsigned long long *tot = acc + kAccTotal + 2 * threadIdx.x;
      const unsigned long long lo = tot[0] + v;
      tot[1] += (lo < v) ? 1ull : 0ull;
      tot[0] = lo;
      acc[threadIdx.x] = 0ull;
    }
  }
  unsigned long long mx1 = 0ull, mx2 = 0ull;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
    unsigned long long t = 0ull;
    for (int c = 0; c < ncopies; ++c) {
      const unsigned long long v = T[(int64_t)c * V + i];
      if (v) {
        t += v;
        T[(int64_t)c * V + i] = 0ull;
      }
    }
    if (t == 0ull) continue;
    const long long s1 = S1[i] + (long long)t;
    S1[i] = s1;
    const unsigned long long lo = S2[2 * i], hi = S2[2 * i + 1];
    const unsigned long long plo = t * t, phi = __umul64hi(t, t);
    const unsigned long long nlo = lo + plo;
    const unsigned long long nhi = hi + phi + (nlo < lo ? 1ull : 0ull);
    S2[2 * i] = nlo;
    S2[2 * i + 1] = nhi;
    mx1 = max(mx1, (unsigned long long)s1);
    mx2 = max(mx2, nhi);
  }
  m1[threadIdx.x] = mx1;
  m2[threadIdx.x] = mx2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      m1[threadIdx.x] = max(m1[threadIdx.x], m1[threadIdx.x + o]);
      m2[threadIdx.x] = max(m2[threadIdx.x], m2[threadIdx.x + o]);
    }
    __syncthreads();
  }
  // Atomics on one address serialize at the memory side, so a block whose
  // maximum does not exceed the recorded one skips its atomic.  The recorded
  // maxima only grow (until the host clears them between launches), so a
  // stale read can only add an atomic, never drop a needed one.
  if (threadIdx.x == 0) {
    const unsigned long long r1 =
        __hip_atomic_load(acc + kAccMaxS1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long r2 =
        __hip_atomic_load(acc + kAccMaxS2Hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (m1[0] > r1) atomicMax(acc + kAccMaxS1, m1[0]);
    if (m2[0] > r2) atomicMax(acc + kAccMaxS2Hi, m2[0]);
  }
}

// Largest XCC id over all workgroups (read-only hardware register).
__global__ void k_xcc_probe(unsigned int *out) {
  if (threadIdx.x == 0) atomicMax(out, xcc_id());
}

// Pack (mat, rho) into 8-byte voxel records; per-material max and min
// density (as float bits, which order like the values for rho >= 0; the min
// stored complemented so that all-zero memory is its neutral start), voxel
// counts, max material id and a count of bad densities.  stats (kPackStats
// words): [0,256) rho max bits, [256,512) voxel count, [512] max material id,
// [513] bad count, [514,770) complemented rho min bits.
__global__ void __launch_bounds__(256) k_pack(const uint8_t *__restrict__ mat,
                                              const float *__restrict__ rho,
                                              uint2 *__restrict__ vox, int64_t V,
                                              unsigned int *stats) {
  __shared__ unsigned int lmax[256], lcnt[256], lmin[256];
  __shared__ unsigned int lmat, lbad;
  for (int i = threadIdx.x; i < 256; i += blockDim.x) { lmax[i] = 0u; lcnt[i] = 0u; lmin[i] = 0u; }
  if (threadIdx.x == 0) { lmat = 0u; lbad = 0u; }
  __syncthreads();
  unsigned int mymat = 0u, mybad = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
    const unsigned int m = mat[i];
    // -0.0 is stored as +0.0: the per-material extremes below (and the cell
    // maxima of MACRO tracking and the bound classes) order densities by
    // their float bits, which only match their values for sign-clear floats
    const float r = rho[i] == 0.0f ? 0.0f : rho[i];
    const bool ok = (r >= 0.0f) && (r <= 3.4e38f);
    vox[i] = make_uint2(__float_as_uint(r), m);
    mymat = max(mymat, m);
    atomicAdd(&lcnt[m], 1u);
    if (ok) {
      atomicMax(&lmax[m], __float_as_uint(r));
      atomicMax(&lmin[m], ~__float_as_uint(r));
    } else {
      mybad += 1u;
    }
  }
  atomicMax(&lmat, mymat);
  if (mybad) atomicAdd(&lbad, mybad);
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    if (lmax[i]) atomicMax(&stats[i], lmax[i]);
    if (lcnt[i]) atomicAdd(&stats[256 + i], lcnt[i]);
    if (lmin[i]) atomicMax(&stats[514 + i], lmin[i]);
  }
  if (threadIdx.x == 0) {
    atomicMax(&stats[512], lmat);
    if (lbad) atomicAdd(&stats[513], lbad);
  }
}

__global__ void __launch_bounds__(256) k_zero(unsigned long long *p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

// sigma-bar, deterministic two-level reductions (fixed grid and block).
__device__ __forceinline__ bool voxel_dose(const long long *s1, const uint2 *vox, int64_t i,
                                           double rho_min, double &d, double &rho) {
  rho = (double)__uint_as_float(vox[i].x);
  if (!(rho >= rho_min) || rho <= 0.0) return false;
  d = (double)s1[i] / rho;
  return true;
}

__global__ void __launch_bounds__(256) k_sigma_max(const long long *s1, const uint2 *vox,
                                                   int64_t V, double rho_min, double *part) {
  __shared__ double sm[256];
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
    double d, r;
    if (voxel_dose(s1, vox, i, rho_min, d, r)) m = fmax(m, d);
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void __launch_bounds__(256) k_sigma_sum(const long long *s1,
                                                   const unsigned long long *s2,
                                                   const uint2 *vox, int64_t V, uint32_t nb,
                                                   double rho_min, double frac, int kind,
                                                   const double *part_max, int nparts,
                                                   double *part) {
  __shared__ double ss[256], sc[256];
  __shared__ double dmax_s;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int b = 0; b < nparts; ++b) m = fmax(m, part_max[b]);
    dmax_s = m;
  }
  __syncthreads();
  const double dmax = dmax_s;
  const double nbd = (double)nb;
  double sum = 0.0, count = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
    double d, rho;
    if (!voxel_dose(s1, vox, i, rho_min, d, rho)) continue;
    if (!(d > frac * dmax) || dmax <= 0.0) continue;
    const double S1 = (double)s1[i];
    const double S2 = (double)s2[2 * i + 1] * 18446744073709551616.0 + (double)s2[2 * i];
    const double var_t = fmax(nbd * S2 - S1 * S1, 0.0) / (nbd * nbd * (nbd - 1.0));
    const double s = sqrt(var_t) * nbd / rho;  // same scale as d = S1 / rho
    sum += (kind == CTD_SIGMA_PAPER) ? s / dmax : s / d;
    count += 1.0;
  }
  ss[threadIdx.x] = sum;
  sc[threadIdx.x] = count;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sc[threadIdx.x] += sc[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ss[0];
    part[2 * blockIdx.x + 1] = sc[0];
  }
}

__global__ void k_sigma_final(const double *part, int nparts, const double *part_max,
                              double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0, c = 0.0, m = 0.0;
  for (int b = 0; b < nparts; ++b) {
    s += part[2 * b];
    c += part[2 * b + 1];
    m = fmax(m, part_max[b]);
  }
  out[0] = c > 0.0 ? s / c : INFINITY;
  out[1] = c;
  out[2] = m;
}

// ------------------------------------------------------- microbenchmarks
// Peaks the transport is measured against: streaming copy, random 64-bit
// atomics (no return), atomics into 64 hot words, random 8-byte gathers.
// Addresses come from a 32-bit integer hash of the operation index.

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void __launch_bounds__(256) k_mb_copy(const uint4 *__restrict__ a,
                                                 uint4 *__restrict__ b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    b[i] = a[i];
}

__global__ void __launch_bounds__(256) k_mb_atomic(unsigned long long *__restrict__ t,
                                                   uint32_t mask_or_n, int hot, int64_t ops) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ops; i += stride) {
    const uint32_t h = mix32((uint32_t)i);
    const uint32_t idx = hot ? (h & 63u) : (uint32_t)(((uint64_t)h * mask_or_n) >> 32);
    __hip_atomic_fetch_add(t + idx, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void __launch_bounds__(256) k_mb_gather(const uint2 *__restrict__ v, uint32_t n,
                                                   int64_t ops, uint32_t *out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ops; i += stride) {
    const uint32_t idx = (uint32_t)(((uint64_t)mix32((uint32_t)i ^ acc) * n) >> 32);
    const uint2 r = v[idx];
    acc += r.x ^ r.y;
  }
  if (acc == 0x12345678u) out[0] = acc;  // keeps the loads live
}

// ------------------------------------------------ static round table

// The launch table of ctd_run_batches_static.  Host code never passes this
// name to a kernel (on the host it is only a stand-in for the symbol): the
// device address comes from static_scratch_address(), once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// One block writes the round's RoundCase, the bin prefix sums and a zero
// chunk counter into the table (all later work on the stream reads them).
__global__ void __launch_bounds__(256) k_static_round_setup(unsigned char *table,
                                                            StaticRoundArgs a) {
  unsigned long long *pre = (unsigned long long *)(table + kStaticPrefixOff);
  for (int i = threadIdx.x; i <= a.nbins; i += blockDim.x) pre[i] = a.prefix[i];
  unsigned long long *ctr = (unsigned long long *)(table + kStaticCounterOff);
  if (threadIdx.x < 32) ctr[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) {
    RoundCase *rc = (RoundCase *)table;
    rc->cd = a.cd;
    rc->prefix = pre;
    rc->h_begin = a.h_begin;
    rc->n = a.n;
    rc->chunk_begin = 0;
    rc->beamlets = a.beamlets;
    rc->wg_lo = 0;
    rc->home_waves = a.home_waves;
  }
}

// ---------------------------------------------------------------- launchers

static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

int static_scratch_address(void **out) {
  *out = nullptr;
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)) == hipSuccess && *out ? 0 : -1;
}

int launch_static_round_setup(void *table, const StaticRoundArgs &args, void *stream) {
  if (args.nbins < 1 || args.nbins > kStaticMaxBins) return -1;
  hipLaunchKernelGGL(k_static_round_setup, dim3(1), dim3(256), 0, (hipStream_t)stream,
                     (unsigned char *)table, args);
  return check_launch();
}

int launch_transport(const RoundCase *rc_dev, int nrc, uint64_t total_chunks,
                     unsigned long long *chunk_ctr, const LaunchCfg &cfg, bool with_log,
                     int step_kind, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  // stage the tables (room for the round's largest case) only where the
  // workgroup's LDS then still allows the resident workgroups the grid is
  // sized for, with the largest source stash (64, 32 or 16 records per wave)
  // that fits beside them; without the tables, the largest stash that fits
  // (16 at least)
  int tab_n = cfg.tab_n, cap = 0;
  if (tab_n > 0) {
    for (int c = 64; c >= 16 && !cap; c >>= 1)
      if (transport_lds_bytes(cfg.block, cfg.tally_mode, tab_n, cfg.tab_ne, c) <= cfg.lds_budget)
        cap = c;
    if (!cap) tab_n = 0;
  }
  if (!cap) {
    cap = 16;
    for (int c = 64; c > 16 && cap == 16; c >>= 1)
      if (transport_lds_bytes(cfg.block, cfg.tally_mode, 0, 0, c) <= cfg.lds_budget) cap = c;
  }
  const size_t lds = transport_lds_bytes(cfg.block, cfg.tally_mode, tab_n, cfg.tab_ne, cap);
  using Kern = void (*)(const RoundCase *, int, uint64_t, unsigned long long *, int, int, int,
                        int, int, int, int, int);
  static const Kern kerns[2][3][2] = {
      {{k_transport<false, kStepPlain, false>, k_transport<false, kStepPlain, true>},
       {k_transport<false, kStepDeferred, false>, k_transport<false, kStepDeferred, true>},
       {k_transport<false, kStepMacro, false>, k_transport<false, kStepMacro, true>}},
      {{k_transport<true, kStepPlain, false>, k_transport<true, kStepPlain, true>},
       {k_transport<true, kStepDeferred, false>, k_transport<true, kStepDeferred, true>},
       {k_transport<true, kStepMacro, false>, k_transport<true, kStepMacro, true>}}};
  if (step_kind < kStepPlain || step_kind > kStepMacro) return -1;
  const Kern kern = kerns[with_log ? 1 : 0][step_kind][tab_n > 0 ? 1 : 0];
  hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(cfg.block), lds, s, rc_dev, nrc, total_chunks,
                     chunk_ctr, cfg.refill_min, cfg.chunk, cfg.tally_mode, cfg.bound_shift,
                     cfg.defer_min, tab_n, tab_n > 0 ? cfg.tab_ne : 0, cap);
  return check_launch();
}

size_t transport_lds_bytes(int block, int tally_mode, int tab_n, int tab_ne, int stash_cap) {
  const size_t nw = (size_t)(block / 64);
  size_t b = kWgSlotsOff + nw * kWaveSlotBytes + (tally_mode == 2 ? nw * kCacheBytesPerWave : 0);
  b += nw * (size_t)stash_cap * kStashRecBytes;
  // majorant nodes, mu/rho rows and (room for) the bound-test sums
  if (tab_n > 0) b += (size_t)((tab_ne + 3) & ~3) * 4 + (size_t)tab_n * 20;
  return b;
}

bool transport_lds_fits(int block, int tally_mode, int device) {
  int lim = 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
      hipSuccess) {
    (void)hipGetLastError();  // not a launch error: leave nothing for check_launch
    return false;
  }
  return transport_lds_bytes(block, tally_mode, 0, 0, 16) <= (size_t)lim;
}

static int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int launch_fold(unsigned long long *tally, int ncopies, long long *s1, unsigned long long *s2,
                int64_t V, unsigned long long *acc, void *stream) {
  // 1024 groups stream the arrays at full rate and keep the per-group
  // maximum records (two loads, at most two atomics each) few
  hipLaunchKernelGGL(k_fold, dim3(grid_for(V, 256, 1024)), dim3(256), 0, (hipStream_t)stream,
                     tally, ncopies, s1, s2, V, acc);
  return check_launch();
}

int launch_xcc_probe(unsigned int *out, int blocks, void *stream) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(blocks), dim3(64), 0, (hipStream_t)stream, out);
  return check_launch();
}

int launch_pack(const uint8_t *mat, const float *rho, uint2 *vox, int64_t V,
                unsigned int *stats, void *stream) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(V, 256, 2048)), dim3(256), 0, (hipStream_t)stream,
                     mat, rho, vox, V, stats);
  return check_launch();
}

int launch_cell_max(const uint2 *vox, int nx, int ny, int nz, int cs, int ncx, int ncy, int M,
                    unsigned int *out, void *stream) {
  const int64_t V = (int64_t)nx * ny * nz;
  if (V <= 0) return 0;
  hipLaunchKernelGGL(k_cell_max, dim3(grid_for(V, 256, 8192)), dim3(256), 0, (hipStream_t)stream,
                     vox, nx, ny, V, cs, ncx, ncy, M, out);
  return check_launch();
}

int launch_block_class(const uint2 *vox, int nx, int ny, int nz, int shift, const uint2 *cls,
                       const int2 *range, uint8_t *out, void *stream) {
  const int e = (1 << shift) - 1;
  const int bx = (nx + e) >> shift, by = (ny + e) >> shift, bz = (nz + e) >> shift;
  const int64_t nb = (int64_t)bx * by * bz;
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(k_block_class, dim3(grid_for(nb, 256, 8192)), dim3(256), 0,
                     (hipStream_t)stream, vox, nx, ny, nz, shift, bx, by, nb, cls, range, out);
  return check_launch();
}

int launch_mh_fill(const float *f, int n_f, int C, uint64_t h_begin, uint64_t n, uint32_t key0,
                   uint32_t key1, int32_t *state, int32_t *out, void *stream) {
  if (C <= 0 || n == 0) return 0;
  hipLaunchKernelGGL(k_mh_fill, dim3((unsigned)((C + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, f, n_f, C, h_begin, n, key0, key1, state, out);
  return check_launch();
}

int launch_zero(void *ptr, size_t bytes, void *stream) {
  const size_t n = bytes / 8;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_zero, dim3(grid_for((int64_t)n, 256, 4096)), dim3(256), 0,
                     (hipStream_t)stream, (unsigned long long *)ptr, n);
  return check_launch();
}

int launch_sigma(const long long *s1, const unsigned long long *s2, const uint2 *vox, int64_t V,
                 uint32_t nb, double rho_min, double frac, int kind, double *scratch,
                 int nblocks, double *out, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  double *pmax = scratch;
  double *psum = scratch + nblocks;
  hipLaunchKernelGGL(k_sigma_max, dim3(nblocks), dim3(256), 0, s, s1, vox, V, rho_min, pmax);
  hipLaunchKernelGGL(k_sigma_sum, dim3(nblocks), dim3(256), 0, s, s1, s2, vox, V, nb, rho_min,
                     frac, kind, pmax, nblocks, psum);
  hipLaunchKernelGGL(k_sigma_final, dim3(1), dim3(64), 0, s, psum, nblocks, pmax, out);
  return check_launch();
}

int launch_microbench(int kind, void *buf_a, void *buf_b, int64_t n, int64_t ops, int grid,
                      void *stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_mb_copy, dim3(grid), dim3(256), 0, s, (const uint4 *)buf_a,
                         (uint4 *)buf_b, n / 16);
      break;
    case 1:
    case 2:
      hipLaunchKernelGGL(k_mb_atomic, dim3(grid), dim3(256), 0, s, (unsigned long long *)buf_a,
                         (uint32_t)(n / 8), kind == 2 ? 1 : 0, ops);
      break;
    case 3:
      hipLaunchKernelGGL(k_mb_gather, dim3(grid), dim3(256), 0, s, (const uint2 *)buf_a,
                         (uint32_t)(n / 8), ops, (uint32_t *)buf_b);
      break;
    default:
      return -1;
  }
  return check_launch();
}

int device_cu_count(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
  return prop.multiProcessorCount;
}

}  // namespace ctd
