/*
 * ctd.h -- C ABI of the MI355X (gfx950) Monte Carlo CT/CBCT imaging-dose
 * transport library (libctd.so).
 *
 * Method: Jia, Yan, Gu & Jiang, "Fast Monte Carlo Simulation for
 * Patient-specific CT/CBCT Imaging Dose Calculation" (arXiv 1109.3266):
 * photons from a cone-beam or pencil source (Sec. 2.2.5 spectrum
 * stratification, Sec. 2.2.6 source trajectory) are transported through a
 * voxel phantom by Woodcock tracking (Sec. 2.1), interacting by photoelectric
 * absorption, Compton and Rayleigh scattering with angles drawn from
 * inverse-CDF "C/R surfaces" (Sec. 2.2.2-2.2.3), depositing electron energy
 * locally; histories run in batches whose spread gives the per-voxel
 * statistical uncertainty (Sec. 2.2.1).
 *
 * Options beside the plain method: bound-electron Compton (one C surface per
 * material, Eq. 2 with S), a helical CT trajectory, a fluence map over the
 * field (Sec. 2.2.4: exact inverse CDF, or Alg. A1 Metropolis-Hastings
 * chains), macro-cell majorants for Woodcock tracking (CTD_TRACK_MACRO, or
 * chosen per case by CTD_TRACK_AUTO), a tally contention strategy chosen per
 * case (ctd_tuning.tally_mode), a batched multi-case engine, a
 * continuous-batching dose server, and the gamma-index comparison of Sec. 3.1.
 *
 * Conventions
 *   - Every call returns an int32 status (CTD_OK or a negative CTD_E* code);
 *     ctd_last_error() gives a message for the last failing call on a ctx.
 *   - Handles are opaque and owned by the library; release them with the
 *     matching *_release / *_destroy call.  One ctx per host thread, or
 *     external locking.  No C++ exception crosses this interface.
 *   - Device work is enqueued on the ctx's stream (ctd_set_stream), in order;
 *     ctd_run* return once the work is enqueued unless stated otherwise.
 *   - Arrays are C order.  Voxel arrays are [nz][ny][nx] (x fastest).
 *   - Energies in keV, lengths in cm, densities in g/cm^3, mass attenuation
 *     coefficients in cm^2/g.
 *   - Deposited energy is tallied exactly in int64 fixed point with unit
 *     q = 2^-24 keV.  Transport arithmetic is float32, so every deposit and
 *     escape is an exact multiple of q and incident = deposited + escaped
 *     holds exactly in q units.
 *   - Determinism: tallies are a pure function of (inputs, seed, the sequence
 *     of batch sizes); they do not depend on the stream, tuning, thread
 *     count or work co-scheduled in a batched launch.
 *   - A ctd_run* call that fails before enqueueing any work leaves its cases
 *     as they were (e.g. CTD_EOVERFLOW from the headroom check).  One that
 *     fails after enqueueing part of a round (a launch or copy error) leaves
 *     their sums, counters and history ids undefined: the calls that run or
 *     read such a case return CTD_EINVAL until ctd_case_reset.
 */
#ifndef CTD_H
#define CTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define CTD_OK 0
#define CTD_EINVAL (-1)     /* invalid argument or input data */
#define CTD_ENOMEM (-2)     /* device or host allocation failed */
#define CTD_EDEVICE (-3)    /* HIP runtime error (message in ctd_last_error) */
#define CTD_EOVERFLOW (-4)  /* fixed-point headroom: N * E_max * 2^24 >= 2^63 */
#define CTD_EBUSY (-5)      /* object still referenced by a live case/request */
#define CTD_ENOTFOUND (-6)  /* unknown ticket */
#define CTD_ECANCELLED (-7) /* request was cancelled */
#define CTD_ESTEPS (-8)     /* a history exceeded the step guard (majorant 0?) */

#define CTD_MEM_HOST 0   /* pointer is host memory; the library copies it */
#define CTD_MEM_DEVICE 1 /* pointer is device memory on the ctx's GPU */

#define CTD_GEOM_PENCIL 0
#define CTD_GEOM_CONE 1

#define CTD_SIGMA_LOCAL 0 /* mean of s/D over voxels with D > f * D_max */
#define CTD_SIGMA_PAPER 1 /* mean of s/D_max over voxels with D > f * D_max (Sec. 3.1) */

typedef struct ctd_ctx ctd_ctx;
typedef struct ctd_phantom ctd_phantom;
typedef struct ctd_matset ctd_matset;
typedef struct ctd_spectrum ctd_spectrum;
typedef struct ctd_geometry ctd_geometry;
typedef struct ctd_case ctd_case;
typedef struct ctd_server ctd_server;

/* Voxel grid: nx*ny*nz voxels of dx*dy*dz cm; origin = corner of voxel 0. */
typedef struct {
  int32_t nx, ny, nz, reserved;
  double dx, dy, dz;
  double origin[3];
} ctd_grid;

/* Uniform energy grid of the attenuation tables and surfaces:
 * E_j = e0 + j*de, j = 0..ne-1 (keV).  Must cover [e_cut, E_max]. */
typedef struct {
  double e0, de;
  int32_t ne, reserved;
} ctd_egrid;

/* Scan geometry (Sec. 2.2.6 source trajectory r(t); the CT use of the
 * method, Sec. 1 and 4, adds table travel).  PENCIL: a fixed point src and
 * direction dir.  CONE: point source at
 *   iso + sad*(sin phi, cos phi, 0) + (0, 0, z_feed*(phi - phi0)/360),
 * aimed at the field rectangle [a0,a1] x [b0,b1] (cm) spanned by
 * e_lat = (cos phi, -sin phi, 0) and e_z around the point of the axis at the
 * source's height; phi = phi0 + p*arc/n_proj for a projection p drawn
 * uniformly (n_proj > 0), or phi0 + u*arc (n_proj = 0, continuous t).
 * z_feed = 0 is the circular (CBCT) orbit; z_feed != 0 with arc spanning
 * several turns is a helical CT scan (pitch = z_feed / (b1 - b0) at the
 * isocentre). */
typedef struct {
  int32_t kind, n_proj;
  double src[3], dir[3];
  double sad, iso[3];
  double a0, a1, b0, b1;
  double phi0_deg, arc_deg;
  double z_feed;            /* cm of travel along z per 360 deg */
  /* Fluence map (Sec. 2.2.4): the field rectangle split into na x nb equal
   * beamlets, beamlet I = ib*na + ia covering [a0 + ia*da, a0 + (ia+1)*da) x
   * [b0 + ib*db, ...), da = (a1-a0)/na, db = (b1-b0)/nb.  A source photon
   * comes from beamlet I with probability f_I / sum f and is uniform inside
   * it.  fluence = NULL (na = nb = 0) is the uniform field.  The map is read
   * during ctd_geometry_set only (copied).  The beamlet is drawn from the
   * first uniform of the history's second source block (Philox counter
   * (0, h_lo, h_hi, 1)) as the smallest I with C_I > u*F, C_I the FP64
   * running sum of f in index order and F = C_{N-1}; the decision is exact
   * in FP64.  CONE only.
   * fluence_chains = C > 0 selects Alg. A1 (Metropolis-Hastings) instead:
   * history h belongs to logical chain h mod C and each chain visits its
   * histories in increasing h, from a uniformly drawn start (counter
   * (0, c_lo, c_hi, 2)); the step of history h proposes J = floor(u0 N) and
   * moves there when u1 * f_{I_last} < f_J (u0, u1 from the second source
   * block; exact in FP64).  Needs every f_I > 0, and the case's runs to
   * follow each other in history order (they do: runs continue at the next
   * id).  Results do not depend on launch configuration. */
  int32_t fluence_na, fluence_nb;
  const float *fluence;     /* [nb][na], f_I >= 0 and finite, sum > 0 */
  int32_t fluence_chains;   /* 0: exact inverse CDF; 1 .. 2^24: Alg. A1 chains */
  int32_t reserved_f;
} ctd_geom;

/* Free-path tracking (Sec. 2.1).  GLOBAL: Woodcock tracking against one
 * majorant mu_max(E) over the whole phantom, as in the paper.  MACRO: the same
 * method with a piecewise-constant majorant over cubic cells of macro_cell^3
 * voxels -- the optical depth -ln(u) to the next tentative collision is spent
 * cell by cell along the ray (boundary crossings draw no random number) and
 * the interaction is selected against the cell's majorant, which bounds
 * every voxel of the cell at every energy.  Both are exact; MACRO consumes
 * random numbers differently, so its histories are not the GLOBAL ones, and it
 * saves the voxel reads of fictitious steps where dense and light tissue mix
 * (a bone-dominated global majorant). */
#define CTD_TRACK_GLOBAL 0
#define CTD_TRACK_MACRO 1
/* AUTO: MACRO where, at the spectrum's mean energy, the largest rho_max *
 * mu/rho over the phantom's materials exceeds 1.5 times that of its most
 * frequent material denser than 0.05 g/cm^3 (a dense minority such as bone
 * sets the global majorant), else GLOBAL.  Decided from the inputs at case
 * creation (ctd_stats.tracking reports it), so results do not depend on the
 * machine. */
#define CTD_TRACK_AUTO 2

typedef struct {
  double e_cut_kev;      /* photon absorption energy (Sec. 3.1 uses 1 keV) */
  uint64_t seed;         /* Philox key */
  int32_t n_batches;     /* batches per ctd_run (Sec. 2.2.1 uses 10), >= 2 */
  int32_t rayleigh;      /* 1 = Rayleigh scattering on */
  double sigma_rho_min;  /* voxels with rho >= this count as "inside" for sigma-bar */
  int32_t tracking;      /* CTD_TRACK_GLOBAL (default), CTD_TRACK_MACRO or CTD_TRACK_AUTO */
  int32_t macro_cell;    /* MACRO cell edge in voxels, 1..64 (0: about 1.6 cm) */
} ctd_params;

/* Energy balance in units of q = 2^-24 keV as exact 128-bit sums (hi:lo). */
typedef struct {
  uint64_t q_incident, q_deposited, q_escaped;          /* low 64 bits */
  uint64_t q_incident_hi, q_deposited_hi, q_escaped_hi; /* high 64 bits */
  uint64_t n_histories, n_missed, n_unscattered, n_cutoff;
} ctd_balance;

typedef struct {
  double sigma_local;    /* CTD_SIGMA_LOCAL with f = 0.5 after the last run */
  double sigma_paper;    /* CTD_SIGMA_PAPER with f = 0.2 after the last run */
  /* n_steps: Woodcock steps (MACRO tracking: flights); n_real: real
   * collisions = n_photo + n_compton + n_rayleigh; n_refills: wave refill
   * steps of the transport kernel */
  uint64_t n_steps, n_real, n_photo, n_compton, n_rayleigh, n_deposits,
      n_escapes, n_refills;
  double transport_ms;   /* GPU time of the transport launches (HIP events) */
  double fold_ms;        /* GPU time of the batch folds */
  uint32_t n_batches;    /* batches folded so far */
  int32_t tracking;      /* CTD_TRACK_GLOBAL or CTD_TRACK_MACRO: the mode in use */
  uint64_t n_histories;  /* histories run so far */
  uint64_t n_crossings;  /* MACRO tracking: macro-cell boundary crossings */
  /* Largest S1 and largest high word of S2 over the voxels, as recorded by
   * the batch folds for the fixed-point headroom check of ctd_run (exact:
   * equal to max(s1) and max(s2_hi) of ctd_read_tally). */
  uint64_t max_s1, max_s2_hi;
} ctd_stats;

/* Launch configuration of the persistent transport kernel. */
typedef struct {
  int32_t block;         /* threads per workgroup: 64, 128, 256, 512 */
  int32_t waves_per_simd;/* resident waves per SIMD to size the grid (1..8) */
  int32_t refill_min;    /* refill a wave when >= this many lanes idle (1..64) */
  int32_t chunk;         /* histories a wave claims per counter atomic (64..65536) */
  int32_t tally_mode;    /* 0: one batch tally, device-scope atomics;
                            1: one batch tally per XCD, updated only by the
                            waves of that XCD (fewer atomics on one address
                            where deposits concentrate) and summed by the
                            fold (only where every XCD id is < 8);
                            2: as 1, behind a 512-slot LDS sub-tally per wave
                            (a voxel's slot is kept by the first voxel that
                            takes it until the wave changes case; the rest go
                            to the XCD tally); 6 KB of LDS per wave, rejected
                            where the workgroup would exceed the LDS limit.
                            Tallies are integer sums: every mode gives the
                            same bits. */
  int32_t bound_block;   /* Early rejection of fictitious collisions (GLOBAL
                            tracking of phantoms stored as 8-byte records):
                            0 off; 1, 2 or 4 = edge in voxels of the blocks
                            of a 1-byte bound grid built at phantom load.  A
                            block of one material carries a density level at
                            or above all of its voxels'; a tentative
                            collision whose xi reaches the level times the
                            material's largest interaction sum over the
                            photon's 1 keV-class energy cell (rounded up
                            with a margin that covers float rounding) is
                            fictitious in every voxel of the block, so it is
                            decided without reading the voxel.  Decisions,
                            and so results, are those of 0, bit for bit. */
  int32_t defer_min;     /* With a bound grid: a tentative collision the
                            bound cannot reject waits, and the wave resolves
                            its waiting collisions together once this many
                            lanes hold one (or every live lane does), so the
                            voxel reads and interaction code run with more
                            lanes active; photons that leave the box add
                            their counters at the wave's next refill.  0:
                            every collision at once (1..64).  Each history's
                            steps are unchanged: same results bit for bit. */
} ctd_tuning;

/* Deposit/event record of the debug log (test use). type: 0 source, 1
 * photoelectric, 2 Compton, 3 Rayleigh, 4 cutoff deposit, 5 escape, 6 miss. */
typedef struct {
  uint64_t h;
  uint32_t seq, k;
  int32_t type, reserved;
  int64_t vox;
  float e;   /* deposited (1,2,4), escaping (5,6) or source (0) energy, keV */
  float E;   /* photon energy after the event */
} ctd_event;

/* ---------------- context ---------------- */

/* Create a context on HIP device `device`.  CTD_EDEVICE if it does not exist. */
int32_t ctd_create(ctd_ctx **out, int32_t device);
/* Destroy the context (waits for its stream, frees its own buffers).  Cases,
 * phantoms, material sets, spectra and geometries created on it must be
 * released first. */
int32_t ctd_destroy(ctd_ctx *ctx);
/* Message of the last failing call on ctx (valid until the next call). */
const char *ctd_last_error(const ctd_ctx *ctx);
/* Enqueue all further work on the caller's hipStream_t (borrowed, never
 * destroyed); NULL restores the context's own stream.  Waits for the work
 * already enqueued on the current stream first. */
int32_t ctd_set_stream(ctd_ctx *ctx, void *hip_stream);

/* ---------------- inputs ----------------
 * Inverse-CDF surface construction (Sec. 2.2.2): pdf [n_e][n_mu] tabulated
 * at n_mu equally spaced mu in [-1, 1] for each energy node.  Host FP64:
 * cumulative distribution by the trapezoid rule, normalised, inverted at
 * zeta_i = i/(n_zeta-1) by linear interpolation; out [n_e][n_zeta] float,
 * caller-allocated.  CTD_EINVAL on sizes < 2 or a negative/zero-mass pdf. */
int32_t ctd_surface_build(int32_t n_e, int32_t n_mu, const double *pdf, int32_t n_zeta,
                          float *out);

/* Voxel phantom (Sec. 2.2.1 inputs): material id mat[] and density rho[].
 * mem = CTD_MEM_HOST or CTD_MEM_DEVICE; both arrays are read during the call
 * only (the library keeps its own packed copy).  CTD_EINVAL on dims <= 0,
 * spacing <= 0, rho not finite or < 0, more than 2^31 - 1 voxels, or
 * ny * nz > 2^24. */
int32_t ctd_phantom_load(ctd_ctx *ctx, const ctd_grid *g, const uint8_t *mat, const float *rho,
                         int32_t mem, ctd_phantom **out);
/* CTD_EBUSY while a case refers to it. */
int32_t ctd_phantom_release(ctd_ctx *ctx, ctd_phantom *ph);

/* Material tables (host memory, copied):
 *   mu_rho   [M][ne][3]  photoelectric, Compton, Rayleigh mass attenuation;
 *   comp     [1 or M][ne][n_zeta_c] Compton surface (one shared, or per
 *            material when comp_per_mat = 1);
 *   rayl     [M][ne][n_zeta_r] Rayleigh surfaces, or NULL.
 * CTD_EINVAL if a surface is not non-decreasing in zeta or leaves [-1, 1],
 * or a coefficient is negative / not finite. */
int32_t ctd_materials_load(ctd_ctx *ctx, const ctd_egrid *eg, int32_t M, const float *mu_rho,
                           const float *comp, int32_t comp_per_mat, int32_t n_zeta_c,
                           const float *rayl, int32_t n_zeta_r, ctd_matset **out);
int32_t ctd_materials_release(ctd_ctx *ctx, ctd_matset *ms);

/* Stratified spectrum (Sec. 2.2.5): nbins bins [e_lo[j], e_lo[j]+width)
 * with relative weights; width = 0 gives monoenergetic lines.  Copied.
 * CTD_EINVAL on a negative weight or zero total. */
int32_t ctd_spectrum_set(ctd_ctx *ctx, int32_t nbins, const double *e_lo, double width,
                         const double *weight, ctd_spectrum **out);
int32_t ctd_spectrum_release(ctd_ctx *ctx, ctd_spectrum *sp);

/* Scan geometry (copied).  CTD_EINVAL on a zero direction, sad <= 0, an
 * empty field, or n_proj < 0. */
int32_t ctd_geometry_set(ctd_ctx *ctx, const ctd_geom *g, ctd_geometry **out);
int32_t ctd_geometry_release(ctd_ctx *ctx, ctd_geometry *geo);

/* ---------------- cases ----------------
 * Bind one dose problem; computes the Woodcock majorant mu_max(E) (Sec. 2.1)
 * from the phantom's per-material maximum density and allocates the batch
 * tally T_b, S1 = sum_b T_b and S2 = sum_b T_b^2 (128-bit).
 * CTD_EINVAL if a material id >= M, the energy grid does not cover
 * [e_cut, E_max], n_batches < 2, e_cut < 1 keV, a spectrum bin starts below
 * 1 keV, or the phantom or material set was loaded through a context on
 * another device; CTD_ENOMEM.  (The 1 keV rules keep the tally exact: a
 * Compton scatter leaves E' > E/2, so every photon energy stays >= 0.5 keV,
 * where float32 values are multiples of q.) */
int32_t ctd_case_create(ctd_ctx *ctx, ctd_phantom *ph, ctd_matset *ms, ctd_spectrum *sp,
                        ctd_geometry *geo, const ctd_params *p, ctd_case **out);
int32_t ctd_case_destroy(ctd_ctx *ctx, ctd_case *cs);
/* Clear all tallies and counters; the next history id is 0 again. */
int32_t ctd_case_reset(ctd_ctx *ctx, ctd_case *cs);
/* Launch configuration for this case (defaults are chosen at creation). */
int32_t ctd_set_tuning(ctd_ctx *ctx, ctd_case *cs, const ctd_tuning *t);
int32_t ctd_get_tuning(ctd_ctx *ctx, const ctd_case *cs, ctd_tuning *t);
/* Time a few launch configurations on `trial_histories` histories of this
 * case (run on a scratch copy of the tallies; the case is left unchanged)
 * and keep the fastest.  Synchronous. */
int32_t ctd_autotune(ctd_ctx *ctx, ctd_case *cs, uint64_t trial_histories, ctd_tuning *best);

/* Run n_histories as n_batches equal batches (the first n mod n_batches
 * one larger), continuing the case's history ids.  Each batch: transport
 * launch, then fold S1 += T_b, S2 += T_b^2, T_b = 0 (Sec. 2.2.1).  Async.
 * CTD_EOVERFLOW if a batch could exceed 2^62 q in one voxel (histories *
 * E_max * 2^24 >= 2^62), or if a voxel's S1 could pass 2^63 or its S2 2^128
 * (checked against the exact per-voxel maxima the folds record). */
int32_t ctd_run(ctd_ctx *ctx, ctd_case *cs, uint64_t n_histories);

/* Run `count` batches of exactly batch_histories each (same per-batch work
 * as ctd_run), continuing the case's history ids.  Async. */
int32_t ctd_run_batches(ctd_ctx *ctx, ctd_case *cs, uint64_t batch_histories, uint64_t count);

/* ctd_run_batches for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same batches with the same results bit for bit, but each round's launch
 * table (its round descriptor, the spectrum's bin prefix sums and the chunk
 * counter, 2816 B) lives in a static device array that each GPU holds until
 * the process ends, written by a set-up kernel; the call enqueues only kernels
 * (no allocation, copy, memset or event).  Limits: at most 256 spectrum bins,
 * and the fixed-point bounds must admit the batches without the exact maxima
 * read-back of ctd_run (else CTD_EOVERFLOW; ctd_run_batches then continues);
 * Alg. A1 cases need a beamlet buffer already sized by a ctd_run_batches call
 * with the same batch size (else CTD_EINVAL).  Every call on one GPU shares
 * its array: calls that overlap on one GPU (work on two streams at once)
 * race, calls in stream order do not.  Kernel times are not added to
 * ctd_stats.transport_ms.  Async. */
int32_t ctd_run_batches_static(ctd_ctx *ctx, ctd_case *cs, uint64_t batch_histories,
                               uint64_t count);

/* Add batches of batch_histories until sigma-bar (sigma_kind, threshold
 * dose_frac * D_max) <= target with >= n_batches batches, or max_histories
 * is reached: a pilot of n_batches batches, then the estimated remainder
 * (sigma ~ batches^-1/2), re-checked.  sigma-bar is the mean relative
 * standard error of the dose over the high-dose region (Sec. 3.1; the
 * standard error from the batch spread of Sec. 2.2.1).  Synchronous;
 * *achieved receives the final sigma-bar (may be NULL).  CTD_EINVAL when the
 * case already holds batches whose size differs from batch_histories by more
 * than one history (the batch statistics need equal batches). */
int32_t ctd_run_to_sigma(ctd_ctx *ctx, ctd_case *cs, double target, double dose_frac,
                         int32_t sigma_kind, uint64_t batch_histories, uint64_t max_histories,
                         double *achieved);

/* Batched engine: run n[i] histories of each case i in ONE persistent launch
 * per batch round over a (case, history-chunk) task queue: each workgroup
 * works on one case at a time, with that case's tables staged in its LDS,
 * and moves on to the next case with chunks left when its case runs out
 * (one launch per step kind when the cases mix MACRO tracking, the bound
 * grid and plain GLOBAL steps), with the launch configuration of cs[0].
 * Per-case results equal ctd_run(cs[i], n[i]) bit for bit.  CTD_EINVAL if a
 * case is listed twice.  Async. */
int32_t ctd_run_many(ctd_ctx *ctx, ctd_case *const *cs, const uint64_t *n, int32_t count);

/* Wait until all work enqueued for the case (its stream) is complete. */
int32_t ctd_sync(ctd_ctx *ctx, ctd_case *cs);

/* Compute sigma-bar (Sec. 3.1, over the batch statistics of Sec. 2.2.1) on
 * the device over the folded batches.  Synchronous.  CTD_EINVAL with fewer
 * than 2 batches or batches whose sizes differ by more than one history. */
int32_t ctd_sigma(ctd_ctx *ctx, ctd_case *cs, int32_t sigma_kind, double dose_frac,
                  double *out);

/* ---------------- readout ----------------
 * Exact integer sums (V-sized caller arrays, host): s1[v] = sum_b T_b[v];
 * s2 as 128-bit (s2_hi:s2_lo) = sum_b T_b[v]^2; *n_batches batches folded.
 * Synchronous. */
int32_t ctd_read_tally(ctd_ctx *ctx, ctd_case *cs, int64_t *s1, uint64_t *s2_hi,
                       uint64_t *s2_lo, uint32_t *n_batches);
/* Dose per history [Gy] and the variance of that mean [Gy^2] per voxel, from
 * the exact sums (Sec. 2.2.1: the mean over batches and its uncertainty from
 * their spread; numerator formed in 192-bit integers).  Voxels of zero
 * density report 0.  Synchronous; CTD_EINVAL unless >= 2 batches were folded
 * and their sizes differ by at most one history (ctd_run's remainder). */
int32_t ctd_read_dose(ctd_ctx *ctx, ctd_case *cs, double *dose, double *var_of_mean);
/* Device pointers of the case's S1 (int64 [V]) and S2 (uint64 [V][2], lo
 * then hi), valid until the case is destroyed. */
int32_t ctd_tally_device(ctd_ctx *ctx, ctd_case *cs, void **s1, void **s2);
int32_t ctd_read_balance(ctd_ctx *ctx, ctd_case *cs, ctd_balance *out);
int32_t ctd_read_stats(ctd_ctx *ctx, ctd_case *cs, ctd_stats *out);
/* Copy the case's majorant nodes mu_max[ne] (float, cm^-1). */
int32_t ctd_read_majorant(ctd_ctx *ctx, ctd_case *cs, float *out);

/* ---------------- microbenchmarks ----------------
 * Device peaks for roofline reporting, timed with HIP events on the ctx
 * stream (synchronous).  kind: 0 streaming copy of `bytes` (result: GB/s of
 * read + write), 1 random 64-bit atomic adds without return into a `bytes`
 * array (ops/s), 2 the same into 64 hot words (ops/s), 3 random 8-byte
 * gathers from a `bytes` array (ops/s).  `ops` is ignored for kind 0.
 * *rate receives the measured rate, *ms the kernel time. */
int32_t ctd_microbench(ctd_ctx *ctx, int32_t kind, uint64_t bytes, uint64_t ops, double *rate,
                       double *ms);

/* ---------------- dose comparison ----------------
 * Gamma index (the agreement test of Sec. 3.1, after Low et al. 1998):
 *   gamma(r) = min_{r'} sqrt((D_ref(r) - D_eval(r'))^2 / dose_tol^2
 *                            + |r - r'|^2 / dta_cm^2)
 * for every voxel centre r with D_ref(r) > region_min.  r' runs over the
 * lattice r + h*(i,j,k), h = dta_cm / substeps, |r' - r| <= gamma_cap*dta_cm,
 * and D_eval(r') is the trilinear interpolant of D_eval between voxel centres,
 * clamped to the outermost centres.  Values that would exceed gamma_cap are
 * reported as gamma_cap.  The paper's test: dose_tol = 0.02 D_max, dta_cm =
 * 0.2, region_min = 0.2 D_max, pass when gamma < 1. */
typedef struct {
  double dose_tol;    /* Delta D, in the arrays' dose units (> 0) */
  double dta_cm;      /* Delta r (> 0) */
  double region_min;  /* voxels with D_ref > region_min are evaluated */
  double gamma_cap;   /* 1 <= gamma_cap <= 4 */
  int32_t substeps;   /* 1 <= substeps <= 20 */
  int32_t reserved;
} ctd_gamma_params;

/* ref, eval: [nz][ny][nx] float doses on grid g, in host (mem = CTD_MEM_HOST)
 * or device memory (CTD_MEM_DEVICE); read only.  gamma: optional [V] output in
 * the same memory kind (NULL to skip), -1 outside the evaluated region.
 * *n_region = evaluated voxels, *n_pass = those with gamma < 1 (decided in
 * FP64).  Synchronous on the context stream.  CTD_EINVAL on bad parameters or
 * more than 2^22 lattice offsets. */
int32_t ctd_gamma(ctd_ctx *ctx, const ctd_grid *g, const float *ref, const float *eval,
                  int32_t mem, const ctd_gamma_params *p, float *gamma, uint64_t *n_region,
                  uint64_t *n_pass);

/* ---------------- debug log (tests) ----------------
 * Arm event logging of histories [h0, h0+nh) for the following runs, with
 * room for `capacity` events (0 disarms).  Read them back with
 * ctd_read_event_log (*n = events recorded; may exceed capacity, in which
 * case only `capacity` were kept). */
int32_t ctd_debug_deposit_log(ctd_ctx *ctx, ctd_case *cs, uint64_t h0, uint64_t nh,
                              uint64_t capacity);
int32_t ctd_read_event_log(ctd_ctx *ctx, ctd_case *cs, ctd_event *out, uint64_t capacity,
                           uint64_t *n);
/* For callers that test their handling of a failed run: the next round on
 * ctx returns CTD_EDEVICE right after its first transport launch (which
 * completes normally), leaving its cases in the failed state described under
 * Conventions.  One-shot. */
int32_t ctd_debug_fail_next_round(ctd_ctx *ctx);

/* ---------------- serving (continuous batching) ----------------
 * A server owns two private contexts on `device` and two host threads: one
 * enqueues the rounds, the other admits requests and copies results out
 * while the rounds run.  Phantoms are registered once (host arrays, copied)
 * and loaded to the device on first use; they stay resident and are evicted
 * least-recently-used when an admission needs the room.  Requests (a phantom
 * key, material set, spectrum, geometry, parameters and a sigma-bar target)
 * queue in arrival order and are admitted while their device footprint fits
 * hbm_budget_bytes.  Each round runs one batch of batch_histories for every
 * admitted request in a single launch of the batched engine; the host waits
 * for the device once per iteration of up to 21 rounds or 2e8 histories,
 * and requests admitted meanwhile join the next iteration.  Every request
 * follows the batch schedule of ctd_run_to_sigma with the same batch size, so
 * its result is identical alone or among others.  Beyond the budget the
 * server keeps staging buffers sized by the largest registered phantom: 5
 * bytes per voxel of device memory and 29 of pinned host memory.
 * Material sets, spectra and geometries may come from any context on the same
 * device; a request holds them from submission until it finishes (releasing
 * one earlier returns CTD_EBUSY).  The calls may come from any host thread,
 * except ctd_server_stop, which must not overlap another call on the same
 * server.  An admission never evicts the phantom it is admitting. */
typedef struct {
  uint64_t hbm_budget_bytes;  /* device memory for request tallies + resident phantoms */
  uint64_t batch_histories;   /* histories per batch, every request */
  uint64_t max_histories;     /* per-request cap */
  double dose_frac;           /* sigma-bar threshold fraction of D_max */
  int32_t sigma_kind;         /* CTD_SIGMA_LOCAL or CTD_SIGMA_PAPER */
  int32_t max_active;         /* cap on concurrently admitted requests */
  ctd_tuning tuning;          /* launch configuration of the rounds; block = 0: default */
} ctd_server_config;

typedef struct {
  int32_t state;    /* 0 queued, 1 running, 2 done, 3 cancelled, 4 failed */
  int32_t status;   /* CTD_* code of a failed or cancelled request */
  double sigma;     /* last sigma-bar */
  uint64_t histories;
  uint32_t batches, reserved;
  double t_submit, t_admit, t_done; /* seconds on the server clock */
} ctd_request_info;

typedef struct {
  uint64_t submitted, completed, rounds, histories;
  uint64_t phantom_loads, phantom_hits, evictions;
  uint64_t resident_bytes;
  uint32_t queued, active;
} ctd_server_stats;

int32_t ctd_server_start(int32_t device, const ctd_server_config *cfg, ctd_server **out);
const char *ctd_server_last_error(const ctd_server *sv);
/* Seconds on the server clock (monotonic, 0 at start). */
double ctd_server_now(const ctd_server *sv);
/* Register a phantom under `key` (arrays copied to host memory).  CTD_EBUSY
 * if the key exists. */
int32_t ctd_server_add_phantom(ctd_server *sv, uint64_t key, const ctd_grid *g,
                               const uint8_t *mat, const float *rho);
/* Queue a request; *ticket identifies it.  CTD_ENOTFOUND for an unknown key. */
int32_t ctd_server_submit(ctd_server *sv, uint64_t phantom_key, ctd_matset *ms,
                          ctd_spectrum *sp, ctd_geometry *geo, const ctd_params *p,
                          double sigma_target, uint64_t *ticket);
int32_t ctd_server_poll(ctd_server *sv, uint64_t ticket, ctd_request_info *info);
/* Block until done (CTD_OK), cancelled (CTD_ECANCELLED) or failed (its
 * status); CTD_ENOTFOUND if the ticket is unknown or released meanwhile. */
int32_t ctd_server_wait(ctd_server *sv, uint64_t ticket, ctd_request_info *info);
/* Exact sums of a done request, copied from host memory into caller arrays
 * of n_voxels entries each (any may be null); CTD_EINVAL unless n_voxels is
 * the phantom's voxel count, CTD_EBUSY before the request is done. */
int32_t ctd_server_read_tally(ctd_server *sv, uint64_t ticket, uint64_t n_voxels, int64_t *s1,
                              uint64_t *s2_hi, uint64_t *s2_lo, uint32_t *n_batches);
/* Forget a finished request (frees its host results). */
int32_t ctd_server_release(ctd_server *sv, uint64_t ticket);
int32_t ctd_server_cancel(ctd_server *sv, uint64_t ticket);
int32_t ctd_server_read_stats(ctd_server *sv, ctd_server_stats *out);
/* Finish the running iteration, copy out the requests that reached their
 * target in it, cancel the rest, free everything. */
int32_t ctd_server_stop(ctd_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* CTD_H */
