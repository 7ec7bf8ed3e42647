/*
 * FP64 CPU oracle for the Monte Carlo CT/CBCT imaging-dose transport of
 * Jia, Yan, Gu & Jiang, "Fast Monte Carlo Simulation for Patient-specific
 * CT/CBCT Imaging Dose Calculation" (arXiv 1109.3266).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library; the two meet only through the seeded synthetic inputs.
 *
 * Plain, slow, obviously correct: one history at a time, in the order of the
 * paper's transport loop (Sec. 2.1, Fig. 2), all arithmetic in double.
 * Tables (attenuation coefficients, inverse-CDF surfaces) are input data and
 * are read as stored (float -> double exactly).
 *
 * Where the paper is silent the following readings are used (the GPU library
 * follows the same rules, written independently):
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (k, history id lo, history id hi, 0); k = 0 is the source
 *     block; blocks k >= 1 give the transport uniforms, taken two at a time
 *     in order (a Woodcock step: free path and selection; a Compton or
 *     Rayleigh scatter: polar-angle sample and azimuth), so two fictitious
 *     steps share a block; u(r) = (2*(r>>9)+1) * 2^-24;
 *   - outside the voxel box is vacuum; entry by the slab method;
 *   - majorant rounded up to float with a 2^-20 relative margin (Sec. 2.1);
 *   - direction update after a scatter: standard polar/azimuth rotation,
 *     pole case when |w| >= 1 - 1e-5, renormalised;
 *   - deposits quantised to q = 2^-24 keV, round-half-even, int64 tallies;
 *     batch statistics by batch means over exact integer sums (Sec. 2.2.1).
 *
 * Every function cites the passage it follows.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ESTEPS (-8)

#define ME_C2_KEV 510.99895
#define TWO_PI 6.283185307179586476925286766559
#define DEG2RAD 0.017453292519943295769236907684886
#define Q_SCALE 16777216.0 /* 2^24: deposits in units of 2^-24 keV */
#define K_MAX 1000000u

enum { EV_SOURCE = 0, EV_PHOTO = 1, EV_COMPTON = 2, EV_RAYLEIGH = 3,
       EV_CUTOFF = 4, EV_ESCAPE = 5, EV_MISS = 6 };

typedef struct {
  int32_t nx, ny, nz, nmat;
  double dx, dy, dz, ox, oy, oz;
  const uint8_t *mat;       /* [nz][ny][nx], x fastest */
  const float *rho;         /* [nz][ny][nx] g/cm^3 */
  int32_t ne, nzeta, rayleigh, kind; /* kind: 0 pencil, 1 cone */
  double e0, de;            /* energy grid: E_j = e0 + j*de */
  const float *mu_rho;      /* [nmat][ne][3] cm^2/g: pe, Compton, Rayleigh */
  const float *comp_surf;   /* [1 or nmat][ne][nzeta] Compton inverse CDF mu(zeta,E) */
  const float *rayl_surf;   /* [nmat][ne][nzeta] Rayleigh inverse CDF or NULL */
  const float *mu_max;      /* [ne] majorant nodes, cm^-1 */
  int32_t nbins, nproj;
  const double *bin_lo;     /* [nbins] keV */
  const double *bin_w;      /* [nbins] relative weights */
  double bin_width;         /* keV; 0 = monoenergetic bins */
  double src[3], dir[3];    /* pencil source */
  double sad, iso[3], a0, a1, b0, b1, phi0_deg, arc_deg; /* cone source */
  double e_cut;             /* keV */
  uint64_t seed;
  int32_t comp_per_mat, pad_c;  /* 1: one Compton surface per material (Eq. 2 with S) */
  double z_feed;            /* cone source: travel along z per 360 deg (helical CT) */
  int32_t fl_na, fl_nb;     /* fluence map beamlets along a and b (0: uniform field) */
  const double *fl_cdf;     /* [fl_na*fl_nb] running sums of the map intensities */
  /* Alg. A1 (Metropolis-Hastings) instead of the inverse CDF when fl_chains > 0:
   * beamlet of history h = fl_beam[h - fl_h0], filled by or_mh_fill */
  int32_t fl_chains, pad_f;
  const float *fl_f;        /* [fl_na*fl_nb] map intensities */
  const int32_t *fl_beam;
  uint64_t fl_h0, fl_nbeam;
} or_case;

typedef struct {
  uint64_t h;
  uint32_t seq, k;
  int32_t type, pad;
  int64_t vox;
  double e;                 /* deposited / escaping / source energy, keV */
  double E;                 /* photon energy after the event */
} or_event;

typedef struct {
  int64_t *s1;              /* [V] sum over batches of batch tallies (q) */
  uint64_t *s2_hi, *s2_lo;  /* [V] sum over batches of squared batch tallies */
  double *shadow;           /* [V] FP64 energy tally summed over batches, keV */
  double *shadow_sq;        /* [V] or NULL: sum of squared FP64 batch tallies */
  double e_inc, e_dep, e_esc;
  int64_t q_inc, q_dep, q_esc;
  uint64_t n_hist, n_steps, n_real, n_pe, n_compton, n_rayleigh, n_deposits,
      n_escapes, n_miss, n_cutoff, n_unscattered;
  double e_unscattered;
  uint32_t n_batches;
  or_event *log;
  uint64_t log_cap, log_n, log_h0, log_h1;
} or_result;

/* ---------------- Philox4x32-10 (Salmon et al., SC'11) ---------------- */

static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  philox4x32_10(ctr, key, out);
}

/* Uniform in (0,1), exactly representable in float and double. */
static double unif(uint32_t r) { return (double)(2u * (r >> 9) + 1u) * (1.0 / Q_SCALE); }

double or_uniform(uint32_t r) { return unif(r); }

/* Four uniforms of history h: counter (k, h_lo, h_hi, s); k = 0 is the
 * source, k >= 1 the transport blocks; s = 1 only for the source's second
 * block (fluence-map beamlet). */
static void block_s(const or_case *c, uint64_t h, uint32_t k, uint32_t s, double u[4]) {
  uint32_t ctr[4] = {k, (uint32_t)h, (uint32_t)(h >> 32), s};
  uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
  uint32_t r[4];
  philox4x32_10(ctr, key, r);
  for (int i = 0; i < 4; ++i) u[i] = unif(r[i]);
}

static void block(const or_case *c, uint64_t h, uint32_t k, double u[4]) { block_s(c, h, k, 0u, u); }

/* Transport uniforms of a history, taken two at a time in order: pair P
 * (P = 0, 1, ...) is uniforms 2 (P mod 2) and 2 (P mod 2) + 1 of block
 * floor(P / 2) + 1.  A Woodcock step takes the next pair (free path,
 * selection); a Compton or Rayleigh scatter takes the pair after its step
 * (polar-angle sample, azimuth). */
typedef struct {
  uint32_t P;     /* pairs taken */
  double u[4];    /* the current block */
} pairs_t;

static void next_pair(const or_case *c, uint64_t h, pairs_t *s, double v[2]) {
  const uint32_t half = s->P & 1u;
  if (half == 0) block(c, h, s->P / 2u + 1u, s->u);
  v[0] = s->u[2 * half];
  v[1] = s->u[2 * half + 1];
  s->P += 1;
}

/* ---------------- Tables: linear interpolation (Sec. 2.2.7 (3)) ---------------- */

static void egrid(const or_case *c, double E, int *j, double *w) {
  double f = (E - c->e0) / c->de;
  double fl = floor(f);
  int jj = (int)fl;
  if (jj < 0) jj = 0;
  if (jj > c->ne - 2) jj = c->ne - 2;
  *j = jj;
  *w = f - (double)jj;
}

static double lerp(double a, double b, double w) { return a + w * (b - a); }

/* Inverse-CDF surface mu(zeta, E), bilinear (Sec. 2.2.2, R/C surface). */
static double surface(const float *S, int nzeta, int j, double wE, double zeta) {
  double f = zeta * (double)(nzeta - 1);
  int i = (int)floor(f);
  if (i < 0) i = 0;
  if (i > nzeta - 2) i = nzeta - 2;
  double wz = f - (double)i;
  const float *r0 = S + (size_t)j * nzeta, *r1 = S + (size_t)(j + 1) * nzeta;
  double s0 = lerp(r0[i], r0[i + 1], wz);
  double s1 = lerp(r1[i], r1[i + 1], wz);
  double mu = lerp(s0, s1, wE);
  if (mu > 1.0) mu = 1.0;
  if (mu < -1.0) mu = -1.0;
  return mu;
}

/* ---------------- Majorant (Sec. 2.1) ----------------
 * mu_max(E_j) = roundup_float( max_m rho_max(m) * sum_k mu/rho(m,j,k) * (1+2^-20) ),
 * the max over materials present in the phantom; the Rayleigh channel counts
 * only when enabled.  Linear interpolation is monotone in the node values, so
 * the interpolated majorant bounds every voxel's interpolated total. */
int or_majorant(const or_case *c, float *out) {
  int64_t V = (int64_t)c->nx * c->ny * c->nz;
  double *rmax = (double *)calloc((size_t)c->nmat, sizeof(double));
  int *seen = (int *)calloc((size_t)c->nmat, sizeof(int));
  if (!rmax || !seen) { free(rmax); free(seen); return OR_ENOMEM; }
  for (int64_t v = 0; v < V; ++v) {
    int m = c->mat[v];
    if (m >= c->nmat) { free(rmax); free(seen); return OR_EINVAL; }
    double r = (double)c->rho[v];
    if (!seen[m] || r > rmax[m]) rmax[m] = r;
    seen[m] = 1;
  }
  for (int j = 0; j < c->ne; ++j) {
    double best = 0.0;
    for (int m = 0; m < c->nmat; ++m) {
      if (!seen[m]) continue;
      const float *t = c->mu_rho + ((size_t)m * c->ne + j) * 3;
      double s = (double)t[0] + (double)t[1];
      if (c->rayleigh) s += (double)t[2];
      double v = rmax[m] * s;
      if (v > best) best = v;
    }
    double x = best * (1.0 + 1.0 / 1048576.0);
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    out[j] = f;
  }
  free(rmax);
  free(seen);
  return OR_OK;
}

/* ---------------- Spectrum stratification (Sec. 2.2.5) ----------------
 * n histories of one batch are split over the 1 keV bins in proportion to the
 * weights by the largest-remainder rule (ties to the lower bin). */
int or_alloc_bins(uint64_t n, int nbins, const double *w, uint64_t *counts) {
  double W = 0.0;
  for (int j = 0; j < nbins; ++j) {
    if (!(w[j] >= 0.0)) return OR_EINVAL;
    W += w[j];
  }
  if (!(W > 0.0)) return OR_EINVAL;
  double *frac = (double *)malloc(sizeof(double) * (size_t)nbins);
  if (!frac) return OR_ENOMEM;
  uint64_t used = 0;
  for (int j = 0; j < nbins; ++j) {
    double q = ((double)n * w[j]) / W;
    double fl = floor(q);
    counts[j] = (uint64_t)fl;
    frac[j] = q - fl;
    used += counts[j];
  }
  if (used > n) { free(frac); return OR_EINVAL; }
  uint64_t rem = n - used;
  /* hand out the remainder one at a time: largest fraction, lowest index */
  char *taken = (char *)calloc((size_t)nbins, 1);
  if (!taken) { free(frac); return OR_ENOMEM; }
  for (uint64_t r = 0; r < rem; ++r) {
    int best = -1;
    for (int j = 0; j < nbins; ++j) {
      if (taken[j]) continue;
      if (best < 0 || frac[j] > frac[best]) best = j;
    }
    if (best < 0) { free(frac); free(taken); return OR_EINVAL; }
    taken[best] = 1;
    counts[best] += 1;
  }
  free(frac);
  free(taken);
  return OR_OK;
}

/* ---------------- One history (Sec. 2.1, Fig. 2 right panel) ---------------- */

typedef struct {
  int64_t *T;          /* per-thread batch tally (q) */
  double *D;           /* per-thread FP64 batch tally (keV) */
  double e_inc, e_dep, e_esc;
  int64_t q_inc, q_dep, q_esc;
  uint64_t n_hist, n_steps, n_real, n_pe, n_compton, n_rayleigh, n_deposits,
      n_escapes, n_miss, n_cutoff, n_unscattered;
  double e_unscattered;
} tally_t;

typedef struct {
  or_event *buf;
  uint64_t cap, n, h0, h1;
  pthread_mutex_t mu;
} log_t;

static int64_t quant(double e) { return (int64_t)llrint(e * Q_SCALE); }

static void log_event(log_t *L, uint64_t h, uint32_t *seq, uint32_t k, int type, int64_t vox,
                      double e, double E) {
  if (!L || h < L->h0 || h >= L->h1) return;
  pthread_mutex_lock(&L->mu);
  if (L->n < L->cap) {
    or_event *ev = &L->buf[L->n];
    ev->h = h; ev->seq = *seq; ev->k = k; ev->type = type; ev->pad = 0;
    ev->vox = vox; ev->e = e; ev->E = E;
  }
  L->n += 1;
  pthread_mutex_unlock(&L->mu);
  *seq += 1;
}

static void deposit(tally_t *t, int64_t vox, double e) {
  int64_t q = quant(e);
  if (t->T) { t->T[vox] += q; t->D[vox] += e; }
  t->e_dep += e;
  t->q_dep += q;
  t->n_deposits += 1;
}

static void escape(tally_t *t, double E, int scattered) {
  t->e_esc += E;
  t->q_esc += quant(E);
  t->n_escapes += 1;
  if (!scattered) { t->n_unscattered += 1; t->e_unscattered += E; }
}

/* Source photon for history h drawn from spectrum bin j (Sec. 2.2.5-2.2.6). */
/* Fluence map (Sec. 2.2.4): beamlet I is drawn with probability f_I / F, by
 * inverse CDF: the smallest I whose running sum C_I exceeds u F. */
static int beamlet_of(const or_case *c, double u) {
  int n = c->fl_na * c->fl_nb;
  double x = u * c->fl_cdf[n - 1];
  int lo = 0, hi = n - 1;   /* C_{n-1} = F > x, so the answer is in [lo, hi] */
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if (c->fl_cdf[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* Alg. A1 on logical chains: history h belongs to chain h mod C and the chain
 * visits its histories in increasing h.  Each step draws a trial beamlet J
 * uniformly and zeta from the history's second source block and moves to J
 * when zeta < f_J / f_{I_last}; the comparison is taken as zeta * f_I < f_J,
 * exact in FP64 (24-bit operands).  A chain starts (at h = c) from a beamlet
 * drawn uniformly from the counter (0, c_lo, c_hi, 2). */
static int mh_initial(const or_case *c, uint64_t chain) {
  double v[4];
  uint32_t ctr[4] = {0u, (uint32_t)chain, (uint32_t)(chain >> 32), 2u};
  uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
  uint32_t r[4];
  philox4x32_10(ctr, key, r);
  for (int i = 0; i < 4; ++i) v[i] = unif(r[i]);
  return (int)(v[0] * (double)(c->fl_na * c->fl_nb));
}

/* Advance the chains over histories [h0, h0 + n) in increasing h; state[C]
 * holds each chain's last beamlet (read for chains already started). */
int or_mh_fill(const or_case *c, uint64_t h0, uint64_t n, int32_t *state, int32_t *out) {
  const uint64_t C = (uint64_t)c->fl_chains;
  const int nf = c->fl_na * c->fl_nb;
  if (C == 0 || nf <= 0 || !c->fl_f) return OR_EINVAL;
  for (uint64_t h = h0; h < h0 + n; ++h) {
    uint64_t chain = h % C;
    int I = h < C ? mh_initial(c, chain) : state[chain];
    double v[4];
    block_s(c, h, 0u, 1u, v);
    int J = (int)(v[0] * (double)nf);           /* 1. uniform trial beamlet */
    double zeta = v[1];                         /* 2. */
    if (zeta * (double)c->fl_f[I] < (double)c->fl_f[J]) I = J;   /* 3. */
    state[chain] = I;                           /* 5. */
    out[h - h0] = I;
  }
  return OR_OK;
}

static int beam_ok(const or_case *c, uint64_t h) {
  return c->fl_chains <= 0 || c->fl_na <= 0 ||
         (c->fl_beam && h >= c->fl_h0 && h - c->fl_h0 < c->fl_nbeam);
}

static void source(const or_case *c, uint64_t h, int j, double x[3], double d[3], double *E,
                   int *beamlet) {
  double u[4];
  block(c, h, 0u, u);
  *beamlet = -1;
  *E = c->bin_lo[j] + u[0] * c->bin_width;
  if (c->kind == 0) {
    double n = sqrt(c->dir[0] * c->dir[0] + c->dir[1] * c->dir[1] + c->dir[2] * c->dir[2]);
    for (int a = 0; a < 3; ++a) { x[a] = c->src[a]; d[a] = c->dir[a] / n; }
    return;
  }
  /* trajectory r(t) = iso + R (sin wt, cos wt, 0) + (0, 0, feed * wt / 2pi):
   * a circle when feed = 0, a helix otherwise; t at a projection angle */
  double swept_deg;
  if (c->nproj > 0) {
    double p = floor(u[1] * (double)c->nproj);
    if (p > (double)(c->nproj - 1)) p = (double)(c->nproj - 1);
    swept_deg = p * c->arc_deg / (double)c->nproj;
  } else {
    swept_deg = u[1] * c->arc_deg;
  }
  double phi = (c->phi0_deg + swept_deg) * DEG2RAD;
  double sp = sin(phi), cp = cos(phi);
  double zs = c->iso[2] + c->z_feed * swept_deg / 360.0;
  double S[3] = {c->iso[0] + c->sad * sp, c->iso[1] + c->sad * cp, zs};
  double a, b;
  if (c->fl_na > 0) {
    int I;
    if (c->fl_chains > 0) {
      I = c->fl_beam[h - c->fl_h0];   /* callers check the range (beam_ok) */
    } else {
      double v[4];
      block_s(c, h, 0u, 1u, v);
      I = beamlet_of(c, v[0]);
    }
    int ia = I % c->fl_na, ib = I / c->fl_na;
    /* uniform inside the beamlet */
    a = c->a0 + (ia + u[2]) * ((c->a1 - c->a0) / c->fl_na);
    b = c->b0 + (ib + u[3]) * ((c->b1 - c->b0) / c->fl_nb);
    *beamlet = I;
  } else {
    a = c->a0 + u[2] * (c->a1 - c->a0);
    b = c->b0 + u[3] * (c->b1 - c->b0);
  }
  /* point on the field rectangle through the axis at the source's height:
   * (iso_x, iso_y, zs) + a e_lat + b e_z */
  double P[3] = {c->iso[0] + a * cp, c->iso[1] - a * sp, zs + b};
  double v[3] = {P[0] - S[0], P[1] - S[1], P[2] - S[2]};
  double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int k = 0; k < 3; ++k) { x[k] = S[k]; d[k] = v[k] / n; }
}

/* Slab-method entry into the voxel box; returns 0 on a miss. */
static int enter_box(const or_case *c, double x[3], const double d[3]) {
  double lo[3] = {c->ox, c->oy, c->oz};
  double hi[3] = {c->ox + c->nx * c->dx, c->oy + c->ny * c->dy, c->oz + c->nz * c->dz};
  double tn = -INFINITY, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (x[a] < lo[a] || x[a] > hi[a]) return 0;
      continue;
    }
    double t1 = (lo[a] - x[a]) / d[a], t2 = (hi[a] - x[a]) / d[a];
    double n = t1 < t2 ? t1 : t2, f = t1 < t2 ? t2 : t1;
    if (n > tn) tn = n;
    if (f < tf) tf = f;
  }
  double tin = tn > 0.0 ? tn : 0.0;
  if (!(tin < tf)) return 0;
  for (int a = 0; a < 3; ++a) x[a] += tin * d[a];
  return 1;
}

/* New direction after deflection cos(theta) = mu and azimuth phi. */
static void rotate(double d[3], double mu, double phi) {
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double cp = cos(phi), sp = sin(phi);
  double u = d[0], v = d[1], w = d[2];
  double nu, nv, nw;
  if (fabs(w) < 1.0 - 1e-5) {
    double r = sqrt(1.0 - w * w);
    nu = u * mu + st * (u * w * cp - v * sp) / r;
    nv = v * mu + st * (v * w * cp + u * sp) / r;
    nw = w * mu - st * cp * r;
  } else {
    nu = st * cp;
    nv = st * sp;
    nw = (w >= 0.0 ? 1.0 : -1.0) * mu;
  }
  double n = sqrt(nu * nu + nv * nv + nw * nw);
  d[0] = nu / n; d[1] = nv / n; d[2] = nw / n;
}

static int history(const or_case *c, uint64_t h, int j, tally_t *t, log_t *L) {
  if (!beam_ok(c, h)) return OR_EINVAL;
  double x[3], d[3], E;
  uint32_t seq = 0;
  int beamlet;
  source(c, h, j, x, d, &E, &beamlet);
  t->n_hist += 1;
  t->e_inc += E;
  t->q_inc += quant(E);
  log_event(L, h, &seq, 0, EV_SOURCE, beamlet, E, E);
  if (!enter_box(c, x, d)) {
    t->n_miss += 1;
    escape(t, E, 0);
    log_event(L, h, &seq, 0, EV_MISS, -1, E, E);
    return OR_OK;
  }
  const double n3[3] = {(double)c->nx, (double)c->ny, (double)c->nz};
  const double o3[3] = {c->ox, c->oy, c->oz};
  const double d3[3] = {c->dx, c->dy, c->dz};
  int scattered = 0;
  pairs_t ps;
  ps.P = 0;
  for (uint32_t k = 1;; ++k) {
    if (ps.P >= K_MAX) return OR_ESTEPS;   /* a guard on the pairs taken */
    double u[2], v[2];
    next_pair(c, h, &ps, u);
    int je;
    double we;
    egrid(c, E, &je, &we);
    double mumax = lerp(c->mu_max[je], c->mu_max[je + 1], we);
    /* Woodcock free path in the homogeneous majorant medium */
    double s = -log(u[0]) / mumax;
    t->n_steps += 1;
    int idx[3];
    int out = 0;
    for (int a = 0; a < 3; ++a) {
      x[a] += s * d[a];
      double f = (x[a] - o3[a]) / d3[a];
      if (!(f >= 0.0 && f < n3[a])) { out = 1; continue; }
      int i = (int)floor(f);
      if (i > (int)n3[a] - 1) i = (int)n3[a] - 1;
      idx[a] = i;
    }
    if (out) {
      escape(t, E, scattered);
      log_event(L, h, &seq, k, EV_ESCAPE, -1, E, E);
      return OR_OK;
    }
    int64_t vox = ((int64_t)idx[2] * c->ny + idx[1]) * c->nx + idx[0];
    int m = c->mat[vox];
    double r = (double)c->rho[vox];
    const float *t0 = c->mu_rho + ((size_t)m * c->ne + je) * 3;
    const float *t1 = t0 + 3;
    double mpe = r * lerp(t0[0], t1[0], we);
    double mc = r * lerp(t0[1], t1[1], we);
    double mr = c->rayleigh ? r * lerp(t0[2], t1[2], we) : 0.0;
    double xi = u[1] * mumax;
    if (xi < mpe) {                                   /* photoelectric */
      t->n_real += 1; t->n_pe += 1;
      deposit(t, vox, E);
      log_event(L, h, &seq, k, EV_PHOTO, vox, E, 0.0);
      return OR_OK;
    } else if (xi < mpe + mc) {                       /* Compton */
      t->n_real += 1; t->n_compton += 1;
      scattered = 1;
      const float *CS = c->comp_surf + (c->comp_per_mat ? (size_t)m * c->ne * c->nzeta : 0);
      next_pair(c, h, &ps, v);
      double mu = surface(CS, c->nzeta, je, we, v[0]);
      double Ep = E / (1.0 + (E / ME_C2_KEV) * (1.0 - mu));
      deposit(t, vox, E - Ep);
      rotate(d, mu, TWO_PI * v[1]);
      log_event(L, h, &seq, k, EV_COMPTON, vox, E - Ep, Ep);
      E = Ep;
      if (E < c->e_cut) {
        t->n_cutoff += 1;
        deposit(t, vox, E);
        log_event(L, h, &seq, k, EV_CUTOFF, vox, E, 0.0);
        return OR_OK;
      }
    } else if (c->rayleigh && xi < mpe + mc + mr) {  /* Rayleigh */
      t->n_real += 1; t->n_rayleigh += 1;
      scattered = 1;
      const float *S = c->rayl_surf + (size_t)m * c->ne * c->nzeta;
      next_pair(c, h, &ps, v);
      double mu = surface(S, c->nzeta, je, we, v[0]);
      rotate(d, mu, TWO_PI * v[1]);
      log_event(L, h, &seq, k, EV_RAYLEIGH, vox, 0.0, E);
    }
    /* else fictitious: state unchanged */
  }
}

/* ---------------- Batches (Sec. 2.2.1) and threads ---------------- */

typedef struct {
  const or_case *c;
  uint64_t h_begin, n;        /* batch ids [h_begin, h_begin+n) */
  const uint64_t *prefix;     /* [nbins+1] bin-major offsets inside the batch */
  uint64_t lo, hi;            /* this thread's slice of [0, n) */
  tally_t *t;
  log_t *L;
  int rc;
} work_t;

static void *worker(void *arg) {
  work_t *w = (work_t *)arg;
  int j = 0;
  for (uint64_t i = w->lo; i < w->hi; ++i) {
    while (i >= w->prefix[j + 1]) ++j;
    int rc = history(w->c, w->h_begin + i, j, w->t, w->L);
    if (rc != OR_OK) { w->rc = rc; return NULL; }
  }
  w->rc = OR_OK;
  return NULL;
}

static void add_u128(uint64_t *hi, uint64_t *lo, unsigned __int128 v) {
  unsigned __int128 cur = ((unsigned __int128)*hi << 64) | *lo;
  cur += v;
  *hi = (uint64_t)(cur >> 64);
  *lo = (uint64_t)cur;
}

/* Run the given batches (sizes in order) starting at history id h0. */
int or_run(const or_case *c, uint64_t h0, const uint64_t *batch_sizes, int n_batches,
           int n_threads, or_result *res) {
  if (!c || !res || n_batches < 0 || n_threads < 1) return OR_EINVAL;
  if (c->ne < 2 || c->nzeta < 2 || c->nbins < 1 || c->nx < 1 || c->ny < 1 || c->nz < 1)
    return OR_EINVAL;
  int64_t V = (int64_t)c->nx * c->ny * c->nz;
  tally_t *tt = (tally_t *)calloc((size_t)n_threads, sizeof(tally_t));
  work_t *ww = (work_t *)calloc((size_t)n_threads, sizeof(work_t));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  uint64_t *cnt = (uint64_t *)calloc((size_t)c->nbins, sizeof(uint64_t));
  uint64_t *prefix = (uint64_t *)calloc((size_t)c->nbins + 1, sizeof(uint64_t));
  int rc = OR_OK;
  if (!tt || !ww || !th || !cnt || !prefix) { rc = OR_ENOMEM; goto done; }
  for (int i = 0; i < n_threads; ++i) {
    tt[i].T = (int64_t *)calloc((size_t)V, sizeof(int64_t));
    tt[i].D = (double *)calloc((size_t)V, sizeof(double));
    if (!tt[i].T || !tt[i].D) { rc = OR_ENOMEM; goto done; }
  }
  log_t L;
  memset(&L, 0, sizeof(L));
  L.buf = res->log; L.cap = res->log_cap; L.h0 = res->log_h0; L.h1 = res->log_h1;
  pthread_mutex_init(&L.mu, NULL);
  log_t *Lp = res->log ? &L : NULL;

  uint64_t h = h0;
  res->n_batches = 0;
  for (int b = 0; b < n_batches && rc == OR_OK; ++b) {
    uint64_t n = batch_sizes[b];
    rc = or_alloc_bins(n, c->nbins, c->bin_w, cnt);
    if (rc != OR_OK) break;
    prefix[0] = 0;
    for (int k = 0; k < c->nbins; ++k) prefix[k + 1] = prefix[k] + cnt[k];
    for (int i = 0; i < n_threads; ++i) {
      ww[i].c = c; ww[i].h_begin = h; ww[i].n = n; ww[i].prefix = prefix;
      ww[i].lo = n * (uint64_t)i / (uint64_t)n_threads;
      ww[i].hi = n * (uint64_t)(i + 1) / (uint64_t)n_threads;
      ww[i].t = &tt[i]; ww[i].L = Lp; ww[i].rc = OR_OK;
    }
    if (n_threads == 1) {
      worker(&ww[0]);
    } else {
      for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, worker, &ww[i]);
      for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    }
    for (int i = 0; i < n_threads; ++i)
      if (ww[i].rc != OR_OK) rc = ww[i].rc;
    if (rc != OR_OK) break;
    /* exact merge of the per-thread batch tallies, then fold into S1, S2 */
    for (int64_t v = 0; v < V; ++v) {
      int64_t tb = 0;
      double db = 0.0;
      for (int i = 0; i < n_threads; ++i) {
        tb += tt[i].T[v]; tt[i].T[v] = 0;
        db += tt[i].D[v]; tt[i].D[v] = 0.0;
      }
      if (tb != 0) {
        res->s1[v] += tb;
        unsigned __int128 sq = (unsigned __int128)(uint64_t)tb * (unsigned __int128)(uint64_t)tb;
        add_u128(&res->s2_hi[v], &res->s2_lo[v], sq);
      }
      if (res->shadow) res->shadow[v] += db;
      if (res->shadow_sq) res->shadow_sq[v] += db * db;
    }
    res->n_batches += 1;
    h += n;
  }
  for (int i = 0; i < n_threads; ++i) {
    tally_t *t = &tt[i];
    res->e_inc += t->e_inc; res->e_dep += t->e_dep; res->e_esc += t->e_esc;
    res->q_inc += t->q_inc; res->q_dep += t->q_dep; res->q_esc += t->q_esc;
    res->n_hist += t->n_hist; res->n_steps += t->n_steps; res->n_real += t->n_real;
    res->n_pe += t->n_pe; res->n_compton += t->n_compton; res->n_rayleigh += t->n_rayleigh;
    res->n_deposits += t->n_deposits; res->n_escapes += t->n_escapes; res->n_miss += t->n_miss;
    res->n_cutoff += t->n_cutoff; res->n_unscattered += t->n_unscattered;
    res->e_unscattered += t->e_unscattered;
  }
  res->log_n = L.n;
  pthread_mutex_destroy(&L.mu);
done:
  for (int i = 0; tt && i < n_threads; ++i) { free(tt[i].T); free(tt[i].D); }
  free(tt); free(ww); free(th); free(cnt); free(prefix);
  return rc;
}

/* One history h from bin j with every event logged (sampled comparisons at
 * full workload size); no volume tally is kept. */
int or_history(const or_case *c, uint64_t h, int j, or_event *buf, uint64_t cap, uint64_t *n_out) {
  tally_t t;
  memset(&t, 0, sizeof(t)); /* no volume tally: events only */
  log_t L;
  memset(&L, 0, sizeof(L));
  L.buf = buf; L.cap = cap; L.h0 = h; L.h1 = h + 1;
  pthread_mutex_init(&L.mu, NULL);
  int rc = history(c, h, j, &t, &L);
  pthread_mutex_destroy(&L.mu);
  *n_out = L.n;
  return rc;
}

/* Sum of quantised deposits per voxel: the tally a deposit list implies. */
int or_tally_replay(uint64_t n, const int64_t *vox, const float *e, int64_t V, int64_t *T) {
  for (uint64_t i = 0; i < n; ++i) {
    if (vox[i] < 0 || vox[i] >= V) return OR_EINVAL;
    T[vox[i]] += quant((double)e[i]);
  }
  return OR_OK;
}

/* ---------------- Batch statistics (Sec. 2.2.1, Sec. 3.1) ----------------
 * Batch means over nb batches: mean of the batch tallies S1/nb, variance of
 * that mean (nb*S2 - S1^2) / (nb^2 (nb-1)).  The numerator is formed exactly
 * in 192-bit integer arithmetic and converted to double last. */
int or_batch_stats(int64_t V, const int64_t *s1, const uint64_t *s2_hi, const uint64_t *s2_lo,
                   uint32_t nb, double *mean, double *var_of_mean) {
  if (nb < 2) return OR_EINVAL;
  for (int64_t v = 0; v < V; ++v) {
    if (s1[v] < 0) return OR_EINVAL;
    /* A = nb * S2 as three 64-bit limbs */
    unsigned __int128 lo = (unsigned __int128)s2_lo[v] * nb;
    unsigned __int128 mid = (unsigned __int128)s2_hi[v] * nb + (uint64_t)(lo >> 64);
    uint64_t a0 = (uint64_t)lo, a1 = (uint64_t)mid, a2 = (uint64_t)(mid >> 64);
    /* B = S1^2 (< 2^126) */
    unsigned __int128 B = (unsigned __int128)(uint64_t)s1[v] * (uint64_t)s1[v];
    uint64_t b0 = (uint64_t)B, b1 = (uint64_t)(B >> 64);
    /* A - B (>= 0 by Cauchy-Schwarz) */
    uint64_t r0 = a0 - b0, br = a0 < b0;
    uint64_t r1 = a1 - b1 - br;
    uint64_t br2 = (a1 < b1) || (a1 - b1 < br);
    uint64_t r2 = a2 - br2;
    if (a2 < br2) return OR_EINVAL;
    double num = (double)r2 * 0x1p128 + (double)r1 * 0x1p64 + (double)r0;
    mean[v] = (double)s1[v] / (double)nb;
    var_of_mean[v] = num / ((double)nb * (double)nb * (double)(nb - 1));
  }
  return OR_OK;
}

/* Test hooks: the transport's own surface lookup and source sampler. */
int or_sample_surface(const float *S, int ne, int nzeta, double e0, double de, double E,
                      const double *zeta, int64_t n, double *out) {
  or_case c;
  memset(&c, 0, sizeof(c));
  c.ne = ne; c.e0 = e0; c.de = de;
  int j;
  double w;
  egrid(&c, E, &j, &w);
  for (int64_t i = 0; i < n; ++i) out[i] = surface(S, nzeta, j, w, zeta[i]);
  return OR_OK;
}

/* out[8] = x, y, z, u, v, w, E, hit (after the slab entry when hit = 1) */
int or_sample_source(const or_case *c, uint64_t h, int j, double *out) {
  if (!beam_ok(c, h)) return OR_EINVAL;
  double x[3], d[3], E;
  int beamlet;
  source(c, h, j, x, d, &E, &beamlet);
  double y[3] = {x[0], x[1], x[2]};
  int hit = enter_box(c, y, d);
  for (int a = 0; a < 3; ++a) { out[a] = x[a]; out[3 + a] = d[a]; }
  out[6] = E;
  out[7] = (double)hit;
  out[8] = (double)beamlet;
  return OR_OK;
}

/* Test hook: the transport's direction update. d[3] in/out. */
void or_rotate(double *d, double mu, double phi) { rotate(d, mu, phi); }
