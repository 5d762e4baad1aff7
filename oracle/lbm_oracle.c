/*
 * FP64 reference ("oracle") for the reactive two-component lattice Boltzmann
 * step.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU
 * baseline leg of the benchmark are its only users.  It shares no code, header
 * or table with the HIP library; the two only see the same host input arrays.
 *
 * What it computes follows Sergi, Grossi, Leidi, Ortona, "Lattice Boltzmann
 * simulation of the surface growth effects for the infiltration of molten Si
 * in carbon preforms", section "LB models":
 *   - BGK collision on a discretised velocity space, bounce-back at the solid
 *     phase, two fluid components;
 *   - fluid-fluid cohesion (surface tension) and solid-fluid adhesion
 *     (wetting) forces of the Martys-Chen/Shan-Chen type;
 *   - a BGK advection-diffusion lattice for the dissolved species, weakly
 *     coupled to the flow (it only reads the flow velocity);
 *   - surface reaction by mass precipitation with rate constant k_r: mass
 *     deposits on the surface and, once the accumulated mass exceeds a
 *     threshold, the node turns solid (surface growth, pore closure).
 * The paper prints no formula for these steps; the readings used (D2Q9 and
 * D2Q5 lattices, the velocity-shift forcing, halfway bounce-back, the first
 * order sink at wall-adjacent nodes, synchronous growth at the end of the step)
 * are listed with the design notes of this repository.  The code is written
 * for checking by eye, one loop per step in the order S1..S8, no fusion.
 *
 * Lattice: nx*ny nodes, index y*nx + x, periodic in x and y; walls exist only
 * through the solid mask.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9: rest, 4 axis links, 4 diagonal links. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* D2Q5 for the solute: the first five D2Q9 vectors, sound speed^2 = 1/3. */
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};

typedef struct {
  int32_t nx, ny;
  double tau;        /* flow relaxation time, both components */
  double G;          /* cohesion strength between the two components */
  double G_ads[2];   /* adhesion strength of component 1 (wetting) and 2 */
  double tau_g;      /* solute relaxation time; 0 = no solute lattice */
  double k_r;        /* reaction-rate constant [lu/ts]; 0 = no reaction */
  double threshold;  /* precipitated mass above which a node turns solid */
  double accel[2];   /* uniform body acceleration (test use) */
  int32_t x_in, x_out, y0, W; /* capillary descriptor, W = 0: none */
  double c_eq;       /* saturation: precipitation k_r n_s phi (C - c_eq) above it */
  double c_hold;     /* held concentration of the source region */
  int32_t hold_x;    /* source region x < hold_x, 0 = none */
  int32_t solute_q;  /* solute lattice: 0/5 = D2Q5, 4 = D2Q4 */
} orc_params;

typedef struct {
  int32_t x, y;
  int64_t step;
} orc_event;

typedef struct {
  int64_t step;
  double mass[2], mass_removed[2];
  double solute, precipitate, solute_removed;
  double front_z, delta_e;
  int64_t closure_step;
  int64_t n_solid, n_events;
  int32_t nonfinite;
  int32_t pad;
  double r_min, r_ave, r_h; /* capillary radii (Fig. 4), NaN without a capillary */
} orc_obs;

typedef struct {
  int32_t x, y;
  int64_t step;
  int32_t decision;
} orc_forced;

typedef struct orc_sim {
  orc_params p;
  long N;
  double *f, *fs;  /* populations [2*9][N]: state and post-collision */
  double *g, *gs;  /* solute populations [5][N] */
  uint8_t *s;      /* solid mask */
  double *m;       /* precipitated mass per node */
  int64_t *solid_step; /* -1 fluid, 0 solid from the start, else step it turned solid */
  double *rho, *jx, *jy, *Fx, *Fy; /* [2][N] scratch: moments and forces */
  double *C, *ux, *uy;             /* [N] scratch */
  uint8_t *grow;                   /* [N] scratch: growth decision */
  double removed[3];               /* mass of component 1, 2 and solute taken out by growth */
  int64_t step;
  orc_event *ev;
  int64_t nev, evcap;
  orc_forced *ov;
  int64_t nov, ovcap;
} orc_sim;

#define F(sim, sg, i, k) ((sim)->f[((long)(sg) * 9 + (i)) * (sim)->N + (k)])
#define FS(sim, sg, i, k) ((sim)->fs[((long)(sg) * 9 + (i)) * (sim)->N + (k)])
#define Gq(sim, i, k) ((sim)->g[(long)(i) * (sim)->N + (k)])
#define GS(sim, i, k) ((sim)->gs[(long)(i) * (sim)->N + (k)])

static long wrap(long a, long n) { return ((a % n) + n) % n; }
static long nbr(const orc_sim *sim, long x, long y, int dx, int dy) {
  return wrap(y + dy, sim->p.ny) * sim->p.nx + wrap(x + dx, sim->p.nx);
}

/* Equilibrium of the D2Q9 BGK model at density rho and velocity (ux, uy):
 * w_i rho [1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u]. */
void orc_feq(double rho, double ux, double uy, double *out9) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; i++) {
    double eu = EX[i] * ux + EY[i] * uy;
    out9[i] = W9[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

/* Solute equilibrium, linear in the advecting velocity: D2Q5 (sound speed^2
 * 1/3) or D2Q4 (the four axis links with weight 1/4, sound speed^2 1/2, no
 * rest link). */
static double geq(const orc_params *p, int k, double C, double ux, double uy) {
  if (p->solute_q == 4) return k == 0 ? 0.0 : 0.25 * C * (1.0 + 2.0 * (EX[k] * ux + EY[k] * uy));
  return W5[k] * C * (1.0 + 3.0 * (EX[k] * ux + EY[k] * uy));
}

int orc_check_params(const orc_params *p) {
  if (!p) return 0;
  if (p->nx < 3 || p->ny < 3) return 0;
  if (!(p->tau > 0.5)) return 0;
  if (!(p->tau_g == 0.0 || p->tau_g > 0.5)) return 0;
  if (!(p->k_r >= 0.0) || 4.0 * p->k_r > 1.0) return 0;
  if (!(p->threshold > 0.0)) return 0;
  if (!(p->c_eq >= 0.0) || !isfinite(p->c_eq)) return 0;
  if (!(p->c_hold >= 0.0) || !isfinite(p->c_hold)) return 0;
  if (p->hold_x < 0 || p->hold_x > p->nx || (p->hold_x > 0 && p->tau_g == 0.0)) return 0;
  if (p->solute_q != 0 && p->solute_q != 4 && p->solute_q != 5) return 0;
  if (p->W < 0) return 0;
  if (p->W > 0) {
    if (p->x_in < 0 || p->x_out > p->nx || p->x_in + 2 > p->x_out) return 0;
    if (p->y0 < 0 || p->y0 + p->W > p->ny) return 0;
  }
  return 1;
}

void orc_destroy(orc_sim *sim) {
  if (!sim) return;
  free(sim->f); free(sim->fs); free(sim->g); free(sim->gs); free(sim->s);
  free(sim->m); free(sim->solid_step); free(sim->rho); free(sim->jx); free(sim->jy);
  free(sim->Fx); free(sim->Fy); free(sim->C); free(sim->ux); free(sim->uy);
  free(sim->grow); free(sim->ev); free(sim->ov);
  free(sim);
}

static orc_sim *alloc_sim(const orc_params *p) {
  if (!orc_check_params(p)) return NULL;
  orc_sim *sim = (orc_sim *)calloc(1, sizeof(orc_sim));
  if (!sim) return NULL;
  sim->p = *p;
  long N = (long)p->nx * p->ny;
  sim->N = N;
  sim->f = (double *)calloc(18 * N, sizeof(double));
  sim->fs = (double *)calloc(18 * N, sizeof(double));
  sim->g = (double *)calloc(5 * N, sizeof(double));
  sim->gs = (double *)calloc(5 * N, sizeof(double));
  sim->s = (uint8_t *)calloc(N, 1);
  sim->m = (double *)calloc(N, sizeof(double));
  sim->solid_step = (int64_t *)calloc(N, sizeof(int64_t));
  sim->rho = (double *)calloc(2 * N, sizeof(double));
  sim->jx = (double *)calloc(2 * N, sizeof(double));
  sim->jy = (double *)calloc(2 * N, sizeof(double));
  sim->Fx = (double *)calloc(2 * N, sizeof(double));
  sim->Fy = (double *)calloc(2 * N, sizeof(double));
  sim->C = (double *)calloc(N, sizeof(double));
  sim->ux = (double *)calloc(N, sizeof(double));
  sim->uy = (double *)calloc(N, sizeof(double));
  sim->grow = (uint8_t *)calloc(N, 1);
  if (!sim->f || !sim->fs || !sim->g || !sim->gs || !sim->s || !sim->m || !sim->solid_step ||
      !sim->rho || !sim->jx || !sim->jy || !sim->Fx || !sim->Fy || !sim->C || !sim->ux ||
      !sim->uy || !sim->grow) {
    orc_destroy(sim);
    return NULL;
  }
  return sim;
}

/* Start from densities at rest: f_i = w_i rho_sigma, g_k = w_k C. */
orc_sim *orc_create(const orc_params *p, const uint8_t *solid, const double *rho1,
                    const double *rho2, const double *conc) {
  orc_sim *sim = alloc_sim(p);
  if (!sim) return NULL;
  long N = sim->N;
  for (long k = 0; k < N; k++) {
    if (solid[k] > 1) { orc_destroy(sim); return NULL; }
    sim->s[k] = solid[k];
    sim->solid_step[k] = solid[k] ? 0 : -1;
    if (solid[k]) continue;
    for (int i = 0; i < 9; i++) {
      F(sim, 0, i, k) = W9[i] * rho1[k];
      F(sim, 1, i, k) = W9[i] * rho2[k];
    }
    if (conc)
      for (int q = 0; q < 5; q++) Gq(sim, q, k) = geq(p, q, conc[k], 0.0, 0.0);
  }
  return sim;
}

/* Arbitrary state: populations f [18][N] (component-major), g [5][N] or NULL,
 * mask, precipitate m or NULL.  Populations at solid nodes are ignored. */
orc_sim *orc_create_state(const orc_params *p, const uint8_t *solid, const double *f,
                          const double *g, const double *m) {
  orc_sim *sim = alloc_sim(p);
  if (!sim) return NULL;
  long N = sim->N;
  for (long k = 0; k < N; k++) {
    if (solid[k] > 1) { orc_destroy(sim); return NULL; }
    sim->s[k] = solid[k];
    sim->solid_step[k] = solid[k] ? 0 : -1;
    if (m) sim->m[k] = m[k];
    if (solid[k]) continue;
    for (int q = 0; q < 18; q++) sim->f[q * N + k] = f[q * N + k];
    if (g)
      for (int q = 0; q < 5; q++) Gq(sim, q, k) = g[q * N + k];
  }
  return sim;
}

/* S1 (moments) and S2 (forces) for the current state.  Solid nodes carry
 * rho = 0, so a solid neighbour adds nothing to the cohesion sum. */
static void moments_and_forces(orc_sim *sim) {
  const orc_params *p = &sim->p;
  const long N = sim->N;
  /* S1 */
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; k++) {
    for (int sg = 0; sg < 2; sg++) {
      double r = 0, jx = 0, jy = 0;
      if (!sim->s[k]) {
        for (int i = 0; i < 9; i++) {
          r += F(sim, sg, i, k);
          jx += F(sim, sg, i, k) * EX[i];
          jy += F(sim, sg, i, k) * EY[i];
        }
      }
      sim->rho[sg * N + k] = r;
      sim->jx[sg * N + k] = jx;
      sim->jy[sg * N + k] = jy;
    }
    double c = 0;
    if (!sim->s[k] && p->tau_g > 0)
      for (int q = 0; q < 5; q++) c += Gq(sim, q, k);
    sim->C[k] = c;
  }
  /* S2: F_s = -G rho_s(x) sum_i w_i rho_other(x+e_i) e_i
   *           - G_ads,s rho_s(x) sum_i w_i s(x+e_i) e_i + rho_s(x) a */
#pragma omp parallel for schedule(static)
  for (long y = 0; y < p->ny; y++) {
    for (long x = 0; x < p->nx; x++) {
      long k = y * p->nx + x;
      for (int sg = 0; sg < 2; sg++) {
        double fx = 0, fy = 0;
        if (!sim->s[k]) {
          double cx = 0, cy = 0, ax = 0, ay = 0;
          for (int i = 1; i < 9; i++) {
            long kn = nbr(sim, x, y, EX[i], EY[i]);
            double other = sim->rho[(1 - sg) * N + kn];
            cx += W9[i] * other * EX[i];
            cy += W9[i] * other * EY[i];
            ax += W9[i] * sim->s[kn] * EX[i];
            ay += W9[i] * sim->s[kn] * EY[i];
          }
          double r = sim->rho[sg * N + k];
          fx = -p->G * r * cx - p->G_ads[sg] * r * ax + r * p->accel[0];
          fy = -p->G * r * cy - p->G_ads[sg] * r * ay + r * p->accel[1];
        }
        sim->Fx[sg * N + k] = fx;
        sim->Fy[sg * N + k] = fy;
      }
      /* physical (barycentric) velocity, half-force corrected */
      double rt = sim->rho[k] + sim->rho[N + k];
      if (!sim->s[k] && rt > 0) {
        sim->ux[k] = (sim->jx[k] + sim->jx[N + k] + 0.5 * (sim->Fx[k] + sim->Fx[N + k])) / rt;
        sim->uy[k] = (sim->jy[k] + sim->jy[N + k] + 0.5 * (sim->Fy[k] + sim->Fy[N + k])) / rt;
      } else {
        sim->ux[k] = 0;
        sim->uy[k] = 0;
      }
    }
  }
}

static int axis_solid_neighbours(const orc_sim *sim, long x, long y) {
  int n = 0;
  for (int i = 1; i <= 4; i++) n += sim->s[nbr(sim, x, y, EX[i], EY[i])];
  return n;
}

static void log_event(orc_sim *sim, int32_t x, int32_t y, int64_t step) {
  if (sim->nev == sim->evcap) {
    int64_t cap = sim->evcap ? 2 * sim->evcap : 1024;
    orc_event *e = (orc_event *)realloc(sim->ev, cap * sizeof(orc_event));
    if (!e) abort();
    sim->ev = e;
    sim->evcap = cap;
  }
  sim->ev[sim->nev].x = x;
  sim->ev[sim->nev].y = y;
  sim->ev[sim->nev].step = step;
  sim->nev++;
}

/* One time step n -> n+1. */
static void step_once(orc_sim *sim) {
  const orc_params *p = &sim->p;
  const long N = sim->N;
  const double tau = p->tau;
  moments_and_forces(sim); /* S1, S2 */

  /* S3 velocities and S4 BGK collision of both components */
#pragma omp parallel for schedule(static)
  for (long k = 0; k < N; k++) {
    if (sim->s[k]) continue;
    double r1 = sim->rho[k], r2 = sim->rho[N + k];
    /* common velocity u' = (sum_s j_s / tau) / (sum_s rho_s / tau) */
    double den = r1 / tau + r2 / tau;
    double upx = (sim->jx[k] / tau + sim->jx[N + k] / tau) / den;
    double upy = (sim->jy[k] / tau + sim->jy[N + k] / tau) / den;
    for (int sg = 0; sg < 2; sg++) {
      double r = sim->rho[sg * N + k];
      double vx = upx, vy = upy;
      if (r > 0) { /* velocity shift u_eq = u' + tau F / rho */
        vx += tau * sim->Fx[sg * N + k] / r;
        vy += tau * sim->Fy[sg * N + k] / r;
      }
      double feq[9];
      orc_feq(r, vx, vy, feq);
      for (int i = 0; i < 9; i++)
        FS(sim, sg, i, k) = F(sim, sg, i, k) - (F(sim, sg, i, k) - feq[i]) / tau;
    }
  }

  if (p->tau_g > 0) {
    /* S5 solute BGK, advected by the physical velocity */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < N; k++) {
      if (sim->s[k]) continue;
      for (int q = 0; q < 5; q++)
        GS(sim, q, k) = Gq(sim, q, k) - (Gq(sim, q, k) - geq(p, q, sim->C[k], sim->ux[k], sim->uy[k])) / p->tau_g;
    }
    /* S6 surface reaction at fluid nodes with n_s >= 1 solid axis neighbours:
     * r = k_r n_s phi, m += r C, solute populations scaled by (1 - r).  With a
     * saturation concentration c_eq > 0 only the excess precipitates:
     * m += r (C - c_eq) when C > c_eq, and the solute keeps C - r (C - c_eq). */
    if (p->k_r > 0) {
#pragma omp parallel for schedule(static)
      for (long y = 0; y < p->ny; y++) {
        for (long x = 0; x < p->nx; x++) {
          long k = y * p->nx + x;
          if (sim->s[k]) continue;
          int ns = axis_solid_neighbours(sim, x, y);
          if (ns == 0) continue;
          double phi = sim->rho[k] / (sim->rho[k] + sim->rho[N + k]);
          double r = p->k_r * ns * phi;
          if (p->c_eq > 0) {
            double excess = sim->C[k] > p->c_eq ? sim->C[k] - p->c_eq : 0.0;
            double dm = r * excess;
            sim->m[k] += dm;
            if (dm > 0)
              for (int q = 0; q < 5; q++) GS(sim, q, k) *= (1.0 - dm / sim->C[k]);
          } else {
            sim->m[k] += r * sim->C[k];
            for (int q = 0; q < 5; q++) GS(sim, q, k) *= (1.0 - r);
          }
        }
      }
    }
    /* held source: the post-collision solute of every fluid node with
     * x < hold_x is the equilibrium at c_hold (a reservoir kept at fixed
     * concentration) */
    if (p->hold_x > 0) {
#pragma omp parallel for schedule(static)
      for (long y = 0; y < p->ny; y++)
        for (long x = 0; x < p->hold_x; x++) {
          long k = y * p->nx + x;
          if (sim->s[k]) continue;
          for (int q = 0; q < 5; q++) GS(sim, q, k) = geq(p, q, p->c_hold, sim->ux[k], sim->uy[k]);
        }
    }
  }

  /* S7 streaming with halfway bounce-back, mask of step n */
#pragma omp parallel for schedule(static)
  for (long y = 0; y < p->ny; y++) {
    for (long x = 0; x < p->nx; x++) {
      long k = y * p->nx + x;
      if (sim->s[k]) continue;
      for (int sg = 0; sg < 2; sg++)
        for (int i = 0; i < 9; i++) {
          long kb = nbr(sim, x, y, -EX[i], -EY[i]);
          F(sim, sg, i, k) = sim->s[kb] ? FS(sim, sg, OPP[i], k) : FS(sim, sg, i, kb);
        }
      if (p->tau_g > 0)
        for (int q = 0; q < 5; q++) {
          long kb = nbr(sim, x, y, -EX[q], -EY[q]);
          Gq(sim, q, k) = sim->s[kb] ? GS(sim, OPP[q], k) : GS(sim, q, kb);
        }
    }
  }

  /* S8 growth, synchronous: every fluid node whose precipitate exceeds the
   * threshold turns solid; its populations leave the fluid and are booked. */
  const int64_t next = sim->step + 1;
  if (p->k_r > 0) {
    for (long k = 0; k < N; k++) sim->grow[k] = !sim->s[k] && sim->m[k] > p->threshold;
    for (int64_t o = 0; o < sim->nov; o++) {
      if (sim->ov[o].step != next) continue;
      long k = (long)sim->ov[o].y * p->nx + sim->ov[o].x;
      if (!sim->s[k]) sim->grow[k] = (uint8_t)(sim->ov[o].decision != 0);
    }
    for (long k = 0; k < N; k++) {
      if (!sim->grow[k]) continue;
      for (int sg = 0; sg < 2; sg++)
        for (int i = 0; i < 9; i++) {
          sim->removed[sg] += F(sim, sg, i, k);
          F(sim, sg, i, k) = 0;
        }
      for (int q = 0; q < 5; q++) {
        sim->removed[2] += Gq(sim, q, k);
        Gq(sim, q, k) = 0;
      }
      sim->s[k] = 1;
      sim->solid_step[k] = next;
      log_event(sim, (int32_t)(k % p->nx), (int32_t)(k / p->nx), next);
    }
  }
  sim->step = next;
}

void orc_step(orc_sim *sim, int64_t n) {
  for (int64_t t = 0; t < n; t++) step_once(sim);
}

/* Deep copy of a simulation (used to rewind a window when comparing growth
 * decisions made at two precisions). */
orc_sim *orc_clone(const orc_sim *src) {
  orc_sim *sim = alloc_sim(&src->p);
  if (!sim) return NULL;
  long N = src->N;
  memcpy(sim->f, src->f, 18 * N * sizeof(double));
  memcpy(sim->g, src->g, 5 * N * sizeof(double));
  memcpy(sim->s, src->s, N);
  memcpy(sim->m, src->m, N * sizeof(double));
  memcpy(sim->solid_step, src->solid_step, N * sizeof(int64_t));
  memcpy(sim->removed, src->removed, sizeof sim->removed);
  sim->step = src->step;
  if (src->nev) {
    sim->ev = (orc_event *)malloc(src->nev * sizeof(orc_event));
    if (!sim->ev) { orc_destroy(sim); return NULL; }
    memcpy(sim->ev, src->ev, src->nev * sizeof(orc_event));
    sim->nev = sim->evcap = src->nev;
  }
  if (src->nov) {
    sim->ov = (orc_forced *)malloc(src->nov * sizeof(orc_forced));
    if (!sim->ov) { orc_destroy(sim); return NULL; }
    memcpy(sim->ov, src->ov, src->nov * sizeof(orc_forced));
    sim->nov = sim->ovcap = src->nov;
  }
  return sim;
}

/* Force the growth decision of node (x, y) at the step that produces state
 * `step` (used when a decision is a certified tie between two precisions). */
int orc_override(orc_sim *sim, int32_t x, int32_t y, int64_t step, int32_t decision) {
  if (x < 0 || y < 0 || x >= sim->p.nx || y >= sim->p.ny) return -1;
  if (sim->nov == sim->ovcap) {
    int64_t cap = sim->ovcap ? 2 * sim->ovcap : 16;
    orc_forced *o = (orc_forced *)realloc(sim->ov, cap * sizeof(orc_forced));
    if (!o) return -1;
    sim->ov = o;
    sim->ovcap = cap;
  }
  orc_forced *o = &sim->ov[sim->nov++];
  o->x = x; o->y = y; o->step = step; o->decision = decision;
  return 0;
}

/* Macroscopic fields of the current state (any pointer may be NULL). */
void orc_fields(orc_sim *sim, double *rho1, double *rho2, double *ux, double *uy, double *conc,
                double *m, uint8_t *solid) {
  moments_and_forces(sim);
  long N = sim->N;
  for (long k = 0; k < N; k++) {
    if (rho1) rho1[k] = sim->rho[k];
    if (rho2) rho2[k] = sim->rho[N + k];
    if (ux) ux[k] = sim->ux[k];
    if (uy) uy[k] = sim->uy[k];
    if (conc) conc[k] = sim->C[k];
    if (m) m[k] = sim->m[k];
    if (solid) solid[k] = sim->s[k];
  }
}

/* Forces on both components for the current state, [2][N] each. */
void orc_forces(orc_sim *sim, double *Fx, double *Fy) {
  moments_and_forces(sim);
  memcpy(Fx, sim->Fx, 2 * sim->N * sizeof(double));
  memcpy(Fy, sim->Fy, 2 * sim->N * sizeof(double));
}

void orc_get_state(const orc_sim *sim, double *f, double *g, double *m) {
  if (f) memcpy(f, sim->f, 18 * sim->N * sizeof(double));
  if (g) memcpy(g, sim->g, 5 * sim->N * sizeof(double));
  if (m) memcpy(m, sim->m, sim->N * sizeof(double));
}

int64_t orc_events(const orc_sim *sim, orc_event *buf, int64_t cap) {
  int64_t n = sim->nev < cap ? sim->nev : cap;
  if (buf && n > 0) memcpy(buf, sim->ev, n * sizeof(orc_event));
  return sim->nev;
}

int64_t orc_step_count(const orc_sim *sim) { return sim->step; }

/* Observables of the current state.  Front: phi = rho1/(rho1+rho2) averaged
 * over the centreline row(s) of the channel; the invading front is the first
 * crossing of phi = 1/2 from the capillary inlet, linearly interpolated and
 * measured from x_in.  Growth: for every capillary column the number of
 * consecutive solid nodes grown from each wall; delta_e is the largest (half
 * the width for a column that is closed). */
void orc_observe(orc_sim *sim, orc_obs *o) {
  const orc_params *p = &sim->p;
  const long N = sim->N;
  moments_and_forces(sim);
  memset(o, 0, sizeof(*o));
  o->step = sim->step;
  for (long k = 0; k < N; k++) {
    if (sim->s[k]) {
      o->n_solid++;
    } else {
      o->mass[0] += sim->rho[k];
      o->mass[1] += sim->rho[N + k];
      o->solute += sim->C[k];
      if (!isfinite(sim->rho[k]) || !isfinite(sim->rho[N + k]) || !isfinite(sim->C[k]))
        o->nonfinite = 1;
    }
    o->precipitate += sim->m[k];
  }
  o->mass_removed[0] = sim->removed[0];
  o->mass_removed[1] = sim->removed[1];
  o->solute_removed = sim->removed[2];
  o->n_events = sim->nev;
  o->front_z = NAN;
  o->delta_e = 0;
  o->closure_step = -1;
  o->r_min = o->r_ave = o->r_h = NAN;
  if (p->W <= 0) return;

  /* centre row(s) */
  int rows[2], nr;
  if (p->W % 2 == 0) {
    rows[0] = p->y0 + p->W / 2 - 1; rows[1] = p->y0 + p->W / 2; nr = 2;
  } else {
    rows[0] = p->y0 + (p->W - 1) / 2; nr = 1;
  }
  double z = (double)(p->x_out - p->x_in); /* no crossing: breakthrough */
  for (long x = p->x_in; x < p->x_out; x++) {
    int blocked = 0;
    double phi = 0;
    for (int r = 0; r < nr; r++) {
      long k = (long)rows[r] * p->nx + x;
      if (sim->s[k]) blocked = 1;
      else phi += sim->rho[k] / (sim->rho[k] + sim->rho[N + k]);
    }
    if (blocked) { z = (double)(x - p->x_in); break; }
    phi /= nr;
    if (x == p->x_in && phi < 0.5) { z = 0; break; }
    if (x + 1 < p->x_out) {
      int nblocked = 0;
      double phin = 0;
      for (int r = 0; r < nr; r++) {
        long k = (long)rows[r] * p->nx + x + 1;
        if (sim->s[k]) nblocked = 1;
        else phin += sim->rho[k] / (sim->rho[k] + sim->rho[N + k]);
      }
      phin /= nr;
      if (!nblocked && phi >= 0.5 && phin < 0.5) {
        z = (double)x + (phi - 0.5) / (phi - phin) - p->x_in;
        break;
      }
    }
  }
  o->front_z = z;

  double de = 0;
  int64_t closure = -1;
  for (long x = p->x_in; x < p->x_out; x++) {
    int db = 0, dt = 0;
    while (db < p->W && sim->s[(long)(p->y0 + db) * p->nx + x]) db++;
    while (dt < p->W && sim->s[(long)(p->y0 + p->W - 1 - dt) * p->nx + x]) dt++;
    double col;
    if (db >= p->W) { /* closed column */
      col = 0.5 * p->W;
      int64_t last = 0;
      for (int y = p->y0; y < p->y0 + p->W; y++) {
        int64_t st = sim->solid_step[(long)y * p->nx + x];
        if (st > last) last = st;
      }
      if (closure < 0 || last < closure) closure = last;
    } else {
      col = db > dt ? db : dt;
    }
    if (col > de) de = col;
  }
  o->delta_e = de;
  o->closure_step = closure;

  /* Radii of the capillary section (section "Results and discussion", Fig. 4),
   * all equal to the width W for the unreacted slit: with w(x) the fluid nodes
   * of column x between the walls and h(x) the solid grown on the lower wall,
   * r_min = min w, r_ave = A / L with A = sum w the open area, and the
   * hydraulic radius r_h = A / P with P the length of the lower wall's
   * profile: one lattice unit per column plus the vertical steps
   * |h(x+1) - h(x)| between neighbouring columns. */
  const long L = p->x_out - p->x_in;
  double area = 0, wmin = p->W, steps = 0;
  int hprev = 0;
  for (long x = p->x_in; x < p->x_out; x++) {
    int w = 0, h = 0;
    for (int y = p->y0; y < p->y0 + p->W; y++)
      if (!sim->s[(long)y * p->nx + x]) w++;
    while (h < p->W && sim->s[(long)(p->y0 + h) * p->nx + x]) h++;
    area += w;
    if (w < wmin) wmin = w;
    if (x > p->x_in) steps += abs(h - hprev);
    hprev = h;
  }
  o->r_min = wmin;
  o->r_ave = area / (double)L;
  o->r_h = area / ((double)L + steps);
}
