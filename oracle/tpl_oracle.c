/*
 * tpl_oracle.c -- FP64 CPU oracle for the two-fluid kinetic scheme of
 * arXiv:2201.10132 (Singh, Subramanian & Ansumali).
 *
 * TEST INFRASTRUCTURE ONLY (see tpl_oracle.h).  Written for reading, not for
 * speed: every step of one time step is a separate loop over the lattice in
 * the order the scheme states it (stream, moments, non-local terms, mixture
 * velocity, equilibria, relaxation).  OpenMP only splits lattice rows.
 *
 * Storage is node-major: XS[y][x][i], XP[y][x][q][k]; the accessors convert
 * to the canonical exchange layouts of the header.
 */
#include "tpl_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0)
#define PI 3.14159265358979323846

/* D2Q9 velocity set and weights (Sec. VI.A).  The angle formula printed for
 * the velocities is garbled; the set below is the standard one, the only one
 * consistent with the printed weights 4/9, 1/9, 1/36. */
static const int C9[9][2] = {{0, 0},  {1, 0},   {0, 1},  {-1, 0}, {0, -1},
                             {1, 1},  {-1, 1},  {-1, -1}, {1, -1}};
static const double W9[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

struct orc_sim {
  orc_config c;
  orc_derived p;
  int nx, ny, nq, nqd;
  int cp[25][4]; /* D4Q25: (v_x, v_y, Qdot_x, Qdot_y) */
  double wp[25];
  int kstar[25];
  double *Q;    /* [nqd][2] Q-disk node positions */
  double *Fh;   /* [nqd][2] spring force / kT      */
  int *nbr;     /* [25][nqd] pull source in Q or -1 */
  double *peq;  /* [nqd] normalised rest distribution */
  /* state (post-collision populations of the last step + lagged fields) */
  double *XS;   /* [ny][nx][9]        */
  double *XP;   /* [ny][nx][nqd][25]  */
  double *psi;  /* [ny][nx][nqd]  psi^n */
  double *U;    /* [ny][nx][2]    U^n   */
  double *rhoS; /* [ny][nx] recorded at the last step */
  double *rhoP; /* [ny][nx] */
  long nstep;
  /* work arrays */
  double *GS, *GP, *psi_new, *U_new;
  double *src;  /* [ny][nx][2] extra body force (NULL: none) */
};

/* ------------------------------------------------------------------------ */
/* SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom   */
/* number generators", OOPSLA 2014).                                         */
uint64_t orc_splitmix64_next(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static double uniform01(uint64_t *st) {
  return (double)(orc_splitmix64_next(st) >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Step 1: lattices.                                                        */

/* D4Q25 (Sec. VI.B, Table I): the rest vector plus every vector with
 * exactly two non-zero entries +-1 among (v_x, v_y, Qdot_x, Qdot_y).
 * Enumeration: coordinate pairs (0,1),(0,2),(0,3),(1,2),(1,3),(2,3), and for
 * each pair the sign pairs (+,+),(+,-),(-,+),(-,-).  Weights w0 = 1/3,
 * w1..24 = 1/36 (Sec. VI.B). */
static void build_d4q25(orc_sim *s) {
  static const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3},
                                  {1, 2}, {1, 3}, {2, 3}};
  static const int sg[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
  memset(s->cp, 0, sizeof s->cp);
  s->wp[0] = 1.0 / 3.0;
  int k = 1;
  for (int p = 0; p < 6; ++p)
    for (int t = 0; t < 4; ++t, ++k) {
      s->cp[k][pairs[p][0]] = sg[t][0];
      s->cp[k][pairs[p][1]] = sg[t][1];
      s->wp[k] = 1.0 / 36.0;
    }
}

/* Q-disk (Sec. VI.B, the Q-domain is a circle of radius sqrt(b) in units of
 * sigma): nodes Q_ab = (a + 1/2 - NQ/2, b + 1/2 - NQ/2), kept when
 * |Q| < R = NQ/2, enumerated row by row (b outer, a inner). */
static int disk_index(const orc_sim *s, int a, int b) {
  if (a < 0 || b < 0 || a >= s->nq || b >= s->nq) return -1;
  double qx = a + 0.5 - 0.5 * s->nq, qy = b + 0.5 - 0.5 * s->nq;
  double R = 0.5 * s->nq;
  if (qx * qx + qy * qy >= R * R) return -1;
  int idx = 0;
  for (int bb = 0; bb < s->nq; ++bb)
    for (int aa = 0; aa < s->nq; ++aa) {
      double x = aa + 0.5 - 0.5 * s->nq, y = bb + 0.5 - 0.5 * s->nq;
      if (x * x + y * y >= R * R) continue;
      if (aa == a && bb == b) return idx;
      ++idx;
    }
  return -1;
}

/* Spring force divided by kT.  Hookean: Q / sigma^2.  FENE (Warner form,
 * singular at |Q| = R = sqrt(b) sigma, Sec. VI.C):
 * Q / (sigma^2 (1 - |Q|^2 / (b sigma^2))). */
static void spring_force(const orc_sim *s, double qx, double qy, double *fx,
                         double *fy) {
  double s2 = s->p.sigma * s->p.sigma;
  double f = 1.0 / s2;
  if (s->c.spring == 0) f /= (1.0 - (qx * qx + qy * qy) / (s->c.b * s2));
  /* lattice caps: the drift D_Q |Fhat| per step may exceed neither
   * drift_cap nor drift_relax times 2 - omega_P, the rate at which the
   * relaxation damps the polymer's non-conserved moments
   * (omega_P = 2 / (2 tau1_P + 1)) */
  double cap = s->c.drift_cap > 0.0 ? s->c.drift_cap : HUGE_VAL;
  if (s->c.drift_relax > 0.0) {
    double omega = 2.0 / (2.0 * s->p.tau1P + 1.0);
    double c2 = s->c.drift_relax * (2.0 - omega);
    if (c2 < cap) cap = c2;
  }
  double mag = f * sqrt(qx * qx + qy * qy);
  if (s->p.DQ * mag > cap) f *= cap / (s->p.DQ * mag);
  *fx = f * qx;
  *fy = f * qy;
}

static void build_qdisk(orc_sim *s) {
  int nq = s->nq;
  s->nqd = 0;
  for (int b = 0; b < nq; ++b)
    for (int a = 0; a < nq; ++a)
      if (disk_index(s, a, b) >= 0) s->nqd++;
  s->Q = malloc(sizeof(double) * 2 * s->nqd);
  s->Fh = malloc(sizeof(double) * 2 * s->nqd);
  s->peq = malloc(sizeof(double) * s->nqd);
  s->nbr = malloc(sizeof(int) * 25 * s->nqd);
  int q = 0;
  int *ia = malloc(sizeof(int) * s->nqd), *ib = malloc(sizeof(int) * s->nqd);
  for (int b = 0; b < nq; ++b)
    for (int a = 0; a < nq; ++a) {
      if (disk_index(s, a, b) < 0) continue;
      s->Q[2 * q] = a + 0.5 - 0.5 * nq;
      s->Q[2 * q + 1] = b + 0.5 - 0.5 * nq;
      ia[q] = a;
      ib[q] = b;
      ++q;
    }
  /* pull source in Q for velocity k: the node at Q_q - Qdot_k */
  for (int k = 0; k < 25; ++k)
    for (q = 0; q < s->nqd; ++q)
      s->nbr[k * s->nqd + q] =
          disk_index(s, ia[q] - s->cp[k][2], ib[q] - s->cp[k][3]);
  /* k* = the velocity with the same v and reversed Qdot */
  for (int k = 0; k < 25; ++k)
    for (int j = 0; j < 25; ++j)
      if (s->cp[j][0] == s->cp[k][0] && s->cp[j][1] == s->cp[k][1] &&
          s->cp[j][2] == -s->cp[k][2] && s->cp[j][3] == -s->cp[k][3])
        s->kstar[k] = j;
  free(ia);
  free(ib);
}

/* Rest distribution over the Q-disk.  FENE: (1 - Q^2/(b sigma^2))^(b/2)
 * (Sec. VI.C initial condition, in units of sigma); Hookean: Gaussian of
 * variance sigma^2 per component.  The printed normaliser is the 3-D one,
 * so the distribution is normalised discretely to sum 1. */
static void build_peq(orc_sim *s) {
  double s2 = s->p.sigma * s->p.sigma, sum = 0.0;
  for (int q = 0; q < s->nqd; ++q) {
    double q2 = s->Q[2 * q] * s->Q[2 * q] + s->Q[2 * q + 1] * s->Q[2 * q + 1];
    double w = (s->c.spring == 0) ? pow(1.0 - q2 / (s->c.b * s2), 0.5 * s->c.b)
                                  : exp(-0.5 * q2 / s2);
    s->peq[q] = w;
    sum += w;
  }
  for (int q = 0; q < s->nqd; ++q) s->peq[q] /= sum;
}

/* ------------------------------------------------------------------------ */
/* Step 0: parameters (Sec. VII definitions of Re, Wi, beta; Sec. IV:
 * viscosity proportional to tau1; App. A: Q-diffusivity 2kT/zeta). */
static int derive(orc_sim *s, char *err) {
  const orc_config *c = &s->c;
  orc_derived *p = &s->p;
  int nyp = c->ny_param > 0 ? c->ny_param : c->ny;
  p->kf = 2.0 * PI * c->periods / nyp;
  p->l = 1.0 / p->kf;
  p->nu = c->u0 * p->l / c->Re;
  p->rhoS0 = 1.0 - c->phi;
  p->rhoP0 = c->phi;
  p->R = 0.5 * c->nq;
  p->sigma = p->R / sqrt(c->b);
  if (c->Wi > 0.0) {
    p->lambda = c->Wi * p->l / c->u0;
    p->nuS = c->beta * p->nu;
    p->G = (1.0 - c->beta) * p->nu / p->lambda; /* eta_p = G lambda, rho = 1 */
  } else { /* Newtonian limit: no elastic stress, passive polymer */
    p->lambda = p->l / c->u0;
    p->nuS = p->nu;
    p->G = 0.0;
  }
  if (c->lambda_set > 0.0) {
    p->G = p->G * p->lambda / c->lambda_set;
    p->lambda = c->lambda_set;
  }
  if (c->qe_model == 2) {
    /* stress-tensor model (Sec. V (ii)): the stresses relax with tau2, so
     * the viscosity is c_s^2 tau2; momenta and fluxes relax with tau1, so
     * tau1 sets the drag and the diffusivities */
    p->tau2S = p->nuS / CS2;
    p->tau1S = c->tau_drag > 0.0 ? c->tau_drag : p->tau2S; /* 0: automatic */
    p->tau1P = p->sigma * p->sigma / (2.0 * CS2 * p->lambda);
    p->tau2P = p->tau1P / c->tau_ratio_p;
    p->DQ = CS2 * p->tau1P;
  } else {
    p->tau1S = p->nuS / CS2; /* trapezoidal scheme: nu = c_s^2 tau1 */
    p->tau2S = c->tau_drag > 0.0 ? c->tau_drag : 1.0; /* 0: automatic */
    /* Q-diffusivity D_Q = c_s^2 tau2_P sets lambda = sigma^2 / (2 D_Q) */
    p->tau2P = p->sigma * p->sigma / (2.0 * CS2 * p->lambda);
    p->tau1P = c->tau_ratio_p * p->tau2P;
    p->DQ = CS2 * p->tau2P;
  }
  p->F0 = c->force_scale * 1.0 * p->nu * c->u0 * p->kf * p->kf;
  p->Sc = p->nuS / p->DQ;
  if (p->tau1S > p->tau2S * (1.0 + 1e-12)) {
    if (err) snprintf(err, 256, "tau1_S=%g exceeds tau2_S=%g", p->tau1S, p->tau2S);
    return -1;
  }
  if (c->qe_model != 1 && c->qe_model != 2) {
    if (err) snprintf(err, 256, "qe_model must be 1 or 2");
    return -1;
  }
  if (c->gradients != 0 && c->gradients != 1) {
    if (err) snprintf(err, 256, "gradients must be 0 or 1");
    return -1;
  }
  if (c->spring_shift != 0 && c->spring_shift != 1) {
    if (err) snprintf(err, 256, "spring_shift must be 0 or 1");
    return -1;
  }
  if (c->tau_ratio_p > 1.0 || c->tau_ratio_p <= 0.0) {
    if (err) snprintf(err, 256, "tau_ratio_p must be in (0,1]");
    return -1;
  }
  return 0;
}

/* kappa converts the Q-sum of the Taylor-expanded spring term into the
 * elastic stress divergence (Sec. III: I = div Theta).  It needs m_eq, the
 * rest value of (1/2) tr sum_q p_eq Q Fhat^T, and so the Q-disk. */
static void derive_kappa(orc_sim *s) {
  double m = 0.0;
  for (int q = 0; q < s->nqd; ++q)
    m += s->peq[q] * (s->Q[2 * q] * s->Fh[2 * q] + s->Q[2 * q + 1] * s->Fh[2 * q + 1]);
  s->p.meq = 0.5 * m;
  /* the polymer flux relaxes with tau2_P (model (i)) or tau1_P (model (ii)) */
  double tJ = s->c.qe_model == 2 ? s->p.tau1P : s->p.tau2P;
  s->p.kappa = (s->p.rhoP0 > 0.0) ? s->p.G * tJ / (s->p.rhoP0 * s->p.meq) : 0.0;
}

/* ------------------------------------------------------------------------ */
orc_sim *orc_new(const orc_config *cfg, char *err) {
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nq < 2 || cfg->Re <= 0.0 ||
      cfg->u0 <= 0.0 || cfg->beta <= 0.0 || cfg->beta > 1.0 || cfg->phi < 0.0 ||
      cfg->phi >= 1.0 || cfg->b <= 0.0 || cfg->Wi < 0.0) {
    if (err) snprintf(err, 256, "invalid configuration");
    return NULL;
  }
  orc_sim *s = calloc(1, sizeof *s);
  s->c = *cfg;
  s->nx = cfg->nx;
  s->ny = cfg->ny;
  s->nq = cfg->nq;
  if (derive(s, err) != 0) {
    free(s);
    return NULL;
  }
  build_d4q25(s);
  build_qdisk(s);
  for (int q = 0; q < s->nqd; ++q)
    spring_force(s, s->Q[2 * q], s->Q[2 * q + 1], &s->Fh[2 * q], &s->Fh[2 * q + 1]);
  build_peq(s);
  derive_kappa(s);
  size_t N = (size_t)s->nx * s->ny, nqd = s->nqd;
  s->XS = calloc(N * 9, sizeof(double));
  s->XP = calloc(N * nqd * 25, sizeof(double));
  s->psi = calloc(N * nqd, sizeof(double));
  s->U = calloc(N * 2, sizeof(double));
  s->rhoS = calloc(N, sizeof(double));
  s->rhoP = calloc(N, sizeof(double));
  s->GS = calloc(N * 9, sizeof(double));
  s->GP = calloc(N * nqd * 25, sizeof(double));
  s->psi_new = calloc(N * nqd, sizeof(double));
  s->U_new = calloc(N * 2, sizeof(double));
  if (!s->XS || !s->XP || !s->GP || !s->GS || !s->psi || !s->psi_new) {
    if (err) snprintf(err, 256, "out of host memory");
    orc_free(s);
    return NULL;
  }
  return s;
}

void orc_free(orc_sim *s) {
  if (!s) return;
  free(s->Q); free(s->Fh); free(s->nbr); free(s->peq);
  free(s->XS); free(s->XP); free(s->psi); free(s->U);
  free(s->rhoS); free(s->rhoP);
  free(s->GS); free(s->GP); free(s->psi_new); free(s->U_new);
  free(s->src);
  free(s);
}

int orc_nqd(const orc_sim *s) { return s->nqd; }

/* Extra body force per r-node, added to the Kolmogorov force in every later
 * step (the momentum source through which a learned correction acts).
 * F is [2][ny][nx] (canonical layout); NULL removes it. */
void orc_set_source(orc_sim *s, const double *F) {
  const size_t N = (size_t)s->nx * s->ny;
  if (!F) {
    free(s->src);
    s->src = NULL;
    return;
  }
  if (!s->src) s->src = malloc(sizeof(double) * 2 * N);
  for (size_t n = 0; n < N; ++n) {
    s->src[2 * n] = F[n];
    s->src[2 * n + 1] = F[N + n];
  }
}
void orc_get_derived(const orc_sim *s, orc_derived *out) { *out = s->p; }
long orc_step_count(const orc_sim *s) { return s->nstep; }

void orc_get_tables(const orc_sim *s, int *cS, double *wS, int *cP,
                    double *wP, double *Q, double *Fhat, int *nbrQ,
                    int *kstar, double *peq) {
  if (cS) memcpy(cS, C9, sizeof C9);
  if (wS) memcpy(wS, W9, sizeof W9);
  if (cP) memcpy(cP, s->cp, sizeof s->cp);
  if (wP) memcpy(wP, s->wp, sizeof s->wp);
  if (Q) memcpy(Q, s->Q, sizeof(double) * 2 * s->nqd);
  if (Fhat) memcpy(Fhat, s->Fh, sizeof(double) * 2 * s->nqd);
  if (nbrQ) memcpy(nbrQ, s->nbr, sizeof(int) * 25 * s->nqd);
  if (kstar) memcpy(kstar, s->kstar, sizeof s->kstar);
  if (peq) memcpy(peq, s->peq, sizeof(double) * s->nqd);
}

/* ------------------------------------------------------------------------ */
/* Step 6: equilibria.                                                      */

/* Quadratic D2Q9 equilibrium about velocity u (Sec. VI.A): used both for
 * the solvent quasi-equilibrium (about u_S) and the equilibrium (about the
 * mixture velocity). */
void orc_solvent_eq(double rho, double ux, double uy, double *out) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double cu = C9[i][0] * ux + C9[i][1] * uy;
    out[i] = W9[i] * rho * (1.0 + cu / CS2 + 0.5 * cu * cu / (CS2 * CS2) -
                            0.5 * uu / CS2);
  }
}

/* Linear D4Q25 equilibrium (Sec. VI.B): w_k [psi + v_k.Jr/c_s^2 +
 * Qdot_k.JQ/c_s^2]; the quasi-equilibrium of the component-momentum model
 * has the same form with the populations' own fluxes. */
void orc_polymer_eq(const orc_sim *s, double psi, const double Jr[2],
                    const double JQ[2], double *out) {
  for (int k = 0; k < 25; ++k)
    out[k] = s->wp[k] * (psi + (s->cp[k][0] * Jr[0] + s->cp[k][1] * Jr[1] +
                                s->cp[k][2] * JQ[0] + s->cp[k][3] * JQ[1]) / CS2);
}

/* Second-order Hermite forms (model (ii)): w [rho + J.c/c_s^2 +
 * (P - rho c_s^2 I):(c c - c_s^2 I) / (2 c_s^4)].  The printed lattice forms
 * omit the 1/(2 c_s^4) normalisation; with it the populations carry exactly
 * the prescribed second moments (both lattices are isotropic to fourth
 * order). */
void orc_solvent_qe2(double rho, const double J[2], const double P[3], double *out) {
  double D[2][2] = {{P[0] - rho * CS2, P[1]}, {P[1], P[2] - rho * CS2}};
  for (int i = 0; i < 9; ++i) {
    double c[2] = {C9[i][0], C9[i][1]};
    double h = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) h += D[a][b] * (c[a] * c[b] - (a == b ? CS2 : 0.0));
    out[i] = W9[i] * (rho + (c[0] * J[0] + c[1] * J[1]) / CS2 + h / (2.0 * CS2 * CS2));
  }
}

void orc_polymer_qe2(const orc_sim *s, double psi, const double J[4], const double P[10],
                     double *out) {
  double D[4][4];
  int n = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) {
      D[a][b] = D[b][a] = P[n++] - (a == b ? psi * CS2 : 0.0);
    }
  for (int k = 0; k < 25; ++k) {
    double lin = 0.0, h = 0.0;
    for (int a = 0; a < 4; ++a) {
      lin += s->cp[k][a] * J[a];
      for (int b = 0; b < 4; ++b)
        h += D[a][b] * (s->cp[k][a] * s->cp[k][b] - (a == b ? CS2 : 0.0));
    }
    out[k] = s->wp[k] * (psi + lin / CS2 + h / (2.0 * CS2 * CS2));
  }
}

/* ------------------------------------------------------------------------ */
/* The g-moments the mixture velocity needs (densities, momenta, solvent
 * second moments, the Q-sum S of the spring terms) and the mixture velocity
 * itself (see orc_collide_node). */
static void mixture(const orc_sim *s, const double *gS, const double *gP, const double *sq,
                    const double Fb[2], double *rhoS_out, double JSg[2], double PSg[3],
                    double *rhoP_out, double JPg[2], double U[2]) {
  const orc_derived *p = &s->p;
  const int nqd = s->nqd;
  const int m2 = s->c.qe_model == 2;
  const double tJS = m2 ? p->tau1S : p->tau2S, tJP = m2 ? p->tau1P : p->tau2P;
  /* solvent moments of g */
  double rhoS = 0;
  JSg[0] = JSg[1] = 0;
  PSg[0] = PSg[1] = PSg[2] = 0;
  for (int i = 0; i < 9; ++i) {
    rhoS += gS[i];
    JSg[0] += C9[i][0] * gS[i];
    JSg[1] += C9[i][1] * gS[i];
    PSg[0] += C9[i][0] * C9[i][0] * gS[i];
    PSg[1] += C9[i][0] * C9[i][1] * gS[i];
    PSg[2] += C9[i][1] * C9[i][1] * gS[i];
  }
  /* polymer moments of g at every Q-node and their Q-sums */
  double rhoP = 0, S[2] = {0, 0};
  JPg[0] = JPg[1] = 0;
  for (int q = 0; q < nqd; ++q) {
    const double *g = gP + 25 * q;
    for (int k = 0; k < 25; ++k) {
      rhoP += g[k];
      JPg[0] += s->cp[k][0] * g[k];
      JPg[1] += s->cp[k][1] * g[k];
    }
    S[0] += sq[2 * q];
    S[1] += sq[2 * q + 1];
  }
  /* mixture velocity */
  double aS = 1.0 / (2.0 * tJS + 1.0), aP = 1.0 / (2.0 * tJP + 1.0);
  double den = rhoS * aS + rhoP * aP;
  for (int a = 0; a < 2; ++a)
    U[a] = ((JSg[a] + 0.5 * Fb[a]) * aS + (JPg[a] + S[a] / (2.0 * tJP)) * aP) / den;
  *rhoS_out = rhoS;
  *rhoP_out = rhoP;
}

/* Steps 4-7 at one r-node.
 *
 * Two quasi-equilibrium models (Sec. V):
 *  (i)  component momenta quasi-conserved: f* carries each species' own
 *       momentum (solvent) or fluxes (polymer); momenta relax to the mixture
 *       with tau2, everything else with tau1;
 *  (ii) component stresses quasi-conserved: f* carries each species' own
 *       second moments and the mixture-velocity momentum (solvent) or the
 *       imposed fluxes (polymer); momenta relax with tau1, stresses with tau2.
 * Write tJ for the momentum relaxation time (tau2 in (i), tau1 in (ii)).
 *
 * Moment inversion (Sec. VI.C, g = f - Omega/2): rho(f) = rho(g);
 *   J(f) = (2 tJ J(g) + J_target) / (2 tJ + 1);
 *   model (ii) also P(f) = (2 tau2 P(g) + P_eq) / (2 tau2 + 1).
 * Mixture velocity: the velocity for which the cross-collision momentum
 * exchange of the two species cancels (Sec. IV/V), expressed in g-moments;
 * with equal tJ it is U(g) + (body force)/2rho + S/(2 tJ rho), the form of
 * Sec. VI.C.  Relaxation (Sec. VI.C, trapezoidal rule made explicit):
 *   g' = (1 - 2 beta) g + 2 beta [(1 - tau1/tau2) f* + (tau1/tau2) f_eq],
 *   beta = 1 / (2 tau1 + 1).
 */
void orc_collide_node(const orc_sim *s, const double *gS, const double *gP,
                      const double K[4], const double *sq, const double Fb[2],
                      double *outS, double *outP, double U[2]) {
  const orc_derived *p = &s->p;
  const int nqd = s->nqd;
  const int m2 = s->c.qe_model == 2;
  const double tJS = m2 ? p->tau1S : p->tau2S, tJP = m2 ? p->tau1P : p->tau2P;
  double rhoS, JSg[2], PSg[3], rhoP, JPg[2];
  mixture(s, gS, gP, sq, Fb, &rhoS, JSg, PSg, &rhoP, JPg, U);
  const double aS = 1.0 / (2.0 * tJS + 1.0), aP = 1.0 / (2.0 * tJP + 1.0);

  /* solvent: target momentum rho_S U + tJ_S F (the body force by a shift of
   * the equilibrium velocity) */
  double fstar[9], feq[9];
  const double vS[2] = {U[0] + tJS * Fb[0] / rhoS, U[1] + tJS * Fb[1] / rhoS};
  orc_solvent_eq(rhoS, vS[0], vS[1], feq);
  if (!m2) {
    double JSf[2];
    for (int a = 0; a < 2; ++a)
      JSf[a] = (2.0 * tJS * JSg[a] + rhoS * U[a] + tJS * Fb[a]) * aS;
    orc_solvent_eq(rhoS, JSf[0] / rhoS, JSf[1] / rhoS, fstar);
  } else {
    /* own stress, inverted against the equilibrium's rho_S (c_s^2 I + v v) */
    const double Peq[3] = {rhoS * (CS2 + vS[0] * vS[0]), rhoS * vS[0] * vS[1],
                           rhoS * (CS2 + vS[1] * vS[1])};
    double PSf[3], JS[2] = {rhoS * vS[0], rhoS * vS[1]};
    for (int c = 0; c < 3; ++c)
      PSf[c] = (2.0 * p->tau2S * PSg[c] + Peq[c]) / (2.0 * p->tau2S + 1.0);
    orc_solvent_qe2(rhoS, JS, PSf, fstar);
  }
  double bS = 1.0 / (2.0 * p->tau1S + 1.0), rS = p->tau1S / p->tau2S;
  for (int i = 0; i < 9; ++i)
    outS[i] = (1.0 - 2.0 * bS) * gS[i] +
              2.0 * bS * ((1.0 - rS) * fstar[i] + rS * feq[i]);

  /* polymer, Q-node by Q-node */
  double bP = 1.0 / (2.0 * p->tau1P + 1.0), rP = p->tau1P / p->tau2P;
  for (int q = 0; q < nqd; ++q) {
    const double *g = gP + 25 * q;
    double psi = 0, Jrg[2] = {0, 0}, JQg[2] = {0, 0}, Pg[10] = {0};
    for (int k = 0; k < 25; ++k) {
      psi += g[k];
      Jrg[0] += s->cp[k][0] * g[k];
      Jrg[1] += s->cp[k][1] * g[k];
      JQg[0] += s->cp[k][2] * g[k];
      JQg[1] += s->cp[k][3] * g[k];
      if (m2) {
        int n = 0;
        for (int a = 0; a < 4; ++a)
          for (int b2 = a; b2 < 4; ++b2) Pg[n++] += s->cp[k][a] * s->cp[k][b2] * g[k];
      }
    }
    const double Qx = s->Q[2 * q], Qy = s->Q[2 * q + 1];
    /* imposed fluxes (Sec. V): J^r_eq = psi U + spring term,
     * J^Q_eq = psi (grad U) . Q - psi 2F/zeta, 2F/zeta = D_Q Fhat */
    double Jreq[2] = {psi * U[0] + sq[2 * q], psi * U[1] + sq[2 * q + 1]};
    double JQeq[2] = {psi * (K[0] * Qx + K[1] * Qy - p->DQ * s->Fh[2 * q]),
                      psi * (K[2] * Qx + K[3] * Qy - p->DQ * s->Fh[2 * q + 1])};
    double fs[25], fe[25];
    orc_polymer_eq(s, psi, Jreq, JQeq, fe);
    if (!m2) {
      double Jrf[2], JQf[2];
      for (int a = 0; a < 2; ++a) {
        Jrf[a] = (2.0 * tJP * Jrg[a] + Jreq[a]) * aP;
        JQf[a] = (2.0 * tJP * JQg[a] + JQeq[a]) * aP;
      }
      orc_polymer_eq(s, psi, Jrf, JQf, fs);
    } else {
      /* own stresses, inverted against the linear equilibrium's psi c_s^2 I */
      double Pf[10], Jeq[4] = {Jreq[0], Jreq[1], JQeq[0], JQeq[1]};
      int n = 0;
      for (int a = 0; a < 4; ++a)
        for (int b2 = a; b2 < 4; ++b2, ++n)
          Pf[n] = (2.0 * p->tau2P * Pg[n] + (a == b2 ? psi * CS2 : 0.0)) /
                  (2.0 * p->tau2P + 1.0);
      orc_polymer_qe2(s, psi, Jeq, Pf, fs);
    }
    double *o = outP + 25 * q;
    for (int k = 0; k < 25; ++k)
      o[k] = (1.0 - 2.0 * bP) * g[k] + 2.0 * bP * ((1.0 - rP) * fs[k] + rP * fe[k]);
  }
}

/* ------------------------------------------------------------------------ */
static inline size_t nid(const orc_sim *s, int x, int y) {
  return (size_t)y * s->nx + x;
}
static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Step 3: pull streaming.  Solvent: periodic D2Q9 shift.  Polymer: shift by
 * v_k in r and by Qdot_k in Q; a population whose Q-source lies outside the
 * disk is replaced by the reversed-Qdot population of the same node
 * (bounce-back on the Q-circle, Sec. VI.C), which keeps v and so r-momentum. */
static void stream(orc_sim *s) {
  const int nx = s->nx, ny = s->ny, nqd = s->nqd;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t n = nid(s, x, y);
      for (int i = 0; i < 9; ++i) {
        size_t m = nid(s, wrap(x - C9[i][0], nx), wrap(y - C9[i][1], ny));
        s->GS[9 * n + i] = s->XS[9 * m + i];
      }
      for (int k = 0; k < 25; ++k) {
        size_t m = nid(s, wrap(x - s->cp[k][0], nx), wrap(y - s->cp[k][1], ny));
        for (int q = 0; q < nqd; ++q) {
          int src = s->nbr[k * nqd + q];
          double v = (src >= 0) ? s->XP[(m * nqd + src) * 25 + k]
                                : s->XP[(m * nqd + q) * 25 + s->kstar[k]];
          s->GP[(n * nqd + q) * 25 + k] = v;
        }
      }
    }
}

/* Central difference with periodic wrap. */
static double ddx(const orc_sim *s, const double *f, int stride, int comp,
                  int x, int y) {
  return 0.5 * (f[nid(s, wrap(x + 1, s->nx), y) * stride + comp] -
                f[nid(s, wrap(x - 1, s->nx), y) * stride + comp]);
}
static double ddy(const orc_sim *s, const double *f, int stride, int comp,
                  int x, int y) {
  return 0.5 * (f[nid(s, x, wrap(y + 1, s->ny)) * stride + comp] -
                f[nid(s, x, wrap(y - 1, s->ny)) * stride + comp]);
}

static double body_force_x(const orc_sim *s, int y) {
  return s->p.F0 * sin(s->p.kf * (double)(y + s->c.y_offset));
}

/* Spring terms of J^r_eq at node (x, y) from the recorded psi, the lattice
 * form of sum_nu (F_nu/zeta) psi(r - R_nu, Q) (Sec. III/V) with the beads at
 * R = -+Q/2 and F_1 = -F_2 = F: s = kappa Fhat(Q) [psi(r + Q/2) - psi(r - Q/2)],
 * or its first-order Taylor expansion kappa Fhat(Q) [Q . grad psi(r, Q)]. */
/* psi(X, Y, q) at a real position by bilinear interpolation between the four
 * surrounding nodes, periodic in both directions.  The weights sum to one and
 * do not depend on the node, so the lattice sum of the interpolated field
 * equals that of psi (sum-preserving). */
static double psi_at(const orc_sim *s, double X, double Y, int q) {
  const double fx0 = floor(X), fy0 = floor(Y);
  const double fx = X - fx0, fy = Y - fy0;
  const int x0 = wrap((int)fx0, s->nx), x1 = wrap((int)fx0 + 1, s->nx);
  const int y0 = wrap((int)fy0, s->ny), y1 = wrap((int)fy0 + 1, s->ny);
  const int nqd = s->nqd;
  return (1.0 - fx) * (1.0 - fy) * s->psi[nid(s, x0, y0) * nqd + q] +
         fx * (1.0 - fy) * s->psi[nid(s, x1, y0) * nqd + q] +
         (1.0 - fx) * fy * s->psi[nid(s, x0, y1) * nqd + q] +
         fx * fy * s->psi[nid(s, x1, y1) * nqd + q];
}

static void spring_terms(const orc_sim *s, int x, int y, double *sq) {
  const int nqd = s->nqd;
  for (int q = 0; q < nqd; ++q) {
    const double Qx = s->Q[2 * q], Qy = s->Q[2 * q + 1];
    double qg;
    if (s->c.spring_shift) {
      /* the two beads at r -+ Q/2 (Sec. V): psi(r + Q/2) - psi(r - Q/2) */
      qg = psi_at(s, x + 0.5 * Qx, y + 0.5 * Qy, q) - psi_at(s, x - 0.5 * Qx, y - 0.5 * Qy, q);
    } else {
      double gx = ddx(s, s->psi, nqd, q, x, y);
      double gy = ddy(s, s->psi, nqd, q, x, y);
      qg = Qx * gx + Qy * gy;
    }
    sq[2 * q] = s->p.kappa * s->Fh[2 * q] * qg;
    sq[2 * q + 1] = s->p.kappa * s->Fh[2 * q + 1] * qg;
  }
}

void orc_spring_terms(const orc_sim *s, int x, int y, double *sq) { spring_terms(s, x, y, sq); }

static void body_force(const orc_sim *s, int y, size_t n, double Fb[2]) {
  Fb[0] = body_force_x(s, y);
  Fb[1] = 0.0;
  if (s->src) {
    Fb[0] += s->src[2 * n];
    Fb[1] += s->src[2 * n + 1];
  }
}

/* Same-step gradients (the reading that takes the gradients at the current
 * time level): replace the recorded psi and U by those of the pulled
 * populations of this step, psi^n(r, Q) = sum_k g_k and U^n the mixture
 * velocity with the spring terms of grad psi^n, before any node collides. */
static void current_observables(orc_sim *s) {
  const int nx = s->nx, ny = s->ny, nqd = s->nqd;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t n = nid(s, x, y);
      for (int q = 0; q < nqd; ++q) {
        double ps = 0;
        for (int k = 0; k < 25; ++k) ps += s->GP[(n * nqd + q) * 25 + k];
        s->psi[n * nqd + q] = ps;
      }
    }
#pragma omp parallel
  {
    double *sq = malloc(sizeof(double) * 2 * nqd);
#pragma omp for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t n = nid(s, x, y);
        double Fb[2], rhoS, JSg[2], PSg[3], rhoP, JPg[2];
        spring_terms(s, x, y, sq);
        body_force(s, y, n, Fb);
        mixture(s, s->GS + 9 * n, s->GP + n * nqd * 25, sq, Fb, &rhoS, JSg, PSg, &rhoP, JPg,
                s->U + 2 * n);
      }
    free(sq);
  }
}

/* One time step: stream; then, per r-node, the non-local terms (from the
 * recorded observables: the previous step's, or with same-step gradients
 * this step's) and the collision; then record the observables. */
static void step_once(orc_sim *s) {
  stream(s);
  if (s->c.gradients == 1) current_observables(s);
  const int nx = s->nx, ny = s->ny, nqd = s->nqd;
#pragma omp parallel
  {
    double *sq = malloc(sizeof(double) * 2 * nqd);
#pragma omp for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t n = nid(s, x, y);
        /* velocity gradient K_ab = d_b U_a of the recorded U */
        double K[4] = {ddx(s, s->U, 2, 0, x, y), ddy(s, s->U, 2, 0, x, y),
                       ddx(s, s->U, 2, 1, x, y), ddy(s, s->U, 2, 1, x, y)};
        spring_terms(s, x, y, sq);
        double Fb[2];
        body_force(s, y, n, Fb);
        double Un[2];
        orc_collide_node(s, s->GS + 9 * n, s->GP + n * nqd * 25, K, sq, Fb,
                         s->XS + 9 * n, s->XP + n * nqd * 25, Un);
        /* observables recorded from the pulled populations */
        double rs = 0, rp = 0;
        for (int i = 0; i < 9; ++i) rs += s->GS[9 * n + i];
        for (int q = 0; q < nqd; ++q) {
          double ps = 0;
          for (int k = 0; k < 25; ++k) ps += s->GP[(n * nqd + q) * 25 + k];
          s->psi_new[n * nqd + q] = ps;
          rp += ps;
        }
        s->rhoS[n] = rs;
        s->rhoP[n] = rp;
        s->U_new[2 * n] = Un[0];
        s->U_new[2 * n + 1] = Un[1];
      }
    free(sq);
  }
  double *t = s->psi; s->psi = s->psi_new; s->psi_new = t;
  t = s->U; s->U = s->U_new; s->U_new = t;
  s->nstep++;
}

void orc_step(orc_sim *s, long n) {
  for (long i = 0; i < n; ++i) step_once(s);
}

/* ------------------------------------------------------------------------ */
/* Step 8: initial state.                                                   */

static void record_densities(orc_sim *s) {
  size_t N = (size_t)s->nx * s->ny;
  for (size_t n = 0; n < N; ++n) {
    double rs = 0, rp = 0;
    for (int i = 0; i < 9; ++i) rs += s->XS[9 * n + i];
    for (int q = 0; q < s->nqd; ++q)
      for (int k = 0; k < 25; ++k) rp += s->XP[(n * s->nqd + q) * 25 + k];
    s->rhoS[n] = rs;
    s->rhoP[n] = rp;
  }
}

/* Rest: solvent at its equilibrium with zero velocity, polymer at the
 * discrete rest distribution carrying mass rho_P (psi sums to rho_P). */
void orc_rest(orc_sim *s) {
  size_t N = (size_t)s->nx * s->ny;
  double feq[9];
  orc_solvent_eq(s->p.rhoS0, 0.0, 0.0, feq);
  for (size_t n = 0; n < N; ++n) {
    for (int i = 0; i < 9; ++i) s->XS[9 * n + i] = feq[i];
    for (int q = 0; q < s->nqd; ++q) {
      double psi = s->p.rhoP0 * s->peq[q];
      s->psi[n * s->nqd + q] = psi;
      for (int k = 0; k < 25; ++k)
        s->XP[(n * s->nqd + q) * 25 + k] = s->wp[k] * psi;
    }
    s->U[2 * n] = s->U[2 * n + 1] = 0.0;
  }
  record_densities(s);
  s->nstep = 0;
}

/* Analytic initial state (Hookean springs, component-momentum model, Wi > 0):
 * the forced laminar Kolmogorov state of Hookean dumbbells, the Oldroyd-B
 * profile with the stress diffusion of the polymer populations, on every
 * column (Sec. VII forcing; Sec. V imposed fluxes; App. A Smoluchowski limit).
 *   U_x = U_L sin(k y), U_L = F0 / (k^2 [eta_s + eta_pk + G lambda / (1 + lambda D k^2)])
 *   with eta_s = rho_S c_s^2 tau1_S, eta_pk = rho_P c_s^2 tau1_P, D = c_s^2 tau2_P;
 *   conformation c_xy = lambda U_L k cos(k y) / (1 + lambda D k^2),
 *   c_xx = 1 + lambda^2 U_L^2 k^2 / (1 + lambda D k^2) [1 + cos(2 k y) / (1 + 4 lambda D k^2)],
 *   c_yy = 1;
 *   psi(y, Q) proportional to exp(-Q^T (sigma^2 c)^-1 Q / 2) over the disk,
 *   summing to rho_P;
 * the solvent at its equilibrium about U, the polymer at its equilibrium
 * with the imposed fluxes J^r = psi U and J^Q = psi (K Q - D_Q Fhat),
 * K_xy = dU_x/dy.  Returns -1 (state unchanged) for other configurations. */
int orc_analytic_state(orc_sim *s) {
  if (s->c.spring != 1 || s->c.qe_model != 1 || !(s->p.G > 0.0)) return -1;
  const int nqd = s->nqd;
  const double k = s->p.kf, lam = s->p.lambda, G = s->p.G;
  const double D = CS2 * s->p.tau2P;
  const double etas = s->p.rhoS0 * CS2 * s->p.tau1S, etap = s->p.rhoP0 * CS2 * s->p.tau1P;
  const double a = 1.0 + lam * D * k * k;
  const double UL = s->p.F0 / (k * k * (etas + etap + G * lam / a));
  const double s2 = s->p.sigma * s->p.sigma;
  double *w = malloc(sizeof(double) * (size_t)nqd);
  for (int y = 0; y < s->ny; ++y) {
    const double Y = (double)(y + s->c.y_offset);
    const double ux = UL * sin(k * Y), Kxy = UL * k * cos(k * Y);
    const double cxy = lam * UL * k * cos(k * Y) / a;
    const double cxx = 1.0 + lam * lam * UL * UL * k * k / a *
                                 (1.0 + cos(2.0 * k * Y) / (1.0 + 4.0 * lam * D * k * k));
    const double cyy = 1.0;
    /* inverse of sigma^2 c */
    const double det = s2 * s2 * (cxx * cyy - cxy * cxy);
    const double ixx = s2 * cyy / det, ixy = -s2 * cxy / det, iyy = s2 * cxx / det;
    double tot = 0.0;
    for (int q = 0; q < nqd; ++q) {
      const double qx = s->Q[2 * q], qy = s->Q[2 * q + 1];
      w[q] = exp(-0.5 * (ixx * qx * qx + 2.0 * ixy * qx * qy + iyy * qy * qy));
      tot += w[q];
    }
    double feq[9];
    orc_solvent_eq(s->p.rhoS0, ux, 0.0, feq);
    for (int x = 0; x < s->nx; ++x) {
      const size_t n = nid(s, x, y);
      for (int i = 0; i < 9; ++i) s->XS[9 * n + i] = feq[i];
      for (int q = 0; q < nqd; ++q) {
        const double psi = s->p.rhoP0 * w[q] / tot;
        const double qy = s->Q[2 * q + 1];
        const double Jr[2] = {psi * ux, 0.0};
        const double JQ[2] = {psi * (Kxy * qy - s->p.DQ * s->Fh[2 * q]),
                              psi * (-s->p.DQ * s->Fh[2 * q + 1])};
        orc_polymer_eq(s, psi, Jr, JQ, s->XP + (n * nqd + q) * 25);
        s->psi[n * nqd + q] = psi;
      }
      s->U[2 * n] = ux;
      s->U[2 * n + 1] = 0.0;
    }
  }
  free(w);
  record_densities(s);
  s->nstep = 0;
  return 0;
}

long orc_default_prerun(const orc_sim *s) {
  double t = s->p.l * s->p.l / s->p.nu;
  if (s->p.lambda > t) t = s->p.lambda;
  return (long)ceil(5.0 * t);
}

/* Base state: the forced laminar state of an x-invariant column, reached by
 * running the scheme itself on nx = 1, then copied to every column. */
void orc_base_state(orc_sim *s, long npre) {
  if (npre < 0) npre = orc_default_prerun(s);
  orc_config cc = s->c;
  cc.nx = 1;
  if (cc.ny_param <= 0) cc.ny_param = s->ny;
  orc_sim *col = orc_new(&cc, NULL);
  orc_rest(col);
  orc_step(col, npre);
  const int nx = s->nx, ny = s->ny, nqd = s->nqd;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t n = nid(s, x, y), m = (size_t)y;
      memcpy(s->XS + 9 * n, col->XS + 9 * m, 9 * sizeof(double));
      memcpy(s->XP + n * nqd * 25, col->XP + m * nqd * 25, nqd * 25 * sizeof(double));
      memcpy(s->psi + n * nqd, col->psi + m * nqd, nqd * sizeof(double));
      s->U[2 * n] = col->U[2 * m];
      s->U[2 * n + 1] = col->U[2 * m + 1];
      s->rhoS[n] = col->rhoS[m];
      s->rhoP[n] = col->rhoP[m];
    }
  orc_free(col);
  s->nstep = 0;
}

/* Perturbation: a divergence-free velocity du added to both species'
 * populations at first order (3 w c.du times the local density) and to the
 * lagged velocity.  Single mode: du_y = amp u0 sin(2 pi x / nx + phi0).
 * Multimode: du = curl of sum_m a_m cos(2 pi (kx x/nx + ky y/ny) + phi_m)
 * over 1 <= |kx| <= 8, |ky| <= 8 (kx outer, ky inner), a_m ~ N(0,1) by
 * Box-Muller from two uniforms, phi_m uniform in [0, 2 pi), then rescaled to
 * RMS amp u0.  All uniforms come from one SplitMix64 stream seeded by seed. */
void orc_perturb(orc_sim *s, uint64_t seed, double amp, int multimode) {
  const int nx = s->nx, ny = s->ny, nqd = s->nqd;
  const int NX = s->c.nx_param > 0 ? s->c.nx_param : nx;
  const int NY = s->c.ny_param > 0 ? s->c.ny_param : ny;
  size_t N = (size_t)nx * ny;
  double *du = calloc(2 * N, sizeof(double));
  uint64_t st = seed;
  if (!multimode) {
    double phi0 = 2.0 * PI * uniform01(&st);
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        du[2 * nid(s, x, y) + 1] =
            amp * s->c.u0 * sin(2.0 * PI * (x + s->c.x_offset) / NX + phi0);
  } else {
    double a[17 * 17], ph[17 * 17];
    int kxs[17 * 17], kys[17 * 17], nm = 0;
    for (int kx = -8; kx <= 8; ++kx) {
      if (kx == 0) continue;
      for (int ky = -8; ky <= 8; ++ky) {
        double u1 = uniform01(&st), u2 = uniform01(&st), u3 = uniform01(&st);
        a[nm] = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * PI * u2);
        ph[nm] = 2.0 * PI * u3;
        kxs[nm] = kx;
        kys[nm] = ky;
        ++nm;
      }
    }
    double ss = 0.0;
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        double ux = 0, uy = 0;
        double X = x + s->c.x_offset, Y = y + s->c.y_offset;
        for (int m = 0; m < nm; ++m) {
          double th = 2.0 * PI * (kxs[m] * X / NX + kys[m] * Y / NY) + ph[m];
          /* du = (d psi/dy, -d psi/dx) of psi = a cos(th) */
          ux += -a[m] * sin(th) * (2.0 * PI * kys[m] / NY);
          uy += a[m] * sin(th) * (2.0 * PI * kxs[m] / NX);
        }
        du[2 * nid(s, x, y)] = ux;
        du[2 * nid(s, x, y) + 1] = uy;
        ss += ux * ux + uy * uy;
      }
    double rms = sqrt(ss / (double)N);
    double f = (rms > 0.0) ? amp * s->c.u0 / rms : 0.0;
    for (size_t i = 0; i < 2 * N; ++i) du[i] *= f;
  }
  for (size_t n = 0; n < N; ++n) {
    double dx = du[2 * n], dy = du[2 * n + 1];
    double rs = 0;
    for (int i = 0; i < 9; ++i) rs += s->XS[9 * n + i];
    for (int i = 0; i < 9; ++i)
      s->XS[9 * n + i] += 3.0 * W9[i] * rs * (C9[i][0] * dx + C9[i][1] * dy);
    for (int q = 0; q < nqd; ++q) {
      double *X = s->XP + (n * nqd + q) * 25;
      double ps = 0;
      for (int k = 0; k < 25; ++k) ps += X[k];
      for (int k = 0; k < 25; ++k)
        X[k] += 3.0 * s->wp[k] * ps * (s->cp[k][0] * dx + s->cp[k][1] * dy);
    }
    s->U[2 * n] += dx;
    s->U[2 * n + 1] += dy;
  }
  free(du);
}

/* ------------------------------------------------------------------------ */
void orc_get_state(const orc_sim *s, double *XS, double *XP, double *psi,
                   double *U) {
  const int nqd = s->nqd;
  size_t N = (size_t)s->nx * s->ny;
  for (size_t n = 0; n < N; ++n) {
    if (XS)
      for (int i = 0; i < 9; ++i) XS[i * N + n] = s->XS[9 * n + i];
    if (XP)
      for (int k = 0; k < 25; ++k)
        for (int q = 0; q < nqd; ++q)
          XP[((size_t)k * nqd + q) * N + n] = s->XP[(n * nqd + q) * 25 + k];
    if (psi)
      for (int q = 0; q < nqd; ++q) psi[(size_t)q * N + n] = s->psi[n * nqd + q];
    if (U) {
      U[n] = s->U[2 * n];
      U[N + n] = s->U[2 * n + 1];
    }
  }
}

void orc_set_state(orc_sim *s, const double *XS, const double *XP,
                   const double *psi, const double *U) {
  const int nqd = s->nqd;
  size_t N = (size_t)s->nx * s->ny;
  for (size_t n = 0; n < N; ++n) {
    if (XS)
      for (int i = 0; i < 9; ++i) s->XS[9 * n + i] = XS[i * N + n];
    if (XP)
      for (int k = 0; k < 25; ++k)
        for (int q = 0; q < nqd; ++q)
          s->XP[(n * nqd + q) * 25 + k] = XP[((size_t)k * nqd + q) * N + n];
    if (psi)
      for (int q = 0; q < nqd; ++q) s->psi[n * nqd + q] = psi[(size_t)q * N + n];
    if (U) {
      s->U[2 * n] = U[n];
      s->U[2 * n + 1] = U[N + n];
    }
  }
  record_densities(s);
}

/* ------------------------------------------------------------------------ */
/* Step 9: observables and diagnostics (Sec. VII: vorticity, enstrophy,
 * RMS extension). */

void orc_observables(const orc_sim *s, double *out) {
  const int nqd = s->nqd;
  size_t N = (size_t)s->nx * s->ny;
  const double s2 = s->p.sigma * s->p.sigma;
  for (size_t n = 0; n < N; ++n) {
    double ps = 0, C[3] = {0, 0, 0}, M[3] = {0, 0, 0};
    for (int q = 0; q < nqd; ++q) {
      double v = s->psi[n * nqd + q], Qx = s->Q[2 * q], Qy = s->Q[2 * q + 1];
      ps += v;
      C[0] += v * Qx * Qx;
      C[1] += v * Qx * Qy;
      C[2] += v * Qy * Qy;
      M[0] += v * Qx * s->Fh[2 * q];
      M[1] += v * Qx * s->Fh[2 * q + 1];
      M[2] += v * Qy * s->Fh[2 * q + 1];
    }
    out[0 * N + n] = s->rhoS[n] + s->rhoP[n];
    out[1 * N + n] = s->U[2 * n];
    out[2 * N + n] = s->U[2 * n + 1];
    out[3 * N + n] = s->rhoP[n];
    for (int c = 0; c < 3; ++c) out[(4 + c) * N + n] = (ps > 0) ? C[c] / (s2 * ps) : 0.0;
    double mref = s->p.rhoP0 * s->p.meq;
    for (int c = 0; c < 3; ++c) {
      double iso = (c == 1) ? 0.0 : 1.0;
      out[(7 + c) * N + n] = (mref > 0) ? s->p.G * (M[c] / mref - iso) : 0.0;
    }
  }
}

/* A(n): RMS over the lattice of the velocity deviation from its x-average at
 * each row, divided by u0. */
double orc_amplitude(const orc_sim *s) {
  const int nx = s->nx, ny = s->ny;
  double acc = 0.0;
  for (int y = 0; y < ny; ++y) {
    double mx = 0, my = 0;
    for (int x = 0; x < nx; ++x) {
      mx += s->U[2 * nid(s, x, y)];
      my += s->U[2 * nid(s, x, y) + 1];
    }
    mx /= nx;
    my /= nx;
    for (int x = 0; x < nx; ++x) {
      double dx = s->U[2 * nid(s, x, y)] - mx, dy = s->U[2 * nid(s, x, y) + 1] - my;
      acc += dx * dx + dy * dy;
    }
  }
  return sqrt(acc / ((double)nx * ny)) / s->c.u0;
}

/* Neumaier's compensated summation, so that the conservation checks see
 * the scheme's round-off rather than that of the diagnostic sum itself. */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

void orc_diagnostics(const orc_sim *s, double *out) {
  const int nx = s->nx, ny = s->ny, nqd = s->nqd;
  nsum mS = {0, 0}, mP = {0, 0}, px = {0, 0}, py = {0, 0};
  double ens = 0, pq2 = 0, pw = 0, minpsi = 1e300;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t n = nid(s, x, y);
      for (int i = 0; i < 9; ++i) {
        nadd(&mS, s->XS[9 * n + i]);
        nadd(&px, C9[i][0] * s->XS[9 * n + i]);
        nadd(&py, C9[i][1] * s->XS[9 * n + i]);
      }
      for (int q = 0; q < nqd; ++q) {
        const double *X = s->XP + (n * nqd + q) * 25;
        for (int k = 0; k < 25; ++k) {
          nadd(&mP, X[k]);
          if (s->cp[k][0]) nadd(&px, s->cp[k][0] * X[k]);
          if (s->cp[k][1]) nadd(&py, s->cp[k][1] * X[k]);
        }
        double v = s->psi[n * nqd + q];
        double q2 = s->Q[2 * q] * s->Q[2 * q] + s->Q[2 * q + 1] * s->Q[2 * q + 1];
        pq2 += v * q2;
        pw += v;
        if (v < minpsi) minpsi = v;
      }
      double w = ddx(s, s->U, 2, 1, x, y) - ddy(s, s->U, 2, 0, x, y);
      ens += 0.5 * w * w;
    }
  out[0] = (double)s->nstep;
  out[1] = nval(&mS);
  out[2] = nval(&mP);
  out[3] = nval(&px);
  out[4] = nval(&py);
  out[5] = orc_amplitude(s);
  out[6] = ens;
  out[7] = (pw > 0) ? sqrt(pq2 / pw) / s->p.R : 0.0;
  out[8] = minpsi;
}

/* Threads of the row loops (for timing the oracle at a given core count). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
