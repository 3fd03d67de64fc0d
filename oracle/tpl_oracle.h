/*
 * tpl_oracle.h -- FP64 CPU oracle for the two-fluid kinetic scheme of
 * Singh, Subramanian & Ansumali, "Two-fluid kinetic theory for dilute polymer
 * solutions" (arXiv:2201.10132).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * reference used by the tests, by the smoke check and by the benchmark's CPU
 * baseline leg.  The product library never includes, links or calls it, and
 * it shares no code, header, table or constant with the GPU path.
 *
 * Units: lattice units, dx = dt = dQ = 1, c_s^2 = 1/3 for both lattices.
 * Solvent: D2Q9 (Sec. VI.A).  Polymer: D4Q25 over (r, Q) (Sec. VI.B, Table I)
 * with Q restricted to a disk of radius NQ/2.
 *
 * Pins (tests/test_oracle_*.py), i.e. what fixes each part independently of
 * this code:
 *   lattices, Q-disk, bounce-back map  -> isotropy conditions, brute force
 *   equilibria                         -> their defining moments
 *   collide_node                       -> implicit trapezoidal rule solved in
 *                                         extended precision; exact momentum
 *                                         exchange
 *   step (solvent)                     -> shear-wave viscosity c_s^2 tau1
 *   step (polymer, r)                  -> density diffusion c_s^2 tau2_P
 *   step (polymer, Q)                  -> Hookean relaxation time lambda
 *   step (coupling, forcing, spring)   -> laminar Oldroyd-B closed form
 *   step (conservation)                -> mass and momentum invariants
 *   non-local spring shift             -> lattice sums (momentum), the
 *                                         Fourier symbol of interpolation,
 *                                         Taylor limit at long wavelength
 *   same-step gradients                -> independence of the lagged fields;
 *                                         the laminar closed form and the
 *                                         invariants as above
 *   perturb                            -> prescribed RMS amplitude
 *   splitmix64                         -> published test vectors
 *   FENE runs                          -> parity unpinned beyond the above
 *                                         invariants (no closed form exists)
 */
#ifndef TPL_ORACLE_H
#define TPL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Physical / numerical configuration.  All fields are plain inputs. */
typedef struct {
  int nx, ny;          /* lattice size (nx = 1 is the x-invariant column)    */
  int nq;              /* Q points per axis; Q-disk radius R = nq/2          */
  int periods;         /* Kolmogorov forcing periods over ny                 */
  double Re, Wi, beta; /* Sec. VII parameter definitions                     */
  double u0;           /* lattice velocity scale                             */
  double phi;          /* polymer mass fraction rho_P / rho                  */
  int spring;          /* 0 = FENE (Warner), 1 = Hookean                     */
  double b;            /* FENE extensibility; sigma = R / sqrt(b)            */
  double tau_drag;     /* solvent drag time: tau2_S (model 1) or tau1_S
                        * (model 2); 0 = automatic (1 or tau2_S)           */
  double tau_ratio_p;  /* tau1_P / tau2_P (<= 1)                             */
  double force_scale;  /* multiplies the Kolmogorov force amplitude F0       */
  double lambda_set;   /* > 0: use this relaxation time instead of Wi*l/u0   */
  int ny_param;        /* > 0: derive k_f (and all scales) from this ny      */
  int y_offset;        /* absolute row index of local row 0 (forcing phase)  */
  int x_offset;        /* absolute column index of local column 0            */
  int nx_param;        /* > 0: x-extent used for the perturbation modes      */
  double drift_cap;    /* > 0: cap on the Q-drift D_Q |Fhat| per step          */
  double drift_relax;  /* > 0: also cap it at drift_relax (2 - omega_P)        */
  int qe_model;        /* 1: component-momentum quasi-equilibria (Sec. V (i));
                        * 2: stress-tensor quasi-equilibria (Sec. V (ii))      */
  int gradients;       /* time level of the velocity gradient and of the
                        * spring term's psi gradient, which the paper leaves
                        * open: 0 = the previous step's observables (lagged);
                        * 1 = the current step's, from the pulled populations */
  int spring_shift;    /* form of the spring term of J^r_eq (Sec. V):
                        * 0 = first-order Taylor expansion,
                        *     kappa Fhat(Q) (Q . grad psi(r, Q));
                        * 1 = the non-local shift itself,
                        *     kappa Fhat(Q) [psi(r + Q/2, Q) - psi(r - Q/2, Q)],
                        *     psi at r +- Q/2 by periodic bilinear interpolation */
} orc_config;

/* Derived lattice parameters (step 0 of the scheme contract). */
typedef struct {
  double kf, l, nu, nuS, lambda, G;
  double tau1S, tau2S, tau1P, tau2P;
  double R, sigma, DQ, F0, kappa, meq;
  double rhoS0, rhoP0, Sc;
} orc_derived;

typedef struct orc_sim orc_sim;

/* Create / destroy.  Returns NULL and fills err (if non-NULL, >= 256 bytes)
 * when the configuration is invalid (e.g. tau1 > tau2, Sec. IV ordering). */
orc_sim *orc_new(const orc_config *cfg, char *err);
void orc_free(orc_sim *s);

int orc_nqd(const orc_sim *s);
void orc_get_derived(const orc_sim *s, orc_derived *out);
/* Lattice tables: cS[9*2], wS[9], cP[25*4], wP[25], Q[nqd*2], Fhat[nqd*2],
 * nbrQ[25*nqd], kstar[25], peq[nqd].  Any pointer may be NULL. */
void orc_get_tables(const orc_sim *s, int *cS, double *wS, int *cP,
                    double *wP, double *Q, double *Fhat, int *nbrQ,
                    int *kstar, double *peq);

/* Initial states (step 8). */
void orc_rest(orc_sim *s);
void orc_base_state(orc_sim *s, long npre); /* npre < 0: default length */
/* Hookean laminar Kolmogorov state in closed form (model 1, Wi > 0); -1 and
 * nothing changed otherwise. */
int orc_analytic_state(orc_sim *s);
long orc_default_prerun(const orc_sim *s);
void orc_perturb(orc_sim *s, uint64_t seed, double amp, int multimode);

/* Advance n steps (steps 3-7 and 9). */
void orc_step(orc_sim *s, long n);
long orc_step_count(const orc_sim *s);

/* State exchange in the canonical layouts:
 *   XS[9][ny][nx], XP[25][nqd][ny][nx], psi[nqd][ny][nx], U[2][ny][nx].
 * Any pointer may be NULL.  orc_set_state also sets the recorded
 * densities from the populations. */
void orc_get_state(const orc_sim *s, double *XS, double *XP, double *psi,
                   double *U);
void orc_set_state(orc_sim *s, const double *XS, const double *XP,
                   const double *psi, const double *U);

/* Observables of the last completed step (step 9), SoA [10][ny][nx]:
 * rho, Ux, Uy, rhoP, Cxx, Cxy, Cyy, tau_xx, tau_xy, tau_yy. */
void orc_observables(const orc_sim *s, double *out);
/* Extra body force F[2][ny][nx] added in every later step; NULL removes it. */
void orc_set_source(orc_sim *s, const double *F);
double orc_amplitude(const orc_sim *s);

/* Second-order Hermite quasi-equilibria of the stress-tensor model (Sec. VI.A,
 * VI.B, model (ii)): the populations with density rho, first moments J and
 * second moments P.  Solvent on D2Q9: J[2], P = (xx, xy, yy).  Polymer on
 * D4Q25 over xi = (v_x, v_y, Qdot_x, Qdot_y): J[4], P = upper triangle of the
 * 4 x 4 tensor, row-major (00 01 02 03 11 12 13 22 23 33). */
void orc_solvent_qe2(double rho, const double J[2], const double P[3], double *out);
void orc_polymer_qe2(const orc_sim *s, double psi, const double J[4], const double P[10],
                     double *out);

/* Threads used by the row loops: set (n > 0) and read back. */
void orc_set_threads(int n);
int orc_max_threads(void);
/* out[9]: step, massS, massP, momx, momy, amplitude, enstrophy, qrms, minpsi */
void orc_diagnostics(const orc_sim *s, double *out);

/* Single-node pieces, exported for the pin tests. */
void orc_solvent_eq(double rho, double ux, double uy, double *out9);
void orc_polymer_eq(const orc_sim *s, double psi, const double Jr[2],
                    const double JQ[2], double *out25);
/* Spring terms sq[nqd][2] of J^r_eq at node (x, y) from the recorded psi
 * (the form spring_shift selects). */
void orc_spring_terms(const orc_sim *s, int x, int y, double *sq);
/* One collision at one r-node from pulled populations gS[9], gP[nqd][25]
 * with lagged velocity gradient K[4] = (dUx/dx, dUx/dy, dUy/dx, dUy/dy),
 * spring terms sq[nqd][2] and body force Fb[2]; writes post-collision
 * populations and the mixture velocity U[2]. */
void orc_collide_node(const orc_sim *s, const double *gS, const double *gP,
                      const double K[4], const double *sq, const double Fb[2],
                      double *outS, double *outP, double U[2]);

/* SplitMix64 (Steele, Lea & Flood 2014), exported for its test vector. */
uint64_t orc_splitmix64_next(uint64_t *state);

#ifdef __cplusplus
}
#endif
#endif
