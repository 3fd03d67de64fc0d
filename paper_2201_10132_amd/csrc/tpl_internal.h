// Internal declarations shared by the device kernels and the host runtime of
// libtpl (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tplk {

// Per-node fields stored next to the populations (double-buffered like them).
enum Field : int {
  F_RHOS = 0,  // solvent density of the last step
  F_RHOP,      // polymer density (sum over Q) of the last step
  F_UX,        // mixture velocity U^n (lagged into the next step)
  F_UY,
  F_MXX,  // M = sum_q psi Q F^T / kT (lagged; its divergence is the
  F_MXY,  //     Q-sum of the spring term)
  F_MYY,
  F_JSX,  // solvent momentum of the post-collision populations
  F_JSY,
  F_M0,  // 9 Q-marginals of the post-collision polymer populations, one per
         // D2Q9 r-direction: they stream exactly like D2Q9 populations, so
         // the next step's polymer density and momentum need no Q-reduction
  NF = F_M0 + 9
};

// One Q-disk node: position, spring force / kT, and for every D4Q25
// velocity k the plane (k' nqd + q') of the population it is pulled from:
// k' = k, q' = the node at Q - Qdot_k when that node is in the disk,
// otherwise k' = the reversed-Qdot velocity and q' = this node
// (bounce-back on the Q-circle).
struct alignas(16) QNode {
  double qx, qy, fx, fy;
  int plane[25];
  int pad[3];
};
static_assert(sizeof(QNode) == 144, "QNode layout");

struct StepParams {
  int nx, ny, nqd, qs;  // lattice, Q-nodes, Q-slices per r-tile
  int ntiles;           // r-tiles of 64 nodes
  int tiles_per_xcd;    // XCD-contiguous tile mapping (0 = off)
  int y0;               // absolute row of local row 0 (forcing phase)
  int pad;
  long long N;  // nx * ny
  double aS, aP;         // 1 / (2 tau2 + 1) per species
  double tau2S, tau2P;
  double c1S, c2S, rS;   // relaxation: g' = c1 g + c2 [(1-r) f* + r f_eq]
  double c1P, c2P, rP;
  double kappa, DQ, F0, kf;
};

struct StateView {  // one half of the double-buffered state
  double *XS, *XP, *PSI, *FLD;
};

// Launchers (tpl_kernels.hip).  All enqueue on stream and return the launch
// status.
hipError_t launch_step_f64(const StepParams &p, StateView a, StateView b,
                           const QNode *qtab, hipStream_t s);
hipError_t launch_rest(int nqd, long long N, double rhoS0, double rhoP0,
                       const double *peq, StateView a, hipStream_t s);
hipError_t launch_refresh(int nqd, long long N, const QNode *qtab,
                          StateView a, hipStream_t s);
hipError_t launch_tile(int nqd, int nx, int ny, StateView col, StateView a,
                       hipStream_t s);
hipError_t launch_perturb_field(int nx, int ny, int x0, int y0, int NX, int NY,
                                int nmodes, const double *modes, double amp_u0,
                                int multimode, double *du, double *partial,
                                hipStream_t s);
hipError_t launch_perturb_apply(int nqd, long long N, const double *du,
                                const double *scale, StateView a,
                                hipStream_t s);
hipError_t launch_sum(const double *partial, int n, int ncomp, double *out,
                      hipStream_t s);
hipError_t launch_amplitude_rows(int nx, int ny, const double *FLD,
                                 double *partial, hipStream_t s);
hipError_t launch_diag(int nx, int ny, int nqd, const QNode *qtab,
                       StateView a, double *partial, int *nblocks,
                       hipStream_t s);
hipError_t launch_diag_final(const double *partial, int nblocks, double *out,
                             hipStream_t s);
hipError_t launch_observables(int nqd, long long N, const QNode *qtab,
                              double inv_s2, double G, double mref,
                              StateView a, double *out, hipStream_t s);
hipError_t launch_nan_check(long long N, const double *FLD, double *partial,
                            int *nblocks, hipStream_t s);
hipError_t launch_window(int nx, int ny, int nqd, int x0, int y0, int w, int h,
                         StateView a, double *dst, hipStream_t s);

constexpr int kDiagComp = 8;  // massS massP momx momy enstrophy psiQ2 psi minpsi
constexpr int kDiagBlock = 256;

}  // namespace tplk
