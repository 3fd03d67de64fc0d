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
// (bounce-back on the Q-circle).  qnb[d]: the node at Q - c_d for the nine
// D2Q9 directions c_d of a Q-velocity, or -1 outside the disk.
struct alignas(16) QNode {
  double qx, qy, fx, fy;
  int plane[25];
  int qnb[9];
  int pad[2];
};
static_assert(sizeof(QNode) == 176, "QNode layout");

struct StepParams {
  int nx, ny, nqd, qs;  // lattice, Q-nodes, Q-slices per r-tile
  int ntiles;           // r-tiles of 64 nodes
  int tiles_per_xcd;    // XCD-contiguous tile mapping (0 = off)
  int y0;               // absolute row of local row 0 (forcing phase)
  int wg;               // tile groups (qs == 1 only): tiles along x in bits 0-7,
                        // rows in bits 8-15, bit 16: barrier per Q-node; 0 = off
  int qe;               // quasi-equilibrium model: 1 component momenta, 2 stresses
  int shift;            // spring term: 0 Taylor form, 1 psi at r +- Q/2 (interpolated)
  long long N;  // nx * ny
  double aS, aP;         // 1 / (2 tJ + 1) per species
  double tJS, tJP;       // momentum relaxation time: tau2 (model 1), tau1 (model 2)
  double pS, pP;         // model 2: 1 / (2 tau2 + 1), the stress inversion
  double c1S, c2S, rS;   // relaxation: g' = c1 g + c2 [(1-r) f* + r f_eq]
  double c1P, c2P, rP;
  double kappa, DQ, F0, kf;
  const double *src;  // extra body force [2][N] added to the forcing (null: none)
  const int *gate;    // non-null: the launch does nothing once *gate != 0 (drift gate)
};

// One half of the double-buffered state.  Populations and the lagged psi are
// stored as T (double, or float for the FP32 form); per-node fields are FP64.
template <typename T>
struct StateT {
  T *XS, *XP, *PSI;
  double *FLD;
  // BF16 form: XP holds [25][nqd][N] BF16 (uint16) deviations.  MOM is
  // unused (kept null).
  float *MOM;
};
using StateView = StateT<double>;
using StateView32 = StateT<float>;

// FP32 form: populations and psi are stored as float deviations from an
// x-invariant reference state (the base state rounded to FP32, so that
// ref + deviation is exact in FP64), laid out [plane][ny].  Unused (null) for
// FP64 storage.
struct RefView {
  const float *XS, *XP, *PSI;
  int ny;
};
// The same reference values regrouped for the step kernel so that one
// Q-node's values are contiguous and wave-uniform (scalar loads):
//   pull[y][q][k]  reference of the population pulled into (k, q) at row y
//   store[y][q][k] reference of (k, q) at row y
//   psi[y][q], spull[y][d], sstore[y][d] likewise for psi and the solvent.
struct StepRef {
  const float *pull, *store, *psi, *spull, *sstore;
};

// One instance of a batch as the batched step kernel sees it: parameters,
// both halves of its state (untyped: the batch's storage type), its FP32
// reference tables, its Q-node table and the index of its first item
// (64-node tile) in the batch's flat item list.  Half (parity ^ cur0) is read.
struct InstDev {
  StepParams p;
  void *XS[2], *XP[2], *PSI[2];
  double *FLD[2];
  const float *rpull, *rstore, *rpsi, *rspull, *rsstore;
  const QNode *qtab;
  int item0;
  int cur0;
};

// Launchers (tpl_kernels.hip).  All enqueue on stream and return the launch
// status.  T = double or float.  ip = 1, 2: the two alternating in-place
// steps (a and b share XS and XP; nx a multiple of 64, one Q-slice, not the
// BF16 form), 0: read a, write b.
template <typename T>
hipError_t launch_step(const StepParams &p, StateT<T> a, StateT<T> b,
                       StepRef ref, const QNode *qtab, hipStream_t s, bool b16 = false,
                       int ip = 0);
// Non-local spring term: S = kappa sum_Q Fhat [psi(r + Q/2) - psi(r - Q/2)]
// of the read half's psi (bilinear interpolation, periodic) into its FLD
// slots F_MXX (S_x) and F_MXY (S_y), where the step with p.shift reads it.
template <typename T>
hipError_t launch_spring_sum(const StepParams &p, StateT<T> a, StepRef ref, const QNode *qtab,
                             hipStream_t s);
// Same-step gradients: overwrite the read half's PSI, M and U with this
// step's psi^n, M^n and U^n (three launches) before launch_step.  ip as there
// (the pull of the step that follows); FP64 and FP32 forms.  With p.shift the
// M pass is replaced by the spring-sum pass over psi^n (launch_spring_sum),
// whose Q-sum the velocity pass and the step read.
template <typename T>
hipError_t launch_same_step_fields(const StepParams &p, StateT<T> a, StepRef ref,
                                   const QNode *qtab, hipStream_t s, int ip = 0);
// The same for every item of a batch (before launch_step_batch; nqd: the
// batch's Q-nodes per r-node; shift: the batch's shifted spring term).
template <typename T>
hipError_t launch_same_step_fields_batch(const InstDev *inst, int ninst, int nitems, int nqd,
                                         int parity, int ip, bool shift, hipStream_t s);
// BF16 form <-> FP32 deviations from the reference: dev [25][nqd][N] =
// the stored BF16 values of XP (decode), and the rounding of dev to BF16
// into XP (encode).
hipError_t launch_bf16_decode(int nqd, long long N, StateT<float> a, float *dev, hipStream_t s);
hipError_t launch_bf16_encode(int nqd, long long N, const float *dev, StateT<float> a,
                              hipStream_t s);
// Build the FP32 form's reference from the FP64 column state (ref = the
// column rounded to FP32) and the step kernel's regrouped tables.
hipError_t launch_make_ref(int nqd, int ny, StateView col, float *ref,
                           hipStream_t s);
hipError_t launch_step_ref(int nqd, int ny, const QNode *qtab, RefView ref,
                           float *pull, float *store, float *psi, float *spull,
                           float *sstore, hipStream_t s);
// dst[plane][N] = (float)(col[plane][y] - ref[plane][y]) for every x.
hipError_t launch_tile_dev(int planes, int nx, int ny, const double *col,
                           const float *ref, float *dst, hipStream_t s);
// group > 1 (qs == 1 only): consecutive items per workgroup, one wave each.
// ip = 1, 2: the in-place step kinds (every instance in place; qs == 1,
// whole tiles), 0: two arrays.  qe2: every instance runs model (ii) (the
// stress quasi-equilibria; not with shift).
template <typename T>
hipError_t launch_step_batch(const InstDev *inst, int ninst, int nitems, int qs, int grid,
                             bool rowtile, int parity, hipStream_t s, int group = 1,
                             int ip = 0, bool shift = false, bool qe2 = false);
// The shifted spring term's Q-sum for every item of a batch (before
// launch_step_batch with shift; grid workgroups of eight waves walk the items).
template <typename T>
hipError_t launch_spring_sum_batch(const InstDev *inst, int ninst, int nitems, int grid,
                                   int parity, hipStream_t s);
// Closed-form Hookean laminar Kolmogorov column (see k_analytic_column):
// velocity amplitude UL, forcing wavenumber k, relaxation time lam,
// Dk2 = lambda D k^2 (stress diffusion D = c_s^2 tau2_P), s2 = sigma^2,
// densities and the Q-diffusivity D_Q.  Writes XS, XP, PSI and U of col
// (nx = 1); the other per-node fields follow from launch_refresh.
struct AnalyticColumn {
  double UL, k, lam, Dk2, s2, rhoS0, rhoP0, DQ;
};
hipError_t launch_analytic_column(int ny, int nqd, const QNode *qtab, AnalyticColumn c,
                                  StateView col, hipStream_t s);
hipError_t launch_rest(int nqd, long long N, double rhoS0, double rhoP0,
                       const double *peq, StateView a, hipStream_t s);
template <typename T>
hipError_t launch_refresh(int nqd, int nx, int ny, const QNode *qtab,
                          StateT<T> a, RefView ref, hipStream_t s);
hipError_t launch_tile(int nqd, int nx, int ny, StateView col, StateView a,
                       hipStream_t s);
hipError_t launch_tile_fields(int nx, int ny, const double *colFLD,
                              double *FLD, hipStream_t s);
hipError_t launch_perturb_field(int nx, int ny, int x0, int y0, int NX, int NY,
                                int nmodes, const double *modes, double amp_u0,
                                int multimode, double *du, double *partial,
                                hipStream_t s);
template <typename T>
hipError_t launch_perturb_apply(int nqd, int nx, int ny, const double *du,
                                const double *scale, StateT<T> a, RefView ref,
                                hipStream_t s);
hipError_t launch_sum(const double *partial, int n, int ncomp, double *out,
                      hipStream_t s);
hipError_t launch_amplitude_rows(int nx, int ny, const double *FLD,
                                 double *partial, hipStream_t s);
template <typename T>
hipError_t launch_diag(int nx, int ny, int nqd, const QNode *qtab,
                       StateT<T> a, RefView ref, double *partial, int *nblocks,
                       hipStream_t s);
hipError_t launch_diag_final(const double *partial, int nblocks, double *out,
                             hipStream_t s);
template <typename T>
hipError_t launch_observables(int nqd, int nx, int ny, const QNode *qtab,
                              double inv_s2, double G, double mref,
                              StateT<T> a, RefView ref, double *out,
                              hipStream_t s);
// Health of a state: out[0] = number of non-finite mixture velocities and
// polymer densities, out[1] / out[2] = smallest / largest psi.  partial holds
// 3 kHealthBlocks doubles.
template <typename T>
hipError_t launch_health(int nx, int ny, int nqd, StateT<T> a, RefView ref,
                         double *partial, double *out, hipStream_t s);
template <typename T>
hipError_t launch_window(int nx, int ny, int nqd, int x0, int y0, int w, int h,
                         StateT<T> a, RefView ref, double *dst, hipStream_t s);
// Whole-array conversion between stored deviations and full FP64 values:
// dst[plane][N] = ref[plane][y] + src[plane][N] (to64) or the inverse.
hipError_t launch_to_f64(int nx, int ny, int planes, const float *src,
                         const float *ref, double *dst, hipStream_t s);
hipError_t launch_from_f64(int nx, int ny, int planes, const double *src,
                           const float *ref, float *dst, hipStream_t s);

// Learned correction: device view of a network 64-wide hidden layers, nin <= 64
// inputs, nout <= 16 outputs (BF16 operand arrays, FP32 biases and output
// standardisation).
struct MlpDev {
  const uint16_t *W1b, *W2b, *W3b, *W2Tb, *W3Tb;
  const float *b1, *b2, *b3;
  const float *out_mean, *out_std;
  int nin, nout;
};
// Floats of one wave's gradient record (see k_mlp_train).
constexpr int kMlpRecord = 4096 + 64 + 4096 + 64 + 1024 + 16 + 1;

hipError_t launch_mlp_forward(const MlpDev &w, const uint16_t *Xb, long long n, float *Y,
                              hipStream_t s);
hipError_t launch_mlp_train(const MlpDev &w, const uint16_t *Xb, const float *T, long long n,
                            int nrec, float *partial, hipStream_t s);
hipError_t launch_mlp_reduce(const float *partial, int nrec, int nin, int nout, float *grad,
                             hipStream_t s);
hipError_t launch_mlp_adam(float *theta, float *m, float *v, const float *grad, int np, float lr,
                           int t, hipStream_t s);
hipError_t launch_mlp_pack(const float *theta, int nin, int nout, const MlpDev &w,
                           hipStream_t s);
hipError_t launch_mlp_prep(const float *X, long long n, int nin, const float *mean,
                           const float *stdv, uint16_t *Xb, hipStream_t s);
hipError_t launch_features(const double *obs, int nx, int ny, const float *mean,
                           const float *stdv, float *X, uint16_t *Xb, hipStream_t s);
hipError_t launch_targets(const double *ref, const double *obs, long long N, float *T,
                          hipStream_t s);
hipError_t launch_source(const float *corr, int nx, int ny, double *F, hipStream_t s);
// Removes the lattice mean of both components of F [2][N]; scratch holds
// 2048 + 2 doubles.
hipError_t launch_source_center(double *F, long long N, double *scratch, hipStream_t s);
hipError_t launch_source_drift(const double *F, const double *FLD, long long N, double *partial,
                               int *nblocks, hipStream_t s);
// The attached correction of one coarse step in two launches, on the
// context's stream with no host synchronisation:
//   launch_correct: per 16-node tile the 54 stencil features straight from
//     the observables obs[10][N] (standardised, BF16), the network, the
//     correction corr [N][5] in physical units, and per wave the sums of its
//     momentum components into partial [waves][2] (waves = correct_waves(N));
//   launch_source_gate: F [2][N] = (dJ - lattice mean of dJ) + div_h(dtau),
//     the mean from those sums in a fixed order; if max |F| / rho exceeds
//     bound (NaN included), gate := tag unless already set; drift holds the
//     largest |F| / rho seen (as the bits of a non-negative double).
// Both do nothing once *gate != 0.
long long correct_waves(long long N);
hipError_t launch_correct(const MlpDev &w, const double *obs, int nx, int ny, const float *mean,
                          const float *stdv, float *corr, double *partial, const int *gate,
                          hipStream_t s);
hipError_t launch_source_gate(const float *corr, int nx, int ny, const double *partial,
                              long long nparts, const double *FLD, double bound, int tag,
                              double *F, int *gate, unsigned long long *drift, hipStream_t s);
template <typename T>
hipError_t launch_restrict(int planes, int nxf, int nyf, int m, const T *src, double *dst,
                           hipStream_t s);

// Workgroup reductions of one double per thread.  Each wavefront folds its
// 64 lanes with cross-lane exchanges in a fixed butterfly order (every lane
// ends with bitwise the same value, since a + b == b + a), then the
// wavefront results are combined in wavefront order.  Deterministic; the
// result is returned to every thread.  sh holds at least blockDim.x / 64
// doubles.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double block_sum(double v, double *sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double out = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) out += sh[w];
  __syncthreads();
  return out;
}
__device__ inline double block_min(double v, double *sh) {
  v = wave_min(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double out = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) out = fmin(out, sh[w]);
  __syncthreads();
  return out;
}
__device__ inline double block_max(double v, double *sh) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double out = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) out = fmax(out, sh[w]);
  __syncthreads();
  return out;
}

constexpr int kDiagComp = 8;  // massS massP momx momy enstrophy psiQ2 psi minpsi
constexpr int kDiagBlocks = 1024;   // workgroups of the diagnostics reduction
constexpr int kHealthBlocks = 1024;  // workgroups of the health check

}  // namespace tplk
