// Host runtime of libtpl: parameter derivation, Q-disk tables, device state,
// initialisation sequence, time stepping and the C ABI of include/tpl.h.
#include "../../include/tpl.h"
#include "tpl_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace tplk;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                       \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(TPL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr double kCs2 = 1.0 / 3.0;

// Configuration (inputs) and everything derived from it (step 0 of the
// scheme: Sec. VII parameter definitions; Sec. IV viscosity ~ tau1; App. A
// Q-diffusivity 2 kT / zeta).
struct Config {
  int nx = 0, ny = 0, periods = 1;
  double Re = 0, Wi = 0, beta = 1, u0 = 0.05;
  int nq = 16, spring = 0, precision = TPL_FP64, pert_modes = 1;
  double b = 25.0, phi = 0.01, tau_drag = 0.0, tau_ratio_p = 1.0;
  double force_scale = 1.0, lambda_set = 0.0, drift_cap = 0.2, drift_relax = 1.0;
  long long pre_steps = -1;
  int qsplit = 0, time_kernels = 0;
  int group_x = 1, group_y = 1, group_sync = 0, autotune = 1;
  int qe_model = 1;
  int inplace = 0;  // one population array, streamed in place
  int gradients = 0;  // 0: lagged (previous step's) gradients; 1: same-step
  int spring_shift = 0;  // spring term: 0 Taylor form, 1 psi at r +- Q/2
  int init_mode = 0;         // 0: base state by a column pre-run; 1: closed form (Hookean)
  long long diag_every = 0;  // health check every k steps of tpl_step (0: at its end)
  double psi_floor = 1.0;    // unstable if min psi < -psi_floor max psi
  int keep_good = 0;         // 1: a failed check restores the last checked state
};

struct Derived {
  double kf, l, nu, nuS, lambda, G, tau1S, tau2S, tau1P, tau2P;
  double R, sigma, DQ, F0, kappa, meq, rhoS0, rhoP0, Sc;
  int nqd;
  std::vector<QNode> qtab;
  std::vector<double> peq;
};

int derive(const Config &c, Derived &d) {
  if (c.nx < 1 || c.ny < 1) return fail(TPL_EINVAL, "nx, ny must be >= 1");
  if (c.periods < 1 || c.ny < 4 * c.periods)
    return fail(TPL_EINVAL, "need periods >= 1 and ny >= 4 periods");
  if (!(c.Re > 0)) return fail(TPL_EINVAL, "Re must be > 0");
  if (!(c.Wi >= 0)) return fail(TPL_EINVAL, "Wi must be >= 0");
  if (!(c.beta > 0 && c.beta <= 1)) return fail(TPL_EINVAL, "beta must be in (0,1]");
  if (!(c.u0 > 0 && c.u0 <= 0.1)) return fail(TPL_EINVAL, "u0 must be in (0,0.1]");
  if (c.nq < 4 || c.nq > 48 || (c.nq & 1)) return fail(TPL_EINVAL, "nq must be even in [4,48]");
  if (!(c.phi >= 0 && c.phi < 1)) return fail(TPL_EINVAL, "phi must be in [0,1)");
  if (!(c.b > 1)) return fail(TPL_EINVAL, "b must be > 1");
  if (!(c.tau_ratio_p > 0 && c.tau_ratio_p <= 1))
    return fail(TPL_EINVAL, "tau_ratio_p must be in (0,1] (tau1 <= tau2)");
  if (c.qe_model != 1 && c.qe_model != 2) return fail(TPL_EINVAL, "qe_model must be 1 or 2");
  if (c.inplace != 0 && c.inplace != 1) return fail(TPL_EINVAL, "inplace must be 0 or 1");
  if (c.inplace && c.precision == TPL_BF16)
    return fail(TPL_EINVAL, "in-place streaming is for the FP64 and FP32 forms");
  if (c.inplace && c.nx % 64)
    return fail(TPL_EINVAL, "in-place streaming needs nx a multiple of 64");
  if (c.gradients != 0 && c.gradients != 1) return fail(TPL_EINVAL, "gradients must be 0 or 1");
  if (c.gradients && c.precision == TPL_BF16)
    return fail(TPL_EINVAL, "same-step gradients are for the FP64 and FP32 forms");
  if (c.spring_shift != 0 && c.spring_shift != 1)
    return fail(TPL_EINVAL, "spring_shift must be 0 or 1");
  if (c.spring_shift && c.precision == TPL_BF16)
    return fail(TPL_EINVAL, "the shifted spring term is for the FP64 and FP32 forms");
  // the step kernel addresses a plane with 32-bit byte offsets: 8 N < 2^32
  if ((long long)c.nx * c.ny >= (1LL << 29)) return fail(TPL_EINVAL, "lattice too large");

  d.kf = 2.0 * kPi * c.periods / c.ny;
  d.l = 1.0 / d.kf;
  d.nu = c.u0 * d.l / c.Re;
  d.rhoS0 = 1.0 - c.phi;
  d.rhoP0 = c.phi;
  d.R = 0.5 * c.nq;
  d.sigma = d.R / std::sqrt(c.b);
  if (c.Wi > 0) {
    d.lambda = c.Wi * d.l / c.u0;
    d.nuS = c.beta * d.nu;
    d.G = (1.0 - c.beta) * d.nu / d.lambda;  // eta_p = G lambda, rho = 1
  } else {  // Newtonian limit: passive polymer, no elastic stress
    d.lambda = d.l / c.u0;
    d.nuS = d.nu;
    d.G = 0.0;
  }
  if (c.lambda_set > 0) {
    d.G *= d.lambda / c.lambda_set;
    d.lambda = c.lambda_set;
  }
  if (c.qe_model == 2) {
    // stress-tensor quasi-equilibria (Sec. V model (ii)): stresses relax with
    // tau2 (viscosity c_s^2 tau2), momenta and fluxes with tau1 (drag,
    // diffusivities)
    d.tau2S = d.nuS / kCs2;
    d.tau1S = c.tau_drag > 0 ? c.tau_drag : d.tau2S;  // 0: automatic
    d.tau1P = d.sigma * d.sigma / (2.0 * kCs2 * d.lambda);
    d.tau2P = d.tau1P / c.tau_ratio_p;
    d.DQ = kCs2 * d.tau1P;
  } else {
    d.tau1S = d.nuS / kCs2;
    d.tau2S = c.tau_drag > 0 ? c.tau_drag : 1.0;  // 0: automatic
    d.tau2P = d.sigma * d.sigma / (2.0 * kCs2 * d.lambda);
    d.tau1P = c.tau_ratio_p * d.tau2P;
    d.DQ = kCs2 * d.tau2P;
  }
  d.F0 = c.force_scale * d.nu * c.u0 * d.kf * d.kf;
  d.Sc = d.nuS / d.DQ;
  if (d.tau1S > d.tau2S * (1.0 + 1e-12))
    return fail(TPL_EINVAL, "solvent tau1 = " + std::to_string(d.tau1S) +
                                " exceeds tau2 = " + std::to_string(d.tau2S) +
                                " (H-theorem ordering)");

  // Q-disk: half-integer nodes strictly inside |Q| < R, row by row.
  const int nq = c.nq;
  std::vector<int> idx(nq * nq, -1);
  std::vector<int> ia, ib;
  for (int bq = 0; bq < nq; ++bq)
    for (int aq = 0; aq < nq; ++aq) {
      const double qx = aq + 0.5 - d.R, qy = bq + 0.5 - d.R;
      if (qx * qx + qy * qy < d.R * d.R) {
        idx[bq * nq + aq] = (int)ia.size();
        ia.push_back(aq);
        ib.push_back(bq);
      }
    }
  d.nqd = (int)ia.size();
  d.qtab.assign(d.nqd, QNode{});
  d.peq.assign(d.nqd, 0.0);
  static const int PVh[25][4] = {
      {0, 0, 0, 0},   {1, 1, 0, 0},   {1, -1, 0, 0},  {-1, 1, 0, 0},
      {-1, -1, 0, 0}, {1, 0, 1, 0},   {1, 0, -1, 0},  {-1, 0, 1, 0},
      {-1, 0, -1, 0}, {1, 0, 0, 1},   {1, 0, 0, -1},  {-1, 0, 0, 1},
      {-1, 0, 0, -1}, {0, 1, 1, 0},   {0, 1, -1, 0},  {0, -1, 1, 0},
      {0, -1, -1, 0}, {0, 1, 0, 1},   {0, 1, 0, -1},  {0, -1, 0, 1},
      {0, -1, 0, -1}, {0, 0, 1, 1},   {0, 0, 1, -1},  {0, 0, -1, 1},
      {0, 0, -1, -1}};
  const double s2 = d.sigma * d.sigma, bs2 = c.b * s2;
  double cap = c.drift_cap > 0 ? c.drift_cap : HUGE_VAL;
  if (c.drift_relax > 0) cap = std::min(cap, c.drift_relax * (2.0 - 2.0 / (2.0 * d.tau1P + 1.0)));
  double wsum = 0.0;
  for (int q = 0; q < d.nqd; ++q) {
    QNode &n = d.qtab[q];
    n.qx = ia[q] + 0.5 - d.R;
    n.qy = ib[q] + 0.5 - d.R;
    const double q2 = n.qx * n.qx + n.qy * n.qy;
    // spring force / kT: Hookean Q/sigma^2 or Warner FENE
    // Q / (sigma^2 (1 - Q^2/(b sigma^2))), capped so that the Q-drift
    // D_Q |F/kT| per step stays <= drift_cap and <= drift_relax (2 - omega_P),
    // the damping rate of the polymer's non-conserved moments
    double f = 1.0 / s2;
    if (c.spring == 0) f /= (1.0 - q2 / bs2);
    const double drift = d.DQ * f * std::sqrt(q2);
    if (drift > cap) f *= cap / drift;
    n.fx = f * n.qx;
    n.fy = f * n.qy;
    for (int k = 0; k < 25; ++k) {
      const int sa = ia[q] - PVh[k][2], sb = ib[q] - PVh[k][3];
      const int src = (sa >= 0 && sb >= 0 && sa < nq && sb < nq) ? idx[sb * nq + sa] : -1;
      int ks = k;  // same r-velocity, reversed Q-velocity
      for (int j = 0; j < 25; ++j)
        if (PVh[j][0] == PVh[k][0] && PVh[j][1] == PVh[k][1] && PVh[j][2] == -PVh[k][2] &&
            PVh[j][3] == -PVh[k][3])
          ks = j;
      n.plane[k] = src >= 0 ? k * d.nqd + src : ks * d.nqd + q;
    }
    static const int C9[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                 {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    for (int dd = 0; dd < 9; ++dd) {
      const int sa = ia[q] - C9[dd][0], sb = ib[q] - C9[dd][1];
      n.qnb[dd] = (sa >= 0 && sb >= 0 && sa < nq && sb < nq) ? idx[sb * nq + sa] : -1;
    }
    n.pad[0] = n.pad[1] = 0;
    const double w = c.spring == 0 ? std::pow(1.0 - q2 / bs2, 0.5 * c.b)
                                   : std::exp(-0.5 * q2 / s2);
    d.peq[q] = w;
    wsum += w;
  }
  double m = 0.0;
  for (int q = 0; q < d.nqd; ++q) {
    d.peq[q] /= wsum;
    m += d.peq[q] * (d.qtab[q].qx * d.qtab[q].fx + d.qtab[q].qy * d.qtab[q].fy);
  }
  d.meq = 0.5 * m;
  // the polymer flux relaxes with tau2_P (model 1) or tau1_P (model 2)
  const double tJ = c.qe_model == 2 ? d.tau1P : d.tau2P;
  d.kappa = d.rhoP0 > 0 ? d.G * tJ / (d.rhoP0 * d.meq) : 0.0;
  return TPL_OK;
}

// Double-buffered state.  XS and PSI hold elements of esize bytes (8: FP64
// values, 4: FP32 deviations from the reference), XP elements of xsize bytes
// (8, 4, or 2: the BF16 deviations of the BF16 form); FLD is FP64.  With in-place streaming
// both halves share one XS and one XP array.
struct Buffers {
  void *XS = nullptr, *XP = nullptr, *PSI = nullptr;
  double *FLD = nullptr;
  float *MOM = nullptr;
  size_t nXS = 0, nXP = 0, nPSI = 0, nFLD = 0, nMOM = 0;  // elements per half
  size_t esize = 8, xsize = 8;
  bool inplace = false;
  int pop_copies() const { return inplace ? 1 : 2; }
  size_t pop_half(int h) const { return inplace ? 0 : (size_t)h; }
  template <typename T>
  StateT<T> half(int h) const {
    return StateT<T>{static_cast<T *>(XS) + pop_half(h) * nXS,
                     reinterpret_cast<T *>(static_cast<char *>(XP) + pop_half(h) * nXP * xsize),
                     static_cast<T *>(PSI) + h * nPSI, FLD + h * nFLD,
                     MOM ? MOM + h * nMOM : nullptr};
  }
  StateView half64(int h) const { return half<double>(h); }
};

}  // namespace

struct tpl_mlp;

struct tpl_ctx {
  Config c;
  Derived d;
  hipStream_t stream = nullptr;
  bool inited = false, owned = true;
  Buffers buf;
  int cur = 0;
  int ip_odd = 0;  // in-place streaming: populations in streamed, reversed order
  long long step = 0;
  QNode *qtab_d = nullptr;
  double *peq_d = nullptr;
  float *ref = nullptr;   // FP32 form: reference state [9 + 26 nqd planes][ny]
  float *sref = nullptr;  // FP32 form: the same values regrouped for the step kernel
  double *scratch = nullptr;  // reductions, perturbation field, windows
  size_t scratch_n = 0;
  double kernel_ms = 0.0;
  long long kernel_launches = 0;
  int qs_used = 0, wg_used = 0;
  bool tuned = false;  // tile-group shape timed (first step)
  int wg_tuned = 0;    // its StepParams::wg (0: one tile per workgroup)
  double tune_ms = 0.0;
  // extra body force [2][N] (a caller's field or an attached correction's)
  double *src_d = nullptr;
  bool src_on = false;
  // attached learned correction and its working arrays
  tpl_mlp *mlp = nullptr;
  double drift_bound = 0.0, last_drift = 0.0;
  double *obs_d = nullptr;    // [10][N] observables
  float *corr_d = nullptr;    // [N][5] correction
  double *part_d = nullptr;   // [waves][2] per-wave sums of the momentum correction
  int *gate_d = nullptr;      // drift gate: 0 open, else the step of the call it stopped
  unsigned long long *drift_d = nullptr;  // largest |F| / rho of the call (double bits)
  // keep_good: copy of the last state that passed a health check
  char *good_d = nullptr;
  size_t good_bytes = 0;
  long long good_step = 0;
  int good_cur = 0, good_ip_odd = 0;
};

namespace {

size_t state_elems(const tpl_ctx *x, int which) {
  const size_t N = (size_t)x->c.nx * x->c.ny, nqd = x->d.nqd;
  switch (which) {
    case 0: return 9 * N;
    // the BF16 form holds a 26th 16-bit plane per Q-node: the lower half of
    // the rest population's FP32 deviation
    case 1: return (x->c.precision == TPL_BF16 ? 26 : 25) * nqd * N;
    case 2: return nqd * N;
    default: return (size_t)NF * N;
  }
}

// Tile groups: gx x gy tiles of 64 nodes (gy consecutive rows) per
// workgroup, one wave each, optionally kept on the same Q-node by a barrier,
// so that the group's overlapping stencil reads (x-shifted pulls across tile
// edges, psi of the rows above and below) meet in the caches.  Only for one
// Q-slice and whole tiles per row; returns false (p unchanged) otherwise.
bool set_group(StepParams &p, int gx, int gy, int sync) {
  if (p.qs != 1 || gx * gy < 2 || gx * gy > 8 || p.nx % 64 || (p.nx / 64) % gx || p.ny % gy)
    return false;
  const int groups = p.ntiles / (gx * gy);
  p.wg = gx | (gy << 8) | (sync ? 1 << 16 : 0);
  p.tiles_per_xcd = groups >= 64 ? (groups + 7) / 8 : 0;
  return true;
}

StepParams make_step_params(const tpl_ctx *x, int nx, int ny, int qs_req) {
  StepParams p{};
  const Derived &d = x->d;
  p.nx = nx;
  p.ny = ny;
  p.N = (long long)nx * ny;
  p.nqd = d.nqd;
  p.ntiles = (int)((p.N + 63) / 64);
  int qs = qs_req;
  if (qs <= 0) {  // aim at >= 2048 waves in flight, at most 8 slices
    qs = 1;
    while (qs < 8 && (long long)p.ntiles * qs < 2048) qs *= 2;
  }
  // in place, every wave owns its nodes' populations: one Q-slice
  if (x->c.inplace && nx == x->c.nx && ny == x->c.ny) qs = 1;
  // 1, 2, 4 or 8 slices (the slice reduction uses qs * 6 KB of LDS)
  qs = qs >= 8 ? 8 : qs >= 4 ? 4 : qs >= 2 ? 2 : 1;
  p.qs = qs;
  p.tiles_per_xcd = p.ntiles >= 64 ? (p.ntiles + 7) / 8 : 0;
  p.wg = 0;
  if (x->c.group_x * x->c.group_y > 1)
    set_group(p, x->c.group_x, x->c.group_y, x->c.group_sync);
  else if (x->tuned && nx == x->c.nx && ny == x->c.ny && x->wg_tuned)
    set_group(p, x->wg_tuned & 255, (x->wg_tuned >> 8) & 255, (x->wg_tuned >> 16) & 1);
  p.y0 = 0;
  const bool m2 = x->c.qe_model == 2;
  p.qe = m2 ? 2 : 1;
  p.shift = x->c.spring_shift;
  p.tJS = m2 ? d.tau1S : d.tau2S;
  p.tJP = m2 ? d.tau1P : d.tau2P;
  p.aS = 1.0 / (2.0 * p.tJS + 1.0);
  p.aP = 1.0 / (2.0 * p.tJP + 1.0);
  p.pS = 1.0 / (2.0 * d.tau2S + 1.0);
  p.pP = 1.0 / (2.0 * d.tau2P + 1.0);
  const double bS = 1.0 / (2.0 * d.tau1S + 1.0), bP = 1.0 / (2.0 * d.tau1P + 1.0);
  p.c1S = 1.0 - 2.0 * bS;
  p.c2S = 2.0 * bS;
  p.rS = d.tau1S / d.tau2S;
  p.c1P = 1.0 - 2.0 * bP;
  p.c2P = 2.0 * bP;
  p.rP = d.tau1P / d.tau2P;
  p.kappa = d.kappa;
  p.DQ = d.DQ;
  p.F0 = d.F0;
  p.kf = d.kf;
  p.src = (x->src_on && nx == x->c.nx && ny == x->c.ny) ? x->src_d : nullptr;
  p.gate = (x->mlp && nx == x->c.nx && ny == x->c.ny) ? x->gate_d : nullptr;
  return p;
}

int ensure_scratch(tpl_ctx *x, size_t n) {
  if (x->scratch_n >= n) return TPL_OK;
  if (x->scratch) HIPCHK(hipFree(x->scratch));
  x->scratch = nullptr;
  x->scratch_n = 0;
  if (hipMalloc(&x->scratch, n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TPL_ENOMEM, "scratch allocation failed");
  }
  x->scratch_n = n;
  return TPL_OK;
}

size_t elem_size(const tpl_ctx *x) { return x->c.precision == TPL_FP64 ? 8 : 4; }
size_t xp_size(const tpl_ctx *x) {
  return x->c.precision == TPL_FP64 ? 8 : x->c.precision == TPL_FP32 ? 4 : 2;
}
// FP32 reference forms (FP32 storage and the BF16 form)
bool fp32(const tpl_ctx *x) { return x->c.precision != TPL_FP64; }
bool bf16(const tpl_ctx *x) { return x->c.precision == TPL_BF16; }

int alloc_state(tpl_ctx *x) {
  if (x->buf.XS) return TPL_OK;
  Buffers &B = x->buf;
  B.nXS = state_elems(x, 0);
  B.nXP = state_elems(x, 1);
  B.nPSI = state_elems(x, 2);
  B.nFLD = state_elems(x, 3);
  B.nMOM = 0;
  B.esize = elem_size(x);
  B.xsize = xp_size(x);
  B.inplace = x->c.inplace != 0;
  void **ptrs[5] = {&B.XS, &B.XP, &B.PSI, reinterpret_cast<void **>(&B.FLD),
                    reinterpret_cast<void **>(&B.MOM)};
  const size_t pc = B.pop_copies();
  size_t bytes[5] = {pc * B.nXS * B.esize, pc * B.nXP * B.xsize, 2 * B.nPSI * B.esize,
                     2 * B.nFLD * sizeof(double), 2 * B.nMOM * sizeof(float)};
  for (int i = 0; i < 4; ++i) {
    if (hipMalloc(ptrs[i], bytes[i]) != hipSuccess) {
      (void)hipGetLastError();
      for (int j = 0; j < i; ++j) {
        (void)hipFree(*ptrs[j]);
        *ptrs[j] = nullptr;
      }
      B.XS = B.XP = B.PSI = nullptr;
      B.FLD = nullptr;
      B.MOM = nullptr;
      char msg[160];
      snprintf(msg, sizeof msg, "device allocation of %.2f GB failed", bytes[i] / 1e9);
      return fail(TPL_ENOMEM, msg);
    }
  }
  x->owned = true;
  return TPL_OK;
}

RefView ref_view(const tpl_ctx *x) {
  const size_t ny = x->c.ny, nqd = x->d.nqd;
  if (!x->ref) return RefView{nullptr, nullptr, nullptr, x->c.ny};
  return RefView{x->ref, x->ref + 9 * ny, x->ref + (9 + 25 * nqd) * ny, x->c.ny};
}
size_t ref_elems(const tpl_ctx *x) { return (9 + 26 * (size_t)x->d.nqd) * x->c.ny; }
size_t sref_elems(const tpl_ctx *x) {
  return (50 * (size_t)x->d.nqd + x->d.nqd + 18) * x->c.ny;
}
StepRef step_ref(const tpl_ctx *x) {
  if (!x->sref) return StepRef{nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t ny = x->c.ny, nqd = x->d.nqd;
  float *p = x->sref;
  return StepRef{p, p + 25 * nqd * ny, p + 50 * nqd * ny, p + 51 * nqd * ny,
                 p + 51 * nqd * ny + 9 * ny};
}
int build_step_ref(tpl_ctx *x) {
  const StepRef r = step_ref(x);
  HIPCHK(launch_step_ref(x->d.nqd, x->c.ny, x->qtab_d, ref_view(x), const_cast<float *>(r.pull),
                         const_cast<float *>(r.store), const_cast<float *>(r.psi),
                         const_cast<float *>(r.spull), const_cast<float *>(r.sstore), x->stream));
  return TPL_OK;
}

// BF16 form: an FP32 view of one half whose polymer
// populations are decoded into a temporary (FP32 deviations), for the
// auxiliary kernels; write-back re-encodes them.
// For the other forms the view is the stored half itself.
struct FloatView {
  StateView32 v{};
  float *tmp = nullptr;
  ~FloatView() {
    if (tmp) (void)hipFree(tmp);
  }
};
int float_view(tpl_ctx *x, int h, FloatView &fv) {
  fv.v = x->buf.half<float>(h);
  if (!bf16(x)) return TPL_OK;
  const long long N = (long long)x->c.nx * x->c.ny;
  if (hipMalloc(&fv.tmp, 25 * (size_t)x->d.nqd * N * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    fv.tmp = nullptr;
    return fail(TPL_ENOMEM, "decode buffer allocation failed");
  }
  HIPCHK(launch_bf16_decode(x->d.nqd, N, fv.v, fv.tmp, x->stream));
  fv.v.XP = fv.tmp;
  return TPL_OK;
}
int float_writeback(tpl_ctx *x, int h, FloatView &fv) {
  if (!bf16(x)) return TPL_OK;
  const long long N = (long long)x->c.nx * x->c.ny;
  HIPCHK(launch_bf16_encode(x->d.nqd, N, fv.tmp, x->buf.half<float>(h), x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

int upload_tables(tpl_ctx *x) {
  if (x->qtab_d) HIPCHK(hipFree(x->qtab_d));
  if (x->peq_d) HIPCHK(hipFree(x->peq_d));
  x->qtab_d = nullptr;
  x->peq_d = nullptr;
  HIPCHK(hipMalloc(&x->qtab_d, sizeof(QNode) * x->d.nqd));
  HIPCHK(hipMalloc(&x->peq_d, sizeof(double) * x->d.nqd));
  HIPCHK(hipMemcpyAsync(x->qtab_d, x->d.qtab.data(), sizeof(QNode) * x->d.nqd,
                        hipMemcpyHostToDevice, x->stream));
  HIPCHK(hipMemcpyAsync(x->peq_d, x->d.peq.data(), sizeof(double) * x->d.nqd,
                        hipMemcpyHostToDevice, x->stream));
  return TPL_OK;
}

// Q-slices of the base-state column steps (single and batched alike, so that
// both produce the same base state).
constexpr int kColumnQs = 8;

// One step of the lattice in B read from half cur: with same-step gradients
// the three field launches, with the shifted spring term its Q-sum, then the
// step (ip: the in-place step kind).
hipError_t enqueue_step(const tpl_ctx *x, const Buffers &B, const StepParams &p,
                        const StepRef &ref, int cur, int ip) {
  hipError_t e = hipSuccess;
  if (B.esize == 4) {
    if (x->c.gradients) e = launch_same_step_fields<float>(p, B.half<float>(cur), ref, x->qtab_d,
                                                           x->stream, ip);
    if (e == hipSuccess && p.shift && !x->c.gradients)
      e = launch_spring_sum<float>(p, B.half<float>(cur), ref, x->qtab_d, x->stream);
    if (e == hipSuccess)
      e = launch_step<float>(p, B.half<float>(cur), B.half<float>(1 - cur), ref, x->qtab_d,
                             x->stream, B.xsize == 2, ip);
  } else {
    if (x->c.gradients) e = launch_same_step_fields<double>(p, B.half<double>(cur), ref,
                                                            x->qtab_d, x->stream, ip);
    if (e == hipSuccess && p.shift && !x->c.gradients)
      e = launch_spring_sum<double>(p, B.half<double>(cur), ref, x->qtab_d, x->stream);
    if (e == hipSuccess)
      e = launch_step<double>(p, B.half<double>(cur), B.half<double>(1 - cur), ref, x->qtab_d,
                              x->stream, false, ip);
  }
  return e;
}

// Enqueue n steps of an nx x ny lattice held in B (halves *cur and 1-*cur)
// with qs_req Q-slices (0: automatic).  B's element size selects the FP64 or
// the FP32 step.
int run_steps(tpl_ctx *x, const Buffers &B, int nx, int ny, int *cur,
              long long n, bool timed, int qs_req) {
  StepParams p = make_step_params(x, nx, ny, qs_req);
  const StepRef ref = B.esize == 4 ? step_ref(x) : StepRef{nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Events {  // destroyed on every return path
    hipEvent_t *a, *b;
    ~Events() {
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } guard{&e0, &e1};
  if (timed) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
  }
  for (long long i = 0; i < n; ++i) {
    if (timed) HIPCHK(hipEventRecord(e0, x->stream));
    const int ip = B.inplace ? (x->ip_odd ? 2 : 1) : 0;
    HIPCHK(enqueue_step(x, B, p, ref, *cur, ip));
    if (B.inplace) x->ip_odd ^= 1;
    if (timed) {
      HIPCHK(hipEventRecord(e1, x->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      x->kernel_ms += ms;
      x->kernel_launches++;
    }
    *cur = 1 - *cur;
  }
  return TPL_OK;
}

// Times the tile-group shapes of the full lattice's step and keeps the
// fastest (every shape computes bitwise the same step).  The timed launches
// read the current half and write the other without swapping, so repeating
// them changes nothing; the first launch of each shape is a warm-up.
constexpr int kTuneShapes = 6;
const int kTuneCand[kTuneShapes][3] = {{1, 1, 0}, {4, 1, 1}, {2, 2, 1},
                                       {8, 1, 0}, {8, 1, 1}, {4, 2, 1}};

int tune_groups(tpl_ctx *x) {
  if (x->buf.inplace) return TPL_OK;  // timed on real steps (tune_groups_inplace)
  x->tuned = true;
  x->wg_tuned = 0;
  StepParams p0 = make_step_params(x, x->c.nx, x->c.ny, x->c.qsplit);
  if (p0.qs != 1 || p0.wg != 0 || x->c.group_x * x->c.group_y > 1) return TPL_OK;
  const Buffers &B = x->buf;
  const bool b16 = B.xsize == 2;
  const auto &cand = kTuneCand;
  const StepRef ref =
      B.esize == 4 ? step_ref(x) : StepRef{nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 0.f;
  int rc = TPL_OK;
  for (const auto &c : cand) {
    StepParams p = p0;
    if (c[0] * c[1] > 1 && !set_group(p, c[0], c[1], c[2])) continue;
    auto launch = [&]() {
      return B.esize == 4
                 ? launch_step<float>(p, B.half<float>(x->cur), B.half<float>(1 - x->cur), ref,
                                      x->qtab_d, x->stream, b16)
                 : launch_step<double>(p, B.half<double>(x->cur), B.half<double>(1 - x->cur),
                                       ref, x->qtab_d, x->stream);
    };
    hipError_t e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, x->stream);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, x->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail(TPL_EHIP, std::string("tile-group tuning: ") + hipGetErrorString(e));
      break;
    }
    x->tune_ms += ms * 1.5;
    if (best == 0.f || ms < best) {
      best = ms;
      x->wg_tuned = p.wg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// In-place steps cannot be repeated without advancing the state, so the
// shapes are timed on real steps: a warm-up pair and a timed pair each
// (every shape computes bitwise the same steps).  Needs kTuneSteps steps;
// returns the number taken in *done.
constexpr int kTuneSteps = 4 * kTuneShapes;
int tune_groups_inplace(tpl_ctx *x, long long *done) {
  *done = 0;
  x->tuned = true;
  x->wg_tuned = 0;
  const StepParams p0 = make_step_params(x, x->c.nx, x->c.ny, x->c.qsplit);
  if (p0.wg != 0 || x->c.group_x * x->c.group_y > 1) return TPL_OK;
  const Buffers &B = x->buf;
  const StepRef ref =
      B.esize == 4 ? step_ref(x) : StepRef{nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 0.f;
  int rc = TPL_OK, best_wg = 0;
  for (const auto &c : kTuneCand) {
    StepParams p = p0;
    if (c[0] * c[1] > 1 && !set_group(p, c[0], c[1], c[2])) continue;
    auto launch = [&]() {
      const hipError_t e = enqueue_step(x, B, p, ref, x->cur, x->ip_odd ? 2 : 1);
      if (e == hipSuccess) {  // a real step
        x->ip_odd ^= 1;
        x->cur = 1 - x->cur;
        ++*done;
      }
      return e;
    };
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, x->stream);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, x->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail(TPL_EHIP, std::string("tile-group tuning: ") + hipGetErrorString(e));
      break;
    }
    x->tune_ms += ms * 2.0;
    if (best == 0.f || ms < best) {
      best = ms;
      best_wg = p.wg;
    }
  }
  x->wg_tuned = best_wg;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// SplitMix64 (Steele, Lea & Flood 2014) and the uniform double it yields.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

int perturb(tpl_ctx *x, uint64_t seed, double amp) {
  const int nx = x->c.nx, ny = x->c.ny;
  const long long N = (long long)nx * ny;
  const int multimode = x->c.pert_modes ? 1 : 0;
  // mode table: (kx, ky, a, phase); a ~ N(0,1) by Box-Muller, phase ~ U[0,2pi)
  std::vector<double> modes;
  SplitMix64 rng{seed};
  if (multimode) {
    for (int kx = -8; kx <= 8; ++kx) {
      if (kx == 0) continue;
      for (int ky = -8; ky <= 8; ++ky) {
        const double u1 = rng.uniform(), u2 = rng.uniform(), u3 = rng.uniform();
        modes.push_back(kx);
        modes.push_back(ky);
        modes.push_back(std::sqrt(-2.0 * std::log(1.0 - u1)) * std::cos(2.0 * kPi * u2));
        modes.push_back(2.0 * kPi * u3);
      }
    }
  } else {
    const double ph = 2.0 * kPi * rng.uniform();
    modes = {1.0, 0.0, 1.0, ph};
  }
  const int nmodes = (int)modes.size() / 4;
  const long long nb = (N + 255) / 256;
  // scratch: modes | du[2N] | partial[nb] | sum[1] | scale[1]
  const size_t need = modes.size() + 2 * N + nb + 2;
  int rc = ensure_scratch(x, need);
  if (rc) return rc;
  double *d_modes = x->scratch, *du = d_modes + modes.size(), *part = du + 2 * N;
  double *sum = part + nb, *scale = sum + 1;
  HIPCHK(hipMemcpyAsync(d_modes, modes.data(), modes.size() * sizeof(double),
                        hipMemcpyHostToDevice, x->stream));
  HIPCHK(launch_perturb_field(nx, ny, 0, 0, nx, ny, nmodes, d_modes,
                              amp * x->c.u0, multimode, du, part, x->stream));
  double h_scale = 1.0;
  if (multimode) {
    HIPCHK(launch_sum(part, (int)nb, 1, sum, x->stream));
    double tot = 0.0;
    HIPCHK(hipMemcpyAsync(&tot, sum, sizeof(double), hipMemcpyDeviceToHost, x->stream));
    HIPCHK(hipStreamSynchronize(x->stream));
    const double rms = std::sqrt(tot / (double)N);
    h_scale = rms > 0 ? amp * x->c.u0 / rms : 0.0;
  }
  HIPCHK(hipMemcpyAsync(scale, &h_scale, sizeof(double), hipMemcpyHostToDevice,
                        x->stream));
  if (fp32(x)) {
    FloatView fv;
    int r2 = float_view(x, x->cur, fv);
    if (r2) return r2;
    HIPCHK(launch_perturb_apply<float>(x->d.nqd, nx, ny, du, scale, fv.v, ref_view(x),
                                       x->stream));
    HIPCHK(launch_refresh<float>(x->d.nqd, nx, ny, x->qtab_d, fv.v, ref_view(x), x->stream));
    r2 = float_writeback(x, x->cur, fv);
    if (r2) return r2;
  } else {
    HIPCHK(launch_perturb_apply<double>(x->d.nqd, nx, ny, du, scale, x->buf.half64(x->cur),
                                        ref_view(x), x->stream));
    HIPCHK(launch_refresh<double>(x->d.nqd, nx, ny, x->qtab_d, x->buf.half64(x->cur),
                                  ref_view(x), x->stream));
  }
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

// Allocate the state and upload the Q-node tables (first part of tpl_init).
int prepare_state(tpl_ctx *x) {
  int rc = alloc_state(x);
  if (rc) return rc;
  if (!x->qtab_d) {
    rc = upload_tables(x);
    if (rc) return rc;
  }
  if (fp32(x) && !x->ref) {
    if (hipMalloc(&x->ref, ref_elems(x) * sizeof(float)) != hipSuccess ||
        hipMalloc(&x->sref, sref_elems(x) * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(TPL_ENOMEM, "reference allocation failed");
    }
  }
  x->cur = 0;
  x->ip_odd = 0;
  x->step = 0;
  x->inited = false;
  return TPL_OK;
}

long long pre_steps_of(const tpl_ctx *x) {
  const Derived &d = x->d;
  long long npre = x->c.pre_steps;
  if (npre < 0) npre = (long long)std::ceil(5.0 * std::max(d.l * d.l / d.nu, d.lambda));
  return npre;
}

// Double-buffered FP64 state of one ny-row column (the x-invariant base state).
struct ColumnBuf {
  Buffers B;
  double *mem = nullptr;
  int alloc(int ny, int nqd) {
    B.nXS = 9 * (size_t)ny;
    B.nXP = 25 * (size_t)nqd * ny;
    B.nPSI = (size_t)nqd * ny;
    B.nFLD = (size_t)NF * ny;
    B.esize = 8;
    const size_t tot = 2 * (B.nXS + B.nXP + B.nPSI + B.nFLD);
    if (hipMalloc(&mem, tot * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      mem = nullptr;
      return fail(TPL_ENOMEM, "column allocation failed");
    }
    B.XS = mem;
    B.XP = mem + 2 * B.nXS;
    B.PSI = mem + 2 * (B.nXS + B.nXP);
    B.FLD = mem + 2 * (B.nXS + B.nXP + B.nPSI);
    return TPL_OK;
  }
  void release() {
    if (mem) (void)hipFree(mem);
    mem = nullptr;
  }
};

// Rest state (equilibrium at zero velocity) in half 0 of a column.
int column_rest(tpl_ctx *x, ColumnBuf &C) {
  const Derived &d = x->d;
  const int ny = x->c.ny;
  const RefView none{nullptr, nullptr, nullptr, ny};
  HIPCHK(launch_rest(d.nqd, ny, d.rhoS0, d.rhoP0, x->peq_d, C.B.half64(0), x->stream));
  HIPCHK(launch_refresh<double>(d.nqd, 1, ny, x->qtab_d, C.B.half64(0), none, x->stream));
  return TPL_OK;
}

// Closed-form Hookean laminar state of the column (init_mode 1): U_L from the
// momentum balance of the Oldroyd-B profile with stress diffusion,
// F0 = k^2 U_L [eta_s + eta_pk + G lambda / (1 + lambda D k^2)], eta_s =
// rho_S c_s^2 tau1_S, eta_pk = rho_P c_s^2 tau1_P, D = c_s^2 tau2_P; the
// kernel sets populations, psi and U, the refresh the other fields.
int column_analytic(tpl_ctx *x, ColumnBuf &C) {
  const Derived &d = x->d;
  const int ny = x->c.ny;
  const double k = d.kf, D = kCs2 * d.tau2P;
  const double Dk2 = d.lambda * D * k * k;
  const double eta = d.rhoS0 * kCs2 * d.tau1S + d.rhoP0 * kCs2 * d.tau1P + d.G * d.lambda / (1.0 + Dk2);
  AnalyticColumn a{d.F0 / (k * k * eta), k, d.lambda, Dk2, d.sigma * d.sigma, d.rhoS0, d.rhoP0,
                   d.DQ};
  const RefView none{nullptr, nullptr, nullptr, ny};
  HIPCHK(launch_analytic_column(ny, d.nqd, x->qtab_d, a, C.B.half64(0), x->stream));
  HIPCHK(launch_refresh<double>(d.nqd, 1, ny, x->qtab_d, C.B.half64(0), none, x->stream));
  return TPL_OK;
}

// Copy the converged column to every column of the lattice (half 0).  FP32
// form: the column rounded to FP32 becomes the reference and the stored
// deviations start as the rounding residual.
int seed_from_column(tpl_ctx *x, const StateView &cv) {
  const Derived &d = x->d;
  const int nx = x->c.nx, ny = x->c.ny;
  if (!fp32(x)) {
    HIPCHK(launch_tile(d.nqd, nx, ny, cv, x->buf.half64(0), x->stream));
  } else {
    HIPCHK(launch_make_ref(d.nqd, ny, cv, x->ref, x->stream));
    int rc = build_step_ref(x);
    if (rc) return rc;
    const RefView rv = ref_view(x);
    const StateView32 h0 = x->buf.half<float>(0);
    HIPCHK(launch_tile_dev(9, nx, ny, cv.XS, rv.XS, h0.XS, x->stream));
    HIPCHK(launch_tile_dev(d.nqd, nx, ny, cv.PSI, rv.PSI, h0.PSI, x->stream));
    HIPCHK(launch_tile_fields(nx, ny, cv.FLD, h0.FLD, x->stream));
    if (!bf16(x)) {
      HIPCHK(launch_tile_dev(25 * d.nqd, nx, ny, cv.XP, rv.XP, h0.XP, x->stream));
    } else {  // FP32 deviations of the column, then their BF16 encoding
      const long long N = (long long)nx * ny;
      float *tmp = nullptr;
      if (hipMalloc(&tmp, 25 * (size_t)d.nqd * N * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TPL_ENOMEM, "encode buffer allocation failed");
      }
      hipError_t e = launch_tile_dev(25 * d.nqd, nx, ny, cv.XP, rv.XP, tmp, x->stream);
      if (e == hipSuccess) e = launch_bf16_encode(d.nqd, N, tmp, h0, x->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
      (void)hipFree(tmp);
      if (e != hipSuccess) return fail(TPL_EHIP, std::string("encode: ") + hipGetErrorString(e));
    }
  }
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

// Perturbation and counters (last part of tpl_init).
int finish_init(tpl_ctx *x, uint64_t seed, double perturbation) {
  x->inited = true;
  if (perturbation > 0) {
    const int rc = perturb(x, seed, perturbation);
    if (rc) return rc;
  }
  x->kernel_ms = 0.0;
  x->kernel_launches = 0;
  return TPL_OK;
}

int check_ready(const tpl_ctx *x) {
  if (!x) return fail(TPL_EINVAL, "null context");
  if (!x->inited) return fail(TPL_ESTATE, "context not initialised (call tpl_init)");
  return TPL_OK;
}

// Calls that read or write populations need them in their plain order,
// which in-place streaming holds after an even number of steps.
int check_populations(const tpl_ctx *x) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (x->ip_odd)
    return fail(TPL_ESTATE, "in-place streaming holds the populations in streamed order after "
                            "an odd number of steps: advance one more step first");
  return TPL_OK;
}

struct Key {
  const char *name;
  double Config::*dbl;
  int Config::*in;
  long long Config::*ll;
};

const Key kKeys[] = {
    {"nq", nullptr, &Config::nq, nullptr},
    {"spring", nullptr, &Config::spring, nullptr},
    {"b", &Config::b, nullptr, nullptr},
    {"phi", &Config::phi, nullptr, nullptr},
    {"tau_drag", &Config::tau_drag, nullptr, nullptr},
    {"tau_ratio_p", &Config::tau_ratio_p, nullptr, nullptr},
    {"force_scale", &Config::force_scale, nullptr, nullptr},
    {"lambda", &Config::lambda_set, nullptr, nullptr},
    {"drift_cap", &Config::drift_cap, nullptr, nullptr},
    {"drift_relax", &Config::drift_relax, nullptr, nullptr},
    {"qe_model", nullptr, &Config::qe_model, nullptr},
    {"inplace", nullptr, &Config::inplace, nullptr},
    {"gradients", nullptr, &Config::gradients, nullptr},
    {"spring_shift", nullptr, &Config::spring_shift, nullptr},
    {"precision", nullptr, &Config::precision, nullptr},
    {"pert_modes", nullptr, &Config::pert_modes, nullptr},
    {"pre_steps", nullptr, nullptr, &Config::pre_steps},
    {"qsplit", nullptr, &Config::qsplit, nullptr},
    {"time_kernels", nullptr, &Config::time_kernels, nullptr},
    {"group_x", nullptr, &Config::group_x, nullptr},
    {"group_y", nullptr, &Config::group_y, nullptr},
    {"group_sync", nullptr, &Config::group_sync, nullptr},
    {"autotune", nullptr, &Config::autotune, nullptr},
    {"u0", &Config::u0, nullptr, nullptr},
    {"periods", nullptr, &Config::periods, nullptr},
    {"init_mode", nullptr, &Config::init_mode, nullptr},
    {"diag_every", nullptr, nullptr, &Config::diag_every},
    {"psi_floor", &Config::psi_floor, nullptr, nullptr},
    {"keep_good", nullptr, &Config::keep_good, nullptr},
};

// Knobs that change no state (launch shape, timing, health checks): they may
// be set at any time and do not take part in matching a checkpoint.
bool is_runtime_knob(const char *key) {
  return !std::strcmp(key, "qsplit") || !std::strcmp(key, "time_kernels") ||
         !std::strncmp(key, "group_", 6) || !std::strcmp(key, "autotune") ||
         !std::strcmp(key, "diag_every") || !std::strcmp(key, "psi_floor") ||
         !std::strcmp(key, "keep_good");
}

// Whether two configurations describe the same lattice and scheme (every
// field but the runtime knobs).
bool same_state_config(const Config &a, const Config &b) {
  if (a.nx != b.nx || a.ny != b.ny || a.Re != b.Re || a.Wi != b.Wi || a.beta != b.beta)
    return false;
  for (const Key &k : kKeys) {
    if (is_runtime_knob(k.name)) continue;
    if (k.dbl && !(a.*(k.dbl) == b.*(k.dbl))) return false;
    if (k.in && a.*(k.in) != b.*(k.in)) return false;
    if (k.ll && a.*(k.ll) != b.*(k.ll)) return false;
  }
  return true;
}

}  // namespace

int learned_begin(tpl_ctx *x);  // attached correction: working arrays, gate opened
int learned_source(tpl_ctx *x, int tag);  // its source for the current state (below)

namespace {

// Device doubles that the diagnostics need as working memory: the
// reduction's partials and result, then the amplitude's row sums and total.
size_t diag_scratch_doubles(int ny) {
  return (size_t)kDiagBlocks * kDiagComp + kDiagComp + (size_t)ny + 1;
}

// A(n) with device working memory w of at least ny + 1 doubles.
double amplitude_with(tpl_ctx *x, double *w) {
  const int nx = x->c.nx, ny = x->c.ny;
  if (launch_amplitude_rows(nx, ny, x->buf.half64(x->cur).FLD, w, x->stream) != hipSuccess ||
      launch_sum(w, ny, 1, w + ny, x->stream) != hipSuccess) {
    fail(TPL_EHIP, "amplitude kernels failed");
    return NAN;
  }
  double tot = 0.0;
  if (hipMemcpyAsync(&tot, w + ny, sizeof(double), hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
      hipStreamSynchronize(x->stream) != hipSuccess) {
    fail(TPL_EHIP, "amplitude copy failed");
    return NAN;
  }
  return std::sqrt(tot / ((double)nx * ny)) / x->c.u0;
}

// tpl_diagnostics with device working memory w of diag_scratch_doubles(ny)
// doubles (the BF16 form also decodes its populations into a buffer of its
// own).
int diagnostics_with(tpl_ctx *x, double *w, tpl_diag *out) {
  int rc;
  int nb = 0;
  FloatView fv;
  if (fp32(x) && (rc = float_view(x, x->cur, fv))) return rc;
  if (fp32(x))
    HIPCHK(launch_diag<float>(x->c.nx, x->c.ny, x->d.nqd, x->qtab_d, fv.v, ref_view(x), w, &nb,
                              x->stream));
  else
    HIPCHK(launch_diag<double>(x->c.nx, x->c.ny, x->d.nqd, x->qtab_d, x->buf.half64(x->cur),
                               ref_view(x), w, &nb, x->stream));
  double *res = w + (size_t)kDiagBlocks * kDiagComp;
  HIPCHK(launch_diag_final(w, nb, res, x->stream));
  double h[kDiagComp];
  HIPCHK(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  const double amp = amplitude_with(x, res + kDiagComp);
  out->step = (double)x->step;
  out->mass_S = h[0];
  out->mass_P = h[1];
  out->mom_x = h[2];
  out->mom_y = h[3];
  out->amplitude = amp;
  out->enstrophy = h[4];
  out->qrms = h[6] > 0 ? std::sqrt(h[5] / h[6]) / x->d.R : 0.0;
  out->min_psi = h[7];
  return TPL_OK;
}

// Working memory of tpl_diagnostics_noalloc, one copy per GPU for the
// life of the process: the diagnostics' partial sums and result and the
// amplitude's row sums, for lattices of at most kNoAllocRows rows.  Every
// call on a GPU reuses it (each call writes every value it later reads, so
// nothing needs clearing); calls that overlap on one GPU race.  Host code
// uses only its device address from noalloc_scratch(), never the name.
constexpr int kNoAllocRows = 1 << 16;
constexpr size_t kNoAllocDoubles = (size_t)kDiagBlocks * kDiagComp + kDiagComp + kNoAllocRows + 1;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of scratch (looked up once per
// device, with that device current).
int noalloc_scratch(double **p) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TPL_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(TPL_EHIP, std::string("hipGetSymbolAddress of the static working memory: ") +
                                hipGetErrorString(e));
    g_noalloc_ptr[dev] = static_cast<double *>(ptr);
  }
  *p = g_noalloc_ptr[dev];
  return TPL_OK;
}

}  // namespace

namespace {

// n steps of the current launch shape (a new source from an attached
// correction before each step).
int advance(tpl_ctx *x, int64_t n) {
  int rc;
  if (x->mlp) {
    // every step: the correction's source from the current state, then the
    // step; the drift gate is checked on the device, and the host learns once
    // at the end how many steps ran
    rc = learned_begin(x);
    if (rc) return rc;
    const int cur0 = x->cur;
    for (int64_t i = 0; i < n; ++i) {
      rc = learned_source(x, (int)(i + 1));
      if (!rc)
        rc = run_steps(x, x->buf, x->c.nx, x->c.ny, &x->cur, 1, x->c.time_kernels != 0,
                       x->c.qsplit);
      if (rc) return rc;
    }
    int gate = 0;
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&gate, x->gate_d, sizeof gate, hipMemcpyDeviceToHost, x->stream));
    HIPCHK(hipMemcpyAsync(&bits, x->drift_d, sizeof bits, hipMemcpyDeviceToHost, x->stream));
    HIPCHK(hipStreamSynchronize(x->stream));
    double dmax;
    std::memcpy(&dmax, &bits, sizeof dmax);
    x->last_drift = dmax / x->c.u0;
    const int64_t ran = gate ? (int64_t)gate - 1 : n;
    x->cur = cur0 ^ (int)(ran & 1);
    x->step += ran;
    if (gate) {
      char msg[200];
      snprintf(msg, sizeof msg, "correction rejected before step %lld: max |F|/rho reached "
               "%.3e u0, above the drift bound %.3e u0", x->step + 1, x->last_drift,
               x->drift_bound);
      return fail(TPL_EREJECTED, msg);
    }
    return TPL_OK;
  }
  if (n == 0) return TPL_OK;
  rc = run_steps(x, x->buf, x->c.nx, x->c.ny, &x->cur, n, x->c.time_kernels != 0, x->c.qsplit);
  if (rc) return rc;
  x->step += n;
  return TPL_OK;
}

// Health of the current state (non-finite U or psi, min and max psi) into
// out[3]; partial and out are device arrays (3 kHealthBlocks and 3 doubles).
int health(tpl_ctx *x, double *partial, double *dout, hipStream_t s, double out[3]) {
  if (fp32(x))
    HIPCHK(launch_health<float>(x->c.nx, x->c.ny, x->d.nqd, x->buf.half<float>(x->cur),
                                ref_view(x), partial, dout, s));
  else
    HIPCHK(launch_health<double>(x->c.nx, x->c.ny, x->d.nqd, x->buf.half64(x->cur),
                                 ref_view(x), partial, dout, s));
  if (out) {
    HIPCHK(hipMemcpyAsync(out, dout, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return TPL_OK;
}

// TPL_EUNSTABLE (with the step and the cause) if the state holds NaN/Inf or
// psi below -psi_floor max psi.
int judge_health(const tpl_ctx *x, const double h[3]) {
  char msg[200];
  if (h[0] != 0.0) {
    snprintf(msg, sizeof msg, "state not finite after step %lld (%.0f non-finite values of U "
             "and psi)", x->step, h[0]);
    return fail(TPL_EUNSTABLE, msg);
  }
  if (h[1] < -x->c.psi_floor * h[2]) {
    snprintf(msg, sizeof msg, "polymer density negative after step %lld: min psi %.3e < "
             "-%.3g max psi (max %.3e)", x->step, h[1], x->c.psi_floor, h[2]);
    return fail(TPL_EUNSTABLE, msg);
  }
  return TPL_OK;
}

int check_health(tpl_ctx *x) {
  int rc = ensure_scratch(x, 3 * (size_t)kHealthBlocks + 3);
  if (rc) return rc;
  double h[3];
  rc = health(x, x->scratch, x->scratch + 3 * (size_t)kHealthBlocks, x->stream, h);
  if (rc) return rc;
  return judge_health(x, h);
}

// The parts of state half h that a step reads (populations: the single array
// when streamed in place; lagged psi; per-node fields; stored moments):
// device addresses and byte counts.
void half_parts(const tpl_ctx *x, int h, char *ptr[5], size_t nb[5]) {
  const Buffers &B = x->buf;
  const size_t hp = B.pop_half(h);
  ptr[0] = static_cast<char *>(B.XS) + hp * B.nXS * B.esize;
  ptr[1] = static_cast<char *>(B.XP) + hp * B.nXP * B.xsize;
  ptr[2] = static_cast<char *>(B.PSI) + (size_t)h * B.nPSI * B.esize;
  ptr[3] = reinterpret_cast<char *>(B.FLD + (size_t)h * B.nFLD);
  ptr[4] = B.MOM ? reinterpret_cast<char *>(B.MOM + (size_t)h * B.nMOM) : nullptr;
  nb[0] = B.nXS * B.esize;
  nb[1] = B.nXP * B.xsize;
  nb[2] = B.nPSI * B.esize;
  nb[3] = B.nFLD * sizeof(double);
  nb[4] = B.MOM ? B.nMOM * sizeof(float) : 0;
}

// keep_good: copy the current state (one half) into the context's spare
// array, allocated on first use, and remember its step.
int keep_state(tpl_ctx *x) {
  char *ptr[5];
  size_t nb[5], total = 0;
  half_parts(x, x->cur, ptr, nb);
  for (size_t b : nb) total += b;
  if (!x->good_d) {
    if (hipMalloc(&x->good_d, total) != hipSuccess) {
      (void)hipGetLastError();
      x->good_d = nullptr;
      return fail(TPL_ENOMEM, "keep_good: no device memory for a copy of the state (" +
                                  std::to_string(total) + " bytes)");
    }
    x->good_bytes = total;
  }
  size_t off = 0;
  for (int i = 0; i < 5; ++i) {
    if (!nb[i]) continue;
    HIPCHK(hipMemcpyAsync(x->good_d + off, ptr[i], nb[i], hipMemcpyDeviceToDevice, x->stream));
    off += nb[i];
  }
  x->good_step = x->step;
  x->good_cur = x->cur;
  x->good_ip_odd = x->ip_odd;
  return TPL_OK;
}

// keep_good: put the kept state back (into the half it came from).
int restore_state(tpl_ctx *x) {
  char *ptr[5];
  size_t nb[5], off = 0;
  half_parts(x, x->good_cur, ptr, nb);
  for (int i = 0; i < 5; ++i) {
    if (!nb[i]) continue;
    HIPCHK(hipMemcpyAsync(ptr[i], x->good_d + off, nb[i], hipMemcpyDeviceToDevice, x->stream));
    off += nb[i];
  }
  HIPCHK(hipStreamSynchronize(x->stream));
  x->step = x->good_step;
  x->cur = x->good_cur;
  x->ip_odd = x->good_ip_odd;
  return TPL_OK;
}

}  // namespace

// ===========================================================================
// C ABI
extern "C" {

const char *tpl_last_error(void) { return g_err.c_str(); }

tpl_ctx *tpl_create(int nx, int ny, double Re, double Wi, double beta,
                    tpl_forcing forcing) {
  g_err.clear();
  tpl_ctx *x = new (std::nothrow) tpl_ctx();
  if (!x) {
    fail(TPL_ENOMEM, "host allocation failed");
    return nullptr;
  }
  x->c.nx = nx;
  x->c.ny = ny;
  x->c.Re = Re;
  x->c.Wi = Wi;
  x->c.beta = beta;
  x->c.periods = forcing.periods;
  x->c.u0 = forcing.u0;
  if (derive(x->c, x->d) != TPL_OK) {
    delete x;
    return nullptr;
  }
  return x;
}

int tpl_set_param(tpl_ctx *x, const char *key, double v) {
  if (!x || !key) return fail(TPL_EINVAL, "null argument");
  // launch, timing and health knobs change no state and may be set at any time
  const bool runtime_knob = is_runtime_knob(key);
  if (x->inited && !runtime_knob)
    return fail(TPL_ESTATE, "parameters are fixed after tpl_init");
  Config c = x->c;
  bool found = false;
  for (const Key &k : kKeys) {
    if (std::strcmp(k.name, key) != 0) continue;
    found = true;
    if (k.dbl) c.*(k.dbl) = v;
    if (k.in) {
      if (v != std::floor(v)) return fail(TPL_EINVAL, std::string(key) + " must be an integer");
      c.*(k.in) = (int)v;
    }
    if (k.ll) {
      if (v != std::floor(v)) return fail(TPL_EINVAL, std::string(key) + " must be an integer");
      c.*(k.ll) = (long long)v;
    }
  }
  if (!found) return fail(TPL_EINVAL, std::string("unknown parameter ") + key);
  if (c.spring != 0 && c.spring != 1) return fail(TPL_EINVAL, "spring must be 0 or 1");
  if (c.precision != TPL_FP64 && c.precision != TPL_FP32 && c.precision != TPL_BF16)
    return fail(TPL_EINVAL, "precision must be TPL_FP64, TPL_FP32 or TPL_BF16");
  if (c.qsplit < 0 || c.qsplit > 8) return fail(TPL_EINVAL, "qsplit must be in [0,8]");
  if (c.group_x < 1 || c.group_y < 1 || c.group_x * c.group_y > 8)
    return fail(TPL_EINVAL, "group_x * group_y must be in [1,8]");
  if (!(c.drift_cap >= 0)) return fail(TPL_EINVAL, "drift_cap must be >= 0");
  if (!(c.drift_relax >= 0)) return fail(TPL_EINVAL, "drift_relax must be >= 0");
  if (c.diag_every < 0) return fail(TPL_EINVAL, "diag_every must be >= 0");
  if (c.init_mode != 0 && c.init_mode != 1) return fail(TPL_EINVAL, "init_mode must be 0 or 1");
  if (!(c.psi_floor >= 0)) return fail(TPL_EINVAL, "psi_floor must be >= 0");
  if (c.keep_good != 0 && c.keep_good != 1) return fail(TPL_EINVAL, "keep_good must be 0 or 1");
  if (runtime_knob) {
    x->c = c;
    return TPL_OK;
  }
  Derived d;
  int rc = derive(c, d);
  if (rc) return rc;
  x->c = c;
  x->d = std::move(d);
  return TPL_OK;
}

int tpl_query(const tpl_ctx *x, const char *key, double *out) {
  if (!x || !key || !out) return fail(TPL_EINVAL, "null argument");
  for (const Key &k : kKeys)
    if (std::strcmp(k.name, key) == 0) {
      *out = k.dbl ? x->c.*(k.dbl) : k.in ? (double)(x->c.*(k.in)) : (double)(x->c.*(k.ll));
      return TPL_OK;
    }
  const Derived &d = x->d;
  const double N = (double)x->c.nx * x->c.ny;
  const double es = x->c.precision == TPL_FP64 ? 8.0 : 4.0;
  const double xs = x->c.precision == TPL_FP64 ? 8.0 : x->c.precision == TPL_FP32 ? 4.0 : 2.0;
  const double ms = 0.0;
  const double xq = (bf16(x) ? 26.0 : 25.0) * xs;  // XP bytes per (r, Q)
  const double pc = x->c.inplace ? 1.0 : 2.0;  // population arrays
  struct {
    const char *n;
    double v;
  } vals[] = {
      {"nx", (double)x->c.nx}, {"ny", (double)x->c.ny}, {"nqd", (double)d.nqd},
      {"Re", x->c.Re}, {"Wi", x->c.Wi}, {"beta", x->c.beta},
      {"kf", d.kf}, {"l", d.l}, {"nu", d.nu}, {"nuS", d.nuS}, {"G", d.G},
      {"tau1S", d.tau1S}, {"tau2S", d.tau2S}, {"tau1P", d.tau1P},
      {"tau2P", d.tau2P}, {"lambda_eff", d.lambda}, {"sigma", d.sigma},
      {"R", d.R}, {"DQ", d.DQ}, {"F0", d.F0}, {"kappa", d.kappa},
      {"meq", d.meq}, {"Sc", d.Sc}, {"rhoS0", d.rhoS0}, {"rhoP0", d.rhoP0},
      {"step", (double)x->step},
      {"bytes_XS", pc * es * 9 * N}, {"bytes_XP", pc * xq * d.nqd * N},
      {"bytes_PSI", 2.0 * es * d.nqd * N}, {"bytes_FLD", 16.0 * NF * N},
      {"bytes_MOM", 2.0 * ms * d.nqd * N},
      {"bytes_state",
       N * (pc * (es * 9 + xq * d.nqd) + 2.0 * (es * d.nqd + ms * d.nqd + 8.0 * NF))},
      // algorithmic HBM bytes of one step: populations read + written,
      // lagged psi written + read, lagged per-node fields written + read
      // (BF16 form: 26 16-bit values per (r, Q)-node); same-step
      // gradients add a second read of the polymer populations, psi written
      // and read, the solvent read and 17 FP64 field values per node; the
      // shifted spring term a second read of psi and its Q-sum written (the
      // step reads the sum where it would read M); both together: the M pass
      // is the spring-sum pass, and the velocity pass reads the sum (13
      // values per node instead of 17, psi read once less)
      {"bytes_per_step",
       N * (2.0 * es * (9 + d.nqd) + 2.0 * (xq + ms) * d.nqd + 8.0 * 2.0 * NF) +
           (x->c.gradients ? N * (xq * d.nqd + 9.0 * es +
                                  (x->c.spring_shift ? es * d.nqd + 104.0
                                                     : 2.0 * es * d.nqd + 136.0))
                           : 0.0) +
           (x->c.spring_shift ? N * (es * d.nqd + 16.0) : 0.0)},
      {"kernel_ms", x->kernel_ms}, {"kernel_launches", (double)x->kernel_launches},
      {"qsplit_used", (double)x->qs_used},
      {"group_x_used", (double)(x->wg_used & 255)},
      {"group_y_used", (double)((x->wg_used >> 8) & 255)},
      {"group_sync_used", (double)((x->wg_used >> 16) & 1)},
      {"tune_ms", x->tune_ms},
      {"inplace_odd", (double)x->ip_odd},
  };
  for (auto &kv : vals)
    if (std::strcmp(kv.n, key) == 0) {
      *out = kv.v;
      return TPL_OK;
    }
  return fail(TPL_EINVAL, std::string("unknown query key ") + key);
}

int tpl_set_stream(tpl_ctx *x, void *s) {
  if (!x) return fail(TPL_EINVAL, "null context");
  x->stream = (hipStream_t)s;
  return TPL_OK;
}

int tpl_adopt_buffers(tpl_ctx *x, void *const *dptrs, const size_t *bytes, int n) {
  if (!x || !dptrs || !bytes) return fail(TPL_EINVAL, "null argument");
  if (x->inited || x->buf.XS) return fail(TPL_ESTATE, "buffers already allocated");
  if (n != 4) return fail(TPL_EINVAL, "expected 4 buffers (XS, XP, PSI, FLD)");
  Buffers B;
  B.nXS = state_elems(x, 0);
  B.nXP = state_elems(x, 1);
  B.nPSI = state_elems(x, 2);
  B.nFLD = state_elems(x, 3);
  B.esize = elem_size(x);
  B.xsize = xp_size(x);
  B.inplace = x->c.inplace != 0;
  const size_t pc = B.pop_copies();
  const size_t need[4] = {pc * B.nXS * B.esize, pc * B.nXP * B.xsize, 2 * B.nPSI * B.esize,
                          2 * B.nFLD * sizeof(double)};
  for (int i = 0; i < 4; ++i) {
    if (!dptrs[i] || bytes[i] < need[i])
      return fail(TPL_EINVAL, "adopted buffer " + std::to_string(i) + " too small");
    if (((uintptr_t)dptrs[i]) & 255) return fail(TPL_EINVAL, "adopted buffer not 256-byte aligned");
  }
  B.XS = dptrs[0];
  B.XP = dptrs[1];
  B.PSI = dptrs[2];
  B.FLD = static_cast<double *>(dptrs[3]);
  x->buf = B;
  x->owned = false;
  return TPL_OK;
}

int tpl_init(tpl_ctx *x, uint64_t seed, double perturbation) {
  if (!x) return fail(TPL_EINVAL, "null context");
  if (!(perturbation >= 0)) return fail(TPL_EINVAL, "perturbation must be >= 0");
  if (x->c.init_mode == 1 && (x->c.spring != 1 || x->c.qe_model != 1 || !(x->d.G > 0.0)))
    return fail(TPL_EINVAL, "init_mode 1 (closed-form state) needs Hookean springs (spring 1), "
                            "qe_model 1 and Wi > 0");
  int rc = prepare_state(x);
  if (rc) return rc;
  const Derived &d = x->d;
  const int ny = x->c.ny;
  // base state on one FP64 column, then copied to every column
  ColumnBuf C;
  rc = C.alloc(ny, d.nqd);
  if (rc) return rc;
  int ccur = 0;
  if (x->c.init_mode == 1) {
    rc = column_analytic(x, C);
  } else {
    rc = column_rest(x, C);
    if (!rc) rc = run_steps(x, C.B, 1, ny, &ccur, pre_steps_of(x), false, kColumnQs);
  }
  if (!rc) rc = seed_from_column(x, C.B.half64(ccur));
  C.release();
  if (rc) return rc;
  return finish_init(x, seed, perturbation);
}

int tpl_step(tpl_ctx *x, int64_t n) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (n < 0) return fail(TPL_EINVAL, "n must be >= 0");
  if (!x->tuned && x->c.autotune && n > 0 && !x->buf.inplace) {
    rc = tune_groups(x);
    if (rc) return rc;
  }
  if (!x->tuned && x->c.autotune && x->buf.inplace && !x->mlp && n >= kTuneSteps) {
    long long done = 0;
    rc = tune_groups_inplace(x, &done);
    x->step += done;
    n -= done;
    if (rc) return rc;
  }
  {
    const StepParams p = make_step_params(x, x->c.nx, x->c.ny, x->c.qsplit);
    x->qs_used = p.qs;
    x->wg_used = p.wg;
  }
  // advance in chunks of diag_every steps (all n if 0), checking the state's
  // health after each chunk; a failed check stops the call there (and with
  // keep_good puts back the state of the last passed check, or of the call's
  // start)
  const bool keep = x->c.keep_good != 0;
  if (keep && (rc = keep_state(x))) return rc;
  int64_t done = 0;
  do {
    const int64_t chunk = x->c.diag_every > 0 ? std::min<int64_t>(x->c.diag_every, n - done)
                                              : n - done;
    rc = advance(x, chunk);
    if (rc) return rc;
    done += chunk;
    rc = check_health(x);
    if (rc == TPL_EUNSTABLE && keep) {
      const std::string why = g_err;
      const int rr = restore_state(x);
      if (rr) return rr;
      return fail(TPL_EUNSTABLE, why + "; state restored to step " + std::to_string(x->step));
    }
    if (rc) return rc;
    if (keep && done < n && (rc = keep_state(x))) return rc;
  } while (done < n);
  return TPL_OK;
}

int tpl_moments_device(tpl_ctx *x, void *dptr, size_t len) {
  int rc = check_ready(x);
  if (rc) return rc;
  const long long N = (long long)x->c.nx * x->c.ny;
  if (!dptr || len < (size_t)TPL_NFIELDS * N) return fail(TPL_EINVAL, "output too small");
  const double s2 = x->d.sigma * x->d.sigma;
  const double G = x->d.G, mref = x->d.rhoP0 * x->d.meq;
  if (fp32(x))
    HIPCHK(launch_observables<float>(x->d.nqd, x->c.nx, x->c.ny, x->qtab_d, 1.0 / s2, G, mref,
                                     x->buf.half<float>(x->cur), ref_view(x), (double *)dptr,
                                     x->stream));
  else
    HIPCHK(launch_observables<double>(x->d.nqd, x->c.nx, x->c.ny, x->qtab_d, 1.0 / s2, G, mref,
                                      x->buf.half64(x->cur), ref_view(x), (double *)dptr,
                                      x->stream));
  return TPL_OK;
}

int tpl_moments(tpl_ctx *x, double *out, size_t len) {
  int rc = check_ready(x);
  if (rc) return rc;
  const long long N = (long long)x->c.nx * x->c.ny;
  if (!out || len < (size_t)TPL_NFIELDS * N) return fail(TPL_EINVAL, "output too small");
  rc = ensure_scratch(x, (size_t)TPL_NFIELDS * N);
  if (rc) return rc;
  rc = tpl_moments_device(x, x->scratch, (size_t)TPL_NFIELDS * N);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(out, x->scratch, sizeof(double) * TPL_NFIELDS * N,
                        hipMemcpyDeviceToHost, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

double tpl_perturbation_amplitude(tpl_ctx *x) {
  if (check_ready(x)) return NAN;
  if (ensure_scratch(x, (size_t)x->c.ny + 1)) return NAN;
  return amplitude_with(x, x->scratch);
}

int tpl_diagnostics(tpl_ctx *x, tpl_diag *out) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (!out) return fail(TPL_EINVAL, "null output");
  rc = ensure_scratch(x, diag_scratch_doubles(x->c.ny));
  if (rc) return rc;
  return diagnostics_with(x, x->scratch, out);
}

int tpl_diagnostics_noalloc(tpl_ctx *x, tpl_diag *out) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (!out) return fail(TPL_EINVAL, "null output");
  if (bf16(x))
    return fail(TPL_EINVAL, "tpl_diagnostics_noalloc: the BF16 form decodes into a buffer "
                            "it would have to allocate");
  if (x->c.ny > kNoAllocRows)
    return fail(TPL_EINVAL, "tpl_diagnostics_noalloc: ny = " + std::to_string(x->c.ny) +
                                " exceeds the static working memory (at most " +
                                std::to_string(kNoAllocRows) + " rows)");
  double *w = nullptr;
  rc = noalloc_scratch(&w);
  if (rc) return rc;
  return diagnostics_with(x, w, out);
}

int tpl_get_window(tpl_ctx *x, int x0, int y0, int w, int h, double *XS,
                   double *XP, double *psi, double *U) {
  int rc = check_populations(x);
  if (rc) return rc;
  if (w < 1 || h < 1) return fail(TPL_EINVAL, "window must be non-empty");
  const size_t nqd = x->d.nqd, wh = (size_t)w * h;
  const size_t planes = 9 + 26 * nqd + 2;
  rc = ensure_scratch(x, planes * wh);
  if (rc) return rc;
  FloatView fv;
  if (fp32(x) && (rc = float_view(x, x->cur, fv))) return rc;
  if (fp32(x))
    HIPCHK(launch_window<float>(x->c.nx, x->c.ny, (int)nqd, x0, y0, w, h, fv.v, ref_view(x),
                                x->scratch, x->stream));
  else
    HIPCHK(launch_window<double>(x->c.nx, x->c.ny, (int)nqd, x0, y0, w, h,
                                 x->buf.half64(x->cur), ref_view(x), x->scratch, x->stream));
  const double *s = x->scratch;
  auto cp = [&](double *dst, size_t off, size_t n) -> int {
    if (dst)
      HIPCHK(hipMemcpyAsync(dst, s + off * wh, n * wh * sizeof(double),
                            hipMemcpyDeviceToHost, x->stream));
    return TPL_OK;
  };
  if ((rc = cp(XS, 0, 9)) || (rc = cp(XP, 9, 25 * nqd)) || (rc = cp(psi, 9 + 25 * nqd, nqd)) ||
      (rc = cp(U, 9 + 26 * nqd, 2)))
    return rc;
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

// One stored array <-> full FP64 host values (planes of N), through scratch
// for the FP32 form.
static int array_to_host(tpl_ctx *x, const void *src, int planes, const float *ref,
                         double *host) {
  const size_t N = (size_t)x->c.nx * x->c.ny;
  if (!fp32(x)) {
    HIPCHK(hipMemcpyAsync(host, src, planes * N * 8, hipMemcpyDeviceToHost, x->stream));
    return TPL_OK;
  }
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(planes, (64u << 20) / (8 * N)));
  int rc = ensure_scratch(x, (size_t)chunk * N);
  if (rc) return rc;
  for (int p0 = 0; p0 < planes; p0 += chunk) {
    const int np = std::min(chunk, planes - p0);
    HIPCHK(launch_to_f64(x->c.nx, x->c.ny, np, static_cast<const float *>(src) + (size_t)p0 * N,
                         ref + (size_t)p0 * x->c.ny, x->scratch, x->stream));
    HIPCHK(hipMemcpyAsync(host + (size_t)p0 * N, x->scratch, np * N * 8, hipMemcpyDeviceToHost,
                          x->stream));
    HIPCHK(hipStreamSynchronize(x->stream));
  }
  return TPL_OK;
}
static int array_from_host(tpl_ctx *x, void *dst, int planes, const float *ref,
                           const double *host) {
  const size_t N = (size_t)x->c.nx * x->c.ny;
  if (!fp32(x)) {
    HIPCHK(hipMemcpyAsync(dst, host, planes * N * 8, hipMemcpyHostToDevice, x->stream));
    return TPL_OK;
  }
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(planes, (64u << 20) / (8 * N)));
  int rc = ensure_scratch(x, (size_t)chunk * N);
  if (rc) return rc;
  for (int p0 = 0; p0 < planes; p0 += chunk) {
    const int np = std::min(chunk, planes - p0);
    HIPCHK(hipMemcpyAsync(x->scratch, host + (size_t)p0 * N, np * N * 8, hipMemcpyHostToDevice,
                          x->stream));
    HIPCHK(launch_from_f64(x->c.nx, x->c.ny, np, x->scratch, ref + (size_t)p0 * x->c.ny,
                           static_cast<float *>(dst) + (size_t)p0 * N, x->stream));
    HIPCHK(hipStreamSynchronize(x->stream));
  }
  return TPL_OK;
}

int tpl_get_state(tpl_ctx *x, double *XS, double *XP, double *psi, double *U) {
  int rc = (XS || XP) ? check_populations(x) : check_ready(x);
  if (rc) return rc;
  const size_t N = (size_t)x->c.nx * x->c.ny;
  const int nqd = x->d.nqd, cur = x->cur;
  const RefView r = ref_view(x);
  const size_t es = x->buf.esize, hp = x->buf.pop_half(cur);
  const char *XSd = static_cast<const char *>(x->buf.XS) + hp * x->buf.nXS * es;
  const char *XPd = static_cast<const char *>(x->buf.XP) + hp * x->buf.nXP * x->buf.xsize;
  const char *PSd = static_cast<const char *>(x->buf.PSI) + cur * x->buf.nPSI * es;
  FloatView fv;
  if (XP && bf16(x)) {
    if ((rc = float_view(x, cur, fv))) return rc;
    XPd = reinterpret_cast<const char *>(fv.v.XP);
  }
  if (XS && (rc = array_to_host(x, XSd, 9, r.XS, XS))) return rc;
  if (XP && (rc = array_to_host(x, XPd, 25 * nqd, r.XP, XP))) return rc;
  if (psi && (rc = array_to_host(x, PSd, nqd, r.PSI, psi))) return rc;
  if (U)
    HIPCHK(hipMemcpyAsync(U, x->buf.half64(cur).FLD + (size_t)F_UX * N, 2 * N * 8,
                          hipMemcpyDeviceToHost, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

int tpl_set_state(tpl_ctx *x, const double *XS, const double *XP,
                  const double *psi, const double *U) {
  int rc = check_populations(x);  // the node fields are refreshed from the populations
  if (rc) return rc;
  const size_t N = (size_t)x->c.nx * x->c.ny;
  const int nqd = x->d.nqd, cur = x->cur;
  const RefView r = ref_view(x);
  const size_t es = x->buf.esize, hp = x->buf.pop_half(cur);
  char *XSd = static_cast<char *>(x->buf.XS) + hp * x->buf.nXS * es;
  char *XPd = static_cast<char *>(x->buf.XP) + hp * x->buf.nXP * x->buf.xsize;
  char *PSd = static_cast<char *>(x->buf.PSI) + cur * x->buf.nPSI * es;
  if (XS && (rc = array_from_host(x, XSd, 9, r.XS, XS))) return rc;
  if (bf16(x) && XP) {
    FloatView fv;
    if ((rc = float_view(x, cur, fv))) return rc;
    if (XP && (rc = array_from_host(x, fv.tmp, 25 * nqd, r.XP, XP))) return rc;
    if (psi && (rc = array_from_host(x, PSd, nqd, r.PSI, psi))) return rc;
    if ((rc = float_writeback(x, cur, fv))) return rc;
  } else {
    if (XP && (rc = array_from_host(x, XPd, 25 * nqd, r.XP, XP))) return rc;
    if (psi && (rc = array_from_host(x, PSd, nqd, r.PSI, psi))) return rc;
  }
  if (U)
    HIPCHK(hipMemcpyAsync(x->buf.half64(cur).FLD + (size_t)F_UX * N, U, 2 * N * 8,
                          hipMemcpyHostToDevice, x->stream));
  FloatView fr;
  if (fp32(x) && (rc = float_view(x, cur, fr))) return rc;
  if (fp32(x))
    HIPCHK(launch_refresh<float>(nqd, x->c.nx, x->c.ny, x->qtab_d, fr.v, r, x->stream));
  else
    HIPCHK(launch_refresh<double>(nqd, x->c.nx, x->c.ny, x->qtab_d, x->buf.half64(cur), r,
                                  x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

int tpl_get_populations(tpl_ctx *x, int species, void *host, size_t bytes) {
  int rc = check_ready(x);
  if (rc) return rc;
  const size_t N = (size_t)x->c.nx * x->c.ny;
  const size_t need = (species == TPL_SOLVENT ? 9 : 25 * (size_t)x->d.nqd) * N * 8;
  if (species != TPL_SOLVENT && species != TPL_POLYMER) return fail(TPL_EINVAL, "bad species");
  if (!host || bytes != need) return fail(TPL_EINVAL, "buffer size mismatch");
  return species == TPL_SOLVENT ? tpl_get_state(x, (double *)host, nullptr, nullptr, nullptr)
                                : tpl_get_state(x, nullptr, (double *)host, nullptr, nullptr);
}

int tpl_set_populations(tpl_ctx *x, int species, const void *host, size_t bytes) {
  int rc = check_ready(x);
  if (rc) return rc;
  const size_t N = (size_t)x->c.nx * x->c.ny;
  const size_t need = (species == TPL_SOLVENT ? 9 : 25 * (size_t)x->d.nqd) * N * 8;
  if (species != TPL_SOLVENT && species != TPL_POLYMER) return fail(TPL_EINVAL, "bad species");
  if (!host || bytes != need) return fail(TPL_EINVAL, "buffer size mismatch");
  return species == TPL_SOLVENT
             ? tpl_set_state(x, (const double *)host, nullptr, nullptr, nullptr)
             : tpl_set_state(x, nullptr, (const double *)host, nullptr, nullptr);
}

static const char kMagic[8] = {'T', 'P', 'L', 'C', 'K', 'P', 'T', '1'};

// Checkpoint layout: magic, Config, step, then each stored array of the
// current half in storage precision (XS, XP, PSI, FLD) and, for the FP32
// form, the FP64 reference.
int tpl_save(tpl_ctx *x, const char *path) {
  int rc = check_populations(x);
  if (rc) return rc;
  if (!path) return fail(TPL_EINVAL, "null path");
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(TPL_EINVAL, std::string("cannot open ") + path);
  HIPCHK(hipStreamSynchronize(x->stream));
  const size_t es = x->buf.esize, xs = x->buf.xsize, cur = x->cur, hp = x->buf.pop_half(x->cur);
  const void *src[6] = {static_cast<const char *>(x->buf.XS) + hp * x->buf.nXS * es,
                        static_cast<const char *>(x->buf.XP) + hp * x->buf.nXP * xs,
                        static_cast<const char *>(x->buf.PSI) + cur * x->buf.nPSI * es,
                        x->buf.FLD + cur * x->buf.nFLD, x->ref,
                        x->buf.MOM ? x->buf.MOM + cur * x->buf.nMOM : nullptr};
  const size_t nb[6] = {x->buf.nXS * es, x->buf.nXP * xs, x->buf.nPSI * es, x->buf.nFLD * 8,
                        x->ref ? ref_elems(x) * sizeof(float) : 0, x->buf.nMOM * sizeof(float)};
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&x->c, sizeof(Config), 1, f) == 1 &&
            std::fwrite(&x->step, sizeof x->step, 1, f) == 1;
  std::vector<char> h;
  for (int i = 0; i < 6 && ok; ++i) {
    if (!nb[i]) continue;
    h.resize(nb[i]);
    if (hipMemcpy(h.data(), src[i], nb[i], hipMemcpyDeviceToHost) != hipSuccess) {
      std::fclose(f);
      return fail(TPL_EHIP, "checkpoint copy failed");
    }
    ok = std::fwrite(h.data(), 1, nb[i], f) == nb[i];
  }
  ok = (std::fclose(f) == 0) && ok;
  return ok ? TPL_OK : fail(TPL_EINVAL, "checkpoint write failed");
}

int tpl_load(tpl_ctx *x, const char *path) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (!path) return fail(TPL_EINVAL, "null path");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(TPL_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  Config c;
  long long step = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
            std::fread(&c, sizeof c, 1, f) == 1 && std::fread(&step, sizeof step, 1, f) == 1;
  if (!ok || !same_state_config(c, x->c)) {
    std::fclose(f);
    return fail(TPL_EINVAL, "checkpoint does not match this context");
  }
  const size_t es = x->buf.esize, xs = x->buf.xsize, cur = x->cur, hp = x->buf.pop_half(x->cur);
  void *dst[6] = {static_cast<char *>(x->buf.XS) + hp * x->buf.nXS * es,
                  static_cast<char *>(x->buf.XP) + hp * x->buf.nXP * xs,
                  static_cast<char *>(x->buf.PSI) + cur * x->buf.nPSI * es,
                  x->buf.FLD + cur * x->buf.nFLD, x->ref,
                  x->buf.MOM ? x->buf.MOM + cur * x->buf.nMOM : nullptr};
  const size_t nb[6] = {x->buf.nXS * es, x->buf.nXP * xs, x->buf.nPSI * es, x->buf.nFLD * 8,
                        x->ref ? ref_elems(x) * sizeof(float) : 0, x->buf.nMOM * sizeof(float)};
  std::vector<char> h;
  HIPCHK(hipStreamSynchronize(x->stream));
  for (int i = 0; i < 6 && ok; ++i) {
    if (!nb[i]) continue;
    h.resize(nb[i]);
    ok = std::fread(h.data(), 1, nb[i], f) == nb[i];
    if (ok && hipMemcpy(dst[i], h.data(), nb[i], hipMemcpyHostToDevice) != hipSuccess) {
      std::fclose(f);
      return fail(TPL_EHIP, "checkpoint upload failed");
    }
  }
  std::fclose(f);
  if (!ok) return fail(TPL_EINVAL, "checkpoint truncated");
  if (x->ref) {
    rc = build_step_ref(x);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(x->stream));
  }
  x->step = step;
  x->ip_odd = 0;  // a checkpoint holds the populations in plain order
  return TPL_OK;
}

void tpl_destroy(tpl_ctx *x) {
  if (!x) return;
  if (x->owned) {
    (void)hipFree(x->buf.XS);
    (void)hipFree(x->buf.XP);
    (void)hipFree(x->buf.PSI);
    (void)hipFree(x->buf.FLD);
    (void)hipFree(x->buf.MOM);
  }
  (void)hipFree(x->qtab_d);
  (void)hipFree(x->peq_d);
  (void)hipFree(x->ref);
  (void)hipFree(x->sref);
  (void)hipFree(x->scratch);
  (void)hipFree(x->src_d);
  (void)hipFree(x->obs_d);
  (void)hipFree(x->part_d);
  (void)hipFree(x->gate_d);
  (void)hipFree(x->corr_d);
  (void)hipFree(x->good_d);
  delete x;
}

}  // extern "C"

// ===========================================================================
// Batched form: many independent lattices, each a full context, advanced
// together by one launch per step over the flat list of all their 64-node
// tiles (the "items"); the launches of several steps are captured in a HIP
// graph.  Unstable instances are dropped from the item list and flagged.

struct tpl_batch {
  std::vector<tpl_ctx *> inst;
  std::vector<tpl_instance> spec;
  std::vector<int> unstable;
  int precision = TPL_FP64;
  hipStream_t stream = nullptr, own_stream = nullptr;
  bool inited = false;
  // launch shape of the batched step
  int qsplit = 0, grid = 0, autotune = 1, graph_steps = 20, time_kernels = 0;
  int qs_used = 0, grid_used = 0, group = 0, group_used = 1;
  bool rowtile = false;
  // device instance table of the active instances
  std::vector<InstDev> tab;
  InstDev *tab_d = nullptr;
  int tab_cap = 0, nitems = 0;
  bool tab_dirty = true;
  // captured graph: graph_steps launches with parities 0, 1, 0, 1, ...
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  // in-place streaming of every instance: the step kind alternates with the
  // batch's step count (ip_odd), which the captured graph starts from (graph_ip)
  int inplace = 0, ip_odd = 0, graph_ip = 0;
  int spring_shift = 0;  // the shifted spring term for every instance
  int gradients = 0;     // same-step gradients for every instance
  bool qe2 = false;      // model (ii) for every instance (set at tpl_batch_init)
  double *scratch = nullptr;
  int scratch_n = 0;
  double kernel_ms = 0.0, tune_ms = 0.0;
  long long kernel_steps = 0;
  long long step = 0;
};

namespace {

void drop_graph(tpl_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

// Instance record of one context for the step kernel: both halves of its
// state, its tables and the batch's Q-slice count.
InstDev inst_record(tpl_ctx *x, const Buffers &B, int nx, int ny, int qs, int item0,
                    int cur0) {
  InstDev r{};
  r.p = make_step_params(x, nx, ny, qs);
  r.p.qs = qs;
  r.p.tiles_per_xcd = 0;
  r.p.wg = 0;
  for (int h = 0; h < 2; ++h) {
    r.XS[h] = static_cast<char *>(B.XS) + B.pop_half(h) * B.nXS * B.esize;
    r.XP[h] = static_cast<char *>(B.XP) + B.pop_half(h) * B.nXP * B.esize;
    r.PSI[h] = static_cast<char *>(B.PSI) + h * B.nPSI * B.esize;
    r.FLD[h] = B.FLD + h * B.nFLD;
  }
  const StepRef ref = B.esize == 4 ? step_ref(x) : StepRef{nullptr, nullptr, nullptr, nullptr, nullptr};
  r.rpull = ref.pull;
  r.rstore = ref.store;
  r.rpsi = ref.psi;
  r.rspull = ref.spull;
  r.rsstore = ref.sstore;
  r.qtab = x->qtab_d;
  r.item0 = item0;
  r.cur0 = cur0;
  return r;
}

int upload_table(tpl_batch *b, const std::vector<InstDev> &tab) {
  if ((int)tab.size() > b->tab_cap) {
    if (b->tab_d) HIPCHK(hipFree(b->tab_d));
    b->tab_d = nullptr;
    b->tab_cap = 0;
    if (hipMalloc(&b->tab_d, sizeof(InstDev) * tab.size()) != hipSuccess) {
      (void)hipGetLastError();
      return fail(TPL_ENOMEM, "instance table allocation failed");
    }
    b->tab_cap = (int)tab.size();
  }
  // synchronous: the host vector may change right after
  HIPCHK(hipMemcpyAsync(b->tab_d, tab.data(), sizeof(InstDev) * tab.size(),
                        hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  return TPL_OK;
}

// inplace: the instances' own lattices, streamed in place when the batch is
// (the base-state columns always keep two arrays).
hipError_t batch_launch(const tpl_batch *b, int esize, int ninst, int nitems, int qs, int grid,
                        bool rowtile, int parity, int group, bool inplace = true) {
  const int ip = (inplace && b->inplace) ? (((b->ip_odd + parity) & 1) ? 2 : 1) : 0;
  const bool sh = b->spring_shift != 0;  // base-state columns as well
  if (b->gradients) {  // base-state columns as well
    int nqd = 1;  // Q-nodes per r-node, the largest of the instances
    for (const tpl_ctx *x : b->inst) nqd = x->d.nqd > nqd ? x->d.nqd : nqd;
    const hipError_t e =
        esize == 4 ? launch_same_step_fields_batch<float>(b->tab_d, ninst, nitems, nqd, parity, ip,
                                                          sh, b->stream)
                   : launch_same_step_fields_batch<double>(b->tab_d, ninst, nitems, nqd, parity,
                                                           ip, sh, b->stream);
    if (e != hipSuccess) return e;
  }
  if (sh && !b->gradients) {  // (with same-step gradients formed above)
    const int sg = nitems < 4096 ? nitems : 4096;
    const hipError_t e =
        esize == 4 ? launch_spring_sum_batch<float>(b->tab_d, ninst, nitems, sg, parity, b->stream)
                   : launch_spring_sum_batch<double>(b->tab_d, ninst, nitems, sg, parity,
                                                     b->stream);
    if (e != hipSuccess) return e;
  }
  return esize == 4 ? launch_step_batch<float>(b->tab_d, ninst, nitems, qs, grid, rowtile, parity,
                                               b->stream, group, ip, sh, b->qe2)
                    : launch_step_batch<double>(b->tab_d, ninst, nitems, qs, grid, rowtile,
                                                parity, b->stream, group, ip, sh, b->qe2);
}

// Enqueue n launches of the uploaded table with parities p0, p0^1, ...
int batch_run(tpl_batch *b, int esize, int ninst, int nitems, int qs, int grid, bool rowtile,
              int p0, long long n, int group = 1, bool inplace = true) {
  for (long long i = 0; i < n; ++i)
    HIPCHK(batch_launch(b, esize, ninst, nitems, qs, grid, rowtile, (int)((p0 + i) & 1), group,
                        inplace));
  return TPL_OK;
}

int batch_scratch(tpl_batch *b, int n) {
  if (b->scratch_n >= n) return TPL_OK;
  if (b->scratch) HIPCHK(hipFree(b->scratch));
  b->scratch = nullptr;
  b->scratch_n = 0;
  if (hipMalloc(&b->scratch, sizeof(double) * n) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TPL_ENOMEM, "batch scratch allocation failed");
  }
  b->scratch_n = n;
  return TPL_OK;
}

// Base states of every instance: all columns stepped together, in phases
// that end when an instance has run its own number of column steps.
int batch_columns(tpl_batch *b) {
  const int n = (int)b->inst.size();
  std::vector<ColumnBuf> col(n);
  std::vector<long long> rem(n);
  std::vector<int> ccur(n, 0);
  int rc = TPL_OK;
  for (int i = 0; i < n && !rc; ++i) {
    tpl_ctx *x = b->inst[i];
    rc = col[i].alloc(x->c.ny, x->d.nqd);
    if (!rc) rc = column_rest(x, col[i]);
    rem[i] = pre_steps_of(x);
  }
  const int qs = kColumnQs;
  while (!rc) {
    long long k = -1;
    for (int i = 0; i < n; ++i)
      if (rem[i] > 0 && (k < 0 || rem[i] < k)) k = rem[i];
    if (k < 0) break;
    std::vector<InstDev> tab;
    int items = 0;
    for (int i = 0; i < n; ++i) {
      if (rem[i] <= 0) continue;
      tpl_ctx *x = b->inst[i];
      tab.push_back(inst_record(x, col[i].B, 1, x->c.ny, qs, items, ccur[i]));
      items += tab.back().p.ntiles;
    }
    rc = upload_table(b, tab);
    if (rc) break;
    rc = batch_run(b, 8, (int)tab.size(), items, qs, items, false, 0, k, 1, false);
    if (rc) break;
    for (int i = 0; i < n; ++i)
      if (rem[i] > 0) {
        rem[i] -= k;
        ccur[i] ^= (int)(k & 1);
      }
  }
  if (!rc) {
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) rc = fail(TPL_EHIP, std::string("column steps: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < n && !rc; ++i) rc = seed_from_column(b->inst[i], col[i].B.half64(ccur[i]));
  for (auto &c : col) c.release();
  return rc;
}

// Table of the active instances for the main step.
int build_main_table(tpl_batch *b, int qs) {
  b->tab.clear();
  int items = 0;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    if (b->unstable[i]) continue;
    tpl_ctx *x = b->inst[i];
    b->tab.push_back(inst_record(x, x->buf, x->c.nx, x->c.ny, qs, items, x->cur));
    items += b->tab.back().p.ntiles;
  }
  b->nitems = items;
  b->tab_dirty = true;
  drop_graph(b);
  return TPL_OK;
}

int batch_esize(const tpl_batch *b) { return b->precision == TPL_FP32 ? 4 : 8; }

// Average duration of one launch of the current table (read half cur0,
// write the other half: repeating it leaves the state unchanged).
int time_shape(tpl_batch *b, int qs, int grid, int reps, double *ms, int group = 1) {
  const int esize = batch_esize(b);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = batch_run(b, esize, (int)b->tab.size(), b->nitems, qs, grid, b->rowtile, 0, 1, group);
  if (!rc) {
    (void)hipEventRecord(e0, b->stream);
    for (int i = 0; i < reps && !rc; ++i)
      rc = batch_run(b, esize, (int)b->tab.size(), b->nitems, qs, grid, b->rowtile, 0, 1,
                     group);
    (void)hipEventRecord(e1, b->stream);
  }
  float t = 0.f;
  if (!rc) {
    const hipError_t e = hipEventSynchronize(e1);
    if (e != hipSuccess) rc = fail(TPL_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    else (void)hipEventElapsedTime(&t, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return rc;
}

// Choose the Q-slice count and the grid: candidates are one workgroup per
// item and persistent grids of one or two waves of workgroups per CU slot.
// Units of `group` consecutive items: what a grouped launch's grid counts.
int batch_units(const tpl_batch *b, int group) { return (b->nitems + group - 1) / group; }

int choose_shape_timed(tpl_batch *b);

// The launch shape, chosen by timing repeated launches on the current half.
// Those launches leave the populations unchanged, but the passes that same-step
// gradients and the shifted spring term run before each step rewrite the
// current half's psi and per-node fields (M, U): those are kept and put back.
int choose_shape(tpl_batch *b) {
  if (!b->autotune || b->inplace || !(b->gradients || b->spring_shift) || !b->inited)
    return choose_shape_timed(b);
  size_t total = 0;
  for (tpl_ctx *x : b->inst) {
    char *ptr[5];
    size_t nb[5];
    half_parts(x, x->cur, ptr, nb);
    total += nb[2] + nb[3];
  }
  char *keep = nullptr;
  if (hipMalloc(&keep, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TPL_ENOMEM, "autotune: no device memory to keep psi and the per-node fields");
  }
  int rc = TPL_OK;
  auto copy = [&](bool save) -> int {
    size_t off = 0;
    for (tpl_ctx *x : b->inst) {
      char *ptr[5];
      size_t nb[5];
      half_parts(x, x->cur, ptr, nb);
      for (int i = 2; i <= 3; ++i) {
        const hipError_t e = save ? hipMemcpyAsync(keep + off, ptr[i], nb[i],
                                                   hipMemcpyDeviceToDevice, b->stream)
                                  : hipMemcpyAsync(ptr[i], keep + off, nb[i],
                                                   hipMemcpyDeviceToDevice, b->stream);
        if (e != hipSuccess) return fail(TPL_EHIP, std::string("autotune keep: ") + hipGetErrorString(e));
        off += nb[i];
      }
    }
    return TPL_OK;
  };
  rc = copy(true);
  if (!rc) rc = choose_shape_timed(b);
  const int rr = copy(false);
  if (!rc) rc = rr;
  const hipError_t e = hipStreamSynchronize(b->stream);
  if (!rc && e != hipSuccess) rc = fail(TPL_EHIP, std::string("autotune: ") + hipGetErrorString(e));
  (void)hipFree(keep);
  return rc;
}

int choose_shape_timed(tpl_batch *b) {
  int qs_list[4] = {1, 2, 4, 8}, nqs = 4;
  if (b->qsplit > 0) {
    const int q = b->qsplit >= 8 ? 8 : b->qsplit >= 4 ? 4 : b->qsplit >= 2 ? 2 : 1;
    qs_list[0] = q;
    nqs = 1;
  }
  if (b->group > 1 && b->qsplit > 1)
    return fail(TPL_EINVAL, "item groups need one Q-slice (qsplit 0 or 1)");
  if (b->group != 0 && b->group != 1 && b->group != 2 && b->group != 4 && b->group != 8)
    return fail(TPL_EINVAL, "group must be 0 (tuned), 1, 2, 4 or 8");
  if (b->inplace) {
    // in place a launch advances the state, so shapes cannot be timed by
    // repeating it: one Q-slice, groups of `group` tiles (4 unless set)
    if (b->qsplit > 1) return fail(TPL_EINVAL, "in-place streaming needs one Q-slice (qsplit 0 or 1)");
    const int grp = b->group > 0 ? b->group : 4;
    b->qs_used = 1;
    b->group_used = grp;
    const int rc = build_main_table(b, 1);
    b->grid_used = b->grid > 0 ? b->grid : batch_units(b, grp);
    return rc;
  }
  int rc0 = build_main_table(b, qs_list[0]);  // sets nitems
  if (rc0) return rc0;
  if (!b->autotune) {
    int qs = qs_list[0];
    const int grp = b->group > 0 ? b->group : 1;
    if (grp > 1) {
      qs = 1;
    } else if (b->qsplit <= 0) {  // as for one lattice: >= 2048 waves, at most 8 slices
      qs = 1;
      while (qs < 8 && (long long)b->nitems * qs < 2048) qs *= 2;
    }
    b->qs_used = qs;
    b->group_used = grp;
    const int rc = build_main_table(b, qs);
    b->grid_used = b->grid > 0 ? b->grid : batch_units(b, grp);
    return rc;
  }
  // first the Q-slice count at one workgroup per item, then item groups
  // (one slice), then persistent grids (one or two workgroups per CU slot) at
  // the best shape
  double best = -1.0;
  int bq = qs_list[0], bg = b->nitems, bgrp = 1;
  b->tune_ms = 0.0;
  auto trial = [&](int qs, int g, int grp) -> int {
    double ms = 0.0;
    const int rc = time_shape(b, qs, g, 2, &ms, grp);
    b->tune_ms += 3 * ms;
    if (!rc && (best < 0 || ms < best)) {
      best = ms;
      bq = qs;
      bg = g;
      bgrp = grp;
    }
    return rc;
  };
  if (b->group <= 1) {
    for (int iq = 0; iq < nqs; ++iq) {
      int rc = build_main_table(b, qs_list[iq]);
      if (!rc) rc = upload_table(b, b->tab);
      if (!rc) rc = trial(qs_list[iq], b->grid > 0 ? b->grid : b->nitems, 1);
      if (rc) return rc;
    }
  }
  if (b->group != 1 && b->qsplit <= 1) {
    int rc = build_main_table(b, 1);
    if (!rc) rc = upload_table(b, b->tab);
    if (rc) return rc;
    const int cand[3] = {2, 4, 8};
    for (int grp : cand) {
      if (b->group > 1 && grp != b->group) continue;
      rc = trial(1, b->grid > 0 ? b->grid : batch_units(b, grp), grp);
      if (rc) return rc;
    }
  }
  if (b->grid <= 0) {
    int rc = build_main_table(b, bq);
    if (!rc) rc = upload_table(b, b->tab);
    if (rc) return rc;
    const int slots = 256 * 12 / (bq * bgrp);  // 256 CUs x 12 waves (3 per SIMD)
    for (int m = 1; m <= 2; ++m) {
      const int g = ((slots * m + 7) / 8) * 8;
      if (g < batch_units(b, bgrp)) {
        rc = trial(bq, g, bgrp);
        if (rc) return rc;
      }
    }
  }
  b->qs_used = bq;
  b->grid_used = bg;
  b->group_used = bgrp;
  return build_main_table(b, bq);
}

int capture_graph(tpl_batch *b) {
  drop_graph(b);
  if (b->graph_steps < 2 || b->stream == nullptr) return TPL_OK;
  const int esize = batch_esize(b);
  HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = batch_run(b, esize, (int)b->tab.size(), b->nitems, b->qs_used, b->grid_used,
                     b->rowtile, 0, b->graph_steps, b->group_used);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(TPL_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  b->graph = g;
  b->graph_ip = b->ip_odd;
  HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
  return TPL_OK;
}

// Health check of every active instance (NaN/Inf in U or psi, psi below
// -psi_floor max psi, as tpl_step judges a context); newly unstable
// instances are flagged and dropped from the table.
int batch_check(tpl_batch *b, int *newly) {
  *newly = 0;
  const int n = (int)b->inst.size();
  int rc = batch_scratch(b, 3 * n);
  if (rc) return rc;
  for (int i = 0; i < n; ++i) {
    if (b->unstable[i]) continue;
    tpl_ctx *x = b->inst[i];
    rc = ensure_scratch(x, 3 * (size_t)kHealthBlocks);
    if (rc) return rc;
    rc = health(x, x->scratch, b->scratch + 3 * i, b->stream, nullptr);
    if (rc) return rc;
  }
  std::vector<double> h(3 * n, 0.0);
  HIPCHK(hipMemcpyAsync(h.data(), b->scratch, sizeof(double) * 3 * n, hipMemcpyDeviceToHost,
                        b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int i = 0; i < n; ++i)
    if (!b->unstable[i] && judge_health(b->inst[i], &h[3 * i]) != TPL_OK) {
      b->unstable[i] = 1;
      ++*newly;
    }
  return TPL_OK;
}

struct BatchKey {
  const char *name;
  int tpl_batch::*field;
};
const BatchKey kBatchKeys[] = {
    {"qsplit", &tpl_batch::qsplit},           {"grid", &tpl_batch::grid},
    {"autotune", &tpl_batch::autotune},       {"graph_steps", &tpl_batch::graph_steps},
    {"group", &tpl_batch::group},
    {"time_kernels", &tpl_batch::time_kernels},
};

}  // namespace

extern "C" {

tpl_batch *tpl_batch_create(const tpl_instance *inst, int n, int precision) {
  if (!inst || n < 1) {
    fail(TPL_EINVAL, "need at least one instance");
    return nullptr;
  }
  if (precision != TPL_FP64 && precision != TPL_FP32) {
    fail(TPL_EINVAL, "a batch runs TPL_FP64 or TPL_FP32");
    return nullptr;
  }
  tpl_batch *b = new tpl_batch;
  b->precision = precision;
  for (int i = 0; i < n; ++i) {
    tpl_ctx *x = tpl_create(inst[i].nx, inst[i].ny, inst[i].Re, inst[i].Wi, inst[i].beta,
                            tpl_forcing{inst[i].periods, inst[i].u0});
    if (!x || tpl_set_param(x, "precision", precision) != TPL_OK) {
      const std::string msg = "instance " + std::to_string(i) + ": " + g_err;
      tpl_destroy(x);
      tpl_batch_destroy(b);
      fail(TPL_EINVAL, msg);
      return nullptr;
    }
    if (!(inst[i].perturbation >= 0)) {
      tpl_destroy(x);
      tpl_batch_destroy(b);
      fail(TPL_EINVAL, "instance " + std::to_string(i) + ": perturbation must be >= 0");
      return nullptr;
    }
    b->inst.push_back(x);
    b->spec.push_back(inst[i]);
  }
  b->unstable.assign(n, 0);
  return b;
}

int tpl_batch_set_param(tpl_batch *b, const char *key, double value) {
  if (!b || !key) return fail(TPL_EINVAL, "null argument");
  for (const BatchKey &k : kBatchKeys)
    if (!strcmp(k.name, key)) {
      if (!(value >= 0 && value <= (1 << 30))) return fail(TPL_EINVAL, "value out of range");
      const int old = b->*k.field;
      b->*k.field = (int)value;
      if (b->inited && strcmp(key, "time_kernels")) {  // new launch shape
        const int rc = choose_shape(b);
        if (rc) {
          b->*k.field = old;  // an invalid shape leaves the previous one
          return rc;
        }
        b->tab_dirty = true;
      }
      return TPL_OK;
    }
  if (!strcmp(key, "precision")) return fail(TPL_EINVAL, "precision is fixed at tpl_batch_create");
  if (!strcmp(key, "inplace") || !strcmp(key, "spring_shift") || !strcmp(key, "gradients")) {
    // set for the whole batch: every instance or none
    int &field = !strcmp(key, "inplace")        ? b->inplace
                 : !strcmp(key, "spring_shift") ? b->spring_shift
                                                : b->gradients;
    if (b->inited) return fail(TPL_ESTATE, std::string(key) + " is fixed after tpl_batch_init");
    if (value != 0 && value != 1) return fail(TPL_EINVAL, std::string(key) + " must be 0 or 1");
    for (size_t i = 0; i < b->inst.size(); ++i) {
      const int rc = tpl_set_param(b->inst[i], key, value);
      if (rc) {  // leave every instance as it was
        const std::string msg = g_err;
        for (size_t j = 0; j < i; ++j) (void)tpl_set_param(b->inst[j], key, field);
        return fail(rc, msg);
      }
    }
    field = (int)value;
    return TPL_OK;
  }
  if (b->inited) return fail(TPL_ESTATE, "instance parameters are fixed after tpl_batch_init");
  for (tpl_ctx *x : b->inst) {
    const int rc = tpl_set_param(x, key, value);
    if (rc) return rc;
  }
  return TPL_OK;
}

int tpl_batch_query(const tpl_batch *b, const char *key, double *out) {
  if (!b || !key || !out) return fail(TPL_EINVAL, "null argument");
  for (const BatchKey &k : kBatchKeys)
    if (!strcmp(k.name, key)) {
      *out = b->*k.field;
      return TPL_OK;
    }
  const std::string s = key;
  double v = 0.0;
  if (s == "instances") v = (double)b->inst.size();
  else if (s == "active") v = (double)b->tab.size();
  else if (s == "unstable") {
    for (int u : b->unstable) v += u;
  } else if (s == "items") v = b->nitems;
  else if (s == "nodes" || s == "bytes_per_step" || s == "bytes_state") {
    for (size_t i = 0; i < b->inst.size(); ++i) {
      if (s != "bytes_state" && b->unstable[i]) continue;
      double q = 0.0;
      const int rc = tpl_query(b->inst[i], s == "nodes" ? "nx" : key, &q);
      if (rc) return rc;
      if (s == "nodes") {
        double ny = 0.0;
        tpl_query(b->inst[i], "ny", &ny);
        q *= ny;
      }
      v += q;
    }
  } else if (s == "qsplit_used") v = b->qs_used;
  else if (s == "group_used") v = b->group_used;
  else if (s == "grid_used") v = b->grid_used;
  else if (s == "rowtile") v = b->rowtile;
  else if (s == "kernel_ms") v = b->kernel_steps ? b->kernel_ms / b->kernel_steps : 0.0;
  else if (s == "kernel_steps") v = (double)b->kernel_steps;
  else if (s == "tune_ms") v = b->tune_ms;
  else if (s == "step") v = (double)b->step;
  else return fail(TPL_EINVAL, "unknown key " + s);
  *out = v;
  return TPL_OK;
}

int tpl_batch_set_stream(tpl_batch *b, void *hip_stream) {
  if (!b) return fail(TPL_EINVAL, "null batch");
  b->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : b->own_stream;
  for (tpl_ctx *x : b->inst) x->stream = b->stream;
  drop_graph(b);
  b->tab_dirty = true;
  return TPL_OK;
}

int tpl_batch_init(tpl_batch *b) {
  if (!b) return fail(TPL_EINVAL, "null batch");
  for (tpl_ctx *x : b->inst) {
    if (x->c.qe_model != b->inst[0]->c.qe_model)
      return fail(TPL_EINVAL, "the instances of a batch share one qe_model");
    if (x->c.qe_model == 2 && x->c.spring_shift)
      return fail(TPL_EINVAL, "the batched step runs model (ii) with the Taylor spring term");
    if (x->c.inplace != b->inplace || x->c.spring_shift != b->spring_shift ||
        x->c.gradients != b->gradients)
      return fail(TPL_EINVAL, "inplace, spring_shift and gradients are set for the whole batch "
                              "(tpl_batch_set_param)");
    if (x->c.init_mode != 0)
      return fail(TPL_EINVAL, "a batch starts every instance from its column pre-run "
                              "(init_mode 0)");
  }
  b->qe2 = !b->inst.empty() && b->inst[0]->c.qe_model == 2;
  b->inited = false;
  drop_graph(b);
  if (!b->stream) {  // the batch's own stream, made on first use
    if (!b->own_stream &&
        hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      b->own_stream = nullptr;
      return fail(TPL_EHIP, "stream creation failed");
    }
    b->stream = b->own_stream;
    for (tpl_ctx *x : b->inst) x->stream = b->stream;
  }
  int rc = TPL_OK;
  for (tpl_ctx *x : b->inst) {
    rc = prepare_state(x);
    if (rc) return rc;
  }
  rc = batch_columns(b);
  if (rc) return rc;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    rc = finish_init(b->inst[i], b->spec[i].seed, b->spec[i].perturbation);
    if (rc) return rc;
  }
  b->unstable.assign(b->inst.size(), 0);
  b->rowtile = true;
  for (tpl_ctx *x : b->inst) b->rowtile = b->rowtile && (x->c.nx % 64 == 0);
  b->ip_odd = 0;
  b->step = 0;
  b->kernel_ms = 0.0;
  b->kernel_steps = 0;
  b->inited = true;
  return choose_shape(b);
}

int tpl_batch_step(tpl_batch *b, int64_t n) {
  if (!b) return fail(TPL_EINVAL, "null batch");
  if (!b->inited) return fail(TPL_ESTATE, "batch not initialised (call tpl_batch_init)");
  if (n < 0) return fail(TPL_EINVAL, "n must be >= 0");
  if (n == 0 || b->tab.empty()) return TPL_OK;
  // instances may have been stepped on their own: refresh the halves read
  for (size_t j = 0, i = 0; i < b->inst.size(); ++i) {
    if (b->unstable[i]) continue;
    if (b->inplace && b->inst[i]->ip_odd != b->ip_odd)
      return fail(TPL_ESTATE, "in place, every instance must be at the batch's step parity "
                              "(instance " + std::to_string(i) + " was stepped on its own)");
    if (b->tab[j].cur0 != b->inst[i]->cur) {
      b->tab[j].cur0 = b->inst[i]->cur;
      b->tab_dirty = true;
    }
    ++j;
  }
  int rc = TPL_OK;
  if (b->tab_dirty) {
    rc = upload_table(b, b->tab);
    if (rc) return rc;
    b->tab_dirty = false;
  }
  const int esize = batch_esize(b), G = b->graph_steps & ~1;
  if (b->gexec && b->inplace && b->graph_ip != b->ip_odd) drop_graph(b);  // other step kind first
  if (G >= 2 && n >= G && !b->gexec) {
    rc = capture_graph(b);
    if (rc) return rc;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (b->time_kernels) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, b->stream));
  }
  long long done = 0;
  if (b->gexec)
    for (; done + G <= n; done += G) HIPCHK(hipGraphLaunch(b->gexec, b->stream));
  rc = batch_run(b, esize, (int)b->tab.size(), b->nitems, b->qs_used, b->grid_used, b->rowtile,
                 0, n - done, b->group_used);
  if (rc) return rc;
  if (b->time_kernels) {
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    b->kernel_ms += ms;
    b->kernel_steps += n;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  for (size_t i = 0; i < b->inst.size(); ++i) {
    if (b->unstable[i]) continue;
    b->inst[i]->cur ^= (int)(n & 1);
    if (b->inplace) b->inst[i]->ip_odd ^= (int)(n & 1);
    b->inst[i]->step += n;
  }
  if (b->inplace) b->ip_odd ^= (int)(n & 1);
  b->step += n;
  int newly = 0;
  rc = batch_check(b, &newly);
  if (rc) return rc;
  if (newly) {
    rc = build_main_table(b, b->qs_used);
    if (rc) return rc;
    const int units = batch_units(b, b->group_used);
    if (b->grid > 0 || b->autotune == 0) b->grid_used = b->grid > 0 ? b->grid : units;
    if (b->grid_used > units && units > 0) b->grid_used = units;
  }
  return TPL_OK;
}

int tpl_batch_amplitudes(tpl_batch *b, double *out, int n) {
  if (!b || !out) return fail(TPL_EINVAL, "null argument");
  if (!b->inited) return fail(TPL_ESTATE, "batch not initialised (call tpl_batch_init)");
  if (n < (int)b->inst.size()) return fail(TPL_EINVAL, "output too small");
  for (size_t i = 0; i < b->inst.size(); ++i)
    out[i] = b->unstable[i] ? NAN : tpl_perturbation_amplitude(b->inst[i]);
  return TPL_OK;
}

int tpl_batch_status(const tpl_batch *b, int *unstable, int n) {
  if (!b || !unstable) return fail(TPL_EINVAL, "null argument");
  if (n < (int)b->inst.size()) return fail(TPL_EINVAL, "output too small");
  for (size_t i = 0; i < b->inst.size(); ++i) unstable[i] = b->unstable[i];
  return TPL_OK;
}

tpl_ctx *tpl_batch_instance(tpl_batch *b, int i) {
  if (!b || i < 0 || i >= (int)b->inst.size()) {
    fail(TPL_EINVAL, "instance index out of range");
    return nullptr;
  }
  return b->inst[i];
}

void tpl_batch_destroy(tpl_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (tpl_ctx *x : b->inst) tpl_destroy(x);
  if (b->tab_d) (void)hipFree(b->tab_d);
  if (b->scratch) (void)hipFree(b->scratch);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  delete b;
}

}  // extern "C"

// ===========================================================================
// Learned coarse-lattice correction: the network object, its training step,
// and the lattice side (restriction, features, targets, momentum source).

struct tpl_mlp {
  int nin = 0, hidden = 64, nout = 0, np = 0;
  hipStream_t stream = nullptr;
  std::vector<float> theta_h;          // master parameters until the device copy exists
  std::vector<float> norm_h;           // in_mean[64] in_std[64] out_mean[16] out_std[16]
  bool on_device = false;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;  // [np] (+1: sse)
  uint16_t *wb = nullptr;              // W1b | W2b | W3b | W2Tb | W3Tb
  float *fb = nullptr;                 // b1[64] b2[64] b3[16] | norm (160)
  float *partial = nullptr;
  int nrec = 0;
  uint16_t *xb = nullptr;
  long long xb_n = 0;
  int t = 0;  // Adam steps taken
};

namespace {

constexpr int kMlpRecs = 512;  // gradient records (waves) of a training pass

MlpDev mlp_dev(const tpl_mlp *m) {
  MlpDev w;
  w.W1b = m->wb;
  w.W2b = m->wb + 4096;
  w.W3b = m->wb + 8192;
  w.W2Tb = m->wb + 9216;
  w.W3Tb = m->wb + 13312;
  w.b1 = m->fb;
  w.b2 = m->fb + 64;
  w.b3 = m->fb + 128;
  w.out_mean = m->fb + 144 + 128;
  w.out_std = m->fb + 144 + 144;
  w.nin = m->nin;
  w.nout = m->nout;
  return w;
}
const float *mlp_in_mean(const tpl_mlp *m) { return m->fb + 144; }
const float *mlp_in_std(const tpl_mlp *m) { return m->fb + 144 + 64; }

// Device arrays of the network, made on first use (the object itself can be
// created and filled without a GPU).
int mlp_ready(tpl_mlp *m) {
  if (m->on_device) return TPL_OK;
  auto alloc = [&](void **p, size_t bytes) -> bool {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return false;
    }
    return true;
  };
  const size_t np = m->np;
  if (!alloc((void **)&m->theta, np * 4) || !alloc((void **)&m->m, np * 4) ||
      !alloc((void **)&m->v, np * 4) || !alloc((void **)&m->grad, (np + 1) * 4) ||
      !alloc((void **)&m->wb, 14336 * 2) || !alloc((void **)&m->fb, (144 + 160) * 4) ||
      !alloc((void **)&m->partial, (size_t)kMlpRecs * kMlpRecord * 4))
    return fail(TPL_ENOMEM, "network allocation failed");
  m->nrec = kMlpRecs;
  HIPCHK(hipMemcpyAsync(m->theta, m->theta_h.data(), np * 4, hipMemcpyHostToDevice, m->stream));
  HIPCHK(hipMemsetAsync(m->m, 0, np * 4, m->stream));
  HIPCHK(hipMemsetAsync(m->v, 0, np * 4, m->stream));
  HIPCHK(hipMemcpyAsync(m->fb + 144, m->norm_h.data(), 160 * 4, hipMemcpyHostToDevice,
                        m->stream));
  m->on_device = true;
  HIPCHK(launch_mlp_pack(m->theta, m->nin, m->nout, mlp_dev(m), m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return TPL_OK;
}

int mlp_inputs(tpl_mlp *m, const float *X, long long n) {
  if (n > m->xb_n) {
    if (m->xb) HIPCHK(hipFree(m->xb));
    m->xb = nullptr;
    m->xb_n = 0;
    if (hipMalloc(&m->xb, (size_t)n * 64 * 2) != hipSuccess) {
      (void)hipGetLastError();
      return fail(TPL_ENOMEM, "input staging allocation failed");
    }
    m->xb_n = n;
  }
  HIPCHK(launch_mlp_prep(X, n, m->nin, mlp_in_mean(m), mlp_in_std(m), m->xb, m->stream));
  return TPL_OK;
}

// One training pass: gradients (canonical layout) and sum of squared errors
// in m->grad[np].
int mlp_pass(tpl_mlp *m, const float *X, const float *T, long long n) {
  int rc = mlp_ready(m);
  if (!rc) rc = mlp_inputs(m, X, n);
  if (rc) return rc;
  HIPCHK(launch_mlp_train(mlp_dev(m), m->xb, T, n, m->nrec, m->partial, m->stream));
  HIPCHK(launch_mlp_reduce(m->partial, m->nrec, m->nin, m->nout, m->grad, m->stream));
  return TPL_OK;
}

int ensure_dev(double **p, size_t n) {
  if (*p) return TPL_OK;
  if (hipMalloc(p, n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(TPL_ENOMEM, "device allocation failed");
  }
  return TPL_OK;
}

int ctx_observables(tpl_ctx *x) {
  const long long N = (long long)x->c.nx * x->c.ny;
  int rc = ensure_dev(&x->obs_d, (size_t)TPL_NFIELDS * N);
  if (rc) return rc;
  return tpl_moments_device(x, x->obs_d, (size_t)TPL_NFIELDS * N);
}

}  // namespace

// Working arrays of an attached network (on first use) and the drift gate
// opened, before a run of corrected steps.
int learned_begin(tpl_ctx *x) {
  const long long N = (long long)x->c.nx * x->c.ny;
  int rc = mlp_ready(x->mlp);
  if (!rc) rc = ensure_dev(&x->src_d, 2 * (size_t)N);
  if (!rc) rc = ensure_dev(&x->part_d, 2 * (size_t)correct_waves(N));
  if (!rc) rc = ensure_dev(&x->obs_d, (size_t)TPL_NFIELDS * N);
  if (rc) return rc;
  if (!x->corr_d && hipMalloc(&x->corr_d, (size_t)N * 5 * 4) != hipSuccess) {
    (void)hipGetLastError();
    x->corr_d = nullptr;
    return fail(TPL_ENOMEM, "correction allocation failed");
  }
  if (!x->gate_d) {
    void *g = nullptr;
    if (hipMalloc(&g, 16) != hipSuccess) {
      (void)hipGetLastError();
      return fail(TPL_ENOMEM, "gate allocation failed");
    }
    x->gate_d = static_cast<int *>(g);
    x->drift_d = reinterpret_cast<unsigned long long *>(static_cast<char *>(g) + 8);
  }
  HIPCHK(hipMemsetAsync(x->gate_d, 0, 16, x->stream));  // gate open, largest drift 0
  x->src_on = true;
  return TPL_OK;
}

// Source of the attached network for the current state, enqueued (no host
// synchronisation): observables, the fused features + network + sums
// (k_correct), the centred source with its divergence and the drift gate
// (k_source_gate; tag = the step of the call it would stop).  Total
// momentum is conserved on both lattices and by the restriction, so the
// exact correction has zero lattice mean: the predicted mean is removed (the
// uniform momentum mode is undamped, a bias there would accumulate).
int learned_source(tpl_ctx *x, int tag) {
  tpl_mlp *m = x->mlp;
  const long long N = (long long)x->c.nx * x->c.ny;
  int rc = tpl_moments_device(x, x->obs_d, (size_t)TPL_NFIELDS * N);
  if (rc) return rc;
  HIPCHK(launch_correct(mlp_dev(m), x->obs_d, x->c.nx, x->c.ny, mlp_in_mean(m), mlp_in_std(m),
                        x->corr_d, x->part_d, x->gate_d, x->stream));
  HIPCHK(launch_source_gate(x->corr_d, x->c.nx, x->c.ny, x->part_d, correct_waves(N),
                            x->buf.half64(x->cur).FLD, x->drift_bound * x->c.u0, tag, x->src_d,
                            x->gate_d, x->drift_d, x->stream));
  return TPL_OK;
}

extern "C" {

tpl_mlp *tpl_mlp_create(int in, int hidden, int out, uint64_t seed) {
  if (hidden != 64 || in < 1 || in > 64 || out < 1 || out > 16) {
    fail(TPL_EINVAL, "network shape must be in (1..64) -> 64 -> 64 -> out (1..16)");
    return nullptr;
  }
  tpl_mlp *m = new tpl_mlp;
  m->nin = in;
  m->nout = out;
  m->np = 64 * in + 64 + 64 * 64 + 64 + out * 64 + out;
  m->theta_h.assign(m->np, 0.0f);
  // U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights from SplitMix64(seed), zero biases
  SplitMix64 rng{seed};
  auto fill = [&](size_t off, int rows, int fan_in) {
    const double a = 1.0 / std::sqrt((double)fan_in);
    for (int i = 0; i < rows * fan_in; ++i)
      m->theta_h[off + i] = (float)(a * (2.0 * rng.uniform() - 1.0));
  };
  fill(0, 64, in);
  fill(64 * in + 64, 64, 64);
  fill(64 * in + 64 + 4096 + 64, out, 64);
  m->norm_h.assign(160, 0.0f);
  for (int i = 0; i < 64; ++i) m->norm_h[64 + i] = 1.0f;
  for (int i = 0; i < 16; ++i) m->norm_h[144 + i] = 1.0f;
  return m;
}

int tpl_mlp_set_stream(tpl_mlp *m, void *hip_stream) {
  if (!m) return fail(TPL_EINVAL, "null network");
  m->stream = static_cast<hipStream_t>(hip_stream);
  return TPL_OK;
}

int tpl_mlp_query(const tpl_mlp *m, const char *key, double *out) {
  if (!m || !key || !out) return fail(TPL_EINVAL, "null argument");
  const std::string k = key;
  if (k == "nparams") *out = m->np;
  else if (k == "in") *out = m->nin;
  else if (k == "hidden") *out = m->hidden;
  else if (k == "out") *out = m->nout;
  else if (k == "adam_steps") *out = m->t;
  else return fail(TPL_EINVAL, "unknown key " + k);
  return TPL_OK;
}

int tpl_mlp_get_params(tpl_mlp *m, float *host, size_t n) {
  if (!m || !host) return fail(TPL_EINVAL, "null argument");
  if (n != (size_t)m->np) return fail(TPL_EINVAL, "parameter count mismatch");
  if (!m->on_device) {
    std::copy(m->theta_h.begin(), m->theta_h.end(), host);
    return TPL_OK;
  }
  HIPCHK(hipMemcpyAsync(host, m->theta, n * 4, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return TPL_OK;
}

int tpl_mlp_set_params(tpl_mlp *m, const float *host, size_t n) {
  if (!m || !host) return fail(TPL_EINVAL, "null argument");
  if (n != (size_t)m->np) return fail(TPL_EINVAL, "parameter count mismatch");
  std::copy(host, host + n, m->theta_h.begin());
  m->t = 0;
  if (!m->on_device) return TPL_OK;
  HIPCHK(hipMemcpyAsync(m->theta, host, n * 4, hipMemcpyHostToDevice, m->stream));
  HIPCHK(hipMemsetAsync(m->m, 0, n * 4, m->stream));
  HIPCHK(hipMemsetAsync(m->v, 0, n * 4, m->stream));
  HIPCHK(launch_mlp_pack(m->theta, m->nin, m->nout, mlp_dev(m), m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return TPL_OK;
}

int tpl_mlp_set_norm(tpl_mlp *m, const float *in_mean, const float *in_std,
                     const float *out_mean, const float *out_std) {
  if (!m || !in_mean || !in_std || !out_mean || !out_std) return fail(TPL_EINVAL, "null argument");
  for (int i = 0; i < m->nin; ++i)
    if (!(in_std[i] > 0)) return fail(TPL_EINVAL, "input scales must be > 0");
  for (int i = 0; i < m->nout; ++i)
    if (!(out_std[i] > 0)) return fail(TPL_EINVAL, "output scales must be > 0");
  for (int i = 0; i < m->nin; ++i) {
    m->norm_h[i] = in_mean[i];
    m->norm_h[64 + i] = in_std[i];
  }
  for (int i = 0; i < m->nout; ++i) {
    m->norm_h[128 + i] = out_mean[i];
    m->norm_h[144 + i] = out_std[i];
  }
  if (!m->on_device) return TPL_OK;
  HIPCHK(hipMemcpyAsync(m->fb + 144, m->norm_h.data(), 160 * 4, hipMemcpyHostToDevice,
                        m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return TPL_OK;
}

int tpl_mlp_forward(tpl_mlp *m, const float *X, float *Y, int64_t n) {
  if (!m || (n > 0 && (!X || !Y))) return fail(TPL_EINVAL, "null argument");
  if (n < 0) return fail(TPL_EINVAL, "n must be >= 0");
  if (n == 0) return TPL_OK;
  int rc = mlp_ready(m);
  if (!rc) rc = mlp_inputs(m, X, n);
  if (rc) return rc;
  HIPCHK(launch_mlp_forward(mlp_dev(m), m->xb, n, Y, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  return TPL_OK;
}

int tpl_mlp_grads(tpl_mlp *m, const float *X, const float *T, int64_t n, float *dW,
                  float *loss) {
  if (!m || !X || !T || !dW) return fail(TPL_EINVAL, "null argument");
  if (n < 1) return fail(TPL_EINVAL, "n must be >= 1");
  int rc = mlp_pass(m, X, T, n);
  if (rc) return rc;
  std::vector<float> g(m->np + 1);
  HIPCHK(hipMemcpyAsync(g.data(), m->grad, (m->np + 1) * 4, hipMemcpyDeviceToHost, m->stream));
  HIPCHK(hipStreamSynchronize(m->stream));
  std::copy(g.begin(), g.begin() + m->np, dW);
  if (loss) *loss = (float)(g[m->np] / ((double)n * m->nout));
  return TPL_OK;
}

int tpl_mlp_train_step(tpl_mlp *m, const float *X, const float *T, int64_t n, float lr,
                       float *loss) {
  if (!m || !X || !T) return fail(TPL_EINVAL, "null argument");
  if (n < 1) return fail(TPL_EINVAL, "n must be >= 1");
  if (!(lr > 0)) return fail(TPL_EINVAL, "lr must be > 0");
  int rc = mlp_pass(m, X, T, n);
  if (rc) return rc;
  m->t += 1;
  HIPCHK(launch_mlp_adam(m->theta, m->m, m->v, m->grad, m->np, lr, m->t, m->stream));
  HIPCHK(launch_mlp_pack(m->theta, m->nin, m->nout, mlp_dev(m), m->stream));
  if (loss) {
    float sse = 0.0f;
    HIPCHK(hipMemcpyAsync(&sse, m->grad + m->np, 4, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    *loss = (float)(sse / ((double)n * m->nout));
  }
  return TPL_OK;
}

void tpl_mlp_destroy(tpl_mlp *m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  (void)hipFree(m->theta);
  (void)hipFree(m->m);
  (void)hipFree(m->v);
  (void)hipFree(m->grad);
  (void)hipFree(m->wb);
  (void)hipFree(m->fb);
  (void)hipFree(m->partial);
  (void)hipFree(m->xb);
  delete m;
}

int tpl_restrict(const tpl_ctx *fine, tpl_ctx *coarse) {
  int rc = check_populations(fine);
  if (!rc) rc = check_populations(coarse);
  if (rc) return rc;
  const int nxf = fine->c.nx, nyf = fine->c.ny, nxc = coarse->c.nx, nyc = coarse->c.ny;
  if (nxc < 1 || nyc < 1 || nxf % nxc || nyf % nyc || nxf / nxc != nyf / nyc)
    return fail(TPL_EINVAL, "fine lattice must be the coarse one refined by one factor");
  const int mfac = nxf / nxc;
  if (mfac < 2 || (mfac & 1)) return fail(TPL_EINVAL, "refinement factor must be even");
  if (fine->d.nqd != coarse->d.nqd) return fail(TPL_EINVAL, "both lattices need the same nq");
  if (fp32(fine) || fp32(coarse)) return fail(TPL_EINVAL, "restriction needs FP64 storage");
  const int nqd = fine->d.nqd;
  const StateView f = fine->buf.half64(fine->cur), c = coarse->buf.half64(coarse->cur);
  hipStream_t s = coarse->stream;
  HIPCHK(hipStreamSynchronize(fine->stream));
  HIPCHK(launch_restrict<double>(9, nxf, nyf, mfac, f.XS, c.XS, s));
  HIPCHK(launch_restrict<double>(25 * nqd, nxf, nyf, mfac, f.XP, c.XP, s));
  HIPCHK(launch_restrict<double>(nqd, nxf, nyf, mfac, f.PSI, c.PSI, s));
  const size_t Nf = (size_t)nxf * nyf, Nc = (size_t)nxc * nyc;
  HIPCHK(launch_restrict<double>(2, nxf, nyf, mfac, f.FLD + F_UX * Nf, c.FLD + F_UX * Nc, s));
  const RefView none{nullptr, nullptr, nullptr, nyc};
  HIPCHK(launch_refresh<double>(nqd, nxc, nyc, coarse->qtab_d, c, none, s));
  HIPCHK(hipStreamSynchronize(s));
  return TPL_OK;
}

int tpl_features(tpl_ctx *x, float *X, size_t len) {
  int rc = check_ready(x);
  if (rc) return rc;
  const long long N = (long long)x->c.nx * x->c.ny;
  if (!X || len < (size_t)N * 54) return fail(TPL_EINVAL, "output too small");
  rc = ctx_observables(x);
  if (rc) return rc;
  HIPCHK(launch_features(x->obs_d, x->c.nx, x->c.ny, nullptr, nullptr, X, nullptr, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

int tpl_targets(tpl_ctx *x, const double *obs_ref, float *T, size_t len) {
  int rc = check_ready(x);
  if (rc) return rc;
  const long long N = (long long)x->c.nx * x->c.ny;
  if (!obs_ref || !T || len < (size_t)N * 5) return fail(TPL_EINVAL, "bad buffer");
  rc = ctx_observables(x);
  if (rc) return rc;
  HIPCHK(launch_targets(obs_ref, x->obs_d, N, T, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

int tpl_set_source(tpl_ctx *x, const double *F, size_t len) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (x->mlp) return fail(TPL_ESTATE, "a network is attached (tpl_attach_mlp(ctx, NULL, 0) first)");
  const size_t N = (size_t)x->c.nx * x->c.ny;
  if (!F) {
    x->src_on = false;
    return TPL_OK;
  }
  if (len != 2 * N) return fail(TPL_EINVAL, "source must hold 2 nx ny doubles");
  rc = ensure_dev(&x->src_d, 2 * N);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(x->src_d, F, 2 * N * sizeof(double), hipMemcpyHostToDevice, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  x->src_on = true;
  return TPL_OK;
}

int tpl_get_source(tpl_ctx *x, double *F, size_t len) {
  int rc = check_ready(x);
  if (rc) return rc;
  const size_t N = (size_t)x->c.nx * x->c.ny;
  if (!F || len != 2 * N) return fail(TPL_EINVAL, "source must hold 2 nx ny doubles");
  if (!x->src_on) {
    std::fill(F, F + 2 * N, 0.0);
    return TPL_OK;
  }
  HIPCHK(hipMemcpyAsync(F, x->src_d, 2 * N * sizeof(double), hipMemcpyDeviceToHost, x->stream));
  HIPCHK(hipStreamSynchronize(x->stream));
  return TPL_OK;
}

int tpl_attach_mlp(tpl_ctx *x, tpl_mlp *m, double drift_bound) {
  int rc = check_ready(x);
  if (rc) return rc;
  if (!m) {
    x->mlp = nullptr;
    x->src_on = false;
    return TPL_OK;
  }
  if (m->nin != 54 || m->nout != 5)
    return fail(TPL_EINVAL, "a correction network maps 54 features to 5 outputs");
  if (x->c.inplace || x->c.gradients || x->c.spring_shift)
    return fail(TPL_EINVAL, "a correction network runs on the two-array step with lagged "
                            "gradients and the Taylor spring term");
  if (!(drift_bound > 0)) return fail(TPL_EINVAL, "drift bound must be > 0");
  x->mlp = m;
  x->drift_bound = drift_bound;
  return TPL_OK;
}

}  // extern "C"
