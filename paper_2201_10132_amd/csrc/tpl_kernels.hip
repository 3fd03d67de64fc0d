// Device kernels of libtpl for gfx950 (MI355X): the fused stream +
// quasi-equilibrium step of the two-fluid polymer scheme (arXiv:2201.10132,
// Sec. VI) and its initialisation and FP64 reduction kernels.
//
// Layout (structure of arrays, r = y*nx + x innermost, so a wave's 64 lanes
// touch 64 consecutive values of one plane):
//   XS[9][N], XP[25][nqd][N], PSI[nqd][N] (storage type T), FLD[NF][N] (FP64)
// T = double stores values; T = float stores deviations from an x-invariant
// FP64 reference (the base state) and every kernel works on the full FP64
// value ref + deviation.
#include "tpl_internal.h"

#include <type_traits>

namespace tplk {

// ---------------------------------------------------------------------------
// Velocity sets.
// D2Q9 (Sec. VI.A; the standard set, the only one matching the weights
// 4/9, 1/9, 1/36).
constexpr int C9X[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int C9Y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr double W9[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// D4Q25 (Sec. VI.B, Table I) as (v_x, v_y, Qdot_x, Qdot_y): the rest vector,
// then for the coordinate pairs (vx,vy) (vx,Qx) (vx,Qy) (vy,Qx) (vy,Qy)
// (Qx,Qy) the sign pairs (+,+) (+,-) (-,+) (-,-).
constexpr int PV[25][4] = {
    {0, 0, 0, 0},                                                    //
    {1, 1, 0, 0},  {1, -1, 0, 0},  {-1, 1, 0, 0},  {-1, -1, 0, 0},   //
    {1, 0, 1, 0},  {1, 0, -1, 0},  {-1, 0, 1, 0},  {-1, 0, -1, 0},   //
    {1, 0, 0, 1},  {1, 0, 0, -1},  {-1, 0, 0, 1},  {-1, 0, 0, -1},   //
    {0, 1, 1, 0},  {0, 1, -1, 0},  {0, -1, 1, 0},  {0, -1, -1, 0},   //
    {0, 1, 0, 1},  {0, 1, 0, -1},  {0, -1, 0, 1},  {0, -1, 0, -1},   //
    {0, 0, 1, 1},  {0, 0, 1, -1},  {0, 0, -1, 1},  {0, 0, -1, -1}};  //

// D2Q9 direction of a D4Q25 velocity's r-part.
__host__ __device__ constexpr int dir9(int vx, int vy) {
  return (vx == 0 && vy == 0)    ? 0
         : (vx == 1 && vy == 0)  ? 1
         : (vx == 0 && vy == 1)  ? 2
         : (vx == -1 && vy == 0) ? 3
         : (vx == 0 && vy == -1) ? 4
         : (vx == 1 && vy == 1)  ? 5
         : (vx == -1 && vy == 1) ? 6
         : (vx == -1 && vy == -1) ? 7
                                  : 8;
}
__host__ __device__ constexpr int pdir(int k) { return dir9(PV[k][0], PV[k][1]); }
// The velocity with the same r-part and reversed Q-part (Q bounce-back).
__host__ __device__ constexpr int kstar(int k) {
  int j = 0;
  for (int i = 0; i < 25; ++i)
    if (PV[i][0] == PV[k][0] && PV[i][1] == PV[k][1] &&
        PV[i][2] == -PV[k][2] && PV[i][3] == -PV[k][3])
      j = i;
  return j;
}
static_assert(kstar(5) == 6 && kstar(21) == 24 && kstar(22) == 23 &&
                  kstar(1) == 1 && pdir(9) == 1 && pdir(16) == 4,
              "D4Q25 table");
// Opposite velocities: -c_d (D2Q9) and -(v_k, Qdot_k) (D4Q25).
__host__ __device__ constexpr int rev9(int d) {
  return dir9(-C9X[d], -C9Y[d]);
}
__host__ __device__ constexpr int krev(int k) {
  int j = 0;
  for (int i = 0; i < 25; ++i)
    if (PV[i][0] == -PV[k][0] && PV[i][1] == -PV[k][1] && PV[i][2] == -PV[k][2] &&
        PV[i][3] == -PV[k][3])
      j = i;
  return j;
}
static_assert(rev9(1) == 3 && rev9(5) == 7 && rev9(8) == 6 && krev(0) == 0 && krev(1) == 4 &&
                  krev(5) == 8 && krev(21) == 24 && krev(13) == 16,
              "opposite velocities");

__device__ __forceinline__ int xcd_tile(int bid, int tiles_per_xcd) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so that stencil neighbours share its L2.
  return tiles_per_xcd > 0 ? (bid & 7) * tiles_per_xcd + (bid >> 3) : bid;
}

// ---------------------------------------------------------------------------
// Storage access.  Loads and stores at a wave-uniform plane base plus a 32-bit
// byte offset (every offset is < sizeof(T) N < 2^32).  The base goes through
// readfirstlane so that it stays in scalar registers; the compiler hoists the
// zero-extended offsets out of the Q-loop and issues the accesses with 64-bit
// per-lane addresses (SGPR base plus offset, one VALU add each).  Forcing the
// SGPR-base instruction form instead (an opaque 32-bit offset per access)
// saves 8-15 VGPRs but measured no faster: the step is bound by DRAM.
template <typename T>
__device__ __forceinline__ T *uni(T *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}
// Accesses go through the global address space explicitly: a generic
// (flat) pointer would force 64-bit per-lane addresses and FLAT instructions.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ldo(const T *base, uint32_t off) {
  const char GLOBAL_AS *b = (const char GLOBAL_AS *)(base);
  return *(const T GLOBAL_AS *)(b + off);
}
template <typename T>
__device__ __forceinline__ void sto(T *base, uint32_t off, T v) {
  char GLOBAL_AS *b = (char GLOBAL_AS *)(base);
  *(T GLOBAL_AS *)(b + off) = v;
}
// Read-only tables (reference values, instance records) are read through the
// constant address space, which the compiler turns into scalar loads whenever
// the address is wave-uniform.
#define CONSTANT_AS __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const T CONSTANT_AS *cst(const T *p) {
  return (const T CONSTANT_AS *)(p);
}

// Full value from a stored one: identity for FP64, reference + deviation for
// the FP32 form (ref = the plane's reference value at this row).
__device__ __forceinline__ double full(double v, double) { return v; }
__device__ __forceinline__ double full(float v, double ref) { return ref + (double)v; }
template <typename T>
__device__ __forceinline__ T stored(double v, double ref);
template <>
__device__ __forceinline__ double stored<double>(double v, double) { return v; }
template <>
__device__ __forceinline__ float stored<float>(double v, double ref) { return (float)(v - ref); }

// BF16 form: a polymer population is stored as the BF16 rounding (nearest
// even) of its deviation from the FP32 reference, the x-invariant base state;
// solvent and psi keep FP32 deviations.  BF16 has FP32's exponent range, so
// the deviations need no scaling.
__device__ __forceinline__ uint16_t to_bf16(double v) {
  uint32_t u = __float_as_uint((float)v);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double from_bf16(uint16_t b) {
  return (double)__uint_as_float(((uint32_t)b) << 16);
}

// ---------------------------------------------------------------------------
// The fused step.  One lane per r-node; the Q-disk of that node is split over
// qs waves (slices) of the workgroup, each walking its Q-nodes in order.  All
// Q-dependent addressing (source Q-node, bounce-back) is wave-uniform.
//
// Per r-node, before any Q-node: solvent pull (9), polymer density and
// momentum from the 9 streamed Q-marginals of the previous step, lagged
// velocity gradient and spring-stress divergence from the 4 neighbours, the
// body force, the mixture velocity, the solvent collision.
// Per (r, Q)-node: pull 25 populations (bounce-back at the disk edge), their
// moments, the spring term from the lagged psi of the 4 neighbours, the
// imposed fluxes, the moment inversion, the blended equilibrium and the
// relaxation; write 25 populations and psi; accumulate the new marginals and
// M.  The slices' partial marginals are summed in LDS in a fixed order.
// Arithmetic is FP64 for both storage types.  ROWTILE: every 64-node tile
// lies in one lattice row (nx % 64 == 0), so the FP32 form's reference values
// are wave-uniform (scalar loads).
// One 64-node tile of one lattice (all qs slices of the workgroup take part).
// red: LDS of qs * 12 * 64 doubles.
// Non-local spring term: psi(r + Q/2) - psi(r - Q/2) of one Q-node's plane P
// (stored T, FP32 reference rpq(row)) at node (x, y), each side by bilinear
// interpolation between its four surrounding nodes, periodic.  The Q-node's
// offsets are wave-uniform; the wrap loops run at most NQ/4 + 1 times (a
// narrow lattice such as the one-column base-state run wraps more than once).
__device__ __forceinline__ int wrap_to(int v, int n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}
template <typename T, typename RefRow>
__device__ __forceinline__ double spring_shift_diff(const T *P, int x, int y, int nx, int ny,
                                                   double qx, double qy, RefRow rpq) {
  const double ax = 0.5 * qx, ay = 0.5 * qy;
  const double flx = floor(ax), fly = floor(ay);
  const double fx = ax - flx, fy = ay - fly;
  const int ix = (int)flx, iy = (int)fly;
  auto at = [&](int xx, int yy) {
    return full(ldo(P, (uint32_t)sizeof(T) * (uint32_t)(yy * nx + xx)), rpq(yy));
  };
  // + side: floor(Q/2) and the next node; - side: floor(-Q/2) = -floor(Q/2) - 1
  // (Q/2 is never an integer: Q-nodes sit at half-integers), weights swapped
  int xp0, xp1, yp0, yp1, xm0, xm1, ym0, ym1;
  if ((ix < 0 ? -ix : ix) + 2 <= nx && (iy < 0 ? -iy : iy) + 2 <= ny) {
    // offsets shorter than the lattice (wave-uniform test): every index lies
    // in [-n, 2n), one conditional add or subtract wraps it
    auto wr = [](int v, int n) {
      v = v < 0 ? v + n : v;
      return v >= n ? v - n : v;
    };
    xp0 = wr(x + ix, nx); xp1 = wr(x + ix + 1, nx);
    yp0 = wr(y + iy, ny); yp1 = wr(y + iy + 1, ny);
    xm0 = wr(x - ix - 1, nx); xm1 = wr(x - ix, nx);
    ym0 = wr(y - iy - 1, ny); ym1 = wr(y - iy, ny);
  } else {
    xp0 = wrap_to(x + ix, nx); xp1 = wrap_to(x + ix + 1, nx);
    yp0 = wrap_to(y + iy, ny); yp1 = wrap_to(y + iy + 1, ny);
    xm0 = wrap_to(x - ix - 1, nx); xm1 = wrap_to(x - ix, nx);
    ym0 = wrap_to(y - iy - 1, ny); ym1 = wrap_to(y - iy, ny);
  }
  const double vp = (1.0 - fx) * (1.0 - fy) * at(xp0, yp0) + fx * (1.0 - fy) * at(xp1, yp0) +
                    (1.0 - fx) * fy * at(xp0, yp1) + fx * fy * at(xp1, yp1);
  const double vm = fx * fy * at(xm0, ym0) + (1.0 - fx) * fy * at(xm1, ym0) +
                    fx * (1.0 - fy) * at(xm0, ym1) + (1.0 - fx) * (1.0 - fy) * at(xm1, ym1);
  return vp - vm;
}

// Mixture velocity: the velocity at which the momentum exchange of the two
// species cancels (Sec. IV/V), from their g-momenta, the body force and the
// Q-sum S of the spring term, weighted by 1 / (2 tJ + 1) per species.
__device__ __forceinline__ void mixture_velocity(const StepParams &p, double rhoS, double JSx,
                                                 double JSy, double rhoP, double JPx, double JPy,
                                                 double Sx, double Sy, double Fbx, double Fby,
                                                 double &Ux, double &Uy) {
  const double den = rhoS * p.aS + rhoP * p.aP;
  Ux = ((JSx + 0.5 * Fbx) * p.aS + (JPx + Sx / (2.0 * p.tJP)) * p.aP) / den;
  Uy = ((JSy + 0.5 * Fby) * p.aS + (JPy + Sy / (2.0 * p.tJP)) * p.aP) / den;
}

// In-place streaming (IP != 0; one population array, a == b for XS and XP;
// the AA pattern of Bailey et al., "Accelerating lattice Boltzmann fluid flow
// simulations using graphics processors", ICPP 2009, with the Q-disk
// bounce-back folded into its address maps).  Steps alternate:
//   IP = 1: pull as in the two-array step, then write the post-collision
//           population of velocity k where the pull of the opposite velocity
//           -k read from (its source node, its plane): each node rewrites
//           exactly the locations it read, so nodes never race;
//   IP = 2: read velocity k's incoming value at the node itself, from the
//           plane of -k, and write the post-collision value to plane k.
// After an IP = 1 step the array holds the streamed populations in reversed
// planes; after the following IP = 2 step it holds exactly what the
// two-array step writes.  Both read and write with the same FP32 reference
// tables as the two-array step, so the three forms agree bitwise.  The
// solvent follows the same maps with the D2Q9 set.  Every wave of a
// workgroup owns its own nodes (one Q-slice), and the per-node fields and
// lagged psi stay double-buffered.
template <typename T, bool ROWTILE, bool B16 = false, bool QE2 = false, int IP = 0,
          bool SHIFT = false>
__device__ __forceinline__ void step_tile(const StepParams &p, const StateT<T> &a,
                                          const StateT<T> &b, const float *__restrict__ rpull,
                                          const float *__restrict__ rstore,
                                          const float *__restrict__ rpsi,
                                          const float *__restrict__ rspull,
                                          const float *__restrict__ rsstore,
                                          const QNode *__restrict__ qtab, const int tile,
                                          double *red) {
  constexpr bool F32 = std::is_same<T, float>::value;
  constexpr uint32_t SZ = sizeof(T);
  const int lane = threadIdx.x & 63;
  const int slice = p.qs > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const long long N = p.N;
  const long long rr = (long long)tile * 64 + lane;
  const bool active = rr < N;
  const int r = (int)(active ? rr : N - 1);
  const int nx = p.nx, ny = p.ny;
  int y = r / nx;
  const int x = r - y * nx;
  if (ROWTILE) y = __builtin_amdgcn_readfirstlane(y);
  const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
  const uint32_t oR = SZ * (uint32_t)r;
  const uint32_t oE = SZ * (uint32_t)(y * nx + xp), oW = SZ * (uint32_t)(y * nx + xm);
  const uint32_t oN = SZ * (uint32_t)(yp * nx + x), oS = SZ * (uint32_t)(ym * nx + x);
  const uint32_t fR = 8u * (uint32_t)r;
  const uint32_t fE = 8u * (uint32_t)(y * nx + xp), fW = 8u * (uint32_t)(y * nx + xm);
  const uint32_t fN = 8u * (uint32_t)(yp * nx + x), fS = 8u * (uint32_t)(ym * nx + x);
  uint32_t osrc[9], fsrc[9];  // byte offsets of the pull source r - c_d
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int sx = C9X[d] == 1 ? xm : (C9X[d] == -1 ? xp : x);
    const int sy = C9Y[d] == 1 ? ym : (C9Y[d] == -1 ? yp : y);
    osrc[d] = SZ * (uint32_t)(sy * nx + sx);
    fsrc[d] = 8u * (uint32_t)(sy * nx + sx);
  }
  auto plane = [&](const T *arr, long long i) { return uni(arr + (size_t)i * N); };
  auto wplane = [&](T *arr, long long i) { return uni(arr + (size_t)i * N); };
  auto fplane = [&](const double *arr, long long i) { return uni(arr + (size_t)i * N); };
  auto wfplane = [&](double *arr, long long i) { return uni(arr + (size_t)i * N); };
  // FP32 form: reference values, [row][q][k] / [row][q] / [row][d]
  auto rq = [&](const float *tab, int row, int q, int k) -> double {
    return F32 ? (double)cst(tab)[((size_t)row * p.nqd + q) * 25 + k] : 0.0;
  };
  auto rpq = [&](int row, int q) -> double {
    return F32 ? (double)cst(rpsi)[(size_t)row * p.nqd + q] : 0.0;
  };
  auto rsd = [&](const float *tab, int d) -> double {
    return F32 ? (double)cst(tab)[(size_t)y * 9 + d] : 0.0;
  };

  // ---- solvent pull and moments
  double gS[9], rhoS = 0.0, JSx = 0.0, JSy = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    gS[d] = IP == 2 ? full(ldo(plane(a.XS, rev9(d)), oR), rsd(rspull, d))
                    : full(ldo(plane(a.XS, d), osrc[d]), rsd(rspull, d));
    rhoS += gS[d];
    if (C9X[d]) JSx += C9X[d] * gS[d];
    if (C9Y[d]) JSy += C9Y[d] * gS[d];
  }
  // ---- polymer density and r-momentum: the streamed Q-marginals
  double rhoP = 0.0, JPx = 0.0, JPy = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const double m = ldo(fplane(a.FLD, F_M0 + d), fsrc[d]);
    rhoP += m;
    if (C9X[d]) JPx += C9X[d] * m;
    if (C9Y[d]) JPy += C9Y[d] * m;
  }
  // ---- lagged non-local terms (central differences)
  auto dX = [&](int f) { return 0.5 * (ldo(fplane(a.FLD, f), fE) - ldo(fplane(a.FLD, f), fW)); };
  auto dY = [&](int f) { return 0.5 * (ldo(fplane(a.FLD, f), fN) - ldo(fplane(a.FLD, f), fS)); };
  const double Kxx = dX(F_UX), Kxy = dY(F_UX), Kyx = dX(F_UY), Kyy = dY(F_UY);
  // Q-sum of the spring terms: the divergence of the lagged M (Taylor form),
  // or summed from the shifted psi by a launch before the step
  const double Sx = SHIFT ? ldo(fplane(a.FLD, F_MXX), fR) : p.kappa * (dX(F_MXX) + dY(F_MXY));
  const double Sy = SHIFT ? ldo(fplane(a.FLD, F_MXY), fR) : p.kappa * (dX(F_MXY) + dY(F_MYY));
  double Fbx = p.F0 * sin(p.kf * (double)(y + p.y0)), Fby = 0.0;
  if (p.src != nullptr) {  // extra body force (a learned correction's source)
    Fbx += p.src[r];
    Fby = p.src[N + r];
  }
  // ---- mixture velocity: exchange of the two species cancels
  double Ux, Uy;
  mixture_velocity(p, rhoS, JSx, JSy, rhoP, JPx, JPy, Sx, Sy, Fbx, Fby, Ux, Uy);
  const bool writer = (slice == 0) && active;

  // ---- solvent collision (slice 0 writes)
  {
    // model 1: f* about the species' own (inverted) momentum; model 2: f*
    // with the equilibrium's momentum and the species' own (inverted) stress
    const double vx = Ux + p.tJS * Fbx / rhoS, vy = Uy + p.tJS * Fby / rhoS;
    const double v2 = vx * vx + vy * vy;
    double usx = 0.0, usy = 0.0, Dxx = 0.0, Dxy = 0.0, Dyy = 0.0;
    if constexpr (!QE2) {
      usx = (2.0 * p.tJS * JSx + rhoS * Ux + p.tJS * Fbx) * p.aS / rhoS;
      usy = (2.0 * p.tJS * JSy + rhoS * Uy + p.tJS * Fby) * p.aS / rhoS;
    } else {
      // P(f) - rho c_s^2 I with P(f) = (2 tau2 P(g) + rho (c_s^2 I + v v)) / (2 tau2 + 1)
      double Pxx = 0.0, Pxy = 0.0, Pyy = 0.0;
#pragma unroll
      for (int d = 0; d < 9; ++d) {
        if (C9X[d]) Pxx += gS[d];
        if (C9Y[d]) Pyy += gS[d];
        if (C9X[d] && C9Y[d]) Pxy += C9X[d] * C9Y[d] * gS[d];
      }
      const double t2 = 1.0 - p.pS;  // 2 tau2 / (2 tau2 + 1)
      Dxx = t2 * Pxx + p.pS * rhoS * (1.0 / 3.0 + vx * vx) - rhoS / 3.0;
      Dyy = t2 * Pyy + p.pS * rhoS * (1.0 / 3.0 + vy * vy) - rhoS / 3.0;
      Dxy = t2 * Pxy + p.pS * rhoS * vx * vy;
    }
    const double us2 = usx * usx + usy * usy;
    double jx = 0.0, jy = 0.0;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      const double cv = C9X[d] * vx + C9Y[d] * vy;
      const double fe = W9[d] * rhoS * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * v2);
      double fs;
      if constexpr (!QE2) {
        const double cu = C9X[d] * usx + C9Y[d] * usy;
        fs = W9[d] * rhoS * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * us2);
      } else {  // second-order Hermite form with the stress D + rho c_s^2 I
        const double h = Dxx * (C9X[d] * C9X[d] - 1.0 / 3.0) +
                         Dyy * (C9Y[d] * C9Y[d] - 1.0 / 3.0) + 2.0 * Dxy * C9X[d] * C9Y[d];
        fs = W9[d] * (rhoS + 3.0 * rhoS * cv + 4.5 * h);
      }
      const double o = p.c1S * gS[d] + p.c2S * ((1.0 - p.rS) * fs + p.rS * fe);
      if (C9X[d]) jx += C9X[d] * o;
      if (C9Y[d]) jy += C9Y[d] * o;
      if (writer) {
        if constexpr (IP == 1)
          sto(wplane(b.XS, rev9(d)), osrc[rev9(d)], stored<T>(o, rsd(rsstore, d)));
        else
          sto(wplane(b.XS, d), oR, stored<T>(o, rsd(rsstore, d)));
      }
    }
    if (writer) {
      sto(wfplane(b.FLD, F_JSX), fR, jx);
      sto(wfplane(b.FLD, F_JSY), fR, jy);
    }
  }

  // ---- polymer, Q-node by Q-node
  double mg[9];
#pragma unroll
  for (int d = 0; d < 9; ++d) mg[d] = 0.0;
  double Mxx = 0.0, Mxy = 0.0, Myy = 0.0;
  const int nqd = p.nqd;
  const double c2w0 = p.c2P * (1.0 / 3.0), c2w1 = p.c2P * (1.0 / 36.0);
  const double one_r = 1.0 - p.rP;
  const bool qsync = (p.wg >> 16) & 1;  // only with qs == 1: equal trip counts
  for (int q = slice; q < nqd; q += p.qs) {
    if (qsync) __syncthreads();  // keep the group's waves on the same Q-node
    const QNode CONSTANT_AS &qn = cst(qtab)[q];  // scalar loads
    // the Q-node's 25 populations: FP64 values, or for the BF16 form their
    // FP32 deviations from the pull reference (the collision's result: from
    // the store reference), which halves the registers they hold
    using GT = std::conditional_t<B16, float, double>;
    GT g[25];
    float rest_res = 0.0f;  // BF16 form: rounding residual of velocities 1..24
    auto G = [&](int k) -> double {
      if constexpr (B16) return rq(rpull, y, q, k) + (double)g[k];
      else return g[k];
    };
    if constexpr (IP == 2) {
      // plane order, each base one plane stride past the last; the stride is
      // kept opaque so that the 25 bases are not hoisted out of the Q-loop
      // (held across it they spill scalar registers, and the spills
      // serialise the loads)
      uint64_t stride = (uint64_t)nqd * (uint64_t)N * SZ;
      asm volatile("" : "+s"(stride));
      const char *pb = reinterpret_cast<const char *>(uni(a.XP + (size_t)q * N));
#pragma unroll
      for (int j = 0; j < 25; ++j)
        g[krev(j)] = full(ldo(reinterpret_cast<const T *>(pb + (size_t)j * stride), oR),
                          rq(rpull, y, q, krev(j)));
    } else if constexpr (!B16) {
#pragma unroll
      for (int k = 0; k < 25; ++k)
        g[k] = full(ldo(plane(a.XP, qn.plane[k]), osrc[pdir(k)]), rq(rpull, y, q, k));
    } else {
      // BF16 form: the 24 pulled deviations, 16 bits each, at half the byte
      // offsets of the FP32 planes; the node's own rest population in FP32
      // from its two 16-bit halves (planes 0 and 25)
      const uint16_t *xp = reinterpret_cast<const uint16_t *>(a.XP);
#pragma unroll
      for (int k = 1; k < 25; ++k)
        g[k] = (float)from_bf16(ldo(uni(xp + (size_t)qn.plane[k] * N), osrc[pdir(k)] >> 1));
      const uint32_t hi = ldo(uni(xp + (size_t)q * N), oR >> 1);
      const uint32_t lo = ldo(uni(xp + (size_t)(25 * nqd + q) * N), oR >> 1);
      g[0] = __uint_as_float((hi << 16) | lo);
    }
    double psi = 0.0, Jrx = 0.0, Jry = 0.0, JQx = 0.0, JQy = 0.0;
    double P2[4][4] = {};  // model 2: second moments sum xi_a xi_b g (a <= b)
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      const double gk = G(k);
      psi += gk;
      if (PV[k][0]) Jrx += PV[k][0] * gk;
      if (PV[k][1]) Jry += PV[k][1] * gk;
      if (PV[k][2]) JQx += PV[k][2] * gk;
      if (PV[k][3]) JQy += PV[k][3] * gk;
      if constexpr (QE2) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b2 = a; b2 < 4; ++b2)
            if (PV[k][a] && PV[k][b2]) P2[a][b2] += PV[k][a] * PV[k][b2] * gk;
      }
    }
    // spring term: kappa Fhat (Q . grad psi^{n-1}), or with the shift
    // kappa Fhat [psi^{n-1}(r + Q/2) - psi^{n-1}(r - Q/2)]
    const T *P = plane(a.PSI, q);
    double qg;
    if constexpr (SHIFT) {
      qg = spring_shift_diff(P, x, y, nx, ny, qn.qx, qn.qy, [&](int row) { return rpq(row, q); });
    } else {
      const double pE = full(ldo(P, oE), rpq(y, q)), pW = full(ldo(P, oW), rpq(y, q));
      const double pN = full(ldo(P, oN), rpq(yp, q)), pS = full(ldo(P, oS), rpq(ym, q));
      const double gx = 0.5 * (pE - pW), gy = 0.5 * (pN - pS);
      qg = qn.qx * gx + qn.qy * gy;
    }
    const double sx = p.kappa * qn.fx * qg, sy = p.kappa * qn.fy * qg;
    // imposed fluxes and moment inversion
    const double Erx = psi * Ux + sx, Ery = psi * Uy + sy;
    const double EQx = psi * (Kxx * qn.qx + Kxy * qn.qy - p.DQ * qn.fx);
    const double EQy = psi * (Kyx * qn.qx + Kyy * qn.qy - p.DQ * qn.fy);
    double A[4];
    if constexpr (!QE2) {
      const double Frx = (2.0 * p.tJP * Jrx + Erx) * p.aP;
      const double Fry = (2.0 * p.tJP * Jry + Ery) * p.aP;
      const double FQx = (2.0 * p.tJP * JQx + EQx) * p.aP;
      const double FQy = (2.0 * p.tJP * JQy + EQy) * p.aP;
      // (1 - r) f* + r f_eq is the linear equilibrium of the blended fluxes
      A[0] = 3.0 * c2w1 * (one_r * Frx + p.rP * Erx);
      A[1] = 3.0 * c2w1 * (one_r * Fry + p.rP * Ery);
      A[2] = 3.0 * c2w1 * (one_r * FQx + p.rP * EQx);
      A[3] = 3.0 * c2w1 * (one_r * FQy + p.rP * EQy);
    } else {
      // f* and f_eq share the imposed fluxes; f* adds the Hermite term of
      // D = P(f) - psi c_s^2 I, P(f) = (2 tau2 P(g) + psi c_s^2 I) / (2 tau2 + 1)
      A[0] = 3.0 * c2w1 * Erx;
      A[1] = 3.0 * c2w1 * Ery;
      A[2] = 3.0 * c2w1 * EQx;
      A[3] = 3.0 * c2w1 * EQy;
      const double t2 = 1.0 - p.pP;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        P2[a][a] = t2 * P2[a][a] + p.pP * psi / 3.0 - psi / 3.0;
#pragma unroll
        for (int b2 = a + 1; b2 < 4; ++b2) P2[a][b2] *= t2;
      }
    }
    const double h = c2w1 * psi;
    // model 2: the Hermite term's factor c2 (1 - r) 4.5 w_k, and -tr(D)/3
    const double hw = 4.5 * one_r * c2w1;
    const double trD3 = QE2 ? (P2[0][0] + P2[1][1] + P2[2][2] + P2[3][3]) / 3.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      double t = (k == 0) ? c2w0 * psi : h;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (PV[k][c]) t += PV[k][c] * A[c];
      if constexpr (QE2) {
        if (k == 0) {
          t -= 4.5 * one_r * c2w0 * trD3;
        } else {
          // sum_ab D_ab (xi_a xi_b - delta_ab / 3) for xi with two unit entries
          double hk = -trD3;
#pragma unroll
          for (int a = 0; a < 4; ++a)
            if (PV[k][a]) {
              hk += P2[a][a];
#pragma unroll
              for (int b2 = a + 1; b2 < 4; ++b2)
                if (PV[k][b2]) hk += 2.0 * PV[k][a] * PV[k][b2] * P2[a][b2];
            }
          t += hw * hk;
        }
      }
      const double go = p.c1P * G(k) + t;  // post-collision population
      mg[pdir(k)] += go;
      if constexpr (B16) {
        // the deviation from the store reference; the rest population (k = 0)
        // collects what BF16 rounding takes from the other 24 (each such
        // residual is exact in FP32)
        const float dv = (float)(go - rq(rstore, y, q, k));
        g[k] = dv;
        if (k > 0) rest_res += dv - (float)from_bf16(to_bf16(dv));
      } else {
        g[k] = go;
      }
    }
    if constexpr (B16) g[0] += rest_res;
    if (active) {
      if constexpr (IP == 1) {
        // the source planes are read again here rather than held across the
        // collision (25 bases in scalar registers spill and serialise the
        // loads); the empty asm keeps the compiler from reusing the earlier
        // reads
        const QNode GLOBAL_AS &qs2 = *(const QNode GLOBAL_AS *)(qtab + q);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < 25; ++k)
          sto(wplane(b.XP, qs2.plane[krev(k)]), osrc[pdir(krev(k))],
              stored<T>(g[k], rq(rstore, y, q, k)));
        sto(wplane(b.PSI, q), oR, stored<T>(psi, rpq(y, q)));
      } else if constexpr (!B16) {
        // plane bases one stride apart, the stride opaque so that they are
        // not hoisted out of the Q-loop (as for the node-local in-place reads)
        uint64_t stride = (uint64_t)nqd * (uint64_t)N * SZ;
        asm volatile("" : "+s"(stride));
        char *pw = reinterpret_cast<char *>(uni(b.XP + (size_t)q * N));
#pragma unroll
        for (int k = 0; k < 25; ++k)
          sto(reinterpret_cast<T *>(pw + (size_t)k * stride), oR,
              stored<T>(g[k], rq(rstore, y, q, k)));
        sto(wplane(b.PSI, q), oR, stored<T>(psi, rpq(y, q)));
      } else {
        // BF16 form: the 24 deviations (from the store reference) rounded to
        // 16 bits, the rest population's FP32 bits split over planes 0 and
        // 25; plane stride opaque as above
        sto(wplane(b.PSI, q), oR, stored<T>(psi, rpq(y, q)));
        uint64_t stride = (uint64_t)nqd * (uint64_t)N * 2u;
        asm volatile("" : "+s"(stride));
        char *pw = reinterpret_cast<char *>(uni(reinterpret_cast<uint16_t *>(b.XP) + (size_t)q * N));
        const uint32_t u0 = __float_as_uint(g[0]);
        sto(reinterpret_cast<uint16_t *>(pw), oR >> 1, (uint16_t)(u0 >> 16));
#pragma unroll
        for (int k = 1; k < 25; ++k)
          sto(reinterpret_cast<uint16_t *>(pw + (size_t)k * stride), oR >> 1, to_bf16(g[k]));
        sto(reinterpret_cast<uint16_t *>(pw + (size_t)25 * stride), oR >> 1,
            (uint16_t)(u0 & 0xffffu));
      }
    }
    Mxx += psi * qn.qx * qn.fx;
    Mxy += psi * qn.qx * qn.fy;
    Myy += psi * qn.qy * qn.fy;
  }

  // ---- combine the slices' partial sums
  if (p.qs > 1) {
    double *mine = red + (size_t)slice * 12 * 64;
#pragma unroll
    for (int d = 0; d < 9; ++d) mine[d * 64 + lane] = mg[d];
    mine[9 * 64 + lane] = Mxx;
    mine[10 * 64 + lane] = Mxy;
    mine[11 * 64 + lane] = Myy;
    __syncthreads();
    if (slice == 0) {
      for (int s = 1; s < p.qs; ++s) {
        const double *o = red + (size_t)s * 12 * 64;
#pragma unroll
        for (int d = 0; d < 9; ++d) mg[d] += o[d * 64 + lane];
        Mxx += o[9 * 64 + lane];
        Mxy += o[10 * 64 + lane];
        Myy += o[11 * 64 + lane];
      }
    }
  }
  if (writer) {
    sto(wfplane(b.FLD, F_RHOS), fR, rhoS);
    sto(wfplane(b.FLD, F_RHOP), fR, rhoP);
    sto(wfplane(b.FLD, F_UX), fR, Ux);
    sto(wfplane(b.FLD, F_UY), fR, Uy);
    sto(wfplane(b.FLD, F_MXX), fR, Mxx);
    sto(wfplane(b.FLD, F_MXY), fR, Mxy);
    sto(wfplane(b.FLD, F_MYY), fR, Myy);
#pragma unroll
    for (int d = 0; d < 9; ++d) sto(wfplane(b.FLD, F_M0 + d), fR, mg[d]);
  }
  if (p.qs > 1) __syncthreads();  // red is reused by the workgroup's next tile
}

template <typename T, int MAXT, bool ROWTILE, bool B16 = false, bool QE2 = false, int IP = 0,
          bool SHIFT = false>
__global__ void __launch_bounds__(MAXT)
    k_step(StepParams p, StateT<T> a, StateT<T> b, const float *__restrict__ rpull,
           const float *__restrict__ rstore, const float *__restrict__ rpsi,
           const float *__restrict__ rspull, const float *__restrict__ rsstore,
           const QNode *__restrict__ qtab) {
  extern __shared__ double red[];  // [qs][12][64]
  if (p.gate && *p.gate) return;  // a learned correction's drift gate closed
  int tile;
  if (p.wg == 0) {
    tile = xcd_tile(blockIdx.x, p.tiles_per_xcd);
    if (tile >= p.ntiles) return;  // whole workgroup leaves together
  } else {
    // a group of gx x gy tiles (one wave each) of gy consecutive rows;
    // tiles_per_xcd counts groups
    const int gx = p.wg & 255, gy = (p.wg >> 8) & 255;
    const int grp = xcd_tile(blockIdx.x, p.tiles_per_xcd);
    if (grp * gx * gy >= p.ntiles) return;  // whole workgroup leaves together
    const int tpr = p.nx >> 6, gpr = tpr / gx;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    tile = ((grp / gpr) * gy + w / gx) * tpr + (grp % gpr) * gx + w % gx;
  }
  step_tile<T, ROWTILE, B16, QE2, IP, SHIFT>(p, a, b, rpull, rstore, rpsi, rspull, rsstore,
                                             qtab, tile, red);
}


// Batched step: one launch advances every instance of a batch by one step.
// Workgroups walk a flat list of (instance, tile) items with a fixed stride;
// the item index is remapped so that each XCD works through a contiguous
// range of items.  parity selects which half of every instance is read.
// With group > 1 (one Q-slice) a workgroup takes `group` consecutive items,
// one wave each, so that neighbouring tiles' overlapping stencil reads meet
// in the caches; units of `group` items are what the grid and the XCD
// mapping count.  IP != 0: every instance streams in place (step_tile);
// SHIFT: the shifted spring term, its Q-sum formed by k_spring_sum_batch.
// QE2: the stress quasi-equilibria (model (ii)) for every instance.
template <typename T, int MAXT, bool ROWTILE, int IP = 0, bool SHIFT = false, bool QE2 = false>
__global__ void __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(3, 8)))
    k_step_batch(const InstDev *__restrict__ inst, int ninst, int nitems, int items_per_xcd,
                 int parity, int group) {
  extern __shared__ double red[];
  const int nunits = (nitems + group - 1) / group;
  const int span = items_per_xcd > 0 ? 8 * items_per_xcd : nunits;
  const int w = group > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  for (int it = blockIdx.x; it < span; it += gridDim.x) {
    const int unit = items_per_xcd > 0 ? (it & 7) * items_per_xcd + (it >> 3) : it;
    const int item = unit * group + w;
    // uniform over the wave; over the workgroup too when group == 1, where
    // Q-slices synchronise (with group > 1 there is one slice and no barrier)
    if (item >= nitems) continue;
    int lo = 0, hi = ninst - 1;    // last instance with item0 <= item
    const InstDev CONSTANT_AS *ci = cst(inst);  // read-only table: scalar loads
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ci[mid].item0 <= item) lo = mid; else hi = mid - 1;
    }
    // Field-by-field reads through the constant address space keep every
    // value in SGPRs (a whole-struct copy would go through private memory).
    const InstDev CONSTANT_AS &d = ci[lo];
    StepParams pp;
#define TPL_LD(f) pp.f = d.p.f;
    TPL_LD(nx) TPL_LD(ny) TPL_LD(nqd) TPL_LD(qs) TPL_LD(ntiles) TPL_LD(tiles_per_xcd)
    TPL_LD(y0) TPL_LD(N) TPL_LD(aS) TPL_LD(aP) TPL_LD(tJS) TPL_LD(tJP) TPL_LD(c1S)
    TPL_LD(c2S) TPL_LD(rS) TPL_LD(c1P) TPL_LD(c2P) TPL_LD(rP) TPL_LD(kappa) TPL_LD(DQ)
    TPL_LD(F0) TPL_LD(kf) TPL_LD(src)
#undef TPL_LD
    pp.wg = 0;
    pp.gate = nullptr;
    pp.qe = QE2 ? 2 : 1;
    pp.shift = 0;
    if constexpr (QE2) {
      pp.pS = d.p.pS;
      pp.pP = d.p.pP;
    } else {
      pp.pS = pp.pP = 0.0;
    }
    const int rd = parity ^ d.cur0;
    const StateT<T> a{static_cast<T *>(d.XS[rd]), static_cast<T *>(d.XP[rd]),
                      static_cast<T *>(d.PSI[rd]), d.FLD[rd]};
    const StateT<T> b{static_cast<T *>(d.XS[rd ^ 1]), static_cast<T *>(d.XP[rd ^ 1]),
                      static_cast<T *>(d.PSI[rd ^ 1]), d.FLD[rd ^ 1]};
    step_tile<T, ROWTILE, false, QE2, IP, SHIFT>(pp, a, b, d.rpull, d.rstore, d.rpsi,
                                                   d.rspull, d.rsstore, d.qtab, item - d.item0,
                                                   red);
  }
}

template <typename T>
hipError_t launch_step_batch(const InstDev *inst, int ninst, int nitems, int qs, int grid,
                             bool rowtile, int parity, hipStream_t s, int group, int ip,
                             bool shift, bool qe2) {
  if (group < 1 || (group > 1 && qs != 1) || qs * group > 8) return hipErrorInvalidValue;
  const size_t lds = qs > 1 ? (size_t)qs * 12 * 64 * sizeof(double) : 0;
  const int nunits = (nitems + group - 1) / group;
  const int per_xcd = (grid % 8 == 0 && nunits >= 64) ? (nunits + 7) / 8 : 0;
  const dim3 g(grid), blk(64 * qs * group);
  if (qe2) {
    // model (ii): two arrays or in place, Taylor form of the spring term
    if (shift) return hipErrorInvalidValue;
    if (ip != 0) {
      if ((ip != 1 && ip != 2) || qs != 1 || !rowtile) return hipErrorInvalidValue;
#define TPL_BATCH_IP2(MAXT, IP)                                                               \
  hipLaunchKernelGGL((k_step_batch<T, MAXT, true, IP, false, true>), g, blk, lds, s, inst,   \
                     ninst, nitems, per_xcd, parity, group)
      if (group <= 4) {
        if (ip == 1) TPL_BATCH_IP2(256, 1); else TPL_BATCH_IP2(256, 2);
      } else {
        if (ip == 1) TPL_BATCH_IP2(512, 1); else TPL_BATCH_IP2(512, 2);
      }
#undef TPL_BATCH_IP2
      return hipGetLastError();
    }
#define TPL_BATCH_QE2(MAXT, RT)                                                               \
  hipLaunchKernelGGL((k_step_batch<T, MAXT, RT, 0, false, true>), g, blk, lds, s, inst, ninst, \
                     nitems, per_xcd, parity, group)
    if (qs * group <= 4) {
      if (rowtile) TPL_BATCH_QE2(256, true); else TPL_BATCH_QE2(256, false);
    } else {
      if (rowtile) TPL_BATCH_QE2(512, true); else TPL_BATCH_QE2(512, false);
    }
#undef TPL_BATCH_QE2
    return hipGetLastError();
  }
  if (shift && ip != 0) {
    // the shifted spring term streamed in place: whole tiles, one Q-slice
    if ((ip != 1 && ip != 2) || qs != 1 || !rowtile) return hipErrorInvalidValue;
#define TPL_BATCH_IPSH(MAXT, IP)                                                            \
  hipLaunchKernelGGL((k_step_batch<T, MAXT, true, IP, true>), g, blk, lds, s, inst, ninst, \
                     nitems, per_xcd, parity, group)
    if (group <= 4) {
      if (ip == 1) TPL_BATCH_IPSH(256, 1); else TPL_BATCH_IPSH(256, 2);
    } else {
      if (ip == 1) TPL_BATCH_IPSH(512, 1); else TPL_BATCH_IPSH(512, 2);
    }
#undef TPL_BATCH_IPSH
    return hipGetLastError();
  }
  if (shift) {
    // the shifted spring term, two arrays
#define TPL_BATCH_SH(MAXT, RT)                                                          \
  hipLaunchKernelGGL((k_step_batch<T, MAXT, RT, 0, true>), g, blk, lds, s, inst, ninst, nitems, \
                     per_xcd, parity, group)
    if (qs * group <= 4) {
      if (rowtile) TPL_BATCH_SH(256, true); else TPL_BATCH_SH(256, false);
    } else {
      if (rowtile) TPL_BATCH_SH(512, true); else TPL_BATCH_SH(512, false);
    }
#undef TPL_BATCH_SH
    return hipGetLastError();
  }
  if (ip != 0) {
    // in place: whole tiles (nx a multiple of 64 for every instance), one Q-slice
    if ((ip != 1 && ip != 2) || qs != 1 || !rowtile) return hipErrorInvalidValue;
#define TPL_BATCH_IP(MAXT, IP)                                                          \
  hipLaunchKernelGGL((k_step_batch<T, MAXT, true, IP>), g, blk, lds, s, inst, ninst, nitems, \
                     per_xcd, parity, group)
    if (group <= 4) {
      if (ip == 1) TPL_BATCH_IP(256, 1); else TPL_BATCH_IP(256, 2);
    } else {
      if (ip == 1) TPL_BATCH_IP(512, 1); else TPL_BATCH_IP(512, 2);
    }
#undef TPL_BATCH_IP
    return hipGetLastError();
  }
  if (qs * group <= 4) {
    if (rowtile)
      hipLaunchKernelGGL((k_step_batch<T, 256, true>), g, blk, lds, s, inst, ninst, nitems,
                         per_xcd, parity, group);
    else
      hipLaunchKernelGGL((k_step_batch<T, 256, false>), g, blk, lds, s, inst, ninst, nitems,
                         per_xcd, parity, group);
  } else {
    if (rowtile)
      hipLaunchKernelGGL((k_step_batch<T, 512, true>), g, blk, lds, s, inst, ninst, nitems,
                         per_xcd, parity, group);
    else
      hipLaunchKernelGGL((k_step_batch<T, 512, false>), g, blk, lds, s, inst, ninst, nitems,
                         per_xcd, parity, group);
  }
  return hipGetLastError();
}
template hipError_t launch_step_batch<double>(const InstDev *, int, int, int, int, bool, int,
                                              hipStream_t, int, int, bool, bool);
template hipError_t launch_step_batch<float>(const InstDev *, int, int, int, int, bool, int,
                                             hipStream_t, int, int, bool, bool);

template <typename T>
hipError_t launch_step(const StepParams &p, StateT<T> a, StateT<T> b,
                       StepRef r, const QNode *qtab, hipStream_t s, bool b16, int ip) {
  const int gsize = p.wg ? (p.wg & 255) * ((p.wg >> 8) & 255) : 1;
  const int grid = p.tiles_per_xcd > 0 ? 8 * p.tiles_per_xcd : p.ntiles / gsize;
  const size_t lds = p.qs > 1 ? (size_t)p.qs * 12 * 64 * sizeof(double) : 0;
  const bool rowtile = (p.nx % 64) == 0;
  if (p.wg && (p.qs != 1 || !rowtile || gsize > 8)) return hipErrorInvalidValue;
  if (p.qe != 1 && p.qe != 2) return hipErrorInvalidValue;
  const dim3 g(grid), blk(64 * p.qs * gsize);
#define TPL_STEP_ARGS p, a, b, r.pull, r.store, r.psi, r.spull, r.sstore, qtab
  if (p.shift != 0 && p.shift != 1) return hipErrorInvalidValue;
  if (p.shift && ip != 0) {
    // shifted spring term streamed in place: whole tiles, one Q-slice
    if (ip != 1 && ip != 2) return hipErrorInvalidValue;
    if (b16 || !rowtile || p.qs != 1 || a.XS != b.XS || a.XP != b.XP) return hipErrorInvalidValue;
#define TPL_STEP_IPSH(QE2, IP)                                                          \
  if (gsize <= 4)                                                                       \
    hipLaunchKernelGGL((k_step<T, 256, true, false, QE2, IP, true>), g, blk, lds, s,    \
                       TPL_STEP_ARGS);                                                  \
  else                                                                                  \
    hipLaunchKernelGGL((k_step<T, 512, true, false, QE2, IP, true>), g, blk, lds, s,    \
                       TPL_STEP_ARGS);
    if (p.qe == 2) {
      if (ip == 1) { TPL_STEP_IPSH(true, 1) } else { TPL_STEP_IPSH(true, 2) }
    } else {
      if (ip == 1) { TPL_STEP_IPSH(false, 1) } else { TPL_STEP_IPSH(false, 2) }
    }
#undef TPL_STEP_IPSH
    return hipGetLastError();
  }
  if (p.shift) {
    // non-local spring term, two arrays: FP64 and FP32 storage
    if (b16) return hipErrorInvalidValue;
#define TPL_STEP_SH(MAXT, RT)                                                                 \
  if (p.qe == 2)                                                                             \
    hipLaunchKernelGGL((k_step<T, MAXT, RT, false, true, 0, true>), g, blk, lds, s,          \
                       TPL_STEP_ARGS);                                                       \
  else                                                                                       \
    hipLaunchKernelGGL((k_step<T, MAXT, RT, false, false, 0, true>), g, blk, lds, s,         \
                       TPL_STEP_ARGS);
    if (p.qs * gsize <= 4) {
      if (rowtile) { TPL_STEP_SH(256, true) } else { TPL_STEP_SH(256, false) }
    } else {
      if (rowtile) { TPL_STEP_SH(512, true) } else { TPL_STEP_SH(512, false) }
    }
#undef TPL_STEP_SH
    return hipGetLastError();
  }
  if (ip != 0) {
    // in place: one population array, whole tiles, one Q-slice
    if (ip != 1 && ip != 2) return hipErrorInvalidValue;
    if (b16 || !rowtile || p.qs != 1 || a.XS != b.XS || a.XP != b.XP) return hipErrorInvalidValue;
#define TPL_STEP_IP(QE2, IP)                                                           \
  if (gsize <= 4)                                                                      \
    hipLaunchKernelGGL((k_step<T, 256, true, false, QE2, IP>), g, blk, lds, s, TPL_STEP_ARGS); \
  else                                                                                 \
    hipLaunchKernelGGL((k_step<T, 512, true, false, QE2, IP>), g, blk, lds, s, TPL_STEP_ARGS);
    if (p.qe == 2) {
      if (ip == 1) { TPL_STEP_IP(true, 1) } else { TPL_STEP_IP(true, 2) }
    } else {
      if (ip == 1) { TPL_STEP_IP(false, 1) } else { TPL_STEP_IP(false, 2) }
    }
#undef TPL_STEP_IP
    return hipGetLastError();
  }
#define TPL_STEP_LAUNCH2(B16, QE2)                                                    \
  if (p.qs * gsize <= 4) {                                                            \
    if (rowtile)                                                                      \
      hipLaunchKernelGGL((k_step<T, 256, true, B16, QE2>), g, blk, lds, s, TPL_STEP_ARGS);  \
    else                                                                              \
      hipLaunchKernelGGL((k_step<T, 256, false, B16, QE2>), g, blk, lds, s, TPL_STEP_ARGS); \
  } else {                                                                            \
    if (rowtile)                                                                      \
      hipLaunchKernelGGL((k_step<T, 512, true, B16, QE2>), g, blk, lds, s, TPL_STEP_ARGS);  \
    else                                                                              \
      hipLaunchKernelGGL((k_step<T, 512, false, B16, QE2>), g, blk, lds, s, TPL_STEP_ARGS); \
  }
#define TPL_STEP_LAUNCH(B16)     \
  if (p.qe == 2) {               \
    TPL_STEP_LAUNCH2(B16, true)  \
  } else {                       \
    TPL_STEP_LAUNCH2(B16, false) \
  }
  if constexpr (std::is_same<T, float>::value) {
    if (b16) {
      TPL_STEP_LAUNCH(true)
    } else {
      TPL_STEP_LAUNCH(false)
    }
  } else {
    if (b16) return hipErrorInvalidValue;
    TPL_STEP_LAUNCH(false)
  }
#undef TPL_STEP_LAUNCH
#undef TPL_STEP_LAUNCH2
#undef TPL_STEP_ARGS
  return hipGetLastError();
}
template hipError_t launch_step<double>(const StepParams &, StateT<double>, StateT<double>,
                                        StepRef, const QNode *, hipStream_t, bool, int);
template hipError_t launch_step<float>(const StepParams &, StateT<float>, StateT<float>,
                                       StepRef, const QNode *, hipStream_t, bool, int);

// Same-step gradients: before the step, the read half's recorded psi, M and
// U are replaced by this step's (the step then reads them where it would
// read the previous step's): psi^n(r, Q) of the pulled populations, one
// thread per (r, Q)-node; M^n = sum_Q psi^n Q Fhat^T per r-node; U^n, the
// mixture velocity with the spring-stress divergence of M^n, per r-node.
// ip selects the pull of the in-place steps as in step_tile.
template <typename T>
__device__ __forceinline__ void pre_psi_node(const StepParams &p, const StateT<T> &a,
                                             const float *rpull, const float *rpsi,
                                             const QNode *qtab, int ip, int r, int q) {
  constexpr bool F32 = std::is_same<T, float>::value;
  constexpr uint32_t SZ = sizeof(T);
  const long long N = p.N;
  const int nx = p.nx, ny = p.ny, nqd = p.nqd;
  const int y = r / nx, x = r - y * nx;
  const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
  const QNode CONSTANT_AS &qn = cst(qtab)[q];
  double psi = 0.0;
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    const int d = pdir(k);
    const int sx = C9X[d] == 1 ? xm : (C9X[d] == -1 ? xp : x);
    const int sy = C9Y[d] == 1 ? ym : (C9Y[d] == -1 ? yp : y);
    const T *pl = ip == 2 ? a.XP + (size_t)(krev(k) * nqd + q) * N : a.XP + (size_t)qn.plane[k] * N;
    const uint32_t off = SZ * (uint32_t)(ip == 2 ? r : sy * nx + sx);
    const double ref = F32 ? (double)rpull[((size_t)y * nqd + q) * 25 + k] : 0.0;
    psi += full(ldo(pl, off), ref);
  }
  sto(a.PSI + (size_t)q * N, SZ * (uint32_t)r,
      stored<T>(psi, F32 ? (double)rpsi[(size_t)y * nqd + q] : 0.0));
}

template <typename T>
__device__ __forceinline__ void pre_m_node(const StepParams &p, const StateT<T> &a,
                                           const float *rpsi, const QNode *qtab, int r) {
  constexpr bool F32 = std::is_same<T, float>::value;
  const long long N = p.N;
  const int y = r / p.nx;
  double Mxx = 0.0, Mxy = 0.0, Myy = 0.0;
  for (int q = 0; q < p.nqd; ++q) {
    const double psi = full(a.PSI[(size_t)q * N + r], F32 ? (double)rpsi[(size_t)y * p.nqd + q] : 0.0);
    const QNode CONSTANT_AS &qn = cst(qtab)[q];
    Mxx += psi * qn.qx * qn.fx;
    Mxy += psi * qn.qx * qn.fy;
    Myy += psi * qn.qy * qn.fy;
  }
  a.FLD[(size_t)F_MXX * N + r] = Mxx;
  a.FLD[(size_t)F_MXY * N + r] = Mxy;
  a.FLD[(size_t)F_MYY * N + r] = Myy;
}

template <typename T>
__device__ __forceinline__ void pre_u_node(const StepParams &p, const StateT<T> &a,
                                           const float *rspull, int ip, int r) {
  constexpr bool F32 = std::is_same<T, float>::value;
  const long long N = p.N;
  const int nx = p.nx, ny = p.ny;
  const int y = r / nx, x = r - y * nx;
  const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
  const double *G = a.FLD;
  double rhoS = 0.0, JSx = 0.0, JSy = 0.0, rhoP = 0.0, JPx = 0.0, JPy = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int sx = C9X[d] == 1 ? xm : (C9X[d] == -1 ? xp : x);
    const int sy = C9Y[d] == 1 ? ym : (C9Y[d] == -1 ? yp : y);
    const size_t src = (size_t)sy * nx + sx;
    const size_t sp = ip == 2 ? (size_t)rev9(d) * N + r : (size_t)d * N + src;
    const double g = full(a.XS[sp], F32 ? (double)rspull[(size_t)y * 9 + d] : 0.0);
    rhoS += g;
    if (C9X[d]) JSx += C9X[d] * g;
    if (C9Y[d]) JSy += C9Y[d] * g;
    const double m = G[(size_t)(F_M0 + d) * N + src];
    rhoP += m;
    if (C9X[d]) JPx += C9X[d] * m;
    if (C9Y[d]) JPy += C9Y[d] * m;
  }
  auto dX = [&](int f) {
    return 0.5 * (G[(size_t)f * N + (size_t)y * nx + xp] - G[(size_t)f * N + (size_t)y * nx + xm]);
  };
  auto dY = [&](int f) {
    return 0.5 * (G[(size_t)f * N + (size_t)yp * nx + x] - G[(size_t)f * N + (size_t)ym * nx + x]);
  };
  // Taylor form: kappa div M of this step's M; shifted form: the Q-sum the
  // spring-sum pass formed from this step's psi (F_MXX, F_MXY slots)
  const double Sx = p.shift ? G[(size_t)F_MXX * N + r] : p.kappa * (dX(F_MXX) + dY(F_MXY));
  const double Sy = p.shift ? G[(size_t)F_MXY * N + r] : p.kappa * (dX(F_MXY) + dY(F_MYY));
  double Fbx = p.F0 * sin(p.kf * (double)(y + p.y0)), Fby = 0.0;
  if (p.src != nullptr) {
    Fbx += p.src[r];
    Fby = p.src[N + r];
  }
  double Ux, Uy;
  mixture_velocity(p, rhoS, JSx, JSy, rhoP, JPx, JPy, Sx, Sy, Fbx, Fby, Ux, Uy);
  a.FLD[(size_t)F_UX * N + r] = Ux;
  a.FLD[(size_t)F_UY * N + r] = Uy;
}

template <typename T>
__global__ void k_pre_psi(StepParams p, StateT<T> a, const float *__restrict__ rpull,
                          const float *__restrict__ rpsi, const QNode *__restrict__ qtab, int ip) {
  const long long rr = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= p.N) return;
  pre_psi_node<T>(p, a, rpull, rpsi, qtab, ip, (int)rr, blockIdx.y);
}

template <typename T>
__global__ void k_pre_m(StepParams p, StateT<T> a, const float *__restrict__ rpsi,
                        const QNode *__restrict__ qtab) {
  const long long rr = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= p.N) return;
  pre_m_node<T>(p, a, rpsi, qtab, (int)rr);
}

template <typename T>
__global__ void k_pre_u(StepParams p, StateT<T> a, const float *__restrict__ rspull, int ip) {
  const long long rr = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= p.N) return;
  pre_u_node<T>(p, a, rspull, ip, (int)rr);
}

// The same three passes over every item (64-node tile) of a batch; the read
// half of each instance chosen by parity as in k_step_batch.  One wave per
// item (and Q-node for the psi pass), items walked with the grid's stride.
__device__ __forceinline__ int batch_instance(const InstDev CONSTANT_AS *ci, int ninst,
                                              int item) {
  int lo = 0, hi = ninst - 1;  // last instance with item0 <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ci[mid].item0 <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}
template <typename T>
__device__ __forceinline__ StateT<T> batch_half(const InstDev &d, int h) {
  return StateT<T>{static_cast<T *>(d.XS[h]), static_cast<T *>(d.XP[h]),
                   static_cast<T *>(d.PSI[h]), d.FLD[h]};
}

template <typename T>
__global__ void k_pre_psi_batch(const InstDev *__restrict__ inst, int ninst, int nitems,
                                int parity, int ip) {
  const InstDev CONSTANT_AS *ci = cst(inst);
  const int q = blockIdx.y;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const InstDev &d = inst[batch_instance(ci, ninst, item)];
    const StepParams pp = d.p;
    if (q >= pp.nqd) continue;
    const long long rr = (long long)(item - d.item0) * 64 + threadIdx.x;
    if (rr < pp.N)
      pre_psi_node<T>(pp, batch_half<T>(d, parity ^ d.cur0), d.rpull, d.rpsi, d.qtab, ip,
                      (int)rr, q);
  }
}

template <typename T>
__global__ void k_pre_m_batch(const InstDev *__restrict__ inst, int ninst, int nitems,
                              int parity) {
  const InstDev CONSTANT_AS *ci = cst(inst);
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const InstDev &d = inst[batch_instance(ci, ninst, item)];
    const StepParams pp = d.p;
    const long long rr = (long long)(item - d.item0) * 64 + threadIdx.x;
    if (rr < pp.N) pre_m_node<T>(pp, batch_half<T>(d, parity ^ d.cur0), d.rpsi, d.qtab, (int)rr);
  }
}

template <typename T>
__global__ void k_pre_u_batch(const InstDev *__restrict__ inst, int ninst, int nitems,
                              int parity, int ip) {
  const InstDev CONSTANT_AS *ci = cst(inst);
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const InstDev &d = inst[batch_instance(ci, ninst, item)];
    const StepParams pp = d.p;
    const long long rr = (long long)(item - d.item0) * 64 + threadIdx.x;
    if (rr < pp.N) pre_u_node<T>(pp, batch_half<T>(d, parity ^ d.cur0), d.rspull, ip, (int)rr);
  }
}

template <typename T>
hipError_t launch_spring_sum_batch(const InstDev *inst, int ninst, int nitems, int grid,
                                   int parity, hipStream_t s);

template <typename T>
hipError_t launch_same_step_fields_batch(const InstDev *inst, int ninst, int nitems, int nqd,
                                         int parity, int ip, bool shift, hipStream_t s) {
  if (ip < 0 || ip > 2 || nitems < 1 || nqd < 1 || nqd > 65535) return hipErrorInvalidValue;
  const unsigned g = (unsigned)(nitems < 16384 ? nitems : 16384);
  hipLaunchKernelGGL(k_pre_psi_batch<T>, dim3(g, (unsigned)nqd), dim3(64), 0, s, inst, ninst,
                     nitems, parity, ip);
  if (shift) {  // the Q-sum of the shifted spring term of this step's psi
    const hipError_t e =
        launch_spring_sum_batch<T>(inst, ninst, nitems, nitems < 4096 ? nitems : 4096, parity, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_pre_m_batch<T>, dim3(g), dim3(64), 0, s, inst, ninst, nitems, parity);
  }
  hipLaunchKernelGGL(k_pre_u_batch<T>, dim3(g), dim3(64), 0, s, inst, ninst, nitems, parity, ip);
  return hipGetLastError();
}
template hipError_t launch_same_step_fields_batch<double>(const InstDev *, int, int, int, int, int,
                                                          bool, hipStream_t);
template hipError_t launch_same_step_fields_batch<float>(const InstDev *, int, int, int, int, int,
                                                         bool, hipStream_t);

// One 64-node tile per workgroup, kSpringSlices waves each summing every
// kSpringSlices-th Q-node; the slices' partial sums are added in slice order
// (the same order for every lattice, so results do not depend on its size).
constexpr int kSpringSlices = 8;
template <typename T>
__global__ void __launch_bounds__(64 * kSpringSlices)
    k_spring_sum(StepParams p, StateT<T> a, const float *__restrict__ rpsi,
                 const QNode *__restrict__ qtab) {
  constexpr bool F32 = std::is_same<T, float>::value;
  __shared__ double part[kSpringSlices][2][64];
  const long long N = p.N;
  const int lane = threadIdx.x & 63;
  const int slice = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long rr = (long long)blockIdx.x * 64 + lane;
  const int r = (int)(rr < N ? rr : N - 1);
  const int nx = p.nx, ny = p.ny, nqd = p.nqd;
  const int y = r / nx, x = r - y * nx;
  double Sx = 0.0, Sy = 0.0;
#pragma unroll 2
  for (int q = slice; q < nqd; q += kSpringSlices) {
    const QNode CONSTANT_AS &qn = cst(qtab)[q];
    const double d = spring_shift_diff(a.PSI + (size_t)q * N, x, y, nx, ny, qn.qx, qn.qy,
                                       [&](int row) {
                                         return F32 ? (double)rpsi[(size_t)row * nqd + q] : 0.0;
                                       });
    Sx += p.kappa * qn.fx * d;
    Sy += p.kappa * qn.fy * d;
  }
  part[slice][0][lane] = Sx;
  part[slice][1][lane] = Sy;
  __syncthreads();
  if (slice == 0 && rr < N) {
    for (int s2 = 1; s2 < kSpringSlices; ++s2) {
      Sx += part[s2][0][lane];
      Sy += part[s2][1][lane];
    }
    a.FLD[(size_t)F_MXX * N + r] = Sx;
    a.FLD[(size_t)F_MXY * N + r] = Sy;
  }
}

template <typename T>
hipError_t launch_spring_sum(const StepParams &p, StateT<T> a, StepRef ref, const QNode *qtab,
                             hipStream_t s) {
  const unsigned nb = (unsigned)((p.N + 63) / 64);
  hipLaunchKernelGGL(k_spring_sum<T>, dim3(nb), dim3(64 * kSpringSlices), 0, s, p, a, ref.psi,
                     qtab);
  return hipGetLastError();
}
template hipError_t launch_spring_sum<double>(const StepParams &, StateT<double>, StepRef,
                                              const QNode *, hipStream_t);
template hipError_t launch_spring_sum<float>(const StepParams &, StateT<float>, StepRef,
                                             const QNode *, hipStream_t);

// The same Q-sum for every item (64-node tile) of a batch, the read half of
// each instance chosen by parity as in k_step_batch.
template <typename T>
__global__ void __launch_bounds__(64 * kSpringSlices)
    k_spring_sum_batch(const InstDev *__restrict__ inst, int ninst, int nitems, int parity) {
  constexpr bool F32 = std::is_same<T, float>::value;
  __shared__ double part[kSpringSlices][2][64];
  const int lane = threadIdx.x & 63;
  const int slice = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const InstDev CONSTANT_AS *ci = cst(inst);
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    int lo = 0, hi = ninst - 1;  // last instance with item0 <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ci[mid].item0 <= item) lo = mid; else hi = mid - 1;
    }
    const InstDev CONSTANT_AS &d = ci[lo];
    const long long N = d.p.N;
    const int nx = d.p.nx, ny = d.p.ny, nqd = d.p.nqd;
    const double kappa = d.p.kappa;
    const int rd = parity ^ d.cur0;
    const T *PSI = static_cast<const T *>(d.PSI[rd]);
    double *FLD = d.FLD[rd];
    const float *rpsi = d.rpsi;
    const QNode *qtab = d.qtab;
    const long long rr = (long long)(item - d.item0) * 64 + lane;
    const int r = (int)(rr < N ? rr : N - 1);
    const int y = r / nx, x = r - y * nx;
    double Sx = 0.0, Sy = 0.0;
#pragma unroll 2
    for (int q = slice; q < nqd; q += kSpringSlices) {
      const QNode CONSTANT_AS &qn = cst(qtab)[q];
      const double dd = spring_shift_diff(PSI + (size_t)q * N, x, y, nx, ny, qn.qx, qn.qy,
                                          [&](int row) {
                                            return F32 ? (double)rpsi[(size_t)row * nqd + q] : 0.0;
                                          });
      Sx += kappa * qn.fx * dd;
      Sy += kappa * qn.fy * dd;
    }
    part[slice][0][lane] = Sx;
    part[slice][1][lane] = Sy;
    __syncthreads();
    if (slice == 0 && rr < N) {
      for (int s2 = 1; s2 < kSpringSlices; ++s2) {
        Sx += part[s2][0][lane];
        Sy += part[s2][1][lane];
      }
      FLD[(size_t)F_MXX * N + r] = Sx;
      FLD[(size_t)F_MXY * N + r] = Sy;
    }
    __syncthreads();  // part is reused by the next item
  }
}

template <typename T>
hipError_t launch_spring_sum_batch(const InstDev *inst, int ninst, int nitems, int grid,
                                   int parity, hipStream_t s) {
  if (grid < 1 || nitems < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_spring_sum_batch<T>, dim3(grid), dim3(64 * kSpringSlices), 0, s, inst,
                     ninst, nitems, parity);
  return hipGetLastError();
}
template hipError_t launch_spring_sum_batch<double>(const InstDev *, int, int, int, int,
                                                    hipStream_t);
template hipError_t launch_spring_sum_batch<float>(const InstDev *, int, int, int, int,
                                                   hipStream_t);

template <typename T>
hipError_t launch_same_step_fields(const StepParams &p, StateT<T> a, StepRef ref,
                                   const QNode *qtab, hipStream_t s, int ip) {
  if (ip < 0 || ip > 2 || p.nqd < 1 || p.nqd > 65535) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)((p.N + 255) / 256);
  hipLaunchKernelGGL(k_pre_psi<T>, dim3(nb, (unsigned)p.nqd), dim3(256), 0, s, p, a, ref.pull,
                     ref.psi, qtab, ip);
  if (p.shift) {  // the Q-sum of the shifted spring term of this step's psi
    const hipError_t e = launch_spring_sum<T>(p, a, ref, qtab, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_pre_m<T>, dim3(nb), dim3(256), 0, s, p, a, ref.psi, qtab);
  }
  hipLaunchKernelGGL(k_pre_u<T>, dim3(nb), dim3(256), 0, s, p, a, ref.spull, ip);
  return hipGetLastError();
}
template hipError_t launch_same_step_fields<double>(const StepParams &, StateT<double>, StepRef,
                                                    const QNode *, hipStream_t, int);
template hipError_t launch_same_step_fields<float>(const StepParams &, StateT<float>, StepRef,
                                                   const QNode *, hipStream_t, int);

// BF16 form: conversions of the polymer populations to and from FP32
// deviations ([25][nqd][N] floats).  Velocities 1..24 are BF16 planes; the
// rest population (velocity 0, which never leaves its node) is kept in full
// FP32, its upper 16 bits in plane 0 and its lower 16 in plane 25, and
// carries the node's rounding residual: the 24 deviations lost to BF16
// rounding are added to it, so the node's density (and the lattice's mass)
// is stored to FP32 accuracy.
__device__ __forceinline__ double rest_with_residual(double rest, const double *d) {
  double e = 0.0;
#pragma unroll
  for (int k = 1; k < 25; ++k) e += d[k] - from_bf16(to_bf16(d[k]));
  return rest + e;
}

__global__ void k_bf16_decode(long long nq, const uint16_t *__restrict__ src,
                              float *__restrict__ dev) {
  // one thread per (Q-node, r) pair; nq = nqd N
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= nq) return;
  dev[j] = __uint_as_float(((uint32_t)src[j] << 16) | (uint32_t)src[25 * nq + j]);
#pragma unroll 4
  for (int k = 1; k < 25; ++k) dev[k * nq + j] = (float)from_bf16(src[k * nq + j]);
}

__global__ void k_bf16_encode(long long nq, const float *__restrict__ dev,
                              uint16_t *__restrict__ dst) {
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= nq) return;
  double d[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) d[k] = dev[k * nq + j];
#pragma unroll
  for (int k = 1; k < 25; ++k) dst[k * nq + j] = to_bf16(d[k]);
  const uint32_t u = __float_as_uint((float)rest_with_residual(d[0], d));
  dst[j] = (uint16_t)(u >> 16);
  dst[25 * nq + j] = (uint16_t)(u & 0xffffu);
}

hipError_t launch_bf16_decode(int nqd, long long N, StateT<float> a, float *dev, hipStream_t s) {
  const long long nq = N * nqd;
  hipLaunchKernelGGL(k_bf16_decode, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nq,
                     reinterpret_cast<const uint16_t *>(a.XP), dev);
  return hipGetLastError();
}
hipError_t launch_bf16_encode(int nqd, long long N, const float *dev, StateT<float> a,
                              hipStream_t s) {
  const long long nq = N * nqd;
  hipLaunchKernelGGL(k_bf16_encode, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nq, dev,
                     reinterpret_cast<uint16_t *>(a.XP));
  return hipGetLastError();
}

// FP32 form reference: ref[plane][y] = (float) column[plane][y] for the 9
// solvent, 25 nqd polymer and nqd psi planes.
__global__ void k_make_ref(int nqd, int ny, StateView col, float *__restrict__ ref) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = blockIdx.y;
  if (y >= ny) return;
  double v;
  if (plane < 9)
    v = col.XS[(size_t)plane * ny + y];
  else if (plane < 9 + 25 * nqd)
    v = col.XP[(size_t)(plane - 9) * ny + y];
  else
    v = col.PSI[(size_t)(plane - 9 - 25 * nqd) * ny + y];
  ref[(size_t)plane * ny + y] = (float)v;
}
hipError_t launch_make_ref(int nqd, int ny, StateView col, float *ref, hipStream_t s) {
  hipLaunchKernelGGL(k_make_ref, dim3((ny + 255) / 256, 9 + 26 * nqd), dim3(256), 0, s, nqd,
                     ny, col, ref);
  return hipGetLastError();
}

// Regroup the reference for the step kernel (one thread per (y, q)).
__global__ void k_step_ref(int nqd, int ny, const QNode *__restrict__ qtab, RefView ref,
                           float *__restrict__ pull, float *__restrict__ store,
                           float *__restrict__ psi, float *__restrict__ spull,
                           float *__restrict__ sstore) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ny * nqd) return;
  const int y = i / nqd, q = i - y * nqd;
  for (int k = 0; k < 25; ++k) {
    const int sy = ((y - PV[k][1]) % ny + ny) % ny;
    pull[(size_t)i * 25 + k] = ref.XP[(size_t)qtab[q].plane[k] * ny + sy];
    store[(size_t)i * 25 + k] = ref.XP[((size_t)k * nqd + q) * ny + y];
  }
  psi[i] = ref.PSI[(size_t)q * ny + y];
  if (q == 0) {
    for (int d = 0; d < 9; ++d) {
      const int sy = ((y - C9Y[d]) % ny + ny) % ny;
      spull[(size_t)y * 9 + d] = ref.XS[(size_t)d * ny + sy];
      sstore[(size_t)y * 9 + d] = ref.XS[(size_t)d * ny + y];
    }
  }
}
hipError_t launch_step_ref(int nqd, int ny, const QNode *qtab, RefView ref, float *pull,
                           float *store, float *psi, float *spull, float *sstore,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_step_ref, dim3((ny * nqd + 255) / 256), dim3(256), 0, s, nqd, ny, qtab,
                     ref, pull, store, psi, spull, sstore);
  return hipGetLastError();
}

// Deviation of the column from the reference, copied to every x.
__global__ void k_tile_dev(int nx, int ny, const double *__restrict__ col,
                           const float *__restrict__ ref, float *__restrict__ dst) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t plane = blockIdx.y;
  if (r >= N) return;
  const int y = (int)(r / nx);
  dst[plane * N + r] = (float)(col[plane * ny + y] - (double)ref[plane * ny + y]);
}
hipError_t launch_tile_dev(int planes, int nx, int ny, const double *col, const float *ref,
                           float *dst, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_tile_dev, dim3((unsigned)((N + 255) / 256), planes), dim3(256), 0, s,
                     nx, ny, col, ref, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial-state kernels.

// Rest (FP64 column): solvent equilibrium at zero velocity; polymer rest
// distribution; zero lagged velocity.
__global__ void k_rest(int nqd, long long N, double rhoS0, double rhoP0,
                       const double *__restrict__ peq, StateView a) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = blockIdx.y;  // 0..8 solvent, then 25*nqd polymer, then psi
  if (r >= N) return;
  if (plane < 9) {
    a.XS[(size_t)plane * N + r] = W9[plane] * rhoS0;
  } else if (plane < 9 + 25 * nqd) {
    const int kq = plane - 9, k = kq / nqd, q = kq - k * nqd;
    a.XP[(size_t)kq * N + r] = (k == 0 ? 1.0 / 3.0 : 1.0 / 36.0) * rhoP0 * peq[q];
  } else {
    const int q = plane - 9 - 25 * nqd;
    a.PSI[(size_t)q * N + r] = rhoP0 * peq[q];
    if (q == 0) {
      a.FLD[(size_t)F_UX * N + r] = 0.0;
      a.FLD[(size_t)F_UY * N + r] = 0.0;
    }
  }
}

hipError_t launch_rest(int nqd, long long N, double rhoS0, double rhoP0,
                       const double *peq, StateView a, hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), 9 + 26 * nqd);
  hipLaunchKernelGGL(k_rest, grid, dim3(256), 0, s, nqd, N, rhoS0, rhoP0, peq,
                     a);
  return hipGetLastError();
}

// Recompute every per-node field except U from the populations and psi of
// the same half (used after any direct change of the state).
template <typename T>
__global__ void k_refresh(int nqd, int nx, int ny, const QNode *__restrict__ qtab,
                          StateT<T> a, RefView ref) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int y = (int)(r / nx);
  constexpr bool F32 = std::is_same<T, float>::value;
  auto rv = [&](const float *tab, long long pl) { return F32 ? (double)tab[(size_t)pl * ny + y] : 0.0; };
  double rs = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const double v = full(a.XS[(size_t)d * N + r], rv(ref.XS, d));
    rs += v;
    jx += C9X[d] * v;
    jy += C9Y[d] * v;
  }
  double mg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double Mxx = 0.0, Mxy = 0.0, Myy = 0.0;
  for (int q = 0; q < nqd; ++q) {
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      const long long pl = (long long)k * nqd + q;
      mg[pdir(k)] += full(a.XP[(size_t)pl * N + r], rv(ref.XP, pl));
    }
    const double ps = full(a.PSI[(size_t)q * N + r], rv(ref.PSI, q));
    Mxx += ps * qtab[q].qx * qtab[q].fx;
    Mxy += ps * qtab[q].qx * qtab[q].fy;
    Myy += ps * qtab[q].qy * qtab[q].fy;
  }
  double rp = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) rp += mg[d];
  double *G = a.FLD;
  G[(size_t)F_RHOS * N + r] = rs;
  G[(size_t)F_RHOP * N + r] = rp;
  G[(size_t)F_JSX * N + r] = jx;
  G[(size_t)F_JSY * N + r] = jy;
  G[(size_t)F_MXX * N + r] = Mxx;
  G[(size_t)F_MXY * N + r] = Mxy;
  G[(size_t)F_MYY * N + r] = Myy;
#pragma unroll
  for (int d = 0; d < 9; ++d) G[(size_t)(F_M0 + d) * N + r] = mg[d];
}

template <typename T>
hipError_t launch_refresh(int nqd, int nx, int ny, const QNode *qtab,
                          StateT<T> a, RefView ref, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_refresh<T>, dim3((unsigned)((N + 255) / 256)), dim3(256),
                     0, s, nqd, nx, ny, qtab, a, ref);
  return hipGetLastError();
}
template hipError_t launch_refresh<double>(int, int, int, const QNode *, StateT<double>,
                                           RefView, hipStream_t);
template hipError_t launch_refresh<float>(int, int, int, const QNode *, StateT<float>,
                                          RefView, hipStream_t);

// Copy an x-invariant column (nx = 1 lattice) to every column.
__global__ void k_tile(int nx, int ny, const double *__restrict__ col,
                       double *__restrict__ dst) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t plane = blockIdx.y;
  if (r >= N) return;
  const int y = (int)(r / nx);
  dst[plane * N + r] = col[plane * ny + y];
}

hipError_t launch_tile(int nqd, int nx, int ny, StateView col, StateView a,
                       hipStream_t s) {
  const long long N = (long long)nx * ny;
  const unsigned gx = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_tile, dim3(gx, 9), dim3(256), 0, s, nx, ny, col.XS, a.XS);
  hipLaunchKernelGGL(k_tile, dim3(gx, 25 * nqd), dim3(256), 0, s, nx, ny,
                     col.XP, a.XP);
  hipLaunchKernelGGL(k_tile, dim3(gx, nqd), dim3(256), 0, s, nx, ny, col.PSI,
                     a.PSI);
  hipLaunchKernelGGL(k_tile, dim3(gx, NF), dim3(256), 0, s, nx, ny, col.FLD,
                     a.FLD);
  return hipGetLastError();
}

hipError_t launch_tile_fields(int nx, int ny, const double *colFLD,
                              double *FLD, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_tile, dim3((unsigned)((N + 255) / 256), NF), dim3(256), 0,
                     s, nx, ny, colFLD, FLD);
  return hipGetLastError();
}

// Whole-array conversions for the FP32 form.
__global__ void k_to_f64(int nx, int ny, const float *__restrict__ src,
                         const float *__restrict__ ref, double *__restrict__ dst) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t plane = blockIdx.y;
  if (r >= N) return;
  dst[plane * N + r] = (double)ref[plane * ny + r / nx] + (double)src[plane * N + r];
}
__global__ void k_from_f64(int nx, int ny, const double *__restrict__ src,
                           const float *__restrict__ ref, float *__restrict__ dst) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t plane = blockIdx.y;
  if (r >= N) return;
  dst[plane * N + r] = (float)(src[plane * N + r] - (double)ref[plane * ny + r / nx]);
}
hipError_t launch_to_f64(int nx, int ny, int planes, const float *src,
                         const float *ref, double *dst, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((N + 255) / 256), planes), dim3(256),
                     0, s, nx, ny, src, ref, dst);
  return hipGetLastError();
}
hipError_t launch_from_f64(int nx, int ny, int planes, const double *src,
                           const float *ref, float *dst, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_from_f64, dim3((unsigned)((N + 255) / 256), planes), dim3(256),
                     0, s, nx, ny, src, ref, dst);
  return hipGetLastError();
}

// Divergence-free perturbation velocity.  modes[m] = (kx, ky, a, phase).
// Multimode: du = (d psi/dy, -d psi/dx) of psi = sum a cos(th),
// th = 2 pi (kx X/NX + ky Y/NY) + phase.  Single mode: du_y = amp_u0
// sin(2 pi X/NX + phase of mode 0).  partial[block] = sum |du|^2.
__global__ void k_perturb_field(int nx, int ny, int x0, int y0, int NX, int NY,
                                int nmodes, const double *__restrict__ modes,
                                double amp_u0, int multimode,
                                double *__restrict__ du,
                                double *__restrict__ partial) {
  __shared__ double sh[16];
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
  double ux = 0.0, uy = 0.0;
  if (r < N) {
    const int y = (int)(r / nx), x = (int)(r - (long long)y * nx);
    const double X = x + x0, Y = y + y0;
    const double twopi = 6.283185307179586476925286766559;
    if (multimode) {
      for (int m = 0; m < nmodes; ++m) {
        const double kx = modes[4 * m], ky = modes[4 * m + 1];
        const double th = twopi * (kx * X / NX + ky * Y / NY) + modes[4 * m + 3];
        const double sa = modes[4 * m + 2] * sin(th);
        ux += -sa * (twopi * ky / NY);
        uy += sa * (twopi * kx / NX);
      }
    } else {
      uy = amp_u0 * sin(twopi * X / NX + modes[3]);
    }
    du[r] = ux;
    du[N + r] = uy;
  }
  const double tot = block_sum(ux * ux + uy * uy, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

hipError_t launch_perturb_field(int nx, int ny, int x0, int y0, int NX, int NY,
                                int nmodes, const double *modes, double amp_u0,
                                int multimode, double *du, double *partial,
                                hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_perturb_field, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, nx, ny, x0, y0, NX, NY, nmodes, modes,
                     amp_u0, multimode, du, partial);
  return hipGetLastError();
}

// Add scale*du at first order to both species and to the lagged U.
template <typename T>
__global__ void k_perturb_apply(int nqd, int nx, int ny, const double *__restrict__ du,
                                const double *__restrict__ scale, StateT<T> a,
                                RefView ref) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int y = (int)(r / nx);
  constexpr bool F32 = std::is_same<T, float>::value;
  auto rv = [&](const float *tab, long long pl) { return F32 ? (double)tab[(size_t)pl * ny + y] : 0.0; };
  const double f = scale[0];
  const double dx = f * du[r], dy = f * du[N + r];
  double rs = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) rs += full(a.XS[(size_t)d * N + r], rv(ref.XS, d));
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    T &v = a.XS[(size_t)d * N + r];
    v = stored<T>(full(v, rv(ref.XS, d)) + 3.0 * W9[d] * rs * (C9X[d] * dx + C9Y[d] * dy),
                  rv(ref.XS, d));
  }
  for (int q = 0; q < nqd; ++q) {
    double ps = 0.0;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      const long long pl = (long long)k * nqd + q;
      ps += full(a.XP[(size_t)pl * N + r], rv(ref.XP, pl));
    }
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      if (PV[k][0] == 0 && PV[k][1] == 0) continue;
      const long long pl = (long long)k * nqd + q;
      T &v = a.XP[(size_t)pl * N + r];
      v = stored<T>(full(v, rv(ref.XP, pl)) +
                        3.0 * (1.0 / 36.0) * ps * (PV[k][0] * dx + PV[k][1] * dy),
                    rv(ref.XP, pl));
    }
  }
  a.FLD[(size_t)F_UX * N + r] += dx;
  a.FLD[(size_t)F_UY * N + r] += dy;
}

template <typename T>
hipError_t launch_perturb_apply(int nqd, int nx, int ny, const double *du,
                                const double *scale, StateT<T> a, RefView ref,
                                hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_perturb_apply<T>, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, nqd, nx, ny, du, scale, a, ref);
  return hipGetLastError();
}
template hipError_t launch_perturb_apply<double>(int, int, int, const double *,
                                                 const double *, StateT<double>, RefView,
                                                 hipStream_t);
template hipError_t launch_perturb_apply<float>(int, int, int, const double *,
                                                const double *, StateT<float>, RefView,
                                                hipStream_t);

// out[c] = sum_i partial[i*ncomp + c] (one workgroup, fixed order).
__global__ void k_sum(const double *__restrict__ partial, int n, int ncomp,
                      double *__restrict__ out) {
  __shared__ double sh[16];
  for (int c = 0; c < ncomp; ++c) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partial[(size_t)i * ncomp + c];
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) out[c] = t;
  }
}

hipError_t launch_sum(const double *partial, int n, int ncomp, double *out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partial, n, ncomp, out);
  return hipGetLastError();
}

// partial[y] = sum_x |U - <U>_x(y)|^2, one workgroup per row.
__global__ void k_amplitude_rows(int nx, int ny, const double *__restrict__ FLD,
                                 double *__restrict__ partial) {
  __shared__ double sh[16];
  const long long N = (long long)nx * ny;
  const int y = blockIdx.x;
  const double *ux = FLD + (size_t)F_UX * N + (size_t)y * nx;
  const double *uy = FLD + (size_t)F_UY * N + (size_t)y * nx;
  double sx = 0.0, sy = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) {
    sx += ux[x];
    sy += uy[x];
  }
  const double mx = block_sum(sx, sh) / nx;
  const double my = block_sum(sy, sh) / nx;
  double acc = 0.0;
  for (int x = threadIdx.x; x < nx; x += 256) {
    const double dx = ux[x] - mx, dy = uy[x] - my;
    acc += dx * dx + dy * dy;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[y] = t;
}

hipError_t launch_amplitude_rows(int nx, int ny, const double *FLD,
                                 double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_amplitude_rows, dim3(ny), dim3(256), 0, s, nx, ny, FLD,
                     partial);
  return hipGetLastError();
}

// Diagnostics, one partial per workgroup: masses, population momentum,
// enstrophy, sum psi |Q|^2, sum psi, min psi.
template <typename T>
__global__ void k_diag(int nx, int ny, int nqd, const QNode *__restrict__ qtab,
                       StateT<T> a, RefView ref, double *__restrict__ partial) {
  __shared__ double sh[16];
  constexpr bool F32 = std::is_same<T, float>::value;
  const long long N = (long long)nx * ny;
  double v[kDiagComp] = {0, 0, 0, 0, 0, 0, 0, 1e300};
  for (long long r = (long long)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (long long)gridDim.x * 256) {
    const double *G = a.FLD;
    v[0] += G[(size_t)F_RHOS * N + r];
    v[1] += G[(size_t)F_RHOP * N + r];
    double px = G[(size_t)F_JSX * N + r], py = G[(size_t)F_JSY * N + r];
#pragma unroll
    for (int d = 1; d < 9; ++d) {
      const double m = G[(size_t)(F_M0 + d) * N + r];
      px += C9X[d] * m;
      py += C9Y[d] * m;
    }
    v[2] += px;
    v[3] += py;
    const int y = (int)(r / nx), x = (int)(r - (long long)y * nx);
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const double *ux = G + (size_t)F_UX * N, *uy = G + (size_t)F_UY * N;
    const double w = 0.5 * (uy[(size_t)y * nx + xp] - uy[(size_t)y * nx + xm]) -
                     0.5 * (ux[(size_t)yp * nx + x] - ux[(size_t)ym * nx + x]);
    v[4] += 0.5 * w * w;
    for (int q = 0; q < nqd; ++q) {
      const double ps = full(a.PSI[(size_t)q * N + r], F32 ? (double)ref.PSI[(size_t)q * ny + y] : 0.0);
      v[5] += ps * (qtab[q].qx * qtab[q].qx + qtab[q].qy * qtab[q].qy);
      v[6] += ps;
      v[7] = fmin(v[7], ps);
    }
  }
  for (int c = 0; c < kDiagComp - 1; ++c) {
    const double t = block_sum(v[c], sh);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kDiagComp + c] = t;
  }
  const double mn = block_min(v[7], sh);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * kDiagComp + 7] = mn;
}

template <typename T>
hipError_t launch_diag(int nx, int ny, int nqd, const QNode *qtab,
                       StateT<T> a, RefView ref, double *partial, int *nblocks,
                       hipStream_t s) {
  const long long N = (long long)nx * ny;
  long long nb = (N + 255) / 256;
  if (nb > kDiagBlocks) nb = kDiagBlocks;
  *nblocks = (int)nb;
  hipLaunchKernelGGL(k_diag<T>, dim3((unsigned)nb), dim3(256), 0, s, nx, ny, nqd,
                     qtab, a, ref, partial);
  return hipGetLastError();
}
template hipError_t launch_diag<double>(int, int, int, const QNode *, StateT<double>,
                                        RefView, double *, int *, hipStream_t);
template hipError_t launch_diag<float>(int, int, int, const QNode *, StateT<float>,
                                       RefView, double *, int *, hipStream_t);

__global__ void k_diag_final(const double *__restrict__ partial, int n,
                             double *__restrict__ out) {
  __shared__ double sh[16];
  for (int c = 0; c < kDiagComp; ++c) {
    double v = (c == kDiagComp - 1) ? 1e300 : 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
      const double p = partial[(size_t)i * kDiagComp + c];
      v = (c == kDiagComp - 1) ? fmin(v, p) : v + p;
    }
    const double t = (c == kDiagComp - 1) ? block_min(v, sh) : block_sum(v, sh);
    if (threadIdx.x == 0) out[c] = t;
  }
}

hipError_t launch_diag_final(const double *partial, int nblocks, double *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, partial, nblocks,
                     out);
  return hipGetLastError();
}

// Observables: rho, Ux, Uy, rhoP, C (3), tau_p (3).
template <typename T>
__global__ void k_observables(int nqd, int nx, int ny, const QNode *__restrict__ qtab,
                              double inv_s2, double G, double mref, StateT<T> a,
                              RefView ref, double *__restrict__ out) {
  constexpr bool F32 = std::is_same<T, float>::value;
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int y = (int)(r / nx);
  double ps = 0.0, cxx = 0.0, cxy = 0.0, cyy = 0.0;
  for (int q = 0; q < nqd; ++q) {
    const double v = full(a.PSI[(size_t)q * N + r], F32 ? (double)ref.PSI[(size_t)q * ny + y] : 0.0);
    ps += v;
    cxx += v * qtab[q].qx * qtab[q].qx;
    cxy += v * qtab[q].qx * qtab[q].qy;
    cyy += v * qtab[q].qy * qtab[q].qy;
  }
  const double *F = a.FLD;
  const double cn = ps > 0.0 ? inv_s2 / ps : 0.0;
  out[0 * N + r] = F[(size_t)F_RHOS * N + r] + F[(size_t)F_RHOP * N + r];
  out[1 * N + r] = F[(size_t)F_UX * N + r];
  out[2 * N + r] = F[(size_t)F_UY * N + r];
  out[3 * N + r] = F[(size_t)F_RHOP * N + r];
  out[4 * N + r] = cxx * cn;
  out[5 * N + r] = cxy * cn;
  out[6 * N + r] = cyy * cn;
  const double g = mref > 0.0 ? G / mref : 0.0;
  out[7 * N + r] = mref > 0.0 ? g * F[(size_t)F_MXX * N + r] - G : 0.0;
  out[8 * N + r] = mref > 0.0 ? g * F[(size_t)F_MXY * N + r] : 0.0;
  out[9 * N + r] = mref > 0.0 ? g * F[(size_t)F_MYY * N + r] - G : 0.0;
}

template <typename T>
hipError_t launch_observables(int nqd, int nx, int ny, const QNode *qtab,
                              double inv_s2, double G, double mref,
                              StateT<T> a, RefView ref, double *out,
                              hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_observables<T>, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, nqd, nx, ny, qtab, inv_s2, G, mref, a, ref, out);
  return hipGetLastError();
}
template hipError_t launch_observables<double>(int, int, int, const QNode *, double, double,
                                               double, StateT<double>, RefView, double *,
                                               hipStream_t);
template hipError_t launch_observables<float>(int, int, int, const QNode *, double, double,
                                              double, StateT<float>, RefView, double *,
                                              hipStream_t);

// Health of a state, per workgroup into partial[3 block + c]: the number of
// non-finite mixture velocities and polymer densities (c = 0), and the
// smallest and largest polymer density psi over all (r, Q)-nodes (c = 1, 2).
// psi is a density of dumbbell configurations (Sec. VI.B): a run whose psi
// goes negative beyond round-off has lost positivity.
template <typename T>
__global__ void k_health(int nx, int ny, int nqd, StateT<T> a, RefView ref,
                         double *__restrict__ partial) {
  __shared__ double sh[16];
  constexpr bool F32 = std::is_same<T, float>::value;
  const long long N = (long long)nx * ny;
  double bad = 0.0, mn = 1e300, mx = -1e300;
  for (long long r = (long long)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (long long)gridDim.x * 256) {
    const double ux = a.FLD[(size_t)F_UX * N + r], uy = a.FLD[(size_t)F_UY * N + r];
    if (!isfinite(ux) || !isfinite(uy)) bad += 1.0;
    const int y = (int)(r / nx);
    for (int q = 0; q < nqd; ++q) {
      const double ps = full(a.PSI[(size_t)q * N + r],
                             F32 ? (double)ref.PSI[(size_t)q * ny + y] : 0.0);
      if (!isfinite(ps)) bad += 1.0;
      mn = fmin(mn, ps);
      mx = fmax(mx, ps);
    }
  }
  const double b = block_sum(bad, sh);
  const double lo = block_min(mn, sh);
  const double hi = block_max(mx, sh);
  if (threadIdx.x == 0) {
    partial[3 * (size_t)blockIdx.x] = b;
    partial[3 * (size_t)blockIdx.x + 1] = lo;
    partial[3 * (size_t)blockIdx.x + 2] = hi;
  }
}

__global__ void k_health_final(const double *__restrict__ partial, int n,
                               double *__restrict__ out) {
  __shared__ double sh[16];
  double b = 0.0, mn = 1e300, mx = -1e300;
  for (int i = threadIdx.x; i < n; i += 256) {
    b += partial[3 * (size_t)i];
    mn = fmin(mn, partial[3 * (size_t)i + 1]);
    mx = fmax(mx, partial[3 * (size_t)i + 2]);
  }
  b = block_sum(b, sh);
  mn = block_min(mn, sh);
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) {
    out[0] = b;
    out[1] = mn;
    out[2] = mx;
  }
}

template <typename T>
hipError_t launch_health(int nx, int ny, int nqd, StateT<T> a, RefView ref,
                         double *partial, double *out, hipStream_t s) {
  const long long N = (long long)nx * ny;
  long long nb = (N + 255) / 256;
  if (nb > kHealthBlocks) nb = kHealthBlocks;
  hipLaunchKernelGGL(k_health<T>, dim3((unsigned)nb), dim3(256), 0, s, nx, ny, nqd, a, ref,
                     partial);
  hipLaunchKernelGGL(k_health_final, dim3(1), dim3(256), 0, s, partial, (int)nb, out);
  return hipGetLastError();
}
template hipError_t launch_health<double>(int, int, int, StateT<double>, RefView, double *,
                                          double *, hipStream_t);
template hipError_t launch_health<float>(int, int, int, StateT<float>, RefView, double *,
                                         double *, hipStream_t);

// Closed-form Hookean laminar Kolmogorov state of one column (nx = 1; one
// workgroup per row y): the Oldroyd-B profile with the polymer populations'
// stress diffusion (Sec. VII forcing, Sec. V imposed fluxes),
//   U_x = UL sin(k y),  c_xy = lambda UL k cos(k y) / (1 + lambda D k^2),
//   c_xx = 1 + lambda^2 UL^2 k^2 / (1 + lambda D k^2) [1 + cos(2 k y) /
//          (1 + 4 lambda D k^2)],  c_yy = 1,
// psi proportional to exp(-Q.(sigma^2 c)^-1 Q / 2) over the disk with the
// row's sum rho_P0, the solvent at its equilibrium about U and the polymer
// at its equilibrium with the imposed fluxes J^r = psi U and
// J^Q = psi (K Q - D_Q Fhat), K_xy = dU_x/dy.  UL comes from the host.
__global__ void k_analytic_column(int ny, int nqd, const QNode *__restrict__ qtab,
                                  AnalyticColumn c, StateView col) {
  __shared__ double sh[16];
  const int y = blockIdx.x;
  const double ky = c.k * (double)y;
  const double ux = c.UL * sin(ky), Kxy = c.UL * c.k * cos(ky);
  const double cxy = c.lam * c.UL * c.k * cos(ky) / (1.0 + c.Dk2);
  const double cxx = 1.0 + c.lam * c.lam * c.UL * c.UL * c.k * c.k / (1.0 + c.Dk2) *
                               (1.0 + cos(2.0 * ky) / (1.0 + 4.0 * c.Dk2));
  // (sigma^2 c)^-1 with c_yy = 1
  const double det = c.s2 * c.s2 * (cxx - cxy * cxy);
  const double ixx = c.s2 / det, ixy = -c.s2 * cxy / det, iyy = c.s2 * cxx / det;
  auto weight = [&](int q) {
    const double qx = qtab[q].qx, qy = qtab[q].qy;
    return exp(-0.5 * (ixx * qx * qx + 2.0 * ixy * qx * qy + iyy * qy * qy));
  };
  double part = 0.0;
  for (int q = threadIdx.x; q < nqd; q += blockDim.x) part += weight(q);
  const double tot = block_sum(part, sh);
  for (int q = threadIdx.x; q < nqd; q += blockDim.x) {
    const double psi = c.rhoP0 * weight(q) / tot;
    const double J[4] = {psi * ux, 0.0, psi * (Kxy * qtab[q].qy - c.DQ * qtab[q].fx),
                         -psi * c.DQ * qtab[q].fy};
#pragma unroll
    for (int k = 0; k < 25; ++k) {
      double t = psi;
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (PV[k][a]) t += 3.0 * PV[k][a] * J[a];
      col.XP[((size_t)k * nqd + q) * ny + y] = (k == 0 ? 1.0 / 3.0 : 1.0 / 36.0) * t;
    }
    col.PSI[(size_t)q * ny + y] = psi;
  }
  if (threadIdx.x == 0) {
    const double uu = ux * ux;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      const double cu = C9X[d] * ux;
      col.XS[(size_t)d * ny + y] = W9[d] * c.rhoS0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
    col.FLD[(size_t)F_UX * ny + y] = ux;
    col.FLD[(size_t)F_UY * ny + y] = 0.0;
  }
}

hipError_t launch_analytic_column(int ny, int nqd, const QNode *qtab, AnalyticColumn c,
                                  StateView col, hipStream_t s) {
  hipLaunchKernelGGL(k_analytic_column, dim3((unsigned)ny), dim3(256), 0, s, ny, nqd, qtab, c,
                     col);
  return hipGetLastError();
}

// Gather a w x h window (periodic wrap) of XS, XP, PSI and U into
// dst[plane][h][w] with planes 9 | 25 nqd | nqd | 2, as full FP64 values.
template <typename T>
__global__ void k_window(int nx, int ny, int nqd, int x0, int y0, int w,
                         int h, StateT<T> a, RefView ref, double *__restrict__ dst) {
  constexpr bool F32 = std::is_same<T, float>::value;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = blockIdx.y;
  if (i >= w * h) return;
  const int wy = i / w, wx = i - wy * w;
  const int x = ((x0 + wx) % nx + nx) % nx, y = ((y0 + wy) % ny + ny) % ny;
  const long long N = (long long)nx * ny;
  const size_t r = (size_t)y * nx + x;
  double v;
  if (plane < 9) {
    v = full(a.XS[(size_t)plane * N + r], F32 ? (double)ref.XS[(size_t)plane * ny + y] : 0.0);
  } else if (plane < 9 + 25 * nqd) {
    const size_t pl = plane - 9;
    v = full(a.XP[pl * N + r], F32 ? (double)ref.XP[pl * ny + y] : 0.0);
  } else if (plane < 9 + 26 * nqd) {
    const size_t pl = plane - 9 - 25 * nqd;
    v = full(a.PSI[pl * N + r], F32 ? (double)ref.PSI[pl * ny + y] : 0.0);
  } else {
    v = a.FLD[(size_t)(F_UX + plane - 9 - 26 * nqd) * N + r];
  }
  dst[(size_t)plane * w * h + i] = v;
}

template <typename T>
hipError_t launch_window(int nx, int ny, int nqd, int x0, int y0, int w, int h,
                         StateT<T> a, RefView ref, double *dst, hipStream_t s) {
  dim3 grid((unsigned)((w * h + 255) / 256), 9 + 26 * nqd + 2);
  hipLaunchKernelGGL(k_window<T>, grid, dim3(256), 0, s, nx, ny, nqd, x0, y0, w,
                     h, a, ref, dst);
  return hipGetLastError();
}
template hipError_t launch_window<double>(int, int, int, int, int, int, int, StateT<double>,
                                          RefView, double *, hipStream_t);
template hipError_t launch_window<float>(int, int, int, int, int, int, int, StateT<float>,
                                         RefView, double *, hipStream_t);

}  // namespace tplk
