// Kernels of the learned coarse-lattice correction: a per-node network
// 54 -> 64 -> 64 -> 5 with exact GELU, BF16 weights and activations, FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16), its training
// step (forward, backward, weight gradients, Adam), and the lattice side:
// full-weighting restriction of a fine state onto a coarse one, the 3x3
// stencil features, the correction targets and the momentum source
// F = dJ + div(dtau) through which a correction acts on the scheme.
//
// Matrix-core layout (16x16x16, wave64, lane l = 16 g + c):
//   A (16 x 16, M x K): lane holds row c, k = 4 g .. 4 g + 3
//   B (16 x 16, K x N): lane holds column c, k = 4 g .. 4 g + 3
//   C (16 x 16, M x N): lane holds column c, rows 4 g .. 4 g + 3
// The network is evaluated transposed, Z^T = W A^T with nodes as the N
// dimension, so that a C tile of one layer (units x nodes) is, register for
// register, the B operand of the next layer.  One wave handles 16 nodes.
#include "tpl_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace tplk {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ v4s pack4(const v4f &v) {
  return v4s{bf16_bits(v[0]), bf16_bits(v[1]), bf16_bits(v[2]), bf16_bits(v[3])};
}

__device__ __forceinline__ v4s ld4(const uint16_t *p) {
  return *reinterpret_cast<const v4s *>(p);
}

__device__ __forceinline__ v4f mfma(const v4s &a, const v4s &b, const v4f &c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

// exact GELU z Phi(z) and its derivative Phi(z) + z phi(z)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * kInvSqrt2)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * kInvSqrt2)) + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

// Forward pass of one 16-node tile (nodes n0 .. n0 + 15, lane column c).
// Outputs z3 (standardised outputs 4 g + i); keeps pre-activations z1, z2
// and the BF16 operands x, h1, h2 for the backward pass.
struct Tile {
  v4s x[4];    // input, B operand per K-block
  v4f z1[4], z2[4];
  v4s h1[4], h2[4];
  v4f z3;
};

// The three layers from the input operands already in t.x.
__device__ __forceinline__ void tile_layers(const MlpDev &w, int c, int g, Tile &t) {
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    v4f acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = w.b1[16 * mb + 4 * g + i];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = mfma(ld4(w.W1b + (16 * mb + c) * 64 + 16 * kb + 4 * g), t.x[kb], acc);
    t.z1[mb] = acc;
    v4f h;
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = gelu(acc[i]);
    t.h1[mb] = pack4(h);
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    v4f acc;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = w.b2[16 * mb + 4 * g + i];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = mfma(ld4(w.W2b + (16 * mb + c) * 64 + 16 * kb + 4 * g), t.h1[kb], acc);
    t.z2[mb] = acc;
    v4f h;
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = gelu(acc[i]);
    t.h2[mb] = pack4(h);
  }
  v4f acc;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = w.b3[4 * g + i];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) acc = mfma(ld4(w.W3b + c * 64 + 16 * kb + 4 * g), t.h2[kb], acc);
  t.z3 = acc;
}

__device__ __forceinline__ void tile_forward(const MlpDev &w, const uint16_t *__restrict__ Xb,
                                             long long n, long long n0, int c, int g, Tile &t) {
  const long long node = n0 + c;
  const bool valid = node < n;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
    t.x[kb] = valid ? ld4(Xb + node * 64 + 16 * kb + 4 * g) : v4s{0, 0, 0, 0};
  tile_layers(w, c, g, t);
}

}  // namespace

// Y[n][nout] = network(standardised X) mapped back to physical units.
__global__ void __launch_bounds__(256) k_mlp_forward(MlpDev w, const uint16_t *__restrict__ Xb,
                                                     long long n, float *__restrict__ Y) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const long long n0 = ((long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16;
  if (n0 >= n) return;  // whole wave
  Tile t;
  tile_forward(w, Xb, n, n0, c, g, t);
  const long long node = n0 + c;
  if (node < n)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * g + i;
      if (o < w.nout) Y[node * w.nout + o] = t.z3[i] * w.out_std[o] + w.out_mean[o];
    }
}

// Training pass: every wave walks 16-node tiles with a fixed stride, runs
// forward and backward and accumulates the weight gradients of
// loss = mean over nodes and outputs of (y - t)^2 (standardised targets) in
// its registers; at the end it writes them to its record in partial[]:
//   dW1 [64][64] | db1 [64] | dW2 [64][64] | db2 [64] | dW3 [16][64] |
//   db3 [16] | sum of squared errors [1]         (kMlpRecord floats)
// Weight gradients contract over the tile's nodes: the tile's operands are
// staged transposed (units x 16 nodes, BF16) in the wave's LDS.
__global__ void __launch_bounds__(64) k_mlp_train(MlpDev w, const uint16_t *__restrict__ Xb,
                                                  const float *__restrict__ T, long long n,
                                                  float scale, float *__restrict__ partial) {
  __shared__ uint16_t XT[64][16], H1T[64][16], H2T[64][16], D1T[64][16], D2T[64][16],
      DYT[16][16];
  const int lane = threadIdx.x, c = lane & 15, g = lane >> 4;
  v4f gW1[4][4], gW2[4][4], gW3[4];
  v4f gb1[4], gb2[4], gb3 = {0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gb1[a] = gb2[a] = gW3[a] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 4; ++b) gW1[a][b] = gW2[a][b] = v4f{0, 0, 0, 0};
  }
  float sse = 0.0f;
  const long long ntiles = (n + 15) / 16;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long n0 = tile * 16, node = n0 + c;
    const bool valid = node < n;
    Tile t;
    tile_forward(w, Xb, n, n0, c, g, t);
    // output error (zero outside the valid nodes and outputs)
    v4f dy;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * g + i;
      float e = 0.0f;
      if (valid && o < w.nout) e = t.z3[i] - (T[node * w.nout + o] - w.out_mean[o]) / w.out_std[o];
      sse += e * e;
      dy[i] = scale * e;
    }
    gb3 += dy;
    const v4s dyb = pack4(dy);
    // dH2 = W3^T dY, dZ2 = dH2 gelu'(z2)
    v4s dz2b[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      v4f acc = mfma(ld4(w.W3Tb + (16 * mb + c) * 16 + 4 * g), dyb, v4f{0, 0, 0, 0});
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] *= gelu_grad(t.z2[mb][i]);
      dz2b[mb] = pack4(acc);
      gb2[mb] += acc;
    }
    // dH1 = W2^T dZ2, dZ1 = dH1 gelu'(z1)
    v4s dz1b[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      v4f acc = {0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        acc = mfma(ld4(w.W2Tb + (16 * mb + c) * 64 + 16 * kb + 4 * g), dz2b[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] *= gelu_grad(t.z1[mb][i]);
      dz1b[mb] = pack4(acc);
      gb1[mb] += acc;
    }
    // stage the operands transposed: unit rows, node columns
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int u = 16 * mb + 4 * g + i;
        XT[u][c] = (uint16_t)t.x[mb][i];
        H1T[u][c] = (uint16_t)t.h1[mb][i];
        H2T[u][c] = (uint16_t)t.h2[mb][i];
        D1T[u][c] = (uint16_t)dz1b[mb][i];
        D2T[u][c] = (uint16_t)dz2b[mb][i];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) DYT[4 * g + i][c] = (uint16_t)dyb[i];
    __syncthreads();
    // dW1 += dZ1^T X, dW2 += dZ2^T H1, dW3 += dY^T H2 (K = the 16 nodes)
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      const v4s a1 = ld4(&D1T[16 * mo + c][4 * g]);
      const v4s a2 = ld4(&D2T[16 * mo + c][4 * g]);
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) {
        gW1[mo][mi] = mfma(a1, ld4(&XT[16 * mi + c][4 * g]), gW1[mo][mi]);
        gW2[mo][mi] = mfma(a2, ld4(&H1T[16 * mi + c][4 * g]), gW2[mo][mi]);
      }
    }
    {
      const v4s a3 = ld4(&DYT[c][4 * g]);
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) gW3[mi] = mfma(a3, ld4(&H2T[16 * mi + c][4 * g]), gW3[mi]);
    }
    __syncthreads();  // the next tile overwrites the staging arrays
  }
  // bias gradients: sum over the 16 node columns of each lane group
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gb1[mb][i] += __shfl_xor(gb1[mb][i], m);
        gb2[mb][i] += __shfl_xor(gb2[mb][i], m);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) gb3[i] += __shfl_xor(gb3[i], m);
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) sse += __shfl_xor(sse, m);
  float *rec = partial + (size_t)blockIdx.x * kMlpRecord;
  float *pW1 = rec, *pb1 = pW1 + 4096, *pW2 = pb1 + 64, *pb2 = pW2 + 4096, *pW3 = pb2 + 64,
        *pb3 = pW3 + 1024, *psse = pb3 + 16;
#pragma unroll
  for (int mo = 0; mo < 4; ++mo)
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pW1[(16 * mo + 4 * g + i) * 64 + 16 * mi + c] = gW1[mo][mi][i];
        pW2[(16 * mo + 4 * g + i) * 64 + 16 * mi + c] = gW2[mo][mi][i];
      }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int i = 0; i < 4; ++i) pW3[(4 * g + i) * 64 + 16 * mi + c] = gW3[mi][i];
  if (c == 0) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pb1[16 * mb + 4 * g + i] = gb1[mb][i];
        pb2[16 * mb + 4 * g + i] = gb2[mb][i];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) pb3[4 * g + i] = gb3[i];
  }
  if (lane == 0) psse[0] = sse;
}

// Sum the per-wave records in FP64 (fixed order) and scatter them to the
// canonical parameter layout W1 [64][nin] b1 W2 [64][64] b2 W3 [nout][64] b3;
// out[nparams] receives the sum of squared errors.
__global__ void k_mlp_reduce(const float *__restrict__ partial, int nrec, int nin, int nout,
                             float *__restrict__ grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kMlpRecord) return;
  double s = 0.0;
  for (int r = 0; r < nrec; ++r) s += partial[(size_t)r * kMlpRecord + j];
  // record position -> canonical position (or -1 for padding)
  int dst = -1;
  const int oW1 = 0, ob1 = 64 * nin, oW2 = ob1 + 64, ob2 = oW2 + 4096, oW3 = ob2 + 64,
            ob3 = oW3 + 64 * nout, osse = ob3 + nout;
  if (j < 4096) {
    const int h = j / 64, i = j % 64;
    if (i < nin) dst = oW1 + h * nin + i;
  } else if (j < 4160) {
    dst = ob1 + (j - 4096);
  } else if (j < 8256) {
    dst = oW2 + (j - 4160);
  } else if (j < 8320) {
    dst = ob2 + (j - 8256);
  } else if (j < 9344) {
    const int o = (j - 8320) / 64, h = (j - 8320) % 64;
    if (o < nout) dst = oW3 + o * 64 + h;
  } else if (j < 9360) {
    if (j - 9344 < nout) dst = ob3 + (j - 9344);
  } else {
    dst = osse;
  }
  if (dst >= 0) grad[dst] = (float)s;
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters; t >= 1.
__global__ void k_mlp_adam(float *__restrict__ theta, float *__restrict__ m,
                           float *__restrict__ v, const float *__restrict__ grad, int np,
                           float lr, float b1, float b2, float eps, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  const float gj = grad[j];
  const float mj = b1 * m[j] + (1.0f - b1) * gj;
  const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  theta[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// Canonical FP32 parameters -> BF16 operand arrays (zero padded) and
// padded FP32 biases: W1b [64][64], W2b [64][64], W3b [16][64],
// W2Tb [64][64] (transposed), W3Tb [64][16] (transposed).
__global__ void k_mlp_pack(const float *__restrict__ theta, int nin, int nout,
                           uint16_t *__restrict__ W1b, uint16_t *__restrict__ W2b,
                           uint16_t *__restrict__ W3b, uint16_t *__restrict__ W2Tb,
                           uint16_t *__restrict__ W3Tb, float *__restrict__ b1,
                           float *__restrict__ b2, float *__restrict__ b3) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const float *W1 = theta, *B1 = W1 + 64 * nin, *W2 = B1 + 64, *B2 = W2 + 4096, *W3 = B2 + 64,
              *B3 = W3 + 64 * nout;
  if (j < 4096) {
    const int r = j / 64, k = j % 64;
    W1b[j] = (uint16_t)bf16_bits(k < nin ? W1[r * nin + k] : 0.0f);
    W2b[j] = (uint16_t)bf16_bits(W2[j]);
    W2Tb[j] = (uint16_t)bf16_bits(W2[k * 64 + r]);  // W2Tb[r][k] = W2[k][r]
  }
  if (j < 1024) {
    const int o = j / 64, h = j % 64;
    W3b[j] = (uint16_t)bf16_bits(o < nout ? W3[o * 64 + h] : 0.0f);
    const int hh = j / 16, oo = j % 16;
    W3Tb[j] = (uint16_t)bf16_bits(oo < nout ? W3[oo * 64 + hh] : 0.0f);
  }
  if (j < 64) {
    b1[j] = B1[j];
    b2[j] = B2[j];
  }
  if (j < 16) b3[j] = j < nout ? B3[j] : 0.0f;
}

// Raw FP32 inputs [n][nin] -> standardised BF16 operand rows [n][64].
__global__ void k_mlp_prep(const float *__restrict__ X, long long n, int nin,
                           const float *__restrict__ mean, const float *__restrict__ stdv,
                           uint16_t *__restrict__ Xb) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n * 64) return;
  const long long node = j / 64;
  const int k = (int)(j % 64);
  Xb[j] = (uint16_t)bf16_bits(k < nin ? (X[node * nin + k] - mean[k]) / stdv[k] : 0.0f);
}

// ---------------------------------------------------------------------------
// Lattice side (FP64).

// Features of every node from the observables obs[10][N]: the 3x3 periodic
// neighbourhood of rho, Ux, Uy, Cxx, Cxy, Cyy, feature 6 s + f for stencil
// position s = 3 (dy + 1) + (dx + 1).  Raw values to X [N][54] (if X) and
// standardised BF16 rows to Xb [N][64] (if Xb).
__global__ void k_features(const double *__restrict__ obs, int nx, int ny,
                           const float *__restrict__ mean, const float *__restrict__ stdv,
                           float *__restrict__ X, uint16_t *__restrict__ Xb) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int y = (int)(r / nx), x = (int)(r - (long long)y * nx);
  const int fields[6] = {0, 1, 2, 4, 5, 6};
#pragma unroll
  for (int s = 0; s < 9; ++s) {
    const int yy = (y + s / 3 - 1 + ny) % ny, xx = (x + s % 3 - 1 + nx) % nx;
    const long long rr = (long long)yy * nx + xx;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const float v = (float)obs[(size_t)fields[f] * N + rr];
      const int k = 6 * s + f;
      if (X) X[r * 54 + k] = v;
      if (Xb) Xb[r * 64 + k] = (uint16_t)bf16_bits((v - mean[k]) / stdv[k]);
    }
  }
  if (Xb)
    for (int k = 54; k < 64; ++k) Xb[r * 64 + k] = 0;
}

// Targets [N][5]: (rho U, tau) of obs_ref minus those of obs.
__global__ void k_targets(const double *__restrict__ ref, const double *__restrict__ obs,
                          long long N, float *__restrict__ T) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  auto ms = [&](const double *o, int j) -> double {
    switch (j) {
      case 0: return o[r] * o[N + r];
      case 1: return o[r] * o[2 * N + r];
      default: return o[(size_t)(5 + j) * N + r];
    }
  };
#pragma unroll
  for (int j = 0; j < 5; ++j) T[r * 5 + j] = (float)(ms(ref, j) - ms(obs, j));
}

// Momentum source F [2][N] = dJ + div_h(dtau) (central differences) from a
// correction corr [N][5] (dJx, dJy, dtau_xx, dtau_xy, dtau_yy).
__global__ void k_source(const float *__restrict__ corr, int nx, int ny,
                         double *__restrict__ F) {
  const long long N = (long long)nx * ny;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int y = (int)(r / nx), x = (int)(r - (long long)y * nx);
  const long long e = (long long)y * nx + (x + 1) % nx, wv = (long long)y * nx + (x - 1 + nx) % nx;
  const long long nn = (long long)((y + 1) % ny) * nx + x, s = (long long)((y - 1 + ny) % ny) * nx + x;
  auto cc = [&](long long i, int j) -> double { return (double)corr[i * 5 + j]; };
  F[r] = cc(r, 0) + 0.5 * (cc(e, 2) - cc(wv, 2)) + 0.5 * (cc(nn, 3) - cc(s, 3));
  F[N + r] = cc(r, 1) + 0.5 * (cc(e, 3) - cc(wv, 3)) + 0.5 * (cc(nn, 4) - cc(s, 4));
}

// Per-workgroup sums of both source components, partial[blk][2] (fixed
// order: the removal of the mean below is deterministic).
__global__ void k_source_sums(const double *__restrict__ F, long long N,
                              double *__restrict__ partial) {
  __shared__ double sx[256], sy[256];
  double a = 0.0, b = 0.0;
  for (long long r = (long long)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (long long)gridDim.x * 256) {
    a += F[r];
    b += F[N + r];
  }
  sx[threadIdx.x] = a;
  sy[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sx[0];
    partial[2 * blockIdx.x + 1] = sy[0];
  }
}

// F -= sum / N per component.
__global__ void k_source_center(double *__restrict__ F, long long N,
                                const double *__restrict__ sums) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const double mx = sums[0] / (double)N, my = sums[1] / (double)N;
  F[r] -= mx;
  F[N + r] -= my;
}

// Largest |F| / rho over the lattice, per workgroup into partial[] (the
// velocity change a source makes in one step).
__global__ void k_source_drift(const double *__restrict__ F, const double *__restrict__ FLD,
                               long long N, double *__restrict__ partial) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (long long r = (long long)blockIdx.x * 256 + threadIdx.x; r < N;
       r += (long long)gridDim.x * 256) {
    const double rho = FLD[(size_t)F_RHOS * N + r] + FLD[(size_t)F_RHOP * N + r];
    const double f = sqrt(F[r] * F[r] + F[N + r] * F[N + r]) / rho;
    mx = (f > mx || !(f == f)) ? f : mx;  // NaN wins
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = sh[threadIdx.x + s];
      if (o > sh[threadIdx.x] || !(o == o)) sh[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Full-weighting restriction by an even factor m of planes of a fine
// lattice (nxf x nyf) onto a coarse one: coarse (X, Y) averages fine
// (m X + i, m Y + j), |i|, |j| <= m/2, weights 1/2 on the window's edges.
template <typename T>
__global__ void k_restrict(int planes, int nxf, int nyf, int m, const T *__restrict__ src,
                           double *__restrict__ dst) {
  const int nxc = nxf / m, nyc = nyf / m;
  const long long Nc = (long long)nxc * nyc, Nf = (long long)nxf * nyf;
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Nc * planes) return;
  const int pl = (int)(j / Nc);
  const long long rc = j - (long long)pl * Nc;
  const int Y = (int)(rc / nxc), X = (int)(rc - (long long)Y * nxc);
  const T *P = src + (size_t)pl * Nf;
  const int h = m / 2;
  double acc = 0.0;
  for (int dj = -h; dj <= h; ++dj) {
    const double wy = (dj == -h || dj == h) ? 0.5 : 1.0;
    const int y = (m * Y + dj + nyf) % nyf;
    double row = 0.0;
    for (int di = -h; di <= h; ++di) {
      const double wx = (di == -h || di == h) ? 0.5 : 1.0;
      const int x = (m * X + di + nxf) % nxf;
      row += wx * (double)P[(long long)y * nxf + x];
    }
    acc += wy * row;
  }
  dst[(size_t)pl * Nc + rc] = acc / ((double)m * m);
}

// ---------------------------------------------------------------------------
// The attached correction of a coarse step, fused.

// Feature k of node (x, y) from the observables, as k_features computes it:
// field f = k % 6 of (rho, Ux, Uy, Cxx, Cxy, Cyy) at stencil position
// s = k / 6 = 3 (dy + 1) + (dx + 1), periodic.
__device__ __forceinline__ float stencil_feature(const double *__restrict__ obs, int nx, int ny,
                                                 int x, int y, int k) {
  const int s = k / 6, f = k - 6 * s;
  const int fld = f < 3 ? f : f + 1;
  const int yy = (y + s / 3 - 1 + ny) % ny, xx = (x + s % 3 - 1 + nx) % nx;
  return (float)obs[(size_t)fld * nx * ny + (size_t)yy * nx + xx];
}

// One wave per 16-node tile: features, network, correction in physical
// units, and the wave's sums of the two momentum corrections.
__global__ void __launch_bounds__(256) k_correct(MlpDev w, const double *__restrict__ obs, int nx,
                                                 int ny, const float *__restrict__ mean,
                                                 const float *__restrict__ stdv,
                                                 float *__restrict__ corr,
                                                 double *__restrict__ partial,
                                                 const int *__restrict__ gate) {
  if (*gate) return;  // uniform: the drift gate stopped an earlier step
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  const long long N = (long long)nx * ny;
  const long long wid = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long long n0 = wid * 16, node = n0 + c;
  const bool valid = node < N;
  double jx = 0.0, jy = 0.0;
  if (n0 < N) {  // whole wave
    Tile t;
    const int y = valid ? (int)(node / nx) : 0, x = valid ? (int)(node - (long long)y * nx) : 0;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      v4s v = {0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * kb + 4 * g + i;
        if (valid && k < w.nin)
          v[i] = bf16_bits((stencil_feature(obs, nx, ny, x, y, k) - mean[k]) / stdv[k]);
      }
      t.x[kb] = v;
    }
    tile_layers(w, c, g, t);
    if (valid)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 4 * g + i;
        if (o < w.nout) {
          const float v = t.z3[i] * w.out_std[o] + w.out_mean[o];
          corr[node * w.nout + o] = v;
          if (o == 0) jx = (double)v;
          if (o == 1) jy = (double)v;
        }
      }
  }
  jx = wave_sum(jx);
  jy = wave_sum(jy);
  if (lane == 0 && n0 < N) {  // one record per wave of correct_waves(N)
    partial[2 * wid] = jx;
    partial[2 * wid + 1] = jy;
  }
}

// F = (dJ - <dJ>) + div_h(dtau) and the drift gate (grid-stride; every
// workgroup forms the lattice mean from the per-wave sums in one fixed
// order).
__global__ void __launch_bounds__(256) k_source_gate(const float *__restrict__ corr, int nx,
                                                     int ny, const double *__restrict__ partial,
                                                     long long nparts,
                                                     const double *__restrict__ FLD, double bound,
                                                     int tag, double *__restrict__ F,
                                                     int *__restrict__ gate,
                                                     unsigned long long *__restrict__ drift) {
  __shared__ double sh[16];
  if (*gate) return;  // uniform
  const long long N = (long long)nx * ny;
  double sx = 0.0, sy = 0.0;
  for (long long i = threadIdx.x; i < nparts; i += blockDim.x) {
    sx += partial[2 * i];
    sy += partial[2 * i + 1];
  }
  const double mx = block_sum(sx, sh) / (double)N, my = block_sum(sy, sh) / (double)N;
  double dmax = 0.0;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N;
       r += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(r / nx), x = (int)(r - (long long)y * nx);
    const long long e = (long long)y * nx + (x + 1) % nx, wv = (long long)y * nx + (x - 1 + nx) % nx;
    const long long nn = (long long)((y + 1) % ny) * nx + x, s = (long long)((y - 1 + ny) % ny) * nx + x;
    auto cc = [&](long long i, int j) -> double { return (double)corr[i * 5 + j]; };
    const double fx = cc(r, 0) - mx + 0.5 * (cc(e, 2) - cc(wv, 2)) + 0.5 * (cc(nn, 3) - cc(s, 3));
    const double fy = cc(r, 1) - my + 0.5 * (cc(e, 3) - cc(wv, 3)) + 0.5 * (cc(nn, 4) - cc(s, 4));
    F[r] = fx;
    F[N + r] = fy;
    const double rho = FLD[(size_t)F_RHOS * N + r] + FLD[(size_t)F_RHOP * N + r];
    const double d = sqrt(fx * fx + fy * fy) / rho;
    dmax = (d > dmax || !(d == d)) ? d : dmax;  // NaN wins
  }
  // a NaN anywhere in the workgroup makes its maximum infinite
  const double bad = block_sum(dmax == dmax ? 0.0 : 1.0, sh);
  dmax = bad > 0.0 ? INFINITY : block_max(dmax, sh);
  if (threadIdx.x == 0) {
    atomicMax(drift, (unsigned long long)__double_as_longlong(dmax));
    if (!(dmax <= bound)) atomicCAS(gate, 0, tag);
  }
}

// ---------------------------------------------------------------------------
// Launchers

hipError_t launch_mlp_forward(const MlpDev &w, const uint16_t *Xb, long long n, float *Y,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long tiles = (n + 15) / 16;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, w, Xb,
                     n, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_train(const MlpDev &w, const uint16_t *Xb, const float *T, long long n,
                            int nrec, float *partial, hipStream_t s) {
  const float scale = 2.0f / (float)((double)n * w.nout);
  hipLaunchKernelGGL(k_mlp_train, dim3(nrec), dim3(64), 0, s, w, Xb, T, n, scale, partial);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float *partial, int nrec, int nin, int nout, float *grad,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpRecord + 255) / 256), dim3(256), 0, s, partial,
                     nrec, nin, nout, grad);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float *theta, float *m, float *v, const float *grad, int np, float lr,
                           int t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - std::pow(0.9, t)), c2 = (float)(1.0 - std::pow(0.999, t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((np + 255) / 256), dim3(256), 0, s, theta, m, v, grad, np,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *theta, int nin, int nout, const MlpDev &w,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(16), dim3(256), 0, s, theta, nin, nout,
                     const_cast<uint16_t *>(w.W1b), const_cast<uint16_t *>(w.W2b),
                     const_cast<uint16_t *>(w.W3b), const_cast<uint16_t *>(w.W2Tb),
                     const_cast<uint16_t *>(w.W3Tb), const_cast<float *>(w.b1),
                     const_cast<float *>(w.b2), const_cast<float *>(w.b3));
  return hipGetLastError();
}

hipError_t launch_mlp_prep(const float *X, long long n, int nin, const float *mean,
                           const float *stdv, uint16_t *Xb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_prep, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, s, X, n,
                     nin, mean, stdv, Xb);
  return hipGetLastError();
}

hipError_t launch_features(const double *obs, int nx, int ny, const float *mean,
                           const float *stdv, float *X, uint16_t *Xb, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, obs, nx,
                     ny, mean, stdv, X, Xb);
  return hipGetLastError();
}

hipError_t launch_targets(const double *ref, const double *obs, long long N, float *T,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_targets, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, ref, obs, N,
                     T);
  return hipGetLastError();
}

hipError_t launch_source(const float *corr, int nx, int ny, double *F, hipStream_t s) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_source, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, corr, nx, ny,
                     F);
  return hipGetLastError();
}

hipError_t launch_source_center(double *F, long long N, double *scratch, hipStream_t s) {
  const long long nb = std::min<long long>(1024, (N + 255) / 256);
  hipLaunchKernelGGL(k_source_sums, dim3((unsigned)nb), dim3(256), 0, s, F, N, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_sum(scratch, (int)nb, 2, scratch + 2048, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_source_center, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, F, N,
                     scratch + 2048);
  return hipGetLastError();
}

hipError_t launch_source_drift(const double *F, const double *FLD, long long N, double *partial,
                               int *nblocks, hipStream_t s) {
  const long long nb = std::min<long long>(1024, (N + 255) / 256);
  *nblocks = (int)nb;
  hipLaunchKernelGGL(k_source_drift, dim3((unsigned)nb), dim3(256), 0, s, F, FLD, N, partial);
  return hipGetLastError();
}

long long correct_waves(long long N) { return (N + 15) / 16; }

hipError_t launch_correct(const MlpDev &w, const double *obs, int nx, int ny, const float *mean,
                          const float *stdv, float *corr, double *partial, const int *gate,
                          hipStream_t s) {
  const long long waves = correct_waves((long long)nx * ny);
  hipLaunchKernelGGL(k_correct, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, w, obs, nx,
                     ny, mean, stdv, corr, partial, gate);
  return hipGetLastError();
}

hipError_t launch_source_gate(const float *corr, int nx, int ny, const double *partial,
                              long long nparts, const double *FLD, double bound, int tag,
                              double *F, int *gate, unsigned long long *drift, hipStream_t s) {
  const long long N = (long long)nx * ny;
  long long nb = (N + 255) / 256;
  if (nb > 128) nb = 128;
  hipLaunchKernelGGL(k_source_gate, dim3((unsigned)nb), dim3(256), 0, s, corr, nx, ny, partial,
                     nparts, FLD, bound, tag, F, gate, drift);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(int planes, int nxf, int nyf, int m, const T *src, double *dst,
                           hipStream_t s) {
  const long long n = (long long)(nxf / m) * (nyf / m) * planes;
  hipLaunchKernelGGL(k_restrict<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, planes,
                     nxf, nyf, m, src, dst);
  return hipGetLastError();
}
template hipError_t launch_restrict<double>(int, int, int, int, const double *, double *,
                                            hipStream_t);

}  // namespace tplk
