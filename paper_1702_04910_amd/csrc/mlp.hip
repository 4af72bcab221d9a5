// Learned solid fraction: an 8 -> 64 -> 64 -> 1 MLP (ReLU) that replaces the
// supersampling (Sec. 2.3.2) of cells cut by a sphere surface.  Inputs: see
// eps_features (signed distance from the surface, sorted direction cosines,
// scaled curvature, zero padding).
//
// All GEMMs run on MFMA (bf16 operands, fp32 accumulation): the K = 64 layer
// of the forward pass on v_mfma_f32_32x32x16_bf16, the others on
// v_mfma_f32_32x32x8bf16_1k.  Layers are chained with the weights as the A operand
// (M = output features) and the activations as the B operand (N = 32 samples
// per wave): the 32x32 fp32 result of one layer, converted to bf16, is in
// exactly the lane/item order of the next layer's B operand.  Operand layout of
// the 32x32x8 instruction (lane l, item e):
//   A[i][k]: i = l % 32, k = 4 (l / 32) + e
//   B[k][j]: j = l % 32, k = 4 (l / 32) + e
//   D[i][j]: j = l % 32, i = 8 (e / 4) + 4 (l / 32) + e % 4
// Weight gradients reduce over samples; for them the bf16 activations and
// back-propagated errors go through LDS as [feature][sample] arrays and are
// read back with the samples on the K axis.
//
// Parameter blob (fp32): W1[64][8] b1[64] W2[64][64] b2[64] W3[64] b3[1].
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace lbm {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int NIN = 8, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;

__device__ __forceinline__ short bfbits(float x) { return __builtin_bit_cast(short, (__bf16)x); }
__device__ __forceinline__ float bfval(float x) { return (float)(__bf16)x; }

__device__ __forceinline__ f16v mfma(s4 a, s4 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

// The K = 16 form of gfx950 (twice the work per instruction).  A sum over k
// does not depend on which k an operand slot holds as long as A and B agree,
// so the 64-feature contraction of layer 2 takes its 16 features per step in
// the order the layer-1 result already has in registers: step m, lane half h,
// item e holds feature 32 (m / 2) + 16 (m % 2) + 4 h + e for e < 4 and
// 32 (m / 2) + 16 (m % 2) + 8 + 4 h + (e - 4) for e >= 4, i.e. the items of
// the two K = 8 groups s = 2 (m % 2) and s + 1 of tile m / 2 side by side.
__device__ __forceinline__ f16v mfma16(s8 a, s8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}
__device__ __forceinline__ int k16_feature(int m, int h, int e) {
  return 32 * (m >> 1) + 16 * (m & 1) + (e < 4 ? 4 * h + e : 8 + 4 * h + (e - 4));
}

__device__ __forceinline__ f16v zero16() {
  f16v z;
#pragma unroll
  for (int e = 0; e < 16; ++e) z[e] = 0.f;
  return z;
}

// Forward pass for the 32 samples of one wave.  xin: the 4 inputs of this lane
// (features 4h..4h+3 of sample l % 32).  Outputs: Z1, Z2 (fp32, D layout, two
// 32-row tiles each), H1 as bf16 B operands, y of sample l % 32.
struct Fwd {
  f16v z1[2], z2[2];
  s4 h1b[2][4];
  float y;
};

// The weight matrices as this lane's bf16 A operands (loaded and converted
// once, reused for every tile of samples a wave processes).
struct MlpA {
  s4 w1[2];
  s8 w2[2][4];  // [output tile][K = 16 step]
};

__device__ __forceinline__ void mlp_load_a(const float* __restrict__ P, MlpA& A) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) A.w1[t][e] = bfbits(P[OFF_W1 + (32 * t + i) * NIN + 4 * h + e]);
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int e = 0; e < 8; ++e) A.w2[t2][m][e] = bfbits(P[OFF_W2 + (32 * t2 + i) * NH + k16_feature(m, h, e)]);
}

// Biases and output weights are read through V (b1[64] b2[64] W3[64] b3, the
// blob's layout from OFF_B1 on with W2 skipped): the parameter blob itself, or
// a copy in LDS.
struct MlpV {
  const float* b1;
  const float* b2;
  const float* w3;
  float b3;
};

__device__ __forceinline__ MlpV mlp_v_global(const float* __restrict__ P) {
  return MlpV{P + OFF_B1, P + OFF_B2, P + OFF_W3, P[OFF_B3]};
}

__device__ __forceinline__ void mlp_forward(const MlpV& V, const MlpA& A, const float (&xin)[4], Fwd& f) {
  const int lane = threadIdx.x & 63, h = lane >> 5;
  s4 xb;
#pragma unroll
  for (int e = 0; e < 4; ++e) xb[e] = bfbits(xin[e]);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f16v d = mfma(A.w1[t], xb, zero16());
#pragma unroll
    for (int e = 0; e < 16; ++e) d[e] += V.b1[32 * t + 8 * (e >> 2) + 4 * h + (e & 3)];
    f.z1[t] = d;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) f.h1b[t][s][e] = bfbits(fmaxf(d[4 * s + e], 0.f));
  }
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2) {
    f16v acc = zero16();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const s4 lo = f.h1b[m >> 1][2 * (m & 1)], hi = f.h1b[m >> 1][2 * (m & 1) + 1];
      s8 b;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        b[e] = lo[e];
        b[4 + e] = hi[e];
      }
      acc = mfma16(A.w2[t2][m], b, acc);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] += V.b2[32 * t2 + 8 * (e >> 2) + 4 * h + (e & 3)];
    f.z2[t2] = acc;
  }
  float part = 0.f;
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int e = 0; e < 16; ++e)
      part += V.w3[32 * t2 + 8 * (e >> 2) + 4 * h + (e & 3)] * fmaxf(f.z2[t2][e], 0.f);
  part += __shfl_xor(part, 32, 64);
  f.y = part + V.b3;
}

// Inference over n samples given as features X[n][8] (fp32); y clamped to [0, 1].
// With `count` non-null the number of samples is min(*count, n).
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                        long long n, const int* __restrict__ count,
                                                        float* __restrict__ y) {
  // biases and output weights in LDS (read by every tile), matrices in registers
  __shared__ float sv[3 * NH];
  for (int k = threadIdx.x; k < 3 * NH; k += blockDim.x)
    sv[k] = P[k < NH ? OFF_B1 + k : OFF_B2 + (k - NH)];  // b2 and W3 are adjacent in the blob
  __syncthreads();
  const MlpV V{sv, sv + NH, sv + 2 * NH, P[OFF_B3]};
  if (count) n = min(n, (long long)*count);
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  MlpA A;
  mlp_load_a(P, A);
  // the inputs of the next PREF tiles are in flight while a tile is evaluated
  constexpr int PREF = 4;
  const long long tile0 = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  float xq[PREF][4];
#pragma unroll
  for (int k = 0; k < PREF; ++k) {
    const long long s = (tile0 + k * nw) * 32 + i;
#pragma unroll
    for (int e = 0; e < 4; ++e) xq[k][e] = s < n ? X[s * NIN + 4 * h + e] : 0.f;
  }
  for (long long tile = tile0; tile * 32 < n; tile += PREF * nw) {
#pragma unroll
    for (int k = 0; k < PREF; ++k) {
      const long long tk = tile + k * nw;
      if (tk * 32 >= n) break;  // whole wave
      const long long s = tk * 32 + i;
      Fwd f;
      mlp_forward(V, A, xq[k], f);
      const long long sn = s + (long long)PREF * nw * 32;  // refill the slot with tile tk + PREF * nw
#pragma unroll
      for (int e = 0; e < 4; ++e) xq[k][e] = sn < n ? X[sn * NIN + 4 * h + e] : 0.f;
      if (h == 0 && s < n) y[s] = fminf(fmaxf(f.y, 0.f), 1.f);
    }
  }
}

// Training: one wave = one tile of 32 samples (indices perm(b0 + tile*32 + i)).
// Writes the tile's gradient (sum over its samples of d(L)/d(params), with
// L = (1/M) sum (y - t)^2 and M = batch) to partial[wave][NPARAM].
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                       const float* __restrict__ T, long long n, long long b0,
                                                       long long mult, long long add, int batch,
                                                       float* __restrict__ partial) {
  __shared__ short lds[4][3 * NH * 32 + 32 * 32];  // per wave: dZ2, H1, dZ1 [64][32], X [32][32] (bf16 bits)
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5, w = threadIdx.x >> 6;
  const int tile = blockIdx.x * (blockDim.x >> 6) + w;
  if ((long long)tile * 32 >= batch) return;  // whole waves only: no barriers below
  short* sdz2 = lds[w];
  short* sh1 = sdz2 + NH * 32;
  short* sdz1 = sh1 + NH * 32;
  short* sx = sdz1 + NH * 32;
  const int local = tile * 32 + i;
  const bool valid = local < batch;
  const long long s = valid ? (b0 + local) % n : 0;
  const long long idx = (s * mult + add) % n;  // affine permutation of the training set
  float xin[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) xin[e] = valid ? X[idx * NIN + 4 * h + e] : 0.f;
  Fwd f;
  MlpA A;
  mlp_load_a(P, A);
  mlp_forward(mlp_v_global(P), A, xin, f);
  const float dy = valid ? 2.f * (f.y - T[idx]) / (float)batch : 0.f;
  float* G = partial + (long long)tile * NPARAM;
  // dZ2 = W3 dy [Z2 > 0]; dW3 = sum_n dy H2; db2 = sum_n dZ2; db3 = sum_n dy
  f16v dz2[2];
  float gw3[2][16], gb2[2][16];
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int o = 32 * t2 + 8 * (e >> 2) + 4 * h + (e & 3);
      const float z = f.z2[t2][e];
      dz2[t2][e] = z > 0.f ? P[OFF_W3 + o] * dy : 0.f;
      gw3[t2][e] = dy * fmaxf(z, 0.f);
      gb2[t2][e] = dz2[t2][e];
    }
  // sum over the 32 samples of this half-wave
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int e = 0; e < 16; ++e)
#pragma unroll
      for (int m = 1; m < 32; m <<= 1) {
        gw3[t2][e] += __shfl_xor(gw3[t2][e], m, 64);
        gb2[t2][e] += __shfl_xor(gb2[t2][e], m, 64);
      }
  if (i == 0) {
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int o = 32 * t2 + 8 * (e >> 2) + 4 * h + (e & 3);
        G[OFF_W3 + o] = gw3[t2][e];
        G[OFF_B2 + o] = gb2[t2][e];
      }
  }
  float gb3 = dy;
#pragma unroll
  for (int m = 1; m < 32; m <<= 1) gb3 += __shfl_xor(gb3, m, 64);
  if (lane == 0) G[OFF_B3] = gb3;
  // dH1 = W2^T dZ2 (MFMA), dZ1 = dH1 [Z1 > 0]
  s4 dz2b[2][4];
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int e = 0; e < 4; ++e) dz2b[t2][s][e] = bfbits(dz2[t2][4 * s + e]);
  f16v dz1[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f16v acc = zero16();
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        s4 a;
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = bfbits(P[OFF_W2 + (32 * t2 + 8 * s + 4 * h + e) * NH + 32 * t + i]);
        acc = mfma(a, dz2b[t2][s], acc);
      }
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = f.z1[t][e] > 0.f ? acc[e] : 0.f;
    dz1[t] = acc;
  }
  // db1 = sum_n dZ1
  float gb1[2][16];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      float v = dz1[t][e];
#pragma unroll
      for (int m = 1; m < 32; m <<= 1) v += __shfl_xor(v, m, 64);
      gb1[t][e] = v;
    }
  if (i == 0) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < 16; ++e) G[OFF_B1 + 32 * t + 8 * (e >> 2) + 4 * h + (e & 3)] = gb1[t][e];
  }
  // stage dZ2, H1, dZ1 (bf16) and X as [feature][sample] in LDS
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int o = 32 * t + 8 * (e >> 2) + 4 * h + (e & 3);
      sdz2[o * 32 + i] = dz2b[t][e >> 2][e & 3];
      sh1[o * 32 + i] = f.h1b[t][e >> 2][e & 3];
      sdz1[o * 32 + i] = bfbits(dz1[t][e]);
    }
#pragma unroll
  for (int e = 0; e < 4; ++e) sx[(4 * h + e) * 32 + i] = bfbits(xin[e]);
  for (int r = 8 + h; r < 32; r += 2) sx[r * 32 + i] = 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // dW2[o][k] = sum_n dZ2[o][n] H1[k][n]: A = dZ2 (o x n), B = H1^T (n x k)
#pragma unroll
  for (int to = 0; to < 2; ++to)
#pragma unroll
    for (int tk = 0; tk < 2; ++tk) {
      f16v acc = zero16();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        s4 a, b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a[e] = sdz2[(32 * to + i) * 32 + 8 * s + 4 * h + e];
          b[e] = sh1[(32 * tk + i) * 32 + 8 * s + 4 * h + e];
        }
        acc = mfma(a, b, acc);
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int o = 32 * to + 8 * (e >> 2) + 4 * h + (e & 3);
        G[OFF_W2 + o * NH + 32 * tk + i] = acc[e];
      }
    }
  // dW1[o][f] = sum_n dZ1[o][n] X[n][f]: A = dZ1 (o x n), B = X (n x f, f < 8 used)
#pragma unroll
  for (int to = 0; to < 2; ++to) {
    f16v acc = zero16();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      s4 a, b;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[e] = sdz1[(32 * to + i) * 32 + 8 * s + 4 * h + e];
        b[e] = sx[i * 32 + 8 * s + 4 * h + e];
      }
      acc = mfma(a, b, acc);
    }
    if (i < NIN) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int o = 32 * to + 8 * (e >> 2) + 4 * h + (e & 3);
        G[OFF_W1 + o * NIN + i] = acc[e];
      }
    }
  }
}

// Sum of the per-tile gradients in tile order; optionally an Adam step on the
// fp32 master weights (bias-corrected, step count `step` >= 1).
__global__ void mlp_reduce_adam_kernel(float* __restrict__ P, const float* __restrict__ partial, int ntiles,
                                       float* __restrict__ grad, float* __restrict__ m, float* __restrict__ v,
                                       int do_adam, float lr, float b1, float b2, float eps, int step) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NPARAM) return;
  float g = 0.f;
  for (int t = 0; t < ntiles; ++t) g += partial[(long long)t * NPARAM + k];
  grad[k] = g;
  if (!do_adam) return;
  const float mk = b1 * m[k] + (1.f - b1) * g;
  const float vk = b2 * v[k] + (1.f - b2) * g * g;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk / (1.f - powf(b1, (float)step));
  const float vh = vk / (1.f - powf(b2, (float)step));
  P[k] -= lr * mh / (sqrtf(vh) + eps);
}

// Features of samples (R, dx, dy, dz) given in FP64; features from index
// n_inputs on are zero (a network trained so has no use for them).
__global__ void mlp_features_kernel(const double* __restrict__ rd, long long n, int n_inputs, float* __restrict__ X) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double d[3] = {rd[4 * s + 1], rd[4 * s + 2], rd[4 * s + 3]};
  float x[NIN];
  eps_features(d, rd[4 * s], x);
#pragma unroll
  for (int k = 0; k < NIN; ++k) X[s * NIN + k] = k < n_inputs ? x[k] : 0.f;
}

// ------------------------------------------------------------------------ launchers
hipError_t launch_mlp_features(const double* rd, long long n, int n_inputs, float* X, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rd, n, n_inputs, X);
  return hipGetLastError();
}

hipError_t launch_mlp_infer_count(const float* P, const float* X, const int* count, long long cap, float* y,
                                  hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  const long long tiles = (cap + 31) / 32;
  // about eight tiles per wave (four waves per workgroup), so that prefetching pays
  const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>((tiles + 31) / 32, 8192));
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(grid), dim3(256), 0, st, P, X, cap, count, y);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* P, const float* X, long long n, float* y, hipStream_t st) {
  return launch_mlp_infer_count(P, X, nullptr, n, y, st);
}

hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, long long n, long long b0, long long mult,
                           long long add, int batch, float* partial, hipStream_t st) {
  const int tiles = (batch + 31) / 32;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((tiles + 3) / 4), dim3(256), 0, st, P, X, T, n, b0, mult, add, batch,
                     partial);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce_adam(float* P, const float* partial, int ntiles, float* grad, float* m, float* v,
                                  int do_adam, float lr, float b1, float b2, float eps, int step, hipStream_t st) {
  hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, P, partial, ntiles, grad, m,
                     v, do_adam, lr, b1, b2, eps, step);
  return hipGetLastError();
}

int mlp_nparam() { return NPARAM; }

}  // namespace lbm
