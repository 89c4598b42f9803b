// Learned warm start: MLP 12 -> 64 -> 64 -> 64 -> 3 with ReLU on the hidden layers,
// forward and backward on gfx950 BF16 MFMA tiles (v_mfma_f32_16x16x16_bf16) with FP32
// accumulation.
//
// Layout: every product is computed transposed, Z^T = W H^T, with the weight tile as
// the A operand (rows = output features) and the activations as the B operand
// (rows = input features, columns = 16 samples).  The accumulator layout of one layer
// (lane l holds rows 4*(l/16)..+3 of column l%16) is then exactly the B-operand layout
// the next layer needs, so activations stay in registers between layers; only the
// weight-gradient products (sum over samples) go through an LDS transpose.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nsn_layout.h"

namespace nsn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = kMlpIn, kH = kMlpHidden, kOut = kMlpOut;
// parameter offsets (floats) in the FP32 master layout
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kOut * kH;
static_assert(oB4 + kOut == kMlpParams, "parameter layout");

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
  return r;
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights staged in LDS as bf16, row-major [out][in] with the input dimension of W1
// padded to 16 and the output dimension of W4 padded to 16 (zeros).
struct MlpLds {
  unsigned short W1[kH * 16];
  unsigned short W2[kH * kH];
  unsigned short W3[kH * kH];
  unsigned short W4[16 * kH];
  float b1[kH], b2[kH], b3[kH], b4[16];
};

__device__ void stage_weights(MlpLds &L, const float *w) {
  for (int i = threadIdx.x; i < kH * 16; i += blockDim.x) {
    const int r = i >> 4, c = i & 15;
    L.W1[i] = c < kIn ? f2bf(w[oW1 + r * kIn + c]) : 0;
  }
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
    L.W2[i] = f2bf(w[oW2 + i]);
    L.W3[i] = f2bf(w[oW3 + i]);
  }
  for (int i = threadIdx.x; i < 16 * kH; i += blockDim.x) {
    const int r = i / kH;
    L.W4[i] = r < kOut ? f2bf(w[oW4 + i]) : 0;
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    L.b1[i] = w[oB1 + i];
    L.b2[i] = w[oB2 + i];
    L.b3[i] = w[oB3 + i];
  }
  for (int i = threadIdx.x; i < 16; i += blockDim.x) L.b4[i] = i < kOut ? w[oB4 + i] : 0.f;
}

// A fragment of a row-major bf16 matrix with `ld` columns: rows r0..r0+15, cols k0..k0+15
__device__ __forceinline__ bf16x4 afrag(const unsigned short *W, int ld, int r0, int k0, int lane) {
  const unsigned short *p = W + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
  bf16x4 r;
  r[0] = (short)p[0]; r[1] = (short)p[1]; r[2] = (short)p[2]; r[3] = (short)p[3];
  return r;
}
// A fragment of the TRANSPOSE of a row-major matrix W [rows x ld]: A[i][k] = W[k][i]
__device__ __forceinline__ bf16x4 afragT(const unsigned short *W, int ld, int i0, int k0, int lane) {
  const int i = i0 + (lane & 15), k = k0 + 4 * (lane >> 4);
  bf16x4 r;
  r[0] = (short)W[(k + 0) * ld + i]; r[1] = (short)W[(k + 1) * ld + i];
  r[2] = (short)W[(k + 2) * ld + i]; r[3] = (short)W[(k + 3) * ld + i];
  return r;
}

struct Acts {
  f32x4 h1[4], h2[4], h3[4];  // post-ReLU activations, tile t holds features 16t + 4*(l/16) + v
  f32x4 y;                    // outputs (rows 0..2 valid in lanes 0..15)
};

// forward of one 16-sample tile; x: the B fragment of the inputs (features 4*(l/16)..+3
// of sample l%16, zero padded to 16)
__device__ __forceinline__ void forward_tile(const MlpLds &L, bf16x4 x, int lane, Acts &a) {
  const int rb = 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(afrag(L.W1, 16, 16 * t, 0, lane), x, acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fmaxf(acc[v] + L.b1[16 * t + rb + v], 0.f);
    a.h1[t] = acc;
  }
  bf16x4 hb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) hb[t] = pack4(a.h1[t][0], a.h1[t][1], a.h1[t][2], a.h1[t][3]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = mfma(afrag(L.W2, kH, 16 * t, 16 * ks, lane), hb[ks], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fmaxf(acc[v] + L.b2[16 * t + rb + v], 0.f);
    a.h2[t] = acc;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) hb[t] = pack4(a.h2[t][0], a.h2[t][1], a.h2[t][2], a.h2[t][3]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = mfma(afrag(L.W3, kH, 16 * t, 16 * ks, lane), hb[ks], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fmaxf(acc[v] + L.b3[16 * t + rb + v], 0.f);
    a.h3[t] = acc;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) hb[t] = pack4(a.h3[t][0], a.h3[t][1], a.h3[t][2], a.h3[t][3]);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = mfma(afrag(L.W4, kH, 0, 16 * ks, lane), hb[ks], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] += L.b4[rb + v];
  a.y = acc;
}

__device__ __forceinline__ bf16x4 load_x(const float *X, long long n, long long s0, int lane,
                                         const float *mean, const float *inv_std) {
  const long long s = s0 + (lane & 15);
  const int k = 4 * (lane >> 4);
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  if (s < n && k < kIn) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float xv = X[s * kIn + k + j];
      if (mean) xv = (xv - mean[k + j]) * inv_std[k + j];
      v[j] = xv;
    }
  }
  return pack4(v[0], v[1], v[2], v[3]);
}

// ---------------------------------------------------------------------------
// forward over n samples (device buffers)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const float *w, const float *X, float *Y, long long n) {
  __shared__ MlpLds L;
  stage_weights(L, w);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const long long ntiles = (n + 15) / 16;
  for (long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); t < ntiles; t += (long long)gridDim.x * 4) {
    Acts a;
    forward_tile(L, load_x(X, n, 16 * t, lane, nullptr, nullptr), lane, a);
    const long long s = 16 * t + (lane & 15);
    if (lane < 16 && s < n) {
#pragma unroll
      for (int o = 0; o < kOut; ++o) Y[s * kOut + o] = a.y[o];
    }
  }
}

// ---------------------------------------------------------------------------
// learned warm start inside a step: every contact of every env, standardised
// features in, de-standardised (lambda_n, lambda_t1, lambda_t2) out.  One block per env.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_warm_mlp(DevScene S, int hybrid) {
  __shared__ MlpLds L;
  __shared__ float xm[kIn], xis[kIn], ym[kOut], ys[kOut];
  const int e = blockIdx.x;
  const int nc = S.n_con[e];
  if (nc == 0) return;
  stage_weights(L, S.mlp);
  const float *norm = S.mlp + kMlpParams;
  if (threadIdx.x < kIn) {
    xm[threadIdx.x] = norm[threadIdx.x];
    xis[threadIdx.x] = 1.f / norm[kIn + threadIdx.x];
  }
  if (threadIdx.x < kOut) {
    ym[threadIdx.x] = norm[2 * kIn + threadIdx.x];
    ys[threadIdx.x] = norm[2 * kIn + kOut + threadIdx.x];
  }
  __syncthreads();
  const EnvInfo E = S.env[e];
  const int lane = threadIdx.x & 63;
  const float *X = S.c_feat + (size_t)E.con_off * kIn;
  for (int t = threadIdx.x >> 6; 16 * t < nc; t += 4) {
    Acts a;
    forward_tile(L, load_x(X, nc, 16 * t, lane, xm, xis), lane, a);
    const int s = 16 * t + (lane & 15);
    // hybrid mode: a contact whose key existed in the previous step (feature 11) keeps
    // the previous-step multipliers already in c_lam0; only new contacts take the
    // prediction
    if (lane < 16 && s < nc && !(hybrid && X[(size_t)s * kIn + 11] != 0.f)) {
      S.c_lam0[E.con_off + s] = make_float4(a.y[0] * ys[0] + ym[0], a.y[1] * ys[1] + ym[1],
                                            a.y[2] * ys[2] + ym[2], 0.f);
    }
  }
}

hipError_t launch_warm_mlp(const DevScene &s, int hybrid, hipStream_t st) {
  hipLaunchKernelGGL(k_warm_mlp, dim3(s.n_envs), dim3(256), 0, st, s, hybrid);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// loss (mean squared error over n x 3) and gradient.  Each block reduces its tiles
// into a partial gradient (fixed order); k_mlp_reduce sums the partials in block
// order, so the result is deterministic (no atomics).
// ---------------------------------------------------------------------------
constexpr int kGradBlocks = 256;

struct GradLds {
  MlpLds L;
  float zt[4][16 * kH];  // per-wave transposed dZ tile [sample][feature]
  float ht[4][16 * kH];  // per-wave transposed activation tile [sample][feature]
};

// dW[o][i] += sum_s dz[o][s] h[i][s] over one tile, with dz and h given in accumulator
// layout (tile t holds features 16t + 4*(l/16) + v of sample l%16); the products run
// on MFMA after an LDS transpose.  acc: [no/16][ni/16] accumulator tiles.
template <int NO, int NI>
__device__ __forceinline__ void accum_wgrad(const f32x4 *dz, const f32x4 *h, float *zt, float *ht, int lane,
                                            f32x4 (&acc)[NO / 16][NI / 16]) {
  const int s = lane & 15, rb = 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < NO / 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) zt[s * kH + 16 * t + rb + v] = dz[t][v];
#pragma unroll
  for (int t = 0; t < NI / 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) ht[s * kH + 16 * t + rb + v] = h[t][v];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // A[o][s] = dz[o][s]: lane holds o = 16mt + l%16, s = 4*(l/16)+j
  // B[s][i] = h[i][s]: lane holds s = 4*(l/16)+j, i = 16nt + l%16
#pragma unroll
  for (int mt = 0; mt < NO / 16; ++mt) {
    const int o = 16 * mt + (lane & 15);
    const bf16x4 a = pack4(zt[(rb + 0) * kH + o], zt[(rb + 1) * kH + o], zt[(rb + 2) * kH + o], zt[(rb + 3) * kH + o]);
#pragma unroll
    for (int nt = 0; nt < NI / 16; ++nt) {
      const int i = 16 * nt + (lane & 15);
      const bf16x4 b = pack4(ht[(rb + 0) * kH + i], ht[(rb + 1) * kH + i], ht[(rb + 2) * kH + i], ht[(rb + 3) * kH + i]);
      acc[mt][nt] = mfma(a, b, acc[mt][nt]);
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int NO, int NI>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[NO / 16][NI / 16]) {
#pragma unroll
  for (int a = 0; a < NO / 16; ++a)
#pragma unroll
    for (int b = 0; b < NI / 16; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// store accumulator tiles (D layout: rows 16mt + 4*(l/16) + v, cols 16nt + l%16) of
// dW [no x ni] into out (row-major with ld = ldo, only ni_valid columns / no_valid rows)
template <int NO, int NI>
__device__ __forceinline__ void store_acc(const f32x4 (&acc)[NO / 16][NI / 16], float *out, int ldo, int no_valid,
                                          int ni_valid, int lane) {
#pragma unroll
  for (int mt = 0; mt < NO / 16; ++mt)
#pragma unroll
    for (int nt = 0; nt < NI / 16; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = 16 * mt + 4 * (lane >> 4) + v, i = 16 * nt + (lane & 15);
        if (o < no_valid && i < ni_valid) out[o * ldo + i] = acc[mt][nt][v];
      }
}

__global__ __launch_bounds__(256) void k_mlp_grad(const float *w, const float *X, const float *T, long long n,
                                                  float *partial, float *loss_part) {
  __shared__ GradLds G;
  stage_weights(G.L, w);
  __syncthreads();
  const MlpLds &L = G.L;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rb = 4 * (lane >> 4);
  float *zt = G.zt[wv], *ht = G.ht[wv];
  f32x4 gW1[kH / 16][1], gW2[kH / 16][kH / 16], gW3[kH / 16][kH / 16], gW4[1][kH / 16];
  zero_acc<kH, 16>(gW1);
  zero_acc<kH, kH>(gW2);
  zero_acc<kH, kH>(gW3);
  zero_acc<16, kH>(gW4);
  float gb1[4][4], gb2[4][4], gb3[4][4], gb4[4];
  for (int t = 0; t < 4; ++t)
    for (int v = 0; v < 4; ++v) gb1[t][v] = gb2[t][v] = gb3[t][v] = 0.f;
  for (int v = 0; v < 4; ++v) gb4[v] = 0.f;
  float loss = 0.f;
  const float scale = 2.f / (float)(n * kOut);
  const long long ntiles = (n + 15) / 16;
  for (long long tile = (long long)blockIdx.x * 4 + wv; tile < ntiles; tile += (long long)gridDim.x * 4) {
    const bf16x4 x = load_x(X, n, 16 * tile, lane, nullptr, nullptr);
    Acts a;
    forward_tile(L, x, lane, a);
    const long long s = 16 * tile + (lane & 15);
    const bool valid = s < n;
    // dY (rows 0..2 live in lanes 0..15)
    f32x4 dy = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = rb + v;
      if (o < kOut && valid) {
        const float e = a.y[v] - T[s * kOut + o];
        loss += e * e;
        dy[v] = scale * e;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) gb4[v] += dy[v];
    // gradient of W4: dy [16(3) x s] times h3^T
    {
      f32x4 dz4[1] = {dy};
      accum_wgrad<16, kH>(dz4, a.h3, zt, ht, lane, gW4);
    }
    // dH3 = W4^T dY, masked by ReLU
    const bf16x4 dyb = pack4(dy[0], dy[1], dy[2], dy[3]);
    f32x4 dz3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(afragT(L.W4, kH, 16 * t, 0, lane), dyb, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = a.h3[t][v] > 0.f ? acc[v] : 0.f;
      dz3[t] = acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) gb3[t][v] += acc[v];
    }
    accum_wgrad<kH, kH>(dz3, a.h2, zt, ht, lane, gW3);
    bf16x4 zb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) zb[t] = pack4(dz3[t][0], dz3[t][1], dz3[t][2], dz3[t][3]);
    f32x4 dz2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mfma(afragT(L.W3, kH, 16 * t, 16 * ks, lane), zb[ks], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = a.h2[t][v] > 0.f ? acc[v] : 0.f;
      dz2[t] = acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) gb2[t][v] += acc[v];
    }
    accum_wgrad<kH, kH>(dz2, a.h1, zt, ht, lane, gW2);
#pragma unroll
    for (int t = 0; t < 4; ++t) zb[t] = pack4(dz2[t][0], dz2[t][1], dz2[t][2], dz2[t][3]);
    f32x4 dz1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mfma(afragT(L.W2, kH, 16 * t, 16 * ks, lane), zb[ks], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = a.h1[t][v] > 0.f ? acc[v] : 0.f;
      dz1[t] = acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) gb1[t][v] += acc[v];
    }
    // gradient of W1: dz1 [64 x s] times x^T (x in accumulator layout: features 4*(l/16)+v)
    f32x4 xa[1];
    {
      const long long ss = 16 * tile + (lane & 15);
      const int k = 4 * (lane >> 4);
      f32x4 xv = {0.f, 0.f, 0.f, 0.f};
      if (ss < n && k < kIn)
        for (int j = 0; j < 4; ++j) xv[j] = X[ss * kIn + k + j];
      xa[0] = xv;
    }
    accum_wgrad<kH, 16>(dz1, xa, zt, ht, lane, gW1);
  }
  // ---- per-block reduction of the four waves (fixed order) into `partial` ----
  float *out = partial + (size_t)blockIdx.x * kMlpParams;
  // each wave writes its part to LDS scratch sequentially: reuse zt/ht as staging
  __syncthreads();
  float *stage = &G.zt[0][0];  // 4 * 16 * 64 floats = 4096 >= one 64x64 matrix
  for (int w = 0; w < 4; ++w) {
    // W2 and W3 (64 x 64) through the stage, one matrix at a time
    for (int m = 0; m < 4; ++m) {
      if (wv == w) {
        if (m == 0) store_acc<kH, kH>(gW2, stage, kH, kH, kH, lane);
        if (m == 1) store_acc<kH, kH>(gW3, stage, kH, kH, kH, lane);
        if (m == 2) store_acc<kH, 16>(gW1, stage, kIn, kH, kIn, lane);
        if (m == 3) store_acc<16, kH>(gW4, stage, kH, kOut, kH, lane);
      }
      __syncthreads();
      const int off = m == 0 ? oW2 : (m == 1 ? oW3 : (m == 2 ? oW1 : oW4));
      const int cnt = m < 2 ? kH * kH : (m == 2 ? kH * kIn : kOut * kH);
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) out[off + i] = (w == 0 ? 0.f : out[off + i]) + stage[i];
      __syncthreads();
    }
  }
  // biases: lanes hold features 16t + 4*(l/16) + v summed over their own sample column;
  // sum over the 16 sample lanes of each row group and over waves in a fixed order
  float *bst = &G.ht[0][0];
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) bst[i] = 0.f;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
      for (int t = 0; t < 4; ++t)
        for (int v = 0; v < 4; ++v) {
          float s1 = gb1[t][v], s2 = gb2[t][v], s3 = gb3[t][v];
          for (int o = 8; o > 0; o >>= 1) {
            s1 += __shfl_xor(s1, o, 16);
            s2 += __shfl_xor(s2, o, 16);
            s3 += __shfl_xor(s3, o, 16);
          }
          if ((lane & 15) == 0) {
            const int f = 16 * t + rb + v;
            bst[f] += s1;
            bst[64 + f] += s2;
            bst[128 + f] += s3;
          }
        }
      for (int v = 0; v < 4; ++v) {
        float s4 = gb4[v];
        for (int o = 8; o > 0; o >>= 1) s4 += __shfl_xor(s4, o, 16);
        if ((lane & 15) == 0 && rb + v < kOut) bst[192 + rb + v] += s4;
      }
      float l = loss;
      for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
      if (lane == 0) bst[256] += l;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    out[oB1 + i] = bst[i];
    out[oB2 + i] = bst[64 + i];
    out[oB3 + i] = bst[128 + i];
  }
  if (threadIdx.x < kOut) out[oB4 + threadIdx.x] = bst[192 + threadIdx.x];
  if (threadIdx.x == 0) loss_part[blockIdx.x] = bst[256];
}

__global__ void k_mlp_reduce(const float *partial, const float *loss_part, int nblocks, float *grad, float *loss,
                             float loss_scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) {
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * kMlpParams + i];
    grad[i] = s;
  }
  if (i == 0 && loss) {
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += loss_part[b];
    *loss = s * loss_scale;
  }
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace nsn

using namespace nsn;

extern "C" {

nsn_status nsn_mlp_forward(const float *w, const float *x, float *y, int64_t n, void *stream) {
  if (!w || !x || !y || n < 0) return NSN_EINVAL;
  if (n == 0) return NSN_OK;
  const long long tiles = (n + 15) / 16;
  const int blocks = (int)std::min<long long>((tiles + 3) / 4, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, (hipStream_t)stream, w, x, y, (long long)n);
  return hipGetLastError() == hipSuccess ? NSN_OK : NSN_EDEVICE;
}

size_t nsn_mlp_scratch_bytes(int64_t n) {
  (void)n;
  return sizeof(float) * ((size_t)kGradBlocks * kMlpParams + kGradBlocks);
}

nsn_status nsn_mlp_loss_grad(const float *w, const float *x, const float *t, int64_t n, float *grad, float *loss_out,
                             void *scratch, void *stream) {
  if (!w || !x || !t || !grad || !scratch || n <= 0) return NSN_EINVAL;
  float *partial = (float *)scratch;
  float *loss_part = partial + (size_t)kGradBlocks * kMlpParams;
  const long long tiles = (n + 15) / 16;
  const int blocks = (int)std::min<long long>((tiles + 3) / 4, kGradBlocks);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, st, w, x, t, (long long)n, partial, loss_part);
  if (hipGetLastError() != hipSuccess) return NSN_EDEVICE;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, partial, loss_part, blocks, grad,
                     loss_out, 1.f / (float)(n * kOut));
  return hipGetLastError() == hipSuccess ? NSN_OK : NSN_EDEVICE;
}

nsn_status nsn_mlp_adam(float *w, const float *grad, float *m, float *v, int64_t n_params, float lr, float beta1,
                        float beta2, float eps, int32_t step, void *stream) {
  if (!w || !grad || !m || !v || n_params <= 0 || step < 1) return NSN_EINVAL;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n_params + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w, grad, m,
                     v, (long long)n_params, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? NSN_OK : NSN_EDEVICE;
}

}  // extern "C"
