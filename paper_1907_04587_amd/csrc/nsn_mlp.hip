// Learned warm start: MLP 12 -> 64 -> 64 -> 64 -> 3 with ReLU on the hidden layers,
// forward and backward on gfx950 BF16 MFMA tiles (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation.
//
// Layout: every product is computed transposed, Z^T = W H^T, with the weight tile as
// the A operand (rows = output features) and the activations as the B operand
// (rows = input features, columns = 16 samples).  One 16x16 accumulator tile leaves
// lane l with rows 4*(l/16)..+3 of column l%16.  A K=32 operand gives lane l eight
// slots; the contraction pairs slot i of lane group g = l/16 in A with the same slot of
// the same group in B, so any assignment of the 32 summed indices to (group, slot)
// serves, as long as both operands use it.  Here slots 0..3 of group g carry index
// 4g + 0..3 and slots 4..7 carry 16 + 4g + 0..3: the two accumulator tiles of one
// layer (features 0..15 and 16..31 of a 32-chunk) are then, as they stand, the B
// operand of the next layer, and activations stay in registers between layers.  The
// weight-gradient products (sums over 32 samples, two 16-sample tiles) go through an
// LDS transpose.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nsn_layout.h"

namespace nsn {

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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

// slots 0..3 from lo, 4..7 from hi (the summed indices 4g+v and 16+4g+v)
__device__ __forceinline__ s16x8 pack8(f32x4 lo, f32x4 hi) {
  s16x8 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    r[v] = (short)f2bf(lo[v]);
    r[4 + v] = (short)f2bf(hi[v]);
  }
  return r;
}
// slots 0..3 from lo, 4..7 zero (a 16-wide contraction on the 32-wide instruction)
__device__ __forceinline__ s16x8 pack8_lo(f32x4 lo) {
  s16x8 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    r[v] = (short)f2bf(lo[v]);
    r[4 + v] = 0;
  }
  return r;
}

__device__ __forceinline__ f32x4 mfma(s16x8 a, s16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
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

// A fragment of a row-major bf16 matrix with `ld` columns: rows r0..r0+15, summed
// columns k0 + (4g + 0..3, 16 + 4g + 0..3) in the slot order above; lo: only the first
// 16 columns exist (slots 4..7 zero)
template <bool LO = false>
__device__ __forceinline__ s16x8 afrag(const unsigned short *W, int ld, int r0, int k0, int lane) {
  const unsigned short *p = W + (r0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4);
  s16x8 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    r[v] = (short)p[v];
    r[4 + v] = LO ? (short)0 : (short)p[16 + v];
  }
  return r;
}
// the same for the TRANSPOSE of a row-major matrix W [rows x ld]: A[i][k] = W[k][i]
template <bool LO = false>
__device__ __forceinline__ s16x8 afragT(const unsigned short *W, int ld, int i0, int k0, int lane) {
  const int i = i0 + (lane & 15), k = k0 + 4 * (lane >> 4);
  s16x8 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    r[v] = (short)W[(k + v) * ld + i];
    r[4 + v] = LO ? (short)0 : (short)W[(k + 16 + v) * ld + i];
  }
  return r;
}

struct Acts {
  f32x4 h1[4], h2[4], h3[4];  // post-ReLU activations, tile t holds features 16t + 4*(l/16) + v
  f32x4 y;                    // outputs (rows 0..2 valid in lanes 0..15)
};

// forward of one 16-sample tile; x: the B fragment of the inputs (slots 0..3: features
// 4*(l/16)..+3 of sample l%16, zero padded to 16; slots 4..7 zero)
__device__ __forceinline__ void forward_tile(const MlpLds &L, s16x8 x, int lane, Acts &a) {
  const int rb = 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(afrag<true>(L.W1, 16, 16 * t, 0, lane), x, acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fmaxf(acc[v] + L.b1[16 * t + rb + v], 0.f);
    a.h1[t] = acc;
  }
  s16x8 hb[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) hb[j] = pack8(a.h1[2 * j], a.h1[2 * j + 1]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) acc = mfma(afrag(L.W2, kH, 16 * t, 32 * j, lane), hb[j], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fmaxf(acc[v] + L.b2[16 * t + rb + v], 0.f);
    a.h2[t] = acc;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) hb[j] = pack8(a.h2[2 * j], a.h2[2 * j + 1]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) acc = mfma(afrag(L.W3, kH, 16 * t, 32 * j, lane), hb[j], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = fmaxf(acc[v] + L.b3[16 * t + rb + v], 0.f);
    a.h3[t] = acc;
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) hb[j] = pack8(a.h3[2 * j], a.h3[2 * j + 1]);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 2; ++j) acc = mfma(afrag(L.W4, kH, 0, 32 * j, lane), hb[j], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] += L.b4[rb + v];
  a.y = acc;
}

// the raw (unpacked) input features of one tile in accumulator layout (features
// 4*(l/16)+v of sample l%16), standardised when mean is given
__device__ __forceinline__ f32x4 load_xf(const float *X, long long n, long long s0, int lane, const float *mean,
                                         const float *inv_std) {
  const long long s = s0 + (lane & 15);
  const int k = 4 * (lane >> 4);
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (s < n && k < kIn) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float xv = X[s * kIn + k + j];
      if (mean) xv = (xv - mean[k + j]) * inv_std[k + j];
      v[j] = xv;
    }
  }
  return v;
}

__device__ __forceinline__ s16x8 load_x(const float *X, long long n, long long s0, int lane, const float *mean,
                                        const float *inv_std) {
  return pack8_lo(load_xf(X, n, s0, lane, mean, inv_std));
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

// Per-wave LDS of the gradient kernel: for each layer, the transposes of dZ and of the
// layer's input over a 32-sample pair of tiles, bf16 [sample][feature] (layer 4: dY 16
// (3 valid) and h3 64; layer 3: dZ3 and h2; layer 2: dZ2 and h1; layer 1: dZ1 64 and x
// 16 (12 valid)), filled by the backward of both tiles before the weight-gradient
// products run.
constexpr int kPairS = 32;
constexpr int kWaveStage = kPairS * (16 + kH + kH + kH + kH + kH + kH + 16);  // bf16 elements
struct WaveStage {
  unsigned short *z4, *h3, *z3, *h2, *z2, *h1, *z1, *x;
  __device__ explicit WaveStage(unsigned short *b)
      : z4(b), h3(z4 + kPairS * 16), z3(h3 + kPairS * kH), h2(z3 + kPairS * kH), z2(h2 + kPairS * kH),
        h1(z2 + kPairS * kH), z1(h1 + kPairS * kH), x(z1 + kPairS * kH) {}
};
constexpr size_t kGradLdsBytes = sizeof(MlpLds) + 4 * sizeof(unsigned short) * (size_t)kWaveStage;
static_assert(kGradLdsBytes <= 160 * 1024, "gradient kernel LDS");

// write one tile's accumulator-layout values (tile t: features 16t + 4*(l/16) + v of
// sample l%16) as bf16 into rows q*16 + sample of a [32][NF] transpose
template <int NF>
__device__ __forceinline__ void stage_t(const f32x4 *v, unsigned short *dst, int q, int lane) {
  const int s = 16 * q + (lane & 15), rb = 4 * (lane >> 4);
#pragma unroll
  for (int t = 0; t < NF / 16; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[s * NF + 16 * t + rb + k] = f2bf(v[t][k]);
}

// dW[o][i] += sum over the 32 staged samples of dz[o][s] h[i][s], on MFMA with the
// samples in the slot order of the header (slots 0..3 of group g: samples 4g + 0..3 of
// the pair's first tile; slots 4..7: the same samples of its second tile).
// acc: [no/16][ni/16] accumulator tiles.
template <int NO, int NI>
__device__ __forceinline__ void wgrad_mfma(const unsigned short *zt, const unsigned short *ht, int lane,
                                           f32x4 (&acc)[NO / 16][NI / 16]) {
  const int rb = 4 * (lane >> 4);
#pragma unroll
  for (int mt = 0; mt < NO / 16; ++mt) {
    const int o = 16 * mt + (lane & 15);
    s16x8 a;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      a[v] = (short)zt[(rb + v) * NO + o];
      a[4 + v] = (short)zt[(16 + rb + v) * NO + o];
    }
#pragma unroll
    for (int nt = 0; nt < NI / 16; ++nt) {
      const int i = 16 * nt + (lane & 15);
      s16x8 b;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        b[v] = (short)ht[(rb + v) * NI + i];
        b[4 + v] = (short)ht[(16 + rb + v) * NI + i];
      }
      acc[mt][nt] = mfma(a, b, acc[mt][nt]);
    }
  }
}

__device__ __forceinline__ void wave_sync() {
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

// dH of a hidden layer from the next layer's dZ (two accumulator tiles per 32-chunk),
// masked by the ReLU of its pre-activation: dz_out[t] = (W^T dz_in)[tile t] * (h > 0)
__device__ __forceinline__ void back_hidden(const unsigned short *W, const f32x4 *dz_in, const f32x4 *h, int lane,
                                            f32x4 *dz_out) {
  s16x8 zb[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) zb[j] = pack8(dz_in[2 * j], dz_in[2 * j + 1]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) acc = mfma(afragT(W, kH, 16 * t, 32 * j, lane), zb[j], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = h[t][v] > 0.f ? acc[v] : 0.f;
    dz_out[t] = acc;
  }
}

__global__ __launch_bounds__(256) void k_mlp_grad(const float *w, const float *X, const float *T, long long n,
                                                  float *partial, float *loss_part) {
  extern __shared__ __align__(16) unsigned char g_lds[];
  MlpLds &L = *reinterpret_cast<MlpLds *>(g_lds);
  unsigned short *stage_base = reinterpret_cast<unsigned short *>(g_lds + sizeof(MlpLds));
  stage_weights(L, w);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rb = 4 * (lane >> 4);
  const WaveStage ws(stage_base + (size_t)wv * kWaveStage);
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
  const long long ntiles = (n + 15) / 16, npairs = (ntiles + 1) / 2;
  // each wave takes pairs of 16-sample tiles; samples beyond n have dY = 0, so every
  // gradient term they touch is zero
  for (long long pr = (long long)blockIdx.x * 4 + wv; pr < npairs; pr += (long long)gridDim.x * 4) {
    for (int q = 0; q < 2; ++q) {
      const long long tile = 2 * pr + q;
      f32x4 xa[1] = {load_xf(X, n, 16 * tile, lane, nullptr, nullptr)};
      Acts a;
      forward_tile(L, pack8_lo(xa[0]), lane, a);
      const long long s = 16 * tile + (lane & 15);
      const bool valid = s < n;
      f32x4 dy[1] = {{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = rb + v;
        if (o < kOut && valid) {
          const float e = a.y[v] - T[s * kOut + o];
          loss += e * e;
          dy[0][v] = scale * e;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) gb4[v] += dy[0][v];
      stage_t<16>(dy, ws.z4, q, lane);
      stage_t<kH>(a.h3, ws.h3, q, lane);
      // dH3 = W4^T dY (a 16-wide contraction: W4 has 16 padded rows), masked by ReLU
      f32x4 dz3[4];
      const s16x8 dyb = pack8_lo(dy[0]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(afragT<true>(L.W4, kH, 16 * t, 0, lane), dyb, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = a.h3[t][v] > 0.f ? acc[v] : 0.f;
        dz3[t] = acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) gb3[t][v] += acc[v];
      }
      stage_t<kH>(dz3, ws.z3, q, lane);
      stage_t<kH>(a.h2, ws.h2, q, lane);
      f32x4 dz2[4];
      back_hidden(L.W3, dz3, a.h2, lane, dz2);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) gb2[t][v] += dz2[t][v];
      stage_t<kH>(dz2, ws.z2, q, lane);
      stage_t<kH>(a.h1, ws.h1, q, lane);
      f32x4 dz1[4];
      back_hidden(L.W2, dz2, a.h1, lane, dz1);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) gb1[t][v] += dz1[t][v];
      stage_t<kH>(dz1, ws.z1, q, lane);
      stage_t<16>(xa, ws.x, q, lane);
    }
    wave_sync();
    wgrad_mfma<16, kH>(ws.z4, ws.h3, lane, gW4);
    wgrad_mfma<kH, kH>(ws.z3, ws.h2, lane, gW3);
    wgrad_mfma<kH, kH>(ws.z2, ws.h1, lane, gW2);
    wgrad_mfma<kH, 16>(ws.z1, ws.x, lane, gW1);
    wave_sync();  // the next pair overwrites the stage
  }
  // ---- per-block reduction of the four waves (fixed order) into `partial` ----
  float *out = partial + (size_t)blockIdx.x * kMlpParams;
  // each wave writes its part to LDS scratch sequentially: reuse zt/ht as staging
  __syncthreads();
  float *stage = reinterpret_cast<float *>(stage_base);  // >= 4096 floats: one 64x64 matrix
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
  float *bst = reinterpret_cast<float *>(stage_base) + 4096;  // 1024 floats after the matrix stage
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

// the gradient kernel's LDS (above the 64 KB default) is enabled once per device
static bool grad_lds_ready() {
  static bool done[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  if (!done[dev]) {
    if (hipFuncSetAttribute((const void *)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kGradLdsBytes) != hipSuccess)
      return false;
    done[dev] = true;
  }
  return true;
}

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
  const long long pairs = ((n + 15) / 16 + 1) / 2;
  const int blocks = (int)std::min<long long>((pairs + 3) / 4, kGradBlocks);
  hipStream_t st = (hipStream_t)stream;
  if (!grad_lds_ready()) return NSN_EDEVICE;
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), kGradLdsBytes, st, w, x, t, (long long)n, partial,
                     loss_part);
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
