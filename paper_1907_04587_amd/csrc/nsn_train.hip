// Training of the warm-start network on the device (nsn_train_warm_start): data
// clipping to per-column quantiles, z-scoring, seeded initialisation, shuffled
// mini-batches and Adam, all as kernels on the caller's stream; the host only
// sequences the launches.  The products run in the library's BF16-MFMA loss/gradient
// kernel (nsn_mlp_loss_grad) and its Adam kernel (nsn_mlp_adam).
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nsn_layout.h"

namespace nsn {
namespace {

constexpr int kCols = kMlpIn + kMlpOut;  // 15 data columns: features then targets

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a counter-based 64-bit mixer.
__host__ __device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// A bijection of [0, n): a balanced 4-round Feistel network on [0, 2^(2 half)) with
// round keys from `key`, walked along its cycle until the value falls below n (a
// permutation restricted this way stays a bijection of [0, n)).
__device__ __forceinline__ unsigned int feistel_perm(unsigned int i, unsigned int n, int half,
                                                     unsigned long long key) {
  const unsigned int mask = (1u << half) - 1u;
  unsigned int x = i;
  do {
    unsigned int l = x >> half, r = x & mask;
#pragma unroll
    for (int round = 0; round < 4; ++round) {
      const unsigned int f = (unsigned int)splitmix64(key + 0x100000000ull * round + r) & mask;
      const unsigned int nl = r, nr = l ^ f;
      l = nl;
      r = nr;
    }
    x = (l << half) | r;
  } while (x >= n);
  return x;
}

// every value finite? (flag stays 0 if so)
__global__ void k_check_finite(const float *a, long long n, int *flag) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(a[i])) *flag = 1;
}

// column c of an [n x ncols] array into a contiguous buffer
__global__ void k_column(const float *a, long long n, int ncols, int c, float *out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = a[i * ncols + c];
}

// clip bounds of one column from its sorted values: the q and 1-q quantiles with
// linear interpolation between order statistics (position q (n-1))
__global__ void k_quantile_bounds(const float *sorted, long long n, double q, float *lo, float *hi) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  auto at = [&](double pos) {
    const long long i = (long long)floor(pos);
    const double f = pos - (double)i;
    const double a = sorted[i], b = sorted[i + 1 < n ? i + 1 : i];
    return (float)(a + f * (b - a));
  };
  *lo = at((double)q * (double)(n - 1));
  *hi = at((1.0 - (double)q) * (double)(n - 1));
}

// clipped copy of column c, mean and standard deviation (population, FP64, fixed
// reduction order: one workgroup per column)
__global__ __launch_bounds__(1024) void k_column_stats(const float *x, const float *t, long long n,
                                                       const float *lo, const float *hi, int clip, double *mean,
                                                       double *sd) {
  __shared__ double red[1024];
  const int c = blockIdx.x;
  const float *a = c < kMlpIn ? x : t;
  const int ncols = c < kMlpIn ? kMlpIn : kMlpOut, cc = c < kMlpIn ? c : c - kMlpIn;
  const float l = clip ? lo[c] : -INFINITY, h = clip ? hi[c] : INFINITY;
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) s += (double)fminf(fmaxf(a[i * ncols + cc], l), h);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double m = red[0] / (double)n;
  __syncthreads();
  double s2 = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = (double)fminf(fmaxf(a[i * ncols + cc], l), h) - m;
    s2 += d * d;
  }
  red[threadIdx.x] = s2;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[c] = m;
    sd[c] = sqrt(red[0] / (double)n);
  }
}

// float32 statistics (a deviation below 1e-6 counts as 1) into the blob tail:
// x_mean[12] x_std[12] y_mean[3] y_std[3]
__global__ void k_stats_out(const double *mean, const double *sd, float *tail) {
  const int c = threadIdx.x;
  if (c >= kCols) return;
  const float m = (float)mean[c];
  float s = (float)sd[c];
  if (!(s > 1e-6f)) s = 1.f;
  if (c < kMlpIn) {
    tail[c] = m;
    tail[kMlpIn + c] = s;
  } else {
    tail[2 * kMlpIn + (c - kMlpIn)] = m;
    tail[2 * kMlpIn + kMlpOut + (c - kMlpIn)] = s;
  }
}

// z-scored, clipped copies of x and t
__global__ void k_standardise(const float *x, const float *t, long long n, const float *lo, const float *hi, int clip,
                              const float *tail, float *xn, float *tn) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n * kCols;
       i += (long long)gridDim.x * blockDim.x) {
    const long long s = i / kCols;
    const int c = (int)(i - s * kCols);
    const float v = c < kMlpIn ? x[s * kMlpIn + c] : t[s * kMlpOut + (c - kMlpIn)];
    const float vc = clip ? fminf(fmaxf(v, lo[c]), hi[c]) : v;
    if (c < kMlpIn) xn[s * kMlpIn + c] = (vc - tail[c]) / tail[kMlpIn + c];
    else tn[s * kMlpOut + (c - kMlpIn)] = (vc - tail[2 * kMlpIn + (c - kMlpIn)]) / tail[2 * kMlpIn + kMlpOut + (c - kMlpIn)];
  }
}

// He initialisation: weights N(0, 2 / fan_in) from counter-based normal draws
// (SplitMix64 of seed and index, Box-Muller), biases 0
__global__ void k_init(float *w, unsigned long long seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  constexpr int oB1 = kMlpHidden * kMlpIn, oW2 = oB1 + kMlpHidden, oB2 = oW2 + kMlpHidden * kMlpHidden,
                oW3 = oB2 + kMlpHidden, oB3 = oW3 + kMlpHidden * kMlpHidden, oW4 = oB3 + kMlpHidden,
                oB4 = oW4 + kMlpOut * kMlpHidden;
  int fan = 0;
  if (i < oB1) fan = kMlpIn;
  else if (i >= oW2 && i < oB2) fan = kMlpHidden;
  else if (i >= oW3 && i < oB3) fan = kMlpHidden;
  else if (i >= oW4 && i < oB4) fan = kMlpHidden;
  if (fan == 0) {
    w[i] = 0.f;
    return;
  }
  const unsigned long long r = splitmix64(seed ^ splitmix64((unsigned long long)i));
  const double u1 = ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((double)(splitmix64(r) >> 11)) * (1.0 / 9007199254740992.0);
  const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  w[i] = (float)(z * sqrt(2.0 / (double)fan));
}

// one mini-batch: rows b0 .. b0+nb of the epoch's permutation
__global__ void k_gather_batch(const float *xn, const float *tn, unsigned int n, int half, unsigned long long key,
                               long long b0, int nb, float *xb, float *tb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const unsigned int s = feistel_perm((unsigned int)(b0 + j), n, half, key);
#pragma unroll
  for (int c = 0; c < kMlpIn; ++c) xb[(size_t)j * kMlpIn + c] = xn[(size_t)s * kMlpIn + c];
#pragma unroll
  for (int c = 0; c < kMlpOut; ++c) tb[(size_t)j * kMlpOut + c] = tn[(size_t)s * kMlpOut + c];
}

__global__ void k_loss_acc(const float *loss, int nb, double *acc, int reset) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *acc = (reset ? 0.0 : *acc) + (double)(*loss) * nb;
}

__global__ void k_copy(const float *src, float *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Sub-allocation of the training workspace (nullptr base: sizes only).
struct TrainWs {
  float *xn, *tn, *xb, *tb, *col, *sorted, *w, *g, *m, *v, *loss, *lo, *hi;
  double *mean, *sd, *acc;
  int *flag;
  void *scratch, *sort_tmp;
  size_t sort_bytes, bytes;
  bool ok;  // the sort's temporary-storage query succeeded
};

TrainWs carve(char *base, long long n, int batch) {
  TrainWs W{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    char *p = base ? base + off : nullptr;
    off += std::max<size_t>(bytes, 1);
    return (void *)p;
  };
  W.sort_bytes = 0;
  W.ok = hipcub::DeviceRadixSort::SortKeys(nullptr, W.sort_bytes, (const float *)nullptr, (float *)nullptr, (int)n) ==
         hipSuccess;
  W.xn = (float *)take(sizeof(float) * kMlpIn * n);
  W.tn = (float *)take(sizeof(float) * kMlpOut * n);
  W.xb = (float *)take(sizeof(float) * kMlpIn * (size_t)batch);
  W.tb = (float *)take(sizeof(float) * kMlpOut * (size_t)batch);
  W.col = (float *)take(sizeof(float) * n);
  W.sorted = (float *)take(sizeof(float) * n);
  W.w = (float *)take(sizeof(float) * kMlpParams);
  W.g = (float *)take(sizeof(float) * kMlpParams);
  W.m = (float *)take(sizeof(float) * kMlpParams);
  W.v = (float *)take(sizeof(float) * kMlpParams);
  W.loss = (float *)take(sizeof(float));
  W.lo = (float *)take(sizeof(float) * kCols);
  W.hi = (float *)take(sizeof(float) * kCols);
  W.mean = (double *)take(sizeof(double) * kCols);
  W.sd = (double *)take(sizeof(double) * kCols);
  W.acc = (double *)take(sizeof(double));
  W.flag = (int *)take(sizeof(int));
  W.scratch = take(nsn_mlp_scratch_bytes(batch));
  W.sort_tmp = take(W.sort_bytes);
  W.bytes = off + 256;
  return W;
}

}  // namespace
}  // namespace nsn

using namespace nsn;

extern "C" {

size_t nsn_train_workspace_bytes(int64_t n, int32_t batch) {
  if (n < 2 || n >= (1ll << 31) || batch < 1) return 0;
  const TrainWs W = carve(nullptr, n, std::min<int64_t>(batch, n));
  return W.ok ? W.bytes : 0;
}

nsn_status nsn_train_warm_start(const float *x, const float *t, int64_t n, const nsn_train_params *tp,
                                const float *w_init, float *blob_out, double *loss_hist, void *workspace,
                                size_t workspace_bytes, void *stream) {
  if (!x || !t || !tp || !blob_out || !workspace || n < 2 || n >= (1ll << 31) || tp->batch < 1 || tp->epochs < 1 ||
      !(tp->lr > 0.f) || !(tp->beta1 >= 0.f && tp->beta1 < 1.f) || !(tp->beta2 >= 0.f && tp->beta2 < 1.f) ||
      !(tp->adam_eps > 0.f) || !(tp->clip_quantile >= 0.f && tp->clip_quantile < 0.5f))
    return NSN_EINVAL;
  const int batch = (int)std::min<long long>(tp->batch, n);
  TrainWs W = carve(nullptr, n, batch);
  if (!W.ok) return NSN_EDEVICE;
  if (workspace_bytes < W.bytes || ((uintptr_t)workspace & 255)) return NSN_ENOMEM;
  W = carve((char *)((uintptr_t)workspace), n, batch);
  hipStream_t st = (hipStream_t)stream;
#define TRY(expr)                                  \
  do {                                             \
    if ((expr) != hipSuccess) return NSN_EDEVICE;  \
  } while (0)
#define LAUNCHED() TRY(hipGetLastError())
  const int grid = 1024;
  // inputs must be finite
  TRY(hipMemsetAsync(W.flag, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_check_finite, dim3(grid), dim3(256), 0, st, x, (long long)n * kMlpIn, W.flag);
  LAUNCHED();
  hipLaunchKernelGGL(k_check_finite, dim3(grid), dim3(256), 0, st, t, (long long)n * kMlpOut, W.flag);
  LAUNCHED();
  int flag = 0;
  TRY(hipMemcpyAsync(&flag, W.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  if (flag) return NSN_EINVAL;
  // 1. per-column quantile bounds from a radix sort of each column
  const int clip = tp->clip_quantile > 0.f ? 1 : 0;
  if (clip) {
    for (int c = 0; c < kCols; ++c) {
      if (c < kMlpIn) hipLaunchKernelGGL(k_column, dim3(grid), dim3(256), 0, st, x, (long long)n, kMlpIn, c, W.col);
      else hipLaunchKernelGGL(k_column, dim3(grid), dim3(256), 0, st, t, (long long)n, kMlpOut, c - kMlpIn, W.col);
      LAUNCHED();
      size_t tb = W.sort_bytes;
      TRY(hipcub::DeviceRadixSort::SortKeys(W.sort_tmp, tb, W.col, W.sorted, (int)n, 0, 32, st));
      hipLaunchKernelGGL(k_quantile_bounds, dim3(1), dim3(1), 0, st, W.sorted, (long long)n,
                         (double)tp->clip_quantile, W.lo + c, W.hi + c);
      LAUNCHED();
    }
  }
  // 2. statistics of the clipped columns and the z-scored data
  hipLaunchKernelGGL(k_column_stats, dim3(kCols), dim3(1024), 0, st, x, t, (long long)n, W.lo, W.hi, clip, W.mean,
                     W.sd);
  LAUNCHED();
  float *tail = blob_out + kMlpParams;
  hipLaunchKernelGGL(k_stats_out, dim3(1), dim3(64), 0, st, W.mean, W.sd, tail);
  LAUNCHED();
  hipLaunchKernelGGL(k_standardise, dim3(grid), dim3(256), 0, st, x, t, (long long)n, W.lo, W.hi, clip, tail, W.xn,
                     W.tn);
  LAUNCHED();
  // 3. initial weights, zero moments
  if (w_init) {
    hipLaunchKernelGGL(k_copy, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, w_init, W.w, kMlpParams);
  } else {
    hipLaunchKernelGGL(k_init, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, W.w, (unsigned long long)tp->seed);
  }
  LAUNCHED();
  TRY(hipMemsetAsync(W.m, 0, sizeof(float) * kMlpParams, st));
  TRY(hipMemsetAsync(W.v, 0, sizeof(float) * kMlpParams, st));
  // 4. epochs of shuffled mini-batches
  int half = 1;
  while ((1ll << (2 * half)) < n) ++half;
  int step = 0;
  for (int ep = 0; ep < tp->epochs; ++ep) {
    const unsigned long long key = splitmix64(tp->seed ^ splitmix64(0xA5A5A5A5ull + (unsigned long long)ep));
    const float lr = tp->lr * 0.5f * (1.f + (float)std::cos(M_PI * (double)ep / (double)tp->epochs));
    for (long long b0 = 0; b0 < n; b0 += batch) {
      const int nb = (int)std::min<long long>(batch, n - b0);
      hipLaunchKernelGGL(k_gather_batch, dim3((nb + 255) / 256), dim3(256), 0, st, W.xn, W.tn, (unsigned int)n, half,
                         key, b0, nb, W.xb, W.tb);
      LAUNCHED();
      nsn_status s = nsn_mlp_loss_grad(W.w, W.xb, W.tb, nb, W.g, W.loss, W.scratch, st);
      if (s) return s;
      s = nsn_mlp_adam(W.w, W.g, W.m, W.v, kMlpParams, lr, tp->beta1, tp->beta2, tp->adam_eps, ++step, st);
      if (s) return s;
      hipLaunchKernelGGL(k_loss_acc, dim3(1), dim3(1), 0, st, W.loss, nb, W.acc, b0 == 0 ? 1 : 0);
      LAUNCHED();
    }
    double acc = 0.0;
    TRY(hipMemcpyAsync(&acc, W.acc, sizeof(double), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    if (!std::isfinite(acc)) return NSN_ENONFINITE;
    if (loss_hist) loss_hist[ep] = acc / (double)n;
  }
  hipLaunchKernelGGL(k_copy, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, W.w, blob_out, kMlpParams);
  LAUNCHED();
  TRY(hipStreamSynchronize(st));
#undef LAUNCHED
#undef TRY
  return NSN_OK;
}

}  // extern "C"
