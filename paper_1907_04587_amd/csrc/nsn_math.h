// Small fixed-size vector/matrix helpers for the device code (float32).
#pragma once
#include <hip/hip_runtime.h>

namespace nsn {

struct V3 {
  float x, y, z;
};

__device__ __forceinline__ V3 mk(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 mk(float4 a) { return V3{a.x, a.y, a.z}; }
__device__ __forceinline__ float4 f4(V3 a, float w) { return make_float4(a.x, a.y, a.z, w); }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator-(V3 a) { return V3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float norm(V3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ float comp(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Row-major 3x3.
struct M3 {
  float m[9];
};

__device__ __forceinline__ V3 mul(const M3 &A, V3 v) {
  return V3{A.m[0] * v.x + A.m[1] * v.y + A.m[2] * v.z, A.m[3] * v.x + A.m[4] * v.y + A.m[5] * v.z,
            A.m[6] * v.x + A.m[7] * v.y + A.m[8] * v.z};
}
__device__ __forceinline__ V3 mulT(const M3 &A, V3 v) {
  return V3{A.m[0] * v.x + A.m[3] * v.y + A.m[6] * v.z, A.m[1] * v.x + A.m[4] * v.y + A.m[7] * v.z,
            A.m[2] * v.x + A.m[5] * v.y + A.m[8] * v.z};
}
__device__ __forceinline__ V3 col(const M3 &A, int c) { return V3{A.m[c], A.m[3 + c], A.m[6 + c]}; }

__device__ __forceinline__ M3 quat_mat(float4 q) {
  float w = q.x, x = q.y, y = q.z, z = q.w;
  M3 R;
  R.m[0] = 1.f - 2.f * (y * y + z * z);
  R.m[1] = 2.f * (x * y - w * z);
  R.m[2] = 2.f * (x * z + w * y);
  R.m[3] = 2.f * (x * y + w * z);
  R.m[4] = 1.f - 2.f * (x * x + z * z);
  R.m[5] = 2.f * (y * z - w * x);
  R.m[6] = 2.f * (x * z - w * y);
  R.m[7] = 2.f * (y * z + w * x);
  R.m[8] = 1.f - 2.f * (x * x + y * y);
  return R;
}

__device__ __forceinline__ float4 quat_normalize(float4 q) {
  float l = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  return make_float4(q.x / l, q.y / l, q.z / l, q.w / l);
}

// symmetric 3x3 stored as (xx yy zz xy xz yz)
__device__ __forceinline__ V3 sym_mul(const float *s, V3 v) {
  return V3{s[0] * v.x + s[3] * v.y + s[4] * v.z, s[3] * v.x + s[1] * v.y + s[5] * v.z,
            s[4] * v.x + s[5] * v.y + s[2] * v.z};
}

__device__ __forceinline__ float det3(const M3 &A) {
  return A.m[0] * (A.m[4] * A.m[8] - A.m[5] * A.m[7]) - A.m[1] * (A.m[3] * A.m[8] - A.m[5] * A.m[6]) +
         A.m[2] * (A.m[3] * A.m[7] - A.m[4] * A.m[6]);
}

// ---- global-memory access through address-space-1 pointers ----
// The scene's arrays are reached through pointers read from memory, which the compiler
// cannot prove global: a plain access through them is a FLAT instruction, and a FLAT
// load counts against the counter of LDS and scalar loads as well, so every wait for an
// LDS read or a pointer reload also waits for the memory loads in flight.  gld / gst
// issue GLOBAL instructions instead (same address, same data).
#define NSN_GLOBAL __attribute__((address_space(1)))
typedef float nsn_f4 __attribute__((ext_vector_type(4)));
typedef int nsn_i4 __attribute__((ext_vector_type(4)));
typedef unsigned nsn_u4 __attribute__((ext_vector_type(4)));
typedef int nsn_i2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float gld(const float *p) { return *(const NSN_GLOBAL float *)p; }
__device__ __forceinline__ int gld(const int *p) { return *(const NSN_GLOBAL int *)p; }
__device__ __forceinline__ float4 gld(const float4 *p) {
  const nsn_f4 v = *(const NSN_GLOBAL nsn_f4 *)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int4 gld(const int4 *p) {
  const nsn_i4 v = *(const NSN_GLOBAL nsn_i4 *)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 gld(const uint4 *p) {
  const nsn_u4 v = *(const NSN_GLOBAL nsn_u4 *)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int2 gld(const int2 *p) {
  const nsn_i2 v = *(const NSN_GLOBAL nsn_i2 *)p;
  return make_int2(v.x, v.y);
}
__device__ __forceinline__ void gst(float *p, float v) { *(NSN_GLOBAL float *)p = v; }
__device__ __forceinline__ void gst(int *p, int v) { *(NSN_GLOBAL int *)p = v; }
__device__ __forceinline__ void gst(float4 *p, float4 v) { *(NSN_GLOBAL nsn_f4 *)p = nsn_f4{v.x, v.y, v.z, v.w}; }


// symmetric 3x3 (xx yy zz xy xz yz) read from global memory, times v
__device__ __forceinline__ V3 sym_mul_g(const float *s, V3 v) {
  float m[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) m[k] = gld(s + k);
  return sym_mul(m, v);
}

}  // namespace nsn
