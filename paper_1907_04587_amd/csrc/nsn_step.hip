// Persistent per-environment kernels of the non-smooth Newton step (gfx950).
//
// One workgroup owns one environment for the whole time step: collision
// detection, start iterate, every Newton iteration (assembly, momentum residual,
// geometric stiffness, residual check, Schur right-hand side, M PCR iterations,
// update).  Environments of a batch are independent, so a launch of one
// workgroup per env keeps every CU busy without grid-wide synchronisation; the
// per-env PCR scalars and early exit fall out naturally.
//
// Paper: Macklin et al., "Non-Smooth Newton Methods for Deformable Multi-Body
// Dynamics" (TOG 2019).  Section / equation references in the comments.
//
// Scatter J^T v (rows -> bodies) is a pull over CSR-ordered adjacency: every body
// sums the contributions of its incident rows in a fixed order (no atomics, so
// results are bitwise reproducible).  Gather J y (bodies -> rows) is a per-element
// read of the body-space vector.
#include <hip/hip_runtime.h>
#include <math.h>

// Multiply-adds are fused only within one expression (the C rule), never across
// statements: the fused operations then follow the source, and the two forms of the
// PCR loop (rows streamed through memory or held in registers) round identically.
#pragma clang fp contract(on)

#include "nsn_layout.h"
#include "nsn_math.h"

namespace nsn {

constexpr float kTauGS = 1e-6f;     // secant smoothing velocity (m/s)
constexpr float kKappaW = 1e-4f;    // FB friction denominator at or below which W is infinite (relative)
constexpr double kTauCR = 1e-12;    // PCR stops once <z, A z> falls below this fraction of its start
constexpr double kWatchBlowup = 1e6; // watchdog: merit growth over the step's best that ends the step
constexpr double kLsSigma = 1e-4;    // line search: sufficient decrease merit <= (1 - sigma t) merit_k
constexpr float kLsTmin = 1.f / 64.f; // line search: smallest step fraction (then accepted)
constexpr float kClampFem = 1e-3f;  // eigenvalue floor of the material Hessian (relative to 2 C1 Ve)
constexpr int kJacobiSweeps = 6;
constexpr float kTauNcp = 1e-6f;    // derivative band around the NCP kink (units of C)
constexpr float kTauEig = 1e-6f;    // relative Jacobi skip / eigenvalue tie tolerance

// --------------------------------------------------------------------------
// block-level reductions (fixed order -> deterministic)
// --------------------------------------------------------------------------
template <int BS>
struct Red {
  static constexpr int NW = BS / 64;
  double d[2][NW > 0 ? NW : 1];
  double d3[3][NW > 0 ? NW : 1];
  float f[2][NW > 0 ? NW : 1];
};

// One lane-permutation step of a wave reduction on a double: each 32-bit half moves
// with the same DPP control (quad_perm, row_half_mirror, row_mirror).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes in a fixed order, returned to every lane: pairs, quads, half
// rows and rows of 16 through DPP moves (no LDS traffic), then the four row sums
// read out and added in row order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 16 * k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 16 * k);
    r[k] = __hiloint2double(hi, lo);
  }
  return (r[0] + r[1]) + (r[2] + r[3]);
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum of the NW (<= 16) per-wave partials p[0..NW-1]: lane i of every wave reads p[i]
// and the same DPP steps add them in a fixed order, so every wave of the block gets
// the identical value from one LDS read per lane.
template <int NW>
__device__ __forceinline__ double partials_sum(const double *p) {
  static_assert(NW <= 16, "one DPP row holds the partials");
  const int lane = threadIdx.x & 63;
  double v = lane < NW ? p[lane] : 0.0;
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 0);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 0);
  return __hiloint2double(hi, lo);
}

template <int BS>
__device__ __forceinline__ double block_sum(double v, Red<BS> &r, int slot) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) r.d[slot][w] = v;
  __syncthreads();
  return partials_sum<Red<BS>::NW>(r.d[slot]);
}

// three sums in one barrier
template <int BS>
__device__ __forceinline__ void block_sum3(double v[3], Red<BS> &r) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = wave_sum(v[k]);
    if (lane == 0) r.d3[k][w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = partials_sum<Red<BS>::NW>(r.d3[k]);
}

template <int BS>
__device__ __forceinline__ float block_max(float v, Red<BS> &r, int slot) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) r.f[slot][w] = v;
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < Red<BS>::NW; ++i) s = fmaxf(s, r.f[slot][i]);
  return s;
}

// exclusive rank of a 0/1 flag within the block; *total = block count
template <int BS>
__device__ __forceinline__ int block_rank(int flag, int *s_wave, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int in_wave = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) s_wave[w] = __popcll(m);
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) {
    int c = s_wave[i];
    before += i < w ? c : 0;
    tot += c;
  }
  *total = tot;
  return before + in_wave;
}

// --------------------------------------------------------------------------
// NCP functions (Sec. 4, Appendix A)
// --------------------------------------------------------------------------
__device__ __forceinline__ void ncp_fb(float C, float lam, float r, float &phi, float &al, float &be) {
  const float rl = r * lam;
  const float rho = sqrtf(C * C + rl * rl);
  phi = C + rl - rho;
  if (rho > kTauNcp) {
    al = 1.f - C / rho;
    be = 1.f - rl / rho;
  } else {  // subgradient choice at (0,0), Sec. 4.2, within rounding of the kink
    al = 0.f;
    be = 1.f;
  }
}

__device__ __forceinline__ void ncp_min(float C, float lam, float r, float &phi, float &al, float &be) {
  const float rl = r * lam;
  phi = fminf(C, rl);
  if (C <= rl + kTauNcp) {
    al = 1.f; be = 0.f;
  } else {
    al = 0.f; be = 1.f;
  }
}

// Friction compliance W (Sec. 4.3 eq. friction_w, Appendix A.2) with the velocity
// magnitude unsquared, W = r num / den with num = sqrt(|v|^2 + r^2 s^2) - r s and
// den = |v| + r |lam_f| - num, s = mu lam_n - |lam_f|.  Both are evaluated free of
// cancellation between large terms, which FP32 cannot afford where W is large (den
// small beside |v|): with root = sqrt(|v|^2 + r^2 s^2) and root - |v| =
// r^2 s^2 / (root + |v|),
//   inside the cone (s > 0): num = |v|^2 / (root + r s),
//       den = r |lam_f| + |v| r s (root + |v| + r s) / ((root + |v|)(root + r s)),
//       a sum of non-negative terms;
//   outside (s <= 0): num = root + r |s|, den = r mu lam_n - r^2 s^2 / (root + |v|),
//       whose remaining cancellation is the limit itself.
// When the fixed point asks for a non-positive friction magnitude (den = r
// |lam_f|^{n+1} at or below kKappaW r mu lam_n) W is infinite: the caller then drives
// lam_f to zero.
__device__ __forceinline__ float friction_w(int ncp, float vn, float lam_n, float lfn, float mu, float r) {
  const float s = mu * lam_n - lfn;
  if (ncp == NSN_NCP_MIN) {
    if (vn <= r * s) return 0.f;
    return (vn - r * s) / (mu * lam_n);
  }
  const float rs = r * s;
  const float root = sqrtf(vn * vn + rs * rs);
  const float rv = root + vn;
  float num, den;
  if (s > 0.f) {
    num = vn * vn / (root + rs);
    den = r * lfn + vn * rs * (rv + rs) / (rv * (root + rs));
  } else {
    num = root - rs;
    den = r * mu * lam_n - (rv > 0.f ? rs * rs / rv : 0.f);
  }
  if (den <= kKappaW * r * mu * lam_n) return __builtin_huge_valf();
  return r * num / den;
}

// --------------------------------------------------------------------------
// 3x3 symmetric eigen-decomposition (cyclic Jacobi, fixed sweeps) and the
// signed SVD of the deformation gradient (Sec. 9.2, Appendix B)
// --------------------------------------------------------------------------
__device__ void sym_eig3(const float *Ain, M3 &Q, float w[3]) {
  float A[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) A[i] = Ain[i];
  float V[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
  // diagonal up to rounding (the rest state): no rotation, so the basis is canonical
  const float tr = fabsf(A[0]) + fabsf(A[4]) + fabsf(A[8]);
  const float off = fmaxf(fabsf(A[1]), fmaxf(fabsf(A[2]), fabsf(A[5])));
  const int sweeps = off <= kTauEig * tr ? 0 : kJacobiSweeps;
  for (int sweep = 0; sweep < sweeps; ++sweep) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int p = k == 2 ? 1 : 0;
      const int q = k == 0 ? 1 : 2;
      const float apq = A[3 * p + q];
      if (apq == 0.f) continue;
      const float theta = (A[3 * q + q] - A[3 * p + p]) / (2.f * apq);
      float t = 1.f / (fabsf(theta) + sqrtf(theta * theta + 1.f));
      if (theta < 0.f) t = -t;
      const float c = 1.f / sqrtf(t * t + 1.f), s = t * c;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float aip = A[3 * i + p], aiq = A[3 * i + q];
        A[3 * i + p] = c * aip - s * aiq;
        A[3 * i + q] = s * aip + c * aiq;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float apj = A[3 * p + j], aqj = A[3 * q + j];
        A[3 * p + j] = c * apj - s * aqj;
        A[3 * q + j] = s * apj + c * aqj;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float vip = V[3 * i + p], viq = V[3 * i + q];
        V[3 * i + p] = c * vip - s * viq;
        V[3 * i + q] = s * vip + c * viq;
      }
    }
  }
  float ev[3] = {A[0], A[4], A[8]};
  int idx[3] = {0, 1, 2};
  // descending insertion sort of three entries; near-ties keep index order
  auto gt = [](float a, float b) { return a - b > kTauEig * (fabsf(a) + fabsf(b)); };
  if (gt(ev[idx[1]], ev[idx[0]])) { int t = idx[0]; idx[0] = idx[1]; idx[1] = t; }
  if (gt(ev[idx[2]], ev[idx[1]])) {
    int t = idx[1]; idx[1] = idx[2]; idx[2] = t;
    if (gt(ev[idx[1]], ev[idx[0]])) { t = idx[0]; idx[0] = idx[1]; idx[1] = t; }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int k = idx[c];
    w[c] = k == 0 ? ev[0] : (k == 1 ? ev[1] : ev[2]);
#pragma unroll
    for (int r = 0; r < 3; ++r) Q.m[3 * r + c] = k == 0 ? V[3 * r] : (k == 1 ? V[3 * r + 1] : V[3 * r + 2]);
  }
}

__device__ __forceinline__ void tangent_basis(V3 n, V3 &d1, V3 &d2) {
  // world axis with the smallest |n_i| (ties -> lowest index)
  const float ax = fabsf(n.x), ay = fabsf(n.y), az = fabsf(n.z);
  int k = 0;
  float best = ax;
  if (ay < best) { best = ay; k = 1; }
  if (az < best) { k = 2; }
  const V3 e = k == 0 ? mk(1.f, 0.f, 0.f) : (k == 1 ? mk(0.f, 1.f, 0.f) : mk(0.f, 0.f, 1.f));
  d1 = cross(n, e);
  const float l = norm(d1);
  d1 = V3{d1.x / l, d1.y / l, d1.z / l};
  d2 = cross(n, d1);
}

// F = U diag(s) V^T, det U = det V = +1, last stretch signed by det F.
__device__ void svd3(const M3 &F, M3 &U, float s[3], M3 &V) {
  float FtF[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      FtF[3 * i + j] = F.m[i] * F.m[j] + F.m[3 + i] * F.m[3 + j] + F.m[6 + i] * F.m[6 + j];
  float w[3];
  sym_eig3(FtF, V, w);
  if (det3(V) < 0.f) { V.m[2] = -V.m[2]; V.m[5] = -V.m[5]; V.m[8] = -V.m[8]; }
  const V3 b0 = mul(F, col(V, 0)), b1 = mul(F, col(V, 1)), b2 = mul(F, col(V, 2));
  V3 u1, u2;
  const float l1 = norm(b0);
  u1 = l1 > 0.f ? V3{b0.x / l1, b0.y / l1, b0.z / l1} : mk(1.f, 0.f, 0.f);
  const float pr = dot(u1, b1);
  u2 = b1 - pr * u1;
  const float l2 = norm(u2);
  if (l2 > 1e-6f * (l1 > 0.f ? l1 : 1.f)) {
    u2 = V3{u2.x / l2, u2.y / l2, u2.z / l2};
  } else {
    V3 t1, t2;
    tangent_basis(u1, t1, t2);
    u2 = t1;
  }
  const V3 u3 = cross(u1, u2);
  U.m[0] = u1.x; U.m[3] = u1.y; U.m[6] = u1.z;
  U.m[1] = u2.x; U.m[4] = u2.y; U.m[7] = u2.z;
  U.m[2] = u3.x; U.m[5] = u3.y; U.m[8] = u3.z;
  s[0] = dot(u1, b0);
  s[1] = dot(u2, b1);
  s[2] = dot(u3, b2);
}

// --------------------------------------------------------------------------
// body helpers
// --------------------------------------------------------------------------
struct Ctx {
  // the scene's table: the kernel argument, or (Newton kernel) its device copy read
  // through a restrict pointer, so that a function that is not inlined receives a
  // small context and the table's fields are reloaded instead of spilled
  const DevScene &S;
  EnvInfo E;
  StepArgs A;
  // LDS mode 2: the tets' J^T v contributions of the env in LDS (three float arrays of
  // cl_n entries, indexed by particle-list position - cl_base) instead of p_cj
  float *cl = nullptr;
  int cl_base = 0, cl_n = 0;
  __device__ Ctx(const DevScene &s, const EnvInfo &e, const StepArgs &a) : S(s), E(e), A(a) {}
};

// The env's descriptor is the same for every lane of a workgroup: read it into scalar
// registers so that its fields take no vector registers in the Newton kernel.
__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float sgpr(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ EnvInfo uniform_env(const EnvInfo &v) {
  EnvInfo u;
  u.rig_off = sgpr(v.rig_off); u.n_rig = sgpr(v.n_rig);
  u.par_off = sgpr(v.par_off); u.n_par = sgpr(v.n_par);
  u.tet_off = sgpr(v.tet_off); u.n_tet = sgpr(v.n_tet);
  u.jnt_off = sgpr(v.jnt_off); u.n_jnt = sgpr(v.n_jnt);
  u.con_off = sgpr(v.con_off); u.max_con = sgpr(v.max_con);
  u.row_off = sgpr(v.row_off); u.row_cap = sgpr(v.row_cap);
  u.dof_off = sgpr(v.dof_off); u.n_dof = sgpr(v.n_dof);
  u.feat_off = sgpr(v.feat_off); u.n_feat = sgpr(v.n_feat);
  u.n_targets = sgpr(v.n_targets); u.ground = sgpr(v.ground);
  u.bcon_off = sgpr(v.bcon_off); u.tet_model = sgpr(v.tet_model);
  u.mu = sgpr(v.mu); u.gx = sgpr(v.gx); u.gy = sgpr(v.gy); u.gz = sgpr(v.gz);
  return u;
}

// world position of a body-fixed point (env-local body id; -1 = world / ground)
__device__ __forceinline__ V3 body_point(const Ctx &c, int body, V3 loc) {
  if (body < 0) return loc;
  if (body < c.E.n_rig) {
    const int g = c.E.rig_off + body;
    return mk(gld(c.S.r_x + g)) + mul(quat_mat(gld(c.S.r_q + g)), loc);
  }
  return mk(gld(c.S.p_x + c.E.par_off + body - c.E.n_rig));
}

__device__ __forceinline__ V3 body_arm(const Ctx &c, int body, V3 loc) {
  if (body < 0 || body >= c.E.n_rig) return mk(0.f, 0.f, 0.f);
  return mul(quat_mat(gld(c.S.r_q + c.E.rig_off + body)), loc);
}

__device__ __forceinline__ bool rigid_static(const Ctx &c, int body) {
  return c.S.r_inertia[c.E.rig_off + body].w == 0.f;
}

// velocity of a point under a body-space vector stored per body (rigid: r_vec 6/body,
// particle: p_vec float4)
__device__ __forceinline__ V3 point_vel(const Ctx &c, const float *rvec, const float4 *pvec, int body, V3 arm) {
  if (body < 0) return mk(0.f, 0.f, 0.f);
  if (body < c.E.n_rig) {
    const int g = c.E.rig_off + body;
    const float *u = rvec + 6 * g;
    return mk(gld(u), gld(u + 1), gld(u + 2)) + cross(mk(gld(u + 3), gld(u + 4), gld(u + 5)), arm);
  }
  return mk(gld(pvec + c.E.par_off + body - c.E.n_rig));
}

// env-local dof index of an env-local body (body-space vectors Y are per env)
__device__ __forceinline__ int ldof(const EnvInfo &E, int body) {
  return body < E.n_rig ? 6 * body : 6 * E.n_rig + 3 * (body - E.n_rig);
}

// velocity of a point under an env-local body-space vector Y
__device__ __forceinline__ V3 point_vel_dof(const Ctx &c, const float *Y, int body, V3 arm) {
  if (body < 0) return mk(0.f, 0.f, 0.f);
  const int d = ldof(c.E, body);
  if (body < c.E.n_rig) return mk(Y[d], Y[d + 1], Y[d + 2]) + cross(mk(Y[d + 3], Y[d + 4], Y[d + 5]), arm);
  return mk(Y[d], Y[d + 1], Y[d + 2]);
}

// J_i M^-1 J_i^T contribution of a direction applied at an arm of one body
__device__ __forceinline__ float effmass_dir(const Ctx &c, int body, V3 arm, V3 dir, bool use_H) {
  if (body < 0) return 0.f;
  if (body < c.E.n_rig) {
    const int g = c.E.rig_off + body;
    const float im = gld(c.S.r_inertia + g).w;
    if (im == 0.f) return 0.f;
    const V3 ad = cross(arm, dir);
    return im * dot(dir, dir) + dot(ad, sym_mul_g(c.S.r_Iwinv + 6 * g, ad));
  }
  const int p = c.E.par_off + body - c.E.n_rig;
  if (use_H) {
    const float4 H = gld(c.S.p_H + p);
    return dir.x * dir.x / H.x + dir.y * dir.y / H.y + dir.z * dir.z / H.z;
  }
  return dot(dir, dir) / gld(c.S.p_m + p);
}

// --------------------------------------------------------------------------
// joints (READING: the paper gives no joint formulas; revolute = 3 anchor rows +
// 2 axis rows, prismatic = 2 point-on-axis rows + 3 orientation rows, optional
// implicit-PD drive row)
// --------------------------------------------------------------------------
struct JFrame {
  V3 PA, PB, rA, rB, a, t1, t2, b, s1, s2;
};

__device__ __forceinline__ JFrame joint_frame(const Ctx &c, int jg) {
  const int4 info = c.S.j_info[jg];
  const float4 *fr = c.S.j_frame + 6 * jg;
  M3 RA = {{1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}};
  V3 xA = mk(0.f, 0.f, 0.f);
  if (info.y >= 0) {
    RA = quat_mat(c.S.r_q[info.y]);
    xA = mk(c.S.r_x[info.y]);
  }
  const M3 RB = quat_mat(c.S.r_q[info.z]);
  JFrame f;
  f.rA = mul(RA, mk(fr[0]));
  f.rB = mul(RB, mk(fr[1]));
  f.PA = xA + f.rA;
  f.PB = mk(c.S.r_x[info.z]) + f.rB;
  f.a = mul(RA, mk(fr[2]));
  f.t1 = mul(RA, mk(fr[4]));
  f.t2 = cross(f.a, f.t1);
  f.b = mul(RB, mk(fr[3]));
  f.s1 = mul(RB, mk(fr[5]));
  f.s2 = cross(f.b, f.s1);
  return f;
}

__device__ __forceinline__ float joint_coordinate(const Ctx &c, int jg) {
  const JFrame f = joint_frame(c, jg);
  if (c.S.j_info[jg].x == NSN_JOINT_REVOLUTE) return atan2f(dot(f.a, cross(f.t1, f.s1)), dot(f.t1, f.s1));
  return dot(f.a, f.PB - f.PA);
}

__device__ __forceinline__ void store_row(float *J, V3 la, V3 aa, V3 lb, V3 ab) {
  J[0] = la.x; J[1] = la.y; J[2] = la.z; J[3] = aa.x; J[4] = aa.y; J[5] = aa.z;
  J[6] = lb.x; J[7] = lb.y; J[8] = lb.z; J[9] = ab.x; J[10] = ab.y; J[11] = ab.z;
}

// Assemble the 6 rows of joint jg: J (world, per side), constraint values c[6].
__device__ __forceinline__ void joint_rows(const Ctx &c, int jg, float *J, float cval[6]) {
  const int4 info = c.S.j_info[jg];
  const JFrame f = joint_frame(c, jg);
  const V3 z = mk(0.f, 0.f, 0.f);
  if (info.x == NSN_JOINT_REVOLUTE) {
    const V3 ex = mk(1.f, 0.f, 0.f), ey = mk(0.f, 1.f, 0.f), ez = mk(0.f, 0.f, 1.f);
    const V3 E3[3] = {ex, ey, ez};
    const V3 d = f.PA - f.PB;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cval[k] = comp(d, k);
      store_row(J + 12 * k, E3[k], cross(f.rA, E3[k]), -E3[k], -cross(f.rB, E3[k]));
    }
    const V3 t1b = cross(f.t1, f.b), t2b = cross(f.t2, f.b);
    cval[3] = dot(f.t1, f.b);
    store_row(J + 36, z, t1b, z, -t1b);
    cval[4] = dot(f.t2, f.b);
    store_row(J + 48, z, t2b, z, -t2b);
    if (info.w) {
      cval[5] = atan2f(dot(f.a, cross(f.t1, f.s1)), dot(f.t1, f.s1));
      store_row(J + 60, z, -f.a, z, f.a);
    } else {
      cval[5] = 0.f;
      store_row(J + 60, z, z, z, z);
    }
  } else {
    const V3 d = f.PB - f.PA;
    cval[0] = dot(f.t1, d);
    store_row(J + 0, -f.t1, cross(f.t1, d) - cross(f.rA, f.t1), f.t1, cross(f.rB, f.t1));
    cval[1] = dot(f.t2, d);
    store_row(J + 12, -f.t2, cross(f.t2, d) - cross(f.rA, f.t2), f.t2, cross(f.rB, f.t2));
    const V3 x0 = cross(f.t1, f.s2), x1 = cross(f.t2, f.b), x2 = cross(f.a, f.s1);
    cval[2] = dot(f.t1, f.s2);
    store_row(J + 24, z, x0, z, -x0);
    cval[3] = dot(f.t2, f.b);
    store_row(J + 36, z, x1, z, -x1);
    cval[4] = dot(f.a, f.s1);
    store_row(J + 48, z, x2, z, -x2);
    if (info.w) {
      cval[5] = dot(f.a, d);
      store_row(J + 60, -f.a, cross(f.a, d) - cross(f.rA, f.a), f.a, cross(f.rB, f.a));
    } else {
      cval[5] = 0.f;
      store_row(J + 60, z, z, z, z);
    }
  }
  if (info.y < 0 || c.S.r_inertia[info.y].w == 0.f)
    for (int r = 0; r < 6; ++r)
      for (int k = 0; k < 6; ++k) J[12 * r + k] = 0.f;
  if (c.S.r_inertia[info.z].w == 0.f)
    for (int r = 0; r < 6; ++r)
      for (int k = 6; k < 12; ++k) J[12 * r + k] = 0.f;
}

__device__ __forceinline__ float row_dot_rigid(const float *J6, const float *Y, int d) {
  return J6[0] * Y[d] + J6[1] * Y[d + 1] + J6[2] * Y[d + 2] + J6[3] * Y[d + 3] + J6[4] * Y[d + 4] +
         J6[5] * Y[d + 5];
}

__device__ __forceinline__ float rigid_quad(const Ctx &c, int g, const float *J6) {
  const float im = gld(c.S.r_inertia + g).w;
  if (im == 0.f) return 0.f;
  const V3 l = mk(J6[0], J6[1], J6[2]), a = mk(J6[3], J6[4], J6[5]);
  return im * dot(l, l) + dot(a, sym_mul_g(c.S.r_Iwinv + 6 * g, a));
}

// --------------------------------------------------------------------------
// element index space of an env: [joints | tets | contacts]; a tet has 3 rows
// (principal stretches) or 6 (strains of a linear tet), uniform over the env
// --------------------------------------------------------------------------
__device__ __forceinline__ bool lin_tets(const EnvInfo &E) { return E.tet_model == NSN_TET_LINEAR; }
__device__ __forceinline__ int tet_nrows(const EnvInfo &E) { return lin_tets(E) ? 6 : 3; }
__device__ __forceinline__ int row_joint(const EnvInfo &E, int jl) { return E.row_off + 6 * jl; }
__device__ __forceinline__ int row_tet(const EnvInfo &E, int tl) { return E.row_off + 6 * E.n_jnt + tet_nrows(E) * tl; }
__device__ __forceinline__ int row_con(const EnvInfo &E, int cl) {
  return E.row_off + 6 * E.n_jnt + tet_nrows(E) * E.n_tet + 3 * cl;
}

// --------------------------------------------------------------------------
// contact geometry (collision detection, Sec. 10; READING of the primitive rules)
// --------------------------------------------------------------------------
__device__ int box_ref_face(const Ctx &c, int A, int B) {
  const int ga = c.E.rig_off + A, gb = c.E.rig_off + B;
  const M3 RA = quat_mat(c.S.r_q[ga]), RB = quat_mat(c.S.r_q[gb]);
  const V3 d = mk(c.S.r_x[ga]) - mk(c.S.r_x[gb]);
  const V3 eA = mk(c.S.r_ext[ga]), eB = mk(c.S.r_ext[gb]);
  int best = 0;
  float bs = 0.f;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int ax = f >> 1;
    const float sg = (f & 1) ? 1.f : -1.f;
    const V3 nf = sg * col(RB, ax);
    float sep = dot(nf, d) - comp(eB, ax);
#pragma unroll
    for (int i = 0; i < 3; ++i) sep -= fabsf(dot(nf, col(RA, i))) * comp(eA, i);
    if (f == 0 || sep > bs) { best = f; bs = sep; }
  }
  return best;
}

__device__ __forceinline__ void setc(V3 &a, int i, float v) {
  if (i == 0) a.x = v; else if (i == 1) a.y = v; else a.z = v;
}

// returns 1 and (n, bL, dist, target thickness) for a point against a target
// (ground plane, box, capsule); see the oracle for the rules
__device__ int target_query(const Ctx &c, int t, V3 pw, bool box_feature, int fbody, V3 &n, V3 &bL,
                            float &dist, float &tthick) {
  tthick = 0.f;
  if (t < 0) {
    n = mk(0.f, 0.f, 1.f);
    bL = mk(pw.x, pw.y, 0.f);
    dist = pw.z;
    return 1;
  }
  const int g = c.E.rig_off + t;
  const M3 R = quat_mat(c.S.r_q[g]);
  const V3 pl = mulT(R, pw - mk(c.S.r_x[g]));
  const V3 ext = mk(c.S.r_ext[g]);
  const int shape = c.S.r_shape[g];
  if (shape == NSN_SHAPE_BOX) {
    V3 nl = mk(0.f, 0.f, 0.f), bl = pl;
    if (box_feature) {
      const int face = box_ref_face(c, fbody, t);
      const int ax = face >> 1;
      const float sg = (face & 1) ? 1.f : -1.f;
#pragma unroll
      for (int o = 0; o < 3; ++o)
        if (o != ax && fabsf(comp(pl, o)) > comp(ext, o) + c.A.p.margin) return 0;
      setc(nl, ax, sg);
      setc(bl, ax, sg * comp(ext, ax));
      dist = sg * comp(pl, ax) - comp(ext, ax);
    } else {
      const bool inside = fabsf(pl.x) <= ext.x && fabsf(pl.y) <= ext.y && fabsf(pl.z) <= ext.z;
      if (inside) {
        int best = -1;
        float bd = 0.f;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int ax = f >> 1;
          const float sg = (f & 1) ? 1.f : -1.f;
          const float depth = comp(ext, ax) - sg * comp(pl, ax);
          if (best < 0 || depth < bd) { best = f; bd = depth; }
        }
        const int ax = best >> 1;
        const float sg = (best & 1) ? 1.f : -1.f;
        setc(nl, ax, sg);
        setc(bl, ax, sg * comp(ext, ax));
        dist = -bd;
      } else {
        bl = mk(fminf(fmaxf(pl.x, -ext.x), ext.x), fminf(fmaxf(pl.y, -ext.y), ext.y),
                fminf(fmaxf(pl.z, -ext.z), ext.z));
        const V3 df = pl - bl;
        const float l = norm(df);
        if (!(l > 1e-9f)) return 0;
        nl = V3{df.x / l, df.y / l, df.z / l};
        dist = l;
      }
    }
    n = mul(R, nl);
    bL = bl;
    return 1;
  }
  if (shape == NSN_SHAPE_CAPSULE) {
    const float L = ext.y;
    const float tp = fminf(fmaxf(pl.x, -L), L);
    const V3 df = mk(pl.x - tp, pl.y, pl.z);
    const float l = norm(df);
    if (!(l > 1e-9f)) return 0;
    n = mul(R, V3{df.x / l, df.y / l, df.z / l});
    bL = mk(tp, 0.f, 0.f);
    dist = l - ext.x;
    tthick = ext.x;
    return 1;
  }
  return 0;
}

// --------------------------------------------------------------------------
// Kernel 1: step set-up (mass at q^-, u~), collision detection in canonical
// candidate order, contact adjacency, warm-start lookup, contact features.
// One workgroup per env.
// --------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(BS) void k_prepare(DevScene S, StepArgs A, int want_features) {
  __shared__ int s_wave[BS / 64];
  __shared__ int s_count;
  const int e = blockIdx.x;
  Ctx c(S, S.env[e], A);
  const EnvInfo &E = c.E;
  const float h = A.h;
  const int tid = threadIdx.x;
  const V3 grav = mk(E.gx, E.gy, E.gz);

  // ---- mass at q^- and u~ = u^- + h M^-1 f (Sec. 5; f = (m g, -w x I w)) ----
  for (int r = tid; r < E.n_rig; r += BS) {
    const int g = E.rig_off + r;
    const float4 q = quat_normalize(S.r_q[g]);
    S.r_q[g] = q;
    S.r_q0[g] = q;
    S.r_x0[g] = S.r_x[g];
    const float4 In = S.r_inertia[g];
    float *Iw = S.r_Iw + 6 * g, *Ii = S.r_Iwinv + 6 * g, *ut = S.r_ut + 6 * g;
    if (In.w == 0.f) {
      for (int k = 0; k < 6; ++k) { Iw[k] = 0.f; Ii[k] = 0.f; ut[k] = 0.f; }
      continue;
    }
    const M3 R = quat_mat(q);
    const float Ib[3] = {In.x, In.y, In.z};
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const float prod = R.m[3 * ia[k] + m] * R.m[3 * ib[k] + m];
        s1 += prod * Ib[m];
        s2 += prod / Ib[m];
      }
      Iw[k] = s1;
      Ii[k] = s2;
    }
    const V3 w = mk(S.r_w[g]);
    const V3 gyro = -cross(w, sym_mul(Iw, w));
    const V3 dw = sym_mul(Ii, gyro);
    const V3 v = mk(S.r_v[g]);
    ut[0] = v.x + h * grav.x; ut[1] = v.y + h * grav.y; ut[2] = v.z + h * grav.z;
    ut[3] = w.x + h * dw.x; ut[4] = w.y + h * dw.y; ut[5] = w.z + h * dw.z;
  }
  for (int p = tid; p < E.n_par; p += BS) {
    const int g = E.par_off + p;
    S.p_x0[g] = S.p_x[g];
    const float4 v = S.p_v[g];
    S.p_ut[g] = make_float4(v.x + h * grav.x, v.y + h * grav.y, v.z + h * grav.z, 0.f);
  }
  if (tid == 0) s_count = 0;
  if (e == 0 && tid == 0) {  // new timing slot for this step
    const int t = S.tick[0] + 1;
    S.tick[0] = t;
    const int slot = t % kTimingRing;
    S.ts[2 * slot] = ~0ull;
    S.ts[2 * slot + 1] = 0ull;
  }
  __syncthreads();
  for (int j = tid; j < E.n_jnt; j += BS) {
    const int jg = E.jnt_off + j;
    S.j_theta0[jg] = S.j_info[jg].w ? joint_coordinate(c, jg) : 0.f;
  }

  // ---- collision detection at q^- (Alg. 1), canonical candidate order:
  //      candidate = feature * n_targets + target, features = rigid features then
  //      particles, targets = ground then rigid bodies ----
  // a caller-given contact list (already in the contact slots) replaces detection
  const int inject = S.c_inject[e];
  const int nfeat = E.n_feat + E.n_par;
  const long long ncand = inject > 0 ? 0 : (long long)nfeat * E.n_targets;
  for (long long base = 0; base < ncand; base += BS) {
    const long long cand = base + tid;
    int keep = 0, fbody = 0, tb = -1;
    V3 n = mk(0.f, 0.f, 0.f), aL = n, bL = n;
    float dtot = 0.f;
    if (cand < ncand) {
      const int fi = (int)(cand / E.n_targets);
      const int ti = (int)(cand - (long long)fi * E.n_targets);
      const int t = E.ground ? ti - 1 : ti;
      const bool is_particle = fi >= E.n_feat;
      bool ok = true;
      float fthick = 0.f;
      int fshape = -1;
      if (!is_particle) {
        const int2 fv = S.feat[E.feat_off + fi];
        fbody = fv.x - E.rig_off;
        fshape = S.r_shape[fv.x];
        if (S.r_inertia[fv.x].w == 0.f) ok = false;
        const float4 ex = S.r_ext[fv.x];
        if (fshape == NSN_SHAPE_BOX) {
          aL = mk((fv.y & 1) ? ex.x : -ex.x, (fv.y & 2) ? ex.y : -ex.y, (fv.y & 4) ? ex.z : -ex.z);
        } else {
          aL = mk((fv.y & 1) ? ex.y : -ex.y, 0.f, 0.f);
          fthick = ex.x;
        }
      } else {
        fbody = E.n_rig + (fi - E.n_feat);
      }
      if (ok && t >= 0) {
        const int ts = S.r_shape[E.rig_off + t];
        if (t == fbody || ts == NSN_SHAPE_NONE) ok = false;
        if (ts == NSN_SHAPE_CAPSULE && !is_particle) ok = false;
        if (fshape == NSN_SHAPE_CAPSULE) ok = false;
        if (!is_particle && ts == NSN_SHAPE_BOX && fshape != NSN_SHAPE_BOX) ok = false;
      }
      if (ok) {
        const V3 pw = body_point(c, fbody, aL);
        float dist, tthick;
        if (target_query(c, t, pw, !is_particle && fshape == NSN_SHAPE_BOX, fbody, n, bL, dist, tthick)) {
          const float gap = dist - fthick;
          const V3 va = point_vel(c, S.r_ut, S.p_ut, fbody, body_arm(c, fbody, aL));
          const V3 vb = t >= 0 ? point_vel(c, S.r_ut, S.p_ut, t, body_arm(c, t, bL)) : mk(0.f, 0.f, 0.f);
          const float vn = dot(n, va - vb);
          const float pred = gap + h * (vn < 0.f ? vn : 0.f);
          if (pred < A.p.margin) {
            keep = 1;
            tb = t;
            dtot = fthick + tthick;
          }
        }
      }
    }
    int total;
    const int rank = block_rank<BS>(keep, s_wave, &total);
    if (keep) {
      const int slot = s_count + rank;
      if (slot < E.max_con) {
        const int gc = E.con_off + slot;
        S.c_key[gc] = (int)cand;
        S.c_body[gc] = make_int2(fbody, tb);
        S.c_n[gc] = f4(n, dtot);
        S.c_aL[gc] = f4(fbody < E.n_rig ? aL : mk(0.f, 0.f, 0.f), 0.f);
        S.c_bL[gc] = f4(bL, 0.f);
      }
    }
    __syncthreads();
    if (tid == 0) s_count += total;
    __syncthreads();
  }
  const int found = inject > 0 ? inject - 1 : s_count;
  const int nc = found < E.max_con ? found : E.max_con;
  __syncthreads();
  if (tid == 0) {
    S.n_con[e] = nc;
    S.overflow[e] = found - nc;
    if (inject > 0) S.c_inject[e] = 0;  // one step only
  }

  // ---- feature-side ranges (contacts come out sorted by feature body) ----
  for (int r = tid; r < E.n_rig; r += BS) {
    S.r_acon_beg[E.rig_off + r] = 0;
    S.r_acon_end[E.rig_off + r] = 0;
  }
  for (int p = tid; p < E.n_par; p += BS) {
    S.p_acon_beg[E.par_off + p] = 0;
    S.p_acon_end[E.par_off + p] = 0;
  }
  __syncthreads();
  for (int i = tid; i < nc; i += BS) {
    const int gc = E.con_off + i;
    const int fa = S.c_body[gc].x;
    const bool first = i == 0 || S.c_body[gc - 1].x != fa;
    const bool last = i == nc - 1 || S.c_body[gc + 1].x != fa;
    if (fa < E.n_rig) {
      if (first) S.r_acon_beg[E.rig_off + fa] = gc;
      if (last) S.r_acon_end[E.rig_off + fa] = gc + 1;
    } else {
      if (first) S.p_acon_beg[E.par_off + fa - E.n_rig] = gc;
      if (last) S.p_acon_end[E.par_off + fa - E.n_rig] = gc + 1;
    }
  }
  // ---- target-side lists: one wave per rigid target, ballot compaction in order ----
  const int lane = tid & 63, wv = tid >> 6;
  for (int t = wv; t < E.n_rig; t += BS / 64) {
    int cnt = 0;
    for (int b0 = 0; b0 < nc; b0 += 64) {
      const int i = b0 + lane;
      const int f = i < nc && S.c_body[E.con_off + i].y == t;
      cnt += __popcll(__ballot(f));
    }
    if (lane == 0) S.r_bcon_cnt[E.rig_off + t] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int t = 0; t < E.n_rig; ++t) {
      S.r_bcon_beg[E.rig_off + t] = E.bcon_off + run;
      run += S.r_bcon_cnt[E.rig_off + t];
    }
  }
  __syncthreads();
  for (int t = wv; t < E.n_rig; t += BS / 64) {
    int run = S.r_bcon_beg[E.rig_off + t];
    for (int b0 = 0; b0 < nc; b0 += 64) {
      const int i = b0 + lane;
      const int f = i < nc && S.c_body[E.con_off + i].y == t;
      const unsigned long long m = __ballot(f);
      if (f) S.bcon_list[run + __popcll(m & ((1ull << lane) - 1ull))] = E.con_off + i;
      run += __popcll(m);
    }
  }

  // ---- contribution slots of the rigid bodies: each body's run holds its joints
  //      (adjacency order), its feature-side contacts, then its target-side contacts,
  //      in the env's region [2 jnt_off + 2 con_off, + 2 n_jnt + 2 max_con) ----
  __syncthreads();
  for (int i = tid; i < nc; i += BS) S.c_slot[E.con_off + i] = make_int2(-1, -1);
  for (int j = tid; j < E.n_jnt; j += BS) S.j_slot[E.jnt_off + j] = make_int2(-1, -1);
  if (tid == 0) {
    int at = 2 * E.jnt_off + 2 * E.con_off;
    for (int r = 0; r < E.n_rig; ++r) {
      const int g = E.rig_off + r;
      const int n = (S.r_jadj_ptr[g + 1] - S.r_jadj_ptr[g]) + (S.r_acon_end[g] - S.r_acon_beg[g]) + S.r_bcon_cnt[g];
      S.r_slot[g] = make_int2(at, at + n);
      at += n;
    }
  }
  __syncthreads();
  for (int r = tid; r < E.n_rig; r += BS) {
    const int g = E.rig_off + r;
    int at = S.r_slot[g].x;
    for (int k = S.r_jadj_ptr[g]; k < S.r_jadj_ptr[g + 1]; ++k, ++at) {
      const int ent = S.r_jadj[k];
      if (ent & 1) S.j_slot[ent >> 1].y = at;
      else S.j_slot[ent >> 1].x = at;
    }
    for (int gc = S.r_acon_beg[g]; gc < S.r_acon_end[g]; ++gc, ++at) S.c_slot[gc].x = at;
    const int b0 = S.r_bcon_beg[g], bn = S.r_bcon_cnt[g];
    for (int k = 0; k < bn; ++k, ++at) S.c_slot[S.bcon_list[b0 + k]].y = at;
  }

  // ---- warm start by key (previous step) and per-contact features ----
  const int np_prev = S.n_prev[e];
  for (int i = tid; i < nc; i += BS) {
    const int gc = E.con_off + i;
    const int key = S.c_key[gc];
    int lo = 0, hi = np_prev - 1, found = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int km = S.c_prev_key[E.con_off + mid];
      if (km == key) { found = mid; break; }
      if (km < key) lo = mid + 1; else hi = mid - 1;
    }
    const float4 lp = found >= 0 ? S.c_prev_lam[E.con_off + found] : make_float4(0.f, 0.f, 0.f, 0.f);
    S.c_lam0[gc] = lp;
    if (want_features) {
      // READING of the 12 features (step start, contact basis): v_n, v_t1, v_t2 under u~,
      // C_n(q^-), previous (lam_n, lam_t1, lam_t2), 1/m_A, 1/m_B, mu, n_z, existed-before flag
      const int2 bd = S.c_body[gc];
      const float4 n4 = S.c_n[gc];
      const V3 n = mk(n4);
      const V3 aL = mk(S.c_aL[gc]), bL = mk(S.c_bL[gc]);
      const V3 va = point_vel(c, S.r_ut, S.p_ut, bd.x, body_arm(c, bd.x, aL));
      V3 vb = mk(0.f, 0.f, 0.f), pb = bL;
      if (bd.y >= 0) {
        vb = point_vel(c, S.r_ut, S.p_ut, bd.y, body_arm(c, bd.y, bL));
        pb = body_point(c, bd.y, bL);
      }
      const V3 pa = body_point(c, bd.x, aL);
      V3 d1, d2;
      tangent_basis(n, d1, d2);
      const V3 vr = va - vb;
      const float ima = bd.x < E.n_rig ? S.r_inertia[E.rig_off + bd.x].w : 1.f / S.p_m[E.par_off + bd.x - E.n_rig];
      const float imb = bd.y >= 0 ? S.r_inertia[E.rig_off + bd.y].w : 0.f;
      float *F = S.c_feat + (size_t)gc * 12;
      F[0] = dot(n, vr); F[1] = dot(d1, vr); F[2] = dot(d2, vr);
      F[3] = dot(n, pa - pb) - n4.w;
      F[4] = lp.x; F[5] = lp.y; F[6] = lp.z;
      F[7] = ima; F[8] = imb; F[9] = E.mu; F[10] = n.z; F[11] = found >= 0 ? 1.f : 0.f;
    }
  }
}

// --------------------------------------------------------------------------
// Newton kernel pieces
// --------------------------------------------------------------------------
__device__ __forceinline__ float tJ(const DevScene &S, int buf, int comp_, int tg) {
  return gld(S.t_J + ((size_t)buf * 18 + comp_) * S.NT + tg);
}

// ---- assembly (Sec. 6.1 eq. newton_system; Appendix A/B) ----
__device__ __forceinline__ void assemble_joint(const Ctx &c, int jl, double tplus) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const float h = c.A.h;
  const int jg = E.jnt_off + jl;
  float cv[6];
  joint_rows(c, jg, S.j_J + (size_t)72 * jg, cv);
  const int r0 = row_joint(E, jl);
  const int4 info = S.j_info[jg];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    float Ec = 0.f, cval = cv[r];
    if (r == 5) {
      if (info.w) {
        // READING: implicit PD as a backward-Euler soft row, k_eff = kp + kd/h,
        // E = 1/k_eff, c = theta(q) - (kp theta*(t+) + (kd/h) theta(q^-)) / k_eff
        const float4 d0 = S.j_drive[2 * jg], d1 = S.j_drive[2 * jg + 1];
        const float keff = d0.x + d0.y / h;
        const double target = (double)d1.y + (double)d0.z * sin(2.0 * M_PI * (double)d0.w * tplus + (double)d1.x);
        const float teff = (float)(((double)d0.x * target + (double)(d0.y / h) * (double)S.j_theta0[jg]) / (double)keff);
        cval = cv[5] - teff;
        Ec = 1.f / keff;
      } else {
        cval = 0.f;  // undriven: empty row that keeps its multiplier at zero
        Ec = h * h;
      }
    }
    S.row_C[r0 + r] = Ec / (h * h);
    S.row_err[r0 + r] = (cval + Ec * S.row_lam[r0 + r]) / h;
  }
}

// ---- linear tets (Sec. 9.2, linear materials): six strains s = (xx yy zz yz xz xy)
// in the element's rotated frame (READING: s = S - I of the polar decomposition
// F = R S, R = U V^T of the signed SVD, rows ds/dx at fixed R), isotropic Hooke
// c = V_e K_e s, constant compliance (V_e K_e)^-1.  The ping-pong Jacobian slot of a
// linear tet holds R (row-major); D_m^-1 is the rest-shape constant.  Row of e_ab at
// vertex j = 1..3: (R_:a (D_m^-1)_jb + R_:b (D_m^-1)_ja) / 2, vertex 0 minus their sum.
constexpr int kLinA[6] = {0, 1, 2, 1, 0, 0}, kLinB[6] = {0, 1, 2, 2, 2, 1};

// the four vertex contributions of a tet, at their particle-list positions dst
__device__ __forceinline__ void store_tet_cj(const Ctx &c, int4 dst, V3 a0, V3 a1, V3 a2, V3 a3) {
  if (c.cl) {
    float *cx = c.cl, *cy = cx + c.cl_n, *cz = cy + c.cl_n;
    const int i[4] = {dst.x - c.cl_base, dst.y - c.cl_base, dst.z - c.cl_base, dst.w - c.cl_base};
    const V3 v[4] = {a0, a1, a2, a3};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cx[i[m]] = v[m].x;
      cy[i[m]] = v[m].y;
      cz[i[m]] = v[m].z;
    }
    return;
  }
  gst(c.S.p_cj + dst.x, f4(a0, 0.f));
  gst(c.S.p_cj + dst.y, f4(a1, 0.f));
  gst(c.S.p_cj + dst.z, f4(a2, 0.f));
  gst(c.S.p_cj + dst.w, f4(a3, 0.f));
}

__device__ __forceinline__ void ltet_load(const DevScene &S, int buf, int tg, float R[9], float B[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = tJ(S, buf, k, tg);
#pragma unroll
  for (int k = 0; k < 9; ++k) B[k] = S.t_Dminv[(size_t)k * S.NT + tg];
}

// Linear-tet tail of the assembly, given the signed SVD F = U diag(sv) V^T;
// stress_only = true: only the warm-start multipliers -c of the start configuration
__device__ __forceinline__ void assemble_ltet_tail(const Ctx &c, int tl, int buf, bool stress_only, const M3 &U,
                                                   const float sv[3], const M3 &V) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const float h = c.A.h;
  const int NT = S.NT;
  const int tg = E.tet_off + tl;
  float eps[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int a = kLinA[q], b = kLinB[q];
    eps[q] = V.m[3 * a] * sv[0] * V.m[3 * b] + V.m[3 * a + 1] * sv[1] * V.m[3 * b + 1] +
             V.m[3 * a + 2] * sv[2] * V.m[3 * b + 2] - (a == b ? 1.f : 0.f);
  }
  const float4 mt = S.t_mat[tg];  // linear tets: (Ve, mu, lambda, -)
  const float Ve = mt.x, mu = mt.y, la = mt.z;
  const float tr = eps[0] + eps[1] + eps[2];
  float cs[6];
#pragma unroll
  for (int q = 0; q < 3; ++q) cs[q] = Ve * (2.f * mu * eps[q] + la * tr);
#pragma unroll
  for (int q = 3; q < 6; ++q) cs[q] = Ve * 4.f * mu * eps[q];
  const int r0 = row_tet(E, tl);
  if (stress_only) {
#pragma unroll
    for (int q = 0; q < 6; ++q) S.row_lam[r0 + q] = -cs[q];
    return;
  }
  float *Jb = S.t_J + (size_t)buf * 18 * NT;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Jb[(size_t)(3 * i + j) * NT + tg] = U.m[3 * i] * V.m[3 * j] + U.m[3 * i + 1] * V.m[3 * j + 1] + U.m[3 * i + 2] * V.m[3 * j + 2];
  // (V_e K_e)^-1: normal block (I - g 1 1^T) / (2 mu V_e) with g = lambda / (2 mu + 3 lambda),
  // shear entries 1 / (4 mu V_e)
  const float f = 1.f / (2.f * mu * Ve), g = la / (2.f * mu + 3.f * la);
  const float En_d = f * (1.f - g), En_o = -f * g, Es = 1.f / (4.f * mu * Ve);
  float cl[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) cl[q] = cs[q] + S.row_lam[r0 + q];
  const float ih = 1.f / h, ih2 = ih * ih;
  const float sn = cl[0] + cl[1] + cl[2];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    S.row_err[r0 + q] = (En_d * cl[q] + En_o * (sn - cl[q])) * ih;
    S.row_C[r0 + q] = En_d * ih2;
  }
#pragma unroll
  for (int q = 3; q < 6; ++q) {
    S.row_err[r0 + q] = Es * cl[q] * ih;
    S.row_C[r0 + q] = Es * ih2;
  }
  // normal block for the matvec, same layout as a neo-Hookean tet's E (xx yy zz xy xz yz)
#pragma unroll
  for (int k = 0; k < 3; ++k) S.t_E[(size_t)k * NT + tg] = En_d * ih2;
#pragma unroll
  for (int k = 3; k < 6; ++k) S.t_E[(size_t)k * NT + tg] = En_o * ih2;
}

// J z of a linear tet: the strain rates of the vertex values y (6 rows)
__device__ __forceinline__ void ltet_JY(const Ctx &c, int tl, const float *Y, int buf, float jy[6]) {
  const DevScene &S = c.S;
  const EnvInfo &E = c.E;
  const int tg = E.tet_off + tl;
  const int4 id = S.t_ids[tg];
  const int base = 6 * E.n_rig - 3 * E.par_off;
  const V3 y0 = mk(Y[base + 3 * id.x], Y[base + 3 * id.x + 1], Y[base + 3 * id.x + 2]);
  const V3 y[3] = {mk(Y[base + 3 * id.y], Y[base + 3 * id.y + 1], Y[base + 3 * id.y + 2]) - y0,
                   mk(Y[base + 3 * id.z], Y[base + 3 * id.z + 1], Y[base + 3 * id.z + 2]) - y0,
                   mk(Y[base + 3 * id.w], Y[base + 3 * id.w + 1], Y[base + 3 * id.w + 2]) - y0};
  float R[9], B[9];
  ltet_load(S, buf, tg, R, B);
  // G = R^T Y_s D_m^-1
  float T[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) T[3 * a + j] = R[a] * y[j].x + R[3 + a] * y[j].y + R[6 + a] * y[j].z;
  float G[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) G[3 * a + b] = T[3 * a] * B[b] + T[3 * a + 1] * B[3 + b] + T[3 * a + 2] * B[6 + b];
#pragma unroll
  for (int q = 0; q < 6; ++q) jy[q] = 0.5f * (G[3 * kLinA[q] + kLinB[q]] + G[3 * kLinB[q] + kLinA[q]]);
}

// J^T z of a linear tet into its particle-list slots: vertex j = 1..3 gets column j of
// R Z D_m^-T with Z the symmetric tensor of z (off-diagonal entries z/2), vertex 0
// minus their sum
__device__ __forceinline__ void ltet_contrib(const Ctx &c, int tl, const float z[6], int buf) {
  const DevScene &S = c.S;
  const int tg = c.E.tet_off + tl;
  float R[9], B[9];
  ltet_load(S, buf, tg, R, B);
  const float Z[9] = {z[0], 0.5f * z[5], 0.5f * z[4], 0.5f * z[5], z[1], 0.5f * z[3], 0.5f * z[4], 0.5f * z[3], z[2]};
  float M[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[3 * k + b] = R[3 * k] * Z[b] + R[3 * k + 1] * Z[3 + b] + R[3 * k + 2] * Z[6 + b];
  V3 a[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    a[j] = mk(M[0] * B[3 * j] + M[1] * B[3 * j + 1] + M[2] * B[3 * j + 2],
              M[3] * B[3 * j] + M[4] * B[3 * j + 1] + M[5] * B[3 * j + 2],
              M[6] * B[3 * j] + M[7] * B[3 * j + 1] + M[8] * B[3 * j + 2]);
  const V3 a0 = mk(0.f, 0.f, 0.f) - (a[0] + a[1] + a[2]);
  store_tet_cj(c, S.t_dst[tg], a0, a[0], a[1], a[2]);
}

// J_i H~^-1 J_i^T of the 6 rows of a linear tet
__device__ __forceinline__ void ltet_hdiag(const Ctx &c, int tl, int buf, float dg[6]) {
  const DevScene &S = c.S;
  const int tg = c.E.tet_off + tl;
  const int4 id = S.t_ids[tg];
  const float4 Hv[4] = {S.p_H[id.x], S.p_H[id.y], S.p_H[id.z], S.p_H[id.w]};
  float R[9], B[9];
  ltet_load(S, buf, tg, R, B);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int a = kLinA[q], b = kLinB[q];
    const V3 ra = mk(R[a], R[3 + a], R[6 + a]), rb = mk(R[b], R[3 + b], R[6 + b]);
    V3 g0 = mk(0.f, 0.f, 0.f);
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const V3 gj = 0.5f * (B[3 * j + b] * ra + B[3 * j + a] * rb);
      g0 = g0 - gj;
      acc += gj.x * gj.x / Hv[j + 1].x + gj.y * gj.y / Hv[j + 1].y + gj.z * gj.z / Hv[j + 1].z;
    }
    dg[q] = acc + g0.x * g0.x / Hv[0].x + g0.y * g0.y / Hv[0].y + g0.z * g0.z / Hv[0].z;
  }
}

// Both tet models share F and its signed SVD (one body, so that the linear-capable
// kernel stays within the inliner's budget); stress_only = true: only the
// warm-start multipliers of the start configuration.
template <bool EXT>
__device__ __forceinline__ void assemble_tet(const Ctx &c, int tl, int buf, bool stress_only) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const float h = c.A.h;
  const int NT = S.NT;
  const int tg = E.tet_off + tl;
  const int4 id = gld(S.t_ids + tg);
  M3 Dmi;
#pragma unroll
  for (int k = 0; k < 9; ++k) Dmi.m[k] = gld(S.t_Dminv + (size_t)k * NT + tg);
  const V3 x0 = mk(gld(S.p_x + id.x));
  const V3 e1 = mk(gld(S.p_x + id.y)) - x0, e2 = mk(gld(S.p_x + id.z)) - x0, e3 = mk(gld(S.p_x + id.w)) - x0;
  // the tet's remaining inputs, read before its first store (see RowIn)
  const int r0 = row_tet(E, tl);
  float4 mt = make_float4(0.f, 0.f, 0.f, 0.f);
  float lam0[3] = {0.f, 0.f, 0.f};
  if (!(EXT && lin_tets(E))) {
    mt = gld(S.t_mat + tg);  // (Ve, C1, D1, alpha)
    if (!stress_only)
#pragma unroll
      for (int r = 0; r < 3; ++r) lam0[r] = gld(S.row_lam + r0 + r);
  }
  M3 Ds = {{e1.x, e2.x, e3.x, e1.y, e2.y, e3.y, e1.z, e2.z, e3.z}};
  M3 F;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F.m[3 * i + j] = Ds.m[3 * i] * Dmi.m[j] + Ds.m[3 * i + 1] * Dmi.m[3 + j] + Ds.m[3 * i + 2] * Dmi.m[6 + j];
  M3 U, V;
  float s[3];
  svd3(F, U, s, V);
  if (EXT && lin_tets(E)) {
    assemble_ltet_tail(c, tl, buf, stress_only, U, s, V);
    return;
  }
  // rows ds_i/dx: u_i * (Dm^-1 v_i)_j for vertices 1..3, minus their sum for vertex 0
  float *Jb = S.t_J + (size_t)buf * 18 * NT;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3 u = col(U, i), w = mul(Dmi, col(V, i));
    gst(Jb + (size_t)(6 * i + 0) * NT + tg, u.x);
    gst(Jb + (size_t)(6 * i + 1) * NT + tg, u.y);
    gst(Jb + (size_t)(6 * i + 2) * NT + tg, u.z);
    gst(Jb + (size_t)(6 * i + 3) * NT + tg, w.x);
    gst(Jb + (size_t)(6 * i + 4) * NT + tg, w.y);
    gst(Jb + (size_t)(6 * i + 5) * NT + tg, w.z);
  }
  const float Ve = mt.x, C1 = mt.y, D1 = mt.z, al = mt.w;
  // stable neo-Hookean (Appendix B) in principal stretches
  const float J = s[0] * s[1] * s[2];
  const float gr[3] = {2.f * C1 * s[0] + 2.f * D1 * (J - al) * s[1] * s[2],
                       2.f * C1 * s[1] + 2.f * D1 * (J - al) * s[0] * s[2],
                       2.f * C1 * s[2] + 2.f * D1 * (J - al) * s[0] * s[1]};
  if (stress_only) {
    // warm start: the stress of the start configuration in its own principal basis,
    // lambda0 = -V_e dPsi/ds (multipliers of the previous step live in another basis)
    gst(S.row_lam + r0, -Ve * gr[0]);
    gst(S.row_lam + r0 + 1, -Ve * gr[1]);
    gst(S.row_lam + r0 + 2, -Ve * gr[2]);
    return;
  }
  const float k0 = 2.f * J - al;
  float H[9];
  H[0] = Ve * 2.f * (D1 * s[1] * s[1] * s[2] * s[2] + C1);
  H[4] = Ve * 2.f * (D1 * s[0] * s[0] * s[2] * s[2] + C1);
  H[8] = Ve * 2.f * (D1 * s[0] * s[0] * s[1] * s[1] + C1);
  H[1] = H[3] = Ve * 2.f * D1 * s[2] * k0;
  H[2] = H[6] = Ve * 2.f * D1 * s[1] * k0;
  H[5] = H[7] = Ve * 2.f * D1 * s[0] * k0;
  const float floor_ = kClampFem * 2.f * C1 * Ve;
  float Em[6];  // xx yy zz xy xz yz
  if (c.A.p.fem_mode == NSN_FEM_DIAGONAL) {
    Em[0] = 1.f / fmaxf(H[0], floor_);
    Em[1] = 1.f / fmaxf(H[4], floor_);
    Em[2] = 1.f / fmaxf(H[8], floor_);
    Em[3] = Em[4] = Em[5] = 0.f;
  } else {
    M3 Q;
    float w[3];
    sym_eig3(H, Q, w);
    const float iw0 = 1.f / fmaxf(w[0], floor_), iw1 = 1.f / fmaxf(w[1], floor_), iw2 = 1.f / fmaxf(w[2], floor_);
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k)
      Em[k] = Q.m[3 * ia[k]] * Q.m[3 * ib[k]] * iw0 + Q.m[3 * ia[k] + 1] * Q.m[3 * ib[k] + 1] * iw1 +
              Q.m[3 * ia[k] + 2] * Q.m[3 * ib[k] + 2] * iw2;
  }
  const V3 cl = mk(Ve * gr[0] + lam0[0], Ve * gr[1] + lam0[1], Ve * gr[2] + lam0[2]);
  const V3 Ecl = sym_mul(Em, cl);
  const float ih = 1.f / h, ih2 = 1.f / (h * h);
  gst(S.row_err + r0, Ecl.x * ih);
  gst(S.row_err + r0 + 1, Ecl.y * ih);
  gst(S.row_err + r0 + 2, Ecl.z * ih);
  gst(S.row_C + r0, Em[0] * ih2);
  gst(S.row_C + r0 + 1, Em[1] * ih2);
  gst(S.row_C + r0 + 2, Em[2] * ih2);
#pragma unroll
  for (int k = 0; k < 6; ++k) gst(S.t_E + (size_t)k * NT + tg, Em[k] * ih2);
}

__device__ __forceinline__ void assemble_contact(const Ctx &c, int cl, int buf) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const float h = c.A.h;
  const int gc = E.con_off + cl;
  const int2 bd = gld(S.c_body + gc);
  const float4 n4 = gld(S.c_n + gc);
  const V3 n = mk(n4);
  const V3 aL = mk(gld(S.c_aL + gc)), bL = mk(gld(S.c_bL + gc));
  const V3 armA = body_arm(c, bd.x, aL);
  const V3 armB = bd.y >= 0 ? body_arm(c, bd.y, bL) : mk(0.f, 0.f, 0.f);
  const V3 pa = body_point(c, bd.x, aL);
  const V3 pb = bd.y >= 0 ? body_point(c, bd.y, bL) : bL;
  const float Cn = dot(n, pa - pb) - n4.w;
  V3 d1, d2;
  tangent_basis(n, d1, d2);
  // complementarity preconditioner (Sec. 7 eq. rscaling)
  float r_n, r_f;
  if (c.A.p.rmode == NSN_R_IDENTITY) {
    r_n = 1.f; r_f = 1.f;
  } else if (c.A.p.rmode == NSN_R_H2) {
    r_n = h * h; r_f = h;
  } else {
    const float Ann = effmass_dir(c, bd.x, armA, n, false) + effmass_dir(c, bd.y, armB, n, false);
    const float A1 = effmass_dir(c, bd.x, armA, d1, false) + effmass_dir(c, bd.y, armB, d1, false);
    const float A2 = effmass_dir(c, bd.x, armA, d2, false) + effmass_dir(c, bd.y, armB, d2, false);
    r_n = h * h * Ann;
    r_f = h * 0.5f * (A1 + A2);
  }
  const int r0 = row_con(E, cl);
  const float lam_n = gld(S.row_lam + r0), lf1 = gld(S.row_lam + r0 + 1), lf2 = gld(S.row_lam + r0 + 2);
  float phi, al, be;
  if (c.A.p.ncp == NSN_NCP_MIN) ncp_min(Cn, lam_n, r_n, phi, al, be);
  else ncp_fb(Cn, lam_n, r_n, phi, al, be);
  float v1 = 0.f, v2 = 0.f, W = __builtin_huge_valf();
  if (E.mu * lam_n > 0.f) {
    const V3 vr = point_vel(c, S.r_u, S.p_u, bd.x, armA) -
                  (bd.y >= 0 ? point_vel(c, S.r_u, S.p_u, bd.y, armB) : mk(0.f, 0.f, 0.f));
    v1 = dot(d1, vr);
    v2 = dot(d2, vr);
    const float vn = sqrtf(v1 * v1 + v2 * v2);
    const float lfn = sqrtf(lf1 * lf1 + lf2 * lf2);
    W = friction_w(c.A.p.ncp, vn, lam_n, lfn, E.mu, r_f);
  }
  const bool active = W < __builtin_huge_valf();
  // every input is read: the stores follow (see RowIn)
  gst(S.c_rA + gc, f4(armA, 0.f));
  gst(S.c_rB + gc, f4(armB, 0.f));
  gst(S.c_alpha + (size_t)buf * S.NC + gc, al);
  gst(S.row_C + r0, be * r_n / (h * h));
  gst(S.row_err + r0, phi / h);
  gst(S.c_active + (size_t)buf * S.NC + gc, active ? 1 : 0);
  if (active) {
    gst(S.row_C + r0 + 1, W / h);
    gst(S.row_C + r0 + 2, W / h);
    gst(S.row_err + r0 + 1, v1 + W * lf1);
    gst(S.row_err + r0 + 2, v2 + W * lf2);
  } else {
    // READING: inactive friction rows (mu lam_n <= 0, or W infinite) are removed
    // (zero J); compliance r_f/h and error r_f lambda_f drive their multipliers to zero
    gst(S.row_C + r0 + 1, r_f / h);
    gst(S.row_C + r0 + 2, r_f / h);
    gst(S.row_err + r0 + 1, r_f * lf1);
    gst(S.row_err + r0 + 2, r_f * lf2);
  }
}

// contact row combination: J_c^T v for one contact as a world-space direction applied
// at the two points: dir = alpha v_n n + [active](v_1 d1 + v_2 d2)
__device__ __forceinline__ V3 contact_dir_core(V3 n, float al, int active, float v0, float v1, float v2) {
  V3 dir = (al * v0) * n;
  if (active) {
    V3 d1, d2;
    tangent_basis(n, d1, d2);
    dir = dir + v1 * d1 + v2 * d2;
  }
  return dir;
}

__device__ __forceinline__ V3 contact_dir(const Ctx &c, int gc, const float *src, int buf) {
  const int r0 = row_con(c.E, gc - c.E.con_off);
  return contact_dir_core(mk(gld(c.S.c_n + gc)), gld(c.S.c_alpha + (size_t)buf * c.S.NC + gc),
                          gld(c.S.c_active + (size_t)buf * c.S.NC + gc), gld(src + r0), gld(src + r0 + 1),
                          gld(src + r0 + 2));
}


// ---- per-element row kernels (one unrolled path per element type) ----
// (J Y) rows of joint jl
// ---- J^T v in two passes: every element writes its contribution once (coalesced,
// element-parallel), then every body sums the contributions of its elements in a
// fixed order (deterministic, no atomics) ----
// v: the joint's six row values
// a joint's J^T v (o: side A's six values, then side B's) into its bodies' slots (none
// for the world)
__device__ __forceinline__ void joint_store_slots(const DevScene &S, int jg, const float o[12]) {
  const int2 js = gld(S.j_slot + jg);
  if (js.x >= 0) {
    gst(S.r_cj + 2 * (size_t)js.x, make_float4(o[0], o[1], o[2], 0.f));
    gst(S.r_cj + 2 * (size_t)js.x + 1, make_float4(o[3], o[4], o[5], 0.f));
  }
  if (js.y >= 0) {
    gst(S.r_cj + 2 * (size_t)js.y, make_float4(o[6], o[7], o[8], 0.f));
    gst(S.r_cj + 2 * (size_t)js.y + 1, make_float4(o[9], o[10], o[11], 0.f));
  }
}

__device__ __forceinline__ void joint_contrib_vals(const Ctx &c, int jl, const float v[6]) {
  const int jg = c.E.jnt_off + jl;
  const float *J = c.S.j_J + (size_t)72 * jg;
  float o[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) o[q] = 0.f;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
#pragma unroll
    for (int q = 0; q < 12; ++q) o[q] += v[r] * gld(J + 12 * r + q);
  }
  joint_store_slots(c.S, jg, o);
}

// A contact's J^T v, dir applied at its two points: a particle feature body reads the
// direction (c_cj); a rigid body's slot gets the force and the torque about its
// centre, with the sign of its side (the target side subtracts)
__device__ __forceinline__ void contact_store(const DevScene &S, int gc, V3 dir, V3 rA, V3 rB) {
  const int2 cs = gld(S.c_slot + gc);
  if (cs.x >= 0) {
    gst(S.r_cj + 2 * (size_t)cs.x, f4(dir, 0.f));
    gst(S.r_cj + 2 * (size_t)cs.x + 1, f4(cross(rA, dir), 0.f));
  } else {
    gst(S.c_cj + gc, f4(dir, 0.f));
  }
  if (cs.y >= 0) {
    const V3 t = cross(rB, dir);
    gst(S.r_cj + 2 * (size_t)cs.y, make_float4(-dir.x, -dir.y, -dir.z, 0.f));
    gst(S.r_cj + 2 * (size_t)cs.y + 1, make_float4(-t.x, -t.y, -t.z, 0.f));
  }
}

__device__ __forceinline__ void joint_contrib(const Ctx &c, int jl, const float *src) {
  const int r0 = row_joint(c.E, jl);
  float v[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) v[r] = gld(src + r0 + r);
  joint_contrib_vals(c, jl, v);
}

// J^T z of a tet from its compressed rows J[18] (u_i, w_i per stretch row), written
// straight into the particles' adjacency order (positions dst fixed at scene creation)
__device__ __forceinline__ void tet_contrib_core(const Ctx &c, const float *J, const float z[3], int4 dst) {
  V3 a0 = mk(0.f, 0.f, 0.f), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3 zu = z[i] * mk(J[6 * i], J[6 * i + 1], J[6 * i + 2]);
    const float w0 = J[6 * i + 3], w1 = J[6 * i + 4], w2 = J[6 * i + 5];
    a1 = a1 + w0 * zu;
    a2 = a2 + w1 * zu;
    a3 = a3 + w2 * zu;
    a0 = a0 - (w0 + w1 + w2) * zu;
  }
  store_tet_cj(c, dst, a0, a1, a2, a3);
}

// z = the tet's three row values (already loaded)
__device__ __forceinline__ void tet_contrib(const Ctx &c, int tl, const float z[3], int buf) {
  const DevScene &S = c.S;
  const int tg = c.E.tet_off + tl;
  float J[18];
#pragma unroll
  for (int m = 0; m < 18; ++m) J[m] = tJ(S, buf, m, tg);
  tet_contrib_core(c, J, z, gld(S.t_dst + tg));
}

// Sums the body's run of contribution slots in order (joints, feature-side contacts,
// target-side contacts), eight slots' loads at a time ahead of their sums.
__device__ __forceinline__ void gather_rigid(const Ctx &c, int g, float out[6]) {
  const DevScene &S = c.S;
  for (int k = 0; k < 6; ++k) out[k] = 0.f;
  const int2 rs = gld(S.r_slot + g);
  for (int k = rs.x; k < rs.y; k += 8) {
    float4 f[8], t[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (k + m >= rs.y) continue;
      f[m] = gld(S.r_cj + 2 * (size_t)(k + m));
      t[m] = gld(S.r_cj + 2 * (size_t)(k + m) + 1);
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (k + m >= rs.y) continue;
      out[0] += f[m].x; out[1] += f[m].y; out[2] += f[m].z;
      out[3] += t[m].x; out[4] += t[m].y; out[5] += t[m].z;
    }
  }
}

// The same sums with the body's slots read by the four lanes sub = 0..3 of an aligned
// group (slots k + sub and k + 4 + sub of each round of eight): every lane adds the
// round's slots in slot order from the lanes' registers, so the result is the one
// gather_rigid gives, in every lane of the group.
__device__ __forceinline__ void gather_rigid_lanes(const DevScene &S, int g, int sub, float out[6]) {
  for (int k = 0; k < 6; ++k) out[k] = 0.f;
  const int2 rs = gld(S.r_slot + g);
  const int lead = (threadIdx.x & 63) & ~3;
  for (int k = rs.x; k < rs.y; k += 8) {
    float4 f[2], t[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int sl = k + sub + 4 * m;
      f[m] = sl < rs.y ? gld(S.r_cj + 2 * (size_t)sl) : make_float4(0.f, 0.f, 0.f, 0.f);
      t[m] = sl < rs.y ? gld(S.r_cj + 2 * (size_t)sl + 1) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int src = lead + l;
        const float fx = __shfl(f[m].x, src, 64), fy = __shfl(f[m].y, src, 64), fz = __shfl(f[m].z, src, 64);
        const float tx = __shfl(t[m].x, src, 64), ty = __shfl(t[m].y, src, 64), tz = __shfl(t[m].z, src, 64);
        if (k + 4 * m + l < rs.y) {
          out[0] += fx; out[1] += fy; out[2] += fz;
          out[3] += tx; out[4] += ty; out[5] += tz;
        }
      }
    }
  }
}

// The tets wrote their contributions in this particle's adjacency order: a contiguous
// run, summed in that order with eight loads in flight.
__device__ __forceinline__ V3 gather_particle(const Ctx &c, int p) {
  const DevScene &S = c.S;
  V3 acc = mk(0.f, 0.f, 0.f);
  const int k0 = gld(S.p_tadj_ptr + p), k1 = gld(S.p_tadj_ptr + p + 1);
  const int c0 = gld(S.p_acon_beg + p), c1 = gld(S.p_acon_end + p);
  int k = k0;
  if (c.cl) {  // the same sums in the same order, from LDS, four entries' reads at a time
    const float *cx = c.cl, *cy = cx + c.cl_n, *cz = cy + c.cl_n;
    for (; k + 4 <= k1; k += 4) {
      float vx[4], vy[4], vz[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int i = k + m - c.cl_base;
        vx[m] = cx[i];
        vy[m] = cy[i];
        vz[m] = cz[i];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) acc = acc + mk(vx[m], vy[m], vz[m]);
    }
    for (; k < k1; ++k) {
      const int i = k - c.cl_base;
      acc = acc + mk(cx[i], cy[i], cz[i]);
    }
  }
  for (; k + 8 <= k1; k += 8) {
    float4 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = gld(S.p_cj + k + m);
#pragma unroll
    for (int m = 0; m < 8; ++m) acc = acc + mk(v[m]);
  }
  for (; k < k1; ++k) acc = acc + mk(gld(S.p_cj + k));
  for (int gc = c0; gc < c1; ++gc) acc = acc + mk(gld(S.c_cj + gc));
  return acc;
}

__device__ __forceinline__ void joint_JY(const Ctx &c, int jl, const float *Y, float jy[6]) {
  const EnvInfo &E = c.E;
  const int jg = E.jnt_off + jl;
  const int4 info = gld(c.S.j_info + jg);
  const float *J = c.S.j_J + (size_t)72 * jg;
  const int dB = ldof(E, info.z - E.rig_off);
  const int dA = info.y >= 0 ? ldof(E, info.y - E.rig_off) : -1;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    float Jr[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) Jr[q] = gld(J + 12 * r + q);
    float acc = row_dot_rigid(Jr + 6, Y, dB);
    if (dA >= 0) acc += row_dot_rigid(Jr, Y, dA);
    jy[r] = acc;
  }
}

// J y of a tet from its compressed rows J[18] and its vertex ids (global particle
// indices) into the env's body-space vector Y
__device__ __forceinline__ void tet_JY_core(const EnvInfo &E, const float *J, int4 id, const float *Y, float jy[3]) {
  const int base = 6 * E.n_rig - 3 * E.par_off;
  const V3 y0 = mk(Y[base + 3 * id.x], Y[base + 3 * id.x + 1], Y[base + 3 * id.x + 2]);
  const V3 y1 = mk(Y[base + 3 * id.y], Y[base + 3 * id.y + 1], Y[base + 3 * id.y + 2]) - y0;
  const V3 y2 = mk(Y[base + 3 * id.z], Y[base + 3 * id.z + 1], Y[base + 3 * id.z + 2]) - y0;
  const V3 y3 = mk(Y[base + 3 * id.w], Y[base + 3 * id.w + 1], Y[base + 3 * id.w + 2]) - y0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3 u = mk(J[6 * i], J[6 * i + 1], J[6 * i + 2]);
    const float w0 = J[6 * i + 3], w1 = J[6 * i + 4], w2 = J[6 * i + 5];
    jy[i] = dot(u, w0 * y1 + w1 * y2 + w2 * y3);
  }
}

__device__ __forceinline__ void tet_JY(const Ctx &c, int tl, const float *Y, int buf, float jy[3]) {
  const DevScene &S = c.S;
  const int tg = c.E.tet_off + tl;
  float J[18];
#pragma unroll
  for (int m = 0; m < 18; ++m) J[m] = tJ(S, buf, m, tg);
  tet_JY_core(c.E, J, gld(S.t_ids + tg), Y, jy);
}

__device__ __forceinline__ void contact_JY_core(const Ctx &c, const float *Y, int2 bd, V3 n, V3 rA, V3 rB, float al,
                                                int active, float jy[3]) {
  const V3 vr = point_vel_dof(c, Y, bd.x, rA) - (bd.y >= 0 ? point_vel_dof(c, Y, bd.y, rB) : mk(0.f, 0.f, 0.f));
  jy[0] = al * dot(n, vr);
  if (active) {
    V3 d1, d2;
    tangent_basis(n, d1, d2);
    jy[1] = dot(d1, vr);
    jy[2] = dot(d2, vr);
  } else {
    jy[1] = 0.f;
    jy[2] = 0.f;
  }
}

__device__ __forceinline__ void contact_JY(const Ctx &c, int cl, const float *Y, int buf, float jy[3]) {
  const DevScene &S = c.S;
  const int gc = c.E.con_off + cl;
  contact_JY_core(c, Y, gld(S.c_body + gc), mk(gld(S.c_n + gc)), mk(gld(S.c_rA + gc)), mk(gld(S.c_rB + gc)),
                  gld(S.c_alpha + (size_t)buf * S.NC + gc), gld(S.c_active + (size_t)buf * S.NC + gc), jy);
}

// J_i H~^-1 J_i^T of every row of an element (preconditioner diagonal without C, eps)
__device__ __forceinline__ void joint_hdiag(const Ctx &c, int jl, float dg[6]) {
  const int jg = c.E.jnt_off + jl;
  const int4 info = gld(c.S.j_info + jg);
  const float *J = c.S.j_J + (size_t)72 * jg;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    float Jr[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) Jr[q] = gld(J + 12 * r + q);
    float acc = rigid_quad(c, info.z, Jr + 6);
    if (info.y >= 0) acc += rigid_quad(c, info.y, Jr);
    dg[r] = acc;
  }
}

__device__ __forceinline__ void tet_hdiag(const Ctx &c, int tl, int buf, float dg[3]) {
  const DevScene &S = c.S;
  const int tg = c.E.tet_off + tl;
  const int4 id = gld(S.t_ids + tg);
  const float4 H0 = gld(S.p_H + id.x), H1 = gld(S.p_H + id.y), H2 = gld(S.p_H + id.z), H3 = gld(S.p_H + id.w);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3 u = mk(tJ(S, buf, 6 * i, tg), tJ(S, buf, 6 * i + 1, tg), tJ(S, buf, 6 * i + 2, tg));
    const float w0 = tJ(S, buf, 6 * i + 3, tg), w1 = tJ(S, buf, 6 * i + 4, tg), w2 = tJ(S, buf, 6 * i + 5, tg);
    const float ws = w0 + w1 + w2;
    const V3 u2 = mk(u.x * u.x, u.y * u.y, u.z * u.z);
    dg[i] = ws * ws * (u2.x / H0.x + u2.y / H0.y + u2.z / H0.z) + w0 * w0 * (u2.x / H1.x + u2.y / H1.y + u2.z / H1.z) +
            w1 * w1 * (u2.x / H2.x + u2.y / H2.y + u2.z / H2.z) + w2 * w2 * (u2.x / H3.x + u2.y / H3.y + u2.z / H3.z);
  }
}

__device__ __forceinline__ void contact_hdiag(const Ctx &c, int cl, int buf, float dg[3]) {
  const DevScene &S = c.S;
  const int gc = c.E.con_off + cl;
  const int2 bd = gld(S.c_body + gc);
  const V3 n = mk(gld(S.c_n + gc));
  const V3 rA = mk(gld(S.c_rA + gc)), rB = mk(gld(S.c_rB + gc));
  const float al = gld(S.c_alpha + (size_t)buf * S.NC + gc);
  dg[0] = al * al * (effmass_dir(c, bd.x, rA, n, true) + effmass_dir(c, bd.y, rB, n, true));
  if (gld(S.c_active + (size_t)buf * S.NC + gc)) {
    V3 d1, d2;
    tangent_basis(n, d1, d2);
    dg[1] = effmass_dir(c, bd.x, rA, d1, true) + effmass_dir(c, bd.y, rB, d1, true);
    dg[2] = effmass_dir(c, bd.x, rA, d2, true) + effmass_dir(c, bd.y, rB, d2, true);
  } else {
    dg[1] = 0.f;
    dg[2] = 0.f;
  }
}

// b and P of an element's N rows from its J Y and Jacobi diagonal (err and C read
// before the first store, see RowIn)
template <int N>
__device__ __forceinline__ void rhs_rows(const DevScene &S, int r0, const float jy[N], const float dg[N], float ih,
                                         float eps) {
  float err[N], C[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    err[r] = gld(S.row_err + r0 + r);
    C[r] = gld(S.row_C + r0 + r);
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    gst(S.row_b + r0 + r, (jy[r] - err[r]) * ih);
    gst(S.row_P + r0 + r, 1.f / (dg[r] + C[r] + eps));
  }
}

// Schur right-hand side b = (J Y - err)/h and Jacobi preconditioner for every row
// (Y = H~^-1 g already in place)
template <int BS, bool EXT>
__device__ __forceinline__ void rhs_and_precond(const Ctx &c, const float *Y, int buf, int nel, float eps) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const float ih = 1.f / c.A.h;
  for (int el = threadIdx.x; el < nel; el += BS) {
    if (el < E.n_jnt) {
      float jy[6], dg[6];
      joint_JY(c, el, Y, jy);
      joint_hdiag(c, el, dg);
      const int r0 = row_joint(E, el);
      rhs_rows<6>(S, r0, jy, dg, ih, eps);
    } else if (EXT && el < E.n_jnt + E.n_tet && lin_tets(E)) {
      float jy[6], dg[6];
      const int tl = el - E.n_jnt;
      ltet_JY(c, tl, Y, buf, jy);
      ltet_hdiag(c, tl, buf, dg);
      rhs_rows<6>(S, row_tet(E, tl), jy, dg, ih, eps);
    } else if (el < E.n_jnt + E.n_tet) {
      float jy[3], dg[3];
      const int tl = el - E.n_jnt;
      tet_JY(c, tl, Y, buf, jy);
      tet_hdiag(c, tl, buf, dg);
      rhs_rows<3>(S, row_tet(E, tl), jy, dg, ih, eps);
    } else {
      float jy[3], dg[3];
      const int cl = el - E.n_jnt - E.n_tet;
      contact_JY(c, cl, Y, buf, jy);
      contact_hdiag(c, cl, buf, dg);
      rhs_rows<3>(S, row_con(E, cl), jy, dg, ih, eps);
    }
  }
}

// a row's parts of <z, w>, <w, P w> and <w, P q>, added to part[0..2]
__device__ __forceinline__ void mv_dots_reg(float z, float w, float P, float q, double part[3]) {
  const float Pw = P * w;
  part[0] += (double)z * (double)w;
  part[1] += (double)w * (double)Pw;
  part[2] += (double)Pw * (double)q;
}

// w = A z = J Y + C z + eps z for every row (Y = H~^-1 J^T z in place); adds the
// thread's parts of <z, w>, <w, P w> and <w, P q> to part[0..2].  FIRST: also q = w
// (initialisation of the PCR).
__device__ __forceinline__ void mv_dots(const DevScene &S, int row, float z, float w, double part[3]) {
  const float Pw = gld(S.row_P + row) * w;
  part[0] += (double)z * (double)w;
  part[1] += (double)w * (double)Pw;
  part[2] += (double)Pw * (double)gld(S.row_q + row);
}

// Island mode (EXT, isl): every element stores its own three partial sums in el_dots
// (summed per island in element order afterwards) instead of adding them to part.
template <int BS, bool FIRST, bool EXT>
__device__ __forceinline__ void matvec_rows(const Ctx &c, const float *Y, int buf, int nel, float eps, double part_[3], bool isl = false) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  // every row of an element is read before its first store (see RowIn); q of the dots
  // is the stored w itself in the first pass
  for (int el = threadIdx.x; el < nel; el += BS) {
    double el3[3] = {0.0, 0.0, 0.0};
    double *part = (EXT && isl) ? el3 : part_;
    if (el < E.n_jnt) {
      const int r0 = row_joint(E, el);
      float z[6], C[6], P[6], q[6], jy[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        z[r] = gld(S.row_z + r0 + r);
        C[r] = gld(S.row_C + r0 + r);
        P[r] = gld(S.row_P + r0 + r);
        q[r] = FIRST ? 0.f : gld(S.row_q + r0 + r);
      }
      joint_JY(c, el, Y, jy);
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        const float w = jy[r] + C[r] * z[r] + eps * z[r];
        gst(S.row_w + r0 + r, w);
        if (FIRST) gst(S.row_q + r0 + r, w);
        mv_dots_reg(z[r], w, P[r], FIRST ? w : q[r], part);
      }
    } else if (EXT && el < E.n_jnt + E.n_tet && lin_tets(E)) {
      // linear tet: normal rows with the 3x3 compliance block, shear rows diagonal
      float jy[6];
      const int tl = el - E.n_jnt;
      const int tg = E.tet_off + tl;
      const int r0 = row_tet(E, tl);
      float Em[6], zr[6], C[6], P[6], q[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        Em[k] = gld(S.t_E + (size_t)k * S.NT + tg);
        zr[k] = gld(S.row_z + r0 + k);
        C[k] = k < 3 ? 0.f : gld(S.row_C + r0 + k);
        P[k] = gld(S.row_P + r0 + k);
        q[k] = FIRST ? 0.f : gld(S.row_q + r0 + k);
      }
      ltet_JY(c, tl, Y, buf, jy);
      const V3 z = mk(zr[0], zr[1], zr[2]);
      const V3 cz = sym_mul(Em, z);
      float w[6];
      w[0] = jy[0] + cz.x + eps * z.x; w[1] = jy[1] + cz.y + eps * z.y; w[2] = jy[2] + cz.z + eps * z.z;
#pragma unroll
      for (int r = 3; r < 6; ++r) w[r] = jy[r] + C[r] * zr[r] + eps * zr[r];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        gst(S.row_w + r0 + r, w[r]);
        if (FIRST) gst(S.row_q + r0 + r, w[r]);
        mv_dots_reg(zr[r], w[r], P[r], FIRST ? w[r] : q[r], part);
      }
    } else if (el < E.n_jnt + E.n_tet) {
      const int tl = el - E.n_jnt;
      const int tg = E.tet_off + tl;
      const int r0 = row_tet(E, tl);
      float J[18], Em[6], zr[3], P[3], q[3], jy[3];
#pragma unroll
      for (int m = 0; m < 18; ++m) J[m] = tJ(S, buf, m, tg);
      const int4 ids = gld(S.t_ids + tg);
#pragma unroll
      for (int k = 0; k < 6; ++k) Em[k] = gld(S.t_E + (size_t)k * S.NT + tg);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        zr[r] = gld(S.row_z + r0 + r);
        P[r] = gld(S.row_P + r0 + r);
        q[r] = FIRST ? 0.f : gld(S.row_q + r0 + r);
      }
      tet_JY_core(E, J, ids, Y, jy);
      const V3 z = mk(zr[0], zr[1], zr[2]);
      const V3 cz = sym_mul(Em, z);
      const float w[3] = {jy[0] + cz.x + eps * z.x, jy[1] + cz.y + eps * z.y, jy[2] + cz.z + eps * z.z};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        gst(S.row_w + r0 + r, w[r]);
        if (FIRST) gst(S.row_q + r0 + r, w[r]);
        mv_dots_reg(zr[r], w[r], P[r], FIRST ? w[r] : q[r], part);
      }
    } else {
      const int cl = el - E.n_jnt - E.n_tet;
      const int r0 = row_con(E, cl);
      float z[3], C[3], P[3], q[3], jy[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        z[r] = gld(S.row_z + r0 + r);
        C[r] = gld(S.row_C + r0 + r);
        P[r] = gld(S.row_P + r0 + r);
        q[r] = FIRST ? 0.f : gld(S.row_q + r0 + r);
      }
      contact_JY(c, cl, Y, buf, jy);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const float w = jy[r] + C[r] * z[r] + eps * z[r];
        gst(S.row_w + r0 + r, w);
        if (FIRST) gst(S.row_q + r0 + r, w);
        mv_dots_reg(z[r], w, P[r], FIRST ? w : q[r], part);
      }
    }
    if (EXT && isl) {
      double *d = S.el_dots + 3 * (size_t)(E.jnt_off + E.tet_off + E.con_off + el);
      d[0] = el3[0]; d[1] = el3[1]; d[2] = el3[2];
    }
  }
}

// H~^-1 applied to a rigid 6-vector (in place), given 1/m and the world inverse inertia
__device__ __forceinline__ void hinv_rigid_vals(float im, const float Iwinv[6], float v[6]) {
  if (im == 0.f) {
    for (int k = 0; k < 6; ++k) v[k] = 0.f;
    return;
  }
  const V3 a = sym_mul(Iwinv, mk(v[3], v[4], v[5]));
  v[0] *= im; v[1] *= im; v[2] *= im;
  v[3] = a.x; v[4] = a.y; v[5] = a.z;
}

// H~^-1 applied to a rigid 6-vector (in place)
__device__ __forceinline__ void hinv_rigid(const Ctx &c, int g, float v[6]) {
  const float im = gld(c.S.r_inertia + g).w;
  if (im == 0.f) {
    for (int k = 0; k < 6; ++k) v[k] = 0.f;
    return;
  }
  const V3 a = sym_mul_g(c.S.r_Iwinv + 6 * g, mk(v[3], v[4], v[5]));
  v[0] *= im; v[1] *= im; v[2] *= im;
  v[3] = a.x; v[4] = a.y; v[5] = a.z;
}

// Y = H~^-1 (sum of the element contributions) for every body of the env
__device__ __forceinline__ void gather_hinv(const Ctx &c, float *Y, int tid, int BS) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int nb = E.n_rig + E.n_par;
  for (int b = tid; b < nb; b += BS) {
    if (b < E.n_rig) {
      const int g = E.rig_off + b;
      float v[6];
      gather_rigid(c, g, v);
      hinv_rigid(c, g, v);
      const int d = 6 * b;
#pragma unroll
      for (int k = 0; k < 6; ++k) Y[d + k] = v[k];
    } else {
      const int p = E.par_off + b - E.n_rig;
      const V3 a = gather_particle(c, p);
      const float4 H = gld(S.p_H + p);
      const int d = 6 * E.n_rig + 3 * (b - E.n_rig);
      Y[d] = a.x / H.x;
      Y[d + 1] = a.y / H.y;
      Y[d + 2] = a.z / H.z;
    }
  }
}

// J^T src contributions of every element (src: one value per row; buf: which
// Jacobian of the ping-pong pair); joints only when their bodies need them.
template <int BS, bool EXT>
__device__ __forceinline__ void contrib_pass(const Ctx &c, const float *src, int buf, int nel, bool joints) {
  const EnvInfo &E = c.E;
  for (int el = threadIdx.x; el < nel; el += BS) {
    if (el < E.n_jnt) {
      if (joints) joint_contrib(c, el, src);
    } else if (EXT && el < E.n_jnt + E.n_tet && lin_tets(E)) {
      const int tl = el - E.n_jnt;
      const int r0 = row_tet(E, tl);
      float z[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) z[r] = gld(src + r0 + r);
      ltet_contrib(c, tl, z, buf);
    } else if (el < E.n_jnt + E.n_tet) {
      const int tl = el - E.n_jnt;
      const int r0 = row_tet(E, tl);
      const float z[3] = {gld(src + r0), gld(src + r0 + 1), gld(src + r0 + 2)};
      tet_contrib(c, tl, z, buf);
    } else {
      const int gc = E.con_off + el - E.n_jnt - E.n_tet;
      contact_store(c.S, gc, contact_dir(c, gc, src, buf), mk(gld(c.S.c_rA + gc)), mk(gld(c.S.c_rB + gc)));
    }
  }
}

// The values of one row that a PCR pass reads.  An element pass reads all the rows
// (and the element data) of an element before it writes any of them: the row arrays
// are reached through pointers the compiler cannot tell apart, so a load placed after
// a store waits for it, and an element that interleaved them would pay one memory
// round trip per row.
struct RowIn {
  float P, z, p, q, x, w;
};

// One PCR row.  INIT: z = P b, x = 0, p = z.  Else the direction update of the
// previous iteration (upd: p = z + beta p, q = w + beta q) followed by this
// iteration's x += alpha p, z -= alpha P q.  pcr_row_load reads the row (INIT: P and b,
// the latter in the z slot), pcr_row_apply updates and stores it.
template <bool INIT>
__device__ __forceinline__ void pcr_row_load(const DevScene &S, int row, bool upd, RowIn &v) {
  v.P = gld(S.row_P + row);
  if (INIT) {
    v.z = gld(S.row_b + row);
    return;
  }
  v.p = gld(S.row_p + row);
  v.q = gld(S.row_q + row);
  v.z = gld(S.row_z + row);
  v.x = gld(S.row_x + row);
  v.w = upd ? gld(S.row_w + row) : 0.f;
}

template <bool INIT>
__device__ __forceinline__ float pcr_row_apply(const DevScene &S, int row, const RowIn &v, float alpha, float beta,
                                               bool upd) {
  if (INIT) {
    const float z = v.P * v.z;
    gst(S.row_x + row, 0.f);
    gst(S.row_z + row, z);
    gst(S.row_p + row, z);
    return z;
  }
  float p = v.p, q = v.q;
  const float z0 = v.z, P = v.P, x = v.x;
  if (upd) {
    p = z0 + beta * p;
    q = v.w + beta * q;
    gst(S.row_p + row, p);
    gst(S.row_q + row, q);
  }
  gst(S.row_x + row, x + alpha * p);
  const float z = z0 - alpha * (P * q);
  gst(S.row_z + row, z);
  return z;
}

template <bool INIT>
__device__ __forceinline__ float pcr_row(const DevScene &S, int row, float alpha, float beta, bool upd) {
  RowIn v;
  pcr_row_load<INIT>(S, row, upd, v);
  return pcr_row_apply<INIT>(S, row, v, alpha, beta, upd);
}

// Element pass of the PCR: the rows of every element are updated (pcr_row) and the
// element then writes its J^T z contribution for the body pass (gather_hinv).
// Island mode (EXT, isl): alpha and beta are the element's island's, and the rows of an
// island that has stopped keep their values (the element still writes its J^T z).
template <int BS, bool INIT, bool EXT>
__device__ __forceinline__ void pcr_update_contrib(const Ctx &c, int buf, int nel, float alpha_, float beta_, bool upd_,
                                   bool isl = false, int ib = 0) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  for (int el = threadIdx.x; el < nel; el += BS) {
    float alpha = alpha_, beta = beta_;
    bool upd = upd_, act = true;
    if (EXT && isl && !INIT) {
      const IslState &I = S.isl[ib + S.el_isl[E.jnt_off + E.tet_off + E.con_off + el]];
      alpha = I.alpha;
      beta = I.beta;
      act = I.active != 0;
    }
    // an element's rows and data are all read before its first store (see RowIn);
    // a row of a stopped island keeps its z
    if (el < E.n_jnt) {
      const int r0 = row_joint(E, el);
      RowIn v[6];
      float z[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        if (act) pcr_row_load<INIT>(S, r0 + r, upd, v[r]);
        else v[r].z = gld(S.row_z + r0 + r);
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) z[r] = act ? pcr_row_apply<INIT>(S, r0 + r, v[r], alpha, beta, upd) : v[r].z;
      joint_contrib_vals(c, el, z);
    } else if (EXT && el < E.n_jnt + E.n_tet && lin_tets(E)) {
      const int tl = el - E.n_jnt;
      const int r0 = row_tet(E, tl);
      RowIn v[6];
      float z[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        if (act) pcr_row_load<INIT>(S, r0 + r, upd, v[r]);
        else v[r].z = gld(S.row_z + r0 + r);
      }
#pragma unroll
      for (int r = 0; r < 6; ++r) z[r] = act ? pcr_row_apply<INIT>(S, r0 + r, v[r], alpha, beta, upd) : v[r].z;
      ltet_contrib(c, tl, z, buf);
    } else if (el < E.n_jnt + E.n_tet) {
      const int tl = el - E.n_jnt, tg = E.tet_off + tl;
      const int r0 = row_tet(E, tl);
      RowIn v[3];
      float z[3], J[18];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (act) pcr_row_load<INIT>(S, r0 + r, upd, v[r]);
        else v[r].z = gld(S.row_z + r0 + r);
      }
#pragma unroll
      for (int m = 0; m < 18; ++m) J[m] = tJ(S, buf, m, tg);
      const int4 dst = gld(S.t_dst + tg);
#pragma unroll
      for (int r = 0; r < 3; ++r) z[r] = act ? pcr_row_apply<INIT>(S, r0 + r, v[r], alpha, beta, upd) : v[r].z;
      tet_contrib_core(c, J, z, dst);
    } else {
      const int cl = el - E.n_jnt - E.n_tet, gc = E.con_off + cl;
      const int r0 = row_con(E, cl);
      RowIn v[3];
      float z[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (act) pcr_row_load<INIT>(S, r0 + r, upd, v[r]);
        else v[r].z = gld(S.row_z + r0 + r);
      }
      const V3 n = mk(gld(S.c_n + gc));
      const float al = gld(S.c_alpha + (size_t)buf * S.NC + gc);
      const int active = gld(S.c_active + (size_t)buf * S.NC + gc);
      const V3 rA = mk(gld(S.c_rA + gc)), rB = mk(gld(S.c_rB + gc));
#pragma unroll
      for (int r = 0; r < 3; ++r) z[r] = act ? pcr_row_apply<INIT>(S, r0 + r, v[r], alpha, beta, upd) : v[r].z;
      contact_store(S, gc, contact_dir_core(n, al, active, z[0], z[1], z[2]), rA, rB);
    }
  }
}

// ---------------------------------------------------------------------------
// Register-resident PCR.  The PCR's row vectors (x, z, p, q, w) and the
// preconditioner P of every tet and contact stay in the registers of the thread that
// owns the element for all the PCR iterations of a Newton iteration: thread t owns
// elements t, t + BS, ..., t + (R-1) BS, so in an env with at most R BS elements the
// row vectors never go through memory inside the loop (the element data -- compressed
// J, compliance, ids -- is still read where it is used).  Joints (six rows each) keep
// their rows in memory.  The arithmetic and its order are those of the streaming form
// (pcr_update_contrib, gather_hinv, matvec_rows), so both give identical results.
// Returns the PCR iterations performed; x is written back to row_x.
// ---------------------------------------------------------------------------

// J^T z of a resident tet or contact (z from registers) for the body pass
__device__ __forceinline__ void resident_contrib(const Ctx &c, int el, int buf, const float z[3]) {
  const EnvInfo &E = c.E;
  if (el < E.n_jnt + E.n_tet) {
    tet_contrib(c, el - E.n_jnt, z, buf);
  } else {
    const int gc = E.con_off + el - E.n_jnt - E.n_tet;
    const DevScene &S = c.S;
    contact_store(S, gc,
                  contact_dir_core(mk(gld(S.c_n + gc)), gld(S.c_alpha + (size_t)buf * S.NC + gc),
                                   gld(S.c_active + (size_t)buf * S.NC + gc), z[0], z[1], z[2]),
                  mk(gld(S.c_rA + gc)), mk(gld(S.c_rB + gc)));
  }
}

// w = J Y + C z + eps z of a resident tet or contact
__device__ __forceinline__ void resident_matvec(const Ctx &c, int el, int buf, const float *Y, float eps,
                                                const float z[3], float w[3]) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  float jy[3];
  if (el < E.n_jnt + E.n_tet) {
    const int tl = el - E.n_jnt, tg = E.tet_off + tl;
    tet_JY(c, tl, Y, buf, jy);
    float Em[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) Em[k] = gld(S.t_E + (size_t)k * S.NT + tg);
    const V3 zz = mk(z[0], z[1], z[2]);
    const V3 cz = sym_mul(Em, zz);
    w[0] = jy[0] + cz.x + eps * zz.x;
    w[1] = jy[1] + cz.y + eps * zz.y;
    w[2] = jy[2] + cz.z + eps * zz.z;
  } else {
    const int cl = el - E.n_jnt - E.n_tet;
    contact_JY(c, cl, Y, buf, jy);
    const int r0 = row_con(E, cl);
#pragma unroll
    for (int r = 0; r < 3; ++r) w[r] = jy[r] + gld(S.row_C + r0 + r) * z[r] + eps * z[r];
  }
}

__device__ __forceinline__ int resident_row0(const EnvInfo &E, int el) {
  return el < E.n_jnt + E.n_tet ? row_tet(E, el - E.n_jnt) : row_con(E, el - E.n_jnt - E.n_tet);
}

// the rows of a joint in memory, as in the streaming form
__device__ __forceinline__ void joint_matvec_mem(const Ctx &c, int jl, const float *Y, float eps, bool first,
                                                 double part[3]) {
  const DevScene &S = c.S;
  float jy[6];
  joint_JY(c, jl, Y, jy);
  const int r0 = row_joint(c.E, jl);
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const float zz = gld(S.row_z + r0 + r);
    const float ww = jy[r] + gld(S.row_C + r0 + r) * zz + eps * zz;
    gst(S.row_w + r0 + r, ww);
    if (first) gst(S.row_q + r0 + r, ww);
    mv_dots(S, r0 + r, zz, ww, part);
  }
}

template <int BS, int R>
__device__ __forceinline__ int pcr_resident(const Ctx &c, float *Y, int buf, int nel, float eps, int cr_iters,
                                            bool dump, Red<BS> &red) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int tid = threadIdx.x;
  const int nj = E.n_jnt;
  float x[R][3], z[R][3], p[R][3], q[R][3], w[R][3], P[R][3];
  // ---- the PCR's start: z = P b, x = 0, p = z; J^T z ----
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int el = tid + j * BS;
    if (el >= nel) continue;
    if (el < nj) {
      const int r0 = row_joint(E, el);
#pragma unroll
      for (int r = 0; r < 6; ++r) pcr_row<true>(S, r0 + r, 0.f, 0.f, false);
      joint_contrib(c, el, S.row_z);
      continue;
    }
    const int r0 = resident_row0(E, el);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      P[j][r] = S.row_P[r0 + r];
      const float zz = P[j][r] * S.row_b[r0 + r];
      x[j][r] = 0.f;
      z[j][r] = zz;
      p[j][r] = zz;
      q[j][r] = 0.f;
      w[j][r] = 0.f;
    }
    resident_contrib(c, el, buf, z[j]);
  }
  __syncthreads();
  gather_hinv(c, Y, tid, BS);
  __syncthreads();
  double dots[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int el = tid + j * BS;
    if (el >= nel) continue;
    if (el < nj) {
      joint_matvec_mem(c, el, Y, eps, true, dots);
      continue;
    }
    resident_matvec(c, el, buf, Y, eps, z[j], w[j]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      q[j][r] = w[j][r];
      mv_dots_reg(z[j][r], w[j][r], P[j][r], q[j][r], dots);
    }
  }
  block_sum3<BS>(dots, red);
  if (dump) {  // A (P b) of the dumped iteration
    for (int r = tid; r < 6 * nj; r += BS) S.row_dump[E.row_off + r] = S.row_w[E.row_off + r];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int el = tid + j * BS;
      if (el < nj || el >= nel) continue;
      const int r0 = resident_row0(E, el);
#pragma unroll
      for (int r = 0; r < 3; ++r) S.row_dump[r0 + r] = w[j][r];
    }
  }
  double rho = dots[0], qs = dots[1];
  // READING: stop once <z, A z> is at rounding level relative to its start
  const double rho_stop = kTauCR * rho;
  float beta = 0.f;
  int done = 0;
  for (int it = 0; it < cr_iters; ++it) {
    if (!(rho > rho_stop) || !(rho > 0.0)) break;
    if (!(qs > 0.0)) break;
    const float alpha = (float)(rho / qs);
    ++done;
    const bool upd = it > 0;
    if (it == cr_iters - 1) {  // the last update needs no further product
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int el = tid + j * BS;
        if (el >= nel) continue;
        if (el < nj) {
          const int r0 = row_joint(E, el);
#pragma unroll
          for (int r = 0; r < 6; ++r) {
            const int row = r0 + r;
            const float pp = upd ? S.row_z[row] + beta * S.row_p[row] : S.row_p[row];
            S.row_x[row] += alpha * pp;
          }
          continue;
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const float pp = upd ? z[j][r] + beta * p[j][r] : p[j][r];
          x[j][r] += alpha * pp;
        }
      }
      break;
    }
    // direction update, x += alpha p, z -= alpha P q, J^T z contributions
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int el = tid + j * BS;
      if (el >= nel) continue;
      if (el < nj) {
        const int r0 = row_joint(E, el);
#pragma unroll
        for (int r = 0; r < 6; ++r) pcr_row<false>(S, r0 + r, alpha, beta, upd);
        joint_contrib(c, el, S.row_z);
        continue;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        float pp = p[j][r], qq = q[j][r];
        const float z0 = z[j][r];
        if (upd) {
          pp = z0 + beta * pp;
          qq = w[j][r] + beta * qq;
          p[j][r] = pp;
          q[j][r] = qq;
        }
        x[j][r] = x[j][r] + alpha * pp;
        z[j][r] = z0 - alpha * (P[j][r] * qq);
      }
      resident_contrib(c, el, buf, z[j]);
    }
    __syncthreads();
    gather_hinv(c, Y, tid, BS);
    __syncthreads();
    dots[0] = dots[1] = dots[2] = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int el = tid + j * BS;
      if (el >= nel) continue;
      if (el < nj) {
        joint_matvec_mem(c, el, Y, eps, false, dots);
        continue;
      }
      resident_matvec(c, el, buf, Y, eps, z[j], w[j]);
#pragma unroll
      for (int r = 0; r < 3; ++r) mv_dots_reg(z[j][r], w[j][r], P[j][r], q[j][r], dots);
    }
    block_sum3<BS>(dots, red);
    const double b = dots[0] / rho;
    qs = dots[1] + 2.0 * b * dots[2] + b * b * qs;
    beta = (float)b;
    rho = dots[0];
  }
  // Delta lambda of the resident rows back to memory
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int el = tid + j * BS;
    if (el < nj || el >= nel) continue;
    const int r0 = resident_row0(E, el);
#pragma unroll
    for (int r = 0; r < 3; ++r) S.row_x[r0 + r] = x[j][r];
  }
  return done;
}

// position update q = q^- + h G(q^k) u (Alg. 1; quaternion normalised every update)
// ---------------------------------------------------------------------------
// One-pass PCR.  The recurrences are those of the single-reduction form above, but
// J^T z is carried in body space instead of being formed from z each iteration: with
// Bz = J^T z and Bq = J^T (P q), the updates q' = w + beta q and z' = z - alpha P q'
// give, by linearity,
//     Bq' = J^T (P w) + beta Bq,      Bz' = Bz - alpha Bq',
// so one element visit per iteration suffices: it applies the deferred row updates of
// the last reduction, forms w = J H~^-1 Bz + C' z at the new z, and writes its
// J^T (P w) contribution in the same visit, reading the element's Jacobian once per
// iteration instead of twice.  The body pass sums those contributions, advances Bq and
// Bz and applies H~^-1.  Bz starts as J^T z0 from an ordinary contribution pass, so
// the first product (the record a dump step keeps) is the streaming form's.
// ---------------------------------------------------------------------------
// Bz is re-formed from the rows (residual replacement) once rho = <z, A z> has fallen
// by this factor since Bz was last formed: the carried Bz's rounding gap grows with the
// updates' size, the size of Bz (~ |z|) with the residual, so the gap relative to Bz
// stays below about (updates since) x eps x 10.
constexpr double kOnePassRefreshDrop = 1e-2;

// The last PCR iteration's x += alpha p (upd: p = z + beta p first) over the env's rows,
// four rows of the thread at a time with their loads before their stores (see RowIn)
template <int BS>
__device__ __forceinline__ void last_x_update(const DevScene &S, int R0, int nrows, int tid, bool upd, float alpha,
                                              float beta) {
  for (int r = tid; r < nrows; r += 4 * BS) {
    float z[4], p[4], x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = R0 + r + j * BS;
      const bool in = r + j * BS < nrows;
      z[j] = in && upd ? gld(S.row_z + row) : 0.f;
      p[j] = in ? gld(S.row_p + row) : 0.f;
      x[j] = in ? gld(S.row_x + row) : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (r + j * BS >= nrows) continue;
      const float pp = upd ? z[j] + beta * p[j] : p[j];
      gst(S.row_x + R0 + r + j * BS, x[j] + alpha * pp);
    }
  }
}

// Deferred row update: MODE 0 keeps the rows as the initialisation set them; 1 applies
// x += alpha p, z -= alpha P q with the starting p and q; 2 first advances
// p = z + beta p, q = w + beta q.  The element visit reads all its rows and element
// data before it writes any (see RowIn).

template <int MODE>
__device__ __forceinline__ void fused_row_load(const DevScene &S, int row, RowIn &v) {
  v.P = gld(S.row_P + row);
  v.z = gld(S.row_z + row);
  if (MODE == 0) return;
  v.p = gld(S.row_p + row);
  v.q = gld(S.row_q + row);
  v.x = gld(S.row_x + row);
  if (MODE == 2) v.w = gld(S.row_w + row);
}

// applies the update to the loaded values and stores them; returns z, q and P
template <int MODE>
__device__ __forceinline__ void fused_row(const DevScene &S, int row, const RowIn &v, float alpha, float beta,
                                          float &z, float &q, float &P) {
  P = v.P;
  if (MODE == 0) {
    z = v.z;
    q = 0.f;
    return;
  }
  float p = v.p;
  q = v.q;
  const float z0 = v.z;
  if (MODE == 2) {
    p = z0 + beta * p;
    q = v.w + beta * q;
    gst(S.row_p + row, p);
    gst(S.row_q + row, q);
  }
  gst(S.row_x + row, v.x + alpha * p);
  z = z0 - alpha * (P * q);
  gst(S.row_z + row, z);
}

// the product's row value w is stored (and, in the first visit, taken as q = A p0);
// returns P w, the value the element's contribution carries
template <int MODE>
__device__ __forceinline__ float fused_finish(const DevScene &S, int row, float z, float w, float P, float &q,
                                              double part[3]) {
  gst(S.row_w + row, w);
  if (MODE == 0) {
    gst(S.row_q + row, w);
    q = w;
  }
  mv_dots_reg(z, w, P, q, part);
  return P * w;
}

template <int BS, int MODE>
__device__ __forceinline__ void fused_visit(const Ctx &c, const float *Y, int buf, int nel, float eps, float alpha,
                                            float beta, double part[3]) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  // Visit slots: eight lanes per joint (one per row, two idle; a group never straddles
  // a wave), then the tets and contacts.  A joint's rows then cost one memory round
  // trip, like a tet's, instead of one per row on a single thread.
  const int nj = E.n_jnt;
  const int nv = nel + 7 * nj;
  for (int i = threadIdx.x; i < nv; i += BS) {
    if (i < 8 * nj) {
      const int jl = i >> 3, r = i & 7, jg = E.jnt_off + jl;
      const bool row = r < 6;
      const int rr = row ? r : 5;  // idle lanes read row 5 and write nothing
      const int r0 = row_joint(E, jl);
      const int4 info = gld(S.j_info + jg);
      RowIn v;
      fused_row_load<MODE>(S, r0 + rr, v);
      const float C = gld(S.row_C + r0 + rr);
      float Jr[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) Jr[k] = gld(S.j_J + (size_t)72 * jg + 12 * rr + k);
      float z = 0.f, q = 0.f, P = 0.f, pw = 0.f;
      if (row) fused_row<MODE>(S, r0 + r, v, alpha, beta, z, q, P);
      const int dB = ldof(E, info.z - E.rig_off);
      const int dA = info.y >= 0 ? ldof(E, info.y - E.rig_off) : -1;
      float jy = row_dot_rigid(Jr + 6, Y, dB);
      if (dA >= 0) jy += row_dot_rigid(Jr, Y, dA);
      if (row) {
        const float w = jy + C * z + eps * z;
        pw = fused_finish<MODE>(S, r0 + r, z, w, P, q, part);
      }
      // J^T (P w) of the joint, summed over its rows in row order as joint_contrib_vals
      // does, from the row lanes' values; the group's first lane stores it
      const int lead = (threadIdx.x & 63) & ~7;
      float o[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = 0.f;
#pragma unroll
      for (int rk = 0; rk < 6; ++rk) {
        const float pk = __shfl(pw, lead + rk, 64);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] += pk * __shfl(Jr[k], lead + rk, 64);
      }
      if (r == 0) joint_store_slots(S, jg, o);
      continue;
    }
    const int el = i - 7 * nj;
    if (el < E.n_jnt + E.n_tet) {
      const int tl = el - E.n_jnt, tg = E.tet_off + tl;
      const int r0 = row_tet(E, tl);
      float z[3], q[3], P[3], jy[3], pw[3];
      // ids and slots first (the Y reads wait for them), decoded after the other loads
      // are issued: from one 16-byte record of env-local 16-bit fields where the
      // scene's envs fit them, else from the two global index tables
      const bool packed = S.tet_loc != 0;
      uint4 L = make_uint4(0u, 0u, 0u, 0u);
      int4 ids = make_int4(0, 0, 0, 0), dst = ids;
      if (packed) {
        L = gld(S.t_loc + tg);
      } else {
        ids = gld(S.t_ids + tg);
        dst = gld(S.t_dst + tg);
      }
      RowIn v[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) fused_row_load<MODE>(S, r0 + r, v[r]);
      float J[18], Em[6];
#pragma unroll
      for (int m = 0; m < 18; ++m) J[m] = tJ(S, buf, m, tg);
#pragma unroll
      for (int k = 0; k < 6; ++k) Em[k] = gld(S.t_E + (size_t)k * S.NT + tg);
      if (packed) {
        const int po = E.par_off, ab = c.cl_base;
        ids = make_int4(po + (int)(L.x & 0xffffu), po + (int)(L.y & 0xffffu), po + (int)(L.z & 0xffffu),
                        po + (int)(L.w & 0xffffu));
        dst = make_int4(ab + (int)(L.x >> 16), ab + (int)(L.y >> 16), ab + (int)(L.z >> 16), ab + (int)(L.w >> 16));
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) fused_row<MODE>(S, r0 + r, v[r], alpha, beta, z[r], q[r], P[r]);
      tet_JY_core(E, J, ids, Y, jy);
      const V3 zz = mk(z[0], z[1], z[2]);
      const V3 cz = sym_mul(Em, zz);
      const float w0 = jy[0] + cz.x + eps * zz.x, w1 = jy[1] + cz.y + eps * zz.y, w2 = jy[2] + cz.z + eps * zz.z;
      pw[0] = fused_finish<MODE>(S, r0, z[0], w0, P[0], q[0], part);
      pw[1] = fused_finish<MODE>(S, r0 + 1, z[1], w1, P[1], q[1], part);
      pw[2] = fused_finish<MODE>(S, r0 + 2, z[2], w2, P[2], q[2], part);
      tet_contrib_core(c, J, pw, dst);
    } else {
      const int cl = el - E.n_jnt - E.n_tet, gc = E.con_off + cl;
      const int r0 = row_con(E, cl);
      float z[3], q[3], P[3], jy[3], pw[3], C[3];
      const int2 bd = gld(S.c_body + gc);  // first: the Y reads wait for it
      RowIn v[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        fused_row_load<MODE>(S, r0 + r, v[r]);
        C[r] = gld(S.row_C + r0 + r);
      }
      const V3 n = mk(gld(S.c_n + gc));
      const float al = gld(S.c_alpha + (size_t)buf * S.NC + gc);
      const int act = gld(S.c_active + (size_t)buf * S.NC + gc);
      const V3 rA = mk(gld(S.c_rA + gc)), rB = mk(gld(S.c_rB + gc));
#pragma unroll
      for (int r = 0; r < 3; ++r) fused_row<MODE>(S, r0 + r, v[r], alpha, beta, z[r], q[r], P[r]);
      contact_JY_core(c, Y, bd, n, rA, rB, al, act, jy);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const float w = jy[r] + C[r] * z[r] + eps * z[r];
        pw[r] = fused_finish<MODE>(S, r0 + r, z[r], w, P[r], q[r], part);
      }
      contact_store(S, gc, contact_dir_core(n, al, act, pw[0], pw[1], pw[2]), rA, rB);
    }
  }
}

// Body pass of the one-pass PCR: G = the summed contributions of the last visit.
// MODE 0: Bz = G (= J^T z0); 1: Bq = G, Bz -= alpha Bq; 2: Bq = G + beta Bq,
// Bz -= alpha Bq.  Then Y = H~^-1 Bz.  Residual replacement (kOnePassRefreshDrop):
// MODE 3 advances Bq only; after a contribution pass of the current z, MODE 4 re-forms
// Bz = G - alpha Bq from it (G = J^T z) and applies H~^-1.
template <int MODE>
__device__ __forceinline__ void fused_body(const Ctx &c, float *Y, float alpha, float beta, int tid, int BS) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  // slots: four lanes per rigid body (they share its gather), then one per particle
  const int nr4 = 4 * E.n_rig;
  const int nv = nr4 + E.n_par;
  for (int i = tid; i < nv; i += BS) {
    if (i < nr4) {
      const int b = i >> 2, g = E.rig_off + b;
      float v[6], oq[6], oz[6], Iw[6];
      const int d = E.dof_off + 6 * b;
      // every load before the first store (see fused_row_load), the body's own values
      // ahead of the gather's chains
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        oq[k] = MODE >= 2 ? gld(S.bq + d + k) : 0.f;
        oz[k] = MODE == 1 || MODE == 2 ? gld(S.bz + d + k) : 0.f;
        Iw[k] = MODE == 3 ? 0.f : gld(S.r_Iwinv + 6 * g + k);
      }
      const float im = MODE == 3 ? 0.f : gld(S.r_inertia + g).w;
      gather_rigid_lanes(S, g, i & 3, v);
      if ((i & 3) != 0) continue;  // the group's first lane finishes the body
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (MODE == 4) {
          v[k] = v[k] - alpha * oq[k];
        } else if (MODE > 0) {
          const float bq = MODE == 1 ? v[k] : v[k] + beta * oq[k];
          gst(S.bq + d + k, bq);
          if (MODE == 3) continue;
          v[k] = oz[k] - alpha * bq;
        }
        gst(S.bz + d + k, v[k]);
      }
      if (MODE == 3) continue;
      hinv_rigid_vals(im, Iw, v);
#pragma unroll
      for (int k = 0; k < 6; ++k) Y[6 * b + k] = v[k];
    } else {
      const int b = i - nr4 + E.n_rig;
      const int p = E.par_off + b - E.n_rig;
      float oq[3], oz[3];
      const int d = E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        oq[k] = MODE >= 2 ? gld(S.bq + d + k) : 0.f;
        oz[k] = MODE == 1 || MODE == 2 ? gld(S.bz + d + k) : 0.f;
      }
      const float4 H = MODE == 3 ? make_float4(1.f, 1.f, 1.f, 0.f) : gld(S.p_H + p);
      const V3 a = gather_particle(c, p);
      float v[3] = {a.x, a.y, a.z};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (MODE == 4) {
          v[k] = v[k] - alpha * oq[k];
        } else if (MODE > 0) {
          const float bq = MODE == 1 ? v[k] : v[k] + beta * oq[k];
          gst(S.bq + d + k, bq);
          if (MODE == 3) continue;
          v[k] = oz[k] - alpha * bq;
        }
        gst(S.bz + d + k, v[k]);
      }
      if (MODE == 3) continue;
      const int y = 6 * E.n_rig + 3 * (b - E.n_rig);
      Y[y] = v[0] / H.x;
      Y[y + 1] = v[1] / H.y;
      Y[y + 2] = v[2] / H.z;
    }
  }
}

__device__ __forceinline__ void update_positions_body(const Ctx &c, int b) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const float h = c.A.h;
  if (b < E.n_rig) {
    const int g = E.rig_off + b;
    if (S.r_inertia[g].w == 0.f) return;
    const float *u = S.r_u + 6 * g;
    const float4 x0 = S.r_x0[g];
    S.r_x[g] = make_float4(x0.x + h * u[0], x0.y + h * u[1], x0.z + h * u[2], 0.f);
    const float4 q = S.r_q[g], q0 = S.r_q0[g];
    // (1/2) Q(theta) omega, Q from Sec. 9 (rigid bodies)
    const float t1 = q.x, t2 = q.y, t3 = q.z, t4 = q.w, w1 = u[3], w2 = u[4], w3 = u[5];
    const float dq0 = -t2 * w1 - t3 * w2 - t4 * w3;
    const float dq1 = t1 * w1 + t4 * w2 - t3 * w3;
    const float dq2 = -t4 * w1 + t1 * w2 + t2 * w3;
    const float dq3 = t3 * w1 - t2 * w2 + t1 * w3;
    S.r_q[g] = quat_normalize(make_float4(q0.x + 0.5f * h * dq0, q0.y + 0.5f * h * dq1, q0.z + 0.5f * h * dq2,
                                          q0.w + 0.5f * h * dq3));
  } else {
    const int p = E.par_off + b - E.n_rig;
    const float4 x0 = S.p_x0[p], u = S.p_u[p];
    S.p_x[p] = make_float4(x0.x + h * u.x, x0.y + h * u.y, x0.z + h * u.z, 0.f);
  }
}

// the env's iterate (multipliers, velocities, positions) into / out of the best slot
__device__ __forceinline__ void keep_best(const Ctx &c, int nrows, bool restore) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int nb = E.n_rig + E.n_par;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
    const int row = E.row_off + r;
    if (restore) S.row_lam[row] = S.row_lam_best[row];
    else S.row_lam_best[row] = S.row_lam[row];
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    if (b < E.n_rig) {
      const int g = E.rig_off + b;
      float *u = S.r_u + 6 * g, *ub = S.r_u_best + 6 * g;
      for (int k = 0; k < 6; ++k) {
        if (restore) u[k] = ub[k];
        else ub[k] = u[k];
      }
      if (restore) { S.r_x[g] = S.r_x_best[g]; S.r_q[g] = S.r_q_best[g]; }
      else { S.r_x_best[g] = S.r_x[g]; S.r_q_best[g] = S.r_q[g]; }
    } else {
      const int p = E.par_off + b - E.n_rig;
      if (restore) { S.p_u[p] = S.p_u_best[p]; S.p_x[p] = S.p_x_best[p]; }
      else { S.p_u_best[p] = S.p_u[p]; S.p_x_best[p] = S.p_x[p]; }
    }
  }
}

// back to q^- (the rerun of a failed warm start)
__device__ __forceinline__ void restore_positions_body(const Ctx &c, int b) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  if (b < E.n_rig) {
    const int g = E.rig_off + b;
    if (S.r_inertia[g].w == 0.f) return;
    S.r_x[g] = S.r_x0[g];
    S.r_q[g] = S.r_q0[g];
  } else {
    const int p = E.par_off + b - E.n_rig;
    S.p_x[p] = S.p_x0[p];
  }
}

template <int BS, bool EXT>
__device__ __forceinline__ void assemble_all(const Ctx &c, int buf, double tplus, int nc) {
  const EnvInfo &E = c.E;
  const int nel = E.n_jnt + E.n_tet + nc;
  for (int el = threadIdx.x; el < nel; el += BS) {
    if (el < E.n_jnt) assemble_joint(c, el, tplus);
    else if (el < E.n_jnt + E.n_tet) assemble_tet<EXT>(c, el - E.n_jnt, buf, false);
    else assemble_contact(c, el - E.n_jnt - E.n_tet, buf);
  }
}

// --------------------------------------------------------------------------
// Islands (option; Sec. 11 names them as the remedy for the Krylov scalars one PCR
// shares over all the bodies of an env).  An island is the dynamic bodies connected
// through joints, tets and contacts (static bodies and the world connect nothing),
// named by its lowest env-local body index; an element belongs to the island of its
// dynamic body (joints: B before A; contacts: the feature body before the target),
// elements without one to the static group n_rig + n_par.  A is block diagonal over
// islands, so each island runs its own PCR with its own scalars and stop.
// --------------------------------------------------------------------------
// labels and counters change through atomics (performed in L2): read them coherently
__device__ __forceinline__ int ld_coherent(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// an island already solved in residual mode (its residual at or below tol)
__device__ __forceinline__ bool island_solved(const Ctx &c, int ib, int k) {
  return c.A.tol > 0.f && __int_as_float(ld_coherent(c.S.isl_res + ib + k)) <= c.A.tol;
}

// rows of element el: first row and count
__device__ __forceinline__ void el_rows(const EnvInfo &E, int el, int &r0, int &nr) {
  if (el < E.n_jnt) { r0 = row_joint(E, el); nr = 6; }
  else if (el < E.n_jnt + E.n_tet) { r0 = row_tet(E, el - E.n_jnt); nr = tet_nrows(E); }
  else { r0 = row_con(E, el - E.n_jnt - E.n_tet); nr = 3; }
}

__device__ __forceinline__ bool body_dyn(const Ctx &c, int b) {
  return b >= 0 && (b >= c.E.n_rig || c.S.r_inertia[c.E.rig_off + b].w != 0.f);
}

// env-local bodies an element unites (joints and contacts: only when both are dynamic)
__device__ __forceinline__ int unite_bodies(const Ctx &c, int el, int bd[4]) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  if (el < E.n_jnt) {
    const int4 info = S.j_info[E.jnt_off + el];
    const int a = info.y >= 0 ? info.y - E.rig_off : -1, b = info.z - E.rig_off;
    if (!body_dyn(c, a) || !body_dyn(c, b)) return 0;
    bd[0] = a; bd[1] = b;
    return 2;
  }
  if (el < E.n_jnt + E.n_tet) {
    const int4 id = S.t_ids[E.tet_off + el - E.n_jnt];
    bd[0] = E.n_rig + id.x - E.par_off; bd[1] = E.n_rig + id.y - E.par_off;
    bd[2] = E.n_rig + id.z - E.par_off; bd[3] = E.n_rig + id.w - E.par_off;
    return 4;
  }
  const int2 cb = S.c_body[E.con_off + el - E.n_jnt - E.n_tet];
  if (!body_dyn(c, cb.x) || !body_dyn(c, cb.y)) return 0;
  bd[0] = cb.x; bd[1] = cb.y;
  return 2;
}

__device__ __forceinline__ int element_island(const Ctx &c, int el, const int *lab) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int nb = E.n_rig + E.n_par;
  if (el < E.n_jnt) {
    const int4 info = S.j_info[E.jnt_off + el];
    const int a = info.y >= 0 ? info.y - E.rig_off : -1, b = info.z - E.rig_off;
    return body_dyn(c, b) ? ld_coherent(lab + b) : (body_dyn(c, a) ? ld_coherent(lab + a) : nb);
  }
  if (el < E.n_jnt + E.n_tet) return ld_coherent(lab + E.n_rig + S.t_ids[E.tet_off + el - E.n_jnt].x - E.par_off);
  const int2 cb = S.c_body[E.con_off + el - E.n_jnt - E.n_tet];
  return body_dyn(c, cb.x) ? ld_coherent(lab + cb.x) : (body_dyn(c, cb.y) ? ld_coherent(lab + cb.y) : nb);
}

// Island of every body and element, and the elements grouped by island in element
// order (el_perm, isl_off); the non-empty islands in isl_list.  Once per step.
template <int BS>
__device__ void island_setup(const Ctx &c, int e, int nel, Red<BS> &red) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int tid = threadIdx.x;
  const int nb = E.n_rig + E.n_par;
  const int eb = E.jnt_off + E.tet_off + E.con_off, ib = E.rig_off + E.par_off + 2 * e;
  int *lab = S.b_lab + E.rig_off + E.par_off;
  for (int b = tid; b < nb; b += BS) lab[b] = body_dyn(c, b) ? b : -1;
  for (int k = tid; k < nb + 2; k += BS) {
    S.isl_cnt[ib + k] = 0;
    S.isl_run[ib + k] = 0;
  }
  __syncthreads();
  // Minimum-label propagation with pointer jumping.  Labels only fall and always name
  // a body of the same island; the fixed point (every uniting element's bodies share a
  // label that labels itself) names each island by its lowest body.  Each round moves
  // the minimum at least one edge further, so nb + 1 rounds reach it.
  for (int round = 0; round <= nb + 1; ++round) {
    float changed = 0.f;
    for (int el = tid; el < nel; el += BS) {
      int bd[4];
      const int n = unite_bodies(c, el, bd);
      if (n < 2) continue;
      int m = ld_coherent(lab + bd[0]);
      for (int i = 1; i < n; ++i) m = min(m, ld_coherent(lab + bd[i]));
      for (int i = 0; i < n; ++i)
        if (atomicMin(&lab[bd[i]], m) > m) changed = 1.f;
    }
    __syncthreads();
    for (int b = tid; b < nb; b += BS) {
      const int l = ld_coherent(lab + b);
      if (l >= 0) {
        const int l2 = ld_coherent(lab + l);
        if (l2 < l && atomicMin(&lab[b], l2) > l2) changed = 1.f;
      }
    }
    if (block_max<BS>(changed, red, 0) == 0.f) break;
    __syncthreads();
  }
  __syncthreads();
  for (int el = tid; el < nel; el += BS) {
    const int k = element_island(c, el, lab);
    S.el_isl[eb + el] = k;
    atomicAdd(&S.isl_cnt[ib + k], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int off = 0, K = 0;
    for (int k = 0; k <= nb; ++k) {
      S.isl_off[ib + k] = off;
      const int n = ld_coherent(S.isl_cnt + ib + k);
      if (n > 0) S.isl_list[ib + K++] = k;
      off += n;
    }
    S.isl_off[ib + nb + 1] = off;
    S.isl_n[e] = K;
  }
  __syncthreads();
  // stable grouping: the first wave walks the elements in order, 64 at a time; a
  // lane's place is its island's start + the island's count so far + the lanes before
  // it with the same island (the count is advanced atomically by the last such lane)
  if (tid < 64) {
    for (int base = 0; base < nel; base += 64) {
      const int el = base + tid;
      const int k = el < nel ? S.el_isl[eb + el] : -1;
      int rank = 0, last = 0;
      for (int j = 0; j < 64; ++j) {
        const int kj = __shfl(k, j, 64);
        if (kj == k) {
          if (j < tid) ++rank;
          last = j;
        }
      }
      int old = 0;
      if (k >= 0 && tid == last) old = atomicAdd(&S.isl_run[ib + k], rank + 1);
      old = __shfl(old, last, 64);
      if (k >= 0) S.el_perm[eb + S.isl_off[ib + k] + old + rank] = el;
    }
  }
  __syncthreads();
}

// One wave per island: its three dots summed in element order (fixed, deterministic),
// then its scalars.  first: the start of the PCR (rho = <z,w>, <q,Pq> = <w,Pw>,
// beta = 0); returns the thread's part of the env's start sum of rho.  Else the
// single-reduction recurrences of an active island, followed by island_check.
template <int BS>
__device__ double island_reduce(const Ctx &c, int e, bool first) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int eb = E.jnt_off + E.tet_off + E.con_off, ib = E.rig_off + E.par_off + 2 * e;
  const int K = S.isl_n[e];
  double rho0 = 0.0;
  for (int i = w; i < K; i += BS / 64) {
    const int k = S.isl_list[ib + i];
    const int o0 = S.isl_off[ib + k], o1 = S.isl_off[ib + k + 1];
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int q = o0 + lane; q < o1; q += 64) {
      const double *d = S.el_dots + 3 * (size_t)(eb + S.el_perm[eb + q]);
      d0 += d[0];
      d1 += d[1];
      d2 += d[2];
    }
    d0 = wave_sum(d0);
    d1 = wave_sum(d1);
    d2 = wave_sum(d2);
    if (lane == 0) {
      IslState I = S.isl[ib + k];
      if (first) {
        I.rho = d0;
        I.qs = d1;
        I.beta = 0.f;
        I.active = 1;
        rho0 += d0;
      } else if (I.active) {
        const double b = d0 / I.rho;
        I.qs = d1 + 2.0 * b * d2 + b * b * I.qs;
        I.beta = (float)b;
        I.rho = d0;
      }
      S.isl[ib + k] = I;
    }
  }
  return rho0;
}

// The check at the top of every PCR iteration, per island (its owner lane): rho above
// the stop level and positive, <q,Pq> positive; then alpha = rho / <q,Pq>.  stop >= 0:
// first call, sets every island's stop level (READING: TAU_CR times the env's start
// rho, the rounding level of the whole system, as in the whole-env PCR).  Returns 1 on
// a lane that saw an active island, else 0.
template <int BS>
__device__ float island_check(const Ctx &c, int e, double stop) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ib = E.rig_off + E.par_off + 2 * e;
  const int K = S.isl_n[e];
  float any = 0.f;
  if (lane != 0) return any;
  for (int i = w; i < K; i += BS / 64) {
    const int k = S.isl_list[ib + i];
    IslState I = S.isl[ib + k];
    if (stop >= 0.0) {
      I.stop = stop;
      if (island_solved(c, ib, k)) I.active = 0;  // READING: early exit of a solved island
    }
    if (I.active) I.active = (I.rho > I.stop) && (I.rho > 0.0) && (I.qs > 0.0);
    if (I.active) {
      I.alpha = (float)(I.rho / I.qs);
      any = 1.f;
    }
    S.isl[ib + k] = I;
  }
  return any;
}

// Residual of every island (the same max(|M~^-1 g|, |err|) as the env's, over the
// island's bodies and rows), for the early exit of solved islands in residual mode.
// Maxima of non-negative floats through integer atomics: independent of the order.
template <int BS>
__device__ void island_residuals(const Ctx &c, int e, int nel) {
  const EnvInfo &E = c.E;
  const DevScene &S = c.S;
  const int tid = threadIdx.x;
  const int nb = E.n_rig + E.n_par;
  const int eb = E.jnt_off + E.tet_off + E.con_off, ib = E.rig_off + E.par_off + 2 * e;
  const int *lab = S.b_lab + E.rig_off + E.par_off;
  for (int k = tid; k < nb + 2; k += BS) S.isl_res[ib + k] = 0;
  __syncthreads();
  for (int b = tid; b < nb; b += BS) {
    const int l = ld_coherent(lab + b);
    if (l < 0) continue;
    float r = 0.f;
    if (b < E.n_rig) {
      const int g = E.rig_off + b;
      const int d = E.dof_off + 6 * b;
      const float im = S.r_inertia[g].w;
      const V3 ia = sym_mul(S.r_Iwinv + 6 * g, mk(S.g[d + 3], S.g[d + 4], S.g[d + 5]));
      r = fmaxf(fmaxf(fabsf(S.g[d] * im), fabsf(S.g[d + 1] * im)), fabsf(S.g[d + 2] * im));
      r = fmaxf(r, fmaxf(fmaxf(fabsf(ia.x), fabsf(ia.y)), fabsf(ia.z)));
    } else {
      const int p = E.par_off + b - E.n_rig;
      const int d = E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
      const float m = S.p_m[p];
      r = fmaxf(fmaxf(fabsf(S.g[d] / m), fabsf(S.g[d + 1] / m)), fabsf(S.g[d + 2] / m));
    }
    atomicMax(S.isl_res + ib + l, __float_as_int(r));
  }
  for (int el = tid; el < nel; el += BS) {
    int r0, nr;
    el_rows(E, el, r0, nr);
    float r = 0.f;
    for (int q = 0; q < nr; ++q) r = fmaxf(r, fabsf(S.row_err[r0 + q]));
    atomicMax(S.isl_res + ib + S.el_isl[eb + el], __float_as_int(r));
  }
  __syncthreads();
}

// --------------------------------------------------------------------------
// Kernel 3: start iterate + Newton loop + write-back.  One workgroup per env.
// --------------------------------------------------------------------------
// LM: 0 body-space vector in global memory, 1 in LDS, 2 in LDS together with the tets'
// contributions
template <int BS, int LM, bool EXT, int R>
__global__ __launch_bounds__(BS) void k_newton(const DevScene *__restrict__ Sp, StepArgs A, int first) {
  __shared__ Red<BS> red;
  extern __shared__ float y_lds[];
  const unsigned long long t_start = wall_clock64();
  const DevScene &S = *Sp;
  const int e = S.env_order[first + blockIdx.x];
  Ctx c(S, uniform_env(S.env[e]), A);
  const EnvInfo &E = c.E;
  const int tid = threadIdx.x;
  const float h = A.h;
  const float damp = A.p.damping, eps = A.p.eps;
  const int nc = sgpr(S.n_con[e]);
  const int nb = E.n_rig + E.n_par;
  const int nel = E.n_jnt + E.n_tet + nc;
  const int nrows = 6 * E.n_jnt + tet_nrows(E) * E.n_tet + 3 * nc;
  const int R0 = E.row_off;
  // island mode: one PCR per island (the extended instantiation only)
  const bool isl_mode = EXT && A.p.islands && A.p.linear == NSN_LINEAR_PCR;
  if (isl_mode) island_setup<BS>(c, e, nel, red);
  const int crow0 = row_con(E, 0);
  const double tplus = S.time[e] + (double)h;
  // env-local body-space vector: in LDS when the bucket's envs fit, else in global memory
  float *Y = LM > 0 ? y_lds : S.y + E.dof_off;
  c.cl_base = sgpr(S.p_tadj_ptr[E.par_off]);  // the env's first particle-list entry
  if (LM == 2) {
    c.cl = y_lds + ((E.n_dof + 3) & ~3);
    c.cl_n = 4 * E.n_tet;
  }

  // ---- start iterate (Sec. 8.1); READING for warm starts: projected lambda0 for
  //      contacts, the previous multipliers for joints, the start-configuration
  //      stress for tets, and u0 = u^- (the previous step's velocity) ----
  int newton_done = 0, cr_total = 0, nonfinite = 0, converged = 0, fallback = 0, watchdog = 0;
  float r_ncp = 0.f, r_con = 0.f, r_first = 0.f;
  double merit = 0.0;
  // READING (recovery, not in the paper): a warm-started step whose iterate turns
  // non-finite is rerun from the plain start u0 = 0, lambda0 = 0 at q^-; the work of
  // both attempts is counted.  nonfinite is block-uniform (a block reduction).
  for (int attempt = 0; attempt < 2; ++attempt) {
  const bool warm = attempt == 0 && A.p.warm != NSN_WARM_ZERO;
  if (attempt == 1) {
    for (int b = tid; b < nb; b += BS) restore_positions_body(c, b);
    nonfinite = 0;
    fallback = 1;
    __syncthreads();
  }
  // Option (Sec. 8.1 names watchdog strategies without using one; off by default, as
  // in the paper): the step keeps its lowest-merit iterate; when the merit grows past
  // kWatchBlowup times that best, or turns non-finite outside a warm attempt, the
  // iteration stops and the step returns the best iterate.  All the quantities
  // deciding this are block-uniform.
  double best_merit = __builtin_huge_val();
  float best_r = 0.f, best_rc = 0.f;
  bool have_best = false, restore = false;
  // Sec. 8.1 (optional globalisation, READING of the details): with line search on,
  // the full step is tried first; while the merit at the trial point exceeds
  // (1 - kLsSigma t) times the accepted iterate's, t is halved down to kLsTmin (then
  // accepted).  Trial points are evaluated like iterates but are not Newton iterations.
  float ls_t = 1.f;
  double merit_k = __builtin_huge_val();
  for (int r = tid; r < nrows; r += BS) {
    const int row = R0 + r;
    if (!warm) {
      S.row_lam[row] = 0.f;
    } else if (row >= crow0) {
      const int cl = (row - crow0) / 3, k = (row - crow0) - 3 * cl;
      float4 l = S.c_lam0[E.con_off + cl];
      if (!(l.x == l.x) || !(l.y == l.y) || !(l.z == l.z)) l = make_float4(0.f, 0.f, 0.f, 0.f);
      const float ln = fmaxf(l.x, 0.f);
      const float lf = sqrtf(l.y * l.y + l.z * l.z), lim = E.mu * ln;
      const float sc = lf > lim ? (lf > 0.f ? lim / lf : 0.f) : 1.f;
      S.row_lam[row] = k == 0 ? ln : (k == 1 ? l.y * sc : l.z * sc);
    }
  }
  for (int b = tid; b < nb; b += BS) {
    if (b < E.n_rig) {
      const int g = E.rig_off + b;
      float *u = S.r_u + 6 * g;
      const bool mv = warm && S.r_inertia[g].w != 0.f;  // static bodies stay at rest
      const float4 v = S.r_v[g], w = S.r_w[g];
      u[0] = mv ? v.x : 0.f; u[1] = mv ? v.y : 0.f; u[2] = mv ? v.z : 0.f;
      u[3] = mv ? w.x : 0.f; u[4] = mv ? w.y : 0.f; u[5] = mv ? w.z : 0.f;
    } else {
      const int p = E.par_off + b - E.n_rig;
      const float4 v = S.p_v[p];
      S.p_u[p] = warm ? make_float4(v.x, v.y, v.z, 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
      S.p_uprev[p] = make_float4(0.f, 0.f, 0.f, 0.f);
      S.p_H[p] = make_float4(S.p_m[p], S.p_m[p], S.p_m[p], 0.f);
    }
  }
  if (warm) {
    for (int t = tid; t < E.n_tet; t += BS) assemble_tet<EXT>(c, t, 0, true);  // stress at q^-
    __syncthreads();
    for (int b = tid; b < nb; b += BS) update_positions_body(c, b);
  }
  __syncthreads();

  for (int k = 0; k <= A.newton_iters; ++k) {
    const int buf = k & 1;
    // dump step: keep iterate k-1 in the watchdog's slot (the watchdog is off)
    if (A.dump_k >= 1 && k == A.dump_k - 1) {
      keep_best(c, nrows, false);
      __syncthreads();
    }
    assemble_all<BS, EXT>(c, buf, tplus, nc);
    __syncthreads();
    // momentum balance g = M~(u - u~) - h J^T lambda (Sec. 6.1); geometric stiffness
    // (Sec. 8.3, READING: secant of J^T lambda at fixed lambda between the last two
    // iterates, particle DOFs only)
    float rg = 0.f;
    double m2 = 0.0;
    contrib_pass<BS, EXT>(c, S.row_lam, buf, nel, true);
    __syncthreads();
    const bool secant = A.p.geo_stiff && k >= 1;
    for (int b = tid; b < nb; b += BS) {
      if (b < E.n_rig) {
        const int g = E.rig_off + b;
        const int d = E.dof_off + 6 * b;
        const float im = S.r_inertia[g].w;
        if (im == 0.f) {
          for (int q = 0; q < 6; ++q) S.g[d + q] = 0.f;
          continue;
        }
        float f6[6];
        gather_rigid(c, g, f6);
        const float *u = S.r_u + 6 * g, *ut = S.r_ut + 6 * g;
        const V3 dv = mk(u[0] - ut[0], u[1] - ut[1], u[2] - ut[2]);
        const V3 dw = sym_mul(S.r_Iw + 6 * g, mk(u[3] - ut[3], u[4] - ut[4], u[5] - ut[5]));
        const float m = 1.f / im;
        float gv[6] = {m * dv.x - h * f6[0], m * dv.y - h * f6[1], m * dv.z - h * f6[2],
                       dw.x - h * f6[3], dw.y - h * f6[4], dw.z - h * f6[5]};
        const V3 ia = sym_mul(S.r_Iwinv + 6 * g, mk(gv[3], gv[4], gv[5]));
        rg = fmaxf(rg, fmaxf(fmaxf(fabsf(gv[0] * im), fabsf(gv[1] * im)), fabsf(gv[2] * im)));
        rg = fmaxf(rg, fmaxf(fmaxf(fabsf(ia.x), fabsf(ia.y)), fabsf(ia.z)));
        for (int q = 0; q < 6; ++q) {
          S.g[d + q] = gv[q];
          m2 += (double)gv[q] * (double)gv[q];
        }
      } else {
        const int p = E.par_off + b - E.n_rig;
        const int d = E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
        const V3 f = gather_particle(c, p);
        const float m = S.p_m[p];
        const float4 u = S.p_u[p], ut = S.p_ut[p];
        const V3 gv = mk(m * (u.x - ut.x) - h * f.x, m * (u.y - ut.y) - h * f.y, m * (u.z - ut.z) - h * f.z);
        if (secant) {
          S.f[d] = f.x; S.f[d + 1] = f.y; S.f[d + 2] = f.z;
        } else {
          S.p_H[p] = make_float4(m, m, m, 0.f);
        }
        S.g[d] = gv.x; S.g[d + 1] = gv.y; S.g[d + 2] = gv.z;
        rg = fmaxf(rg, fmaxf(fmaxf(fabsf(gv.x / m), fabsf(gv.y / m)), fabsf(gv.z / m)));
        m2 += (double)gv.x * gv.x + (double)gv.y * gv.y + (double)gv.z * gv.z;
      }
    }
    if (secant) {
      // the same forces with the previous iterate's Jacobians (particles only)
      __syncthreads();
      contrib_pass<BS, EXT>(c, S.row_lam, buf ^ 1, nel, false);
      __syncthreads();
      for (int b = E.n_rig + tid; b < nb; b += BS) {
        const int p = E.par_off + b - E.n_rig;
        const int d = E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
        const V3 fh = gather_particle(c, p);
        const float m = S.p_m[p];
        const float4 u = S.p_u[p], up = S.p_uprev[p];
        const float du[3] = {u.x - up.x, u.y - up.y, u.z - up.z};
        const float df[3] = {S.f[d] - fh.x, S.f[d + 1] - fh.y, S.f[d + 2] - fh.z};
        float hh[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float cj = h * df[a] * du[a] / (du[a] * du[a] + kTauGS * kTauGS);
          hh[a] = m - (cj < 0.f ? cj : 0.f);
        }
        S.p_H[p] = make_float4(hh[0], hh[1], hh[2], 0.f);
      }
    }
    float re = 0.f, rc = 0.f;
    for (int r = tid; r < nrows; r += BS) {
      const float ev = S.row_err[R0 + r];
      const float a = fabsf(ev);
      re = fmaxf(re, a);
      if (R0 + r >= crow0) rc = fmaxf(rc, a);
      m2 += (double)ev * ev;
    }
    // residual (READING: r_ncp = max(|M~^-1 g|_inf, |err|_inf)), merit |[g; err]|_2 in FP64
    const float rmax = block_max<BS>(fmaxf(rg, re), red, 0);
    const float rcon = block_max<BS>(rc, red, 1);
    const double msum = block_sum<BS>(m2, red, 0);
    r_ncp = rmax;
    r_con = rcon;
    merit = sqrt(msum);
    if (k == 0) r_first = rmax;
    const bool finite_now = rmax == rmax && !isinf(rmax) && msum == msum && !isinf(msum);
    if (EXT && isl_mode && A.tol > 0.f) island_residuals<BS>(c, e, nel);
    if (A.p.line_search && k > 0 && ls_t > kLsTmin &&
        (!finite_now || merit > (1.0 - kLsSigma * (double)ls_t) * merit_k)) {
      ls_t *= 0.5f;
      for (int r = tid; r < nrows; r += BS) S.row_lam[R0 + r] = S.row_lam_k[R0 + r] + ls_t * S.row_x[R0 + r];
      for (int b = tid; b < nb; b += BS) {
        if (b < E.n_rig) {
          const int g = E.rig_off + b;
          if (S.r_inertia[g].w == 0.f) continue;
          float *u = S.r_u + 6 * g;
          const float *uk = S.r_u_k + 6 * g, *dv = S.du + E.dof_off + 6 * b;
          for (int q = 0; q < 6; ++q) u[q] = uk[q] + ls_t * dv[q];
          S.r_q[g] = S.r_q_k[g];  // positions from G(q^k)
        } else {
          const int p = E.par_off + b - E.n_rig;
          const float *dv = S.du + E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
          const float4 uk = S.p_uprev[p];
          S.p_u[p] = make_float4(uk.x + ls_t * dv[0], uk.y + ls_t * dv[1], uk.z + ls_t * dv[2], 0.f);
        }
        update_positions_body(c, b);
      }
      __syncthreads();
      --k;
      continue;
    }
    if (A.p.watchdog && finite_now && merit < best_merit) {
      best_merit = merit;
      best_r = rmax;
      best_rc = rcon;
      have_best = true;
      keep_best(c, nrows, false);
    }
    if (!finite_now) {
      if (!A.p.watchdog || warm || !have_best) { nonfinite = 1; break; }
      restore = true;
      break;
    }
    if (A.p.watchdog && merit > kWatchBlowup * best_merit) { restore = true; break; }
    if (A.tol > 0.f && rmax <= A.tol) { converged = 1; break; }
    if (k == A.newton_iters) break;

    // Schur right-hand side b = (1/h)(J H~^-1 g - err) and Jacobi preconditioner
    // P = 1/(J H~^-1 J^T + C + eps)_ii (Sec. 6.2, 8.2, 8.4)
    for (int b = tid; b < nb; b += BS) {
      if (b < E.n_rig) {
        const int g = E.rig_off + b;
        const int d = E.dof_off + 6 * b;
        float v[6];
        for (int q = 0; q < 6; ++q) v[q] = S.g[d + q];
        hinv_rigid(c, g, v);
        for (int q = 0; q < 6; ++q) Y[6 * b + q] = v[q];
      } else {
        const int p = E.par_off + b - E.n_rig;
        const int d = E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
        const int dl = 6 * E.n_rig + 3 * (b - E.n_rig);
        const float4 H = S.p_H[p];
        Y[dl] = S.g[d] / H.x; Y[dl + 1] = S.g[d + 1] / H.y; Y[dl + 2] = S.g[d + 2] / H.z;
      }
    }
    __syncthreads();
    rhs_and_precond<BS, EXT>(c, Y, buf, nel, eps);
    __syncthreads();

    // ---- preconditioned conjugate residual (Sec. 8.2), x0 = 0, FP64 scalars ----
    // per iteration: [p = z + beta p, q = w + beta q, s = P q, <q,s>] -> element pass:
    // x += alpha p, z -= alpha s, J^T z per element -> body pass: Y = H~^-1 (sum) ->
    // element pass: w = J Y + C z + eps z, <z,w>
    int done = 0;
    if (A.p.linear == NSN_LINEAR_PCG) {
      // ---- preconditioned conjugate gradient (the comparison solver), x0 = 0 ----
      // storage: direction d in row_z (so that the contribution and matvec passes
      // apply A to it), residual r in row_p, A d in row_w
      double rz = 0.0;
      for (int r = tid; r < nrows; r += BS) {
        const int row = R0 + r;
        const float rv = S.row_b[row], zv = S.row_P[row] * rv;
        S.row_x[row] = 0.f;
        S.row_p[row] = rv;
        S.row_z[row] = zv;
        rz += (double)rv * (double)zv;
      }
      rz = block_sum<BS>(rz, red, 0);
      const double rz_stop = kTauCR * rz;
      for (int it = 0; it < A.cr_iters; ++it) {
        if (!(rz > rz_stop) || !(rz > 0.0)) break;
        contrib_pass<BS, EXT>(c, S.row_z, buf, nel, true);
        __syncthreads();
        gather_hinv(c, Y, tid, BS);
        __syncthreads();
        double dots[3] = {0.0, 0.0, 0.0};
        matvec_rows<BS, false, EXT>(c, Y, buf, nel, eps, dots);
        block_sum3<BS>(dots, red);
        if (it == 0 && k == A.dump_k)
          for (int r = tid; r < nrows; r += BS) S.row_dump[R0 + r] = S.row_w[R0 + r];
        const double pw = dots[0];
        if (!(pw > 0.0)) break;
        const float alpha = (float)(rz / pw);
        ++done;
        double part = 0.0;
        for (int r = tid; r < nrows; r += BS) {
          const int row = R0 + r;
          S.row_x[row] += alpha * S.row_z[row];
          const float rv = S.row_p[row] - alpha * S.row_w[row];
          S.row_p[row] = rv;
          part += (double)rv * (double)(S.row_P[row] * rv);
        }
        const double rz_new = block_sum<BS>(part, red, 1);
        if (it == A.cr_iters - 1) break;
        const float beta = (float)(rz_new / rz);
        rz = rz_new;
        for (int r = tid; r < nrows; r += BS) {
          const int row = R0 + r;
          S.row_z[row] = S.row_P[row] * S.row_p[row] + beta * S.row_z[row];
        }
        __syncthreads();
      }
    } else if (EXT && isl_mode) {
      // ---- one PCR per island: the single-reduction recurrences below with each
      //      island's own scalars and stop; done counts the iterations in which some
      //      island was active (the largest island count) ----
      const int ib = E.rig_off + E.par_off + 2 * e, eb = E.jnt_off + E.tet_off + E.con_off;
      pcr_update_contrib<BS, true, EXT>(c, buf, nel, 0.f, 0.f, false);
      __syncthreads();
      gather_hinv(c, Y, tid, BS);
      __syncthreads();
      double dots[3] = {0.0, 0.0, 0.0};
      matvec_rows<BS, true, EXT>(c, Y, buf, nel, eps, dots, true);
      __syncthreads();
      if (k == A.dump_k)
        for (int r = tid; r < nrows; r += BS) S.row_dump[R0 + r] = S.row_w[R0 + r];
      const double rho_env = block_sum<BS>(island_reduce<BS>(c, e, true), red, 0);
      float any = block_max<BS>(island_check<BS>(c, e, kTauCR * rho_env), red, 1);
      for (int it = 0; it < A.cr_iters; ++it) {
        if (any == 0.f) break;
        ++done;
        if (it == A.cr_iters - 1) {  // the last update needs no further product
          for (int el = tid; el < nel; el += BS) {
            const IslState &I = S.isl[ib + S.el_isl[eb + el]];
            if (!I.active) continue;
            int r0, nr;
            el_rows(E, el, r0, nr);
            for (int r = 0; r < nr; ++r) {
              const int row = r0 + r;
              const float p = it > 0 ? S.row_z[row] + I.beta * S.row_p[row] : S.row_p[row];
              S.row_x[row] += I.alpha * p;
            }
          }
          break;
        }
        pcr_update_contrib<BS, false, EXT>(c, buf, nel, 0.f, 0.f, it > 0, true, ib);
        __syncthreads();
        gather_hinv(c, Y, tid, BS);
        __syncthreads();
        matvec_rows<BS, false, EXT>(c, Y, buf, nel, eps, dots, true);
        __syncthreads();
        (void)island_reduce<BS>(c, e, false);
        any = block_max<BS>(island_check<BS>(c, e, -1.0), red, 1);
      }
    } else {
      bool resident = false;
      if constexpr (!EXT && R > 0) {
        // register-resident form where every element of the env has a register slot
        if (nel <= R * BS) {
          done = pcr_resident<BS, R>(c, Y, buf, nel, eps, A.cr_iters, k == A.dump_k, red);
          resident = true;
        }
      }
      if constexpr (!EXT && R < 0) {
        // one-pass form (fused_visit / fused_body)
        pcr_update_contrib<BS, true, EXT>(c, buf, nel, 0.f, 0.f, false);  // z0 = P b, x = 0, p = z0; J^T z0
        __syncthreads();
        fused_body<0>(c, Y, 0.f, 0.f, tid, BS);
        __syncthreads();
        double dots[3] = {0.0, 0.0, 0.0};
        fused_visit<BS, 0>(c, Y, buf, nel, eps, 0.f, 0.f, dots);
        block_sum3<BS>(dots, red);
        if (k == A.dump_k)
          for (int r = tid; r < nrows; r += BS) S.row_dump[R0 + r] = S.row_w[R0 + r];
        double rho = dots[0], qs = dots[1];
        const double rho_stop = kTauCR * rho;
        double rho_ref = rho;  // rho when Bz was last formed from the rows
        float beta = 0.f;
        for (int it = 0; it < A.cr_iters; ++it) {
          if (!(rho > rho_stop) || !(rho > 0.0)) break;
          if (!(qs > 0.0)) break;
          const float alpha = (float)(rho / qs);
          ++done;
          if (it == A.cr_iters - 1) {  // the last update needs no further product
            last_x_update<BS>(S, R0, nrows, tid, it > 0, alpha, beta);
            break;
          }
          if (it == 0) {
            fused_body<1>(c, Y, alpha, beta, tid, BS);
          } else if (rho <= kOnePassRefreshDrop * rho_ref) {  // residual replacement of Bz
            rho_ref = rho;
            fused_body<3>(c, Y, alpha, beta, tid, BS);
            __syncthreads();
            contrib_pass<BS, EXT>(c, S.row_z, buf, nel, true);  // J^T z of the current z
            __syncthreads();
            fused_body<4>(c, Y, alpha, beta, tid, BS);
          } else {
            fused_body<2>(c, Y, alpha, beta, tid, BS);
          }
          __syncthreads();
          dots[0] = dots[1] = dots[2] = 0.0;
          if (it == 0) fused_visit<BS, 1>(c, Y, buf, nel, eps, alpha, beta, dots);
          else fused_visit<BS, 2>(c, Y, buf, nel, eps, alpha, beta, dots);
          block_sum3<BS>(dots, red);
          const double b = dots[0] / rho;
          qs = dots[1] + 2.0 * b * dots[2] + b * b * qs;
          beta = (float)b;
          rho = dots[0];
        }
        resident = true;
      }
      if (!resident) {
        // Single-reduction form of the same recurrences: the matvec pass also sums
        // <w, P w> and <w, P q>, so that <q', P q'> of the next direction q' = w + beta q
        // follows as <w,Pw> + 2 beta <w,Pq> + beta^2 <q,Pq>, and the direction update is
        // fused into the next element pass (one pass and one barrier fewer per iteration).
        pcr_update_contrib<BS, true, EXT>(c, buf, nel, 0.f, 0.f, false);
        __syncthreads();
        gather_hinv(c, Y, tid, BS);
        __syncthreads();
        double dots[3] = {0.0, 0.0, 0.0};
        matvec_rows<BS, true, EXT>(c, Y, buf, nel, eps, dots);
        block_sum3<BS>(dots, red);
        if (k == A.dump_k)
          for (int r = tid; r < nrows; r += BS) S.row_dump[R0 + r] = S.row_w[R0 + r];
        double rho = dots[0], qs = dots[1];
        // READING: stop once <z, A z> is at rounding level relative to its start
        const double rho_stop = kTauCR * rho;
        float beta = 0.f;
        for (int it = 0; it < A.cr_iters; ++it) {
          if (!(rho > rho_stop) || !(rho > 0.0)) break;
          if (!(qs > 0.0)) break;
          const float alpha = (float)(rho / qs);
          ++done;
          if (it == A.cr_iters - 1) {  // the last update needs no further product
            last_x_update<BS>(S, R0, nrows, tid, it > 0, alpha, beta);
            break;
          }
          // direction update, x += alpha p, z -= alpha P q, J^T z contributions
          pcr_update_contrib<BS, false, EXT>(c, buf, nel, alpha, beta, it > 0);
          __syncthreads();
          gather_hinv(c, Y, tid, BS);
          __syncthreads();
          dots[0] = dots[1] = dots[2] = 0.0;
          matvec_rows<BS, false, EXT>(c, Y, buf, nel, eps, dots);
          block_sum3<BS>(dots, red);
          const double b = dots[0] / rho;
          qs = dots[1] + 2.0 * b * dots[2] + b * b * qs;
          beta = (float)b;
          rho = dots[0];
        }

      }
    }
    cr_total += done;
    __syncthreads();
    if (k == A.dump_k) break;  // dump step: iteration k's data stays in place

    // ---- update: du = H~^-1 (h J^T dlambda - g), damped step t (Sec. 6.2, 8.1) ----
    const float tstep = A.p.line_search ? 1.f : damp;
    if (A.p.line_search) {
      merit_k = merit;
      ls_t = 1.f;
    }
    contrib_pass<BS, EXT>(c, S.row_x, buf, nel, true);
    __syncthreads();
    // READING (island mode, residual mode): a solved island keeps its velocities
    auto frozen = [&](int b) {
      const int l = ld_coherent(S.b_lab + E.rig_off + E.par_off + b);
      return A.tol > 0.f && l >= 0 && island_solved(c, E.rig_off + E.par_off + 2 * e, l);
    };
    for (int b = tid; b < nb; b += BS) {
      if (b < E.n_rig) {
        const int g = E.rig_off + b;
        const int d = E.dof_off + 6 * b;
        float v[6];
        gather_rigid(c, g, v);
        for (int q = 0; q < 6; ++q) v[q] = h * v[q] - S.g[d + q];
        hinv_rigid(c, g, v);
        if (EXT && isl_mode && frozen(b))
          for (int q = 0; q < 6; ++q) v[q] = 0.f;
        float *u = S.r_u + 6 * g;
        if (A.p.line_search) {
          for (int q = 0; q < 6; ++q) {
            S.r_u_k[6 * g + q] = u[q];
            S.du[d + q] = v[q];
          }
          S.r_q_k[g] = S.r_q[g];
        }
        for (int q = 0; q < 6; ++q) u[q] += tstep * v[q];
      } else {
        const int p = E.par_off + b - E.n_rig;
        const int d = E.dof_off + 6 * E.n_rig + 3 * (b - E.n_rig);
        const V3 a = gather_particle(c, p);
        const float4 H = S.p_H[p];
        const float4 u = S.p_u[p];
        float dv[3] = {(h * a.x - S.g[d]) / H.x, (h * a.y - S.g[d + 1]) / H.y, (h * a.z - S.g[d + 2]) / H.z};
        if (EXT && isl_mode && frozen(b)) dv[0] = dv[1] = dv[2] = 0.f;
        if (A.p.line_search) {
          S.du[d] = dv[0]; S.du[d + 1] = dv[1]; S.du[d + 2] = dv[2];
        }
        S.p_uprev[p] = u;
        S.p_u[p] = make_float4(u.x + tstep * dv[0], u.y + tstep * dv[1], u.z + tstep * dv[2], 0.f);
      }
    }
    __syncthreads();
    if (A.p.line_search) {
      for (int r = tid; r < nrows; r += BS) {
        const int row = R0 + r;
        S.row_lam_k[row] = S.row_lam[row];
        S.row_lam[row] += tstep * S.row_x[row];
      }
    } else {
      // four rows of the thread at a time, loads before stores (see RowIn)
      for (int r = tid; r < nrows; r += 4 * BS) {
        float l[4], x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = r + j * BS;
          l[j] = rr < nrows ? gld(S.row_lam + R0 + rr) : 0.f;
          x[j] = rr < nrows ? gld(S.row_x + R0 + rr) : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (r + j * BS < nrows) gst(S.row_lam + R0 + r + j * BS, l[j] + tstep * x[j]);
      }
    }
    for (int b = tid; b < nb; b += BS) update_positions_body(c, b);
    __syncthreads();
    ++newton_done;
  }
  if (restore) {
    __syncthreads();
    keep_best(c, nrows, true);
    r_ncp = best_r;
    r_con = best_rc;
    merit = best_merit;
    watchdog = 1;
    __syncthreads();
  }
  if (!nonfinite || !warm) break;
  }

  // ---- write-back (a dump step leaves velocities, time and warm-start data alone) ----
  const bool dumping = A.dump_k >= 0;
  for (int b = tid; b < nb && !dumping; b += BS) {
    if (b < E.n_rig) {
      const int g = E.rig_off + b;
      if (S.r_inertia[g].w == 0.f) continue;
      const float *u = S.r_u + 6 * g;
      S.r_v[g] = make_float4(u[0], u[1], u[2], 0.f);
      S.r_w[g] = make_float4(u[3], u[4], u[5], 0.f);
    } else {
      const int p = E.par_off + b - E.n_rig;
      S.p_v[p] = S.p_u[p];
    }
  }
  for (int i = tid; i < nc && !dumping; i += BS) {
    const int gc = E.con_off + i;
    const int r0 = row_con(E, i);
    S.c_prev_key[gc] = S.c_key[gc];
    S.c_prev_lam[gc] = make_float4(S.row_lam[r0], S.row_lam[r0 + 1], S.row_lam[r0 + 2], 0.f);
  }
  if (tid == 0) {
    if (!dumping) {
      S.n_prev[e] = nc;
      S.time[e] = tplus;
    }
    nsn_step_stats st;
    st.newton_iters = newton_done;
    st.cr_iters = cr_total;
    st.n_contacts = nc;
    st.overflow = S.overflow[e];
    st.nonfinite = nonfinite;
    st.converged = converged;
    st.fallback = fallback;
    st.watchdog = watchdog;
    st.r_ncp = r_ncp;
    st.r_contact = r_con;
    st.merit = merit;
    st.r_ncp_first = r_first;
    S.stats[e] = st;
    if (!dumping) {
      nsn_accum a = S.acc[e];
      a.steps += 1;
      a.newton_iters += newton_done;
      a.cr_iters += cr_total;
      a.converged += converged;
      a.nonfinite += nonfinite;
      a.fallbacks += fallback;
      a.watchdogs += watchdog;
      a.cr_bytes += (double)cr_total * ((lin_tets(E) ? kBytesLinTet : kBytesTet) * E.n_tet + kBytesContact * nc +
                                        kBytesJoint * E.n_jnt +
                                        kBytesDof * (6.0 * E.n_rig + 3.0 * E.n_par));
      S.acc[e] = a;
    }
    const int slot = S.tick[0] % kTimingRing;
    atomicMin(S.ts + 2 * slot, t_start);
    atomicMax(S.ts + 2 * slot + 1, (unsigned long long)wall_clock64());
  }
}

// --------------------------------------------------------------------------
// launchers.  The extended instantiation (EXT: linear tets, islands) is built in its
// own translation unit (nsn_step_ext.hip includes this file with NSN_STEP_EXT_TU),
// with a larger basic-block budget for the inliner: at the default budget that
// kernel leaves functions taking the Ctx out of line, which puts the Ctx (about 1 KB)
// in scratch memory.  The default instantiation keeps the default budget.
// --------------------------------------------------------------------------
// register slots per thread of the resident PCR (18 registers each) that fit the
// 256-VGPR budget without spilling below 1024 threads; none at 1024 threads (128 VGPRs)
template <int BS, bool EXT>
constexpr int resident_slots() {
  return EXT ? 0 : (BS >= 1024 ? 0 : 2);
}
// PCR form of a launch: 0 streaming, 1 register-resident where the env fits, 2 one-pass
constexpr int kFormStream = 0, kFormResident = 1, kFormOnePass = 2;

// what: kLaunchAttr sets the kernel's dynamic-LDS limit (a call that must stay outside
// a stream capture), kLaunchRun enqueues the launch; both by default.
template <int BS, int LM, bool EXT, int RS>
static void launch_one(const DevScene &s, const StepArgs &a, int first, int count, size_t bytes, hipStream_t st,
                       int what) {
  if ((what & kLaunchAttr) && bytes > 16384 * sizeof(float))
    (void)hipFuncSetAttribute((const void *)k_newton<BS, LM, EXT, RS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
  if (what & kLaunchRun)
    hipLaunchKernelGGL((k_newton<BS, LM, EXT, RS>), dim3(count), dim3(BS), bytes, st, s.dev, a, first);
}

template <int BS, bool EXT>
static void launch_bs(const DevScene &s, const StepArgs &a, int first, int count, int lds_floats, int lds_mode,
                      int resident, hipStream_t st, int what) {
  const size_t bytes = lds_mode > 0 ? sizeof(float) * (size_t)lds_floats : 0;
  constexpr int B2 = BS >= 128 ? BS : 128;  // mode 2 from 128 threads up
  constexpr int R2 = resident_slots<B2, EXT>(), R1 = resident_slots<BS, EXT>();
  if (lds_mode == 2 && BS >= 128) {
    if constexpr (!EXT)
      if (resident == kFormOnePass) return launch_one<B2, 2, EXT, -1>(s, a, first, count, bytes, st, what);
    if (resident == kFormResident && R2 > 0) launch_one<B2, 2, EXT, R2>(s, a, first, count, bytes, st, what);
    else launch_one<B2, 2, EXT, 0>(s, a, first, count, bytes, st, what);
  } else if (lds_mode >= 1) {
    if constexpr (!EXT)
      if (resident == kFormOnePass) return launch_one<BS, 1, EXT, -1>(s, a, first, count, bytes, st, what);
    if (resident == kFormResident && R1 > 0) launch_one<BS, 1, EXT, R1>(s, a, first, count, bytes, st, what);
    else launch_one<BS, 1, EXT, 0>(s, a, first, count, bytes, st, what);
  } else {
    if constexpr (!EXT)
      if (resident == kFormOnePass) return launch_one<BS, 0, EXT, -1>(s, a, first, count, 0, st, what);
    if (resident == kFormResident && R1 > 0) launch_one<BS, 0, EXT, R1>(s, a, first, count, 0, st, what);
    else launch_one<BS, 0, EXT, 0>(s, a, first, count, 0, st, what);
  }
}

#ifdef NSN_STEP_EXT_TU
constexpr bool kExtTU = true;
#else
constexpr bool kExtTU = false;
#endif

static hipError_t launch_tu(const DevScene &s, const StepArgs &a, int block, int first, int count, int lds_floats,
                            int lds_mode, int resident, hipStream_t st, int what) {
  switch (block) {
    case 64: launch_bs<64, kExtTU>(s, a, first, count, lds_floats, lds_mode, resident, st, what); break;
    case 128: launch_bs<128, kExtTU>(s, a, first, count, lds_floats, lds_mode, resident, st, what); break;
    case 256: launch_bs<256, kExtTU>(s, a, first, count, lds_floats, lds_mode, resident, st, what); break;
    case 512: launch_bs<512, kExtTU>(s, a, first, count, lds_floats, lds_mode, resident, st, what); break;
    case 1024: launch_bs<1024, kExtTU>(s, a, first, count, lds_floats, lds_mode, resident, st, what); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#ifdef NSN_STEP_EXT_TU
hipError_t launch_newton_ext(const DevScene &s, const StepArgs &a, int block, int first, int count, int lds_floats,
                             int lds_mode, hipStream_t st, int what) {
  return launch_tu(s, a, block, first, count, lds_floats, lds_mode, 0, st, what);
}
#else
hipError_t launch_prepare(const DevScene &s, const StepArgs &a, int want_features, hipStream_t st) {
  hipLaunchKernelGGL(k_prepare<256>, dim3(s.n_envs), dim3(256), 0, st, s, a, want_features);
  return hipGetLastError();
}

hipError_t launch_newton(const DevScene &s, const StepArgs &a, int block, int first, int count, int lds_floats,
                         int lds_mode, int resident, hipStream_t st, int what) {
  if (count <= 0) return hipSuccess;
  if (s.any_linear || (a.p.islands && a.p.linear == NSN_LINEAR_PCR))
    return launch_newton_ext(s, a, block, first, count, lds_floats, lds_mode, st, what);
  return launch_tu(s, a, block, first, count, lds_floats, lds_mode, resident, st, what);
}
#endif

}  // namespace nsn
