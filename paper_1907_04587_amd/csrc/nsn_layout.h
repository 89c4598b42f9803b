// Device-side layout of a scene: per-env tables and the structure-of-arrays
// buffers that live in the caller's workspace.  Shared by the host builder
// (nsn_api.cpp) and the kernels (nsn_step.hip, nsn_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/nsn.h"

namespace nsn {

constexpr int kMlpIn = 12;
constexpr int kMlpHidden = 64;
constexpr int kMlpOut = 3;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + 2 * (kMlpHidden * kMlpHidden + kMlpHidden) +
                           kMlpOut * kMlpHidden + kMlpOut;  // 9347
constexpr int kMlpBlob = kMlpParams + 2 * kMlpIn + 2 * kMlpOut;

// Per-environment table (read once per workgroup).
struct EnvInfo {
  int rig_off, n_rig;      // rigid bodies [rig_off, rig_off + n_rig)
  int par_off, n_par;      // particles
  int tet_off, n_tet;      // tetrahedra
  int jnt_off, n_jnt;      // joints
  int con_off, max_con;    // contact slots
  int row_off, row_cap;    // rows: joints (6 each), tets (3 or 6 each), contacts (3 each)
  int dof_off, n_dof;      // body space: 6 per rigid body, 3 per particle
  int feat_off, n_feat;    // rigid collision features (box vertices, capsule ends)
  int n_targets, ground;   // (ground ? 1 : 0) + n_rig
  int bcon_off, tet_model; // target-side contact lists; NSN_TET_* of all the env's tets
  float mu, gx, gy, gz;
};

// PCR scalars of one island (island mode)
struct IslState {
  double rho, qs, stop;
  float alpha, beta;
  int active, pad;
};

// Pointers into the workspace.  Indices stored in the tables are global
// (already offset by the env's base) unless noted.
struct DevScene {
  const DevScene *dev;  // this table's copy in the workspace (the Newton kernel's argument)
  int n_envs;
  int NR, NP, NT, NJ, NC, NROW, NDOF;  // totals over all envs
  int any_linear;                      // some env has NSN_TET_LINEAR tets
  const EnvInfo *env;
  const int *env_order;  // envs sorted by decreasing work (launch order)

  // rigid bodies
  float4 *r_x, *r_q, *r_v, *r_w;  // state at the end of the last step
  float4 *r_x0, *r_q0;             // state at the start of the current step
  const float4 *r_inertia;         // (Ix, Iy, Iz, 1/m), 1/m = 0 for static bodies
  const float4 *r_ext;             // shape extents
  const int *r_shape;
  float *r_Iw, *r_Iwinv;           // world inertia / inverse, 6 per body (xx yy zz xy xz yz)
  float *r_ut, *r_u;               // u~ and the Newton iterate, 6 per body (v, omega)

  // particles
  float4 *p_x, *p_v, *p_x0;
  const float *p_m;                // lumped mass
  float4 *p_ut, *p_u, *p_uprev, *p_H;

  // collision features of rigid bodies: (body, vertex)
  const int2 *feat;

  // tets (component-major SoA)
  const int4 *t_ids;
  const float *t_Dminv;            // 9 x NT
  const float4 *t_mat;             // (Ve, C1, D1, alpha); linear tets (Ve, mu, lambda, 0)
  float *t_J;                      // 2 x 18 x NT, ping-pong: u_i(3), w_i(3) per stretch row;
                                   // linear tets: the rotation R (9, row-major)
  float *t_E;                      // 6 x NT : E / h^2 (xx yy zz xy xz yz); linear tets: normal block
  const int4 *t_dst;               // per tet: positions of its 4 slots in the particle lists
  const uint4 *t_loc;              // per tet, vertex k: (env-local particle id) | (slot position
                                   // from the env's first particle list entry) << 16
  int tet_loc;                     // 1 if every env's ids and slot positions fit 16 bits
  float4 *p_cj;                    // NTADJ : J^T v of the tets, in particle-list order

  // joints
  const int4 *j_info;              // (type, A global or -1, B global, has_drive)
  const float4 *j_frame;           // 6 per joint: pA, pB, aA, aB, tA, tB
  const float4 *j_drive;           // 2 per joint: (kp, kd, amp, freq), (phase, offset, -, -)
  float *j_theta0;                 // drive coordinate at q^-
  float *j_J;                      // NJ x 6 rows x 12 (J_A, J_B)
  int2 *j_slot;                    // NJ : (side A, side B) contribution slot, -1 for the world

  // contacts (capacity NC)
  int *c_key;
  int2 *c_body;                    // (feature body, target body): env-local numbering,
                                   // rigid i -> i, particle p -> n_rig + p, ground -> -1
  float4 *c_n;                     // normal, thickness
  float4 *c_aL, *c_bL;             // feature / target points (body frame or world)
  float4 *c_rA, *c_rB;             // world arms at the current iterate
  float4 *c_cj;                    // world direction of a contact's J^T v (particle feature bodies)
  int2 *c_slot;                    // (feature side, target side) contribution slot, -1 if not rigid
  float *c_alpha;                  // 2 x NC ping-pong (normal row scale alpha)
  int *c_active;                   // 2 x NC ping-pong (friction rows active)
  float4 *c_lam0;                  // warm-start multipliers
  float *c_feat;                   // NC x 12 features (contact-major)
  int *c_prev_key;                 // last step's contacts (sorted keys) and multipliers
  float4 *c_prev_lam;
  int *n_prev;

  // contact adjacency (rebuilt every step)
  int *r_acon_beg, *r_acon_end;    // rigid body as feature body: contact range
  int *p_acon_beg, *p_acon_end;    // particle as feature body
  int *r_bcon_beg, *r_bcon_cnt;    // rigid body as target: range in bcon_list
  int *bcon_list;                  // contact indices (global)
  // rigid bodies' J^T v contributions: one run of slots per body, its joints (adjacency
  // order), then the contacts where it is the feature body, then those where it is the
  // target (list order); a slot is a force and a torque, two float4, with the target
  // side's sign applied.  Slots are assigned with the contacts every step.
  float4 *r_cj;                    // 2 x (2 NJ + 2 NC)
  int2 *r_slot;                    // NR : (first, end) slot of a body's run

  // static adjacency
  const int *p_tadj_ptr, *p_tadj;  // particle -> (tet << 2 | slot)
  const int *r_jadj_ptr, *r_jadj;  // rigid body -> (joint << 1 | side)

  // rows (capacity NROW)
  float *row_lam, *row_x, *row_z, *row_p, *row_q, *row_w, *row_err, *row_P, *row_C, *row_b;
  // the step's lowest-merit iterate (watchdog); in a dump step, iterate k-1
  float *row_lam_best, *r_u_best;
  float4 *r_x_best, *r_q_best, *p_u_best, *p_x_best;
  // line search: the accepted iterate k (particle velocities in p_uprev) and its direction
  float *row_lam_k, *r_u_k, *du;
  float4 *r_q_k;

  // dump step: A (P b) of the dumped iteration
  float *row_dump;

  // body space (NDOF)
  float *y, *g, *f;
  float *bz, *bq;  // one-pass PCR: J^T z and J^T (P q) in body space (NDOF each)

  // islands (rebuilt every step in island mode).  Element index space of an env:
  // [joints | tets | contact slots] from jnt_off + tet_off + con_off; island slots of
  // an env: rig_off + par_off + 2 env, one per body (named by the island's lowest
  // env-local body index) plus the static group (index n_rig + n_par)
  int *b_lab;                      // NR + NP: island of every body (-1: static)
  int *el_isl, *el_perm;           // island of every element; elements grouped by island
  double *el_dots;                 // 3 per element: its part of the PCR dots
  int *isl_cnt, *isl_off, *isl_run, *isl_list;  // per island slot: size, start in el_perm,
                                                // placement counter; non-empty islands
  IslState *isl;
  int *isl_n;                      // per env: number of non-empty islands
  int *isl_res;                    // per island slot: its residual (bits of a float >= 0)

  // per env dynamic; c_inject: 1 + the number of caller-given contacts that replace
  // collision detection in the next step (0: none)
  int *n_con, *overflow, *c_inject;
  double *time;
  nsn_step_stats *stats;

  // learned warm start
  const float *mlp;
  int have_mlp;

  // launch timing: step counter and per-step (first start, last end) wall clock of
  // the Newton kernel(s), a ring of kTimingRing steps
  int *tick;
  unsigned long long *ts;
  nsn_accum *acc;
};

// algorithmic bytes of one PCR iteration (see nsn_accum)
constexpr double kBytesTet = 332.0, kBytesContact = 228.0, kBytesJoint = 880.0, kBytesDof = 12.0;
constexpr double kBytesLinTet = 476.0;  // a linear tet (6 rows)

constexpr int kTimingRing = 1024;

struct StepArgs {
  float h;
  int newton_iters, cr_iters;
  float tol;
  int dump_k;  // >= 0: stop inside Newton iteration dump_k and keep its data (dump step)
  nsn_solver_params p;
};

// sets the calling thread's nsn_last_error() message and returns st (nsn_api.cpp)
nsn_status set_error(nsn_status st, const std::string &msg);

// kernel launchers (nsn_step.hip)
hipError_t launch_prepare(const DevScene &s, const StepArgs &a, int want_features, hipStream_t st);
// envs S.env_order[first .. first+count) with `block` threads per workgroup;
// lds_mode 0: the body-space vector in global memory; 1: in `lds_floats` floats of
// dynamic LDS; 2: in LDS together with the tets' contributions
// (align4(n_dof) + 12 n_tet floats per env)
// resident: the register-resident PCR for the envs whose elements all have a register
// slot (neo-Hookean instantiation only; others take the streaming form)
// what: kLaunchAttr sets the chosen kernel's dynamic-LDS limit (not allowed inside a
// stream capture), kLaunchRun enqueues it
constexpr int kLaunchAttr = 1, kLaunchRun = 2;
hipError_t launch_newton(const DevScene &s, const StepArgs &a, int block, int first, int count, int lds_floats,
                         int lds_mode, int resident, hipStream_t st, int what = kLaunchAttr | kLaunchRun);
// the same for the extended instantiation (linear tets, islands; nsn_step_ext.hip)
hipError_t launch_newton_ext(const DevScene &s, const StepArgs &a, int block, int first, int count, int lds_floats,
                             int lds_mode, hipStream_t st, int what);
constexpr int kMaxLdsFloats = 24 * 1024;  // 96 KB of LDS for the body-space vector
constexpr int kMaxLdsFloatsCl = 39 * 1024;  // 156 KB: body-space vector + tet contributions (mode 2)
// learned warm start: MLP prediction for every contact of every env (nsn_mlp.hip)
// hybrid: contacts that existed in the previous step keep their previous-step multipliers
hipError_t launch_warm_mlp(const DevScene &s, int hybrid, hipStream_t st);

}  // namespace nsn
