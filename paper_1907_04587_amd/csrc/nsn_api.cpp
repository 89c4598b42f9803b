// Host side of the C ABI (include/nsn.h): validation, the device layout inside the
// caller's workspace, static adjacency, graph capture of the step, state I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "nsn_layout.h"

using namespace nsn;

namespace {

thread_local std::string g_err;

nsn_status fail(nsn_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return fail(NSN_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// Sequential sub-allocator: a dry run computes the size, a real run assigns pointers.
struct Arena {
  char *base;
  size_t off = 0;
  explicit Arena(void *b) : base((char *)b) {}
  template <class T>
  T *take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? (T *)(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

struct HostEnv {
  int n_rig, n_par, n_tet, n_jnt, max_con, n_feat, n_targets, tet_rows;
};

struct Sizes {
  int NR = 0, NP = 0, NT = 0, NJ = 0, NC = 0, NROW = 0, NDOF = 0, NF = 0, NTADJ = 0, NJADJ = 0;
  int any_linear = 0;
};

nsn_status validate_env(const nsn_env_desc &d, int e, HostEnv &he) {
  auto bad = [&](const std::string &m) { return fail(NSN_EINVAL, "env " + std::to_string(e) + ": " + m); };
  if (d.n_rigid < 0 || d.n_particles < 0 || d.n_tets < 0 || d.n_joints < 0 || d.max_contacts < 0)
    return bad("negative count");
  if (d.n_rigid > 0 && (!d.rigid_mass || !d.rigid_inertia || !d.rigid_x || !d.rigid_q || !d.rigid_v ||
                        !d.rigid_w || !d.rigid_shape || !d.rigid_extent))
    return bad("missing rigid arrays");
  if (d.n_particles > 0 && (!d.particle_x || !d.particle_v || !d.particle_rest))
    return bad("missing particle arrays");
  if (d.n_tets > 0 && (!d.tet_ids || !d.tet_material)) return bad("missing tet arrays");
  if (d.tet_model != NSN_TET_NEOHOOKEAN && d.tet_model != NSN_TET_LINEAR) return bad("unknown tet model");
  if (d.n_joints > 0 && (!d.joint_type || !d.joint_body || !d.joint_anchor || !d.joint_axis || !d.joint_ref ||
                         !d.joint_drive))
    return bad("missing joint arrays");
  int nfeat = 0;
  for (int i = 0; i < d.n_rigid; ++i) {
    const float m = d.rigid_mass[i];
    if (!(m >= 0.f) || !std::isfinite(m)) return bad("rigid " + std::to_string(i) + ": bad mass");
    if (m > 0.f)
      for (int k = 0; k < 3; ++k)
        if (!(d.rigid_inertia[3 * i + k] > 0.f)) return bad("rigid " + std::to_string(i) + ": bad inertia");
    const int sh = d.rigid_shape[i];
    if (sh < 0 || sh > 2) return bad("rigid " + std::to_string(i) + ": bad shape");
    float ql = 0.f;
    for (int k = 0; k < 4; ++k) ql += d.rigid_q[4 * i + k] * d.rigid_q[4 * i + k];
    if (!(ql > 0.f)) return bad("rigid " + std::to_string(i) + ": zero quaternion");
    nfeat += sh == NSN_SHAPE_BOX ? 8 : (sh == NSN_SHAPE_CAPSULE ? 2 : 0);
  }
  std::vector<float> mass(d.n_particles, 0.f);
  for (int p = 0; p < d.n_particles; ++p) mass[p] = d.particle_mass ? d.particle_mass[p] : 0.f;
  for (int t = 0; t < d.n_tets; ++t) {
    for (int k = 0; k < 4; ++k) {
      const int id = d.tet_ids[4 * t + k];
      if (id < 0 || id >= d.n_particles) return bad("tet " + std::to_string(t) + ": bad particle id");
    }
    const float E = d.tet_material[3 * t], nu = d.tet_material[3 * t + 1], rho = d.tet_material[3 * t + 2];
    if (!(E > 0.f) || !(nu > -1.f && nu < 0.5f) || !(rho > 0.f)) return bad("tet " + std::to_string(t) + ": bad material");
  }
  for (int j = 0; j < d.n_joints; ++j) {
    const int a = d.joint_body[2 * j], b = d.joint_body[2 * j + 1], ty = d.joint_type[j];
    if (a < -1 || a >= d.n_rigid || b < 0 || b >= d.n_rigid || a == b || (ty != 0 && ty != 1))
      return bad("joint " + std::to_string(j) + ": bad bodies or type");
  }
  he.n_rig = d.n_rigid;
  he.n_par = d.n_particles;
  he.n_tet = d.n_tets;
  he.tet_rows = d.tet_model == NSN_TET_LINEAR ? 6 : 3;
  he.n_jnt = d.n_joints;
  he.max_con = d.max_contacts;
  he.n_feat = nfeat;
  he.n_targets = (d.ground ? 1 : 0) + d.n_rigid;
  const long long ncand = (long long)(nfeat + d.n_particles) * he.n_targets;
  if (ncand >= (1ll << 31)) return fail(NSN_EUNSUPPORTED, "env " + std::to_string(e) + ": too many collision candidates");
  return NSN_OK;
}

// Which optional buffers a workspace holds (decided by the parameters at creation).
struct Options {
  bool islands = false, line_search = false;
};

Options options_of(const nsn_solver_params *p) {
  Options o;
  if (p) {
    o.islands = p->islands != 0;
    o.line_search = p->line_search != 0;
  }
  return o;
}

bool params_ok(const nsn_solver_params *p) {
  return p->ncp >= 0 && p->ncp <= 1 && p->rmode >= 0 && p->rmode <= 2 && p->warm >= 0 && p->warm <= 3 &&
         p->fem_mode >= 0 && p->fem_mode <= 1 && p->damping > 0.f && p->eps >= 0.f && p->margin >= 0.f &&
         p->line_search >= 0 && p->line_search <= 1 && p->linear >= 0 && p->linear <= 1 && p->islands >= 0 &&
         p->islands <= 1 && p->watchdog >= 0 && p->watchdog <= 1 && p->geo_stiff >= 0 && p->geo_stiff <= 1;
}

// Assign every workspace buffer; with base == nullptr only the size is computed.
void layout(const Sizes &z, int n_envs, const Options &opt, Arena &a, DevScene &S, EnvInfo *&env, int *&order) {
  S.dev = a.take<DevScene>(1);
  S.n_envs = n_envs;
  S.NR = z.NR; S.NP = z.NP; S.NT = z.NT; S.NJ = z.NJ; S.NC = z.NC; S.NROW = z.NROW; S.NDOF = z.NDOF;
  S.any_linear = z.any_linear;
  env = a.take<EnvInfo>(n_envs);
  order = a.take<int>(n_envs);
  S.env = env;
  S.env_order = order;
  S.r_x = a.take<float4>(z.NR); S.r_q = a.take<float4>(z.NR); S.r_v = a.take<float4>(z.NR);
  S.r_w = a.take<float4>(z.NR); S.r_x0 = a.take<float4>(z.NR); S.r_q0 = a.take<float4>(z.NR);
  S.r_inertia = a.take<float4>(z.NR); S.r_ext = a.take<float4>(z.NR); S.r_shape = a.take<int>(z.NR);
  S.r_Iw = a.take<float>(6 * (size_t)z.NR); S.r_Iwinv = a.take<float>(6 * (size_t)z.NR);
  S.r_ut = a.take<float>(6 * (size_t)z.NR); S.r_u = a.take<float>(6 * (size_t)z.NR);
  S.p_x = a.take<float4>(z.NP); S.p_v = a.take<float4>(z.NP); S.p_x0 = a.take<float4>(z.NP);
  S.p_m = a.take<float>(z.NP); S.p_ut = a.take<float4>(z.NP); S.p_u = a.take<float4>(z.NP);
  S.p_uprev = a.take<float4>(z.NP); S.p_H = a.take<float4>(z.NP);
  S.feat = a.take<int2>(z.NF);
  S.t_ids = a.take<int4>(z.NT); S.t_Dminv = a.take<float>(9 * (size_t)z.NT); S.t_mat = a.take<float4>(z.NT);
  S.t_J = a.take<float>(2 * 18 * (size_t)z.NT); S.t_E = a.take<float>(6 * (size_t)z.NT);
  S.t_dst = a.take<int4>(z.NT); S.p_cj = a.take<float4>(z.NTADJ); S.t_loc = a.take<uint4>(z.NT);
  S.j_info = a.take<int4>(z.NJ); S.j_frame = a.take<float4>(6 * (size_t)z.NJ);
  S.j_drive = a.take<float4>(2 * (size_t)z.NJ); S.j_theta0 = a.take<float>(z.NJ);
  S.j_J = a.take<float>(72 * (size_t)z.NJ);
  S.j_slot = a.take<int2>(z.NJ);
  S.c_key = a.take<int>(z.NC); S.c_body = a.take<int2>(z.NC); S.c_n = a.take<float4>(z.NC);
  S.c_aL = a.take<float4>(z.NC); S.c_bL = a.take<float4>(z.NC); S.c_rA = a.take<float4>(z.NC);
  S.c_rB = a.take<float4>(z.NC); S.c_cj = a.take<float4>(z.NC); S.c_alpha = a.take<float>(2 * (size_t)z.NC);
  S.c_active = a.take<int>(2 * (size_t)z.NC); S.c_lam0 = a.take<float4>(z.NC);
  S.c_feat = a.take<float>(12 * (size_t)z.NC); S.c_prev_key = a.take<int>(z.NC);
  S.c_prev_lam = a.take<float4>(z.NC); S.n_prev = a.take<int>(n_envs);
  S.r_acon_beg = a.take<int>(z.NR); S.r_acon_end = a.take<int>(z.NR);
  S.p_acon_beg = a.take<int>(z.NP); S.p_acon_end = a.take<int>(z.NP);
  S.r_bcon_beg = a.take<int>(z.NR); S.r_bcon_cnt = a.take<int>(z.NR); S.bcon_list = a.take<int>(z.NC);
  S.r_cj = a.take<float4>(2 * (2 * (size_t)z.NJ + 2 * (size_t)z.NC)); S.r_slot = a.take<int2>(z.NR);
  S.c_slot = a.take<int2>(z.NC);
  S.p_tadj_ptr = a.take<int>(z.NP + 1); S.p_tadj = a.take<int>(z.NTADJ);
  S.r_jadj_ptr = a.take<int>(z.NR + 1); S.r_jadj = a.take<int>(z.NJADJ);
  S.row_lam = a.take<float>(z.NROW); S.row_x = a.take<float>(z.NROW); S.row_z = a.take<float>(z.NROW);
  S.row_p = a.take<float>(z.NROW); S.row_q = a.take<float>(z.NROW); S.row_w = a.take<float>(z.NROW);
  S.row_err = a.take<float>(z.NROW); S.row_P = a.take<float>(z.NROW); S.row_C = a.take<float>(z.NROW);
  S.row_b = a.take<float>(z.NROW);
  S.row_lam_best = a.take<float>(z.NROW); S.r_u_best = a.take<float>(6 * (size_t)z.NR);
  S.r_x_best = a.take<float4>(z.NR); S.r_q_best = a.take<float4>(z.NR);
  S.p_u_best = a.take<float4>(z.NP); S.p_x_best = a.take<float4>(z.NP);
  // line search (only when reserved)
  const size_t ls = opt.line_search ? 1 : 0;
  S.row_lam_k = a.take<float>(ls * z.NROW); S.r_u_k = a.take<float>(ls * 6 * (size_t)z.NR);
  S.r_q_k = a.take<float4>(ls * z.NR); S.du = a.take<float>(ls * z.NDOF);
  S.row_dump = a.take<float>(z.NROW);
  S.y = a.take<float>(z.NDOF); S.g = a.take<float>(z.NDOF); S.f = a.take<float>(z.NDOF);
  S.bz = a.take<float>(z.NDOF); S.bq = a.take<float>(z.NDOF);
  // islands: per element (joints, tets, contact slots), per body, and per env
  // n_rig + n_par + 2 island slots (the bodies, the static group, one spare)
  const size_t isl = opt.islands ? 1 : 0;
  const size_t nel = isl * ((size_t)z.NJ + z.NT + z.NC), nslot = isl * ((size_t)z.NR + z.NP + 2 * (size_t)n_envs);
  S.b_lab = a.take<int>(isl * ((size_t)z.NR + z.NP));
  S.el_isl = a.take<int>(nel); S.el_perm = a.take<int>(nel); S.el_dots = a.take<double>(3 * nel);
  S.isl_cnt = a.take<int>(nslot); S.isl_off = a.take<int>(nslot); S.isl_run = a.take<int>(nslot);
  S.isl_list = a.take<int>(nslot); S.isl = a.take<IslState>(nslot); S.isl_n = a.take<int>(isl * n_envs);
  S.isl_res = a.take<int>(nslot);
  S.n_con = a.take<int>(n_envs); S.overflow = a.take<int>(n_envs); S.c_inject = a.take<int>(n_envs);
  S.time = a.take<double>(n_envs);
  S.stats = a.take<nsn_step_stats>(n_envs);
  S.mlp = a.take<float>(kMlpBlob);
  S.have_mlp = 0;
  S.tick = a.take<int>(1);
  S.ts = a.take<unsigned long long>(2 * kTimingRing);
  S.acc = a.take<nsn_accum>(n_envs);
}

Sizes sizes_of(const std::vector<HostEnv> &he) {
  Sizes z;
  for (const auto &h : he) {
    z.NR += h.n_rig; z.NP += h.n_par; z.NT += h.n_tet; z.NJ += h.n_jnt; z.NC += h.max_con;
    z.NROW += 6 * h.n_jnt + h.tet_rows * h.n_tet + 3 * h.max_con;
    if (h.tet_rows == 6 && h.n_tet > 0) z.any_linear = 1;
    z.NDOF += 6 * h.n_rig + 3 * h.n_par;
    z.NF += h.n_feat;
    z.NTADJ += 4 * h.n_tet;
    z.NJADJ += 2 * h.n_jnt;
  }
  return z;
}

}  // namespace

nsn_status nsn::set_error(nsn_status st, const std::string &msg) { return fail(st, msg); }

struct GraphKey {
  float h;
  int n, m;
  float tol;
  bool operator<(const GraphKey &o) const {
    return std::tie(h, n, m, tol) < std::tie(o.h, o.n, o.m, o.tol);
  }
};

struct Bucket {
  int first, count, block;
  int lds_floats;  // dynamic LDS floats of a workgroup
  int lds_mode;    // 0: body-space vector in global memory, 1: in LDS, 2: with the tet contributions
};

struct nsn_scene_s {
  DevScene S;
  hipStream_t stream = nullptr;
  nsn_solver_params p;
  Options reserved;   // optional buffers present in the workspace
  int dumped_k = -1;  // iteration of the last dump step (-1: none)
  std::vector<nsn_env_desc> desc_sizes;  // counts only (pointers cleared)
  std::vector<EnvInfo> env;
  std::vector<int> order;
  std::vector<Bucket> buckets;
  std::map<GraphKey, hipGraphExec_t> graphs;
  bool use_graphs = true;
  int lds_max = 2;  // the largest LDS mode the buckets may use (nsn_set_lds_mode)
  int pcr_form = 2;  // the PCR loop's form (nsn_set_pcr_form): one-pass by default
  int want_features = 0;
  // side streams (default priority) for concurrent schedule buckets, and fork/join events
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  ~nsn_scene_s() {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto st : side) (void)hipStreamDestroy(st);
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// LDS of each bucket: the body-space vector and the tets' contributions (mode 2) when
// every env's fit in the LDS share that keeps the register-limited occupancy (one
// workgroup per CU at 512 and 1024 threads, two at 256, four at 128); else the
// body-space vector alone (mode 1) when it fits.
static void set_bucket_lds(nsn_scene s) {
  int dev = 0, max_bytes = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    max_bytes = 0;
  // room for the kernel's static LDS (the block reductions, < 1 KB)
  const int max_cl = std::min(kMaxLdsFloatsCl, (max_bytes - 2048) / 4);
  for (Bucket &b : s->buckets) {
    int mx = 0, mx_cl = 0;
    for (int i = b.first; i < b.first + b.count; ++i) {
      const EnvInfo &E = s->env[s->order[i]];
      mx = std::max(mx, E.n_dof);
      mx_cl = std::max(mx_cl, ((E.n_dof + 3) & ~3) + 12 * E.n_tet);
    }
    b.lds_mode = 0;
    b.lds_floats = 0;
    // workgroups per CU at the kernel's register use (8 waves per CU): the LDS share
    // that keeps them resident
    const int per_cu = std::max(1, 512 / b.block);
    if (s->lds_max >= 2 && b.block >= 128 && mx_cl > 0 && mx_cl <= max_cl / per_cu) {
      b.lds_mode = 2;
      b.lds_floats = mx_cl;
    } else if (s->lds_max >= 1 && mx > 0 && mx <= kMaxLdsFloats) {
      b.lds_mode = 1;
      b.lds_floats = mx;
    }
  }
}

// The dynamic state: every array a step reads that an earlier step wrote (Alg. 1 reads
// q^-, u^- and the time; a warm start, Sec. 8.1, also the previous step's contact keys
// and multipliers and the joint rows' multipliers, which stay in row_lam).  Each block
// starts at a 256-byte boundary of the snapshot.
template <class F>
static size_t for_each_state_block(const DevScene &S, F f) {
  size_t off = 0;
  auto blk = [&](const void *p, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    if (bytes) f((char *)p, off, bytes);
    off += bytes;
  };
  blk(S.r_x, sizeof(float4) * S.NR);
  blk(S.r_q, sizeof(float4) * S.NR);
  blk(S.r_v, sizeof(float4) * S.NR);
  blk(S.r_w, sizeof(float4) * S.NR);
  blk(S.p_x, sizeof(float4) * S.NP);
  blk(S.p_v, sizeof(float4) * S.NP);
  blk(S.time, sizeof(double) * S.n_envs);
  blk(S.c_prev_key, sizeof(int) * S.NC);
  blk(S.c_prev_lam, sizeof(float4) * S.NC);
  blk(S.n_prev, sizeof(int) * S.n_envs);
  blk(S.row_lam, sizeof(float) * S.NROW);
  return off;
}

extern "C" {

const char *nsn_last_error(void) { return g_err.c_str(); }

nsn_status nsn_query_workspace(const nsn_env_desc *envs, int32_t n_envs, const nsn_solver_params *params,
                               size_t *bytes) {
  if (!envs || n_envs < 1 || !bytes) return fail(NSN_EINVAL, "nsn_query_workspace: bad arguments");
  if (params && !params_ok(params)) return fail(NSN_EINVAL, "bad solver parameters");
  std::vector<HostEnv> he(n_envs);
  for (int e = 0; e < n_envs; ++e) {
    nsn_status st = validate_env(envs[e], e, he[e]);
    if (st) return st;
  }
  Sizes z = sizes_of(he);
  Arena a(nullptr);
  DevScene S{};
  EnvInfo *env;
  int *order;
  layout(z, n_envs, options_of(params), a, S, env, order);
  *bytes = a.off + 256;
  return NSN_OK;
}

static bool learned_warm(int w) { return w == NSN_WARM_LEARNED || w == NSN_WARM_HYBRID; }

nsn_status nsn_create_scene(const nsn_env_desc *envs, int32_t n_envs, const nsn_solver_params *p,
                            void *hip_stream, void *workspace, size_t workspace_bytes, nsn_scene *out) {
  if (!envs || n_envs < 1 || !p || !out) return fail(NSN_EINVAL, "nsn_create_scene: bad arguments");
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(NSN_EINVAL, "workspace must be a 256-byte aligned device pointer");
  if (!params_ok(p)) return fail(NSN_EINVAL, "bad solver parameters");
  size_t need = 0;
  nsn_status st = nsn_query_workspace(envs, n_envs, p, &need);
  if (st) return st;
  if (workspace_bytes < need) return fail(NSN_ENOMEM, "workspace too small: need " + std::to_string(need));
  std::vector<HostEnv> he(n_envs);
  for (int e = 0; e < n_envs; ++e) validate_env(envs[e], e, he[e]);
  Sizes z = sizes_of(he);
  auto *s = new nsn_scene_s();
  s->stream = (hipStream_t)hip_stream;
  s->p = *p;
  s->reserved = options_of(p);
  Arena a(workspace);
  EnvInfo *env_dev;
  int *order_dev;
  layout(z, n_envs, s->reserved, a, s->S, env_dev, order_dev);
  DevScene &S = s->S;

  // ---- host staging of every static and initial array ----
  std::vector<EnvInfo> env(n_envs);
  std::vector<float4> r_x(z.NR), r_q(z.NR), r_v(z.NR), r_w(z.NR), r_in(z.NR), r_ext(z.NR);
  std::vector<int> r_shape(z.NR);
  std::vector<float4> p_x(z.NP), p_v(z.NP);
  std::vector<float> p_m(z.NP, 0.f);
  std::vector<int2> feat(std::max(z.NF, 1));
  std::vector<int4> t_ids(z.NT);
  std::vector<float> t_Dminv(9 * (size_t)z.NT);
  std::vector<float4> t_mat(z.NT);
  std::vector<int4> j_info(z.NJ);
  std::vector<float4> j_frame(6 * (size_t)z.NJ), j_drive(2 * (size_t)z.NJ);
  std::vector<int> tadj_ptr(z.NP + 1, 0), tadj(std::max(z.NTADJ, 1)), jadj_ptr(z.NR + 1, 0), jadj(std::max(z.NJADJ, 1));
  std::vector<int4> t_dst(std::max(z.NT, 1));
  int ro = 0, po = 0, to = 0, jo = 0, co = 0, rowo = 0, dofo = 0, fo = 0;
  for (int e = 0; e < n_envs; ++e) {
    const nsn_env_desc &d = envs[e];
    const HostEnv &h = he[e];
    EnvInfo &E = env[e];
    E.rig_off = ro; E.n_rig = h.n_rig; E.par_off = po; E.n_par = h.n_par;
    E.tet_off = to; E.n_tet = h.n_tet; E.jnt_off = jo; E.n_jnt = h.n_jnt;
    E.con_off = co; E.max_con = h.max_con; E.row_off = rowo;
    E.row_cap = 6 * h.n_jnt + h.tet_rows * h.n_tet + 3 * h.max_con;
    E.dof_off = dofo; E.n_dof = 6 * h.n_rig + 3 * h.n_par;
    E.feat_off = fo; E.n_feat = h.n_feat; E.n_targets = h.n_targets; E.ground = d.ground ? 1 : 0;
    E.bcon_off = co; E.tet_model = d.tet_model;
    E.mu = d.mu; E.gx = d.gravity[0]; E.gy = d.gravity[1]; E.gz = d.gravity[2];
    for (int i = 0; i < h.n_rig; ++i) {
      const int g = ro + i;
      float q[4];
      float ql = 0.f;
      for (int k = 0; k < 4; ++k) { q[k] = d.rigid_q[4 * i + k]; ql += q[k] * q[k]; }
      ql = std::sqrt(ql);
      for (int k = 0; k < 4; ++k) q[k] /= ql;
      const float m = d.rigid_mass[i];
      const bool stat = !(m > 0.f);
      r_x[g] = make_float4(d.rigid_x[3 * i], d.rigid_x[3 * i + 1], d.rigid_x[3 * i + 2], 0.f);
      r_q[g] = make_float4(q[0], q[1], q[2], q[3]);
      r_v[g] = stat ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(d.rigid_v[3 * i], d.rigid_v[3 * i + 1], d.rigid_v[3 * i + 2], 0.f);
      r_w[g] = stat ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(d.rigid_w[3 * i], d.rigid_w[3 * i + 1], d.rigid_w[3 * i + 2], 0.f);
      r_in[g] = make_float4(d.rigid_inertia[3 * i], d.rigid_inertia[3 * i + 1], d.rigid_inertia[3 * i + 2], stat ? 0.f : 1.f / m);
      r_ext[g] = make_float4(d.rigid_extent[3 * i], d.rigid_extent[3 * i + 1], d.rigid_extent[3 * i + 2], 0.f);
      r_shape[g] = d.rigid_shape[i];
      const int nf = r_shape[g] == NSN_SHAPE_BOX ? 8 : (r_shape[g] == NSN_SHAPE_CAPSULE ? 2 : 0);
      for (int v = 0; v < nf; ++v) feat[fo++] = make_int2(g, v);
    }
    for (int i = 0; i < h.n_par; ++i) {
      const int g = po + i;
      p_x[g] = make_float4(d.particle_x[3 * i], d.particle_x[3 * i + 1], d.particle_x[3 * i + 2], 0.f);
      p_v[g] = make_float4(d.particle_v[3 * i], d.particle_v[3 * i + 1], d.particle_v[3 * i + 2], 0.f);
      p_m[g] = d.particle_mass ? d.particle_mass[i] : 0.f;
    }
    for (int t = 0; t < h.n_tet; ++t) {
      const int g = to + t;
      const int *id = d.tet_ids + 4 * t;
      t_ids[g] = make_int4(po + id[0], po + id[1], po + id[2], po + id[3]);
      // rest shape D_m and its inverse (Sec. 9.2 constant-strain tetrahedron), in double
      double Dm[9];
      const float *r0 = d.particle_rest + 3 * id[0];
      for (int c = 0; c < 3; ++c) {
        const float *rc = d.particle_rest + 3 * id[c + 1];
        for (int r = 0; r < 3; ++r) Dm[3 * r + c] = (double)rc[r] - (double)r0[r];
      }
      const double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6]) +
                         Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
      if (!(std::fabs(det) > 1e-15)) {
        delete s;
        return fail(NSN_EINVAL, "env " + std::to_string(e) + ": tet " + std::to_string(t) + " has a degenerate rest shape");
      }
      double Di[9];
      Di[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) / det; Di[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) / det;
      Di[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) / det; Di[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) / det;
      Di[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) / det; Di[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) / det;
      Di[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) / det; Di[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) / det;
      Di[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) / det;
      for (int k = 0; k < 9; ++k) t_Dminv[(size_t)k * z.NT + g] = (float)Di[k];
      const double Ve = std::fabs(det) / 6.0;
      const double E = d.tet_material[3 * t], nu = d.tet_material[3 * t + 1], rho = d.tet_material[3 * t + 2];
      // READING of the material constants: C1 = mu/2, D1 = (lambda+mu)/2, alpha = 1 + mu/(lambda+mu)
      const double mu = E / (2.0 * (1.0 + nu)), la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
      if (d.tet_model == NSN_TET_LINEAR) t_mat[g] = make_float4((float)Ve, (float)mu, (float)la, 0.f);
      else t_mat[g] = make_float4((float)Ve, (float)(0.5 * mu), (float)(0.5 * (la + mu)), (float)(1.0 + mu / (la + mu)));
      // READING: lumped particle mass rho V_e / 4 per vertex (Sec. 9.3)
      for (int k = 0; k < 4; ++k) p_m[po + id[k]] += (float)(rho * Ve / 4.0);
    }
    for (int i = 0; i < h.n_par; ++i)
      if (!(p_m[po + i] > 0.f)) {
        delete s;
        return fail(NSN_EINVAL, "env " + std::to_string(e) + ": particle " + std::to_string(i) + " has no mass");
      }
    for (int j = 0; j < h.n_jnt; ++j) {
      const int g = jo + j;
      const int A = d.joint_body[2 * j], B = d.joint_body[2 * j + 1];
      const float *dr = d.joint_drive + 6 * j;
      const int has_drive = (dr[0] != 0.f || dr[1] != 0.f) ? 1 : 0;
      j_info[g] = make_int4(d.joint_type[j], A >= 0 ? ro + A : -1, ro + B, has_drive);
      const float *an = d.joint_anchor + 6 * j, *ax = d.joint_axis + 6 * j, *rf = d.joint_ref + 6 * j;
      j_frame[6 * g + 0] = make_float4(an[0], an[1], an[2], 0.f);
      j_frame[6 * g + 1] = make_float4(an[3], an[4], an[5], 0.f);
      j_frame[6 * g + 2] = make_float4(ax[0], ax[1], ax[2], 0.f);
      j_frame[6 * g + 3] = make_float4(ax[3], ax[4], ax[5], 0.f);
      j_frame[6 * g + 4] = make_float4(rf[0], rf[1], rf[2], 0.f);
      j_frame[6 * g + 5] = make_float4(rf[3], rf[4], rf[5], 0.f);
      j_drive[2 * g] = make_float4(dr[0], dr[1], dr[2], dr[3]);
      j_drive[2 * g + 1] = make_float4(dr[4], dr[5], 0.f, 0.f);
    }
    ro += h.n_rig; po += h.n_par; to += h.n_tet; jo += h.n_jnt; co += h.max_con;
    rowo += E.row_cap; dofo += E.n_dof;
  }
  // static adjacency: particle -> (tet, slot) and rigid -> (joint, side), in element order
  for (int t = 0; t < z.NT; ++t) {
    const int4 id = t_ids[t];
    tadj_ptr[id.x + 1]++; tadj_ptr[id.y + 1]++; tadj_ptr[id.z + 1]++; tadj_ptr[id.w + 1]++;
  }
  for (int i = 0; i < z.NP; ++i) tadj_ptr[i + 1] += tadj_ptr[i];
  {
    std::vector<int> fill(tadj_ptr.begin(), tadj_ptr.end() - 1);
    for (int t = 0; t < z.NT; ++t) {
      const int ids[4] = {t_ids[t].x, t_ids[t].y, t_ids[t].z, t_ids[t].w};
      int pos[4];
      for (int k = 0; k < 4; ++k) {
        pos[k] = fill[ids[k]]++;
        tadj[pos[k]] = (t << 2) | k;
      }
      t_dst[t] = make_int4(pos[0], pos[1], pos[2], pos[3]);
    }
  }
  for (int j = 0; j < z.NJ; ++j) {
    if (j_info[j].y >= 0) jadj_ptr[j_info[j].y + 1]++;
    jadj_ptr[j_info[j].z + 1]++;
  }
  for (int i = 0; i < z.NR; ++i) jadj_ptr[i + 1] += jadj_ptr[i];
  {
    std::vector<int> fill(jadj_ptr.begin(), jadj_ptr.end() - 1);
    for (int j = 0; j < z.NJ; ++j) {
      if (j_info[j].y >= 0) jadj[fill[j_info[j].y]++] = (j << 1) | 0;
      jadj[fill[j_info[j].z]++] = (j << 1) | 1;
    }
  }
  // launch order: most work first (longest-processing-time first)
  std::vector<int> order(n_envs);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const long long wa = (long long)env[a].row_cap + env[a].n_dof, wb = (long long)env[b].row_cap + env[b].n_dof;
    return wa > wb;
  });

  // ---- upload ----
  hipStream_t st_ = s->stream;
  HIP_TRY(hipMemsetAsync(workspace, 0, need - 256, st_));
  auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_);
  };
  HIP_TRY(up(env_dev, env.data(), sizeof(EnvInfo) * n_envs));
  HIP_TRY(up(order_dev, order.data(), sizeof(int) * n_envs));
  HIP_TRY(up(S.r_x, r_x.data(), sizeof(float4) * z.NR));
  HIP_TRY(up(S.r_q, r_q.data(), sizeof(float4) * z.NR));
  HIP_TRY(up(S.r_v, r_v.data(), sizeof(float4) * z.NR));
  HIP_TRY(up(S.r_w, r_w.data(), sizeof(float4) * z.NR));
  HIP_TRY(up((void *)S.r_inertia, r_in.data(), sizeof(float4) * z.NR));
  HIP_TRY(up((void *)S.r_ext, r_ext.data(), sizeof(float4) * z.NR));
  HIP_TRY(up((void *)S.r_shape, r_shape.data(), sizeof(int) * z.NR));
  HIP_TRY(up(S.p_x, p_x.data(), sizeof(float4) * z.NP));
  HIP_TRY(up(S.p_v, p_v.data(), sizeof(float4) * z.NP));
  HIP_TRY(up((void *)S.p_m, p_m.data(), sizeof(float) * z.NP));
  HIP_TRY(up((void *)S.feat, feat.data(), sizeof(int2) * z.NF));
  HIP_TRY(up((void *)S.t_ids, t_ids.data(), sizeof(int4) * z.NT));
  HIP_TRY(up((void *)S.t_Dminv, t_Dminv.data(), sizeof(float) * 9 * (size_t)z.NT));
  HIP_TRY(up((void *)S.t_mat, t_mat.data(), sizeof(float4) * z.NT));
  HIP_TRY(up((void *)S.j_info, j_info.data(), sizeof(int4) * z.NJ));
  HIP_TRY(up((void *)S.j_frame, j_frame.data(), sizeof(float4) * 6 * (size_t)z.NJ));
  HIP_TRY(up((void *)S.j_drive, j_drive.data(), sizeof(float4) * 2 * (size_t)z.NJ));
  HIP_TRY(up((void *)S.p_tadj_ptr, tadj_ptr.data(), sizeof(int) * (z.NP + 1)));
  HIP_TRY(up((void *)S.p_tadj, tadj.data(), sizeof(int) * z.NTADJ));
  HIP_TRY(up((void *)S.t_dst, t_dst.data(), sizeof(int4) * z.NT));
  {  // the same indices packed to 16 bits per field, env-local, for the one-pass PCR
    std::vector<uint4> t_loc(std::max(z.NT, 1));
    S.tet_loc = 1;
    for (int e = 0; e < n_envs && S.tet_loc; ++e) {
      const EnvInfo &E = env[e];
      const int abase = tadj_ptr[E.par_off];
      for (int t = E.tet_off; t < E.tet_off + E.n_tet; ++t) {
        const int id[4] = {t_ids[t].x, t_ids[t].y, t_ids[t].z, t_ids[t].w};
        const int ds[4] = {t_dst[t].x, t_dst[t].y, t_dst[t].z, t_dst[t].w};
        unsigned w[4];
        for (int k = 0; k < 4; ++k) {
          const int l = id[k] - E.par_off, d = ds[k] - abase;
          if (l < 0 || l > 0xffff || d < 0 || d > 0xffff) S.tet_loc = 0;
          w[k] = (unsigned)(l & 0xffff) | ((unsigned)(d & 0xffff) << 16);
        }
        t_loc[t] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    HIP_TRY(up((void *)S.t_loc, t_loc.data(), sizeof(uint4) * z.NT));
  }
  HIP_TRY(up((void *)S.r_jadj_ptr, jadj_ptr.data(), sizeof(int) * (z.NR + 1)));
  HIP_TRY(up((void *)S.r_jadj, jadj.data(), sizeof(int) * z.NJADJ));
  HIP_TRY(up((void *)S.dev, &S, sizeof(DevScene)));  // the table itself, for the Newton kernel
  HIP_TRY(hipStreamSynchronize(st_));

  s->env = env;
  s->order = order;
  s->desc_sizes.assign(envs, envs + n_envs);
  for (auto &d : s->desc_sizes) {
    d.rigid_mass = d.rigid_inertia = d.rigid_x = d.rigid_q = d.rigid_v = d.rigid_w = d.rigid_extent = nullptr;
    d.rigid_shape = nullptr;
    d.particle_x = d.particle_v = d.particle_rest = d.particle_mass = nullptr;
    d.tet_ids = nullptr; d.tet_material = nullptr;
    d.joint_type = d.joint_body = nullptr;
    d.joint_anchor = d.joint_axis = d.joint_ref = d.joint_drive = nullptr;
  }
  // default schedule.  Large batches of heavy envs, in launch order (decreasing work):
  // the heaviest 3/8 of the envs with 1024 threads each, the next 3/8 with 512, the
  // lightest quarter with 128 (measured best on the uneven 4096-env batch with tet
  // blocks: 1185 ms per step against 1191 with 1/2 at 512 and 1/8 at 128, and 1206 with
  // the light quarter at 256).  "Heavy" counts the rows and DOFs an env always has
  // (joints, tets, bodies), not its contact capacity, which is mostly unused: when the
  // env at 3/8 of the order has fewer than 1024 of them, a large batch is one launch of
  // 128 threads per env (the same batch without tets: 18.7 ms per step against 35.5 ms
  // with the three buckets, 19.5 at 64 threads, 21.5 at 256).  Batches with linear tets
  // run the extended instantiation, which spills at 1024 threads: three quarters at 512
  // and a quarter at 128 (the batch with linear tet blocks: 1644 ms per step against
  // 1863 with the three buckets, 1652 all at 512).  Small batches: one launch with the
  // block size from the largest env.
  auto fixed_rows = [&](const EnvInfo &E) {
    return 6 * E.n_jnt + (E.tet_model == NSN_TET_LINEAR ? 6 : 3) * E.n_tet + 6 * E.n_rig + 3 * E.n_par;
  };
  if (n_envs >= 1024 && fixed_rows(env[order[3 * (n_envs / 8)]]) >= 1024 && z.any_linear) {
    const int a = 3 * (n_envs / 4);
    s->buckets = {Bucket{0, a, 512, 0}, Bucket{a, n_envs - a, 128, 0}};
  } else if (n_envs >= 1024 && fixed_rows(env[order[3 * (n_envs / 8)]]) >= 1024) {
    const int a1 = 3 * (n_envs / 8), a2 = 3 * (n_envs / 4);
    s->buckets = {Bucket{0, a1, 1024, 0}, Bucket{a1, a2 - a1, 512, 0}, Bucket{a2, n_envs - a2, 128, 0}};
  } else if (n_envs >= 1024) {
    s->buckets = {Bucket{0, n_envs, 128, 0}};
  } else {
    int max_el = 0;
    for (auto &E : env) max_el = std::max(max_el, E.n_jnt + E.n_tet + E.max_con + E.n_rig + E.n_par);
    int block = 64;
    while (block < 256 && block * 4 < max_el) block *= 2;
    s->buckets = {Bucket{0, n_envs, block, 0}};
  }
  set_bucket_lds(s);
  s->use_graphs = s->stream != nullptr;
  *out = s;
  return NSN_OK;
}

nsn_status nsn_destroy_scene(nsn_scene s) {
  if (!s) return NSN_OK;
  delete s;
  return NSN_OK;
}

nsn_status nsn_set_params(nsn_scene s, const nsn_solver_params *p) {
  if (!s || !p) return fail(NSN_EINVAL, "nsn_set_params: bad arguments");
  if (!params_ok(p)) return fail(NSN_EINVAL, "bad solver parameters");
  if ((p->islands && !s->reserved.islands) || (p->line_search && !s->reserved.line_search))
    return fail(NSN_ESTATE, "islands / line search need a workspace sized with them (nsn_query_workspace params)");
  if (learned_warm(p->warm) && !s->S.have_mlp) return fail(NSN_ESTATE, "learned warm start needs nsn_set_warm_start_model first");
  s->p = *p;
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return NSN_OK;
}

// Buckets after the first run on side streams forked from the scene stream, so the
// launches of different size classes overlap; the scene stream joins them.
static hipError_t ensure_side_streams(nsn_scene s, size_t nb) {
  while (s->side.size() + 1 < nb) {
    hipStream_t st;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    s->side.push_back(st);
  }
  while (s->ev.size() < 2 * nb) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    s->ev.push_back(ev);
  }
  return hipSuccess;
}

// Everything a step's launches need that is not a stream operation -- the side streams
// and events of the buckets, the dynamic-LDS limit of each bucket's kernel -- set up
// before a capture begins (such calls are not allowed inside one).
static hipError_t prime_step(nsn_scene s, const StepArgs &a) {
  if (s->stream != nullptr && s->buckets.size() > 1) {
    hipError_t e = ensure_side_streams(s, s->buckets.size());
    if (e != hipSuccess) return e;
  }
  for (const Bucket &b : s->buckets) {
    hipError_t e = launch_newton(s->S, a, b.block, b.first, b.count, b.lds_floats, b.lds_mode, s->pcr_form, s->stream,
                                 kLaunchAttr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Enqueues one step; with `capturing` set only stream operations are issued (prime_step
// has run first).
static hipError_t enqueue_step(nsn_scene s, const StepArgs &a, bool capturing = false) {
  const int what = capturing ? kLaunchRun : (kLaunchAttr | kLaunchRun);
  hipError_t e = launch_prepare(s->S, a, s->want_features || learned_warm(a.p.warm), s->stream);
  if (e != hipSuccess) return e;
  if (learned_warm(a.p.warm)) {
    e = launch_warm_mlp(s->S, a.p.warm == NSN_WARM_HYBRID, s->stream);
    if (e != hipSuccess) return e;
  }
  const size_t nb = s->buckets.size();
  if (s->stream == nullptr || nb == 1) {
    for (const Bucket &b : s->buckets) {
      e = launch_newton(s->S, a, b.block, b.first, b.count, b.lds_floats, b.lds_mode, s->pcr_form, s->stream, what);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (s->side.size() + 1 < nb || s->ev.size() < 2 * nb) {
    if (capturing) return hipErrorStreamCaptureUnsupported;  // prime_step creates them
    e = ensure_side_streams(s, nb);
    if (e != hipSuccess) return e;
  }
  e = hipEventRecord(s->ev[0], s->stream);
  if (e != hipSuccess) return e;
  for (size_t i = 1; i < nb; ++i) {
    e = hipStreamWaitEvent(s->side[i - 1], s->ev[0], 0);
    if (e != hipSuccess) return e;
  }
  for (size_t i = 0; i < nb; ++i) {
    const Bucket &b = s->buckets[i];
    e = launch_newton(s->S, a, b.block, b.first, b.count, b.lds_floats, b.lds_mode, s->pcr_form,
                      i == 0 ? s->stream : s->side[i - 1], what);
    if (e != hipSuccess) return e;
  }
  for (size_t i = 1; i < nb; ++i) {
    e = hipEventRecord(s->ev[i], s->side[i - 1]);
    if (e != hipSuccess) return e;
    e = hipStreamWaitEvent(s->stream, s->ev[i], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

nsn_status nsn_step(nsn_scene s, double h, int32_t newton_iters, int32_t cr_iters, double tol,
                    nsn_step_stats *stats) {
  if (!s) return fail(NSN_EINVAL, "nsn_step: null scene");
  if (!(h > 0.0) || newton_iters < 0 || cr_iters < 0 || !(tol >= 0.0)) return fail(NSN_EINVAL, "nsn_step: bad h, iteration counts or tol");
  if (learned_warm(s->p.warm) && !s->S.have_mlp) return fail(NSN_ESTATE, "learned warm start needs nsn_set_warm_start_model first");
  StepArgs a;
  a.h = (float)h;
  a.newton_iters = newton_iters;
  a.cr_iters = cr_iters;
  a.tol = (float)tol;
  a.dump_k = -1;
  a.p = s->p;
  s->dumped_k = -1;
  if (!s->use_graphs) {
    HIP_TRY(enqueue_step(s, a));
    return stats ? nsn_get_stats(s, stats) : NSN_OK;
  }
  GraphKey k{a.h, newton_iters, cr_iters, a.tol};
  auto it = s->graphs.find(k);
  if (it == s->graphs.end()) {
    hipGraph_t graph;
    HIP_TRY(prime_step(s, a));
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = enqueue_step(s, a, true);
    hipError_t ce = hipStreamEndCapture(s->stream, &graph);
    if (le != hipSuccess) return fail(NSN_EDEVICE, std::string("capture: ") + hipGetErrorString(le));
    if (ce != hipSuccess) return fail(NSN_EDEVICE, std::string("end capture: ") + hipGetErrorString(ce));
    hipGraphExec_t exec;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(NSN_EDEVICE, std::string("instantiate: ") + hipGetErrorString(ie));
    it = s->graphs.emplace(k, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, s->stream));
  return stats ? nsn_get_stats(s, stats) : NSN_OK;
}

nsn_status nsn_get_stats(nsn_scene s, nsn_step_stats *out) {
  if (!s || !out) return fail(NSN_EINVAL, "nsn_get_stats: bad arguments");
  HIP_TRY(hipMemcpyAsync(out, s->S.stats, sizeof(nsn_step_stats) * s->S.n_envs, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NSN_OK;
}

static nsn_status check_env(nsn_scene s, int env) {
  if (!s) return fail(NSN_EINVAL, "null scene");
  if (env < 0 || env >= s->S.n_envs) return fail(NSN_EINVAL, "env index out of range");
  return NSN_OK;
}

static hipError_t d2h_f4(float *dst, const float4 *src, int n, int ncomp, hipStream_t st) {
  if (!dst || n <= 0) return hipSuccess;
  std::vector<float4> tmp(n);
  hipError_t e = hipMemcpyAsync(tmp.data(), src, sizeof(float4) * n, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    const float v[4] = {tmp[i].x, tmp[i].y, tmp[i].z, tmp[i].w};
    for (int k = 0; k < ncomp; ++k) dst[ncomp * i + k] = v[k];
  }
  return hipSuccess;
}

nsn_status nsn_read_state(nsn_scene s, int32_t env, float *rigid_x, float *rigid_q, float *rigid_v,
                          float *rigid_w, float *particle_x, float *particle_v, double *time) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  const EnvInfo &E = s->env[env];
  const DevScene &S = s->S;
  HIP_TRY(d2h_f4(rigid_x, S.r_x + E.rig_off, E.n_rig, 3, s->stream));
  HIP_TRY(d2h_f4(rigid_q, S.r_q + E.rig_off, E.n_rig, 4, s->stream));
  HIP_TRY(d2h_f4(rigid_v, S.r_v + E.rig_off, E.n_rig, 3, s->stream));
  HIP_TRY(d2h_f4(rigid_w, S.r_w + E.rig_off, E.n_rig, 3, s->stream));
  HIP_TRY(d2h_f4(particle_x, S.p_x + E.par_off, E.n_par, 3, s->stream));
  HIP_TRY(d2h_f4(particle_v, S.p_v + E.par_off, E.n_par, 3, s->stream));
  if (time) {
    HIP_TRY(hipMemcpyAsync(time, S.time + env, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return NSN_OK;
}

static hipError_t h2d_f4(float4 *dst, const float *src, int n, int ncomp, hipStream_t st, bool normalize_q) {
  if (!src || n <= 0) return hipSuccess;
  std::vector<float4> tmp(n);
  for (int i = 0; i < n; ++i) {
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < ncomp; ++k) v[k] = src[ncomp * i + k];
    if (normalize_q) {
      const float l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
      for (int k = 0; k < 4; ++k) v[k] /= l;
    }
    tmp[i] = make_float4(v[0], v[1], v[2], v[3]);
  }
  hipError_t e = hipMemcpyAsync(dst, tmp.data(), sizeof(float4) * n, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);  // the staging vector dies on return
}

nsn_status nsn_write_state(nsn_scene s, int32_t env, const float *rigid_x, const float *rigid_q,
                           const float *rigid_v, const float *rigid_w, const float *particle_x,
                           const float *particle_v, const double *time) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  const EnvInfo &E = s->env[env];
  DevScene &S = s->S;
  const nsn_env_desc &d = s->desc_sizes[env];
  (void)d;
  HIP_TRY(h2d_f4(S.r_x + E.rig_off, rigid_x, E.n_rig, 3, s->stream, false));
  HIP_TRY(h2d_f4(S.r_q + E.rig_off, rigid_q, E.n_rig, 4, s->stream, true));
  // static bodies keep zero velocity
  if (rigid_v || rigid_w) {
    std::vector<float4> inr(E.n_rig);
    HIP_TRY(hipMemcpyAsync(inr.data(), S.r_inertia + E.rig_off, sizeof(float4) * E.n_rig, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<float> v(rigid_v ? rigid_v : rigid_w, (rigid_v ? rigid_v : rigid_w) + 3 * E.n_rig);
    if (rigid_v) {
      std::vector<float> vv(rigid_v, rigid_v + 3 * E.n_rig);
      for (int i = 0; i < E.n_rig; ++i)
        if (inr[i].w == 0.f) vv[3 * i] = vv[3 * i + 1] = vv[3 * i + 2] = 0.f;
      HIP_TRY(h2d_f4(S.r_v + E.rig_off, vv.data(), E.n_rig, 3, s->stream, false));
    }
    if (rigid_w) {
      std::vector<float> ww(rigid_w, rigid_w + 3 * E.n_rig);
      for (int i = 0; i < E.n_rig; ++i)
        if (inr[i].w == 0.f) ww[3 * i] = ww[3 * i + 1] = ww[3 * i + 2] = 0.f;
      HIP_TRY(h2d_f4(S.r_w + E.rig_off, ww.data(), E.n_rig, 3, s->stream, false));
    }
  }
  HIP_TRY(h2d_f4(S.p_x + E.par_off, particle_x, E.n_par, 3, s->stream, false));
  HIP_TRY(h2d_f4(S.p_v + E.par_off, particle_v, E.n_par, 3, s->stream, false));
  if (time) {
    HIP_TRY(hipMemcpyAsync(S.time + env, time, sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return NSN_OK;
}

nsn_status nsn_state_bytes(nsn_scene s, size_t *bytes) {
  if (!s || !bytes) return fail(NSN_EINVAL, "nsn_state_bytes: null argument");
  *bytes = for_each_state_block(s->S, [](char *, size_t, size_t) {});
  return NSN_OK;
}

nsn_status nsn_save_state(nsn_scene s, void *buf) {
  if (!s || !buf) return fail(NSN_EINVAL, "nsn_save_state: null argument");
  hipError_t e = hipSuccess;
  for_each_state_block(s->S, [&](char *p, size_t off, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync((char *)buf + off, p, bytes, hipMemcpyDeviceToDevice, s->stream);
  });
  HIP_TRY(e);
  return NSN_OK;
}

nsn_status nsn_load_state(nsn_scene s, const void *buf) {
  if (!s || !buf) return fail(NSN_EINVAL, "nsn_load_state: null argument");
  hipError_t e = hipSuccess;
  for_each_state_block(s->S, [&](char *p, size_t off, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(p, (const char *)buf + off, bytes, hipMemcpyDeviceToDevice, s->stream);
  });
  HIP_TRY(e);
  s->dumped_k = -1;  // the working arrays no longer hold a dump step's iterate
  return NSN_OK;
}

nsn_status nsn_read_contacts(nsn_scene s, int32_t env, int32_t cap, int32_t *n, int32_t *keys, int32_t *bodies,
                             float *geom, float *lam) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  if (!n || cap < 0) return fail(NSN_EINVAL, "nsn_read_contacts: bad arguments");
  const EnvInfo &E = s->env[env];
  const DevScene &S = s->S;
  int nc = 0;
  HIP_TRY(hipMemcpyAsync(&nc, S.n_con + env, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *n = nc;
  const int m = std::min(nc, cap);
  if (m <= 0) return NSN_OK;
  std::vector<int> k(m);
  std::vector<int2> b(m);
  std::vector<float4> nn(m), aa(m), bb(m), ll(m);
  HIP_TRY(hipMemcpyAsync(k.data(), S.c_key + E.con_off, sizeof(int) * m, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(b.data(), S.c_body + E.con_off, sizeof(int2) * m, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(nn.data(), S.c_n + E.con_off, sizeof(float4) * m, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(aa.data(), S.c_aL + E.con_off, sizeof(float4) * m, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(bb.data(), S.c_bL + E.con_off, sizeof(float4) * m, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(ll.data(), S.c_prev_lam + E.con_off, sizeof(float4) * m, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int i = 0; i < m; ++i) {
    if (keys) keys[i] = k[i];
    if (bodies) { bodies[2 * i] = b[i].x; bodies[2 * i + 1] = b[i].y; }
    if (geom) {
      float *g = geom + 10 * i;
      g[0] = nn[i].x; g[1] = nn[i].y; g[2] = nn[i].z;
      g[3] = aa[i].x; g[4] = aa[i].y; g[5] = aa[i].z;
      g[6] = bb[i].x; g[7] = bb[i].y; g[8] = bb[i].z;
      g[9] = nn[i].w;
    }
    if (lam) { lam[3 * i] = ll[i].x; lam[3 * i + 1] = ll[i].y; lam[3 * i + 2] = ll[i].z; }
  }
  return NSN_OK;
}

nsn_status nsn_read_lambda(nsn_scene s, int32_t env, int32_t cap, int32_t *n, float *lam) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  if (!n || cap < 0) return fail(NSN_EINVAL, "nsn_read_lambda: bad arguments");
  const EnvInfo &E = s->env[env];
  int nc = 0;
  HIP_TRY(hipMemcpyAsync(&nc, s->S.n_con + env, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const int rows = 6 * E.n_jnt + (E.tet_model == NSN_TET_LINEAR ? 6 : 3) * E.n_tet + 3 * nc;
  *n = rows;
  const int m = std::min(rows, cap);
  if (m > 0 && lam) {
    HIP_TRY(hipMemcpyAsync(lam, s->S.row_lam + E.row_off, sizeof(float) * m, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return NSN_OK;
}

nsn_status nsn_set_warm_start_model(nsn_scene s, const float *blob, int64_t n) {
  if (!s || !blob || n != kMlpBlob) return fail(NSN_EINVAL, "warm-start model must hold " + std::to_string(kMlpBlob) + " floats");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(blob[i])) return fail(NSN_EINVAL, "warm-start model has non-finite values");
  HIP_TRY(hipMemcpyAsync((void *)s->S.mlp, blob, sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->S.have_mlp = 1;
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return NSN_OK;
}

nsn_status nsn_read_features(nsn_scene s, int32_t env, int32_t cap, int32_t *n, float *feat) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  if (!n || cap < 0) return fail(NSN_EINVAL, "nsn_read_features: bad arguments");
  if (!s->want_features && !learned_warm(s->p.warm))
    return fail(NSN_ESTATE, "features are only computed after nsn_enable_features(scene, 1) or in learned mode");
  const EnvInfo &E = s->env[env];
  int nc = 0;
  HIP_TRY(hipMemcpyAsync(&nc, s->S.n_con + env, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *n = nc;
  const int m = std::min(nc, cap);
  if (m > 0 && feat) {
    HIP_TRY(hipMemcpyAsync(feat, s->S.c_feat + (size_t)E.con_off * 12, sizeof(float) * 12 * m, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return NSN_OK;
}

// ---- extras used by the Python layer (declared in include/nsn_ext.h) ----
nsn_status nsn_enable_features(nsn_scene s, int32_t on) {
  if (!s) return fail(NSN_EINVAL, "null scene");
  s->want_features = on ? 1 : 0;
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return NSN_OK;
}

nsn_status nsn_set_use_graphs(nsn_scene s, int32_t on) {
  if (!s) return fail(NSN_EINVAL, "null scene");
  s->use_graphs = on && s->stream != nullptr;
  return NSN_OK;
}

nsn_status nsn_get_env_order(nsn_scene s, int32_t *order) {
  if (!s || !order) return fail(NSN_EINVAL, "bad arguments");
  std::copy(s->order.begin(), s->order.end(), order);
  return NSN_OK;
}

nsn_status nsn_set_schedule(nsn_scene s, int32_t n_buckets, const int32_t *first, const int32_t *count,
                            const int32_t *block) {
  if (!s || n_buckets < 1 || !first || !count || !block) return fail(NSN_EINVAL, "bad schedule");
  std::vector<Bucket> b;
  int expect = 0;
  for (int i = 0; i < n_buckets; ++i) {
    if (first[i] != expect || count[i] < 0) return fail(NSN_EINVAL, "schedule buckets must tile the env order");
    const int bl = block[i];
    if (bl != 64 && bl != 128 && bl != 256 && bl != 512 && bl != 1024) return fail(NSN_EINVAL, "block size must be 64..1024 (power of two)");
    b.push_back(Bucket{first[i], count[i], bl, 0, 0});
    expect += count[i];
  }
  if (expect != s->S.n_envs) return fail(NSN_EINVAL, "schedule must cover every env");
  s->buckets = b;
  set_bucket_lds(s);
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return NSN_OK;
}

nsn_status nsn_set_lds_mode(nsn_scene s, int32_t max_mode) {
  if (!s || max_mode < 0 || max_mode > 2) return fail(NSN_EINVAL, "LDS mode must be 0, 1 or 2");
  s->lds_max = max_mode;
  set_bucket_lds(s);
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return NSN_OK;
}

nsn_status nsn_get_schedule(nsn_scene s, int32_t cap, int32_t *n, int32_t *first, int32_t *count, int32_t *block) {
  if (!s || !n) return fail(NSN_EINVAL, "bad arguments");
  *n = (int)s->buckets.size();
  for (int i = 0; i < std::min<int>(cap, *n); ++i) {
    first[i] = s->buckets[i].first;
    count[i] = s->buckets[i].count;
    block[i] = s->buckets[i].block;
  }
  return NSN_OK;
}

nsn_status nsn_set_pcr_form(nsn_scene s, int32_t form) {
  if (!s || form < 0 || form > 2) return fail(NSN_EINVAL, "PCR form must be 0, 1 or 2");
  s->pcr_form = form;
  for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return NSN_OK;
}

nsn_status nsn_get_lds_modes(nsn_scene s, int32_t cap, int32_t *n, int32_t *mode) {
  if (!s || !n || (cap > 0 && !mode)) return fail(NSN_EINVAL, "bad arguments");
  *n = (int)s->buckets.size();
  for (int i = 0; i < std::min<int>(cap, *n); ++i) mode[i] = s->buckets[i].lds_mode;
  return NSN_OK;
}

nsn_status nsn_read_accumulators(nsn_scene s, nsn_accum *out) {
  if (!s || !out) return fail(NSN_EINVAL, "bad arguments");
  HIP_TRY(hipMemcpyAsync(out, s->S.acc, sizeof(nsn_accum) * s->S.n_envs, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NSN_OK;
}

nsn_status nsn_reset_accumulators(nsn_scene s) {
  if (!s) return fail(NSN_EINVAL, "null scene");
  HIP_TRY(hipMemsetAsync(s->S.acc, 0, sizeof(nsn_accum) * s->S.n_envs, s->stream));
  return NSN_OK;
}

nsn_status nsn_read_kernel_times(nsn_scene s, int32_t cap, int32_t *n, double *ms) {
  if (!s || !n || cap < 0) return fail(NSN_EINVAL, "bad arguments");
  int tick = 0;
  std::vector<unsigned long long> ts(2 * kTimingRing);
  HIP_TRY(hipMemcpyAsync(&tick, s->S.tick, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(ts.data(), s->S.ts, sizeof(unsigned long long) * 2 * kTimingRing, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  int dev = 0, rate_khz = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
  if (rate_khz <= 0) return fail(NSN_EDEVICE, "wall clock rate unavailable");
  const int avail = std::min(tick, kTimingRing);
  const int m = std::min(avail, cap);
  *n = m;
  for (int i = 0; i < m; ++i) {
    const int step = tick - m + 1 + i;
    const int slot = step % kTimingRing;
    const unsigned long long a = ts[2 * slot], b = ts[2 * slot + 1];
    ms[i] = (b > a) ? (double)(b - a) / (double)rate_khz : 0.0;
  }
  return NSN_OK;
}

// device pointer of the per-env stats array (for asynchronous readers)
nsn_status nsn_stats_device_ptr(nsn_scene s, void **ptr) {
  if (!s || !ptr) return fail(NSN_EINVAL, "bad arguments");
  *ptr = s->S.stats;
  return NSN_OK;
}

nsn_status nsn_set_contacts(nsn_scene s, int32_t env, const nsn_contact *contacts, int32_t n) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  const EnvInfo &E = s->env[env];
  if (n < 0 || n > E.max_con || (n > 0 && !contacts))
    return fail(NSN_EINVAL, "nsn_set_contacts: count must be in [0, max_contacts]");
  std::vector<int> key(std::max(n, 1));
  std::vector<int2> body(std::max(n, 1));
  std::vector<float4> nrm(std::max(n, 1)), aL(std::max(n, 1)), bL(std::max(n, 1));
  const int nb = E.n_rig + E.n_par;
  for (int i = 0; i < n; ++i) {
    const nsn_contact &c = contacts[i];
    const std::string at = "nsn_set_contacts: contact " + std::to_string(i) + ": ";
    if (i > 0 && !(c.key > contacts[i - 1].key)) return fail(NSN_EINVAL, at + "keys must be strictly ascending");
    if (i > 0 && c.body_a < contacts[i - 1].body_a) return fail(NSN_EINVAL, at + "feature bodies must be non-decreasing");
    if (c.body_a < 0 || c.body_a >= nb) return fail(NSN_EINVAL, at + "bad feature body");
    if (c.body_b < -1 || c.body_b >= E.n_rig || c.body_b == c.body_a) return fail(NSN_EINVAL, at + "bad target body");
    if (c.body_b == -1 && !E.ground) return fail(NSN_EINVAL, at + "the env has no ground plane");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c.normal[k]) || !std::isfinite(c.a_local[k]) || !std::isfinite(c.b_local[k]))
        return fail(NSN_EINVAL, at + "non-finite geometry");
    if (!std::isfinite(c.thickness)) return fail(NSN_EINVAL, at + "non-finite thickness");
    key[i] = c.key;
    body[i] = make_int2(c.body_a, c.body_b);
    nrm[i] = make_float4(c.normal[0], c.normal[1], c.normal[2], c.thickness);
    const bool particle = c.body_a >= E.n_rig;
    aL[i] = particle ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(c.a_local[0], c.a_local[1], c.a_local[2], 0.f);
    bL[i] = make_float4(c.b_local[0], c.b_local[1], c.b_local[2], 0.f);
  }
  const DevScene &S = s->S;
  const hipStream_t st_ = s->stream;
  if (n > 0) {
    HIP_TRY(hipMemcpyAsync(S.c_key + E.con_off, key.data(), sizeof(int) * n, hipMemcpyHostToDevice, st_));
    HIP_TRY(hipMemcpyAsync(S.c_body + E.con_off, body.data(), sizeof(int2) * n, hipMemcpyHostToDevice, st_));
    HIP_TRY(hipMemcpyAsync(S.c_n + E.con_off, nrm.data(), sizeof(float4) * n, hipMemcpyHostToDevice, st_));
    HIP_TRY(hipMemcpyAsync(S.c_aL + E.con_off, aL.data(), sizeof(float4) * n, hipMemcpyHostToDevice, st_));
    HIP_TRY(hipMemcpyAsync(S.c_bL + E.con_off, bL.data(), sizeof(float4) * n, hipMemcpyHostToDevice, st_));
  }
  const int flag = n + 1;
  HIP_TRY(hipMemcpyAsync(S.c_inject + env, &flag, sizeof(int), hipMemcpyHostToDevice, st_));
  HIP_TRY(hipStreamSynchronize(st_));  // the staging vectors die on return
  return NSN_OK;
}

nsn_status nsn_dump_iteration(nsn_scene s, double h, int32_t k, int32_t cr_iters) {
  if (!s) return fail(NSN_EINVAL, "nsn_dump_iteration: null scene");
  if (!(h > 0.0) || k < 0 || cr_iters < 0) return fail(NSN_EINVAL, "nsn_dump_iteration: bad h, k or cr_iters");
  if (s->p.line_search) return fail(NSN_EUNSUPPORTED, "nsn_dump_iteration: not with line search");
  if (learned_warm(s->p.warm) && !s->S.have_mlp) return fail(NSN_ESTATE, "learned warm start needs nsn_set_warm_start_model first");
  StepArgs a;
  a.h = (float)h;
  a.newton_iters = k + 1;
  a.cr_iters = cr_iters;
  a.tol = 0.f;
  a.dump_k = k;
  a.p = s->p;
  a.p.watchdog = 0;  // the watchdog's slot holds iterate k-1
  HIP_TRY(enqueue_step(s, a));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->dumped_k = k;
  return NSN_OK;
}

nsn_status nsn_read_iteration(nsn_scene s, int32_t env, int32_t field, int32_t cap, int32_t *n, float *out) {
  nsn_status st = check_env(s, env);
  if (st) return st;
  if (!n || cap < 0 || (cap > 0 && !out)) return fail(NSN_EINVAL, "nsn_read_iteration: bad arguments");
  if (field < 0 || field >= NSN_IT_NFIELDS) return fail(NSN_EINVAL, "nsn_read_iteration: unknown field");
  if (s->dumped_k < 0) return fail(NSN_ESTATE, "nsn_read_iteration: no dump step since the last nsn_step");
  const bool prev = field >= NSN_IT_PREV_LAM;
  if (prev && s->dumped_k < 1) return fail(NSN_ESTATE, "nsn_read_iteration: iterate k-1 needs k >= 1");
  const EnvInfo &E = s->env[env];
  const DevScene &S = s->S;
  const hipStream_t st_ = s->stream;
  int nc = 0;
  HIP_TRY(hipMemcpyAsync(&nc, S.n_con + env, sizeof(int), hipMemcpyDeviceToHost, st_));
  HIP_TRY(hipStreamSynchronize(st_));
  const int tet_rows = E.tet_model == NSN_TET_LINEAR ? 6 : 3;
  const int rows = 6 * E.n_jnt + tet_rows * E.n_tet + 3 * nc;
  std::vector<float> v;
  auto rowf = [&](const float *src) -> hipError_t {
    v.resize(rows);
    if (!rows) return hipSuccess;
    return hipMemcpyAsync(v.data(), src + E.row_off, sizeof(float) * rows, hipMemcpyDeviceToHost, st_);
  };
  auto f4 = [&](const float4 *src, int count, int ncomp) -> hipError_t {
    std::vector<float4> t(std::max(count, 1));
    v.resize((size_t)ncomp * count);
    if (!count) return hipSuccess;
    hipError_t e = hipMemcpyAsync(t.data(), src, sizeof(float4) * count, hipMemcpyDeviceToHost, st_);
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    for (int i = 0; i < count; ++i) {
      const float c4[4] = {t[i].x, t[i].y, t[i].z, t[i].w};
      for (int q = 0; q < ncomp; ++q) v[(size_t)ncomp * i + q] = c4[q];
    }
    return e;
  };
  // body-space velocities: 6 per rigid body (from a 6-float array), 3 per particle (float4)
  auto bodyu = [&](const float *ru, const float4 *pu) -> hipError_t {
    std::vector<float> r(std::max(6 * E.n_rig, 1));
    std::vector<float4> p(std::max(E.n_par, 1));
    hipError_t e = hipSuccess;
    if (E.n_rig) e = hipMemcpyAsync(r.data(), ru + 6 * (size_t)E.rig_off, sizeof(float) * 6 * E.n_rig, hipMemcpyDeviceToHost, st_);
    if (e == hipSuccess && E.n_par) e = hipMemcpyAsync(p.data(), pu + E.par_off, sizeof(float4) * E.n_par, hipMemcpyDeviceToHost, st_);
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    v.assign(r.begin(), r.begin() + 6 * E.n_rig);
    for (int i = 0; i < E.n_par; ++i) { v.push_back(p[i].x); v.push_back(p[i].y); v.push_back(p[i].z); }
    return e;
  };
  switch (field) {
    case NSN_IT_LAM: HIP_TRY(rowf(S.row_lam)); break;
    case NSN_IT_ERR: HIP_TRY(rowf(S.row_err)); break;
    case NSN_IT_CDIAG: HIP_TRY(rowf(S.row_C)); break;
    case NSN_IT_P: HIP_TRY(rowf(S.row_P)); break;
    case NSN_IT_B: HIP_TRY(rowf(S.row_b)); break;
    case NSN_IT_AZ: HIP_TRY(rowf(S.row_dump)); break;
    case NSN_IT_DLAM: HIP_TRY(rowf(S.row_x)); break;
    case NSN_IT_PREV_LAM: HIP_TRY(rowf(S.row_lam_best)); break;
    case NSN_IT_TETC: {
      v.resize(6 * (size_t)E.n_tet);
      for (int q = 0; q < 6 && E.n_tet; ++q) {
        std::vector<float> t(E.n_tet);
        HIP_TRY(hipMemcpyAsync(t.data(), S.t_E + (size_t)q * S.NT + E.tet_off, sizeof(float) * E.n_tet,
                               hipMemcpyDeviceToHost, st_));
        HIP_TRY(hipStreamSynchronize(st_));
        for (int i = 0; i < E.n_tet; ++i) v[6 * (size_t)i + q] = t[i];
      }
      break;
    }
    case NSN_IT_ALPHA:
    case NSN_IT_ACTIVE: {
      // the dumped iteration's half of the ping-pong pair
      const int buf = s->dumped_k & 1;
      v.resize(nc);
      if (nc && field == NSN_IT_ALPHA) {
        HIP_TRY(hipMemcpyAsync(v.data(), S.c_alpha + (size_t)buf * S.NC + E.con_off, sizeof(float) * nc,
                               hipMemcpyDeviceToHost, st_));
      } else if (nc) {
        std::vector<int> t(nc);
        HIP_TRY(hipMemcpyAsync(t.data(), S.c_active + (size_t)buf * S.NC + E.con_off, sizeof(int) * nc,
                               hipMemcpyDeviceToHost, st_));
        HIP_TRY(hipStreamSynchronize(st_));
        for (int i = 0; i < nc; ++i) v[i] = (float)t[i];
      }
      break;
    }
    case NSN_IT_G:
      v.resize(E.n_dof);
      if (E.n_dof) HIP_TRY(hipMemcpyAsync(v.data(), S.g + E.dof_off, sizeof(float) * E.n_dof, hipMemcpyDeviceToHost, st_));
      break;
    case NSN_IT_U: HIP_TRY(bodyu(S.r_u, S.p_u)); break;
    case NSN_IT_PREV_U: HIP_TRY(bodyu(S.r_u_best, S.p_u_best)); break;
    case NSN_IT_HDIAG: HIP_TRY(f4(S.p_H + E.par_off, E.n_par, 3)); break;
    case NSN_IT_RX: HIP_TRY(f4(S.r_x + E.rig_off, E.n_rig, 3)); break;
    case NSN_IT_RQ: HIP_TRY(f4(S.r_q + E.rig_off, E.n_rig, 4)); break;
    case NSN_IT_PX: HIP_TRY(f4(S.p_x + E.par_off, E.n_par, 3)); break;
    case NSN_IT_PREV_RX: HIP_TRY(f4(S.r_x_best + E.rig_off, E.n_rig, 3)); break;
    case NSN_IT_PREV_RQ: HIP_TRY(f4(S.r_q_best + E.rig_off, E.n_rig, 4)); break;
    case NSN_IT_PREV_PX: HIP_TRY(f4(S.p_x_best + E.par_off, E.n_par, 3)); break;
  }
  HIP_TRY(hipStreamSynchronize(st_));
  *n = (int)v.size();
  const int m = std::min<int>(cap, (int)v.size());
  if (m > 0) std::copy(v.begin(), v.begin() + m, out);
  return NSN_OK;
}

}  // extern "C"
