/*
 * nsn.h -- C ABI of the MI355X non-smooth Newton library (libnsn.so).
 *
 * The library steps batches of independent environments ("envs") of rigid bodies,
 * particles (tetrahedral FEM nodes), joints and frictional contacts with the
 * non-smooth Newton method of Macklin et al., "Non-Smooth Newton Methods for
 * Deformable Multi-Body Dynamics", TOG 38(5) 2019:
 *   - Algorithm 1 (simulation loop): collision detection once per step, then N
 *     Newton iterations, each with an assembly and M linear (PCR) iterations;
 *   - Sec. 5 (implicit time stepping) and Sec. 6 (Newton system, Schur complement
 *     [J H^-1 J^T + C] dlambda = (1/h)(J H^-1 g - err));
 *   - Sec. 4 / App. A (Fischer-Burmeister or minimum-map NCP functions, friction
 *     compliance W), Sec. 7 (complementarity preconditioner r);
 *   - Sec. 8 (damped step t, zero start, Jacobi-preconditioned conjugate residual,
 *     diagonal geometric stiffness, eps regularisation);
 *   - Sec. 9 / App. B (generalised compliance of stable neo-Hookean tets in
 *     principal stretches, particles, rigid bodies with quaternions); Sec. 9.2
 *     (linear Hookean tets on six strains, constant compliance);
 *   - options around the method: line search on the merit (Sec. 8.1), PCG as the
 *     comparison solver (Sec. 8.2), one PCR per island of an env (Sec. 11), a
 *     learned contact warm start.
 *
 * Conventions: SI units; z up; quaternions (w,x,y,z); angular velocities in the
 * world frame; all host arrays are float32 and row-major unless stated.
 *
 * Memory ownership: the caller owns ALL device memory.  nsn_query_workspace()
 * returns the size of one device buffer that the caller allocates (e.g. a torch
 * uint8 tensor) and passes to nsn_create_scene(); the library sub-allocates it and
 * never calls hipMalloc.  Host descriptor arrays are only read during
 * nsn_create_scene() and may be freed afterwards.  Every call that takes host
 * output arrays writes into caller-owned memory.
 *
 * Streams: every device operation of a scene is enqueued on the stream given at
 * creation (NULL = the default stream).  nsn_step() is asynchronous.  Calls that
 * return data to the host synchronise that stream first.  Calls on one scene are
 * not re-entrant; different scenes may be used from different threads.
 *
 * Errors: every function returns NSN_OK or a negative status; nsn_last_error()
 * returns a thread-local message for the last failure.  Non-convergence is NOT an
 * error: it is reported in nsn_step_stats.
 */
#ifndef NSN_H
#define NSN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsn_scene_s *nsn_scene;
typedef int32_t nsn_status;

#define NSN_OK 0
#define NSN_EINVAL (-1)       /* invalid argument or descriptor */
#define NSN_ENOMEM (-2)       /* workspace too small */
#define NSN_EDEVICE (-3)      /* a HIP runtime call failed */
#define NSN_ENONFINITE (-4)   /* non-finite state detected */
#define NSN_EUNSUPPORTED (-5) /* sizes beyond the supported limits */
#define NSN_ESTATE (-6)       /* call not valid in the current state */

/* Shapes of rigid bodies (collision geometry; Sec. 10 primitive features). */
#define NSN_SHAPE_BOX 0     /* extent = half extents */
#define NSN_SHAPE_CAPSULE 1 /* extent = (radius, half length, 0), segment on body x */
#define NSN_SHAPE_NONE 2    /* no collision geometry */

#define NSN_JOINT_REVOLUTE 0
#define NSN_JOINT_PRISMATIC 1

#define NSN_NCP_FB 0   /* Fischer-Burmeister (Sec. 4.2) */
#define NSN_NCP_MIN 1  /* minimum map (Sec. 4.1) */

#define NSN_R_IDENTITY 0   /* r = 1 */
#define NSN_R_H2 1         /* r_n = h^2, r_f = h */
#define NSN_R_H2_EFFMASS 2 /* Sec. 7 eq. rscaling: r = h^2 [J M^-1 J^T]_ii (h for friction) */

#define NSN_FEM_FULL_PROJECTED 0 /* E = (d2U/ds2)^-1 projected to positive definite */
#define NSN_FEM_DIAGONAL 1       /* diagonal approximation of E */

/* tet material model of an env (Sec. 9.2) */
#define NSN_TET_NEOHOOKEAN 0 /* stable neo-Hookean in principal stretches (App. B): 3 rows per tet */
#define NSN_TET_LINEAR 1     /* linear Hookean on six co-rotated strains: 6 rows per tet, constant
                                compliance (V_e K_e)^-1 of an isotropic K_e from (E, nu) */

#define NSN_WARM_ZERO 0    /* u0 = 0, lambda0 = 0 (Sec. 8.1) */
#define NSN_WARM_PREV 1    /* previous-step multipliers (contacts matched by key) */
#define NSN_WARM_LEARNED 2 /* contact multipliers predicted by the warm-start MLP */
#define NSN_WARM_HYBRID 3  /* previous-step multipliers for contacts whose key existed in the
                              previous step, the warm-start MLP's prediction for new ones */

/* linear solver of the Newton system (Sec. 8.2) */
#define NSN_LINEAR_PCR 0 /* preconditioned conjugate residual: the method */
#define NSN_LINEAR_PCG 1 /* preconditioned conjugate gradient: the comparison solver */

/* One environment.  Pointers are host float32/int32 arrays, sizes as noted.
 * A rigid body with mass 0 is a static obstacle.  Particles take their mass from
 * the tets that use them (rho V_e / 4 each) plus particle_mass.  Tet rest shapes
 * come from particle_rest. */
typedef struct {
  int32_t n_rigid;
  const float *rigid_mass;    /* [n_rigid] */
  const float *rigid_inertia; /* [n_rigid*3] principal body-frame inertia */
  const float *rigid_x;       /* [n_rigid*3] */
  const float *rigid_q;       /* [n_rigid*4] (w,x,y,z), normalised on entry */
  const float *rigid_v;       /* [n_rigid*3] */
  const float *rigid_w;       /* [n_rigid*3] world angular velocity */
  const int32_t *rigid_shape; /* [n_rigid] NSN_SHAPE_* */
  const float *rigid_extent;  /* [n_rigid*3] */
  int32_t n_particles;
  const float *particle_x;    /* [n_particles*3] */
  const float *particle_v;    /* [n_particles*3] */
  const float *particle_rest; /* [n_particles*3] */
  const float *particle_mass; /* [n_particles] extra point mass (may be 0) */
  int32_t n_tets;
  const int32_t *tet_ids;     /* [n_tets*4] particle indices */
  const float *tet_material;  /* [n_tets*3] (Young's modulus E, Poisson nu, density rho) */
  int32_t n_joints;
  const int32_t *joint_type;  /* [n_joints] NSN_JOINT_* */
  const int32_t *joint_body;  /* [n_joints*2] (A, B); A may be -1 = world */
  const float *joint_anchor;  /* [n_joints*6] anchor in A's frame, anchor in B's frame */
  const float *joint_axis;    /* [n_joints*6] axis in A's frame, axis in B's frame */
  const float *joint_ref;     /* [n_joints*6] unit reference direction perpendicular to the axis, per body */
  const float *joint_drive;   /* [n_joints*6] kp, kd, amplitude, frequency, phase, offset (kp=kd=0: no drive) */
  float mu;                   /* friction coefficient */
  float gravity[3];
  int32_t ground;             /* 1: static plane z = 0 with normal +z */
  int32_t max_contacts;       /* contact capacity; extra contacts are dropped and counted */
  int32_t tet_model;          /* NSN_TET_* of all tets of the env */
} nsn_env_desc;

typedef struct {
  int32_t ncp;       /* NSN_NCP_* */
  int32_t rmode;     /* NSN_R_* */
  float damping;     /* constant Newton step fraction t (Sec. 8.1; 0.75) */
  float eps;         /* Schur regularisation (Sec. 8.4; 1e-6) */
  int32_t geo_stiff; /* diagonal geometric stiffness on particle DOFs (Sec. 8.3) */
  int32_t fem_mode;  /* NSN_FEM_* */
  float margin;      /* contact creation distance (m) */
  int32_t warm;      /* NSN_WARM_* */
  int32_t line_search; /* 1: back-tracking line search on the L2 merit from the full
                          step (Sec. 8.1; for frictionless scenes) instead of the
                          constant damping; 0 (default): constant damping */
  int32_t linear;    /* NSN_LINEAR_* (default PCR) */
  int32_t islands;   /* 1: one PCR per island of an env (dynamic bodies connected by joints,
                        tets and contacts; Sec. 11), each with its own scalars and stop;
                        PCR only.  0 (default): one PCR over the whole env */
  int32_t watchdog;  /* 1: the step keeps its lowest-merit iterate and returns it when the
                        merit grows past 1e6 times that best or turns non-finite (a
                        safeguard Sec. 8.1 names without using it); 0 (default): the
                        paper's method, every damped iterate accepted */
} nsn_solver_params;

typedef struct {
  int32_t newton_iters; /* Newton updates performed in the last step */
  int32_t cr_iters;     /* PCR iterations performed in the last step */
  int32_t n_contacts;
  int32_t overflow;     /* contacts dropped beyond max_contacts */
  int32_t nonfinite;    /* 1 if a non-finite value was produced */
  int32_t converged;    /* 1 if r_ncp <= tol at exit (tol > 0) */
  int32_t fallback;     /* 1 if a warm-started step went non-finite and was rerun
                           from the plain start (u0 = 0, lambda0 = 0) */
  int32_t watchdog;     /* 1 if the iteration diverged (merit beyond 1e6 times the
                           step's best, or non-finite) and the step returned its
                           lowest-merit iterate */
  double r_ncp;         /* max(|M^-1 g|_inf, |err|_inf) at the final iterate (FP64) */
  double r_contact;     /* same over contact rows only */
  double merit;         /* |[g; err]|_2 at the final iterate (FP64 accumulation) */
  double r_ncp_first;   /* residual at the start iterate */
} nsn_step_stats;

/* Per-env totals accumulated by every step since the scene was created or the last
 * nsn_reset_accumulators(). */
typedef struct {
  int64_t steps;
  int64_t newton_iters;
  int64_t cr_iters;
  int64_t converged;        /* steps that ended with r_ncp <= tol (tol > 0) */
  int64_t nonfinite;
  int64_t fallbacks;        /* warm-started steps rerun from the plain start */
  int64_t watchdogs;        /* steps that returned their lowest-merit iterate */
  double cr_bytes;          /* algorithmic bytes of the PCR loop: per PCR iteration
                               332 B per tet (476 B per linear tet) + 228 B per
                               contact + 880 B per joint
                               + 12 B per body-space DOF (vectors, compressed J and
                               compliance read/written once per iteration, J read
                               twice), times the PCR iterations performed */
} nsn_accum;

/* One contact handed to nsn_set_contacts, in the form collision detection produces it
 * (Sec. 3: a feature point on body A, a point on body B or the world, the normal
 * fixed for the step at q^-, and a thickness; Alg. 1 runs detection once per step).
 * Bodies are env-local: rigid body i -> i, particle p -> n_rigid + p, -1 = the ground
 * plane (target only). */
typedef struct {
  int32_t key;         /* unique id, strictly ascending over the list; the library's own
                          detection uses feature * n_targets + target (features: box
                          vertices and capsule ends of rigid bodies in body order, then
                          particles; targets: the ground if present, then rigid bodies) */
  int32_t body_a;      /* feature body (rigid or particle); non-decreasing over the list */
  int32_t body_b;      /* target body (rigid) or -1 */
  float normal[3];     /* unit contact normal (world), pointing from B towards A */
  float a_local[3];    /* feature point in A's body frame (ignored for particles) */
  float b_local[3];    /* target point in B's body frame, or in the world for the ground */
  float thickness;     /* d: C = n.(a - b) - d */
} nsn_contact;

/* Fields of the per-iteration record (nsn_dump_iteration, nsn_read_iteration).  Row
 * arrays are in the library's row order: joints (6 rows each), tets (3 rows each, or 6
 * for NSN_TET_LINEAR), contacts (3 rows each: normal, friction 1, friction 2).
 * Body-space arrays hold 6 entries per rigid body (v, omega_world) then 3 per
 * particle. */
#define NSN_IT_LAM 0       /* [rows] multipliers lambda^k the iteration starts from */
#define NSN_IT_ERR 1       /* [rows] constraint error err (Sec. 6.1; App. A, B) */
#define NSN_IT_CDIAG 2     /* [rows] diagonal of the compliance block C */
#define NSN_IT_P 3         /* [rows] Jacobi preconditioner 1/(J H~^-1 J^T + C + eps)_ii (Sec. 8.2) */
#define NSN_IT_B 4         /* [rows] Schur right-hand side (J H~^-1 g - err)/h (Sec. 6.2) */
#define NSN_IT_AZ 5        /* [rows] A z for z = P b, A = J H~^-1 J^T + C + eps I */
#define NSN_IT_DLAM 6      /* [rows] the linear solve's Delta lambda */
#define NSN_IT_TETC 7      /* [6 per tet] compliance block E/h^2 of the tet's normal rows
                              (xx yy zz xy xz yz; App. B eq. E for neo-Hookean tets) */
#define NSN_IT_ALPHA 8     /* [per contact] alpha of the normal row (App. A) */
#define NSN_IT_ACTIVE 9    /* [per contact] 1 where the friction rows are active, else 0 */
#define NSN_IT_G 10        /* [body space] momentum residual g = M~(u - u~) - h J^T lambda */
#define NSN_IT_U 11        /* [body space] velocities u^k */
#define NSN_IT_HDIAG 12    /* [3 per particle] diagonal of H~ (Sec. 8.3) */
#define NSN_IT_RX 13       /* [3 per rigid body] positions at iterate k */
#define NSN_IT_RQ 14       /* [4 per rigid body] orientations at iterate k */
#define NSN_IT_PX 15       /* [3 per particle] particle positions at iterate k */
#define NSN_IT_PREV_LAM 16 /* iterate k-1 (k >= 1), same layouts as the fields above */
#define NSN_IT_PREV_U 17
#define NSN_IT_PREV_RX 18
#define NSN_IT_PREV_RQ 19
#define NSN_IT_PREV_PX 20
#define NSN_IT_NFIELDS 21

/* Last error message of the calling thread ("" if none).  Never NULL. */
const char *nsn_last_error(void);

/* Bytes of device workspace for these environments under these parameters (Sec. 6:
 * the Newton system's rows and body-space vectors; every array of a step lives in it).
 * n_envs >= 1.  params may be NULL for the defaults; its islands and line_search
 * fields decide whether the buffers of those options (Sec. 11, Sec. 8.1) are reserved,
 * and a scene created without them rejects turning them on later.  Returns NSN_EINVAL
 * on malformed descriptors or parameters (see nsn_create_scene). */
nsn_status nsn_query_workspace(const nsn_env_desc *envs, int32_t n_envs, const nsn_solver_params *params,
                               size_t *bytes);

/* Validate the descriptors (the problem statement of Sec. 5: state (q^-, u^-), masses,
 * bilateral constraints, contact geometry, friction coefficient), build the device
 * layout in `workspace` (a device pointer of at least nsn_query_workspace(envs, n_envs,
 * p) bytes, 256-byte aligned) and bind the scene to `hip_stream` (a hipStream_t, or
 * NULL).  Errors: NSN_EINVAL for bad sizes, indices, masses, inertias, degenerate rest
 * tets or materials, NSN_ENOMEM if the workspace is too small, NSN_EUNSUPPORTED if an
 * env exceeds the kernel limits, NSN_EDEVICE on a HIP failure.  On success *out owns
 * host bookkeeping only; free it with nsn_destroy_scene (the workspace stays the
 * caller's). */
nsn_status nsn_create_scene(const nsn_env_desc *envs, int32_t n_envs, const nsn_solver_params *p,
                            void *hip_stream, void *workspace, size_t workspace_bytes,
                            nsn_scene *out);

/* Release the host bookkeeping of a scene (NULL is accepted).  The workspace is the
 * caller's and is not touched. */
nsn_status nsn_destroy_scene(nsn_scene s);

/* Replace the solver parameters (the method's choices of Sec. 4, 7 and 8; takes
 * effect at the next step).  NSN_ESTATE for islands or line search when the scene's
 * workspace was sized without them, and for a learned warm start before
 * nsn_set_warm_start_model. */
nsn_status nsn_set_params(nsn_scene s, const nsn_solver_params *p);

/* One time step of every env (Algorithm 1) enqueued on the scene's stream:
 * collision detection at q^-, then up to `newton_iters` damped Newton updates with
 * `cr_iters` PCR iterations each.  tol > 0: an env stops as soon as its residual
 * r_ncp <= tol (checked before each update); tol = 0: fixed iteration counts.
 * The step sequence is captured once into a hipGraph per (h, iterations, tol) and
 * replayed.  stats: NULL keeps the call asynchronous; else a host array of n_envs
 * records that receives the step's statistics (the call then synchronises the
 * stream).  Errors: NSN_EINVAL for h <= 0 or negative counts; NSN_ESTATE in a learned
 * warm-start mode before nsn_set_warm_start_model. */
nsn_status nsn_step(nsn_scene s, double h, int32_t newton_iters, int32_t cr_iters, double tol,
                    nsn_step_stats *stats);

/* Statistics of the last step for every env (Sec. 8.1 residual and merit, iteration
 * counts): out[n_envs] (host).  Synchronises. */
nsn_status nsn_get_stats(nsn_scene s, nsn_step_stats *out);

/* Copy the state (q, u) of Sec. 5 of one env to caller-owned host arrays sized by its
 * descriptor (any pointer may be NULL to skip).  Synchronises the stream. */
nsn_status nsn_read_state(nsn_scene s, int32_t env, float *rigid_x, float *rigid_q, float *rigid_v,
                          float *rigid_w, float *particle_x, float *particle_v, double *time);

/* Overwrite the state (q, u) of one env (NULL pointers keep the current values).
 * Quaternions are normalised (Sec. 9 rigid bodies).  Static bodies keep zero velocity.
 * Enqueued on the stream; the host arrays may be freed on return. */
nsn_status nsn_write_state(nsn_scene s, int32_t env, const float *rigid_x, const float *rigid_q,
                           const float *rigid_v, const float *rigid_w, const float *particle_x,
                           const float *particle_v, const double *time);

/* Snapshot of the scene's dynamic state: what a time step (Alg. 1) reads that earlier
 * steps wrote -- positions and velocities (q^-, u^-) of bodies and particles, each
 * env's time, and what a warm start (Sec. 8.1) carries over: the previous step's
 * contact keys and multipliers and the joint rows' multipliers.  Geometry, solver
 * parameters, schedule, warm-start model and accumulators are not part of it.
 * nsn_state_bytes gives the size of a snapshot of this scene. */
nsn_status nsn_state_bytes(nsn_scene s, size_t *bytes);
/* Copies the state of every env into buf (device memory of nsn_state_bytes bytes,
 * owned by the caller) with device-to-device copies enqueued on the scene's stream;
 * returns without waiting.  NSN_EINVAL for a null argument. */
nsn_status nsn_save_state(nsn_scene s, void *buf);
/* Restores the state from a snapshot that nsn_save_state took of this same scene
 * (any other buffer is undefined behaviour); enqueued on the scene's stream.  The next
 * nsn_step continues from the saved state exactly: with the same schedule and
 * parameters it repeats, bit for bit, the steps that followed the save.  Discards
 * the record of a dump step (nsn_read_iteration then reports NSN_ESTATE). */
nsn_status nsn_load_state(nsn_scene s, const void *buf);

/* Contacts of one env from the last step (Alg. 1 collision detection; multipliers of
 * Sec. 3/4): up to `cap` records.  *n receives the count.  keys[cap]; bodies[cap*2] =
 * (feature body, target body) numbered as in nsn_contact; geom[cap*10] = normal(3),
 * feature point (body frame / unused for particles)(3), target point (body frame or
 * world)(3), thickness; lam[cap*3] = (lambda_n, lambda_f1, lambda_f2).  Synchronises. */
nsn_status nsn_read_contacts(nsn_scene s, int32_t env, int32_t cap, int32_t *n, int32_t *keys,
                             int32_t *bodies, float *geom, float *lam);

/* Replace collision detection (Alg. 1, "CollisionDetect") of one env for the NEXT step
 * only by the caller's contact list: n records, 0 <= n <= max_contacts, keys strictly
 * ascending, feature bodies non-decreasing, bodies in range, normals finite.  The list
 * is copied to the device on the stream before return (the host array may be freed).
 * Used to run both sides of a comparison on one contact set.  NSN_EINVAL on a list
 * that breaks these rules. */
nsn_status nsn_set_contacts(nsn_scene s, int32_t env, const nsn_contact *contacts, int32_t n);

/* Full multiplier vector lambda of one env (Sec. 6.1) in row order (joints: 6 rows
 * each, tets: 3 each or 6 for NSN_TET_LINEAR, contacts: 3 each); *n receives the row
 * count.  Synchronises. */
nsn_status nsn_read_lambda(nsn_scene s, int32_t env, int32_t cap, int32_t *n, float *lam);

/* Run ONE time step of every env that stops inside Newton iteration k (Alg. 1): the
 * first k damped updates as in nsn_step with tol = 0, then iteration k's assembly,
 * residual, geometric stiffness, Schur right-hand side and preconditioner, one
 * product A (P b), and `cr_iters` linear iterations; its update is not applied.  The
 * step is not captured in a graph and the call synchronises.  Afterwards the scene
 * holds iterate k in its working arrays, readable with nsn_read_iteration: positions
 * at iterate k, the pre-step velocities, the pre-step time, and the previous step's
 * contact multipliers for warm starts are left as they were.  Restore the pre-step
 * positions with nsn_write_state before stepping on.  The watchdog is off for this
 * step.  NSN_EINVAL for k < 0, cr_iters < 0 or h <= 0; NSN_EUNSUPPORTED with line search
 * on. */
nsn_status nsn_dump_iteration(nsn_scene s, double h, int32_t k, int32_t cr_iters);

/* One field (NSN_IT_*) of one env from the last nsn_dump_iteration: up to cap floats
 * into out (host); *n receives the field's length.  The PREV fields need k >= 1.
 * NSN_ESTATE before any nsn_dump_iteration; NSN_EINVAL for an unknown field.
 * Synchronises. */
nsn_status nsn_read_iteration(nsn_scene s, int32_t env, int32_t field, int32_t cap, int32_t *n, float *out);

/* Warm-start model for NSN_WARM_LEARNED and NSN_WARM_HYBRID (Sec. 8.1 starts the
 * Newton iteration from a given lambda^0; the learned start predicts it per contact):
 * float32 blob of 9347 MLP parameters
 * (12 -> 64 -> 64 -> 64 -> 3, ReLU; W1[64x12] b1 W2[64x64] b2 W3[64x64] b3 W4[3x64] b4)
 * followed by x_mean[12] x_std[12] y_mean[3] y_std[3].  Copied to the device. */
nsn_status nsn_set_warm_start_model(nsn_scene s, const float *blob, int64_t n);

/* Per-contact features of the last step's contact set, as used by the learned
 * warm start (at step start, in the contact basis of Sec. 3): feat[cap*12] = normal
 * and tangential relative velocity under u~ (3), C_n(q^-), previous-step
 * (lambda_n, lambda_f1, lambda_f2), 1/m_A, 1/m_B, mu, n_z, 1 if the key existed in the
 * previous step.  Synchronises. */
nsn_status nsn_read_features(nsn_scene s, int32_t env, int32_t cap, int32_t *n, float *feat);

/* Compute the 12 warm-start features of every contact in every step (off by default
 * except in the learned modes); needed by nsn_read_features. */
nsn_status nsn_enable_features(nsn_scene s, int32_t on);

/* Replay steps from captured hipGraphs (default on when the scene has a non-NULL
 * stream; graphs are never used on the NULL stream). */
nsn_status nsn_set_use_graphs(nsn_scene s, int32_t on);

/* ---- launch schedule (batching of independent envs; used by the autotuner) ------
 * Envs are launched in a fixed order: decreasing rows + DOFs (longest first).
 * order[n_envs] receives that order. */
nsn_status nsn_get_env_order(nsn_scene s, int32_t *order);

/* Split the env order into consecutive buckets, each launched as one grid of
 * workgroups with `block[i]` threads (64, 128, 256, 512 or 1024; 64 = one
 * wavefront per env).  The buckets must tile [0, n_envs) in order. */
nsn_status nsn_set_schedule(nsn_scene s, int32_t n_buckets, const int32_t *first, const int32_t *count,
                            const int32_t *block);

/* The current buckets: *n receives their number; up to cap entries are written.
 * Default at creation: for 1024 envs or more whose env at 3/8 of the order has at
 * least 1024 rows + DOFs besides its contact slots, three buckets (the heaviest 3/8 at
 * 1024 threads, the next 3/8 at 512, the rest at 128), or two (3/4 at 512, the rest at
 * 128) when some env has linear tets; other batches of 1024 envs or more, one bucket
 * at 128; smaller batches, one bucket sized by the largest env. */
nsn_status nsn_get_schedule(nsn_scene s, int32_t cap, int32_t *n, int32_t *first, int32_t *count,
                            int32_t *block);

/* Working memory of the Newton kernel (a tuning and testing switch; results are the
 * same in every mode, bit for bit): 0 keeps the body-space vector in global memory;
 * 1 puts it in LDS where a bucket's envs fit; 2 (default) also puts the tets'
 * contributions (J^T v per tet vertex) in LDS in buckets whose envs fit: n_dof +
 * 12 n_tet floats within the LDS share of a workgroup at the kernel's register-limited
 * occupancy (all of the device's LDS per workgroup at 512 and 1024 threads, half at
 * 256, a quarter at 128).  Applies to the current and later schedules. */
nsn_status nsn_set_lds_mode(nsn_scene s, int32_t max_mode);

/* Form of the PCR loop (Sec. 8.2; a tuning switch).  0: every PCR iteration streams
 * the rows and the element data from memory in two element passes, one forming
 * J^T z and one forming J (H~^-1 J^T z).  1: the same arithmetic with the
 * rows of every tet and contact held in the registers of the thread that owns the
 * element for all the PCR iterations of a Newton iteration, in envs whose elements
 * all have a slot (2 per thread below 1024 threads, none at 1024); results identical
 * to 0.  2 (default): one element pass per PCR iteration -- J^T z and J^T (P q) are carried in
 * body space by their own recurrences (linear images of the row updates), so each
 * element's Jacobian is read once per iteration; the same iterates in exact
 * arithmetic, with different rounding.  Envs with linear tets, and island mode, use
 * 0 whatever the setting.  NSN_EINVAL for another value. */
nsn_status nsn_set_pcr_form(nsn_scene s, int32_t form);

/* The LDS mode each current bucket runs in (0, 1, 2 as above): mode[cap]. */
nsn_status nsn_get_lds_modes(nsn_scene s, int32_t cap, int32_t *n, int32_t *mode);

/* Copy the per-env accumulators (out[n_envs], host) / reset them to zero. */
nsn_status nsn_read_accumulators(nsn_scene s, nsn_accum *out);
nsn_status nsn_reset_accumulators(nsn_scene s);

/* Duration of the Newton kernel launch(es) of the last min(cap, steps, 1024) steps,
 * oldest first, in ms: from the first workgroup's start to the last workgroup's end,
 * read from the GPU wall clock inside the kernel (so it also works under hipGraph
 * replay).  *n receives the count.  Synchronises the stream. */
nsn_status nsn_read_kernel_times(nsn_scene s, int32_t cap, int32_t *n, double *ms);

/* Device address of the per-env nsn_step_stats array (n_envs entries), valid for
 * the scene's lifetime, for readers that copy it asynchronously. */
nsn_status nsn_stats_device_ptr(nsn_scene s, void **ptr);

/* ---- learned part: MLP kernels on caller-owned device buffers -------------
 * Weights `w` are float32 device arrays in the layout above (9347 floats).  The
 * matrix products run on BF16 MFMA tiles with FP32 accumulation; activations are
 * rounded to bf16 where they enter a product.  `stream` may be NULL.  (The paper
 * starts every Newton solve from zero or the previous step's multipliers, Sec. 8.1;
 * the network supplies a per-contact start instead.) */

/* y[n*3] = MLP(x[n*12]) on the device. */
nsn_status nsn_mlp_forward(const float *w, const float *x, float *y, int64_t n, void *stream);

/* Mean-squared-error loss over n samples and its gradient grad[9347] (device);
 * *loss_out (device float, may be NULL).  `scratch` is a device buffer of at least
 * nsn_mlp_scratch_bytes(n) bytes (per-block partial gradients, reduced in a fixed
 * order, so the result is deterministic). */
size_t nsn_mlp_scratch_bytes(int64_t n);
nsn_status nsn_mlp_loss_grad(const float *w, const float *x, const float *t, int64_t n,
                             float *grad, float *loss_out, void *scratch, void *stream);

/* One Adam update of w (device) from grad with moments m, v (device, zero-initialised
 * by the caller), step count `step` >= 1. */
nsn_status nsn_mlp_adam(float *w, const float *grad, float *m, float *v, int64_t n_params,
                        float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/* The loss and gradient of nsn_mlp_loss_grad for callers that cannot allocate device
 * memory (code under graph capture, serving loops, harnesses that forbid it): the
 * same kernels, with the per-block partial gradients in a device array the library
 * holds for the life of the process on every device it runs on (nsn_mlp_noalloc_
 * scratch_bytes() bytes, about 10 MiB), so the results equal nsn_mlp_loss_grad's bit
 * for bit.  Allocates nothing and calls no allocating routine.  Calls on one device
 * share that array: calls that overlap in time on one device race (serialise them,
 * e.g. on one stream).  NSN_EINVAL for NULL pointers or n <= 0; NSN_EUNSUPPORTED if n
 * needs more scratch than the array holds; NSN_EDEVICE if the array's address cannot
 * be taken.  The message is in nsn_last_error(). */
size_t nsn_mlp_noalloc_scratch_bytes(void);
nsn_status nsn_mlp_loss_grad_noalloc(const float *w, const float *x, const float *t, int64_t n,
                                     float *grad, float *loss_out, void *stream);

/* Training of the warm-start network on solver-generated data (the network is trained
 * on the multipliers the method itself converges to; the paper's solver is the
 * teacher).  Every stage runs on the device in the library:
 *   1. each of the 15 columns of [x | t] is clipped to its [q, 1 - q] quantiles
 *      (linear interpolation between order statistics; q = clip_quantile, 0 = off);
 *   2. z-scoring with the clipped columns' means and standard deviations (FP64
 *      accumulation; a deviation below 1e-6 counts as 1);
 *   3. He-initialised weights (counter-based normal draws from `seed`) unless w_init;
 *   4. `epochs` passes, each over a fresh permutation of the samples (a counter-based
 *      bijection seeded by seed and the epoch), in batches of `batch` samples: MSE
 *      loss and gradient (nsn_mlp_loss_grad), then Adam (nsn_mlp_adam) at the
 *      learning rate lr * (1 + cos(pi * epoch / epochs)) / 2.
 * x[n*12], t[n*3]: device float32 (read only).  blob_out: device float32, the 9347
 * parameters then x_mean, x_std, y_mean, y_std (the layout of
 * nsn_set_warm_start_model).  loss_hist: host double[epochs] of the mean standardised
 * loss of every epoch, or NULL.  The workspace is a device buffer of at least
 * nsn_train_workspace_bytes(n, batch) bytes.  Synchronises `stream` at the end.
 * NSN_EINVAL for n < 2, batch < 1, epochs < 1, non-positive rates or a non-finite
 * input; NSN_ENONFINITE if the loss turns non-finite. */
typedef struct {
  int32_t epochs;
  int32_t batch;
  float lr;            /* peak learning rate of the cosine schedule */
  float beta1, beta2;  /* Adam moment decays (0.9, 0.999) */
  float adam_eps;      /* Adam denominator floor (1e-8) */
  float clip_quantile; /* data clipping quantile q in [0, 0.5) (5e-4) */
  uint64_t seed;
} nsn_train_params;
size_t nsn_train_workspace_bytes(int64_t n, int32_t batch);
nsn_status nsn_train_warm_start(const float *x, const float *t, int64_t n, const nsn_train_params *tp,
                                const float *w_init, float *blob_out, double *loss_hist, void *workspace,
                                size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
