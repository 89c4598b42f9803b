/*
 * FP64 CPU oracle of the non-smooth Newton step -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * this library.  It shares no code with the GPU library (include/nsn.h and the
 * package's csrc/), and neither side includes the other.
 *
 * The oracle steps ONE environment at a time, in double precision, following
 * Macklin et al., "Non-Smooth Newton Methods for Deformable Multi-Body Dynamics"
 * (TOG 2019): Algorithm 1 (simulation loop), Sec. 3 (models), Sec. 4 (NCP
 * functions), Sec. 5 (implicit time stepping), Sec. 6 (Newton system, Schur
 * complement), Sec. 7 (complementarity preconditioner), Sec. 8 (damping, start
 * iterate, PCR, geometric stiffness, regularisation), Sec. 9 (generalised
 * compliance, particles, rigid bodies) and Appendices A/B.
 */
#ifndef NSN_ORACLE_H
#define NSN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_rigid;
  const double *rigid_mass;      /* [n_rigid]; 0 = static obstacle */
  const double *rigid_inertia;   /* [n_rigid*3] principal body-frame inertia */
  const double *rigid_x;         /* [n_rigid*3] */
  const double *rigid_q;         /* [n_rigid*4] (w,x,y,z) */
  const double *rigid_v;         /* [n_rigid*3] */
  const double *rigid_w;         /* [n_rigid*3] world-frame angular velocity */
  const int32_t *rigid_shape;    /* [n_rigid] 0 box, 1 capsule, 2 none */
  const double *rigid_extent;    /* [n_rigid*3] box half extents / (radius, half length, 0) */
  int32_t n_particles;
  const double *particle_x, *particle_v, *particle_rest; /* [n_particles*3] */
  const double *particle_mass;   /* [n_particles] extra point mass */
  int32_t n_tets;
  const int32_t *tet_ids;        /* [n_tets*4] */
  const double *tet_material;    /* [n_tets*3] (E, nu, rho) */
  int32_t n_joints;
  const int32_t *joint_type;     /* [n_joints] 0 revolute, 1 prismatic */
  const int32_t *joint_body;     /* [n_joints*2] (A, B), -1 = world */
  const double *joint_anchor;    /* [n_joints*6] pA (A frame), pB (B frame) */
  const double *joint_axis;      /* [n_joints*6] aA, aB */
  const double *joint_ref;       /* [n_joints*6] tA, tB (perpendicular to the axis) */
  const double *joint_drive;     /* [n_joints*6] kp, kd, amp, freq, phase, offset */
  double mu;
  double gravity[3];
  int32_t ground;                /* plane z = 0 with normal +z */
  int32_t max_contacts;
  int32_t tet_model;             /* ORC_TET_NEOHOOKEAN (3 rows per tet) or ORC_TET_LINEAR (6) */
} orc_desc;

#define ORC_TET_NEOHOOKEAN 0 /* stable neo-Hookean in principal stretches (App. B) */
#define ORC_TET_LINEAR 1     /* linear Hookean on six co-rotated strains (Sec. 9.2) */

typedef struct {
  int32_t ncp;        /* 0 Fischer-Burmeister, 1 minimum map */
  int32_t rmode;      /* 0 identity, 1 h^2, 2 h^2 * effective mass */
  double damping;     /* constant step fraction t */
  double eps;         /* Schur regularisation */
  int32_t geo_stiff;  /* diagonal geometric stiffness on particle DOFs */
  int32_t fem_mode;   /* 0 projected full 3x3 compliance, 1 diagonal */
  double margin;      /* contact creation distance */
  int32_t warm;       /* 0 zero start, 1 previous-step multipliers, 2 learned, 3 previous-step
                         multipliers for known contact keys and learned for new ones */
  int32_t line_search; /* 1: back-tracking on the L2 merit from t = 1 instead of the constant damping */
  int32_t linear;      /* 0 preconditioned conjugate residual (the method), 1 preconditioned conjugate gradient */
  int32_t islands;     /* 1: one PCR per island of the env (independent CR scalars) */
  int32_t watchdog;    /* 1: keep the step's lowest-merit iterate and return it when the merit
                          blows up (Sec. 8.1 names such safeguards without using one); 0: the
                          method as the paper runs it, every iterate accepted */
} orc_params;

typedef struct {
  int32_t newton_iters;   /* Newton updates performed */
  int32_t cr_iters;       /* total PCR iterations */
  int32_t n_contacts;
  int32_t overflow;       /* contacts dropped beyond max_contacts */
  int32_t nonfinite;
  int32_t fallback;       /* 1 if a warm-started step went non-finite and was rerun from the plain start */
  int32_t watchdog;       /* 1 if the step diverged and returned its lowest-merit iterate */
  int32_t pad;
  double r_ncp;           /* final max(|M^-1 g|_inf, |err|_inf) */
  double r_contact;       /* same, contact rows only */
  double merit;           /* final |[g; err]|_2 */
  double r_ncp_first;     /* residual at the start iterate */
} orc_stats;

void *orc_create(const orc_desc *d, char *err, int errlen);
void orc_destroy(void *env);
int orc_step(void *env, const orc_params *p, double h, int newton_iters, int cr_iters,
             double tol, orc_stats *st);
void orc_get_state(void *env, double *rx, double *rq, double *rv, double *rw,
                   double *px, double *pv);
void orc_set_state(void *env, const double *rx, const double *rq, const double *rv,
                   const double *rw, const double *px, const double *pv);
double orc_get_time(void *env);
void orc_set_time(void *env, double t);
int orc_num_contacts(void *env);
/* contacts of the last step: key, feature body, target body, n, aL, bL, d, lambda(3) */
int orc_get_contacts(void *env, int64_t *key, int32_t *bodies, double *geom, double *lam, int cap);
int orc_num_rows(void *env);
void orc_get_lambda(void *env, double *lam);   /* full multiplier vector of the last step */
void orc_set_mlp(void *env, const double *weights, int64_t n);
/* per-iteration residual history of the last step (r_ncp per assembly) */
int orc_get_history(void *env, double *r, int cap);
/* Merit |[g; err]|_2 of every accepted iterate of the last step (count returned). */
int orc_get_merit_history(void *env, double *m, int cap);
/* Previous-step multipliers for a warm start (keys ascending); 0 or -1 (bad input). */
int orc_set_prev(void *env, int n, const int64_t *keys, const double *lam3, const double *lam_joint);
/* per-row data of the final assembly of the last step */
int orc_get_rows_debug(void *env, double *err, double *cdiag, double *pdiag, int cap);

/* ---- per-iteration record (test support) ----
 * orc_set_record(env, k): the following steps record Newton iteration k (-1 = off;
 * with line search, the accepted point of iteration k): the iterate it starts from
 * and its assembly, residual, geometric stiffness, Schur system and PCR solution.
 * orc_get_record(env, field, out, cap) copies one field (ORC_REC_*), returns its length
 * (0 when iteration k was not reached).  Rows are in the oracle's order: joints
 * (6 each), contacts (3 each), tets (3 or 6 each). */
#define ORC_REC_LAM 0     /* [rows] multipliers lambda^k */
#define ORC_REC_U 1       /* [ndof] velocities u^k (6 per rigid body, then 3 per particle) */
#define ORC_REC_RX 2      /* [3 n_rigid] positions at iterate k */
#define ORC_REC_RQ 3      /* [4 n_rigid] */
#define ORC_REC_PX 4      /* [3 n_particles] */
#define ORC_REC_ERR 5     /* [rows] constraint error vector */
#define ORC_REC_CDIAG 6   /* [rows] diagonal of the compliance block C */
#define ORC_REC_P 7       /* [rows] Jacobi preconditioner 1/(J H~^-1 J^T + C + eps)_ii */
#define ORC_REC_B 8       /* [rows] Schur right-hand side (J H~^-1 g - err)/h */
#define ORC_REC_AZ 9      /* [rows] A z for z = P b, A = J H~^-1 J^T + C + eps I */
#define ORC_REC_DLAM 10   /* [rows] PCR solution Delta lambda */
#define ORC_REC_G 11      /* [ndof] momentum residual g = M~(u - u~) - h J^T lambda */
#define ORC_REC_HDIAG 12  /* [3 n_particles] diagonal of H~ on particle DOFs */
#define ORC_REC_ALPHA 13  /* [n_contacts] alpha of the normal row */
#define ORC_REC_RN 14     /* [n_contacts] r of the normal row */
#define ORC_REC_RF 15     /* [n_contacts] r of the friction rows */
#define ORC_REC_CBLK 16   /* [9 rows] compliance block, 3x3 row-major, at the block's first row */
#define ORC_REC_F 17      /* [ndof] J^T lambda^k */
#define ORC_REC_FHAT 18   /* [ndof] (J^{k-1})^T lambda^k, the secant's other force (0 if none) */
#define ORC_REC_UPREV 19  /* [ndof] u^{k-1} (0 if none) */
#define ORC_REC_ACTIVE 20 /* [n_contacts] 1 where the friction rows are active */
#define ORC_REC_RESID 21  /* [4] r_ncp, r_contact, merit, cr iterations of iteration k */
void orc_set_record(void *env, int k);
int orc_get_record(void *env, int field, double *out, int cap);

/* Evaluate one Newton iteration at a given iterate (test support).  Runs the step
 * set-up and collision detection at the env's current state (q^-, u^-), puts the
 * iterate (lam, u, rx, rq, px) in place of the start iterate, and records iteration 0
 * of that step (orc_get_record): assembly, residual, Schur system, PCR of M
 * iterations.  The previous iterate (lam_p, u_p, rx_p, rq_p, px_p), when given, is
 * assembled first and supplies J^{k-1} and u^{k-1} to the geometric-stiffness secant
 * (NULL: no previous iterate, no secant).  lam and lam_p hold the rows of the contact
 * set found at q^- (orc_num_contacts after the call tells its size; -2 if it differs
 * from n_contacts).  The env's state and previous-step data are left unchanged. */
int orc_eval_iterate(void *env, const orc_params *p, double h, int M, int n_contacts,
                     const double *lam, const double *u, const double *rx, const double *rq,
                     const double *px, const double *lam_p, const double *u_p, const double *rx_p,
                     const double *rq_p, const double *px_p);

/* ---- primitives exposed for the pins ---- */
void orc_ncp_fb(double C, double lam, double r, double *phi, double *alpha, double *beta);
void orc_ncp_min(double C, double lam, double r, double *phi, double *alpha, double *beta);
double orc_friction_w(int ncp, double vnorm, double lam_n, double lamf_norm, double mu, double r);
void orc_svd3(const double *F, double *U, double *s, double *V);
void orc_sym_eig3(const double *A, double *Q, double *w);
void orc_lame(double E, double nu, double *C1, double *D1, double *alpha);
void orc_neohookean(const double *s, double C1, double D1, double alpha, double *psi,
                    double *grad, double *hess);
void orc_compliance3(const double *H, double floor_, int mode, double *E);
/* Linear tet of Sec. 9.2 at node positions x12 (4 x 3): strains eps6 (xx yy zz yz xz
 * xy), constraint rows rows72 (6 x 12, node-major), stress c6 = V_e K_e eps6 and the
 * compliance C36 = (V_e K_e)^-1 (6 x 6). */
void orc_linear_tet(const double *Dminv, const double *x12, double E, double nu, double Ve, double *eps6,
                    double *rows72, double *c6, double *C36);
int orc_pcg_dense(int n, const double *A, const double *b, const double *P, int iters, double *x, double *hist);
int orc_pcr_dense(int n, const double *A, const double *b, const double *P, int iters,
                  double *x, double *hist);
void orc_quat_kinematic(const double *q, double *Q /* 4x3 */);
void orc_tangent_basis(const double *n, double *d1, double *d2);

/* ---- learned warm start (FP64 MLP: 12 -> 64 -> 64 -> 64 -> 3, ReLU) ---- */
int64_t orc_mlp_num_params(void);
void orc_mlp_forward(const double *w, int64_t n, const double *x, double *y);
double orc_mlp_loss_grad(const double *w, int64_t n, const double *x, const double *t,
                         double *grad);
/* the same with every product operand rounded to bfloat16 (the GPU's MFMA operands) */
double orc_mlp_loss_grad_bf16(const double *w, int64_t n, const double *x, const double *t,
                              double *grad);
/* pre-activations (3 x 64) of that rounded forward pass for one sample */
void orc_mlp_preact_bf16(const double *w, const double *x, double *pre);
/* 12 features of every contact of the current state (computed as at step start) */
int orc_contact_features(void *env, const orc_params *p, double h, double *feat, int64_t *key,
                         int cap);

#ifdef __cplusplus
}
#endif
#endif
