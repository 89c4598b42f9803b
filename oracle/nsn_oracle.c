/*
 * FP64 CPU oracle of the non-smooth Newton step -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow and written to be checked against the paper by eye:
 *   Macklin, Erleben, Mueller, Chentanez, Jeschke, Makoviychuk,
 *   "Non-Smooth Newton Methods for Deformable Multi-Body Dynamics", TOG 38(5), 2019.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load it.
 * It shares no code with the GPU library.  Every function names the passage it
 * follows.  Readings of passages the paper leaves open are marked READING.
 *
 * Parity-unpinned parts (checked only GPU-vs-oracle): the exact iterate path at a
 * fixed Newton x PCR budget (FP rounding at the non-smooth points, SVD bases at
 * repeated singular values, the geometric-stiffness secant), contact generation
 * rules for the primitive shapes.
 */
#include "nsn_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXENT 4
#define TAU_GS 1e-6      /* READING: secant smoothing velocity scale (m/s) */
#define KAPPA_W 1e-4     /* READING: FB friction denominator at or below which W is infinite, relative to r*mu*lambda_n */
#define TAU_CR 1e-12     /* READING: PCR stops once <z, A z> falls below this fraction of its start */
#define WATCH_BLOWUP 1e6 /* READING: watchdog, merit growth over the step's best that ends the step */
#define LS_SIGMA 1e-4    /* READING: line search, sufficient decrease merit <= (1 - sigma t) merit_k */
#define LS_TMIN (1.0 / 64.0) /* READING: line search, smallest step fraction (then accepted) */
#define CLAMP_FEM 1e-3   /* READING: eigenvalue floor of the material Hessian, relative to 2*C1*Ve */
#define JACOBI_SWEEPS 6
#define TAU_NCP 1e-6      /* READING: derivative band around the NCP kink (units of C) */
#define TAU_EIG 1e-6      /* READING: relative size below which Jacobi skips a rotation / treats
                             eigenvalues as tied */
#define MAX_HIST 256
#define ORC_REC_NFIELDS 22
#define MLP_IN 12
#define MLP_H 64
#define MLP_OUT 3

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
static void v3_cross(const double *a, const double *b, double *c) {
  double t0 = a[1] * b[2] - a[2] * b[1];
  double t1 = a[2] * b[0] - a[0] * b[2];
  double t2 = a[0] * b[1] - a[1] * b[0];
  c[0] = t0; c[1] = t1; c[2] = t2;
}
static double v3_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double v3_norm(const double *a) { return sqrt(v3_dot(a, a)); }
static void m3_vec(const double *M, const double *v, double *o) { /* row-major 3x3 */
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = M[3 * i] * v[0] + M[3 * i + 1] * v[1] + M[3 * i + 2] * v[2];
  o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
static void m3_tvec(const double *M, const double *v, double *o) {
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = M[i] * v[0] + M[3 + i] * v[1] + M[6 + i] * v[2];
  o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
static void m3_mul(const double *A, const double *B, double *C) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      T[3 * i + j] = s;
    }
  memcpy(C, T, sizeof T);
}
static double m3_det(const double *A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
static void m3_inv(const double *A, double *B) {
  double d = m3_det(A), T[9];
  T[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  T[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  T[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  T[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  T[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  T[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  T[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  T[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  T[8] = (A[0] * A[4] - A[1] * A[3]) / d;
  memcpy(B, T, sizeof T);
}

/* Orientations must be unit quaternions; inputs are normalised on entry. */
static void normalize_quat(double *q) {
  double l = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  q[0] /= l; q[1] /= l; q[2] /= l; q[3] /= l;
}

/* Rotation matrix of a unit quaternion (w,x,y,z). */
static void quat_to_mat(const double *q, double *R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Sec. 9 (rigid bodies): the 4x3 matrix Q(theta) of the kinematic map G = diag(I, Q/2). */
void orc_quat_kinematic(const double *t, double *Q) {
  double t1 = t[0], t2 = t[1], t3 = t[2], t4 = t[3];
  double M[12] = {-t2, -t3, -t4,
                  t1, t4, -t3,
                  -t4, t1, t2,
                  t3, -t2, t1};
  memcpy(Q, M, sizeof M);
}

/* READING: tangent basis of a contact normal.  The paper needs only a 2-D basis
 * D = [d1 d2] orthogonal to n (Sec. 3, friction); isotropy makes results basis-free.
 * e = world axis with the smallest |n_i| (ties -> lowest index), d1 = n x e / |n x e|,
 * d2 = n x d1. */
void orc_tangent_basis(const double *n, double *d1, double *d2) {
  int k = 0;
  double best = fabs(n[0]);
  for (int i = 1; i < 3; ++i)
    if (fabs(n[i]) < best) { best = fabs(n[i]); k = i; }
  double e[3] = {0, 0, 0};
  e[k] = 1.0;
  v3_cross(n, e, d1);
  double l = v3_norm(d1);
  d1[0] /= l; d1[1] /= l; d1[2] /= l;
  v3_cross(n, d1, d2);
}

/* ------------------------------------------------------------------------- */
/* NCP functions (Sec. 4, Appendix A)                                        */
/* ------------------------------------------------------------------------- */

/* Appendix A.1, FB form with the r factor: phi = C + r lam - sqrt(C^2 + r^2 lam^2);
 * alpha = d phi / dC, beta = 1 - r lam / sqrt(..) so that d phi / d lam = beta r.
 * At (0,0) the subgradient choice alpha = 0, beta = 1 of Sec. 4.2.  READING: the
 * derivative takes that choice whenever sqrt(C^2 + r^2 lam^2) <= TAU_NCP, i.e. when the
 * point is (0,0) up to the rounding of positions (every resting contact starts there at
 * the zero start iterate); phi itself is always exact. */
void orc_ncp_fb(double C, double lam, double r, double *phi, double *alpha, double *beta) {
  double rl = r * lam;
  double rho = sqrt(C * C + rl * rl);
  *phi = C + rl - rho;
  if (rho > TAU_NCP) {
    *alpha = 1.0 - C / rho;
    *beta = 1.0 - rl / rho;
  } else {
    *alpha = 0.0;
    *beta = 1.0;
  }
}

/* Appendix A.1, minimum map with r: phi = min(C, r lam); derivative of the C branch
 * when C <= r lam.  READING: the branch test is C <= r lam + TAU_NCP so that ties up to
 * the rounding of positions take the C branch on every precision; phi is exact. */
void orc_ncp_min(double C, double lam, double r, double *phi, double *alpha, double *beta) {
  double rl = r * lam;
  *phi = C < rl ? C : rl;
  if (C <= rl + TAU_NCP) {
    *alpha = 1.0; *beta = 0.0;
  } else {
    *alpha = 0.0; *beta = 1.0;
  }
}

/* Sec. 4.3 eq. (friction_w) and Appendix A.2: the friction compliance W of one
 * contact with mu*lam_n > 0.  FB form (READING of the A.2 expressions: the
 * velocity magnitude enters unsquared; the fixed-point numerator is evaluated in a
 * cancellation-free way):
 *   s   = mu lam_n - |lam_f|
 *   num = sqrt(|v|^2 + r^2 s^2) - r s       (= |D^T u|^{n+1})
 *   den = |v| + r |lam_f| - num             (= r |lam_f|^{n+1})
 *   W   = r num / den
 * READING: once |lam_f| leaves the cone far enough (about 2 mu lam_n at small slip),
 * the fixed point asks for a friction magnitude |lam_f|^{n+1} <= 0, i.e. no friction
 * force; W is then infinite (returned as INFINITY for den <= KAPPA_W r mu lam_n), and
 * the row takes its W -> infinity limit, lam_f -> 0 (the form of inactive friction).
 * Minimum map: W = 0 if |v| <= r s, else (|v| - r s) / (mu lam_n). */
double orc_friction_w(int ncp, double vnorm, double lam_n, double lamf_norm, double mu, double r) {
  double s = mu * lam_n - lamf_norm;
  if (ncp == 1) {
    if (vnorm <= r * s) return 0.0;
    return (vnorm - r * s) / (mu * lam_n);
  }
  double root = sqrt(vnorm * vnorm + r * r * s * s);
  double num;
  if (s > 0.0)
    num = vnorm * vnorm / (root + r * s);
  else
    num = root - r * s;
  double den = vnorm + r * lamf_norm - num;
  if (den <= KAPPA_W * r * mu * lam_n) return INFINITY;
  return r * num / den;
}

/* ------------------------------------------------------------------------- */
/* 3x3 symmetric eigen-decomposition and signed SVD (Sec. 9.2, Appendix B)   */
/* ------------------------------------------------------------------------- */

/* Cyclic Jacobi on a symmetric 3x3 (row-major).  Fixed sweep count; pairs in the
 * order (0,1), (0,2), (1,2).  On return w holds the eigenvalues sorted descending
 * and Q the matching eigenvectors as columns.  READING for repeated singular values
 * (the rest state F = I): a matrix whose off-diagonals are all below TAU_EIG times its
 * trace is taken as diagonal (no rotation), and eigenvalues within TAU_EIG relative of
 * each other are ties that keep index order, so a basis that is arbitrary in exact
 * arithmetic comes out the same on every precision. */
void orc_sym_eig3(const double *Ain, double *Q, double *w) {
  double A[9], V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  memcpy(A, Ain, sizeof A);
  static const int PP[3] = {0, 0, 1}, QQ[3] = {1, 2, 2};
  double tr = fabs(A[0]) + fabs(A[4]) + fabs(A[8]);
  double off = fabs(A[1]);
  if (fabs(A[2]) > off) off = fabs(A[2]);
  if (fabs(A[5]) > off) off = fabs(A[5]);
  int sweeps = off <= TAU_EIG * tr ? 0 : JACOBI_SWEEPS;
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    for (int k = 0; k < 3; ++k) {
      int p = PP[k], q = QQ[k];
      double apq = A[3 * p + q];
      if (apq == 0.0) continue;
      double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
      double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
      if (theta < 0) t = -t;
      double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      /* A <- J^T A J with J the rotation in the (p,q) plane */
      for (int i = 0; i < 3; ++i) {
        double aip = A[3 * i + p], aiq = A[3 * i + q];
        A[3 * i + p] = c * aip - s * aiq;
        A[3 * i + q] = s * aip + c * aiq;
      }
      for (int j = 0; j < 3; ++j) {
        double apj = A[3 * p + j], aqj = A[3 * q + j];
        A[3 * p + j] = c * apj - s * aqj;
        A[3 * q + j] = s * apj + c * aqj;
      }
      for (int i = 0; i < 3; ++i) {
        double vip = V[3 * i + p], viq = V[3 * i + q];
        V[3 * i + p] = c * vip - s * viq;
        V[3 * i + q] = s * vip + c * viq;
      }
    }
  }
  double ev[3] = {A[0], A[4], A[8]};
  int idx[3] = {0, 1, 2};
  /* stable descending sort of 3 entries */
  for (int i = 1; i < 3; ++i) {
    int j = i;
    while (j > 0 && ev[idx[j]] - ev[idx[j - 1]] > TAU_EIG * (fabs(ev[idx[j]]) + fabs(ev[idx[j - 1]]))) {
      int t = idx[j]; idx[j] = idx[j - 1]; idx[j - 1] = t;
      --j;
    }
  }
  for (int c = 0; c < 3; ++c) {
    w[c] = ev[idx[c]];
    for (int r = 0; r < 3; ++r) Q[3 * r + c] = V[3 * r + idx[c]];
  }
}

/* Signed SVD F = U diag(s) V^T with det U = det V = +1 (READING of the principal
 * stretches of Sec. 9.2 for inverted elements: the last stretch carries the sign of
 * det F).  V from the eigenvectors of F^T F (descending), b_i = F v_i,
 * u1 = b1/|b1|, u2 = Gram-Schmidt(b2), u3 = u1 x u2, s_i = u_i . b_i. */
void orc_svd3(const double *F, double *U, double *s, double *V) {
  double FtF[9], w[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += F[3 * k + i] * F[3 * k + j];
      FtF[3 * i + j] = acc;
    }
  orc_sym_eig3(FtF, V, w);
  if (m3_det(V) < 0) { V[2] = -V[2]; V[5] = -V[5]; V[8] = -V[8]; }
  double b[3][3];
  for (int c = 0; c < 3; ++c) {
    double vc[3] = {V[c], V[3 + c], V[6 + c]};
    m3_vec(F, vc, b[c]);
  }
  double u1[3], u2[3], u3[3];
  double l1 = v3_norm(b[0]);
  if (l1 > 0) { u1[0] = b[0][0] / l1; u1[1] = b[0][1] / l1; u1[2] = b[0][2] / l1; }
  else { u1[0] = 1; u1[1] = 0; u1[2] = 0; }
  double pr = v3_dot(u1, b[1]);
  u2[0] = b[1][0] - pr * u1[0]; u2[1] = b[1][1] - pr * u1[1]; u2[2] = b[1][2] - pr * u1[2];
  double l2 = v3_norm(u2);
  if (l2 > 1e-6 * (l1 > 0 ? l1 : 1.0)) {
    u2[0] /= l2; u2[1] /= l2; u2[2] /= l2;
  } else { /* any unit vector orthogonal to u1 */
    double t1[3], t2[3];
    orc_tangent_basis(u1, t1, t2);
    u2[0] = t1[0]; u2[1] = t1[1]; u2[2] = t1[2];
  }
  v3_cross(u1, u2, u3);
  for (int r = 0; r < 3; ++r) { U[3 * r] = u1[r]; U[3 * r + 1] = u2[r]; U[3 * r + 2] = u3[r]; }
  s[0] = v3_dot(u1, b[0]);
  s[1] = v3_dot(u2, b[1]);
  s[2] = v3_dot(u3, b[2]);
}

/* ------------------------------------------------------------------------- */
/* Stable neo-Hookean in principal stretches (Appendix B)                    */
/* ------------------------------------------------------------------------- */

/* READING of "relate to the Lame parameters according to the original paper":
 * mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu)), C1 = mu/2, D1 = (lambda+mu)/2,
 * alpha = 1 + mu/(lambda+mu); with these the rest state is stress free. */
void orc_lame(double E, double nu, double *C1, double *D1, double *alpha) {
  double mu = E / (2.0 * (1.0 + nu));
  double la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  *C1 = 0.5 * mu;
  *D1 = 0.5 * (la + mu);
  *alpha = 1.0 + mu / (la + mu);
}

/* Appendix B: Psi = C1 (I_C - 3) + D1 (J - alpha)^2 with I_C = sum s_i^2, J = s1 s2 s3.
 * Gradient READING: (J - alpha) in the gradient, consistent with the energy and
 * with the Hessian printed there (k0 = 2J - alpha). */
void orc_neohookean(const double *s, double C1, double D1, double alpha, double *psi,
                    double *grad, double *hess) {
  double s1 = s[0], s2 = s[1], s3 = s[2];
  double J = s1 * s2 * s3;
  double IC = s1 * s1 + s2 * s2 + s3 * s3;
  if (psi) *psi = C1 * (IC - 3.0) + D1 * (J - alpha) * (J - alpha);
  if (grad) {
    grad[0] = 2.0 * C1 * s1 + 2.0 * D1 * (J - alpha) * s2 * s3;
    grad[1] = 2.0 * C1 * s2 + 2.0 * D1 * (J - alpha) * s1 * s3;
    grad[2] = 2.0 * C1 * s3 + 2.0 * D1 * (J - alpha) * s1 * s2;
  }
  if (hess) {
    double k0 = 2.0 * J - alpha;
    double k1 = D1 * s3 * k0, k2 = D1 * s2 * k0, k3 = D1 * s1 * k0;
    hess[0] = 2.0 * (D1 * s2 * s2 * s3 * s3 + C1);
    hess[4] = 2.0 * (D1 * s1 * s1 * s3 * s3 + C1);
    hess[8] = 2.0 * (D1 * s1 * s1 * s2 * s2 + C1);
    hess[1] = hess[3] = 2.0 * k1;
    hess[2] = hess[6] = 2.0 * k2;
    hess[5] = hess[7] = 2.0 * k3;
  }
}

/* Sec. 9.2 (hyperelastic materials): E = (d^2 U / ds^2)^-1, projected to the positive
 * definite cone when indefinite (READING: eigenvalues clamped to >= floor_), or its
 * diagonal approximation (mode 1). */
void orc_compliance3(const double *H, double floor_, int mode, double *E) {
  if (mode == 1) {
    memset(E, 0, 9 * sizeof(double));
    for (int i = 0; i < 3; ++i) {
      double d = H[4 * i];
      if (d < floor_) d = floor_;
      E[4 * i] = 1.0 / d;
    }
    return;
  }
  double Q[9], w[3];
  orc_sym_eig3(H, Q, w);
  for (int i = 0; i < 3; ++i)
    if (w[i] < floor_) w[i] = floor_;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += Q[3 * i + k] * Q[3 * j + k] / w[k];
      E[3 * i + j] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* Linear Hookean constant-strain tet (Sec. 9.2, linear materials)            */
/* ------------------------------------------------------------------------- */

/* strain order of Sec. 9.2: (e_xx, e_yy, e_zz, e_yz, e_xz, e_xy) as index pairs */
static const int LIN_A[6] = {0, 1, 2, 1, 0, 0}, LIN_B[6] = {0, 1, 2, 2, 2, 1};

/* READING: the strain of a linear tet is taken in the element's rotated frame (the
 * paper's material-extension test names the linear model co-rotational):
 * e = S - I with F = R S the polar decomposition, R = U V^T and S = V diag(s) V^T from
 * the signed SVD (det R = +1 also for inverted elements).  Shear entries are tensor
 * components, e_yz = (S_yz + S_zy)/2 - 0. */
static void corot_strain(const double *F, double *R, double *eps6) {
  double U[9], s[3], V[9];
  orc_svd3(F, U, s, V);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double r = 0.0;
      for (int k = 0; k < 3; ++k) r += U[3 * i + k] * V[3 * j + k];
      R[3 * i + j] = r;
    }
  for (int q = 0; q < 6; ++q) {
    int a = LIN_A[q], b = LIN_B[q];
    double Sab = 0.0;
    for (int k = 0; k < 3; ++k) Sab += V[3 * a + k] * s[k] * V[3 * b + k];
    eps6[q] = Sab - (a == b ? 1.0 : 0.0);
  }
}

/* READING: ds/dx at fixed R.  With D_s = [x1-x0, x2-x0, x3-x0] and F = D_s D_m^-1,
 * (R^T F)_ab = sum_j R_:a . (x_j - x0) (D_m^-1)_jb, so the row of e_ab has the entry
 * (R_:a (D_m^-1)_jb + R_:b (D_m^-1)_ja)/2 at vertex j = 1..3 and minus their sum at
 * vertex 0.  For an isotropic K_e, J^T c is then the exact gradient of the energy
 * (the rotation's derivative pairs a skew matrix with the symmetric S c). */
static void corot_rows(const double *R, const double *Dminv, double g[6][4][3]) {
  for (int q = 0; q < 6; ++q) {
    int a = LIN_A[q], b = LIN_B[q];
    for (int k = 0; k < 3; ++k) g[q][0][k] = 0.0;
    for (int j = 1; j <= 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double v = 0.5 * (R[3 * k + a] * Dminv[3 * (j - 1) + b] + R[3 * k + b] * Dminv[3 * (j - 1) + a]);
        g[q][j][k] = v;
        g[q][0][k] -= v;
      }
  }
}

/* Sec. 9.2: U = V_e (1/2) s^T K_e s, c = dU/ds = V_e K_e s.  READING: isotropic K_e from
 * the Lame parameters, for tensor shear strains: normal block lambda 1 1^T + 2 mu I,
 * shear diagonal 4 mu (so that s^T K_e s / 2 = mu e:e + lambda tr(e)^2 / 2). */
static void lin_stiffness(double mu, double la, double *K36) {
  memset(K36, 0, 36 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K36[6 * i + j] = la + (i == j ? 2.0 * mu : 0.0);
  for (int i = 3; i < 6; ++i) K36[6 * i + i] = 4.0 * mu;
}

/* E = (V_e K_e)^-1 (Sec. 9.2, a constant): the normal block inverted as a 3x3 matrix,
 * the shear diagonal entry by entry. */
static void lin_compliance(double mu, double la, double Ve, double *C36) {
  double K[36], Kn[9], En[9];
  lin_stiffness(mu, la, K);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Kn[3 * i + j] = Ve * K[6 * i + j];
  m3_inv(Kn, En);
  memset(C36, 0, 36 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C36[6 * i + j] = En[3 * i + j];
  for (int i = 3; i < 6; ++i) C36[6 * i + i] = 1.0 / (Ve * K[6 * i + i]);
}

static void lame_mu_lambda(double E, double nu, double *mu, double *la) {
  *mu = E / (2.0 * (1.0 + nu));
  *la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

void orc_linear_tet(const double *Dminv, const double *x12, double E, double nu, double Ve, double *eps6,
                    double *rows72, double *c6, double *C36) {
  double Ds[9], F[9], R[9], g[6][4][3], K[36], mu, la;
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) Ds[3 * r + c] = x12[3 * (c + 1) + r] - x12[r];
  m3_mul(Ds, Dminv, F);
  corot_strain(F, R, eps6);
  corot_rows(R, Dminv, g);
  for (int q = 0; q < 6; ++q)
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 3; ++k) rows72[12 * q + 3 * j + k] = g[q][j][k];
  lame_mu_lambda(E, nu, &mu, &la);
  lin_stiffness(mu, la, K);
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 6; ++j) acc += K[6 * i + j] * eps6[j];
    c6[i] = Ve * acc;
  }
  lin_compliance(mu, la, Ve, C36);
}

/* ------------------------------------------------------------------------- */
/* Preconditioned conjugate residual (Sec. 8.2; Saad's CR with a left Jacobi  */
/* preconditioner).  READING: x0 = 0, at most `iters` iterations; stops when   */
/* rho = <z, Az> <= TAU_CR rho_0 (the residual is at rounding level: further   */
/* steps only amplify rounding) or <q, Pq> <= 0.                               */
/* ------------------------------------------------------------------------- */
typedef void (*orc_apply_fn)(void *ctx, const double *in, double *out);

static int pcr_solve_ref(int n, orc_apply_fn apply, void *ctx, const double *b, const double *P,
                         int iters, double *x, double *hist, double rho_ref);
static int pcr_solve(int n, orc_apply_fn apply, void *ctx, const double *b, const double *P,
                     int iters, double *x, double *hist) {
  return pcr_solve_ref(n, apply, ctx, b, P, iters, x, hist, -1.0);
}

/* rho_ref >= 0: the stop level is TAU_CR * rho_ref instead of TAU_CR times the solve's
 * own start (the island mode: the rounding level of the whole env's system). */
static int pcr_solve_ref(int n, orc_apply_fn apply, void *ctx, const double *b, const double *P,
                         int iters, double *x, double *hist, double rho_ref) {
  double *r = calloc(n, sizeof(double)), *z = calloc(n, sizeof(double));
  double *p = calloc(n, sizeof(double)), *q = calloc(n, sizeof(double));
  double *w = calloc(n, sizeof(double)), *s = calloc(n, sizeof(double));
  int done = 0;
  for (int i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; z[i] = P[i] * r[i]; p[i] = z[i]; }
  if (iters > 0) {
    apply(ctx, z, w);
    double rho = 0.0;
    for (int i = 0; i < n; ++i) { q[i] = w[i]; rho += z[i] * w[i]; }
    const double rho_stop = TAU_CR * (rho_ref >= 0.0 ? rho_ref : rho);
    for (int it = 0; it < iters; ++it) {
      if (!(rho > rho_stop) || !(rho > 0.0)) break;
      double qs = 0.0;
      for (int i = 0; i < n; ++i) { s[i] = P[i] * q[i]; qs += q[i] * s[i]; }
      if (!(qs > 0.0)) break;
      double alpha = rho / qs;
      for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; z[i] -= alpha * s[i]; }
      ++done;
      if (hist) {
        double rr = 0;
        for (int i = 0; i < n; ++i) rr += r[i] * P[i] * r[i];
        hist[it] = sqrt(rr);
      }
      if (it == iters - 1) break;  /* the last update needs no further product */
      apply(ctx, z, w);
      double rho_new = 0.0;
      for (int i = 0; i < n; ++i) rho_new += z[i] * w[i];
      double beta = rho_new / rho;
      rho = rho_new;
      for (int i = 0; i < n; ++i) { p[i] = z[i] + beta * p[i]; q[i] = w[i] + beta * q[i]; }
    }
  }
  free(r); free(z); free(p); free(q); free(w); free(s);
  return done;
}

/* ------------------------------------------------------------------------- */
/* Preconditioned conjugate gradient (the comparison solver of Sec. 8.2 and    */
/* the solver study): Jacobi preconditioner P, x0 = 0, at most `iters`        */
/* iterations; READING: stops when <r, P r> <= TAU_CR <r0, P r0> or            */
/* <p, A p> <= 0.  hist[k] = sqrt(r^T P r) after iteration k.                  */
/* ------------------------------------------------------------------------- */
static int pcg_solve(int n, orc_apply_fn apply, void *ctx, const double *b, const double *P,
                     int iters, double *x, double *hist) {
  double *r = calloc(n, sizeof(double)), *z = calloc(n, sizeof(double));
  double *p = calloc(n, sizeof(double)), *w = calloc(n, sizeof(double));
  int done = 0;
  double rz = 0.0;
  for (int i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; z[i] = P[i] * r[i]; p[i] = z[i]; rz += r[i] * z[i]; }
  const double rz_stop = TAU_CR * rz;
  for (int it = 0; it < iters; ++it) {
    if (!(rz > rz_stop) || !(rz > 0.0)) break;
    apply(ctx, p, w);
    double pw = 0.0;
    for (int i = 0; i < n; ++i) pw += p[i] * w[i];
    if (!(pw > 0.0)) break;
    double alpha = rz / pw;
    for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * w[i]; }
    ++done;
    double rz_new = 0.0;
    for (int i = 0; i < n; ++i) { z[i] = P[i] * r[i]; rz_new += r[i] * z[i]; }
    if (hist) hist[it] = sqrt(rz_new);
    if (it == iters - 1) break;
    double beta = rz_new / rz;
    rz = rz_new;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  free(r); free(z); free(p); free(w);
  return done;
}

typedef struct { int n; const double *A; } dense_ctx;
static void dense_apply(void *c, const double *in, double *out) {
  dense_ctx *d = (dense_ctx *)c;
  for (int i = 0; i < d->n; ++i) {
    double acc = 0;
    for (int j = 0; j < d->n; ++j) acc += d->A[(size_t)i * d->n + j] * in[j];
    out[i] = acc;
  }
}
int orc_pcr_dense(int n, const double *A, const double *b, const double *P, int iters,
                  double *x, double *hist) {
  dense_ctx c = {n, A};
  return pcr_solve(n, dense_apply, &c, b, P, iters, x, hist);
}

int orc_pcg_dense(int n, const double *A, const double *b, const double *P, int iters,
                  double *x, double *hist) {
  dense_ctx c = {n, A};
  return pcg_solve(n, dense_apply, &c, b, P, iters, x, hist);
}

/* ------------------------------------------------------------------------- */
/* Environment state                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t key;
  int fa;          /* feature body: rigid index, or n_rigid + particle index */
  int tb;          /* target body: -1 world, else rigid index */
  double n[3];     /* world normal, fixed for the step (Sec. 3.3) */
  double aL[3];    /* feature point: body frame (rigid) / unused (particle) */
  double bL[3];    /* target point: body frame (rigid) / world point (world) */
  double d;        /* thickness */
  double lam[3];   /* (lambda_n, lambda_f1, lambda_f2) */
} contact;

typedef struct {
  int nent;
  int dof[MAXENT];
  int nd[MAXENT];
  double c[MAXENT][6];
} jrow;

typedef struct {
  orc_desc d;  /* pointers not retained; sizes only */
  int nr, np, nt, nj, maxc;
  /* rigid */
  double *rm, *rI, *rx, *rq, *rv, *rw, *rext;
  int *rshape;
  /* particles */
  double *px, *pv, *pm;
  /* tets */
  int *tid;
  double *Dminv, *Ve, *C1, *D1, *alph;
  double *lmu, *llam;      /* Lame parameters (linear tets) */
  int tet_model, tet_rows; /* ORC_TET_*; rows per tet: 3 (principal stretches) or 6 (strains) */
  /* joints */
  int *jtype, *jbody;
  double *janc, *jaxis, *jref, *jdrive;
  double mu, grav[3];
  int ground;
  double time;
  /* contacts of the current/last step */
  contact *con;
  int nc, overflow;
  contact *prev;   /* last step's contacts (sorted by key) */
  int nprev;
  double *lam_joint_prev, *lam_tet_prev;  /* joint rows (6 each), tet rows (tet_rows each) */
  int have_prev;
  /* scratch sized at create */
  int ndof, maxrows;
  double *hist, *mhist;  /* r_ncp and merit of every accepted iterate of the last step */
  int nhist;
  double *dbg_err, *dbg_cdiag, *dbg_pdiag;
  int dbg_rows;
  double *lam_last;
  int nrows_last;
  /* learned warm start */
  double *mlp;
  int64_t mlp_n;
  /* per-iteration record (orc_set_record): iteration to record (-1 off), the fields */
  int rec_k;
  double *rec[ORC_REC_NFIELDS];
  int rec_len[ORC_REC_NFIELDS];
  /* orc_eval_iterate: the iterate put in place of the start iterate (and the previous
   * one, for the secant) during one step */
  int inj, inj_nc;
  const double *inj_lam, *inj_u, *inj_rx, *inj_rq, *inj_px;
  const double *inj_lam_p, *inj_u_p, *inj_rx_p, *inj_rq_p, *inj_px_p;
} env_t;

static int is_static_rigid(const env_t *e, int i) { return e->rm[i] <= 0.0; }

/* Number of joint rows: 5 hard rows + a drive row when kp or kd is non-zero. */
static int joint_has_drive(const env_t *e, int j) {
  return e->jdrive[6 * j] != 0.0 || e->jdrive[6 * j + 1] != 0.0;
}

void *orc_create(const orc_desc *d, char *err, int errlen) {
  env_t *e = calloc(1, sizeof(env_t));
  e->nr = d->n_rigid; e->np = d->n_particles; e->nt = d->n_tets; e->nj = d->n_joints;
  e->maxc = d->max_contacts;
  e->tet_model = d->tet_model;
  e->tet_rows = d->tet_model == ORC_TET_LINEAR ? 6 : 3;
  int nr = e->nr, np = e->np, nt = e->nt, nj = e->nj;
#define ALLOC(p, n) p = calloc((size_t)((n) > 0 ? (n) : 1), sizeof(*(p)))
  ALLOC(e->rm, nr); ALLOC(e->rI, 3 * nr); ALLOC(e->rx, 3 * nr); ALLOC(e->rq, 4 * nr);
  ALLOC(e->rv, 3 * nr); ALLOC(e->rw, 3 * nr); ALLOC(e->rext, 3 * nr); ALLOC(e->rshape, nr);
  ALLOC(e->px, 3 * np); ALLOC(e->pv, 3 * np); ALLOC(e->pm, np);
  ALLOC(e->tid, 4 * nt); ALLOC(e->Dminv, 9 * nt); ALLOC(e->Ve, nt); ALLOC(e->C1, nt);
  ALLOC(e->D1, nt); ALLOC(e->alph, nt); ALLOC(e->lmu, nt); ALLOC(e->llam, nt);
  ALLOC(e->jtype, nj); ALLOC(e->jbody, 2 * nj); ALLOC(e->janc, 6 * nj); ALLOC(e->jaxis, 6 * nj);
  ALLOC(e->jref, 6 * nj); ALLOC(e->jdrive, 6 * nj);
  ALLOC(e->con, e->maxc); ALLOC(e->prev, e->maxc);
  ALLOC(e->lam_joint_prev, 6 * nj); ALLOC(e->lam_tet_prev, e->tet_rows * nt);
  if (d->tet_model != ORC_TET_NEOHOOKEAN && d->tet_model != ORC_TET_LINEAR) {
    snprintf(err, errlen, "unknown tet model %d", d->tet_model);
    orc_destroy(e);
    return NULL;
  }
  for (int i = 0; i < nr; ++i) {
    e->rm[i] = d->rigid_mass[i];
    for (int k = 0; k < 3; ++k) {
      e->rI[3 * i + k] = d->rigid_inertia[3 * i + k];
      e->rx[3 * i + k] = d->rigid_x[3 * i + k];
      e->rv[3 * i + k] = d->rigid_v[3 * i + k];
      e->rw[3 * i + k] = d->rigid_w[3 * i + k];
      e->rext[3 * i + k] = d->rigid_extent[3 * i + k];
    }
    for (int k = 0; k < 4; ++k) e->rq[4 * i + k] = d->rigid_q[4 * i + k];
    normalize_quat(e->rq + 4 * i);
    e->rshape[i] = d->rigid_shape[i];
    if (e->rm[i] < 0 || (e->rm[i] > 0 && (e->rI[3 * i] <= 0 || e->rI[3 * i + 1] <= 0 || e->rI[3 * i + 2] <= 0))) {
      snprintf(err, errlen, "rigid body %d: invalid mass or inertia", i);
      orc_destroy(e);
      return NULL;
    }
    if (is_static_rigid(e, i)) { /* static obstacles do not move */
      for (int k = 0; k < 3; ++k) { e->rv[3 * i + k] = 0; e->rw[3 * i + k] = 0; }
    }
  }
  for (int p = 0; p < np; ++p) {
    for (int k = 0; k < 3; ++k) { e->px[3 * p + k] = d->particle_x[3 * p + k]; e->pv[3 * p + k] = d->particle_v[3 * p + k]; }
    e->pm[p] = d->particle_mass[p];
  }
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < 4; ++k) {
      int id = d->tet_ids[4 * t + k];
      if (id < 0 || id >= np) { snprintf(err, errlen, "tet %d: bad particle id", t); orc_destroy(e); return NULL; }
      e->tid[4 * t + k] = id;
    }
    /* Sec. 9.2: constant-strain tetrahedron; rest shape D_m from the rest positions. */
    const double *r0 = d->particle_rest + 3 * e->tid[4 * t];
    double Dm[9];
    for (int c = 0; c < 3; ++c) {
      const double *rc = d->particle_rest + 3 * e->tid[4 * t + c + 1];
      for (int r = 0; r < 3; ++r) Dm[3 * r + c] = rc[r] - r0[r];
    }
    double det = m3_det(Dm);
    if (!(fabs(det) > 1e-15)) { snprintf(err, errlen, "tet %d: degenerate rest shape", t); orc_destroy(e); return NULL; }
    m3_inv(Dm, e->Dminv + 9 * t);
    e->Ve[t] = fabs(det) / 6.0;
    double E = d->tet_material[3 * t], nu = d->tet_material[3 * t + 1], rho = d->tet_material[3 * t + 2];
    if (!(E > 0) || !(nu > -1 && nu < 0.5) || !(rho > 0)) { snprintf(err, errlen, "tet %d: bad material", t); orc_destroy(e); return NULL; }
    orc_lame(E, nu, &e->C1[t], &e->D1[t], &e->alph[t]);
    lame_mu_lambda(E, nu, &e->lmu[t], &e->llam[t]);
    /* READING: lumped particle mass, rho V_e / 4 per tet vertex (Sec. 9.3). */
    for (int k = 0; k < 4; ++k) e->pm[e->tid[4 * t + k]] += rho * e->Ve[t] / 4.0;
  }
  for (int p = 0; p < np; ++p)
    if (!(e->pm[p] > 0)) { snprintf(err, errlen, "particle %d has no mass", p); orc_destroy(e); return NULL; }
  for (int j = 0; j < nj; ++j) {
    e->jtype[j] = d->joint_type[j];
    e->jbody[2 * j] = d->joint_body[2 * j];
    e->jbody[2 * j + 1] = d->joint_body[2 * j + 1];
    for (int k = 0; k < 6; ++k) {
      e->janc[6 * j + k] = d->joint_anchor[6 * j + k];
      e->jaxis[6 * j + k] = d->joint_axis[6 * j + k];
      e->jref[6 * j + k] = d->joint_ref[6 * j + k];
      e->jdrive[6 * j + k] = d->joint_drive[6 * j + k];
    }
    int a = e->jbody[2 * j], b = e->jbody[2 * j + 1];
    if (a < -1 || a >= nr || b < 0 || b >= nr || a == b || (e->jtype[j] != 0 && e->jtype[j] != 1)) {
      snprintf(err, errlen, "joint %d: bad bodies or type", j); orc_destroy(e); return NULL;
    }
  }
  e->mu = d->mu;
  for (int k = 0; k < 3; ++k) e->grav[k] = d->gravity[k];
  e->ground = d->ground;
  e->ndof = 6 * nr + 3 * np;
  e->maxrows = 6 * nj + 3 * e->maxc + e->tet_rows * nt;
  ALLOC(e->hist, MAX_HIST); ALLOC(e->mhist, MAX_HIST);
  ALLOC(e->dbg_err, e->maxrows); ALLOC(e->dbg_cdiag, e->maxrows); ALLOC(e->dbg_pdiag, e->maxrows);
  ALLOC(e->lam_last, e->maxrows);
#undef ALLOC
  e->rec_k = -1;
  return e;
}

void orc_destroy(void *p) {
  env_t *e = (env_t *)p;
  if (!e) return;
  free(e->rm); free(e->rI); free(e->rx); free(e->rq); free(e->rv); free(e->rw); free(e->rext); free(e->rshape);
  free(e->px); free(e->pv); free(e->pm);
  free(e->tid); free(e->Dminv); free(e->Ve); free(e->C1); free(e->D1); free(e->alph); free(e->lmu); free(e->llam);
  free(e->jtype); free(e->jbody); free(e->janc); free(e->jaxis); free(e->jref); free(e->jdrive);
  free(e->con); free(e->prev); free(e->lam_joint_prev); free(e->lam_tet_prev);
  free(e->hist); free(e->mhist); free(e->dbg_err); free(e->dbg_cdiag); free(e->dbg_pdiag); free(e->lam_last);
  free(e->mlp);
  for (int f = 0; f < ORC_REC_NFIELDS; ++f) free(e->rec[f]);
  free(e);
}

/* ------------------------------------------------------------------------- */
/* Per-step working set                                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
  env_t *e;
  const orc_params *p;
  double h;
  int ndof, nrows;
  /* start-of-step state */
  double *x0, *q0;        /* rigid x^-, theta^- */
  double *px0;            /* particle x^- */
  double *Iw, *Iwinv;     /* world inertia at q^- (9 per rigid) */
  double *ut;             /* u tilde */
  double *u, *uprev;      /* current / previous Newton iterate velocities */
  double *Hdiag;          /* particle DOF diagonal of H~ (3 per particle) */
  double *lam;            /* multipliers [nrows] */
  /* assembly of the current iterate */
  jrow *J, *Jprev;
  double *err;
  double *Cblk;           /* 9 per row: block entries stored at the block's first row */
  int *blk_start, *blk_size;  /* per row */
  int *row_kind;          /* 0 joint, 1 contact normal, 2 friction, 3 tet */
  double *c_alpha, *c_rn, *c_rf;  /* per contact: alpha of the normal row, r factors */
  int *c_act;             /* per contact: friction rows active */
  int have_prev;
  double *theta_minus;    /* joint drive coordinate at q^- */
  double t_plus;
} step_t;

static int particle_dof(const env_t *e, int p) { return 6 * e->nr + 3 * p; }

/* world position of a body-fixed point; velocity of the point under u */
static void body_point(const env_t *e, int body, const double *local, double *out) {
  if (body < 0) { out[0] = local[0]; out[1] = local[1]; out[2] = local[2]; return; }
  if (body < e->nr) {
    double R[9];
    quat_to_mat(e->rq + 4 * body, R);
    m3_vec(R, local, out);
    for (int k = 0; k < 3; ++k) out[k] += e->rx[3 * body + k];
    return;
  }
  int p = body - e->nr;
  for (int k = 0; k < 3; ++k) out[k] = e->px[3 * p + k];
}

static void body_arm(const env_t *e, int body, const double *local, double *arm) {
  if (body < 0 || body >= e->nr) { arm[0] = arm[1] = arm[2] = 0; return; }
  double R[9];
  quat_to_mat(e->rq + 4 * body, R);
  m3_vec(R, local, arm);
}

static void point_velocity(const env_t *e, const double *u, int body, const double *arm, double *v) {
  v[0] = v[1] = v[2] = 0;
  if (body < 0) return;
  if (body < e->nr) {
    if (is_static_rigid(e, body)) return;
    const double *ub = u + 6 * body;
    double wxr[3];
    v3_cross(ub + 3, arm, wxr);
    for (int k = 0; k < 3; ++k) v[k] = ub[k] + wxr[k];
    return;
  }
  const double *ub = u + particle_dof(e, body - e->nr);
  for (int k = 0; k < 3; ++k) v[k] = ub[k];
}

/* Append a Jacobian entry for a direction `dir` applied at arm `arm` of body
 * (linear part dir, angular part arm x dir), scaled by sgn.  Static and world bodies
 * carry no DOFs and contribute nothing (Sec. 5: J = grad(c) G). */
static void jrow_add_point(const env_t *e, jrow *r, int body, const double *arm, const double *dir, double sgn) {
  if (body < 0) return;
  if (body < e->nr) {
    if (is_static_rigid(e, body)) return;
    int k = r->nent++;
    r->dof[k] = 6 * body; r->nd[k] = 6;
    double axd[3];
    v3_cross(arm, dir, axd);
    for (int i = 0; i < 3; ++i) { r->c[k][i] = sgn * dir[i]; r->c[k][3 + i] = sgn * axd[i]; }
    return;
  }
  int k = r->nent++;
  r->dof[k] = particle_dof(e, body - e->nr); r->nd[k] = 3;
  for (int i = 0; i < 3; ++i) r->c[k][i] = sgn * dir[i];
  for (int i = 3; i < 6; ++i) r->c[k][i] = 0;
}

/* angular-only entry (rotation rows of joints) */
static void jrow_add_ang(const env_t *e, jrow *r, int body, const double *ang) {
  if (body < 0 || is_static_rigid(e, body)) return;
  int k = r->nent++;
  r->dof[k] = 6 * body; r->nd[k] = 6;
  for (int i = 0; i < 3; ++i) { r->c[k][i] = 0; r->c[k][3 + i] = ang[i]; }
}

static double jrow_dot(const jrow *r, const double *v) {
  double acc = 0;
  for (int k = 0; k < r->nent; ++k)
    for (int i = 0; i < r->nd[k]; ++i) acc += r->c[k][i] * v[r->dof[k] + i];
  return acc;
}

static void jrow_scatter(const jrow *r, double s, double *out) {
  for (int k = 0; k < r->nent; ++k)
    for (int i = 0; i < r->nd[k]; ++i) out[r->dof[k] + i] += s * r->c[k][i];
}

static void jrow_scale(jrow *r, double s) {
  for (int k = 0; k < r->nent; ++k)
    for (int i = 0; i < 6; ++i) r->c[k][i] *= s;
}

/* Apply H~^-1 (block diagonal: rigid [1/m I, I_w^-1], particle diag 1/H~_jj). */
static void apply_Hinv(const step_t *S, const double *in, double *out) {
  const env_t *e = S->e;
  for (int i = 0; i < e->nr; ++i) {
    double *o = out + 6 * i;
    const double *v = in + 6 * i;
    if (is_static_rigid(e, i)) { for (int k = 0; k < 6; ++k) o[k] = 0; continue; }
    for (int k = 0; k < 3; ++k) o[k] = v[k] / e->rm[i];
    m3_vec(S->Iwinv + 9 * i, v + 3, o + 3);
  }
  for (int p = 0; p < e->np; ++p)
    for (int k = 0; k < 3; ++k) {
      int dd = particle_dof(e, p) + k;
      out[dd] = in[dd] / S->Hdiag[3 * p + k];
    }
}

/* Apply the mass matrix M~ (Sec. 9: particle m I, rigid diag(m I, I_w)). */
static void apply_M(const step_t *S, const double *in, double *out) {
  const env_t *e = S->e;
  for (int i = 0; i < e->nr; ++i) {
    double *o = out + 6 * i;
    const double *v = in + 6 * i;
    if (is_static_rigid(e, i)) { for (int k = 0; k < 6; ++k) o[k] = 0; continue; }
    for (int k = 0; k < 3; ++k) o[k] = e->rm[i] * v[k];
    m3_vec(S->Iw + 9 * i, v + 3, o + 3);
  }
  for (int p = 0; p < e->np; ++p)
    for (int k = 0; k < 3; ++k) {
      int dd = particle_dof(e, p) + k;
      out[dd] = e->pm[p] * in[dd];
    }
}

static void apply_Minv(const step_t *S, const double *in, double *out) {
  const env_t *e = S->e;
  for (int i = 0; i < e->nr; ++i) {
    double *o = out + 6 * i;
    const double *v = in + 6 * i;
    if (is_static_rigid(e, i)) { for (int k = 0; k < 6; ++k) o[k] = 0; continue; }
    for (int k = 0; k < 3; ++k) o[k] = v[k] / e->rm[i];
    m3_vec(S->Iwinv + 9 * i, v + 3, o + 3);
  }
  for (int p = 0; p < e->np; ++p)
    for (int k = 0; k < 3; ++k) {
      int dd = particle_dof(e, p) + k;
      out[dd] = in[dd] / e->pm[p];
    }
}

/* J_i M~^-1 J_i^T for one row, with M~ (not H~), used for the r factors (Sec. 7). */
static double row_effmass(const step_t *S, const jrow *r) {
  const env_t *e = S->e;
  double acc = 0;
  for (int k = 0; k < r->nent; ++k) {
    int dof = r->dof[k];
    if (dof < 6 * e->nr) {
      int i = dof / 6;
      acc += (r->c[k][0] * r->c[k][0] + r->c[k][1] * r->c[k][1] + r->c[k][2] * r->c[k][2]) / e->rm[i];
      double t[3];
      m3_vec(S->Iwinv + 9 * i, r->c[k] + 3, t);
      acc += v3_dot(r->c[k] + 3, t);
    } else {
      int p = (dof - 6 * e->nr) / 3;
      acc += (r->c[k][0] * r->c[k][0] + r->c[k][1] * r->c[k][1] + r->c[k][2] * r->c[k][2]) / e->pm[p];
    }
  }
  return acc;
}

/* J_i H~^-1 J_i^T for one row (the Jacobi diagonal of Sec. 8.2 without C, eps). */
static double row_hdiag(const step_t *S, const jrow *r) {
  const env_t *e = S->e;
  double acc = 0;
  for (int k = 0; k < r->nent; ++k) {
    int dof = r->dof[k];
    if (dof < 6 * e->nr) {
      int i = dof / 6;
      acc += (r->c[k][0] * r->c[k][0] + r->c[k][1] * r->c[k][1] + r->c[k][2] * r->c[k][2]) / e->rm[i];
      double t[3];
      m3_vec(S->Iwinv + 9 * i, r->c[k] + 3, t);
      acc += v3_dot(r->c[k] + 3, t);
    } else {
      int p = (dof - 6 * e->nr) / 3;
      for (int a = 0; a < 3; ++a) acc += r->c[k][a] * r->c[k][a] / S->Hdiag[3 * p + a];
    }
  }
  return acc;
}

/* ------------------------------------------------------------------------- */
/* Collision detection (Sec. 10: once per step at q^-, candidates from the    */
/* unconstrained velocity).  READING: primitive features and targets:        */
/*   features = box vertices, capsule end spheres, particles;                 */
/*   targets  = ground plane z=0, boxes, capsules (particles only);           */
/* a pair is kept when dist - d + h min(0, n.v_rel(u~)) < margin.            */
/* Candidates are enumerated in a canonical order (features, then targets),   */
/* key = feature_index * n_targets + target_index.                            */
/* ------------------------------------------------------------------------- */
static int n_features_of(const env_t *e, int i) {
  if (e->rshape[i] == 0) return 8;
  if (e->rshape[i] == 1) return 2;
  return 0;
}

static void feature_local(const env_t *e, int i, int v, double *loc, double *thick) {
  const double *ext = e->rext + 3 * i;
  if (e->rshape[i] == 0) {
    loc[0] = (v & 1) ? ext[0] : -ext[0];
    loc[1] = (v & 2) ? ext[1] : -ext[1];
    loc[2] = (v & 4) ? ext[2] : -ext[2];
    *thick = 0.0;
  } else {
    loc[0] = (v & 1) ? ext[1] : -ext[1];
    loc[1] = 0; loc[2] = 0;
    *thick = ext[0];
  }
}

/* Closest-feature query of a world point against target t; returns 0 if no contact
 * geometry (degenerate), else fills n (world), bL (target-local / world), dist
 * (distance of the point from the target's surface-reference minus target thickness),
 * and the target thickness. */
static int target_query(const env_t *e, int t, const double *pw, double *n, double *bL, double *dist,
                        double *tthick) {
  if (t < 0) { /* ground */
    n[0] = 0; n[1] = 0; n[2] = 1;
    bL[0] = pw[0]; bL[1] = pw[1]; bL[2] = 0.0;
    *dist = pw[2];
    *tthick = 0.0;
    return 1;
  }
  double R[9];
  quat_to_mat(e->rq + 4 * t, R);
  double rel[3] = {pw[0] - e->rx[3 * t], pw[1] - e->rx[3 * t + 1], pw[2] - e->rx[3 * t + 2]};
  double pl[3];
  m3_tvec(R, rel, pl);
  const double *ext = e->rext + 3 * t;
  if (e->rshape[t] == 0) {
    int inside = fabs(pl[0]) <= ext[0] && fabs(pl[1]) <= ext[1] && fabs(pl[2]) <= ext[2];
    double nl[3] = {0, 0, 0};
    *tthick = 0.0;
    if (inside) {
      /* least-penetration face, faces ordered -x,+x,-y,+y,-z,+z, ties -> lowest */
      int best = -1;
      double bd = 0;
      for (int f = 0; f < 6; ++f) {
        int ax = f >> 1;
        double sg = (f & 1) ? 1.0 : -1.0;
        double depth = ext[ax] - sg * pl[ax];
        if (best < 0 || depth < bd) { best = f; bd = depth; }
      }
      int ax = best >> 1;
      double sg = (best & 1) ? 1.0 : -1.0;
      nl[ax] = sg;
      bL[0] = pl[0]; bL[1] = pl[1]; bL[2] = pl[2];
      bL[ax] = sg * ext[ax];
      *dist = -bd;
    } else {
      double cl[3];
      for (int k = 0; k < 3; ++k) cl[k] = pl[k] < -ext[k] ? -ext[k] : (pl[k] > ext[k] ? ext[k] : pl[k]);
      double df[3] = {pl[0] - cl[0], pl[1] - cl[1], pl[2] - cl[2]};
      double l = v3_norm(df);
      if (!(l > 1e-9)) return 0;
      for (int k = 0; k < 3; ++k) nl[k] = df[k] / l;
      bL[0] = cl[0]; bL[1] = cl[1]; bL[2] = cl[2];
      *dist = l;
    }
    m3_vec(R, nl, n);
    return 1;
  }
  if (e->rshape[t] == 1) { /* capsule: segment along local x */
    double L = ext[1];
    double tpar = pl[0];
    if (tpar < -L) tpar = -L;
    if (tpar > L) tpar = L;
    double cl[3] = {tpar, 0, 0};
    double df[3] = {pl[0] - cl[0], pl[1], pl[2]};
    double l = v3_norm(df);
    if (!(l > 1e-9)) return 0;
    double nl[3] = {df[0] / l, df[1] / l, df[2] / l};
    m3_vec(R, nl, n);
    bL[0] = cl[0]; bL[1] = cl[1]; bL[2] = cl[2];
    *dist = l - ext[0];
    *tthick = ext[0];
    return 1;
  }
  return 0;
}

/* READING (box vertex against a box): the contact plane is the face of the target
 * box B whose outward normal n_f separates the two boxes best,
 *   sep_f = n_f.(x_A - x_B) - ext_B[axis(f)] - sum_i |n_f . R_A e_i| ext_A[i],
 * faces ordered -x,+x,-y,+y,-z,+z, ties -> lowest index.  Every vertex of A whose
 * projection falls on that face (extended by the margin) gets a vertex-plane
 * contact with it; this keeps stacked boxes on face normals. */
static int box_ref_face(const env_t *e, int A, int B) {
  double RA[9], RB[9];
  quat_to_mat(e->rq + 4 * A, RA);
  quat_to_mat(e->rq + 4 * B, RB);
  double d[3] = {e->rx[3 * A] - e->rx[3 * B], e->rx[3 * A + 1] - e->rx[3 * B + 1], e->rx[3 * A + 2] - e->rx[3 * B + 2]};
  const double *eA = e->rext + 3 * A, *eB = e->rext + 3 * B;
  int best = 0;
  double bs = 0;
  for (int f = 0; f < 6; ++f) {
    int ax = f >> 1;
    double sg = (f & 1) ? 1.0 : -1.0;
    double nf[3] = {sg * RB[ax], sg * RB[3 + ax], sg * RB[6 + ax]};
    double sep = v3_dot(nf, d) - eB[ax];
    for (int i = 0; i < 3; ++i) {
      double ai[3] = {RA[i], RA[3 + i], RA[6 + i]};
      sep -= fabs(v3_dot(nf, ai)) * eA[i];
    }
    if (f == 0 || sep > bs) { best = f; bs = sep; }
  }
  return best;
}

static int box_face_query(const env_t *e, int t, int face, const double *pw, double margin, double *n,
                          double *bL, double *dist) {
  double R[9];
  quat_to_mat(e->rq + 4 * t, R);
  double rel[3] = {pw[0] - e->rx[3 * t], pw[1] - e->rx[3 * t + 1], pw[2] - e->rx[3 * t + 2]};
  double pl[3];
  m3_tvec(R, rel, pl);
  const double *ext = e->rext + 3 * t;
  int ax = face >> 1;
  double sg = (face & 1) ? 1.0 : -1.0;
  for (int o = 0; o < 3; ++o)
    if (o != ax && fabs(pl[o]) > ext[o] + margin) return 0;
  double nl[3] = {0, 0, 0};
  nl[ax] = sg;
  m3_vec(R, nl, n);
  bL[0] = pl[0]; bL[1] = pl[1]; bL[2] = pl[2];
  bL[ax] = sg * ext[ax];
  *dist = sg * pl[ax] - ext[ax];
  return 1;
}

static void generate_contacts(step_t *S) {
  env_t *e = S->e;
  const double h = S->h, margin = S->p->margin;
  int ntargets = (e->ground ? 1 : 0) + e->nr;
  int64_t feat_index = 0;
  e->nc = 0;
  e->overflow = 0;
  int nfeat_total = 0;
  for (int i = 0; i < e->nr; ++i) nfeat_total += n_features_of(e, i);
  nfeat_total += e->np;
  (void)nfeat_total;
  /* features: rigid body features in body order, then particles */
  for (int pass = 0; pass < 2; ++pass) {
    int nitems = pass == 0 ? e->nr : e->np;
    for (int it = 0; it < nitems; ++it) {
      int nf = pass == 0 ? n_features_of(e, it) : 1;
      for (int v = 0; v < nf; ++v, ++feat_index) {
        int fbody = pass == 0 ? it : e->nr + it;
        int fis_particle = pass == 1;
        int fis_capsule = pass == 0 && e->rshape[it] == 1;
        if (pass == 0 && is_static_rigid(e, it)) continue;
        double loc[3] = {0, 0, 0}, fthick = 0.0;
        if (pass == 0) feature_local(e, it, v, loc, &fthick);
        double pw[3];
        body_point(e, fbody, loc, pw);
        double arm_a[3];
        body_arm(e, fbody, loc, arm_a);
        int fis_box = pass == 0 && e->rshape[it] == 0;
        for (int ti = 0; ti < ntargets; ++ti) {
          int t = e->ground ? ti - 1 : ti;
          if (t >= 0) {
            if (t == fbody) continue;
            int ts = e->rshape[t];
            if (ts == 2) continue;
            if (ts == 1 && !fis_particle) continue;          /* capsules are targets of particles only */
            if (fis_capsule && t >= 0) continue;             /* capsule ends collide with the ground only */
            if (pass == 0 && ts == 0 && e->rshape[it] != 0) continue;
          }
          double n[3], bL[3], dist, tthick = 0.0;
          if (fis_box && t >= 0) {
            if (!box_face_query(e, t, box_ref_face(e, it, t), pw, margin, n, bL, &dist)) continue;
          } else if (!target_query(e, t, pw, n, bL, &dist, &tthick)) {
            continue;
          }
          double dtot = fthick + tthick;
          double gap = dist - fthick; /* target_query already removed the target thickness */
          /* relative velocity of the two points under u~ */
          double va[3], vb[3], arm_b[3];
          point_velocity(e, S->ut, fbody, arm_a, va);
          if (t >= 0) { body_arm(e, t, bL, arm_b); point_velocity(e, S->ut, t, arm_b, vb); }
          else { vb[0] = vb[1] = vb[2] = 0; }
          double vn = n[0] * (va[0] - vb[0]) + n[1] * (va[1] - vb[1]) + n[2] * (va[2] - vb[2]);
          double pred = gap + h * (vn < 0 ? vn : 0.0);
          if (!(pred < margin)) continue;
          if (e->nc >= e->maxc) { e->overflow++; continue; }
          contact *c = &e->con[e->nc++];
          c->key = feat_index * (int64_t)ntargets + ti;
          c->fa = fbody;
          c->tb = t;
          for (int k = 0; k < 3; ++k) { c->n[k] = n[k]; c->aL[k] = loc[k]; c->bL[k] = bL[k]; }
          c->d = dtot;
          c->lam[0] = c->lam[1] = c->lam[2] = 0;
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Row assembly (Sec. 6.1 eq. newton_system, Appendix A/B)                    */
/* ------------------------------------------------------------------------- */

/* Joint frames at the current configuration. */
typedef struct {
  double PA[3], PB[3], rA[3], rB[3];
  double a[3], t1[3], t2[3];     /* A's axis and perpendiculars (world) */
  double b[3], s1[3], s2[3];     /* B's axis and perpendiculars (world) */
} jframe;

static void joint_frame(const env_t *e, int j, jframe *f) {
  int A = e->jbody[2 * j], B = e->jbody[2 * j + 1];
  const double *pA = e->janc + 6 * j, *pB = pA + 3, *aA = e->jaxis + 6 * j, *aB = aA + 3;
  const double *tA = e->jref + 6 * j, *tB = tA + 3;
  double RA[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, RB[9], xA[3] = {0, 0, 0};
  if (A >= 0) { quat_to_mat(e->rq + 4 * A, RA); for (int k = 0; k < 3; ++k) xA[k] = e->rx[3 * A + k]; }
  quat_to_mat(e->rq + 4 * B, RB);
  m3_vec(RA, pA, f->rA);
  m3_vec(RB, pB, f->rB);
  for (int k = 0; k < 3; ++k) { f->PA[k] = xA[k] + f->rA[k]; f->PB[k] = e->rx[3 * B + k] + f->rB[k]; }
  m3_vec(RA, aA, f->a); m3_vec(RA, tA, f->t1); v3_cross(f->a, f->t1, f->t2);
  m3_vec(RB, aB, f->b); m3_vec(RB, tB, f->s1); v3_cross(f->b, f->s1, f->s2);
}

/* READING (the paper gives no joint formulas): joint coordinate of the drive row.
 * Revolute: angle of B's reference direction about A's axis, atan2(a.(t1 x s1), t1.s1).
 * Prismatic: displacement of B's anchor along A's axis. */
static double joint_coordinate(const env_t *e, int j) {
  jframe f;
  joint_frame(e, j, &f);
  if (e->jtype[j] == 0) {
    double c[3];
    v3_cross(f.t1, f.s1, c);
    return atan2(v3_dot(f.a, c), v3_dot(f.t1, f.s1));
  }
  double d[3] = {f.PB[0] - f.PA[0], f.PB[1] - f.PA[1], f.PB[2] - f.PA[2]};
  return v3_dot(f.a, d);
}

/* Joint rows at the current configuration (READING of Sec. 3.1-3.2 for revolute and
 * prismatic joints): five hard rows c(q) = 0 and, when driven, one soft row.
 * J rows are grad(c) G, i.e. derivatives w.r.t. (v, omega_world).
 * Returns the constraint values in c[6] and fills 6 rows (row 5 empty if undriven). */
static void joint_rows(const env_t *e, int j, jrow *rows, double *c) {
  int A = e->jbody[2 * j], B = e->jbody[2 * j + 1];
  jframe f;
  joint_frame(e, j, &f);
  for (int r = 0; r < 6; ++r) { rows[r].nent = 0; c[r] = 0; }
  if (e->jtype[j] == 0) {
    /* anchor coincidence: c_k = e_k . (PA - PB) */
    for (int k = 0; k < 3; ++k) {
      double ek[3] = {0, 0, 0};
      ek[k] = 1.0;
      c[k] = f.PA[k] - f.PB[k];
      jrow_add_point(e, &rows[k], A, f.rA, ek, 1.0);
      jrow_add_point(e, &rows[k], B, f.rB, ek, -1.0);
    }
    /* axis alignment: c = t_j . b for the two perpendiculars of A's axis */
    const double *tj[2] = {f.t1, f.t2};
    for (int k = 0; k < 2; ++k) {
      double txb[3];
      v3_cross(tj[k], f.b, txb);
      c[3 + k] = v3_dot(tj[k], f.b);
      jrow_add_ang(e, &rows[3 + k], A, txb);
      double m[3] = {-txb[0], -txb[1], -txb[2]};
      jrow_add_ang(e, &rows[3 + k], B, m);
    }
    if (joint_has_drive(e, j)) {
      c[5] = joint_coordinate(e, j);
      double ma[3] = {-f.a[0], -f.a[1], -f.a[2]};
      jrow_add_ang(e, &rows[5], A, ma);
      jrow_add_ang(e, &rows[5], B, f.a);
    }
  } else {
    double d[3] = {f.PB[0] - f.PA[0], f.PB[1] - f.PA[1], f.PB[2] - f.PA[2]};
    const double *tj[2] = {f.t1, f.t2};
    /* point on axis: c = t_j . (PB - PA) */
    for (int k = 0; k < 2; ++k) {
      c[k] = v3_dot(tj[k], d);
      double txd[3], rxt[3];
      v3_cross(tj[k], d, txd);
      v3_cross(f.rA, tj[k], rxt);
      if (A >= 0 && !is_static_rigid(e, A)) {
        int q = rows[k].nent++;
        rows[k].dof[q] = 6 * A; rows[k].nd[q] = 6;
        for (int i = 0; i < 3; ++i) { rows[k].c[q][i] = -tj[k][i]; rows[k].c[q][3 + i] = txd[i] - rxt[i]; }
      }
      jrow_add_point(e, &rows[k], B, f.rB, tj[k], 1.0);
    }
    /* orientation lock: c = (t1.s2, t2.b, a.s1) */
    const double *ea[3] = {f.t1, f.t2, f.a}, *eb[3] = {f.s2, f.b, f.s1};
    for (int k = 0; k < 3; ++k) {
      double x[3];
      v3_cross(ea[k], eb[k], x);
      c[2 + k] = v3_dot(ea[k], eb[k]);
      jrow_add_ang(e, &rows[2 + k], A, x);
      double m[3] = {-x[0], -x[1], -x[2]};
      jrow_add_ang(e, &rows[2 + k], B, m);
    }
    if (joint_has_drive(e, j)) {
      c[5] = v3_dot(f.a, d);
      double axd[3], rxa[3];
      v3_cross(f.a, d, axd);
      v3_cross(f.rA, f.a, rxa);
      if (A >= 0 && !is_static_rigid(e, A)) {
        int q = rows[5].nent++;
        rows[5].dof[q] = 6 * A; rows[5].nd[q] = 6;
        for (int i = 0; i < 3; ++i) { rows[5].c[q][i] = -f.a[i]; rows[5].c[q][3 + i] = axd[i] - rxa[i]; }
      }
      jrow_add_point(e, &rows[5], B, f.rB, f.a, 1.0);
    }
  }
}

/* Physical contact rows (Sec. 3.3-3.4 with Sec. 5): normal [n; r_A x n | -n; -r_B x n],
 * tangents likewise with d1, d2.  Also returns C_n = n.(a - b) - d and the
 * relative velocity projections. */
static void contact_rows(const env_t *e, const contact *c, jrow *rn, jrow *rt1, jrow *rt2, double *Cn) {
  double armA[3], armB[3], pa[3], pb[3], d1[3], d2[3];
  body_arm(e, c->fa, c->aL, armA);
  body_point(e, c->fa, c->aL, pa);
  if (c->tb >= 0) { body_arm(e, c->tb, c->bL, armB); body_point(e, c->tb, c->bL, pb); }
  else { armB[0] = armB[1] = armB[2] = 0; pb[0] = c->bL[0]; pb[1] = c->bL[1]; pb[2] = c->bL[2]; }
  *Cn = c->n[0] * (pa[0] - pb[0]) + c->n[1] * (pa[1] - pb[1]) + c->n[2] * (pa[2] - pb[2]) - c->d;
  orc_tangent_basis(c->n, d1, d2);
  rn->nent = rt1->nent = rt2->nent = 0;
  jrow_add_point(e, rn, c->fa, armA, c->n, 1.0);
  jrow_add_point(e, rn, c->tb, armB, c->n, -1.0);
  jrow_add_point(e, rt1, c->fa, armA, d1, 1.0);
  jrow_add_point(e, rt1, c->tb, armB, d1, -1.0);
  jrow_add_point(e, rt2, c->fa, armA, d2, 1.0);
  jrow_add_point(e, rt2, c->tb, armB, d2, -1.0);
}

/* Tet rows (Sec. 9.1-9.2, Appendix B): F = D_s D_m^-1, signed SVD, s_i; rows
 * ds_i/dx_j = u_i (D_m^-1 v_i)_j for vertices 1..3 and minus their sum for vertex 0. */
static void tet_rows(const env_t *e, int t, jrow *rows, double *s, double *Sout_U, double *Sout_W) {
  const int *id = e->tid + 4 * t;
  const double *x0 = e->px + 3 * id[0];
  double Ds[9], F[9], U[9], V[9];
  for (int c = 0; c < 3; ++c) {
    const double *xc = e->px + 3 * id[c + 1];
    for (int r = 0; r < 3; ++r) Ds[3 * r + c] = xc[r] - x0[r];
  }
  m3_mul(Ds, e->Dminv + 9 * t, F);
  orc_svd3(F, U, s, V);
  for (int i = 0; i < 3; ++i) {
    double ui[3] = {U[i], U[3 + i], U[6 + i]};
    double vi[3] = {V[i], V[3 + i], V[6 + i]};
    double wi[3];
    m3_vec(e->Dminv + 9 * t, vi, wi);
    jrow *r = &rows[i];
    r->nent = 4;
    double wsum = wi[0] + wi[1] + wi[2];
    for (int k = 0; k < 4; ++k) {
      r->dof[k] = particle_dof(e, id[k]);
      r->nd[k] = 3;
      double coef = k == 0 ? -wsum : wi[k - 1];
      for (int a = 0; a < 3; ++a) r->c[k][a] = coef * ui[a];
      for (int a = 3; a < 6; ++a) r->c[k][a] = 0;
    }
    if (Sout_U) for (int a = 0; a < 3; ++a) Sout_U[3 * i + a] = ui[a];
    if (Sout_W) for (int a = 0; a < 3; ++a) Sout_W[3 * i + a] = wi[a];
  }
}

/* Linear tet rows (Sec. 9.2): the six strains of the current configuration and their
 * rows ds/dx (READING: at fixed R, see corot_rows); the stress c = V_e K_e s. */
static void linear_tet_rows(const env_t *e, int t, jrow *rows, double *eps6, double *c6) {
  const int *id = e->tid + 4 * t;
  double x12[12], Ds[9], F[9], R[9], g[6][4][3];
  for (int k = 0; k < 4; ++k)
    for (int a = 0; a < 3; ++a) x12[3 * k + a] = e->px[3 * id[k] + a];
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) Ds[3 * r + c] = x12[3 * (c + 1) + r] - x12[r];
  m3_mul(Ds, e->Dminv + 9 * t, F);
  corot_strain(F, R, eps6);
  if (rows) {
    corot_rows(R, e->Dminv + 9 * t, g);
    for (int q = 0; q < 6; ++q) {
      jrow *r = &rows[q];
      r->nent = 4;
      for (int k = 0; k < 4; ++k) {
        r->dof[k] = particle_dof(e, id[k]);
        r->nd[k] = 3;
        for (int a = 0; a < 3; ++a) r->c[k][a] = g[q][k][a];
        for (int a = 3; a < 6; ++a) r->c[k][a] = 0;
      }
    }
  }
  double K[36];
  lin_stiffness(e->lmu[t], e->llam[t], K);
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 6; ++j) acc += K[6 * i + j] * eps6[j];
    c6[i] = e->Ve[t] * acc;
  }
}

/* Row layout of an environment: joints (6 rows each), contacts (3 each), tets (3 or 6 each). */
static int row_joint(const env_t *e, int j) { (void)e; return 6 * j; }
static int row_contact(const env_t *e, int c) { return 6 * e->nj + 3 * c; }
static int row_tet(const env_t *e, int t) { return 6 * e->nj + 3 * e->nc + e->tet_rows * t; }

/* r-factors of one contact (Sec. 7 eq. rscaling).  READING: friction uses the mean of
 * the two tangent diagonals, identity mode r = 1, h^2 mode r_n = h^2, r_f = h. */
static void contact_r(const step_t *S, const jrow *rn, const jrow *rt1, const jrow *rt2, double *r_n, double *r_f) {
  double h = S->h;
  if (S->p->rmode == 0) { *r_n = 1.0; *r_f = 1.0; return; }
  if (S->p->rmode == 1) { *r_n = h * h; *r_f = h; return; }
  *r_n = h * h * row_effmass(S, rn);
  *r_f = h * 0.5 * (row_effmass(S, rt1) + row_effmass(S, rt2));
}

/* Full assembly at the current iterate (q^k, u^k, lambda^k):
 * rows J, compliance blocks C, constraint errors err (Sec. 6.1). */
static void assemble(step_t *S) {
  env_t *e = S->e;
  const double h = S->h;
  const orc_params *p = S->p;
  /* joints */
  for (int j = 0; j < e->nj; ++j) {
    int r0 = row_joint(e, j);
    double c[6];
    joint_rows(e, j, S->J + r0, c);
    for (int r = 0; r < 6; ++r) {
      int row = r0 + r;
      S->blk_start[row] = row; S->blk_size[row] = 1; S->row_kind[row] = 0;
      memset(S->Cblk + 9 * row, 0, 9 * sizeof(double));
      double Ecomp = 0.0, cval = c[r];
      if (r == 5) {
        if (joint_has_drive(e, j)) {
          /* READING: implicit PD drive as a soft row under backward Euler:
           * k_eff = kp + kd/h, E = 1/k_eff, target theta_eff =
           * (kp theta*(t+) + (kd/h) theta(q^-)) / k_eff; c = theta(q) - theta_eff. */
          const double *dr = e->jdrive + 6 * j;
          double keff = dr[0] + dr[1] / h;
          double target = dr[5] + dr[2] * sin(2.0 * M_PI * dr[3] * S->t_plus + dr[4]);
          double teff = (dr[0] * target + (dr[1] / h) * S->theta_minus[j]) / keff;
          cval = c[5] - teff;
          Ecomp = 1.0 / keff;
        } else {
          /* undriven: an empty row that keeps its multiplier at zero */
          cval = 0.0;
          Ecomp = h * h;  /* gives C = 1 */
        }
      }
      S->Cblk[9 * row] = Ecomp / (h * h);
      S->err[row] = (cval + Ecomp * S->lam[row]) / h;
    }
  }
  /* contacts */
  for (int ci = 0; ci < e->nc; ++ci) {
    contact *c = &e->con[ci];
    int r0 = row_contact(e, ci);
    jrow *rn = S->J + r0, *rt1 = rn + 1, *rt2 = rn + 2;
    double Cn;
    contact_rows(e, c, rn, rt1, rt2, &Cn);
    double r_n, r_f;
    contact_r(S, rn, rt1, rt2, &r_n, &r_f);
    double lam_n = S->lam[r0], lf1 = S->lam[r0 + 1], lf2 = S->lam[r0 + 2];
    double phi, al, be;
    if (p->ncp == 1) orc_ncp_min(Cn, lam_n, r_n, &phi, &al, &be);
    else orc_ncp_fb(Cn, lam_n, r_n, &phi, &al, &be);
    /* Sec. 4 eq. fb_grad1 / Sec. 6.1: J_n = alpha grad(C) G, C_nn = S/h^2 with S = beta r,
     * err_n = phi / h.  READING: the same alpha-scaled rows are used in the momentum
     * balance (literal form). */
    jrow_scale(rn, al);
    S->c_alpha[ci] = al; S->c_rn[ci] = r_n; S->c_rf[ci] = r_f; S->c_act[ci] = 0;
    for (int k = 0; k < 3; ++k) {
      S->blk_start[r0 + k] = r0 + k; S->blk_size[r0 + k] = 1;
      memset(S->Cblk + 9 * (r0 + k), 0, 9 * sizeof(double));
    }
    S->row_kind[r0] = 1; S->row_kind[r0 + 1] = 2; S->row_kind[r0 + 2] = 2;
    S->Cblk[9 * r0] = be * r_n / (h * h);
    S->err[r0] = phi / h;
    /* friction (Sec. 4.3, Appendix A.2): active iff mu lam_n > 0 */
    double v1 = 0.0, v2 = 0.0, W = INFINITY;
    if (e->mu * lam_n > 0.0) {
      v1 = jrow_dot(rt1, S->u); v2 = jrow_dot(rt2, S->u);
      double vn = sqrt(v1 * v1 + v2 * v2);
      double lfn = sqrt(lf1 * lf1 + lf2 * lf2);
      W = orc_friction_w(p->ncp, vn, lam_n, lfn, e->mu, r_f);
    }
    if (isfinite(W)) {
      S->c_act[ci] = 1;
      S->Cblk[9 * (r0 + 1)] = W / h;
      S->Cblk[9 * (r0 + 2)] = W / h;
      S->err[r0 + 1] = v1 + W * lf1;
      S->err[r0 + 2] = v2 + W * lf2;
    } else {
      /* READING: inactive friction rows (mu lam_n <= 0, or W infinite) are zeroed;
       * compliance r_f/h and error r_f lambda_f drive the multipliers to zero
       * (Delta lambda_f = -lambda_f). */
      rt1->nent = 0; rt2->nent = 0;
      S->Cblk[9 * (r0 + 1)] = r_f / h;
      S->Cblk[9 * (r0 + 2)] = r_f / h;
      S->err[r0 + 1] = r_f * lf1;
      S->err[r0 + 2] = r_f * lf2;
    }
  }
  /* tets (Sec. 9.1-9.2: generalised compliance of a continuum material) */
  for (int t = 0; t < e->nt && e->tet_model == ORC_TET_LINEAR; ++t) {
    /* linear material: 6 strain rows, constant compliance E = (V_e K_e)^-1, which is
     * block diagonal (normal strains 3x3, shears 1x1); err = E (c + lambda) / h */
    int r0 = row_tet(e, t);
    double eps[6], c6[6], C36[36];
    linear_tet_rows(e, t, S->J + r0, eps, c6);
    lin_compliance(e->lmu[t], e->llam[t], e->Ve[t], C36);
    for (int q = 0; q < 6; ++q) {
      double acc = 0.0;
      for (int k = 0; k < 6; ++k) acc += C36[6 * q + k] * (c6[k] + S->lam[r0 + k]);
      S->err[r0 + q] = acc / h;
      S->row_kind[r0 + q] = 3;
      S->blk_start[r0 + q] = q < 3 ? r0 : r0 + q;
      S->blk_size[r0 + q] = q < 3 ? 3 : 1;
      memset(S->Cblk + 9 * (r0 + q), 0, 9 * sizeof(double));
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S->Cblk[9 * r0 + 3 * i + j] = C36[6 * i + j] / (h * h);
    for (int q = 3; q < 6; ++q) S->Cblk[9 * (r0 + q)] = C36[6 * q + q] / (h * h);
  }
  for (int t = 0; t < e->nt && e->tet_model == ORC_TET_NEOHOOKEAN; ++t) {
    int r0 = row_tet(e, t);
    double s[3];
    tet_rows(e, t, S->J + r0, s, NULL, NULL);
    double grad[3], hs[9], E[9];
    orc_neohookean(s, e->C1[t], e->D1[t], e->alph[t], NULL, grad, hs);
    double Ve = e->Ve[t];
    double cst[3] = {Ve * grad[0], Ve * grad[1], Ve * grad[2]};
    for (int k = 0; k < 9; ++k) hs[k] *= Ve;
    orc_compliance3(hs, CLAMP_FEM * 2.0 * e->C1[t] * Ve, p->fem_mode, E);
    double cl[3] = {cst[0] + S->lam[r0], cst[1] + S->lam[r0 + 1], cst[2] + S->lam[r0 + 2]};
    double Ecl[3];
    m3_vec(E, cl, Ecl);
    for (int k = 0; k < 3; ++k) {
      S->blk_start[r0 + k] = r0; S->blk_size[r0 + k] = 3; S->row_kind[r0 + k] = 3;
      S->err[r0 + k] = Ecl[k] / h;   /* J dq + E dlam = -E (c + lam) divided by h */
    }
    for (int k = 0; k < 9; ++k) S->Cblk[9 * r0 + k] = E[k] / (h * h);
  }
}

/* A z = J H~^-1 J^T z + C z + eps z (Sec. 6.2 eq. schur_system with Sec. 8.4). */
typedef struct { step_t *S; double *tmp1, *tmp2; } schur_ctx;
static void schur_apply(void *vc, const double *z, double *out) {
  schur_ctx *sc = (schur_ctx *)vc;
  step_t *S = sc->S;
  memset(sc->tmp1, 0, S->ndof * sizeof(double));
  for (int r = 0; r < S->nrows; ++r) jrow_scatter(&S->J[r], z[r], sc->tmp1);
  apply_Hinv(S, sc->tmp1, sc->tmp2);
  for (int r = 0; r < S->nrows; ++r) {
    double acc = jrow_dot(&S->J[r], sc->tmp2);
    int b0 = S->blk_start[r], bs = S->blk_size[r], ri = r - b0;
    for (int k = 0; k < bs; ++k) acc += S->Cblk[9 * b0 + 3 * ri + k] * z[b0 + k];
    out[r] = acc + S->p->eps * z[r];
  }
}

/* Position update (Alg. 1; READING: q^{k+1} = q^- + h G(q^k) u^{k+1}, quaternion
 * normalised after every update). */
static void update_positions(step_t *S) {
  env_t *e = S->e;
  const double h = S->h;
  for (int i = 0; i < e->nr; ++i) {
    if (is_static_rigid(e, i)) continue;
    const double *u = S->u + 6 * i;
    for (int k = 0; k < 3; ++k) e->rx[3 * i + k] = S->x0[3 * i + k] + h * u[k];
    double Q[12], th[4];
    orc_quat_kinematic(e->rq + 4 * i, Q);
    for (int r = 0; r < 4; ++r)
      th[r] = S->q0[4 * i + r] + 0.5 * h * (Q[3 * r] * u[3] + Q[3 * r + 1] * u[4] + Q[3 * r + 2] * u[5]);
    double l = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2] + th[3] * th[3]);
    for (int r = 0; r < 4; ++r) e->rq[4 * i + r] = th[r] / l;
  }
  for (int p = 0; p < e->np; ++p)
    for (int k = 0; k < 3; ++k) e->px[3 * p + k] = S->px0[3 * p + k] + h * S->u[particle_dof(e, p) + k];
}

/* ------------------------------------------------------------------------- */
/* Islands (Sec. 11 suggests them): dynamic bodies connected by joints, tets  */
/* or contacts; static bodies and the world connect nothing.  Union by the    */
/* smaller index, so every island is named by its lowest body (deterministic). */
/* Rows take the island of their element's dynamic body; rows touching no     */
/* dynamic body form one extra group.                                          */
/* ------------------------------------------------------------------------- */
static int uf_find(int *par, int a) {
  while (par[a] != a) { par[a] = par[par[a]]; a = par[a]; }
  return a;
}
static void uf_union(int *par, int a, int b) {
  a = uf_find(par, a); b = uf_find(par, b);
  if (a < b) par[b] = a; else if (b < a) par[a] = b;
}
static int body_dynamic(const env_t *e, int b) { return b >= 0 && (b >= e->nr || !is_static_rigid(e, b)); }

static void row_islands(const env_t *e, int *row_isl, int *body_isl) {
  int nb = e->nr + e->np;
  int *par = malloc((nb + 1) * sizeof(int));
  for (int i = 0; i <= nb; ++i) par[i] = i;
  for (int j = 0; j < e->nj; ++j) {
    int a = e->jbody[2 * j], b = e->jbody[2 * j + 1];
    if (body_dynamic(e, a) && body_dynamic(e, b)) uf_union(par, a, b);
  }
  for (int t = 0; t < e->nt; ++t)
    for (int k = 1; k < 4; ++k) uf_union(par, e->nr + e->tid[4 * t], e->nr + e->tid[4 * t + k]);
  for (int ci = 0; ci < e->nc; ++ci) {
    const contact *c = &e->con[ci];
    if (body_dynamic(e, c->fa) && body_dynamic(e, c->tb)) uf_union(par, c->fa, c->tb);
  }
  for (int j = 0; j < e->nj; ++j) {
    int a = e->jbody[2 * j], b = e->jbody[2 * j + 1];
    int isl = body_dynamic(e, b) ? uf_find(par, b) : (body_dynamic(e, a) ? uf_find(par, a) : nb);
    for (int r = 0; r < 6; ++r) row_isl[6 * j + r] = isl;
  }
  for (int ci = 0; ci < e->nc; ++ci) {
    const contact *c = &e->con[ci];
    int isl = body_dynamic(e, c->fa) ? uf_find(par, c->fa) : (body_dynamic(e, c->tb) ? uf_find(par, c->tb) : nb);
    for (int r = 0; r < 3; ++r) row_isl[6 * e->nj + 3 * ci + r] = isl;
  }
  for (int t = 0; t < e->nt; ++t) {
    int isl = uf_find(par, e->nr + e->tid[4 * t]);
    for (int r = 0; r < e->tet_rows; ++r) row_isl[row_tet(e, t) + r] = isl;
  }
  for (int b = 0; b < nb; ++b) body_isl[b] = body_dynamic(e, b) ? uf_find(par, b) : -1;
  free(par);
}

static int prev_lookup(const env_t *e, int64_t key) {
  int lo = 0, hi = e->nprev - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (e->prev[mid].key == key) return mid;
    if (e->prev[mid].key < key) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

static void mlp_predict(const env_t *e, const double *feat, double *out);
static void contact_features(const step_t *S, const contact *c, double *f);

/* Start iterate (Sec. 8.1).  Zero start: u0 = 0, lambda0 = 0.  READING for warm
 * starts: lambda0 projected into the admissible set and u0 = u~ + h M~^-1 J(q^-)^T lambda0. */
static void start_iterate(step_t *S) {
  env_t *e = S->e;
  memset(S->lam, 0, S->nrows * sizeof(double));
  memset(S->u, 0, S->ndof * sizeof(double));
  if (S->p->warm == 0) return;
  for (int ci = 0; ci < e->nc; ++ci) {
    contact *c = &e->con[ci];
    double l[3] = {0, 0, 0};
    /* mode 3: the previous-step multipliers where the key existed in the previous
     * step, the network's prediction for a new contact */
    const int known = e->have_prev && prev_lookup(e, c->key) >= 0;
    if ((S->p->warm == 2 || (S->p->warm == 3 && !known)) && e->mlp) {
      double f[MLP_IN];
      contact_features(S, c, f);
      mlp_predict(e, f, l);
    } else {
      int k = e->have_prev ? prev_lookup(e, c->key) : -1;
      if (k >= 0) { l[0] = e->prev[k].lam[0]; l[1] = e->prev[k].lam[1]; l[2] = e->prev[k].lam[2]; }
    }
    if (!(l[0] == l[0]) || !(l[1] == l[1]) || !(l[2] == l[2])) { l[0] = l[1] = l[2] = 0; }
    if (l[0] < 0) l[0] = 0;
    double lf = sqrt(l[1] * l[1] + l[2] * l[2]), lim = e->mu * l[0];
    if (lf > lim) { double sc = lf > 0 ? lim / lf : 0.0; l[1] *= sc; l[2] *= sc; }
    int r0 = row_contact(e, ci);
    S->lam[r0] = l[0]; S->lam[r0 + 1] = l[1]; S->lam[r0 + 2] = l[2];
  }
  if (e->have_prev)
    for (int j = 0; j < e->nj; ++j)
      for (int r = 0; r < 6; ++r) S->lam[row_joint(e, j) + r] = e->lam_joint_prev[6 * j + r];
  /* READING: a tet's multipliers are stresses in the principal basis of the current
   * configuration, and that basis (even its row order) changes from step to step, so
   * the previous step's values do not carry over; the warm start uses the stress of
   * the start configuration instead, lambda0 = -V_e dPsi/ds(s(q^-)), whose force
   * J^T lambda0 is the elastic force at q^-.  The strains of a linear tet live in its
   * rotated frame, which turns with the element, and take the same rule,
   * lambda0 = -V_e K_e s(q^-). */
  for (int t = 0; t < e->nt && e->tet_model == ORC_TET_LINEAR; ++t) {
    double eps[6], c6[6];
    linear_tet_rows(e, t, NULL, eps, c6);
    for (int r = 0; r < 6; ++r) S->lam[row_tet(e, t) + r] = -c6[r];
  }
  for (int t = 0; t < e->nt && e->tet_model == ORC_TET_NEOHOOKEAN; ++t) {
    jrow rows3[3];
    double s3[3], grad[3];
    tet_rows(e, t, rows3, s3, NULL, NULL);
    orc_neohookean(s3, e->C1[t], e->D1[t], e->alph[t], NULL, grad, NULL);
    for (int r = 0; r < 3; ++r) S->lam[row_tet(e, t) + r] = -e->Ve[t] * grad[r];
  }
  /* READING: the paper leaves u0 of a warm start open.  The start velocity is the
   * previous step's velocity u^- (static bodies stay at rest), so a warm start takes
   * both halves of the previous solution; only lambda0 differs between the modes.
   * (Mapping lambda0 to velocities through the inverse mass made light FEM particles
   * overshoot under contact forces balanced by the end-of-step stress.) */
  for (int i = 0; i < e->nr; ++i) {
    if (is_static_rigid(e, i)) continue;
    for (int k = 0; k < 3; ++k) { S->u[6 * i + k] = e->rv[3 * i + k]; S->u[6 * i + 3 + k] = e->rw[3 * i + k]; }
  }
  for (int pi = 0; pi < e->np; ++pi)
    for (int k = 0; k < 3; ++k) S->u[particle_dof(e, pi) + k] = e->pv[3 * pi + k];
  update_positions(S);
}

/* ---- per-iteration record (test support, not part of the method) ---- */
static void rec_put(env_t *e, int f, const double *v, int n) {
  e->rec[f] = realloc(e->rec[f], (size_t)(n > 0 ? n : 1) * sizeof(double));
  if (n > 0) {
    if (v) memcpy(e->rec[f], v, (size_t)n * sizeof(double));
    else memset(e->rec[f], 0, (size_t)n * sizeof(double));
  }
  e->rec_len[f] = n;
}
static void rec_put_int(env_t *e, int f, const int *v, int n) {
  rec_put(e, f, NULL, n);
  for (int i = 0; i < n; ++i) e->rec[f][i] = v[i];
}

/* orc_eval_iterate: the given iterate in place of the start iterate.  The previous
 * iterate, when given, is assembled first: its Jacobians and velocities are the
 * secant's J^{k-1} and u^{k-1}. */
static void inject_iterate(step_t *S) {
  env_t *e = S->e;
  const size_t nrow = (size_t)S->nrows, nd = (size_t)S->ndof;
  if (e->inj_lam_p) {
    if (nrow) memcpy(S->lam, e->inj_lam_p, nrow * sizeof(double));
    if (nd) memcpy(S->u, e->inj_u_p, nd * sizeof(double));
    if (e->nr) { memcpy(e->rx, e->inj_rx_p, 3 * e->nr * sizeof(double)); memcpy(e->rq, e->inj_rq_p, 4 * e->nr * sizeof(double)); }
    if (e->np) memcpy(e->px, e->inj_px_p, 3 * e->np * sizeof(double));
    assemble(S);
    memcpy(S->Jprev, S->J, nrow * sizeof(jrow));
    if (nd) memcpy(S->uprev, e->inj_u_p, nd * sizeof(double));
    S->have_prev = 1;
  }
  if (nrow) memcpy(S->lam, e->inj_lam, nrow * sizeof(double));
  if (nd) memcpy(S->u, e->inj_u, nd * sizeof(double));
  if (e->nr) { memcpy(e->rx, e->inj_rx, 3 * e->nr * sizeof(double)); memcpy(e->rq, e->inj_rq, 4 * e->nr * sizeof(double)); }
  if (e->np) memcpy(e->px, e->inj_px, 3 * e->np * sizeof(double));
}

int orc_step(void *envp, const orc_params *p, double h, int N, int M, double tol, orc_stats *st) {
  env_t *e = (env_t *)envp;
  memset(st, 0, sizeof *st);
  if (!(h > 0) || N < 0 || M < 0) return -1;
  step_t S;
  memset(&S, 0, sizeof S);
  S.e = e; S.p = p; S.h = h;
  S.ndof = e->ndof;
  S.t_plus = e->time + h;
  int nd = S.ndof > 0 ? S.ndof : 1;
  S.x0 = calloc(3 * e->nr + 1, sizeof(double)); S.q0 = calloc(4 * e->nr + 1, sizeof(double));
  S.px0 = calloc(3 * e->np + 1, sizeof(double));
  S.Iw = calloc(9 * e->nr + 1, sizeof(double)); S.Iwinv = calloc(9 * e->nr + 1, sizeof(double));
  S.ut = calloc(nd, sizeof(double)); S.u = calloc(nd, sizeof(double)); S.uprev = calloc(nd, sizeof(double));
  S.Hdiag = calloc(3 * e->np + 1, sizeof(double));
  S.theta_minus = calloc(e->nj + 1, sizeof(double));
  memcpy(S.x0, e->rx, 3 * e->nr * sizeof(double));
  memcpy(S.q0, e->rq, 4 * e->nr * sizeof(double));
  memcpy(S.px0, e->px, 3 * e->np * sizeof(double));

  /* Sec. 5 (implicit time stepping) and Sec. 9: mass at q^-; u~ = u^- + h M~^-1 f,
   * READING f = (m g, -omega x I omega) for rigid bodies, m g for particles. */
  for (int i = 0; i < e->nr; ++i) {
    double R[9];
    quat_to_mat(e->rq + 4 * i, R);
    const double *Ib = e->rI + 3 * i;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s1 = 0, s2 = 0;
        for (int k = 0; k < 3; ++k) {
          s1 += R[3 * a + k] * Ib[k] * R[3 * b + k];
          s2 += is_static_rigid(e, i) ? 0.0 : R[3 * a + k] / Ib[k] * R[3 * b + k];
        }
        S.Iw[9 * i + 3 * a + b] = s1;
        S.Iwinv[9 * i + 3 * a + b] = s2;
      }
    if (is_static_rigid(e, i)) continue;
    double *ut = S.ut + 6 * i;
    const double *w = e->rw + 3 * i;
    double Iw_w[3], gyro[3], dw[3];
    m3_vec(S.Iw + 9 * i, w, Iw_w);
    v3_cross(w, Iw_w, gyro);
    gyro[0] = -gyro[0]; gyro[1] = -gyro[1]; gyro[2] = -gyro[2];
    m3_vec(S.Iwinv + 9 * i, gyro, dw);
    for (int k = 0; k < 3; ++k) {
      ut[k] = e->rv[3 * i + k] + h * e->grav[k];
      ut[3 + k] = w[k] + h * dw[k];
    }
  }
  for (int pi = 0; pi < e->np; ++pi)
    for (int k = 0; k < 3; ++k) {
      S.ut[particle_dof(e, pi) + k] = e->pv[3 * pi + k] + h * e->grav[k];
      S.Hdiag[3 * pi + k] = e->pm[pi];
    }
  for (int j = 0; j < e->nj; ++j) S.theta_minus[j] = joint_has_drive(e, j) ? joint_coordinate(e, j) : 0.0;

  /* collision detection once per step (Alg. 1) */
  generate_contacts(&S);
  if (e->inj && e->nc != e->inj_nc) {  /* orc_eval_iterate: not the caller's contact set */
    free(S.x0); free(S.q0); free(S.px0); free(S.Iw); free(S.Iwinv); free(S.ut); free(S.u); free(S.uprev);
    free(S.Hdiag); free(S.theta_minus);
    return -2;
  }
  if (e->rec_k >= 0)
    for (int f = 0; f < ORC_REC_NFIELDS; ++f) e->rec_len[f] = 0;
  st->n_contacts = e->nc;
  st->overflow = e->overflow;
  S.nrows = 6 * e->nj + 3 * e->nc + e->tet_rows * e->nt;
  int nr_alloc = S.nrows > 0 ? S.nrows : 1;
  S.lam = calloc(nr_alloc, sizeof(double));
  S.J = calloc(nr_alloc, sizeof(jrow)); S.Jprev = calloc(nr_alloc, sizeof(jrow));
  S.err = calloc(nr_alloc, sizeof(double));
  S.Cblk = calloc(9 * nr_alloc, sizeof(double));
  S.blk_start = calloc(nr_alloc, sizeof(int)); S.blk_size = calloc(nr_alloc, sizeof(int));
  S.row_kind = calloc(nr_alloc, sizeof(int));
  const int nc_alloc = e->nc > 0 ? e->nc : 1;
  S.c_alpha = calloc(nc_alloc, sizeof(double)); S.c_rn = calloc(nc_alloc, sizeof(double));
  S.c_rf = calloc(nc_alloc, sizeof(double)); S.c_act = calloc(nc_alloc, sizeof(int));
  double *g = calloc(nd, sizeof(double)), *f = calloc(nd, sizeof(double)), *fhat = calloc(nd, sizeof(double));
  double *tmp = calloc(nd, sizeof(double)), *tmp2 = calloc(nd, sizeof(double));
  double *b = calloc(nr_alloc, sizeof(double)), *P = calloc(nr_alloc, sizeof(double));
  double *x = calloc(nr_alloc, sizeof(double)), *du = calloc(nd, sizeof(double));
  int *row_isl = calloc(nr_alloc, sizeof(int));
  int *body_isl = calloc(e->nr + e->np + 1, sizeof(int));
  double *isl_r = calloc(e->nr + e->np + 1, sizeof(double));  /* residual of every island */
  if (p->islands) row_islands(e, row_isl, body_isl);

  int newton_done = 0, cr_total = 0;
  double r_ncp = 0, r_con = 0, merit = 0;
  /* the step's best iterate (lowest merit) for the watchdog */
  double *best_lam = calloc(nr_alloc, sizeof(double)), *best_u = calloc(nd, sizeof(double));
  double *best_rx = calloc(3 * e->nr + 1, sizeof(double)), *best_rq = calloc(4 * e->nr + 1, sizeof(double));
  double *best_px = calloc(3 * e->np + 1, sizeof(double));
  /* line search: the accepted iterate k and its direction */
  double *lam_k = calloc(nr_alloc, sizeof(double)), *rq_k = calloc(4 * e->nr + 1, sizeof(double));
  orc_params pzero = *p;
  pzero.warm = 0;
  /* READING (recovery, not in the paper): a warm-started step whose iterate turns
   * non-finite is rerun from the paper's plain start u0 = 0, lambda0 = 0 at q^-;
   * the work of both attempts is counted. */
  for (int attempt = 0; attempt < 2; ++attempt) {
  if (attempt == 1) {
    S.p = &pzero;
    memcpy(e->rx, S.x0, 3 * e->nr * sizeof(double));
    memcpy(e->rq, S.q0, 4 * e->nr * sizeof(double));
    memcpy(e->px, S.px0, 3 * e->np * sizeof(double));
    for (int pi = 0; pi < e->np; ++pi)
      for (int k = 0; k < 3; ++k) S.Hdiag[3 * pi + k] = e->pm[pi];
    S.have_prev = 0;
    st->nonfinite = 0;
    st->fallback = 1;
  }
  start_iterate(&S);
  if (e->inj && attempt == 0) inject_iterate(&S);
  e->nhist = 0;
  /* READING (Sec. 8.1 names watchdog strategies without using one): the step keeps
   * its lowest-merit iterate; when the merit grows past WATCH_BLOWUP times that best,
   * or turns non-finite outside a warm attempt, the iteration stops and the step
   * returns the best iterate.  Ordinary non-monotone steps are far below that. */
  double best_merit = INFINITY, best_r = 0, best_rc = 0;
  int have_best = 0, restore = 0;
  /* Sec. 8.1 (optional globalisation, READING of the details): with line search on,
   * the full Newton step (t = 1) is tried first; while the merit at the trial point
   * exceeds (1 - LS_SIGMA t) times the accepted iterate's, t is halved down to LS_TMIN
   * (then accepted).  Trial points are assembled and evaluated like iterates but do
   * not count as Newton iterations. */
  double ls_t = 1.0, merit_k = INFINITY;
  for (int k = 0; k <= N; ++k) {
    const int rec = k == e->rec_k;  /* test support: record this iteration */
    if (rec) {
      rec_put(e, ORC_REC_LAM, S.lam, S.nrows);
      rec_put(e, ORC_REC_U, S.u, S.ndof);
      rec_put(e, ORC_REC_UPREV, S.have_prev ? S.uprev : NULL, S.ndof);
      rec_put(e, ORC_REC_RX, e->rx, 3 * e->nr);
      rec_put(e, ORC_REC_RQ, e->rq, 4 * e->nr);
      rec_put(e, ORC_REC_PX, e->px, 3 * e->np);
    }
    assemble(&S);
    /* momentum balance g = M~(u - u~) - h J^T lambda (Sec. 6.1) */
    memset(f, 0, nd * sizeof(double));
    for (int r = 0; r < S.nrows; ++r) jrow_scatter(&S.J[r], S.lam[r], f);
    for (int i = 0; i < S.ndof; ++i) tmp[i] = S.u[i] - S.ut[i];
    apply_M(&S, tmp, g);
    for (int i = 0; i < S.ndof; ++i) g[i] -= h * f[i];
    /* Sec. 8.3 geometric stiffness, READING: secant of J^T lambda at fixed lambda^k
     * between the last two iterates, particle DOFs only; H~_jj = M~_jj - min(0, c_j). */
    for (int pi = 0; pi < e->np; ++pi)
      for (int a = 0; a < 3; ++a) S.Hdiag[3 * pi + a] = e->pm[pi];
    memset(fhat, 0, nd * sizeof(double));
    if (p->geo_stiff && S.have_prev) {
      for (int r = 0; r < S.nrows; ++r) jrow_scatter(&S.Jprev[r], S.lam[r], fhat);
      for (int pi = 0; pi < e->np; ++pi)
        for (int a = 0; a < 3; ++a) {
          int dd = particle_dof(e, pi) + a;
          double dU = S.u[dd] - S.uprev[dd];
          double cj = h * (f[dd] - fhat[dd]) * dU / (dU * dU + TAU_GS * TAU_GS);
          S.Hdiag[3 * pi + a] = e->pm[pi] - (cj < 0 ? cj : 0.0);
        }
    }
    if (rec) {
      rec_put(e, ORC_REC_ERR, S.err, S.nrows);
      rec_put(e, ORC_REC_CDIAG, NULL, S.nrows);
      for (int r = 0; r < S.nrows; ++r) {
        int b0 = S.blk_start[r], ri = r - b0;
        e->rec[ORC_REC_CDIAG][r] = S.Cblk[9 * b0 + 3 * ri + ri];
      }
      rec_put(e, ORC_REC_CBLK, S.Cblk, 9 * S.nrows);
      rec_put(e, ORC_REC_ALPHA, S.c_alpha, e->nc);
      rec_put(e, ORC_REC_RN, S.c_rn, e->nc);
      rec_put(e, ORC_REC_RF, S.c_rf, e->nc);
      rec_put_int(e, ORC_REC_ACTIVE, S.c_act, e->nc);
      rec_put(e, ORC_REC_G, g, S.ndof);
      rec_put(e, ORC_REC_F, f, S.ndof);
      rec_put(e, ORC_REC_FHAT, fhat, S.ndof);
      rec_put(e, ORC_REC_HDIAG, S.Hdiag, 3 * e->np);
    }
    /* READING of "residual": r_ncp = max(|M~^-1 g|_inf, |err|_inf), merit |[g; err]|_2 */
    apply_Minv(&S, g, tmp);
    double rg = 0, re = 0, rc = 0, m2 = 0;
    for (int i = 0; i < S.ndof; ++i) { double a = fabs(tmp[i]); if (a > rg) rg = a; m2 += g[i] * g[i]; }
    for (int r = 0; r < S.nrows; ++r) {
      double a = fabs(S.err[r]);
      if (a > re) re = a;
      if (S.row_kind[r] == 1 || S.row_kind[r] == 2) { if (a > rc) rc = a; }
      m2 += S.err[r] * S.err[r];
    }
    r_ncp = rg > re ? rg : re;
    r_con = rc;
    merit = sqrt(m2);
    if (k == 0) st->r_ncp_first = r_ncp;
    if (p->islands) {
      /* the same residual per island (its bodies' DOFs and its rows) */
      for (int i = 0; i <= e->nr + e->np; ++i) isl_r[i] = 0.0;
      for (int i = 0; i < S.ndof; ++i) {
        int b = i < 6 * e->nr ? i / 6 : e->nr + (i - 6 * e->nr) / 3;
        if (body_isl[b] >= 0 && fabs(tmp[i]) > isl_r[body_isl[b]]) isl_r[body_isl[b]] = fabs(tmp[i]);
      }
      for (int r = 0; r < S.nrows; ++r)
        if (fabs(S.err[r]) > isl_r[row_isl[r]]) isl_r[row_isl[r]] = fabs(S.err[r]);
    }
    if (rec) {
      double rs[4] = {r_ncp, r_con, merit, 0.0};
      rec_put(e, ORC_REC_RESID, rs, 4);
    }
    int finite_now = r_ncp == r_ncp && !isinf(r_ncp) && merit == merit && !isinf(merit);
    if (p->line_search && k > 0 && ls_t > LS_TMIN && (!finite_now || merit > (1.0 - LS_SIGMA * ls_t) * merit_k)) {
      ls_t *= 0.5;
      for (int r = 0; r < S.nrows; ++r) S.lam[r] = lam_k[r] + ls_t * x[r];
      for (int i = 0; i < S.ndof; ++i) S.u[i] = S.uprev[i] + ls_t * du[i];
      memcpy(e->rq, rq_k, 4 * e->nr * sizeof(double));
      update_positions(&S);
      --k;
      continue;
    }
    if (e->nhist < MAX_HIST) { e->mhist[e->nhist] = merit; e->hist[e->nhist++] = r_ncp; }
    if (S.p->watchdog && finite_now && merit < best_merit) {
      best_merit = merit; best_r = r_ncp; best_rc = r_con; have_best = 1;
      memcpy(best_lam, S.lam, S.nrows * sizeof(double));
      memcpy(best_u, S.u, S.ndof * sizeof(double));
      memcpy(best_rx, e->rx, 3 * e->nr * sizeof(double));
      memcpy(best_rq, e->rq, 4 * e->nr * sizeof(double));
      memcpy(best_px, e->px, 3 * e->np * sizeof(double));
    }
    if (!finite_now) {
      if (!S.p->watchdog || S.p->warm != 0 || !have_best) { st->nonfinite = 1; break; }
      restore = 1;
      break;
    }
    if (S.p->watchdog && merit > WATCH_BLOWUP * best_merit) { restore = 1; break; }
    if (k == N || r_ncp <= tol) break;
    /* Schur right-hand side and Jacobi preconditioner (Sec. 6.2, 8.2, 8.4) */
    apply_Hinv(&S, g, tmp);
    for (int r = 0; r < S.nrows; ++r) {
      b[r] = (jrow_dot(&S.J[r], tmp) - S.err[r]) / h;
      int b0 = S.blk_start[r], ri = r - b0;
      P[r] = 1.0 / (row_hdiag(&S, &S.J[r]) + S.Cblk[9 * b0 + 3 * ri + ri] + p->eps);
    }
    schur_ctx sc = {&S, tmp, tmp2};
    if (rec) {
      rec_put(e, ORC_REC_B, b, S.nrows);
      rec_put(e, ORC_REC_P, P, S.nrows);
      /* one product A z with z = P b (the first product of the PCR) */
      double *z = calloc(nr_alloc, sizeof(double)), *az = calloc(nr_alloc, sizeof(double));
      for (int r = 0; r < S.nrows; ++r) z[r] = P[r] * b[r];
      schur_apply(&sc, z, az);
      rec_put(e, ORC_REC_AZ, az, S.nrows);
      free(z); free(az);
    }
    int done = 0;
    if (p->islands && p->linear == 0) {
      /* READING of Sec. 11's island remedy: one PCR per island.  A is block diagonal
       * over islands, so the PCR of the right-hand side restricted to an island stays
       * in that island's rows; the solution is the sum of the island solutions.
       * READING of the stop: an island's rounding level is that of the env's whole
       * system, so each island stops once its <z, A z> falls to TAU_CR of the env's
       * start <P b, A P b> (= the sum of the islands' starts), the stop of the
       * whole-env PCR.  Relative to its own start, an ill-conditioned small island in
       * FP32 never reaches that level and iterates on rounding with its own scalars.
       * READING of the early exit: in residual mode (tol > 0) an island whose own
       * residual is at or below tol is solved already: it skips its PCR and keeps its
       * multipliers and velocities (Delta lambda = 0, Delta u = 0); the env's iteration
       * still ends when every island is. */
      for (int r = 0; r < S.nrows; ++r) x[r] = 0.0;
      double *bi = calloc(nr_alloc, sizeof(double)), *xi = calloc(nr_alloc, sizeof(double));
      double rho_env = 0.0;
      for (int r = 0; r < S.nrows; ++r) bi[r] = P[r] * b[r];
      schur_apply(&sc, bi, xi);
      for (int r = 0; r < S.nrows; ++r) rho_env += bi[r] * xi[r];
      for (int r0 = 0; r0 < S.nrows; ++r0) {
        int isl = row_isl[r0], first = 1;
        for (int r = 0; r < r0; ++r) if (row_isl[r] == isl) { first = 0; break; }
        if (!first) continue;
        if (tol > 0.0 && isl_r[isl] <= tol) continue;
        for (int r = 0; r < S.nrows; ++r) bi[r] = row_isl[r] == isl ? b[r] : 0.0;
        int di = pcr_solve_ref(S.nrows, schur_apply, &sc, bi, P, M, xi, NULL, rho_env);
        if (di > done) done = di;
        for (int r = 0; r < S.nrows; ++r) if (row_isl[r] == isl) x[r] = xi[r];
      }
      free(bi); free(xi);
    } else {
      done = p->linear == 1 ? pcg_solve(S.nrows, schur_apply, &sc, b, P, M, x, NULL)
                            : pcr_solve(S.nrows, schur_apply, &sc, b, P, M, x, NULL);
    }
    cr_total += done;
    if (rec) {
      rec_put(e, ORC_REC_DLAM, x, S.nrows);
      if (e->rec_len[ORC_REC_RESID] == 4) e->rec[ORC_REC_RESID][3] = done;
    }
    /* du = H~^-1 (h J^T dlambda - g); damped update (Sec. 6.2, 8.1) */
    memset(f, 0, nd * sizeof(double));
    for (int r = 0; r < S.nrows; ++r) jrow_scatter(&S.J[r], x[r], f);
    for (int i = 0; i < S.ndof; ++i) tmp2[i] = h * f[i] - g[i];
    apply_Hinv(&S, tmp2, du);
    if (p->islands && p->linear == 0 && tol > 0.0)  /* a solved island keeps its velocities */
      for (int i = 0; i < S.ndof; ++i) {
        int bb = i < 6 * e->nr ? i / 6 : e->nr + (i - 6 * e->nr) / 3;
        if (body_isl[bb] >= 0 && isl_r[body_isl[bb]] <= tol) du[i] = 0.0;
      }
    memcpy(S.uprev, S.u, S.ndof * sizeof(double));
    memcpy(S.Jprev, S.J, S.nrows * sizeof(jrow));
    S.have_prev = 1;
    const double tstep = p->line_search ? 1.0 : p->damping;
    if (p->line_search) {
      memcpy(lam_k, S.lam, S.nrows * sizeof(double));
      memcpy(rq_k, e->rq, 4 * e->nr * sizeof(double));
      merit_k = merit;
      ls_t = 1.0;
    }
    for (int r = 0; r < S.nrows; ++r) S.lam[r] += tstep * x[r];
    for (int i = 0; i < S.ndof; ++i) S.u[i] += tstep * du[i];
    update_positions(&S);
    ++newton_done;
  }
  if (restore) {
    memcpy(S.lam, best_lam, S.nrows * sizeof(double));
    memcpy(S.u, best_u, S.ndof * sizeof(double));
    memcpy(e->rx, best_rx, 3 * e->nr * sizeof(double));
    memcpy(e->rq, best_rq, 4 * e->nr * sizeof(double));
    memcpy(e->px, best_px, 3 * e->np * sizeof(double));
    r_ncp = best_r; r_con = best_rc; merit = best_merit;
    st->watchdog = 1;
  }
  if (!st->nonfinite || S.p->warm == 0) break;
  }
  free(best_lam); free(best_u); free(best_rx); free(best_rq); free(best_px);
  free(lam_k); free(rq_k);
  S.p = p;
  st->newton_iters = newton_done;
  st->cr_iters = cr_total;
  st->r_ncp = r_ncp;
  st->r_contact = r_con;
  st->merit = merit;
  /* debug copy of the final assembly */
  e->dbg_rows = S.nrows;
  for (int r = 0; r < S.nrows; ++r) {
    int b0 = S.blk_start[r], ri = r - b0;
    e->dbg_err[r] = S.err[r];
    e->dbg_cdiag[r] = S.Cblk[9 * b0 + 3 * ri + ri];
    e->dbg_pdiag[r] = row_hdiag(&S, &S.J[r]);
    e->lam_last[r] = S.lam[r];
  }
  e->nrows_last = S.nrows;
  /* velocities u+ and bookkeeping for warm starts */
  for (int i = 0; i < e->nr; ++i) {
    if (is_static_rigid(e, i)) continue;
    for (int k = 0; k < 3; ++k) { e->rv[3 * i + k] = S.u[6 * i + k]; e->rw[3 * i + k] = S.u[6 * i + 3 + k]; }
  }
  for (int pi = 0; pi < e->np; ++pi)
    for (int k = 0; k < 3; ++k) e->pv[3 * pi + k] = S.u[particle_dof(e, pi) + k];
  for (int ci = 0; ci < e->nc; ++ci) {
    int r0 = row_contact(e, ci);
    for (int k = 0; k < 3; ++k) e->con[ci].lam[k] = S.lam[r0 + k];
  }
  memcpy(e->prev, e->con, e->nc * sizeof(contact));
  e->nprev = e->nc;
  for (int j = 0; j < e->nj; ++j)
    for (int r = 0; r < 6; ++r) e->lam_joint_prev[6 * j + r] = S.lam[row_joint(e, j) + r];
  for (int t = 0; t < e->nt; ++t)
    for (int r = 0; r < e->tet_rows; ++r) e->lam_tet_prev[e->tet_rows * t + r] = S.lam[row_tet(e, t) + r];
  e->have_prev = 1;
  e->time = S.t_plus;
  for (int i = 0; i < e->nr && !st->nonfinite; ++i)
    for (int k = 0; k < 3; ++k) if (!isfinite(e->rx[3 * i + k])) st->nonfinite = 1;
  for (int pi = 0; pi < e->np && !st->nonfinite; ++pi)
    for (int k = 0; k < 3; ++k) if (!isfinite(e->px[3 * pi + k])) st->nonfinite = 1;

  free(S.x0); free(S.q0); free(S.px0); free(S.Iw); free(S.Iwinv); free(S.ut); free(S.u); free(S.uprev);
  free(S.Hdiag); free(S.theta_minus); free(S.lam); free(S.J); free(S.Jprev); free(S.err); free(S.Cblk);
  free(S.blk_start); free(S.blk_size); free(S.row_kind);
  free(S.c_alpha); free(S.c_rn); free(S.c_rf); free(S.c_act);
  free(g); free(f); free(fhat); free(tmp); free(tmp2); free(b); free(P); free(x); free(du); free(row_isl); free(body_isl); free(isl_r);
  return st->nonfinite ? -4 : 0;
}

/* ------------------------------------------------------------------------- */
/* state access                                                               */
/* ------------------------------------------------------------------------- */
void orc_get_state(void *p, double *rx, double *rq, double *rv, double *rw, double *px, double *pv) {
  env_t *e = (env_t *)p;
  if (rx) memcpy(rx, e->rx, 3 * e->nr * sizeof(double));
  if (rq) memcpy(rq, e->rq, 4 * e->nr * sizeof(double));
  if (rv) memcpy(rv, e->rv, 3 * e->nr * sizeof(double));
  if (rw) memcpy(rw, e->rw, 3 * e->nr * sizeof(double));
  if (px) memcpy(px, e->px, 3 * e->np * sizeof(double));
  if (pv) memcpy(pv, e->pv, 3 * e->np * sizeof(double));
}

void orc_set_state(void *p, const double *rx, const double *rq, const double *rv, const double *rw,
                   const double *px, const double *pv) {
  env_t *e = (env_t *)p;
  if (rx) memcpy(e->rx, rx, 3 * e->nr * sizeof(double));
  if (rq) memcpy(e->rq, rq, 4 * e->nr * sizeof(double));
  if (rv) memcpy(e->rv, rv, 3 * e->nr * sizeof(double));
  if (rw) memcpy(e->rw, rw, 3 * e->nr * sizeof(double));
  if (px) memcpy(e->px, px, 3 * e->np * sizeof(double));
  if (pv) memcpy(e->pv, pv, 3 * e->np * sizeof(double));
  for (int i = 0; i < e->nr; ++i) normalize_quat(e->rq + 4 * i);
  for (int i = 0; i < e->nr; ++i)
    if (is_static_rigid(e, i))
      for (int k = 0; k < 3; ++k) { e->rv[3 * i + k] = 0; e->rw[3 * i + k] = 0; }
}

double orc_get_time(void *p) { return ((env_t *)p)->time; }
void orc_set_time(void *p, double t) { ((env_t *)p)->time = t; }
int orc_num_contacts(void *p) { return ((env_t *)p)->nc; }
int orc_num_rows(void *p) { return ((env_t *)p)->nrows_last; }

int orc_get_contacts(void *p, int64_t *key, int32_t *bodies, double *geom, double *lam, int cap) {
  env_t *e = (env_t *)p;
  int n = e->nc < cap ? e->nc : cap;
  for (int i = 0; i < n; ++i) {
    const contact *c = &e->con[i];
    key[i] = c->key;
    bodies[2 * i] = c->fa; bodies[2 * i + 1] = c->tb;
    for (int k = 0; k < 3; ++k) { geom[10 * i + k] = c->n[k]; geom[10 * i + 3 + k] = c->aL[k]; geom[10 * i + 6 + k] = c->bL[k]; }
    geom[10 * i + 9] = c->d;
    for (int k = 0; k < 3; ++k) lam[3 * i + k] = c->lam[k];
  }
  return n;
}

void orc_get_lambda(void *p, double *lam) {
  env_t *e = (env_t *)p;
  memcpy(lam, e->lam_last, e->nrows_last * sizeof(double));
}

/* Loads the previous-step multipliers (what a warm start reads): contacts by key,
 * keys ascending, lam3 = (lambda_n, lambda_f1, lambda_f2) each, and the joint rows
 * (6 per joint).  Lets a test start the oracle from another solver's previous step. */
int orc_set_prev(void *p, int n, const int64_t *keys, const double *lam3, const double *lam_joint) {
  env_t *e = (env_t *)p;
  if (n < 0 || n > e->maxc) return -1;
  for (int i = 1; i < n; ++i) if (keys[i] <= keys[i - 1]) return -1;
  memset(e->prev, 0, (size_t)(e->maxc > 0 ? e->maxc : 0) * sizeof(contact));
  for (int i = 0; i < n; ++i) {
    e->prev[i].key = keys[i];
    for (int k = 0; k < 3; ++k) e->prev[i].lam[k] = lam3[3 * i + k];
  }
  e->nprev = n;
  for (int j = 0; j < 6 * e->nj; ++j) e->lam_joint_prev[j] = lam_joint ? lam_joint[j] : 0.0;
  e->have_prev = 1;
  return 0;
}

int orc_get_history(void *p, double *r, int cap) {
  env_t *e = (env_t *)p;
  int n = e->nhist < cap ? e->nhist : cap;
  memcpy(r, e->hist, n * sizeof(double));
  return n;
}

int orc_get_merit_history(void *p, double *m, int cap) {
  env_t *e = (env_t *)p;
  int n = e->nhist < cap ? e->nhist : cap;
  memcpy(m, e->mhist, n * sizeof(double));
  return n;
}

void orc_set_record(void *p, int k) {
  env_t *e = (env_t *)p;
  e->rec_k = k;
  for (int f = 0; f < ORC_REC_NFIELDS; ++f) e->rec_len[f] = 0;
}

int orc_get_record(void *p, int field, double *out, int cap) {
  env_t *e = (env_t *)p;
  if (field < 0 || field >= ORC_REC_NFIELDS) return -1;
  int n = e->rec_len[field];
  if (out && n > 0) memcpy(out, e->rec[field], (size_t)(n < cap ? n : cap) * sizeof(double));
  return n;
}

static double *dup_d(const double *a, int n) {
  double *b = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (n > 0) memcpy(b, a, (size_t)n * sizeof(double));
  return b;
}

int orc_eval_iterate(void *p, const orc_params *prm, double h, int M, int n_contacts, const double *lam,
                     const double *u, const double *rx, const double *rq, const double *px, const double *lam_p,
                     const double *u_p, const double *rx_p, const double *rq_p, const double *px_p) {
  env_t *e = (env_t *)p;
  if (!lam || !u || (e->nr && (!rx || !rq)) || (e->np && !px) || n_contacts < 0) return -1;
  if (lam_p && (!u_p || (e->nr && (!rx_p || !rq_p)) || (e->np && !px_p))) return -1;
  /* the state and previous-step bookkeeping the step would change */
  double *rx0 = dup_d(e->rx, 3 * e->nr), *rq0 = dup_d(e->rq, 4 * e->nr), *rv0 = dup_d(e->rv, 3 * e->nr);
  double *rw0 = dup_d(e->rw, 3 * e->nr), *px0 = dup_d(e->px, 3 * e->np), *pv0 = dup_d(e->pv, 3 * e->np);
  double *lj0 = dup_d(e->lam_joint_prev, 6 * e->nj), *lt0 = dup_d(e->lam_tet_prev, e->tet_rows * e->nt);
  contact *prev0 = malloc((size_t)(e->maxc > 0 ? e->maxc : 1) * sizeof(contact));
  memcpy(prev0, e->prev, (size_t)e->nprev * sizeof(contact));
  const int nprev0 = e->nprev, have_prev0 = e->have_prev, rec_k0 = e->rec_k;
  const double time0 = e->time;
  e->inj = 1; e->inj_nc = n_contacts;
  e->inj_lam = lam; e->inj_u = u; e->inj_rx = rx; e->inj_rq = rq; e->inj_px = px;
  e->inj_lam_p = lam_p; e->inj_u_p = u_p; e->inj_rx_p = rx_p; e->inj_rq_p = rq_p; e->inj_px_p = px_p;
  e->rec_k = 0;
  orc_params q = *prm;
  q.warm = 0;          /* the injected iterate replaces any start iterate */
  q.line_search = 0;
  orc_stats st;
  int rc = orc_step(e, &q, h, 1, M, 0.0, &st);
  e->inj = 0;
  e->rec_k = rec_k0;
  memcpy(e->rx, rx0, 3 * e->nr * sizeof(double)); memcpy(e->rq, rq0, 4 * e->nr * sizeof(double));
  memcpy(e->rv, rv0, 3 * e->nr * sizeof(double)); memcpy(e->rw, rw0, 3 * e->nr * sizeof(double));
  memcpy(e->px, px0, 3 * e->np * sizeof(double)); memcpy(e->pv, pv0, 3 * e->np * sizeof(double));
  memcpy(e->lam_joint_prev, lj0, 6 * e->nj * sizeof(double));
  memcpy(e->lam_tet_prev, lt0, (size_t)e->tet_rows * e->nt * sizeof(double));
  memcpy(e->prev, prev0, (size_t)nprev0 * sizeof(contact));
  e->nprev = nprev0; e->have_prev = have_prev0; e->time = time0;
  free(rx0); free(rq0); free(rv0); free(rw0); free(px0); free(pv0); free(lj0); free(lt0); free(prev0);
  return rc;
}

int orc_get_rows_debug(void *p, double *err, double *cdiag, double *pdiag, int cap) {
  env_t *e = (env_t *)p;
  int n = e->dbg_rows < cap ? e->dbg_rows : cap;
  memcpy(err, e->dbg_err, n * sizeof(double));
  memcpy(cdiag, e->dbg_cdiag, n * sizeof(double));
  memcpy(pdiag, e->dbg_pdiag, n * sizeof(double));
  return n;
}

/* ------------------------------------------------------------------------- */
/* Learned warm start: FP64 MLP 12 -> 64 -> 64 -> 64 -> 3 with ReLU           */
/* Parameter layout: W1[64x12] b1[64] W2[64x64] b2[64] W3[64x64] b3[64]       */
/* W4[3x64] b4[3]; weights blob for the warm start appends x_mean[12]         */
/* x_std[12] y_mean[3] y_std[3].                                              */
/* ------------------------------------------------------------------------- */
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT)
int64_t orc_mlp_num_params(void) { return MLP_NPARAM; }

static void dense_layer(const double *W, const double *bvec, int nout, int nin, const double *x, double *y, int relu) {
  for (int o = 0; o < nout; ++o) {
    double acc = bvec[o];
    for (int i = 0; i < nin; ++i) acc += W[o * nin + i] * x[i];
    y[o] = relu && acc < 0 ? 0.0 : acc;
  }
}

void orc_mlp_forward(const double *w, int64_t n, const double *x, double *y) {
  const double *W1 = w, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
  const double *W3 = b2 + MLP_H, *b3 = W3 + MLP_H * MLP_H, *W4 = b3 + MLP_H, *b4 = W4 + MLP_OUT * MLP_H;
  for (int64_t s = 0; s < n; ++s) {
    double h1[MLP_H], h2[MLP_H], h3[MLP_H];
    dense_layer(W1, b1, MLP_H, MLP_IN, x + MLP_IN * s, h1, 1);
    dense_layer(W2, b2, MLP_H, MLP_H, h1, h2, 1);
    dense_layer(W3, b3, MLP_H, MLP_H, h2, h3, 1);
    dense_layer(W4, b4, MLP_OUT, MLP_H, h3, y + MLP_OUT * s, 0);
  }
}

/* Mean squared error over n samples and outputs, loss = sum (y - t)^2 / (n * 3),
 * and its gradient w.r.t. every parameter (plain backpropagation). */
double orc_mlp_loss_grad(const double *w, int64_t n, const double *x, const double *t, double *grad) {
  const double *W1 = w, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
  const double *W3 = b2 + MLP_H, *b3 = W3 + MLP_H * MLP_H, *W4 = b3 + MLP_H, *b4 = W4 + MLP_OUT * MLP_H;
  double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H;
  double *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_H * MLP_H, *gW4 = gb3 + MLP_H, *gb4 = gW4 + MLP_OUT * MLP_H;
  memset(grad, 0, MLP_NPARAM * sizeof(double));
  double loss = 0;
  double scale = 1.0 / ((double)n * MLP_OUT);
  for (int64_t s = 0; s < n; ++s) {
    const double *xs = x + MLP_IN * s;
    double h1[MLP_H], h2[MLP_H], h3[MLP_H], y[MLP_OUT];
    dense_layer(W1, b1, MLP_H, MLP_IN, xs, h1, 1);
    dense_layer(W2, b2, MLP_H, MLP_H, h1, h2, 1);
    dense_layer(W3, b3, MLP_H, MLP_H, h2, h3, 1);
    dense_layer(W4, b4, MLP_OUT, MLP_H, h3, y, 0);
    double dy[MLP_OUT], d3[MLP_H], d2[MLP_H], d1[MLP_H];
    for (int o = 0; o < MLP_OUT; ++o) {
      double e = y[o] - t[MLP_OUT * s + o];
      loss += e * e * scale;
      dy[o] = 2.0 * e * scale;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
      gb4[o] += dy[o];
      for (int i = 0; i < MLP_H; ++i) gW4[o * MLP_H + i] += dy[o] * h3[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0;
      for (int o = 0; o < MLP_OUT; ++o) acc += W4[o * MLP_H + i] * dy[o];
      d3[i] = h3[i] > 0 ? acc : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
      gb3[o] += d3[o];
      for (int i = 0; i < MLP_H; ++i) gW3[o * MLP_H + i] += d3[o] * h2[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0;
      for (int o = 0; o < MLP_H; ++o) acc += W3[o * MLP_H + i] * d3[o];
      d2[i] = h2[i] > 0 ? acc : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
      gb2[o] += d2[o];
      for (int i = 0; i < MLP_H; ++i) gW2[o * MLP_H + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0;
      for (int o = 0; o < MLP_H; ++o) acc += W2[o * MLP_H + i] * d2[o];
      d1[i] = h1[i] > 0 ? acc : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
      gb1[o] += d1[o];
      for (int i = 0; i < MLP_IN; ++i) gW1[o * MLP_IN + i] += d1[o] * xs[i];
    }
  }
  return loss;
}

/* bfloat16 rounding of a value held in float32 (round to nearest, ties to even on the
 * 16 dropped mantissa bits): the operand format of the network's products on the GPU. */
static double bf16_round(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, sizeof u);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  memcpy(&f, &u, sizeof f);
  return (double)f;
}

static void dense_layer_rounded(const double *W, const double *bvec, int nout, int nin, const double *x_r,
                                double *pre) {
  for (int o = 0; o < nout; ++o) {
    double acc = bvec[o];
    for (int i = 0; i < nin; ++i) acc += bf16_round(W[o * nin + i]) * x_r[i];
    pre[o] = acc;
  }
}

/* The same loss and gradient with the rounding the BF16 matrix units apply: every
 * operand of a product (weights, inputs, activations, back-propagated errors) is
 * rounded to bfloat16 where it enters the product; biases, ReLU masks, the loss and
 * all sums stay in double.  Backpropagation in the order of the plain version:
 * dy = 2 (y - t) / (3 n); for each layer, weight gradient = sum over samples of
 * bf16(delta) bf16(input), bias gradient = sum of delta, and the next delta =
 * mask (W^T bf16(delta)) with W rounded. */
double orc_mlp_loss_grad_bf16(const double *w, int64_t n, const double *x, const double *t, double *grad) {
  const double *W1 = w, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
  const double *W3 = b2 + MLP_H, *b3 = W3 + MLP_H * MLP_H, *W4 = b3 + MLP_H, *b4 = W4 + MLP_OUT * MLP_H;
  double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H, *gb2 = gW2 + MLP_H * MLP_H;
  double *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_H * MLP_H, *gW4 = gb3 + MLP_H, *gb4 = gW4 + MLP_OUT * MLP_H;
  memset(grad, 0, MLP_NPARAM * sizeof(double));
  double loss = 0;
  const double scale = 1.0 / ((double)n * MLP_OUT);
  for (int64_t s = 0; s < n; ++s) {
    double xr[MLP_IN], p1[MLP_H], p2[MLP_H], p3[MLP_H], h1r[MLP_H], h2r[MLP_H], h3r[MLP_H], y[MLP_OUT];
    for (int i = 0; i < MLP_IN; ++i) xr[i] = bf16_round(x[MLP_IN * s + i]);
    dense_layer_rounded(W1, b1, MLP_H, MLP_IN, xr, p1);
    for (int i = 0; i < MLP_H; ++i) h1r[i] = bf16_round(p1[i] > 0 ? p1[i] : 0.0);
    dense_layer_rounded(W2, b2, MLP_H, MLP_H, h1r, p2);
    for (int i = 0; i < MLP_H; ++i) h2r[i] = bf16_round(p2[i] > 0 ? p2[i] : 0.0);
    dense_layer_rounded(W3, b3, MLP_H, MLP_H, h2r, p3);
    for (int i = 0; i < MLP_H; ++i) h3r[i] = bf16_round(p3[i] > 0 ? p3[i] : 0.0);
    dense_layer_rounded(W4, b4, MLP_OUT, MLP_H, h3r, y);
    double dy[MLP_OUT], dyr[MLP_OUT], d3[MLP_H], d2[MLP_H], d1[MLP_H], dr[MLP_H];
    for (int o = 0; o < MLP_OUT; ++o) {
      const double e = y[o] - t[MLP_OUT * s + o];
      loss += e * e * scale;
      dy[o] = 2.0 * e * scale;
      dyr[o] = bf16_round(dy[o]);
    }
    for (int o = 0; o < MLP_OUT; ++o) {
      gb4[o] += dy[o];
      for (int i = 0; i < MLP_H; ++i) gW4[o * MLP_H + i] += dyr[o] * h3r[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0;
      for (int o = 0; o < MLP_OUT; ++o) acc += bf16_round(W4[o * MLP_H + i]) * dyr[o];
      d3[i] = p3[i] > 0 ? acc : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) dr[o] = bf16_round(d3[o]);
    for (int o = 0; o < MLP_H; ++o) {
      gb3[o] += d3[o];
      for (int i = 0; i < MLP_H; ++i) gW3[o * MLP_H + i] += dr[o] * h2r[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0;
      for (int o = 0; o < MLP_H; ++o) acc += bf16_round(W3[o * MLP_H + i]) * dr[o];
      d2[i] = p2[i] > 0 ? acc : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) dr[o] = bf16_round(d2[o]);
    for (int o = 0; o < MLP_H; ++o) {
      gb2[o] += d2[o];
      for (int i = 0; i < MLP_H; ++i) gW2[o * MLP_H + i] += dr[o] * h1r[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
      double acc = 0;
      for (int o = 0; o < MLP_H; ++o) acc += bf16_round(W2[o * MLP_H + i]) * dr[o];
      d1[i] = p1[i] > 0 ? acc : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) dr[o] = bf16_round(d1[o]);
    for (int o = 0; o < MLP_H; ++o) {
      gb1[o] += d1[o];
      for (int i = 0; i < MLP_IN; ++i) gW1[o * MLP_IN + i] += dr[o] * xr[i];
    }
  }
  return loss;
}

/* Pre-activations of the rounded forward pass of one sample (the ReLU decisions the
 * BF16 network takes): pre[3 * 64] = layers 1, 2, 3. */
void orc_mlp_preact_bf16(const double *w, const double *x, double *pre) {
  const double *W1 = w, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
  const double *W3 = b2 + MLP_H, *b3 = W3 + MLP_H * MLP_H;
  double xr[MLP_IN], hr[MLP_H];
  for (int i = 0; i < MLP_IN; ++i) xr[i] = bf16_round(x[i]);
  dense_layer_rounded(W1, b1, MLP_H, MLP_IN, xr, pre);
  for (int i = 0; i < MLP_H; ++i) hr[i] = bf16_round(pre[i] > 0 ? pre[i] : 0.0);
  dense_layer_rounded(W2, b2, MLP_H, MLP_H, hr, pre + MLP_H);
  for (int i = 0; i < MLP_H; ++i) hr[i] = bf16_round(pre[MLP_H + i] > 0 ? pre[MLP_H + i] : 0.0);
  dense_layer_rounded(W3, b3, MLP_H, MLP_H, hr, pre + 2 * MLP_H);
}

void orc_set_mlp(void *p, const double *weights, int64_t n) {
  env_t *e = (env_t *)p;
  free(e->mlp);
  e->mlp = NULL;
  e->mlp_n = 0;
  if (!weights || n <= 0) return;
  e->mlp = malloc(n * sizeof(double));
  memcpy(e->mlp, weights, n * sizeof(double));
  e->mlp_n = n;
}

/* prediction with the standardisation stored after the parameters */
static void mlp_predict(const env_t *e, const double *feat, double *out) {
  const double *w = e->mlp;
  const double *xm = w + MLP_NPARAM, *xs = xm + MLP_IN, *ym = xs + MLP_IN, *ys = ym + MLP_OUT;
  double xin[MLP_IN], y[MLP_OUT];
  for (int i = 0; i < MLP_IN; ++i) xin[i] = (feat[i] - xm[i]) / xs[i];
  orc_mlp_forward(w, 1, xin, y);
  for (int o = 0; o < MLP_OUT; ++o) out[o] = y[o] * ys[o] + ym[o];
}

/* READING of the 12 per-contact features, all at step start in the contact basis:
 * [v_n, v_t1, v_t2] relative velocity under u~, C_n(q^-), previous-step
 * (lambda_n, lambda_t1, lambda_t2) of the same contact key (0 if new), inverse masses
 * of the two bodies (0 for static/world), mu, n_z, and a flag that is 1 when the
 * contact key existed in the previous step. */
static void contact_features(const step_t *S, const contact *c, double *f) {
  const env_t *e = S->e;
  double armA[3], armB[3], va[3], vb[3], pa[3], pb[3], d1[3], d2[3];
  body_arm(e, c->fa, c->aL, armA);
  body_point(e, c->fa, c->aL, pa);
  point_velocity(e, S->ut, c->fa, armA, va);
  if (c->tb >= 0) {
    body_arm(e, c->tb, c->bL, armB);
    body_point(e, c->tb, c->bL, pb);
    point_velocity(e, S->ut, c->tb, armB, vb);
  } else {
    pb[0] = c->bL[0]; pb[1] = c->bL[1]; pb[2] = c->bL[2];
    vb[0] = vb[1] = vb[2] = 0;
  }
  double vr[3] = {va[0] - vb[0], va[1] - vb[1], va[2] - vb[2]};
  orc_tangent_basis(c->n, d1, d2);
  f[0] = v3_dot(c->n, vr);
  f[1] = v3_dot(d1, vr);
  f[2] = v3_dot(d2, vr);
  f[3] = c->n[0] * (pa[0] - pb[0]) + c->n[1] * (pa[1] - pb[1]) + c->n[2] * (pa[2] - pb[2]) - c->d;
  int k = e->have_prev ? prev_lookup(e, c->key) : -1;
  f[4] = k >= 0 ? e->prev[k].lam[0] : 0.0;
  f[5] = k >= 0 ? e->prev[k].lam[1] : 0.0;
  f[6] = k >= 0 ? e->prev[k].lam[2] : 0.0;
  double ima = 0, imb = 0;
  if (c->fa < e->nr) ima = is_static_rigid(e, c->fa) ? 0.0 : 1.0 / e->rm[c->fa];
  else ima = 1.0 / e->pm[c->fa - e->nr];
  if (c->tb >= 0) imb = is_static_rigid(e, c->tb) ? 0.0 : 1.0 / e->rm[c->tb];
  f[7] = ima;
  f[8] = imb;
  f[9] = e->mu;
  f[10] = c->n[2];
  f[11] = k >= 0 ? 1.0 : 0.0;  /* the contact existed in the previous step */
}

int orc_contact_features(void *envp, const orc_params *p, double h, double *feat, int64_t *key, int cap) {
  /* Runs the step set-up and collision detection of the current state without
   * changing it, and returns the features of the contacts found. */
  env_t *e = (env_t *)envp;
  step_t S;
  memset(&S, 0, sizeof S);
  S.e = e; S.p = p; S.h = h; S.ndof = e->ndof;
  int nd = S.ndof > 0 ? S.ndof : 1;
  S.ut = calloc(nd, sizeof(double));
  S.Iw = calloc(9 * e->nr + 1, sizeof(double)); S.Iwinv = calloc(9 * e->nr + 1, sizeof(double));
  for (int i = 0; i < e->nr; ++i) {
    if (is_static_rigid(e, i)) continue;
    double R[9];
    quat_to_mat(e->rq + 4 * i, R);
    const double *Ib = e->rI + 3 * i;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s1 = 0, s2 = 0;
        for (int k = 0; k < 3; ++k) { s1 += R[3 * a + k] * Ib[k] * R[3 * b + k]; s2 += R[3 * a + k] / Ib[k] * R[3 * b + k]; }
        S.Iw[9 * i + 3 * a + b] = s1; S.Iwinv[9 * i + 3 * a + b] = s2;
      }
    const double *w = e->rw + 3 * i;
    double Iw_w[3], gyro[3], dw[3];
    m3_vec(S.Iw + 9 * i, w, Iw_w);
    v3_cross(w, Iw_w, gyro);
    gyro[0] = -gyro[0]; gyro[1] = -gyro[1]; gyro[2] = -gyro[2];
    m3_vec(S.Iwinv + 9 * i, gyro, dw);
    for (int k = 0; k < 3; ++k) { S.ut[6 * i + k] = e->rv[3 * i + k] + h * e->grav[k]; S.ut[6 * i + 3 + k] = w[k] + h * dw[k]; }
  }
  for (int pi = 0; pi < e->np; ++pi)
    for (int k = 0; k < 3; ++k) S.ut[particle_dof(e, pi) + k] = e->pv[3 * pi + k] + h * e->grav[k];
  int nc_saved = e->nc;
  contact *saved = malloc((size_t)(e->maxc > 0 ? e->maxc : 1) * sizeof(contact));
  memcpy(saved, e->con, e->nc * sizeof(contact));
  generate_contacts(&S);
  int n = e->nc < cap ? e->nc : cap;
  for (int i = 0; i < n; ++i) {
    contact_features(&S, &e->con[i], feat + MLP_IN * i);
    key[i] = e->con[i].key;
  }
  int total = e->nc;
  memcpy(e->con, saved, nc_saved * sizeof(contact));
  e->nc = nc_saved;
  free(saved); free(S.ut); free(S.Iw); free(S.Iwinv);
  return total;
}
