/*
 * oracle.c -- plain FP64 CPU oracle of the edge-timing path.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it to check the GPU library; the product path
 * never links, loads or calls it, and it shares no code, header or constant
 * generator with the GPU library.
 *
 * Paper: "Becoming a Fruit Ninja" (FRUITNINJA planner).  Every routine
 * follows the passage it cites, in double precision, in the paper's order
 * and notation, with no blocking, fusion or reordering.  Build with
 * -O2 -ffp-contract=off and without -ffast-math, so that every operation is
 * rounded separately in IEEE binary64.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - the S evaluation times are t_s = T * s / (S-1), endpoints included;
 *  - the velocity taper is the braking law
 *        qdbar_i(q, v) = min(qdmax_i, sqrt(2 acc_i max(0, dist)))
 *    with dist the distance to the joint limit the motion heads for;
 *  - rho_v is taken at the three candidate peaks of each joint's quadratic
 *    velocity profile (t = 0, t = T, and the vertex when it is interior);
 *  - position limits add rho_q (exact position extrema of the cubic), and
 *    clearance adds rho_c = (r_a + r_o + margin) / |c_a - c_o|, both checked
 *    once at the searched T, like rho_v;
 *  - the search predicate of Def. 7 uses rho_tau and rho_P only; feasibility
 *    is inclusive (rho <= 1);
 *  - Alg. 1 and-s the clearance into the edge's flag after the limit checks
 *    (ok_p <- ok_p and Clear): clearance is evaluated only for an edge that
 *    passed them (rho_tau, rho_P, rho_v, rho_q <= 1); otherwise rho_c is
 *    reported as NaN (not evaluated) and never sets the collision bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OJ 8      /* max joints */
#define OSPH 64   /* max arm spheres */

/* dynamics terms of Eq. (4) that are switched on */
#define T_RIGID 1
#define T_ARMATURE 2
#define T_FRICTION 4
#define T_GRAVITY 8

/* per-edge status bits */
#define S_NONE 1     /* no slot with rho_tau, rho_P <= 1 */
#define S_VEL 2      /* rho_v > 1 at the searched T */
#define S_POS 4      /* rho_q > 1 at the searched T */
#define S_COLL 8     /* rho_c > 1 at the searched T */
#define S_BAD 128    /* non-finite input */
#define S_NOPARENT 512 /* padded parent (index -1) */
#define S_SELF 1024    /* two of the arm's own spheres closer than the margin (full recheck) */

typedef struct {
  int32_t n;       /* joints */
  int32_t terms;   /* T_* bits */
  double alpha[OJ], a[OJ], d[OJ];  /* modified DH: alpha_{i-1}, a_{i-1}, d_i */
  double m[OJ], rc[OJ][3], I[OJ][3]; /* mass, COM and diagonal inertia in frame i */
  double Im[OJ], psi1[OJ], psi2[OJ], psi3[OJ];
  double qmin[OJ], qmax[OJ], qdmax[OJ], taumax[OJ], acc[OJ];
  double wmax;
  double g[3];
  double tool[3];
  int32_t nsph;
  int32_t sph_link[OSPH]; /* 1..n */
  double sph[OSPH][4];    /* centre in link frame, radius */
} oarm;

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static void matvec(const double R[3][3], const double v[3], double o[3]) {
  for (int r = 0; r < 3; ++r) o[r] = R[r][0] * v[0] + R[r][1] * v[1] + R[r][2] * v[2];
}
static void matTvec(const double R[3][3], const double v[3], double o[3]) {
  for (int c = 0; c < 3; ++c) o[c] = R[0][c] * v[0] + R[1][c] * v[1] + R[2][c] * v[2];
}
static double dmax(double a, double b) { return a > b ? a : b; }

/* Rotation of frame i in frame i-1 for modified DH: Rx(alpha) Rz(q). */
static void dh_rot(double alpha, double q, double R[3][3]) {
  double ca = cos(alpha), sa = sin(alpha), cq = cos(q), sq = sin(q);
  R[0][0] = cq;      R[0][1] = -sq;     R[0][2] = 0.0;
  R[1][0] = sq * ca; R[1][1] = cq * ca; R[1][2] = -sa;
  R[2][0] = sq * sa; R[2][1] = cq * sa; R[2][2] = ca;
}
/* Origin of frame i in frame i-1: Rx(alpha) (a,0,0) + Rx(alpha) Rz(q) (0,0,d). */
static void dh_org(double alpha, double a, double d, double p[3]) {
  p[0] = a;
  p[1] = -sin(alpha) * d;
  p[2] = cos(alpha) * d;
}

/* ------------------------------------------------------------------ */
/* Eq. (6), Def. 5: the cubic edge                                     */
/* ------------------------------------------------------------------ */
/* sigma_T(t) = q0 + qd0 t + (3 d1/T^2 - d2/T) t^2 + (d2/T^2 - 2 d1/T^3) t^3,
 * d1 = q1 - q0 - qd0 T, d2 = qd1 - qd0; first and second derivatives too.
 * x0, x1 are states (q[n], qd[n]). */
void oracle_cubic(int n, const double* x0, const double* x1, double T, double t,
                  double* s, double* sd, double* sdd) {
  for (int i = 0; i < n; ++i) {
    double q0 = x0[i], qd0 = x0[n + i], q1 = x1[i], qd1 = x1[n + i];
    double d1 = q1 - q0 - qd0 * T;
    double d2 = qd1 - qd0;
    double c2 = 3.0 * d1 / (T * T) - d2 / T;
    double c3 = d2 / (T * T) - 2.0 * d1 / (T * T * T);
    s[i] = q0 + qd0 * t + c2 * t * t + c3 * t * t * t;
    sd[i] = qd0 + 2.0 * c2 * t + 3.0 * c3 * t * t;
    sdd[i] = 2.0 * c2 + 6.0 * c3 * t;
  }
}

/* ------------------------------------------------------------------ */
/* Eq. (5): sigmoid friction, zero at zero velocity                    */
/* ------------------------------------------------------------------ */
static double logistic(double x) {  /* 1/(1+e^-x), evaluated without overflow */
  if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
  double e = exp(x);
  return e / (1.0 + e);
}
double oracle_friction(double psi1, double psi2, double psi3, double qd) {
  return psi1 * logistic(psi2 * (qd + psi3)) - psi1 * logistic(psi2 * psi3);
}

/* ------------------------------------------------------------------ */
/* Eq. (4): tau = M(q) qdd + c(q, qd) + g(q) + I_m qdd + tau_f(qd).    */
/* The rigid-body part is recursive Newton-Euler in link frames        */
/* (outward velocities/accelerations, inward forces/moments).         */
/* ------------------------------------------------------------------ */
void oracle_rnea(const oarm* A, const double* q, const double* qd, const double* qdd,
                 double* tau) {
  int n = A->n;
  double R[OJ][3][3], P[OJ][3];
  double F[OJ][3], N[OJ][3];
  double w[3] = {0, 0, 0}, wd[3] = {0, 0, 0}, vd[3] = {0, 0, 0};
  if (A->terms & T_GRAVITY) {  /* base acceleration -g carries gravity */
    vd[0] = -A->g[0]; vd[1] = -A->g[1]; vd[2] = -A->g[2];
  }
  for (int i = 0; i < n; ++i) {
    dh_rot(A->alpha[i], q[i], R[i]);
    dh_org(A->alpha[i], A->a[i], A->d[i], P[i]);
  }
  for (int i = 0; i < n; ++i) {
    double t1[3], t2[3], t3[3], tmp[3];
    /* vd_i = R^T (wd_{i-1} x p_i + w_{i-1} x (w_{i-1} x p_i) + vd_{i-1}) */
    cross(wd, P[i], t1);
    cross(w, P[i], t2);
    cross(w, t2, t3);
    for (int r = 0; r < 3; ++r) tmp[r] = t1[r] + t3[r] + vd[r];
    double vdi[3];
    matTvec(R[i], tmp, vdi);
    /* w_i = R^T w_{i-1} + qd_i z ;  wd_i = R^T wd_{i-1} + (R^T w_{i-1}) x qd_i z + qdd_i z */
    double rw[3], rwd[3], wi[3], wdi[3], zq[3] = {0, 0, qd[i]}, c[3];
    matTvec(R[i], w, rw);
    matTvec(R[i], wd, rwd);
    cross(rw, zq, c);
    for (int r = 0; r < 3; ++r) {
      wi[r] = rw[r] + zq[r];
      wdi[r] = rwd[r] + c[r];
    }
    wdi[2] += qdd[i];
    /* COM acceleration, Newton and Euler equations */
    double a1[3], a2[3], a3[3], vc[3];
    cross(wdi, A->rc[i], a1);
    cross(wi, A->rc[i], a2);
    cross(wi, a2, a3);
    for (int r = 0; r < 3; ++r) vc[r] = a1[r] + a3[r] + vdi[r];
    double Iw[3], Iwd[3], wIw[3];
    for (int r = 0; r < 3; ++r) {
      Iw[r] = A->I[i][r] * wi[r];
      Iwd[r] = A->I[i][r] * wdi[r];
    }
    cross(wi, Iw, wIw);
    for (int r = 0; r < 3; ++r) {
      F[i][r] = A->m[i] * vc[r];
      N[i][r] = Iwd[r] + wIw[r];
      w[r] = wi[r];
      wd[r] = wdi[r];
      vd[r] = vdi[r];
    }
  }
  double f[3] = {0, 0, 0}, nn[3] = {0, 0, 0};
  for (int i = n - 1; i >= 0; --i) {
    double Rf[3] = {0, 0, 0}, Rn[3] = {0, 0, 0}, pxRf[3] = {0, 0, 0}, rxF[3];
    if (i + 1 < n) {
      matvec(R[i + 1], f, Rf);
      matvec(R[i + 1], nn, Rn);
      cross(P[i + 1], Rf, pxRf);
    }
    cross(A->rc[i], F[i], rxF);
    for (int r = 0; r < 3; ++r) {
      f[r] = Rf[r] + F[i][r];
      nn[r] = N[i][r] + Rn[r] + rxF[r] + pxRf[r];
    }
    tau[i] = (A->terms & T_RIGID) ? nn[2] : 0.0;
  }
  for (int i = 0; i < n; ++i) {
    if (A->terms & T_ARMATURE) tau[i] += A->Im[i] * qdd[i];
    if (A->terms & T_FRICTION) tau[i] += oracle_friction(A->psi1[i], A->psi2[i], A->psi3[i], qd[i]);
  }
}

/* ------------------------------------------------------------------ */
/* Forward kinematics of the collision spheres (Sec. IV-E, collision   */
/* checking): world centre of every arm sphere at configuration q.     */
/* ------------------------------------------------------------------ */
/* World rotation Rw[i] and origin pw[i] of every link frame i = 0..n
 * (frame 0: the base) at configuration q, by the modified DH chain. */
static void fk_frames(const oarm* A, const double* q, double Rw[OJ + 1][3][3], double pw[OJ + 1][3]) {
  memset(Rw[0], 0, sizeof(Rw[0]));
  Rw[0][0][0] = Rw[0][1][1] = Rw[0][2][2] = 1.0;
  pw[0][0] = pw[0][1] = pw[0][2] = 0.0;
  for (int i = 0; i < A->n; ++i) {
    double R[3][3], p[3], pr[3];
    dh_rot(A->alpha[i], q[i], R);
    dh_org(A->alpha[i], A->a[i], A->d[i], p);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Rw[i + 1][r][c] = Rw[i][r][0] * R[0][c] + Rw[i][r][1] * R[1][c] + Rw[i][r][2] * R[2][c];
    matvec(Rw[i], p, pr);
    for (int r = 0; r < 3; ++r) pw[i + 1][r] = pw[i][r] + pr[r];
  }
}

void oracle_fk_spheres(const oarm* A, const double* q, double* centres /*[nsph][3]*/) {
  double Rw[OJ + 1][3][3], pw[OJ + 1][3];
  fk_frames(A, q, Rw, pw);
  for (int k = 0; k < A->nsph; ++k) {
    int l = A->sph_link[k];
    double c[3];
    matvec(Rw[l], A->sph[k], c);
    for (int r = 0; r < 3; ++r) centres[3 * k + r] = pw[l][r] + c[r];
  }
}

/* World position of a point given in the frame of link `link` (1..n), for
 * n configurations q [n][stride] (the blade point p_n of Eq. (8)). */
void oracle_fk_point(const oarm* A, int n, const double* q, int stride, int link,
                     const double* local, double* out /*[n][3]*/) {
  for (int i = 0; i < n; ++i) {
    double Rw[OJ + 1][3][3], pw[OJ + 1][3], c[3];
    fk_frames(A, q + (size_t)i * stride, Rw, pw);
    matvec(Rw[link], local, c);
    for (int r = 0; r < 3; ++r) out[3 * i + r] = pw[link][r] + c[r];
  }
}

/* ------------------------------------------------------------------ */
/* Def. 6, Eq. (7): torque and power ratios of one edge at one T       */
/* ------------------------------------------------------------------ */
/* Evaluates the cubic at S equally spaced times t_s = T s/(S-1) and
 * returns rho_tau = max_{i,s} |tau_i|/taumax_i and
 * rho_P = max_s |sum_i tau_i sd_i| / W_max.  tau_out[S][n] optional. */
void oracle_slot_rho(const oarm* A, const double* x0, const double* x1, double T, int S,
                     double* rho_tau, double* rho_p, double* tau_out) {
  int n = A->n;
  double rt = 0.0, rp = 0.0;
  for (int s = 0; s < S; ++s) {
    double u = (S > 1) ? (double)s / (double)(S - 1) : 0.0;
    double t = u * T;
    double sg[OJ], sd[OJ], sdd[OJ], tau[OJ];
    oracle_cubic(n, x0, x1, T, t, sg, sd, sdd);
    oracle_rnea(A, sg, sd, sdd, tau);
    double pw = 0.0;
    for (int i = 0; i < n; ++i) {
      rt = dmax(rt, fabs(tau[i]) / A->taumax[i]);
      pw += tau[i] * sd[i];
      if (tau_out) tau_out[(size_t)s * n + i] = tau[i];
    }
    rp = dmax(rp, fabs(pw) / A->wmax);
  }
  *rho_tau = rt;
  *rho_p = rp;
}

/* ------------------------------------------------------------------ */
/* Post-checks at the searched T (Sec. IV-D after Def. 7; Sec. IV-E).  */
/* ------------------------------------------------------------------ */
/* Velocity taper of Def. 1 (braking-law reading). */
static double taper(const oarm* A, int i, double q, double v) {
  double dist = (v >= 0.0) ? (A->qmax[i] - q) : (q - A->qmin[i]);
  double b = sqrt(2.0 * A->acc[i] * dmax(0.0, dist));
  return b < A->qdmax[i] ? b : A->qdmax[i];
}
static double vel_ratio(const oarm* A, int i, double q, double v) {
  if (v == 0.0) return 0.0;
  double lim = taper(A, i, q, v);
  if (lim <= 0.0) return INFINITY;
  return fabs(v) / lim;
}
/* cubic coefficients in t for joint i */
static void coeffs(int n, const double* x0, const double* x1, double T, int i,
                   double* c0, double* c1, double* c2, double* c3) {
  double q0 = x0[i], qd0 = x0[n + i], q1 = x1[i], qd1 = x1[n + i];
  double d1 = q1 - q0 - qd0 * T, d2 = qd1 - qd0;
  *c0 = q0;
  *c1 = qd0;
  *c2 = 3.0 * d1 / (T * T) - d2 / T;
  *c3 = d2 / (T * T) - 2.0 * d1 / (T * T * T);
}
/* rho_v: exact peaks of the quadratic velocity profile, ratio to the taper
 * at the position reached at that instant. */
double oracle_rho_v(const oarm* A, const double* x0, const double* x1, double T) {
  int n = A->n;
  double r = 0.0;
  for (int i = 0; i < n; ++i) {
    double c0, c1, c2, c3;
    coeffs(n, x0, x1, T, i, &c0, &c1, &c2, &c3);
    double ts[3];
    int nt = 0;
    ts[nt++] = 0.0;
    ts[nt++] = T;
    if (c3 != 0.0) {
      double tv = -c2 / (3.0 * c3);
      if (tv > 0.0 && tv < T) ts[nt++] = tv;
    }
    for (int k = 0; k < nt; ++k) {
      double t = ts[k];
      double q = c0 + c1 * t + c2 * t * t + c3 * t * t * t;
      double v = c1 + 2.0 * c2 * t + 3.0 * c3 * t * t;
      r = dmax(r, vel_ratio(A, i, q, v));
    }
  }
  return r;
}
/* rho_q: exact position extrema over [0, T] (endpoints and the real roots of
 * the velocity in (0, T), stable quadratic formula), relative to the joint
 * range: |sigma - centre| / half-range. */
double oracle_rho_q(const oarm* A, const double* x0, const double* x1, double T) {
  int n = A->n;
  double r = 0.0;
  for (int i = 0; i < n; ++i) {
    double c0, c1, c2, c3;
    coeffs(n, x0, x1, T, i, &c0, &c1, &c2, &c3);
    double ts[4];
    int nt = 0;
    ts[nt++] = 0.0;
    ts[nt++] = T;
    double qa = 3.0 * c3, qb = 2.0 * c2, qc = c1;  /* velocity qa t^2 + qb t + qc */
    if (qa == 0.0) {
      if (qb != 0.0) ts[nt++] = -qc / qb;
    } else {
      double disc = qb * qb - 4.0 * qa * qc;
      if (disc >= 0.0) {
        double sq = sqrt(disc);
        double qq = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
        if (qq != 0.0) {
          ts[nt++] = qq / qa;
          ts[nt++] = qc / qq;
        } else {
          ts[nt++] = 0.0;  /* qb = qc = 0: double root at 0 */
        }
      }
    }
    double cen = 0.5 * (A->qmax[i] + A->qmin[i]);
    double half = 0.5 * (A->qmax[i] - A->qmin[i]);
    for (int k = 0; k < nt; ++k) {
      double t = ts[k];
      if (!(t >= 0.0 && t <= T)) continue;
      double q = c0 + c1 * t + c2 * t * t + c3 * t * t * t;
      r = dmax(r, fabs(q - cen) / half);
    }
  }
  return r;
}
/* The world an edge is checked against (Sec. IV-E, collision checking):
 * obstacle spheres [n_sph][4] = (centre, radius) and obstacle capsules
 * [n_cap][7] = (segment end p0, segment end p1, radius), both with the
 * clearance margin `margin`; and the arm's self-collision sphere pairs
 * [n_pairs][2] (indices into the arm's spheres, the pairs that survive the
 * offline pruning) with margin `margin_self`, checked by the fixed-duration
 * check (the full-resolution recheck of the plan sent to the controller). */
typedef struct {
  const double* sph;
  int32_t n_sph;
  const double* cap;
  int32_t n_cap;
  double margin;
  const int32_t* pairs;
  int32_t n_pairs;
  double margin_self;
} oworld;

/* Distance from point c to the segment p0 p1: the closest point is
 * p0 + t (p1 - p0) with t the projection clamped to [0, 1]. */
double oracle_point_segment(const double* c, const double* p0, const double* p1) {
  double d[3], w[3];
  for (int r = 0; r < 3; ++r) {
    d[r] = p1[r] - p0[r];
    w[r] = c[r] - p0[r];
  }
  double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double t = dd > 0.0 ? (w[0] * d[0] + w[1] * d[1] + w[2] * d[2]) / dd : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double e[3];
  for (int r = 0; r < 3; ++r) e[r] = w[r] - t * d[r];
  return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
}

/* rho_c: clearance of every arm sphere against every obstacle sphere and
 * capsule at the S evaluation times, as (r_a + r_o + margin) / distance
 * (distance to the capsule's segment). */
double oracle_rho_c(const oarm* A, const double* x0, const double* x1, double T, int S,
                    const oworld* W) {
  int n = A->n;
  double r = 0.0;
  if (W->n_sph + W->n_cap <= 0) return 0.0;
  double cen[OSPH * 3];
  for (int s = 0; s < S; ++s) {
    double u = (S > 1) ? (double)s / (double)(S - 1) : 0.0;
    double t = u * T;
    double sg[OJ], sd[OJ], sdd[OJ];
    oracle_cubic(n, x0, x1, T, t, sg, sd, sdd);
    oracle_fk_spheres(A, sg, cen);
    for (int k = 0; k < A->nsph; ++k) {
      for (int o = 0; o < W->n_sph; ++o) {
        const double* ob = W->sph + 4 * o;
        double dx = cen[3 * k] - ob[0], dy = cen[3 * k + 1] - ob[1], dz = cen[3 * k + 2] - ob[2];
        double dist = sqrt(dx * dx + dy * dy + dz * dz);
        double need = A->sph[k][3] + ob[3] + W->margin;
        r = dmax(r, dist > 0.0 ? need / dist : INFINITY);
      }
      for (int o = 0; o < W->n_cap; ++o) {
        const double* cp = W->cap + 7 * o;
        double dist = oracle_point_segment(cen + 3 * k, cp, cp + 3);
        double need = A->sph[k][3] + cp[6] + W->margin;
        r = dmax(r, dist > 0.0 ? need / dist : INFINITY);
      }
    }
  }
  return r;
}

/* rho_self: clearance of the arm's self-collision pairs at the S
 * evaluation times, (r_a + r_b + margin_self) / |c_a - c_b|. */
double oracle_rho_self(const oarm* A, const double* x0, const double* x1, double T, int S,
                       const oworld* W) {
  int n = A->n;
  double r = 0.0;
  if (W->n_pairs <= 0) return 0.0;
  double cen[OSPH * 3];
  for (int s = 0; s < S; ++s) {
    double u = (S > 1) ? (double)s / (double)(S - 1) : 0.0;
    double t = u * T;
    double sg[OJ], sd[OJ], sdd[OJ];
    oracle_cubic(n, x0, x1, T, t, sg, sd, sdd);
    oracle_fk_spheres(A, sg, cen);
    for (int p = 0; p < W->n_pairs; ++p) {
      int a = W->pairs[2 * p], b = W->pairs[2 * p + 1];
      double dx = cen[3 * a] - cen[3 * b], dy = cen[3 * a + 1] - cen[3 * b + 1],
             dz = cen[3 * a + 2] - cen[3 * b + 2];
      double dist = sqrt(dx * dx + dy * dy + dz * dz);
      double need = A->sph[a][3] + A->sph[b][3] + W->margin_self;
      r = dmax(r, dist > 0.0 ? need / dist : INFINITY);
    }
  }
  return r;
}

static int finite_state(int n, const double* x) {
  for (int i = 0; i < 2 * n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

/* ------------------------------------------------------------------ */
/* Def. 7 on the T grid + post-checks: one edge                        */
/* ------------------------------------------------------------------ */
/* Search the grid slots 0..jmax for the first slot with rho_tau <= 1 and
 * rho_P <= 1 (Def. 7; "one iteration of an N-ary search" over all slots,
 * Sec. IV-E).  scan = 0 evaluates every slot (dense definition), scan = 1
 * stops at the first feasible slot (same result: it is the first).
 * Outputs: j* (or -1), status bits, margin = the smallest |rho - 1| over the
 * slots up to j* (all slots when none) and the post-check ratios at j*,
 * rho4 = (rho_tauP(j*), rho_v, rho_q, rho_c), nslots = slots evaluated;
 * rho_c is NaN when rho_v or rho_q already fails (not evaluated). */
static void edge_one(const oarm* A, const double* x0, const double* x1, int NT,
                     const double* grid, int S, int jmax, const oworld* W, int scan, int16_t* out_j, uint16_t* out_st,
                     double* out_m, double* rho4, int* nslots) {
  int n = A->n;
  rho4[0] = rho4[1] = rho4[2] = rho4[3] = 0.0;
  *nslots = 0;
  if (!finite_state(n, x0) || !finite_state(n, x1)) {
    *out_j = -1;
    *out_st = S_BAD;
    *out_m = 0.0;
    return;
  }
  if (jmax > NT - 1) jmax = NT - 1;
  int jstar = -1;
  double m = INFINITY, last = 0.0;
  for (int j = 0; j <= jmax; ++j) {
    double rt, rp;
    oracle_slot_rho(A, x0, x1, grid[j], S, &rt, &rp, NULL);
    double rho = dmax(rt, rp);
    (*nslots)++;
    if (jstar < 0) {
      m = fmin(m, fabs(rho - 1.0));
      last = rho;
      if (rho <= 1.0) {
        jstar = j;
        rho4[0] = rho;
        if (scan) break;
      }
    }
  }
  uint16_t st = 0;
  if (jstar < 0) {
    st |= S_NONE;
    rho4[0] = last;
  } else {
    double T = grid[jstar];
    double rv = oracle_rho_v(A, x0, x1, T);
    double rq = oracle_rho_q(A, x0, x1, T);
    /* Clear is and-ed after the limit checks (Alg. 1): evaluated only when
     * they pass; fmin below ignores the NaN of an unevaluated clearance */
    double rc = (rv <= 1.0 && rq <= 1.0) ? oracle_rho_c(A, x0, x1, T, S, W) : NAN;
    rho4[1] = rv;
    rho4[2] = rq;
    rho4[3] = rc;
    if (rv > 1.0) st |= S_VEL;
    if (rq > 1.0) st |= S_POS;
    if (rc > 1.0) st |= S_COLL;
    m = fmin(m, fabs(rv - 1.0));
    m = fmin(m, fabs(rq - 1.0));
    m = fmin(m, fabs(rc - 1.0));
  }
  *out_j = (int16_t)jstar;
  *out_st = st;
  *out_m = m;
}

/* Batched edge timing: edges e = (parent state x0[e], candidate x1[e]).
 * parent_ok[e] == 0 marks a padded parent (no edge).  jmax may be NULL. */
void oracle_edge_time(const oarm* A, int E, const double* x0, const double* x1,
                      const int32_t* parent_ok, int NT, const double* grid, int S,
                      const int16_t* jmax, const oworld* W, int scan, int16_t* out_j, uint16_t* out_st, double* out_m,
                      double* out_rho, int32_t* out_nslots) {
  int w = 2 * A->n;
  for (int e = 0; e < E; ++e) {
    double rho4[4];
    int ns = 0;
    if (parent_ok && !parent_ok[e]) {
      out_j[e] = -1;
      out_st[e] = S_NOPARENT;
      out_m[e] = INFINITY;
      rho4[0] = rho4[1] = rho4[2] = rho4[3] = 0.0;
    } else {
      int jm = jmax ? jmax[e] : NT - 1;
      edge_one(A, x0 + (size_t)e * w, x1 + (size_t)e * w, NT, grid, S, jm, W, scan, &out_j[e],
               &out_st[e], &out_m[e], rho4, &ns);
    }
    if (out_rho)
      for (int r = 0; r < 4; ++r) out_rho[(size_t)e * 4 + r] = rho4[r];
    if (out_nslots) out_nslots[e] = ns;
  }
}

/* Dense table of (rho_tau, rho_P) for every edge and every grid slot. */
void oracle_edge_dense(const oarm* A, int E, const double* x0, const double* x1, int NT,
                       const double* grid, int S, double* rho /*[E][NT][2]*/) {
  int w = 2 * A->n;
  for (int e = 0; e < E; ++e)
    for (int j = 0; j < NT; ++j)
      oracle_slot_rho(A, x0 + (size_t)e * w, x1 + (size_t)e * w, grid[j], S,
                      &rho[((size_t)e * NT + j) * 2], &rho[((size_t)e * NT + j) * 2 + 1], NULL);
}

/* The paper's multi-round N-ary search over the slot index range (Sec.
 * IV-D after Def. 7): each round evaluates N evenly spaced slots of the
 * current range and keeps the sub-range ending at the first feasible one.
 * It assumes feasibility is monotone in T; on such edges it returns the
 * dense result.  Returns j (or -1) per edge. */
void oracle_edge_nary(const oarm* A, int E, const double* x0, const double* x1, int NT,
                      const double* grid, int S, int N, int16_t* out_j) {
  int w = 2 * A->n;
  for (int e = 0; e < E; ++e) {
    const double* a = x0 + (size_t)e * w;
    const double* b = x1 + (size_t)e * w;
    int lo = 0, hi = NT - 1, found = -1;
    /* is the top of the range feasible at all? */
    double rt, rp;
    oracle_slot_rho(A, a, b, grid[hi], S, &rt, &rp, NULL);
    if (dmax(rt, rp) > 1.0) {
      out_j[e] = -1;
      continue;
    }
    found = hi;
    while (hi - lo > 0) {
      int span = hi - lo;
      int npts = N < span ? N : span;
      int prev = lo - 1, first = hi;
      for (int k = 0; k < npts; ++k) {
        int j = lo + (int)(((long)span * k) / npts);
        oracle_slot_rho(A, a, b, grid[j], S, &rt, &rp, NULL);
        if (dmax(rt, rp) <= 1.0) {
          first = j;
          break;
        }
        prev = j;
      }
      found = first;
      hi = first;
      lo = prev + 1;
      if (hi == lo) break;
    }
    out_j[e] = (int16_t)found;
  }
}

/* Multi-round N-ary refinement of the minimum feasible time below the grid
 * (Sec. IV-D after Def. 7: the interval [T_lo, T_hi] is cut into N equal
 * slots, their ends are evaluated, and the slot whose end is the first
 * feasible one is cut again, until it is no wider than eps).  It starts from
 * the grid search's result j (the first feasible slot): T_hi = grid[j] is
 * feasible, T_lo = grid[j-1] is not (T_lo = 0 for j = 0).  A round
 * evaluates t_i = T_lo + i (T_hi - T_lo)/N for i = 1 .. N-1 in ascending
 * order; the first feasible t_i becomes T_hi and t_{i-1} becomes T_lo; when
 * none is feasible, T_lo = t_{N-1}.  The result is T_hi, a feasible duration
 * within eps of the boundary below it.  Velocity taper, position limits and
 * clearance are then checked at that duration as in the grid search
 * (clearance only when the limits pass).  Edges with j < 0 are not refined
 * (T = NaN, status S_NONE).  out_lo: the final T_lo; out_rounds: rounds run;
 * rho4 = (rho_tauP(T), rho_v, rho_q, rho_c). */
void oracle_edge_refine(const oarm* A, int E, const double* x0, const double* x1,
                        const int16_t* j_in, int NT, const double* grid, int S, int N,
                        double eps, const oworld* W,
                        double* out_T, double* out_lo, uint16_t* out_st, double* out_rho,
                        int32_t* out_rounds) {
  int w = 2 * A->n;
  for (int e = 0; e < E; ++e) {
    const double* a = x0 + (size_t)e * w;
    const double* b = x1 + (size_t)e * w;
    double* r4 = out_rho + (size_t)e * 4;
    int j = j_in[e];
    r4[0] = r4[1] = r4[2] = r4[3] = 0.0;
    out_rounds[e] = 0;
    if (j < 0 || j >= NT || !finite_state(A->n, a) || !finite_state(A->n, b)) {
      out_T[e] = NAN;
      out_lo[e] = NAN;
      out_st[e] = (j < 0 || j >= NT) ? S_NONE : S_BAD;
      continue;
    }
    double hi = grid[j];
    double lo = j > 0 ? grid[j - 1] : 0.0;
    int rounds = 0;
    while (hi - lo > eps) {
      double wd = (hi - lo) / (double)N;
      int first = N;
      for (int i = 1; i < N; ++i) {
        double rt, rp;
        oracle_slot_rho(A, a, b, lo + (double)i * wd, S, &rt, &rp, NULL);
        if (dmax(rt, rp) <= 1.0) {
          first = i;
          break;
        }
      }
      double nlo = lo + (double)(first - 1) * wd;
      double nhi = first < N ? lo + (double)first * wd : hi;
      lo = nlo;
      hi = nhi;
      rounds++;
    }
    double rt, rp;
    oracle_slot_rho(A, a, b, hi, S, &rt, &rp, NULL);
    double rv = oracle_rho_v(A, a, b, hi);
    double rq = oracle_rho_q(A, a, b, hi);
    double rc = (rv <= 1.0 && rq <= 1.0) ? oracle_rho_c(A, a, b, hi, S, W) : NAN;
    uint16_t st = 0;
    if (rv > 1.0) st |= S_VEL;
    if (rq > 1.0) st |= S_POS;
    if (rc > 1.0) st |= S_COLL;
    r4[0] = dmax(rt, rp);
    r4[1] = rv;
    r4[2] = rq;
    r4[3] = rc;
    out_T[e] = hi;
    out_lo[e] = lo;
    out_st[e] = st;
    out_rounds[e] = rounds;
  }
}

/* ------------------------------------------------------------------ */
/* The 1 kHz tracking controller (Sec. IV-F, Eq. (9))                  */
/* ------------------------------------------------------------------ */
/* Control status bits */
#define C_ACC 1      /* the desired acceleration was clipped to [l, u] */
#define C_SLEW 2     /* the torque was clipped to the slew limit */
#define C_TORQUE 4   /* the torque was clipped to the torque limit */
#define C_POWER 8    /* the torque was scaled to the power limit */
#define C_BAD 128    /* non-finite input or horizon T <= 0: zero torque */

/* One control step per instance.  The controller refits the cubic of
 * Eq. (6) from the measured state (q, qd) to the rendezvous (qg, qdg) over
 * the horizon T and takes its initial acceleration, Eq. (9):
 *   qdd_des = 6 (qg - q) / T^2 - (4 qd + 2 qdg) / T.
 * Readings: [l, u] keeps the velocity after one period dt inside the taper
 * of Def. 1 (braking law), l = (-qdbar(q, -) - qd) / dt,
 * u = (qdbar(q, +) - qd) / dt, where qdbar(q, +) = min(qdmax, sqrt(2 acc
 * (qmax - q)_+)) and qdbar(q, -) = min(qdmax, sqrt(2 acc (q - qmin)_+));
 * the torque of Eq. (4) at (q, qd, qdd) is then clipped in the order slew
 * (|tau - tau_prev| <= slew dt), torque (|tau| <= taumax), power (when
 * |sum tau qd| > W_max the torque is scaled by W_max / |sum tau qd|).
 * Outputs: tau [n][dof], the clipped acceleration qdd [n][dof], status. */
void oracle_control(const oarm* A, int n_inst, const double* q, const double* qd,
                    const double* tau_prev, const double* qg, const double* qdg, const double* T,
                    double dt, const double* slew, double* out_tau, double* out_qdd,
                    uint16_t* out_st) {
  int n = A->n;
  for (int e = 0; e < n_inst; ++e) {
    const double* qe = q + (size_t)e * n;
    const double* ve = qd + (size_t)e * n;
    const double* pe = tau_prev + (size_t)e * n;
    const double* ge = qg + (size_t)e * n;
    const double* we = qdg + (size_t)e * n;
    double* te = out_tau + (size_t)e * n;
    double* ae = out_qdd + (size_t)e * n;
    int ok = isfinite(T[e]) && T[e] > 0.0;
    for (int i = 0; i < n; ++i)
      ok = ok && isfinite(qe[i]) && isfinite(ve[i]) && isfinite(pe[i]) && isfinite(ge[i]) &&
           isfinite(we[i]);
    if (!ok) {
      for (int i = 0; i < n; ++i) te[i] = ae[i] = 0.0;
      out_st[e] = C_BAD;
      continue;
    }
    uint16_t st = 0;
    double Te = T[e];
    for (int i = 0; i < n; ++i) {
      double a = 6.0 * (ge[i] - qe[i]) / (Te * Te) - (4.0 * ve[i] + 2.0 * we[i]) / Te;
      double vp = sqrt(2.0 * A->acc[i] * dmax(0.0, A->qmax[i] - qe[i]));
      double vm = sqrt(2.0 * A->acc[i] * dmax(0.0, qe[i] - A->qmin[i]));
      if (vp > A->qdmax[i]) vp = A->qdmax[i];
      if (vm > A->qdmax[i]) vm = A->qdmax[i];
      double lo = (-vm - ve[i]) / dt, hi = (vp - ve[i]) / dt;
      if (a < lo) {
        a = lo;
        st |= C_ACC;
      } else if (a > hi) {
        a = hi;
        st |= C_ACC;
      }
      ae[i] = a;
    }
    oracle_rnea(A, qe, ve, ae, te);
    for (int i = 0; i < n; ++i) {
      double d = slew[i] * dt;
      if (te[i] > pe[i] + d) {
        te[i] = pe[i] + d;
        st |= C_SLEW;
      } else if (te[i] < pe[i] - d) {
        te[i] = pe[i] - d;
        st |= C_SLEW;
      }
      if (te[i] > A->taumax[i]) {
        te[i] = A->taumax[i];
        st |= C_TORQUE;
      } else if (te[i] < -A->taumax[i]) {
        te[i] = -A->taumax[i];
        st |= C_TORQUE;
      }
    }
    double p = 0.0;
    for (int i = 0; i < n; ++i) p += te[i] * ve[i];
    if (fabs(p) > A->wmax) {
      double s = A->wmax / fabs(p);
      for (int i = 0; i < n; ++i) te[i] *= s;
      st |= C_POWER;
    }
    out_st[e] = st;
  }
}

/* Fixed-duration check of one edge (goal candidates, Alg. 1 fixed-T branch;
 * also the full-resolution recheck of a sent plan, Sec. IV-E).
 * rho5 = (rho_tau, rho_P, rho_v, rho_q, rho_c); T <= 0 is infeasible; rho_c is
 * NaN unless rho_tau, rho_P, rho_v and rho_q all pass. */
void oracle_edge_check(const oarm* A, int E, const double* x0, const double* x1,
                       const double* T, int S, const oworld* W,
                       uint16_t* out_st, double* out_rho /*[E][5]*/, double* out_tau /*[E][S][n]*/) {
  int n = A->n, w = 2 * n;
  for (int e = 0; e < E; ++e) {
    const double* a = x0 + (size_t)e * w;
    const double* b = x1 + (size_t)e * w;
    double* r5 = out_rho + (size_t)e * 5;
    double* tau = out_tau ? out_tau + (size_t)e * S * n : NULL;
    for (int r = 0; r < 5; ++r) r5[r] = 0.0;
    if (!finite_state(n, a) || !finite_state(n, b) || !isfinite(T[e])) {
      out_st[e] = S_BAD;
      if (tau) memset(tau, 0, sizeof(double) * S * n);
      continue;
    }
    if (!(T[e] > 0.0)) {
      out_st[e] = S_NONE;
      if (tau) memset(tau, 0, sizeof(double) * S * n);
      continue;
    }
    oracle_slot_rho(A, a, b, T[e], S, &r5[0], &r5[1], tau);
    r5[2] = oracle_rho_v(A, a, b, T[e]);
    r5[3] = oracle_rho_q(A, a, b, T[e]);
    /* clearance only for an edge that passed every limit check (Alg. 1) */
    const int lim_ok = r5[0] <= 1.0 && r5[1] <= 1.0 && r5[2] <= 1.0 && r5[3] <= 1.0;
    /* the full recheck adds the arm's self-collision pairs to the obstacles */
    double rs = lim_ok ? oracle_rho_self(A, a, b, T[e], S, W) : NAN;
    r5[4] = lim_ok ? dmax(oracle_rho_c(A, a, b, T[e], S, W), rs) : NAN;
    uint16_t st = 0;
    if (r5[0] > 1.0 || r5[1] > 1.0) st |= S_NONE;
    if (r5[2] > 1.0) st |= S_VEL;
    if (r5[3] > 1.0) st |= S_POS;
    if (r5[4] > 1.0) st |= S_COLL;
    if (rs > 1.0) st |= S_SELF;
    out_st[e] = st;
  }
}

/* ------------------------------------------------------------------ */
/* Parents(T, x, M) of Alg. 1: brute-force nearest tree nodes          */
/* ------------------------------------------------------------------ */
/* d^2 = sum_{j=0..13} (x_j - y_j)^2 in order j = 0..13, each operation
 * rounded separately; ranking by (d^2, node index); the first k are kept,
 * padded with -1 / +inf when there are fewer than k nodes. */
typedef struct {
  double d2;
  int32_t idx;
} okey;
static int okey_cmp(const void* pa, const void* pb) {
  const okey* a = (const okey*)pa;
  const okey* b = (const okey*)pb;
  if (a->d2 < b->d2) return -1;
  if (a->d2 > b->d2) return 1;
  return (a->idx > b->idx) - (a->idx < b->idx);
}
void oracle_plan_knn(int N, const double* nodes /*[N][dim]*/, int B, const double* qs /*[B][dim]*/,
                     int dim, int k, int32_t* out_idx, double* out_d2) {
  okey* keys = (okey*)malloc(sizeof(okey) * (size_t)(N > 0 ? N : 1));
  for (int b = 0; b < B; ++b) {
    const double* x = qs + (size_t)b * dim;
    for (int i = 0; i < N; ++i) {
      const double* y = nodes + (size_t)i * dim;
      double d = 0.0;
      for (int j = 0; j < dim; ++j) {
        double t = x[j] - y[j];
        double sq = t * t;
        d = d + sq;
      }
      keys[i].d2 = d;
      keys[i].idx = i;
    }
    qsort(keys, (size_t)N, sizeof(okey), okey_cmp);
    for (int r = 0; r < k; ++r) {
      out_idx[(size_t)b * k + r] = r < N ? keys[r].idx : -1;
      if (out_d2) out_d2[(size_t)b * k + r] = r < N ? keys[r].d2 : INFINITY;
    }
  }
  free(keys);
}

/* ------------------------------------------------------------------ */
/* Risk objective, Eq. (2) with the terms of Eq. (3) (Sec. IV-B)       */
/* ------------------------------------------------------------------ */
typedef struct {
  double gz;                  /* vertical gravity component of Eq. (1) */
  int32_t sigma_mode;         /* 0: sigma^2 = sp^2 + (sv t)^2 + (sa t^2/2)^2; 1: s0 + s1 t */
  double sp, sv, sa, s0, s1;
  double wv, vtarget, wp, wr, wx, r, nu0, lam;
} orisk;

static double sigma_of(const orisk* R, double t) {
  if (R->sigma_mode == 1) return R->s0 + R->s1 * t;
  double a = R->sp, b = R->sv * t, c = 0.5 * R->sa * t * t;
  return sqrt(a * a + b * b + c * c);
}
/* log of the standard normal CDF; for z < -20 the asymptotic series
 * log Phi(z) = -z^2/2 - log(-z) - log(2 pi)/2 + log(1 - 1/z^2 + 3/z^4 - 15/z^6 + 105/z^8). */
double oracle_log_phi(double z) {
  if (z >= -20.0) return log(0.5 * erfc(-z / sqrt(2.0)));
  double z2 = z * z;
  double s = 1.0 - 1.0 / z2 + 3.0 / (z2 * z2) - 15.0 / (z2 * z2 * z2) + 105.0 / (z2 * z2 * z2 * z2);
  return -0.5 * z2 - log(-z) - 0.5 * log(2.0 * M_PI) + log(s);
}
static double log_erf(double x) {
  if (x < 0.5) return log(erf(x));
  return log1p(-erfc(x));
}
/* J of one rendezvous with arrival time T, relative speed v_rel, peak
 * velocity fraction nu, on a flight with vertical launch velocity vz0 that
 * leaves reach at t_fall (the vertical speed there is |vz0 + gz t_fall|). */
double oracle_risk_one(const orisk* R, double T, double v_rel, double nu, double vz0,
                       double t_fall) {
  double sg = sigma_of(R, T);
  double lpo = log_erf(R->r / (sg * sqrt(2.0)));
  double xdz = vz0 + R->gz * t_fall;
  double st = sg / fabs(xdz);
  double lpr = oracle_log_phi((t_fall - T) / st);
  double lpa = (nu > R->nu0) ? -R->lam * (nu - R->nu0) * T * (1.0 - R->nu0 / nu) : 0.0;
  double vr = v_rel < R->vtarget ? v_rel : R->vtarget;
  return R->wv * vr + R->wp * lpo + R->wr * lpr + R->wx * lpa;
}
void oracle_risk_score(const orisk* R, int n, const double* T, const double* v_rel,
                       const double* nu, const double* vz0, const double* t_fall,
                       double* out_J) {
  for (int i = 0; i < n; ++i) out_J[i] = oracle_risk_one(R, T[i], v_rel[i], nu[i], vz0[i], t_fall[i]);
}
