/*
 * FP64 CPU oracle for softened direct-summation gravity.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant with the
 * GPU path.
 *
 * Every function is the plain definition written out, in double precision,
 * summing j in ascending index order with Neumaier-compensated sums so that
 * the oracle's own rounding error stays near 1e-16 relative.  OpenMP only
 * distributes independent rows i; each row's arithmetic is sequential, so the
 * result does not depend on the thread count.
 *
 * Layout: vectors are SoA, x[c*n + i] for component c in {0,1,2}; masses m[i].
 *
 * Sources (the paper: "Assessing Performance and Porting Strategies for
 * Gravitational N-Body Simulations on the RISC-V-Based Tenstorrent Wormhole"):
 *   - acceleration: Eq. (1) of Sec. 2.1 divided by m_i, with the softening
 *     parameter of App. A read as Plummer softening |d|^2 + eps^2;
 *   - pair arithmetic order: App. A, Algorithm 3 (displacement, squared
 *     distance, inverse root, cube, weight times cube, accumulate);
 *   - integrator: kick-drift-kick leapfrog (the paper's Sec. 2.1 uses a Hermite
 *     predictor-corrector; the workloads use KDK);
 *   - diagnostics: kinetic + softened pair potential (self pair excluded),
 *     linear and angular momentum (Sec. 4.1 compares particle energies);
 *   - adjoint: the exact reverse-mode derivative of the KDK map above;
 *   - jerk: App. A, Algorithm 3 (t_j = p_w r^-3, A = -3 r^-2, v_r = r . v,
 *     q = A v_r, a += t_j r_ij, jerk += t_j (v_ij + q r_ij)), with the
 *     softened r^2 = |d|^2 + eps^2, i.e. the time derivative of the softened
 *     acceleration along the motion;
 *   - Hermite: the fourth-order predictor-evaluator-corrector with a shared
 *     time step (Sec. 2.1 describes the sixth-order member of this family:
 *     predict, evaluate acceleration and jerk, correct);
 *   - sixth-order Hermite (Sec. 2.1, after the scheme of Nitadori & Makino
 *     2008 that the paper cites): the evaluation also returns the snap, the
 *     second time derivative of the softened acceleration along paths of
 *     constant acceleration, and the predictor uses the crackle of the
 *     quintic that interpolates a, jerk and snap at both ends of the
 *     previous step (zero before the first step).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Neumaier compensated sum ----------------------------------------- */
typedef struct { double s, c; } nsum;

static inline void nadd(nsum* a, double t) {
    double s = a->s + t;
    if (fabs(a->s) >= fabs(t)) a->c += (a->s - s) + t;
    else a->c += (t - s) + a->s;
    a->s = s;
}
static inline double nval(const nsum* a) { return a->s + a->c; }

/* ---- O1: acceleration of one row i (Eq. 1 / m_i, softened) -------------- */
static void accel_row(int64_t n, const double* x, const double* m, double G, double eps,
                      int64_t i, double out[3]) {
    const double* X = x;
    const double* Y = x + n;
    const double* Z = x + 2 * n;
    const double e2 = eps * eps;
    nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;                    /* the sum in Eq. (1) skips j = i */
        double dx = X[j] - X[i];                 /* r_ij = r_j - r_i */
        double dy = Y[j] - Y[i];
        double dz = Z[j] - Z[i];
        double r2 = dx * dx + dy * dy + dz * dz + e2;
        double rinv = 1.0 / sqrt(r2);
        double rinv3 = rinv * rinv * rinv;
        double t = m[j] * rinv3;                 /* weight of j times r^-3 */
        nadd(&ax, t * dx);
        nadd(&ay, t * dy);
        nadd(&az, t * dz);
    }
    out[0] = G * nval(&ax);
    out[1] = G * nval(&ay);
    out[2] = G * nval(&az);
}

void oracle_accel(int64_t n, const double* x, const double* m, double G, double eps, double* a) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double o[3];
        accel_row(n, x, m, G, eps, i, o);
        a[i] = o[0];
        a[n + i] = o[1];
        a[2 * n + i] = o[2];
    }
}

/* Rows listed in `rows` only (each exact as in oracle_accel); out is [3][nrows]. */
void oracle_accel_rows(int64_t n, const double* x, const double* m, double G, double eps,
                       int64_t nrows, const int64_t* rows, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nrows; ++k) {
        double o[3];
        accel_row(n, x, m, G, eps, rows[k], o);
        out[k] = o[0];
        out[nrows + k] = o[1];
        out[2 * nrows + k] = o[2];
    }
}

/* Per-row scale of the terms: G * sum_{j != i} m_j / (|d|^2 + eps^2), used to
 * normalise errors of rows whose acceleration nearly cancels. */
void oracle_term_scale_rows(int64_t n, const double* x, const double* m, double G, double eps,
                            int64_t nrows, const int64_t* rows, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        nsum s = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            nadd(&s, m[j] / (dx * dx + dy * dy + dz * dz + eps * eps));
        }
        out[k] = fabs(G) * nval(&s);
    }
}

/* Per-row scales of the VJP terms, the condition of the sums of
 * oracle_accel_vjp: for each listed row k,
 *   sx[k] = G sum_{j != k} |K(d_kj) u_kj|_2   (u_kj = m_k w_j - m_j w_k),
 *   sm[k] = G sum_{j != k} |s^-3/2 (d_kj . w_j)|,
 * so that |gx_k| <= sx[k] and |gm_k| <= sm[k], with equality for one term. */
void oracle_accel_vjp_scale_rows(int64_t n, const double* x, const double* m, const double* w, double G,
                                 double eps, int64_t nrows, const int64_t* rows, double* sx, double* sm) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t k = rows[r];
        nsum ax = {0, 0}, am = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == k) continue;
            double d[3], u[3];
            for (int c = 0; c < 3; ++c) {
                d[c] = x[c * n + j] - x[c * n + k];
                u[c] = m[k] * w[c * n + j] - m[j] * w[c * n + k];
            }
            double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
            double s32 = 1.0 / (s * sqrt(s));
            double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
            double t[3];
            for (int c = 0; c < 3; ++c) t[c] = s32 * u[c] - 3.0 * (s32 / s) * du * d[c];
            nadd(&ax, sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]));
            double dw = d[0] * w[j] + d[1] * w[n + j] + d[2] * w[2 * n + j];
            nadd(&am, fabs(s32 * dw));
        }
        sx[r] = fabs(G) * nval(&ax);
        sm[r] = fabs(G) * nval(&am);
    }
}

/* ---- O2: kick-drift-kick leapfrog -------------------------------------- */
/* Advances (x, v) in place by nsteps steps of size dt.  If traj != NULL it
 * receives the positions x_0 .. x_nsteps, traj[s*3n + c*n + i]. */
void oracle_kdk(int64_t n, double* x, double* v, const double* m, double G, double eps,
                double dt, int64_t nsteps, double* traj) {
    const int64_t n3 = 3 * n;
    double* a = (double*)malloc(sizeof(double) * (size_t)(n3 > 0 ? n3 : 1));
    oracle_accel(n, x, m, G, eps, a);
    if (traj) memcpy(traj, x, sizeof(double) * (size_t)n3);
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t k = 0; k < n3; ++k) v[k] = v[k] + 0.5 * dt * a[k];   /* half kick */
        for (int64_t k = 0; k < n3; ++k) x[k] = x[k] + dt * v[k];         /* drift */
        oracle_accel(n, x, m, G, eps, a);                                  /* a(x_{s+1}) */
        for (int64_t k = 0; k < n3; ++k) v[k] = v[k] + 0.5 * dt * a[k];   /* half kick */
        if (traj) memcpy(traj + (size_t)(s + 1) * n3, x, sizeof(double) * (size_t)n3);
    }
    free(a);
}

/* ---- O3: diagnostics --------------------------------------------------- */
/* out = {K, W, E, Px, Py, Pz, Lx, Ly, Lz}.  W sums the softened pair potential
 * -G m_i m_j / sqrt(|d|^2 + eps^2) over unordered pairs i < j only. */
void oracle_energy(int64_t n, const double* x, const double* v, const double* m, double G,
                   double eps, double* out) {
    const double *X = x, *Y = x + n, *Z = x + 2 * n;
    const double *VX = v, *VY = v + n, *VZ = v + 2 * n;
    double* wrow = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum w = {0, 0};
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
            nadd(&w, m[i] * m[j] / r);
        }
        wrow[i] = nval(&w);
    }
    nsum W = {0, 0}, K = {0, 0};
    nsum P[3] = {{0, 0}, {0, 0}, {0, 0}}, L[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t i = 0; i < n; ++i) {
        nadd(&W, wrow[i]);
        nadd(&K, 0.5 * m[i] * (VX[i] * VX[i] + VY[i] * VY[i] + VZ[i] * VZ[i]));
        nadd(&P[0], m[i] * VX[i]);
        nadd(&P[1], m[i] * VY[i]);
        nadd(&P[2], m[i] * VZ[i]);
        nadd(&L[0], m[i] * (Y[i] * VZ[i] - Z[i] * VY[i]));
        nadd(&L[1], m[i] * (Z[i] * VX[i] - X[i] * VZ[i]));
        nadd(&L[2], m[i] * (X[i] * VY[i] - Y[i] * VX[i]));
    }
    free(wrow);
    out[0] = nval(&K);
    out[1] = -G * nval(&W);
    out[2] = out[0] + out[1];
    for (int c = 0; c < 3; ++c) {
        out[3 + c] = nval(&P[c]);
        out[6 + c] = nval(&L[c]);
    }
}

/* ---- O6: vector-Jacobian products of the acceleration ------------------ */
/* With d_kj = x_j - x_k, s = |d|^2 + eps^2 and K(d) = s^-3/2 I - 3 s^-5/2 d d^T:
 *   gx_k = G sum_{j != k} K(d_kj) (m_k w_j - m_j w_k)      (d a / d x)^T w
 *   gm_k = -G sum_{j != k} s^-3/2 (d_kj . w_j)              (d a / d m)^T w
 * Both follow from differentiating Eq. (1) / m_i term by term. */
/* One row k of the VJP: out4 = (gx_k, gy_k, gz_k, gm_k). */
static void vjp_row(int64_t n, const double* x, const double* m, const double* w, double G, double eps,
                    int64_t k, double* out4) {
    const double *X = x, *Y = x + n, *Z = x + 2 * n;
    const double *WX = w, *WY = w + n, *WZ = w + 2 * n;
    nsum gxs = {0, 0}, gys = {0, 0}, gzs = {0, 0}, gms = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
        if (j == k) continue;
        double d[3] = {X[j] - X[k], Y[j] - Y[k], Z[j] - Z[k]};
        double u[3] = {m[k] * WX[j] - m[j] * WX[k], m[k] * WY[j] - m[j] * WY[k],
                       m[k] * WZ[j] - m[j] * WZ[k]};
        double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
        double s32 = 1.0 / (s * sqrt(s));
        double s52 = s32 / s;
        double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
        nadd(&gxs, s32 * u[0] - 3.0 * s52 * du * d[0]);
        nadd(&gys, s32 * u[1] - 3.0 * s52 * du * d[1]);
        nadd(&gzs, s32 * u[2] - 3.0 * s52 * du * d[2]);
        double dw = d[0] * WX[j] + d[1] * WY[j] + d[2] * WZ[j];
        nadd(&gms, -s32 * dw);
    }
    out4[0] = G * nval(&gxs);
    out4[1] = G * nval(&gys);
    out4[2] = G * nval(&gzs);
    out4[3] = G * nval(&gms);
}

void oracle_accel_vjp(int64_t n, const double* x, const double* m, const double* w, double G,
                      double eps, double* gx, double* gm) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double o[4];
        vjp_row(n, x, m, w, G, eps, k, o);
        gx[k] = o[0];
        gx[n + k] = o[1];
        gx[2 * n + k] = o[2];
        gm[k] = o[3];
    }
}

/* The rows `rows` of oracle_accel_vjp only: gx (3 x nrows), gm (nrows). */
void oracle_accel_vjp_rows(int64_t n, const double* x, const double* m, const double* w, double G,
                           double eps, int64_t nrows, const int64_t* rows, double* gx, double* gm) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nrows; ++k) {
        double o[4];
        vjp_row(n, x, m, w, G, eps, rows[k], o);
        gx[k] = o[0];
        gx[nrows + k] = o[1];
        gx[2 * nrows + k] = o[2];
        gm[k] = o[3];
    }
}

/* Directional derivative of the acceleration: (da/dx) dx + (da/dm) dm, the
 * forward-mode counterpart used by the dot-product test. */
void oracle_accel_jvp(int64_t n, const double* x, const double* m, const double* tx,
                      const double* tm, double G, double eps, double* out) {
    const double *X = x, *Y = x + n, *Z = x + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum o[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {X[j] - X[i], Y[j] - Y[i], Z[j] - Z[i]};
            double dd[3] = {tx[j] - tx[i], tx[n + j] - tx[n + i], tx[2 * n + j] - tx[2 * n + i]};
            double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
            double s32 = 1.0 / (s * sqrt(s));
            double s52 = s32 / s;
            double ddot = d[0] * dd[0] + d[1] * dd[1] + d[2] * dd[2];
            for (int c = 0; c < 3; ++c)
                nadd(&o[c], m[j] * (s32 * dd[c] - 3.0 * s52 * ddot * d[c]) + tm[j] * s32 * d[c]);
        }
        for (int c = 0; c < 3; ++c) out[c * n + i] = G * nval(&o[c]);
    }
}

/* ---- O6: reverse sweep of the KDK map ---------------------------------- */
/* Given cotangents (gxT, gvT) of the final state after nsteps KDK steps from
 * (x0, v0), returns the cotangents (gx0, gv0, gm) of the initial state and the
 * masses.  The whole position trajectory is stored (no checkpointing), and the
 * two Jacobian products at each interior position are taken separately. */
void oracle_kdk_adjoint(int64_t n, const double* x0, const double* v0, const double* m, double G,
                        double eps, double dt, int64_t nsteps, const double* gxT,
                        const double* gvT, double* gx0, double* gv0, double* gm) {
    const int64_t n3 = 3 * n;
    const size_t nb = sizeof(double) * (size_t)(n3 > 0 ? n3 : 1);
    double* traj = (double*)malloc(nb * (size_t)(nsteps + 1));
    double* xw = (double*)malloc(nb);
    double* vw = (double*)malloc(nb);
    memcpy(xw, x0, sizeof(double) * (size_t)n3);
    memcpy(vw, v0, sizeof(double) * (size_t)n3);
    oracle_kdk(n, xw, vw, m, G, eps, dt, nsteps, traj);

    double* lx = (double*)malloc(nb);
    double* lv = (double*)malloc(nb);
    double* w = (double*)malloc(nb);
    double* jx = (double*)malloc(nb);
    double* jm = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    memcpy(lx, gxT, sizeof(double) * (size_t)n3);
    memcpy(lv, gvT, sizeof(double) * (size_t)n3);
    for (int64_t i = 0; i < n; ++i) gm[i] = 0.0;
    const double h = 0.5 * dt;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double* xs1 = traj + (size_t)(s + 1) * n3;
        const double* xs = traj + (size_t)s * n3;
        /* v_{s+1} = vh + h a(x_{s+1}) */
        for (int64_t k = 0; k < n3; ++k) w[k] = h * lv[k];
        oracle_accel_vjp(n, xs1, m, w, G, eps, jx, jm);
        for (int64_t k = 0; k < n3; ++k) lx[k] += jx[k];
        for (int64_t i = 0; i < n; ++i) gm[i] += jm[i];
        /* x_{s+1} = x_s + dt vh */
        for (int64_t k = 0; k < n3; ++k) lv[k] += dt * lx[k];
        /* vh = v_s + h a(x_s) */
        for (int64_t k = 0; k < n3; ++k) w[k] = h * lv[k];
        oracle_accel_vjp(n, xs, m, w, G, eps, jx, jm);
        for (int64_t k = 0; k < n3; ++k) lx[k] += jx[k];
        for (int64_t i = 0; i < n; ++i) gm[i] += jm[i];
    }
    memcpy(gx0, lx, sizeof(double) * (size_t)n3);
    memcpy(gv0, lv, sizeof(double) * (size_t)n3);
    free(traj); free(xw); free(vw); free(lx); free(lv); free(w); free(jx); free(jm);
}

/* ---- acceleration and jerk (App. A, Algorithm 3) ----------------------- */
static void accel_jerk_row(int64_t n, const double* x, const double* v, const double* m, double G,
                           double eps, int64_t i, double a[3], double jk[3]) {
    nsum sa[3] = {{0, 0}, {0, 0}, {0, 0}}, sj[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double r[3], w[3];
        for (int c = 0; c < 3; ++c) {
            r[c] = x[c * n + j] - x[c * n + i];       /* r_ij = r_j - r_i */
            w[c] = v[c * n + j] - v[c * n + i];       /* v_ij = v_j - v_i */
        }
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps * eps;
        double rinv = 1.0 / sqrt(r2);
        double rinv2 = rinv * rinv;
        double t = m[j] * rinv2 * rinv;               /* t_j = p_w,j r^-3 */
        double A = -3.0 * rinv2;                      /* A = -3 r^-2 */
        double vr = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
        double q = A * vr;                            /* q = A v_r */
        for (int c = 0; c < 3; ++c) {
            nadd(&sa[c], t * r[c]);
            nadd(&sj[c], t * (w[c] + q * r[c]));
        }
    }
    for (int c = 0; c < 3; ++c) {
        a[c] = G * nval(&sa[c]);
        jk[c] = G * nval(&sj[c]);
    }
}

void oracle_accel_jerk(int64_t n, const double* x, const double* v, const double* m, double G, double eps,
                       double* a, double* jk) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double ai[3], ji[3];
        accel_jerk_row(n, x, v, m, G, eps, i, ai, ji);
        for (int c = 0; c < 3; ++c) {
            a[c * n + i] = ai[c];
            jk[c * n + i] = ji[c];
        }
    }
}

/* The listed rows of oracle_accel_jerk (the same per-row computation), out
 * arrays of shape (3, nrows). */
void oracle_accel_jerk_rows(int64_t n, const double* x, const double* v, const double* m, double G, double eps,
                            int64_t nrows, const int64_t* rows, double* a, double* jk) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        double ai[3], ji[3];
        accel_jerk_row(n, x, v, m, G, eps, rows[r], ai, ji);
        for (int c = 0; c < 3; ++c) {
            a[c * nrows + r] = ai[c];
            jk[c * nrows + r] = ji[c];
        }
    }
}

/* Fourth-order Hermite predictor-evaluator-corrector, shared step dt:
 *   predict  xp = x + v dt + a dt^2/2 + j dt^3/6,  vp = v + a dt + j dt^2/2
 *   evaluate a1, j1 at (xp, vp)
 *   correct  v1 = v + (a0 + a1) dt/2 + (j0 - j1) dt^2/12
 *            x1 = x + (v + v1) dt/2 + (a0 - a1) dt^2/12
 * (x, v) advance in place by nsteps steps. */
void oracle_hermite4(int64_t n, double* x, double* v, const double* m, double G, double eps, double dt,
                     int64_t nsteps) {
    const int64_t n3 = 3 * n;
    const size_t nb = sizeof(double) * (size_t)(n3 > 0 ? n3 : 1);
    double *a0 = (double*)malloc(nb), *j0 = (double*)malloc(nb), *a1 = (double*)malloc(nb),
           *j1 = (double*)malloc(nb), *xp = (double*)malloc(nb), *vp = (double*)malloc(nb);
    oracle_accel_jerk(n, x, v, m, G, eps, a0, j0);
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t k = 0; k < n3; ++k) {
            xp[k] = x[k] + v[k] * dt + a0[k] * (dt * dt / 2.0) + j0[k] * (dt * dt * dt / 6.0);
            vp[k] = v[k] + a0[k] * dt + j0[k] * (dt * dt / 2.0);
        }
        oracle_accel_jerk(n, xp, vp, m, G, eps, a1, j1);
        for (int64_t k = 0; k < n3; ++k) {
            double v1 = v[k] + (a0[k] + a1[k]) * (dt / 2.0) + (j0[k] - j1[k]) * (dt * dt / 12.0);
            x[k] = x[k] + (v[k] + v1) * (dt / 2.0) + (a0[k] - a1[k]) * (dt * dt / 12.0);
            v[k] = v1;
            a0[k] = a1[k];
            j0[k] = j1[k];
        }
    }
    free(a0); free(j0); free(a1); free(j1); free(xp); free(vp);
}

/* Per-particle potential phi_i = -G sum_{j != i} m_j / (|x_j - x_i|^2 + eps^2)^(1/2)
 * (the softened pair potential of the diagnostics, per particle): the specific
 * energy of particle i is |v_i|^2 / 2 + phi_i, whose distribution Sec. 4.1
 * (Fig. 4) compares against the double-precision reference. */
void oracle_potential(int64_t n, const double* x, const double* m, double G, double eps, double* phi) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum sp = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            nadd(&sp, m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps * eps));
        }
        phi[i] = -G * nval(&sp);
    }
}

/* ---- acceleration, jerk and snap (sixth-order Hermite, Sec. 2.1) --------
 * Each particle moves on x_k(t) = x_k + v_k t + acc_k t^2 / 2.  The pair term
 * P(t) = m_j d / s^(3/2), d = x_j - x_i, s = |d|^2 + eps^2, has at t = 0, with
 * w = v_j - v_i and u = acc_j - acc_i,
 *   t_j   = m_j s^(-3/2)
 *   alpha = (d . w) / s
 *   beta  = (w . w + d . u) / s + alpha^2
 *   P     = t_j d
 *   P'    = t_j w - 3 alpha P                 (the jerk term of Algorithm 3)
 *   P''   = t_j u - 6 alpha P' - 3 beta P
 * (differentiate t_j' = -3 alpha t_j and alpha' = (w.w + d.u)/s - 2 alpha^2).
 * a, jerk and snap are G times the sums of P, P' and P'' over j != i. */
static void accel_jerk_snap_row(int64_t n, const double* x, const double* v, const double* acc,
                                const double* m, double G, double eps, int64_t i, double* a, double* jk,
                                double* sn) {
    nsum sa[3] = {{0, 0}, {0, 0}, {0, 0}}, sj[3] = {{0, 0}, {0, 0}, {0, 0}}, ss[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3], w[3], u[3];
        for (int c = 0; c < 3; ++c) {
            d[c] = x[c * n + j] - x[c * n + i];
            w[c] = v[c * n + j] - v[c * n + i];
            u[c] = acc[c * n + j] - acc[c * n + i];
        }
        double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
        double sinv = 1.0 / s2;
        double t = m[j] * sinv / sqrt(s2);
        double alpha = (d[0] * w[0] + d[1] * w[1] + d[2] * w[2]) * sinv;
        double beta = (w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + d[0] * u[0] + d[1] * u[1] + d[2] * u[2]) * sinv +
                      alpha * alpha;
        for (int c = 0; c < 3; ++c) {
            double P0 = t * d[c];
            double P1 = t * w[c] - 3.0 * alpha * P0;
            double P2 = t * u[c] - 6.0 * alpha * P1 - 3.0 * beta * P0;
            nadd(&sa[c], P0);
            nadd(&sj[c], P1);
            nadd(&ss[c], P2);
        }
    }
    for (int c = 0; c < 3; ++c) {
        a[c] = G * nval(&sa[c]);
        jk[c] = G * nval(&sj[c]);
        sn[c] = G * nval(&ss[c]);
    }
}

void oracle_accel_jerk_snap(int64_t n, const double* x, const double* v, const double* acc, const double* m,
                            double G, double eps, double* a, double* jk, double* sn) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double ai[3], ji[3], si[3];
        accel_jerk_snap_row(n, x, v, acc, m, G, eps, i, ai, ji, si);
        for (int c = 0; c < 3; ++c) {
            a[c * n + i] = ai[c];
            jk[c * n + i] = ji[c];
            sn[c * n + i] = si[c];
        }
    }
}

/* The listed rows of oracle_accel_jerk_snap, out arrays of shape (3, nrows). */
void oracle_accel_jerk_snap_rows(int64_t n, const double* x, const double* v, const double* acc, const double* m,
                                 double G, double eps, int64_t nrows, const int64_t* rows, double* a, double* jk,
                                 double* sn) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        double ai[3], ji[3], si[3];
        accel_jerk_snap_row(n, x, v, acc, m, G, eps, rows[r], ai, ji, si);
        for (int c = 0; c < 3; ++c) {
            a[c * nrows + r] = ai[c];
            jk[c * nrows + r] = ji[c];
            sn[c * nrows + r] = si[c];
        }
    }
}

/* Third derivative at the end t = h of the quintic q(t) with q(0) = a0,
 * q'(0) = j0, q''(0) = s0, q(h) = a1, q'(h) = j1, q''(h) = s1.  Writing
 * q = a0 + j0 t + s0 t^2/2 + k3 t^3 + k4 t^4 + k5 t^5 and
 *   A = (a1 - a0 - j0 h - s0 h^2/2) / h^3 = k3 + k4 h + k5 h^2
 *   B = (j1 - j0 - s0 h) / h^2             = 3 k3 + 4 k4 h + 5 k5 h^2
 *   C = (s1 - s0) / h                      = 6 k3 + 12 k4 h + 20 k5 h^2,
 * the solution k3 = 10A - 4B + C/2, k4 h = 7B - 15A - C, k5 h^2 = (C + 12A - 6B)/2
 * gives q'''(h) = 6 k3 + 24 k4 h + 60 k5 h^2 = 60 A - 36 B + 9 C. */
void oracle_hermite6_crackle(int64_t cnt, double h, const double* a0, const double* j0, const double* s0,
                             const double* a1, const double* j1, const double* s1, double* c1) {
    for (int64_t k = 0; k < cnt; ++k) {
        double A = (a1[k] - a0[k] - j0[k] * h - s0[k] * (h * h / 2.0)) / (h * h * h);
        double B = (j1[k] - j0[k] - s0[k] * h) / (h * h);
        double C = (s1[k] - s0[k]) / h;
        c1[k] = 60.0 * A - 36.0 * B + 9.0 * C;
    }
}

/* Sixth-order Hermite predictor-evaluator-corrector, shared step h = dt:
 *   predict  xp = x + v h + a h^2/2 + j h^3/6 + s h^4/24 + c h^5/120
 *            vp = v + a h + j h^2/2 + s h^3/6 + c h^4/24
 *            ap = a + j h + s h^2/2 + c h^3/6
 *   evaluate a1, j1, s1 at (xp, vp, ap)
 *   correct  v1 = v + (a + a1) h/2 - (j1 - j) h^2/10 + (s + s1) h^3/120
 *            x1 = x + (v + v1) h/2 - (a1 - a) h^2/10 + (j + j1) h^3/120
 *   crackle  c1 from oracle_hermite6_crackle
 * Start: a, j at (x, v) (Algorithm 3), then a, j, s at (x, v, a); c = 0.
 * (x, v) advance in place by nsteps steps. */
void oracle_hermite6(int64_t n, double* x, double* v, const double* m, double G, double eps, double dt,
                     int64_t nsteps) {
    const int64_t n3 = 3 * n;
    const size_t nb = sizeof(double) * (size_t)(n3 > 0 ? n3 : 1);
    double *a = (double*)malloc(nb), *j = (double*)malloc(nb), *s = (double*)malloc(nb), *c = (double*)malloc(nb);
    double *a1 = (double*)malloc(nb), *j1 = (double*)malloc(nb), *s1 = (double*)malloc(nb);
    double *xp = (double*)malloc(nb), *vp = (double*)malloc(nb), *ap = (double*)malloc(nb);
    const double h = dt;
    oracle_accel_jerk(n, x, v, m, G, eps, a1, j1);
    oracle_accel_jerk_snap(n, x, v, a1, m, G, eps, a, j, s);
    for (int64_t k = 0; k < n3; ++k) c[k] = 0.0;
    for (int64_t st = 0; st < nsteps; ++st) {
        for (int64_t k = 0; k < n3; ++k) {
            xp[k] = x[k] + v[k] * h + a[k] * (h * h / 2.0) + j[k] * (h * h * h / 6.0) +
                    s[k] * (h * h * h * h / 24.0) + c[k] * (h * h * h * h * h / 120.0);
            vp[k] = v[k] + a[k] * h + j[k] * (h * h / 2.0) + s[k] * (h * h * h / 6.0) + c[k] * (h * h * h * h / 24.0);
            ap[k] = a[k] + j[k] * h + s[k] * (h * h / 2.0) + c[k] * (h * h * h / 6.0);
        }
        oracle_accel_jerk_snap(n, xp, vp, ap, m, G, eps, a1, j1, s1);
        oracle_hermite6_crackle(n3, h, a, j, s, a1, j1, s1, c);
        for (int64_t k = 0; k < n3; ++k) {
            double v1 = v[k] + (a[k] + a1[k]) * (h / 2.0) - (j1[k] - j[k]) * (h * h / 10.0) +
                        (s[k] + s1[k]) * (h * h * h / 120.0);
            x[k] = x[k] + (v[k] + v1) * (h / 2.0) - (a1[k] - a[k]) * (h * h / 10.0) +
                   (j[k] + j1[k]) * (h * h * h / 120.0);
            v[k] = v1;
            a[k] = a1[k];
            j[k] = j1[k];
            s[k] = s1[k];
        }
    }
    free(a); free(j); free(s); free(c); free(a1); free(j1); free(s1); free(xp); free(vp); free(ap);
}

/* Mean squared distance of positions to a target: (1/N) sum_i |x_i - t_i|^2. */
double oracle_msd_loss(int64_t n, const double* x, const double* tgt) {
    nsum s = {0, 0};
    for (int64_t k = 0; k < 3 * n; ++k) {
        double d = x[k] - tgt[k];
        nadd(&s, d * d);
    }
    return n > 0 ? nval(&s) / (double)n : 0.0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the following oracle calls (timing of the single-thread baseline). */
void oracle_set_num_threads(int k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
