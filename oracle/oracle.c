/*
 * FP64 CPU oracle for the regularized 2D Biot-Savart pair sum and the
 * computations built on it (projection-tree ROM, arXiv 2103.01983).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product path: only
 * tests, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code, header or constant with the HIP library.
 *
 * Everything is plain double-precision loops in the order the paper states
 * the operation; OpenMP only distributes independent targets.  No tiling, no
 * fusion, no compensated summation.
 *
 * Conventions (problem formulation, eqs. "pairwise_ode" / "BS_kernel" and the
 * state-vector definition that follows them):
 *   state xy[2N]  : xy[0..N) = chi_i (x), xy[N..2N) = psi_i (y)   (SoA)
 *   velocity f[2N]: same layout
 *   kernel        : f_i = sum_{j != i} Gamma_j/(2 pi) * (-r_y, r_x)/(|r|^2 + delta^2),
 *                   r = x_i - x_j (target minus source).
 *                   The paper writes the core as "+ delta_k"; delta enters
 *                   squared here (delta is a length), one reading of an
 *                   inconsistent passage (kernel equation vs HyperPair).
 *   self pair     : excluded by index (j != i), never by testing r == 0.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TWO_PI 6.283185307179586476925286766559
#define OR_FOUR_PI 12.566370614359172953850573533118

/* ------------------------------------------------------------------------ */
/* Pair sum and its derivatives (problem formulation, kernel equation).      */
/* ------------------------------------------------------------------------ */

/* velocity of target i from all sources j != i */
static void vel_one(int64_t n, const double *xy, const double *gam, double d2,
                    int64_t i, double *fx, double *fy) {
  double sx = 0.0, sy = 0.0;
  const double xi = xy[i], yi = xy[n + i];
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    const double rx = xi - xy[j];
    const double ry = yi - xy[n + j];
    const double s = rx * rx + ry * ry + d2;
    sx += gam[j] * (-ry) / s;
    sy += gam[j] * rx / s;
  }
  *fx = sx / OR_TWO_PI;
  *fy = sy / OR_TWO_PI;
}

void or_velocity(int64_t n, const double *xy, const double *gam, double delta, double *f) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) vel_one(n, xy, gam, d2, i, &f[i], &f[n + i]);
}

/* velocity at a subset of targets: out[0..nt) = x-components, out[nt..2nt) = y */
void or_velocity_at(int64_t n, const double *xy, const double *gam, double delta, int64_t nt,
                    const int64_t *idx, double *out) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) vel_one(n, xy, gam, d2, idx[t], &out[t], &out[nt + t]);
}

/*
 * Derivative of the pair term with respect to r = x_i - x_j.  With
 * s = rx^2 + ry^2 + d^2 and u(r) = (-ry, rx)/s,
 *   du/dr = (1/s^2) [[ 2 rx ry,            ry^2 - rx^2 - d^2 ],
 *                    [ ry^2 - rx^2 + d^2, -2 rx ry           ]]
 * (differentiate u component-wise).  h[0..3] = row-major entries.
 */
static void du_dr(double rx, double ry, double d2, double h[4]) {
  const double s = rx * rx + ry * ry + d2;
  const double inv2 = 1.0 / (s * s);
  h[0] = 2.0 * rx * ry * inv2;
  h[1] = (ry * ry - rx * rx - d2) * inv2;
  h[2] = (ry * ry - rx * rx + d2) * inv2;
  h[3] = -2.0 * rx * ry * inv2;
}

/* (J v)_i = sum_{j != i} gamma_j/(2pi) * du/dr(r_ij) (v_i - v_j) */
static void jvp_one(int64_t n, const double *xy, const double *gam, double d2, const double *v,
                    int64_t i, double *ox, double *oy) {
  double ax = 0.0, ay = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double h[4];
    du_dr(xy[i] - xy[j], xy[n + i] - xy[n + j], d2, h);
    const double dvx = v[i] - v[j], dvy = v[n + i] - v[n + j];
    ax += gam[j] * (h[0] * dvx + h[1] * dvy);
    ay += gam[j] * (h[2] * dvx + h[3] * dvy);
  }
  *ox = ax / OR_TWO_PI;
  *oy = ay / OR_TWO_PI;
}

void or_jvp(int64_t n, const double *xy, const double *gam, double delta, const double *v,
            double *jv) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) jvp_one(n, xy, gam, d2, v, i, &jv[i], &jv[n + i]);
}

void or_jvp_at(int64_t n, const double *xy, const double *gam, double delta, const double *v,
               int64_t nt, const int64_t *idx, double *out) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) jvp_one(n, xy, gam, d2, v, idx[t], &out[t], &out[nt + t]);
}

/* Per-target 2x2 block of df/dx (the paper's inexact "diagonal block"
 * Jacobian): B_i = sum_{j != i} gamma_j du/dr(r_ij), entries row-major. */
static void bjac_one(int64_t n, const double *xy, const double *gam, double d2, int64_t i, double b[4]) {
  for (int q = 0; q < 4; ++q) b[q] = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double h[4];
    du_dr(xy[i] - xy[j], xy[n + i] - xy[n + j], d2, h);
    for (int q = 0; q < 4; ++q) b[q] += gam[j] * h[q];
  }
  for (int q = 0; q < 4; ++q) b[q] /= OR_TWO_PI;
}

/* All blocks, layout [4][N]. */
void or_block_jacobian(int64_t n, const double *xy, const double *gam, double delta, double *B) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double b[4];
    bjac_one(n, xy, gam, d2, i, b);
    for (int q = 0; q < 4; ++q) B[q * n + i] = b[q];
  }
}

/* The blocks of the targets idx[0..nt), layout [4][nt]. */
void or_block_jacobian_at(int64_t n, const double *xy, const double *gam, double delta, int64_t nt,
                          const int64_t *idx, double *out) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) {
    double b[4];
    bjac_one(n, xy, gam, d2, idx[t], b);
    for (int q = 0; q < 4; ++q) out[q * nt + t] = b[q];
  }
}

/*
 * Adjoint of the pair sum.  For a cotangent w:
 *   (J^T w)_k = sum_i (df_i/dx_k)^T w_i
 *             = sum_{j != k} H(r_kj)^T (gamma_j w_k - gamma_k w_j),
 * with H = du/dr (even in r) and gamma = Gamma/(2pi); and
 *   d(w.f)/dGamma_k = (1/2pi) sum_{i != k} w_i . u(x_i - x_k).
 */
static void vjp_one(int64_t n, const double *xy, const double *gam, double d2, const double *w,
                    int64_t k, double *gx, double *gy, double *gg) {
  double ax = 0.0, ay = 0.0, ag = 0.0;
  const double gk = gam[k];
  for (int64_t j = 0; j < n; ++j) {
    if (j == k) continue;
    double h[4];
    du_dr(xy[k] - xy[j], xy[n + k] - xy[n + j], d2, h);
    const double qx = gam[j] * w[k] - gk * w[j];
    const double qy = gam[j] * w[n + k] - gk * w[n + j];
    /* H^T q */
    ax += h[0] * qx + h[2] * qy;
    ay += h[1] * qx + h[3] * qy;
    /* u(x_j - x_k) = (-(y_j - y_k), x_j - x_k)/s */
    const double rx = xy[j] - xy[k], ry = xy[n + j] - xy[n + k];
    const double s = rx * rx + ry * ry + d2;
    ag += (w[j] * (-ry) + w[n + j] * rx) / s;
  }
  *gx = ax / OR_TWO_PI;
  *gy = ay / OR_TWO_PI;
  *gg = ag / OR_TWO_PI;
}

void or_vjp(int64_t n, const double *xy, const double *gam, double delta, const double *w,
            double *gxy, double *ggam) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) vjp_one(n, xy, gam, d2, w, k, &gxy[k], &gxy[n + k], &ggam[k]);
}

void or_vjp_at(int64_t n, const double *xy, const double *gam, double delta, const double *w,
               int64_t nt, const int64_t *idx, double *gxy_out, double *gg_out) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t)
    vjp_one(n, xy, gam, d2, w, idx[t], &gxy_out[t], &gxy_out[nt + t], &gg_out[t]);
}

/* Regularized Hamiltonian H_d = -(1/4pi) sum_{i != j} G_i G_j (1/2) log(|r|^2 + d^2),
 * the invariant of the regularized flow.  At d = 0 it is the paper's
 * Hamiltonian up to an overall sign convention. */
double or_hamiltonian(int64_t n, const double *xy, const double *gam, double delta) {
  const double d2 = delta * delta;
  double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double rx = xy[i] - xy[j], ry = xy[n + i] - xy[n + j];
      acc += gam[j] * 0.5 * log(rx * rx + ry * ry + d2);
    }
    total += gam[i] * acc;
  }
  return -total / OR_FOUR_PI;
}

/* Stream function of the regularized flow at every body, induced by the
 * others: psi_i = -(1/4pi) sum_{j != i} G_j log(|r|^2 + d^2).  The velocity is
 * its perpendicular gradient in the target position, f_i = (d psi_i/dy_i,
 * -d psi_i/dx_i), and the Hamiltonian is H = 1/2 sum_i G_i psi_i. */
static double psi_one(int64_t n, const double *xy, const double *gam, double d2, int64_t i) {
  double acc = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    const double rx = xy[i] - xy[j], ry = xy[n + i] - xy[n + j];
    acc += gam[j] * log(rx * rx + ry * ry + d2);
  }
  return -acc / OR_FOUR_PI;
}

void or_stream_function(int64_t n, const double *xy, const double *gam, double delta, double *psi) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) psi[i] = psi_one(n, xy, gam, d2, i);
}

/* stream function at a subset of targets */
void or_stream_function_at(int64_t n, const double *xy, const double *gam, double delta, int64_t nt,
                           const int64_t *idx, double *out) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) out[t] = psi_one(n, xy, gam, d2, idx[t]);
}

/* Velocity induced at nt arbitrary points p [2][nt] by all n bodies (no
 * exclusion): the grid velocity field of the metrics section. */
void or_velocity_points(int64_t nt, const double *p, int64_t n, const double *xy, const double *gam,
                        double delta, double *out) {
  const double d2 = delta * delta;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) {
    double sx = 0.0, sy = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double rx = p[t] - xy[j], ry = p[nt + t] - xy[n + j];
      const double s = rx * rx + ry * ry + d2;
      sx += gam[j] * (-ry) / s;
      sy += gam[j] * rx / s;
    }
    out[t] = sx / OR_TWO_PI;
    out[nt + t] = sy / OR_TWO_PI;
  }
}

/* ------------------------------------------------------------------------ */
/* Explicit RK4 (classic four-stage scheme).                                 */
/* ------------------------------------------------------------------------ */

static void axpy_into(int64_t m, double *out, const double *x, double a, const double *y) {
  for (int64_t q = 0; q < m; ++q) out[q] = x[q] + a * y[q];
}

/* One RK4 step x <- x + h/6 (k1 + 2k2 + 2k3 + k4).  `work` holds 5*2N doubles. */
static void rk4_step(int64_t n, double *x, const double *gam, double delta, double h, double *work) {
  const int64_t m = 2 * n;
  double *k1 = work, *k2 = work + m, *k3 = work + 2 * m, *k4 = work + 3 * m, *s = work + 4 * m;
  or_velocity(n, x, gam, delta, k1);
  axpy_into(m, s, x, 0.5 * h, k1);
  or_velocity(n, s, gam, delta, k2);
  axpy_into(m, s, x, 0.5 * h, k2);
  or_velocity(n, s, gam, delta, k3);
  axpy_into(m, s, x, h, k3);
  or_velocity(n, s, gam, delta, k4);
  for (int64_t q = 0; q < m; ++q) x[q] += h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
}

int or_rk4(int64_t n, double *xy, const double *gam, double delta, double dt, int nsteps) {
  double *work = (double *)malloc(sizeof(double) * 10 * n);
  if (!work) return -2;
  for (int s = 0; s < nsteps; ++s) rk4_step(n, xy, gam, delta, dt, work);
  free(work);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Implicit one-step linear multistep schemes (eq. "linKstep" with k = 1):   */
/*   r(xi) = xi - x_prev - dt (beta0 f(xi) + beta1 f(x_prev))                */
/*   backward Euler: beta0 = 1, beta1 = 0; trapezoid: beta0 = beta1 = 1/2.   */
/* Newton's method on r(xi) = 0; each Newton system (I - dt beta0 J) d = -r  */
/* is solved by restarted GMRES with the exact matrix-free Jacobian product. */
/* ------------------------------------------------------------------------ */

static double dot(int64_t m, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t q = 0; q < m; ++q) s += a[q] * b[q];
  return s;
}

typedef struct {
  int64_t n;
  const double *xi;
  const double *gam;
  double delta;
  double c; /* dt * beta0 */
  double *tmp;
} newton_op;

/* y = (I - c J(xi)) v */
static void newton_apply(const newton_op *op, const double *v, double *y) {
  or_jvp(op->n, op->xi, op->gam, op->delta, v, op->tmp);
  for (int64_t q = 0; q < 2 * op->n; ++q) y[q] = v[q] - op->c * op->tmp[q];
}

/* Restarted GMRES(mr) with modified Gram-Schmidt and Givens rotations.
 * Solves A x = b from x = 0 until |b - A x| <= rtol |b|.  Returns matvecs used. */
static int gmres(const newton_op *op, const double *b, double *x, int mr, double rtol, int maxit) {
  const int64_t m = 2 * op->n;
  double *V = (double *)malloc(sizeof(double) * m * (mr + 1));
  double *w = (double *)malloc(sizeof(double) * m);
  double *H = (double *)calloc((size_t)(mr + 1) * mr, sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * mr), *sn = (double *)malloc(sizeof(double) * mr);
  double *g = (double *)malloc(sizeof(double) * (mr + 1)), *yk = (double *)malloc(sizeof(double) * mr);
  memset(x, 0, sizeof(double) * m);
  const double bnorm = sqrt(dot(m, b, b));
  int used = 0;
  if (bnorm == 0.0) goto done;
  while (used < maxit) {
    /* r = b - A x */
    newton_apply(op, x, w);
    for (int64_t q = 0; q < m; ++q) V[q] = b[q] - w[q];
    double beta = sqrt(dot(m, V, V));
    if (beta <= rtol * bnorm) break;
    for (int64_t q = 0; q < m; ++q) V[q] /= beta;
    memset(g, 0, sizeof(double) * (mr + 1));
    g[0] = beta;
    int kk = 0;
    for (; kk < mr && used < maxit; ++kk) {
      newton_apply(op, V + kk * m, w);
      ++used;
      for (int i = 0; i <= kk; ++i) {
        const double hij = dot(m, w, V + i * m);
        H[i * mr + kk] = hij;
        for (int64_t q = 0; q < m; ++q) w[q] -= hij * V[i * m + q];
      }
      const double hn = sqrt(dot(m, w, w));
      H[(kk + 1) * mr + kk] = hn;
      if (hn > 0.0)
        for (int64_t q = 0; q < m; ++q) V[(kk + 1) * m + q] = w[q] / hn;
      for (int i = 0; i < kk; ++i) {
        const double a = H[i * mr + kk], c = H[(i + 1) * mr + kk];
        H[i * mr + kk] = cs[i] * a + sn[i] * c;
        H[(i + 1) * mr + kk] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[kk * mr + kk], c = H[(kk + 1) * mr + kk];
      const double rr = sqrt(a * a + c * c);
      cs[kk] = (rr == 0.0) ? 1.0 : a / rr;
      sn[kk] = (rr == 0.0) ? 0.0 : c / rr;
      H[kk * mr + kk] = rr;
      H[(kk + 1) * mr + kk] = 0.0;
      g[kk + 1] = -sn[kk] * g[kk];
      g[kk] = cs[kk] * g[kk];
      if (fabs(g[kk + 1]) <= rtol * bnorm || hn == 0.0) {
        ++kk;
        break;
      }
    }
    /* back-substitute the kk x kk triangle and update x */
    for (int i = kk - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < kk; ++j) s -= H[i * mr + j] * yk[j];
      yk[i] = s / H[i * mr + i];
    }
    for (int i = 0; i < kk; ++i)
      for (int64_t q = 0; q < m; ++q) x[q] += yk[i] * V[i * m + q];
    if (kk > 0 && fabs(g[kk]) <= rtol * bnorm) break;
  }
done:
  free(V); free(w); free(H); free(cs); free(sn); free(g); free(yk);
  return used;
}

typedef struct {
  int32_t newton_iters; /* total Newton iterations over all steps */
  int32_t krylov_iters; /* total GMRES matvecs */
  int32_t nonconverged_steps;
  int32_t pad;
  double max_final_rel_residual;
} or_newton_stats;

/* scheme 0 = backward Euler, 1 = trapezoid.  Newton stops when
 * |r(xi)| <= newton_tol |r(x_prev)|.  u [2n] (may be NULL) is a background
 * velocity added to every body's right-hand side, dx_i/dt = f_i(x) + u_i:
 * the inflow of the mushroom-cloud experiment (parametric results).  It does
 * not depend on x, so the Jacobian is unchanged. */
int or_implicit_forced(int64_t n, double *xy, const double *gam, double delta, const double *u, double dt,
                       int nsteps, int scheme, double newton_tol, int max_newton, double gmres_tol,
                       int gmres_restart, int gmres_maxit, or_newton_stats *st) {
  const int64_t m = 2 * n;
  const double beta0 = (scheme == 0) ? 1.0 : 0.5, beta1 = (scheme == 0) ? 0.0 : 0.5;
  double *xprev = (double *)malloc(sizeof(double) * m), *fprev = (double *)malloc(sizeof(double) * m);
  double *f = (double *)malloc(sizeof(double) * m), *r = (double *)malloc(sizeof(double) * m);
  double *d = (double *)malloc(sizeof(double) * m), *tmp = (double *)malloc(sizeof(double) * m);
  memset(st, 0, sizeof(*st));
  for (int step = 0; step < nsteps; ++step) {
    memcpy(xprev, xy, sizeof(double) * m);
    or_velocity(n, xprev, gam, delta, fprev);
    if (u)
      for (int64_t q = 0; q < m; ++q) fprev[q] += u[q];
    double r0 = -1.0, rn = 0.0;
    int it = 0;
    for (;; ++it) {
      or_velocity(n, xy, gam, delta, f);
      if (u)
        for (int64_t q = 0; q < m; ++q) f[q] += u[q];
      for (int64_t q = 0; q < m; ++q)
        r[q] = xy[q] - xprev[q] - dt * (beta0 * f[q] + beta1 * fprev[q]);
      rn = sqrt(dot(m, r, r));
      if (r0 < 0.0) r0 = rn;
      if (rn <= newton_tol * r0 || r0 == 0.0) break;
      if (it >= max_newton) {
        st->nonconverged_steps++;
        break;
      }
      for (int64_t q = 0; q < m; ++q) r[q] = -r[q];
      newton_op op = {n, xy, gam, delta, dt * beta0, tmp};
      /* op.xi aliases xy: GMRES only reads it while xy is unchanged */
      st->krylov_iters += gmres(&op, r, d, gmres_restart, gmres_tol, gmres_maxit);
      for (int64_t q = 0; q < m; ++q) xy[q] += d[q];
    }
    st->newton_iters += it;
    const double rel = (r0 > 0.0) ? rn / r0 : 0.0;
    if (rel > st->max_final_rel_residual) st->max_final_rel_residual = rel;
  }
  free(xprev); free(fprev); free(f); free(r); free(d); free(tmp);
  return st->nonconverged_steps ? 1 : 0;
}

/* The paper's FOM solver (problem formulation, after eq. "linKstep"): an
 * inexact Newton method whose Jacobian keeps only the diagonal 2x2 blocks
 * of the kernel Jacobian, B_i = df_i/dx_i.  Each Newton correction solves
 * (I - dt beta0 B_i) d_i = -r_i body by body (Cramer's rule); the converged
 * state is a root of the same residual as the exact Newton iteration.
 * jac_period = 0 evaluates B at every Newton iterate; p >= 1 evaluates it
 * at the first iterate (x_prev) of steps 0, p, 2p, ... of this call and
 * keeps it in between (the paper's Jacobian update every p_it steps). */
int or_implicit_block(int64_t n, double *xy, const double *gam, double delta, const double *u, double dt,
                      int nsteps, int scheme, double newton_tol, int max_newton, int jac_period,
                      or_newton_stats *st) {
  const int64_t m = 2 * n;
  const double beta0 = (scheme == 0) ? 1.0 : 0.5, beta1 = (scheme == 0) ? 0.0 : 0.5;
  double *xprev = (double *)malloc(sizeof(double) * m), *fprev = (double *)malloc(sizeof(double) * m);
  double *f = (double *)malloc(sizeof(double) * m), *r = (double *)malloc(sizeof(double) * m);
  double *B = (double *)malloc(sizeof(double) * 4 * n);
  memset(st, 0, sizeof(*st));
  for (int step = 0; step < nsteps; ++step) {
    memcpy(xprev, xy, sizeof(double) * m);
    or_velocity(n, xprev, gam, delta, fprev);
    if (u)
      for (int64_t q = 0; q < m; ++q) fprev[q] += u[q];
    double r0 = -1.0, rn = 0.0;
    int it = 0;
    for (;; ++it) {
      or_velocity(n, xy, gam, delta, f);
      if (u)
        for (int64_t q = 0; q < m; ++q) f[q] += u[q];
      for (int64_t q = 0; q < m; ++q)
        r[q] = xy[q] - xprev[q] - dt * (beta0 * f[q] + beta1 * fprev[q]);
      rn = sqrt(dot(m, r, r));
      if (r0 < 0.0) r0 = rn;
      if (rn <= newton_tol * r0 || r0 == 0.0) break;
      if (it >= max_newton) {
        st->nonconverged_steps++;
        break;
      }
      if (jac_period == 0 || (it == 0 && step % jac_period == 0)) or_block_jacobian(n, xy, gam, delta, B);
      const double c = dt * beta0;
      for (int64_t i = 0; i < n; ++i) {
        /* A = I - c B_i acting on (dx_i, dy_i) */
        const double a00 = 1.0 - c * B[i], a01 = -c * B[n + i];
        const double a10 = -c * B[2 * n + i], a11 = 1.0 - c * B[3 * n + i];
        const double det = a00 * a11 - a01 * a10;
        const double bx = -r[i], by = -r[n + i];
        xy[i] += (bx * a11 - a01 * by) / det;
        xy[n + i] += (a00 * by - a10 * bx) / det;
      }
    }
    st->newton_iters += it;
    const double rel = (r0 > 0.0) ? rn / r0 : 0.0;
    if (rel > st->max_final_rel_residual) st->max_final_rel_residual = rel;
  }
  free(xprev); free(fprev); free(f); free(r); free(B);
  return st->nonconverged_steps ? 1 : 0;
}

int or_implicit(int64_t n, double *xy, const double *gam, double delta, double dt, int nsteps,
                int scheme, double newton_tol, int max_newton, double gmres_tol, int gmres_restart,
                int gmres_maxit, or_newton_stats *st) {
  return or_implicit_forced(n, xy, gam, delta, NULL, dt, nsteps, scheme, newton_tol, max_newton, gmres_tol,
                            gmres_restart, gmres_maxit, st);
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the RK4 map.  For y = x + h/6 (k1 + 2k2 + 2k3 + k4)   */
/* with stage inputs s1 = x, s2 = x + h/2 k1, s3 = x + h/2 k2, s4 = x + h k3 */
/* and lam = dQ/dy, the chain rule taken stage by stage backwards gives      */
/*   kap4 = h/6 lam,                 a4 = J(s4)^T kap4                        */
/*   kap3 = h/3 lam + h a4,          a3 = J(s3)^T kap3                        */
/*   kap2 = h/3 lam + h/2 a3,        a2 = J(s2)^T kap2                        */
/*   kap1 = h/6 lam + h/2 a2,        a1 = J(s1)^T kap1                        */
/*   dQ/dx = lam + a1 + a2 + a3 + a4                                          */
/* and dQ/dGamma accumulates the Gamma-partials of kap_s . f(s_s).            */
/* The oracle stores every step state (no checkpointing).                    */
/* ------------------------------------------------------------------------ */

int or_rk4_adjoint(int64_t n, const double *xy0, const double *gam, double delta, double dt,
                   int nsteps, const double *lamT, const double *gg_direct, double *xyT,
                   double *lam0, double *gg) {
  const int64_t m = 2 * n;
  double *states = (double *)malloc(sizeof(double) * m * (size_t)(nsteps + 1));
  double *work = (double *)malloc(sizeof(double) * 5 * m);
  double *st[4], *kap[4], *a[4];
  double *buf = (double *)malloc(sizeof(double) * 12 * m);
  double *gpart = (double *)malloc(sizeof(double) * n);
  if (!states || !work || !buf || !gpart) return -2;
  for (int q = 0; q < 4; ++q) {
    st[q] = buf + q * m;
    kap[q] = buf + (4 + q) * m;
    a[q] = buf + (8 + q) * m;
  }
  memcpy(states, xy0, sizeof(double) * m);
  for (int s = 0; s < nsteps; ++s) {
    memcpy(states + (size_t)(s + 1) * m, states + (size_t)s * m, sizeof(double) * m);
    rk4_step(n, states + (size_t)(s + 1) * m, gam, delta, dt, work);
  }
  if (xyT) memcpy(xyT, states + (size_t)nsteps * m, sizeof(double) * m);
  memcpy(lam0, lamT, sizeof(double) * m);
  for (int64_t q = 0; q < n; ++q) gg[q] = gg_direct ? gg_direct[q] : 0.0;
  const double h = dt;
  double *k = work; /* stage velocity scratch */
  for (int s = nsteps - 1; s >= 0; --s) {
    const double *x = states + (size_t)s * m;
    /* recompute the stage inputs of this step */
    memcpy(st[0], x, sizeof(double) * m);
    or_velocity(n, st[0], gam, delta, k);
    axpy_into(m, st[1], x, 0.5 * h, k);
    or_velocity(n, st[1], gam, delta, k);
    axpy_into(m, st[2], x, 0.5 * h, k);
    or_velocity(n, st[2], gam, delta, k);
    axpy_into(m, st[3], x, h, k);
    const double *lam = lam0;
    for (int64_t q = 0; q < m; ++q) kap[3][q] = h / 6.0 * lam[q];
    or_vjp(n, st[3], gam, delta, kap[3], a[3], gpart);
    for (int64_t q = 0; q < n; ++q) gg[q] += gpart[q];
    for (int64_t q = 0; q < m; ++q) kap[2][q] = h / 3.0 * lam[q] + h * a[3][q];
    or_vjp(n, st[2], gam, delta, kap[2], a[2], gpart);
    for (int64_t q = 0; q < n; ++q) gg[q] += gpart[q];
    for (int64_t q = 0; q < m; ++q) kap[1][q] = h / 3.0 * lam[q] + 0.5 * h * a[2][q];
    or_vjp(n, st[1], gam, delta, kap[1], a[1], gpart);
    for (int64_t q = 0; q < n; ++q) gg[q] += gpart[q];
    for (int64_t q = 0; q < m; ++q) kap[0][q] = h / 6.0 * lam[q] + 0.5 * h * a[1][q];
    or_vjp(n, st[0], gam, delta, kap[0], a[0], gpart);
    for (int64_t q = 0; q < n; ++q) gg[q] += gpart[q];
    for (int64_t q = 0; q < m; ++q) lam0[q] += a[0][q] + a[1][q] + a[2][q] + a[3][q];
  }
  free(states); free(work); free(buf); free(gpart);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Online PTROM step: HyperPair (Algorithm "HyperPair") inside the online    */
/* Gauss-Newton loop (Algorithm "Gauss-Newton").                             */
/*                                                                           */
/* Artifacts (all produced offline):                                         */
/*   ns sampled bodies, nd = 2 ns sampled rows ordered [chi of samples,      */
/*   psi of samples] like the full state vector;                             */
/*   Phibar[nd][M], xbar0[nd]  : rows of Phi and x^0 at the sampled rows;    */
/*   Nc unique surrogate sources: xqt0[Nc][2], Phit[Nc][2][M], Gt[Nc];       */
/*   CSR lists off[ns+1], ids[nnz]: the sources each sampled target sees      */
/*   (its own body is never listed);                                         */
/*   A[Mr][nd] = [P Phi_r]^+  (NULL means the identity, Mr = nd: plain LSPG). */
/* jac_mode 0 = the paper's inexact Jacobian (target 2x2 block only),        */
/*          1 = exact (adds the motion of the surrogate sources).            */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t M, Mr, ns, jac_mode;
  int64_t Nc;
  const double *Phibar, *xbar0, *xqt0, *Phit, *Gt, *A;
  const int64_t *off, *ids;
  double delta, dt;
  const double *ubar; /* [nd] background velocity at the sampled rows, or NULL */
} or_rom;

/* One HyperPair evaluation at generalized coordinates xhat (source clustering
 * with the Biot-Savart kernel of the governing equations).
 * Outputs: xbar[nd] (sampled positions), fbar[nd] (sampled velocities, with
 * the background velocity ubar when there is one),
 * rbar[nd] (trapezoid residual rows), C[nd][M] (residual Jacobian times Phi). */
static void rom_hyperpair(const or_rom *R, const double *xhat, const double *xbar_prev,
                          const double *fbar_prev, double *xbar, double *fbar, double *rbar,
                          double *C) {
  const int M = R->M, ns = R->ns, nd = 2 * ns;
  const double d2 = R->delta * R->delta, hdt = 0.5 * R->dt;
  /* sampled targets: xbar = xbar0 + Phibar xhat */
  for (int q = 0; q < nd; ++q) {
    double s = R->xbar0[q];
    for (int c = 0; c < M; ++c) s += R->Phibar[(size_t)q * M + c] * xhat[c];
    xbar[q] = s;
  }
  /* surrogate sources: p_c = xqt0_c + Phit_c xhat */
  double *p = (double *)malloc(sizeof(double) * 2 * (size_t)(R->Nc > 0 ? R->Nc : 1));
  for (int64_t c = 0; c < R->Nc; ++c)
    for (int d = 0; d < 2; ++d) {
      double s = R->xqt0[2 * c + d];
      for (int q = 0; q < M; ++q) s += R->Phit[(2 * c + d) * (size_t)M + q] * xhat[q];
      p[2 * c + d] = s;
    }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < ns; ++i) {
    const double tx = xbar[i], ty = xbar[ns + i];
    double fx = 0.0, fy = 0.0, b[4] = {0, 0, 0, 0};
    double *E = (double *)calloc(2 * (size_t)M, sizeof(double));
    for (int64_t e = R->off[i]; e < R->off[i + 1]; ++e) {
      const int64_t c = R->ids[e];
      const double rx = tx - p[2 * c], ry = ty - p[2 * c + 1];
      const double s = rx * rx + ry * ry + d2;
      /* A surrogate can sit exactly on its target when delta = 0 (its
       * Gamma-weighted mean is taken in physical space, its cell was chosen
       * in the weighted POD space): such a pair, like the self pair, adds
       * neither velocity nor Jacobian. */
      if (s == 0.0) continue;
      const double g = R->Gt[c] / OR_TWO_PI;
      fx += g * (-ry) / s;
      fy += g * rx / s;
      double h[4];
      du_dr(rx, ry, d2, h);
      for (int q = 0; q < 4; ++q) b[q] += g * h[q];
      if (R->jac_mode == 1)
        for (int q = 0; q < M; ++q) {
          const double px = R->Phit[(2 * c) * (size_t)M + q], py = R->Phit[(2 * c + 1) * (size_t)M + q];
          E[q] += g * (h[0] * px + h[1] * py);
          E[M + q] += g * (h[2] * px + h[3] * py);
        }
    }
    if (R->ubar) {
      fx += R->ubar[i];
      fy += R->ubar[ns + i];
    }
    fbar[i] = fx;
    fbar[ns + i] = fy;
    rbar[i] = tx - xbar_prev[i] - hdt * (fx + fbar_prev[i]);
    rbar[ns + i] = ty - xbar_prev[ns + i] - hdt * (fy + fbar_prev[ns + i]);
    for (int q = 0; q < M; ++q) {
      const double phx = R->Phibar[(size_t)i * M + q], phy = R->Phibar[(size_t)(ns + i) * M + q];
      /* d fbar_i / d xhat = B_i Phibar_i - E (E only in the exact mode) */
      const double dfx = b[0] * phx + b[1] * phy - E[q];
      const double dfy = b[2] * phx + b[3] * phy - E[M + q];
      C[(size_t)i * M + q] = phx - hdt * dfx;
      C[(size_t)(ns + i) * M + q] = phy - hdt * dfy;
    }
    free(E);
  }
  free(p);
}

/* Least squares min |G x - b| for G[m][n] (m >= n, full column rank) by
 * Householder QR.  G and b are overwritten. */
static void householder_lstsq(int m, int n, double *G, double *b, double *x) {
  for (int k = 0; k < n; ++k) {
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += G[(size_t)i * n + k] * G[(size_t)i * n + k];
    nrm = sqrt(nrm);
    if (nrm == 0.0) continue;
    const double alpha = (G[(size_t)k * n + k] > 0.0) ? -nrm : nrm;
    /* v = g_k - alpha e_k, stored in column k below and on the diagonal */
    G[(size_t)k * n + k] -= alpha;
    double vnorm2 = 0.0;
    for (int i = k; i < m; ++i) vnorm2 += G[(size_t)i * n + k] * G[(size_t)i * n + k];
    for (int j = k + 1; j < n; ++j) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += G[(size_t)i * n + k] * G[(size_t)i * n + j];
      s = 2.0 * s / vnorm2;
      for (int i = k; i < m; ++i) G[(size_t)i * n + j] -= s * G[(size_t)i * n + k];
    }
    double s = 0.0;
    for (int i = k; i < m; ++i) s += G[(size_t)i * n + k] * b[i];
    s = 2.0 * s / vnorm2;
    for (int i = k; i < m; ++i) b[i] -= s * G[(size_t)i * n + k];
    G[(size_t)k * n + k] = alpha; /* R's diagonal */
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= G[(size_t)k * n + j] * x[j];
    x[k] = s / G[(size_t)k * n + k];
  }
}

int or_lstsq(int m, int n, const double *G, const double *b, double *x) {
  double *Gc = (double *)malloc(sizeof(double) * (size_t)m * n), *bc = (double *)malloc(sizeof(double) * m);
  memcpy(Gc, G, sizeof(double) * (size_t)m * n);
  memcpy(bc, b, sizeof(double) * m);
  householder_lstsq(m, n, Gc, bc, x);
  free(Gc); free(bc);
  return 0;
}

/* HyperPair at one xhat, for kernel-level comparisons. */
void or_rom_hyperpair(const or_rom *R, const double *xhat, const double *xbar_prev,
                      const double *fbar_prev, double *xbar, double *fbar, double *rbar, double *C) {
  rom_hyperpair(R, xhat, xbar_prev, fbar_prev, xbar, fbar, rbar, C);
}

/*
 * nsteps online time steps from xhat (in/out).  Per step n, starting from
 * xhat^{n-1}:
 *   repeat: HyperPair at xhat_k -> rbar, C;  G = A C, b = A rbar;
 *           d = -argmin |G nu + b|;  xhat_{k+1} = xhat_k + alpha d;
 *           eps_k = |G^T b| / |G_1^T b_1|;  k += 1
 *   while eps_k > tol and k <= max_iter.
 * The previous-step terms of the trapezoid residual are the sampled
 * positions at the accepted xhat^{n-1} and the velocity of the last
 * HyperPair evaluation of step n-1 (step 0: HyperPair at the initial xhat).
 * Optional records: xhat_hist[nsteps][M], iters[nsteps], and every residual
 * rbar in resid_hist[cap][nd] (the residual snapshots of offline stage 3).
 * Returns 0, or 1 when some step stopped at max_iter.
 */
int or_rom_run(const or_rom *R, double alpha, double tol, int max_iter, int nsteps, double *xhat,
               double *xhat_hist, int32_t *iters, double *resid_hist, int64_t resid_cap,
               int64_t *resid_count) {
  const int M = R->M, nd = 2 * R->ns;
  const int Mr = R->A ? R->Mr : nd;
  double *xbar = (double *)malloc(sizeof(double) * nd), *fbar = (double *)malloc(sizeof(double) * nd);
  double *rbar = (double *)malloc(sizeof(double) * nd), *C = (double *)malloc(sizeof(double) * (size_t)nd * M);
  double *xbar_prev = (double *)malloc(sizeof(double) * nd), *fbar_prev = (double *)malloc(sizeof(double) * nd);
  double *G = (double *)malloc(sizeof(double) * (size_t)Mr * M), *b = (double *)malloc(sizeof(double) * Mr);
  double *d = (double *)malloc(sizeof(double) * M), *gvec = (double *)malloc(sizeof(double) * M);
  int status = 0;
  int64_t nrec = 0;
  /* initial previous-step terms: HyperPair at the initial xhat; its residual is not used */
  {
    double *zeros = (double *)calloc(nd, sizeof(double));
    rom_hyperpair(R, xhat, zeros, zeros, xbar_prev, fbar_prev, rbar, C);
    free(zeros);
  }
  for (int step = 0; step < nsteps; ++step) {
    int k = 1;
    double g1 = 0.0, eps = 1.0;
    do {
      rom_hyperpair(R, xhat, xbar_prev, fbar_prev, xbar, fbar, rbar, C);
      if (resid_hist && nrec < resid_cap) memcpy(resid_hist + nrec * nd, rbar, sizeof(double) * nd);
      ++nrec;
      if (R->A) {
        for (int r = 0; r < Mr; ++r) {
          double sb = 0.0;
          for (int q = 0; q < nd; ++q) sb += R->A[(size_t)r * nd + q] * rbar[q];
          b[r] = sb;
          for (int c = 0; c < M; ++c) {
            double s = 0.0;
            for (int q = 0; q < nd; ++q) s += R->A[(size_t)r * nd + q] * C[(size_t)q * M + c];
            G[(size_t)r * M + c] = s;
          }
        }
      } else {
        memcpy(G, C, sizeof(double) * (size_t)nd * M);
        memcpy(b, rbar, sizeof(double) * nd);
      }
      double gn = 0.0;
      for (int c = 0; c < M; ++c) {
        double s = 0.0;
        for (int r = 0; r < Mr; ++r) s += G[(size_t)r * M + c] * b[r];
        gvec[c] = s;
        gn += s * s;
      }
      gn = sqrt(gn);
      if (k == 1) g1 = gn;
      householder_lstsq(Mr, M, G, b, d);
      for (int c = 0; c < M; ++c) xhat[c] -= alpha * d[c];
      eps = (g1 > 0.0) ? gn / g1 : 0.0;
      ++k;
    } while (eps > tol && k <= max_iter);
    if (eps > tol) status = 1;
    if (iters) iters[step] = k - 1;
    if (xhat_hist) memcpy(xhat_hist + (size_t)step * M, xhat, sizeof(double) * M);
    /* previous-step terms for the next step */
    for (int q = 0; q < nd; ++q) {
      double s = R->xbar0[q];
      for (int c = 0; c < M; ++c) s += R->Phibar[(size_t)q * M + c] * xhat[c];
      xbar_prev[q] = s;
    }
    memcpy(fbar_prev, fbar, sizeof(double) * nd);
  }
  if (resid_count) *resid_count = nrec;
  free(xbar); free(fbar); free(rbar); free(C); free(xbar_prev); free(fbar_prev);
  free(G); free(b); free(d); free(gvec);
  return status;
}

/* Thread count of the OpenMP loops (for timing the oracle on one core);
 * returns the previous maximum. */
int or_set_threads(int n) {
  const int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
}
