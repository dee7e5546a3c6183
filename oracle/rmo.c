/*
 * rmo.c -- plain, slow FP64 CPU oracle for the outer-region R-matrix energy loop.
 *
 * TEST INFRASTRUCTURE ONLY (see rmo.h).  Written for readability: every stage is
 * the textbook definition or a published algorithm in its plain form, computed
 * in long double.  No blocking, no fusion, no reordering beyond what the
 * definitions state.
 *
 * Stage map (PSTGF paper):
 *   form_R            eq. (rmatrix)
 *   channel split     eps_i = E - e_i, open iff eps_i > 0 (text after eq. (radial))
 *   open_channel      Coulomb F, G at r = a (section "Overview", asymptotic form)
 *   closed_channel    exponentially decaying Whittaker function at r = a (Glossary)
 *   match_and_solve   eq. (match) with the asymptotic forms substituted
 *   s_and_omega       Glossary: T-matrix, collision strength
 */
#include "rmo.h"

#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
typedef long double _Complex cld;

#define CF_TOL 1e-17L        /* relative agreement of successive depths */
#define CF_MAXDEPTH (1 << 22) /* iteration cap -> RMO_PT_NOCONV */

static double nan_value(void) { return (double)NAN; }

/* ------------------------------------------------------------------------- */
/* Stage 1: R-matrix, eq. (rmatrix): R_ij = (1/2a) sum_k w_ik w_jk / (E_k - E) */
/* ------------------------------------------------------------------------- */
static int32_t form_R_one(const rmo_pw *pw, double E, double *R) {
  const int n = pw->nchan, M = pw->npole;
  for (int k = 0; k < M; ++k)
    if (pw->Ek[k] == E) {
      for (long t = 0; t < (long)n * n; ++t) R[t] = nan_value();
      return RMO_PT_POLE;
    }
  /* lower triangle, row i holds columns 0..i.  When called outside a parallel
     region (one energy at a time) the rows are shared among threads; each row's
     sum still runs over k in ascending order. */
  ld *acc = (ld *)calloc((size_t)n * (n + 1) / 2, sizeof(ld));
#ifdef _OPENMP
  const int par = !omp_in_parallel() && n >= 128;
#pragma omp parallel if (par)
#endif
  for (int k = 0; k < M; ++k) {
    const double *wk = pw->w + (size_t)k * n;
    const ld d = 1.0L / ((ld)pw->Ek[k] - (ld)E);
#ifdef _OPENMP
#pragma omp for schedule(static, 1)
#endif
    for (int i = 0; i < n; ++i) {
      const ld wi = (ld)wk[i] * d;
      ld *row = acc + (size_t)i * (i + 1) / 2;
      for (int j = 0; j <= i; ++j) row[j] += wi * (ld)wk[j];
    }
  }
  const ld scale = 1.0L / (2.0L * (ld)pw->a);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      const double v = (double)(acc[(size_t)i * (i + 1) / 2 + j] * scale);
      R[(size_t)i * n + j] = v;
      R[(size_t)j * n + i] = v;
    }
  free(acc);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Radial ODE u'' = (l(l+1)/r^2 - 2z/r - eps) u, Taylor-series steps inward.   */
/* The only singular point is r = 0, so a series about r0 converges for       */
/* |h| < r0; steps use |h| <= r0/2 and at most ~1.5 local wavelengths/decay    */
/* lengths.  Coefficients follow from (r0+x)^2 u'' = (L2 - 2z(r0+x) -          */
/* eps (r0+x)^2) u, written for d_n = c_n h^n.                                */
/* ------------------------------------------------------------------------- */
static int taylor_inward(ld z, ld eps, ld L2, ld r0, ld r1, ld *u, ld *up, int renorm) {
  ld r = r0, U = *u, Up = *up;
  long steps = 0;
  enum { NT = 400 };
  ld d[NT + 3];
  while (r > r1) {
    ld kl = sqrtl(fabsl(eps + 2.0L * z / r - L2 / (r * r))) + 1e-3L;
    ld h = -fminl(0.5L * r, 1.5L / kl);
    if (r + h < r1) h = r1 - r;
    const ld A = L2 - 2.0L * z * r - eps * r * r;
    const ld B = -(2.0L * z + 2.0L * eps * r);
    const ld C = -eps;
    d[0] = U;
    d[1] = Up * h;
    ld su = d[0] + d[1], sd = d[1];
    int small = 0, n;
    for (n = 0; n < NT; ++n) {
      const ld dm1 = n >= 1 ? d[n - 1] : 0.0L;
      const ld dm2 = n >= 2 ? d[n - 2] : 0.0L;
      const ld num = (A - (ld)n * (n - 1)) * d[n] * h * h - 2.0L * r * (ld)n * (n + 1) * d[n + 1] * h +
                     B * dm1 * h * h * h + C * dm2 * h * h * h * h;
      d[n + 2] = num / (r * r * (ld)(n + 1) * (n + 2));
      su += d[n + 2];
      sd += (ld)(n + 2) * d[n + 2];
      if (fabsl(d[n + 2]) < 1e-22L * (fabsl(su) + fabsl(sd))) {
        if (++small >= 3) break;
      } else {
        small = 0;
      }
    }
    if (n >= NT) return -1;
    U = su;
    Up = sd / h;
    if (renorm) {
      const ld s = 1.0L / fmaxl(fabsl(U), fabsl(Up));
      U *= s;
      Up *= s;
    }
    r += h;
    if (++steps > 50000000L) return -1;
  }
  *u = U;
  *up = Up;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Coulomb functions by Steed's method (Barnett, Feng, Steed & Goldfarb,      */
/* Comput. Phys. Commun. 8 (1974) 377), with two changes of evaluation order:  */
/*  - CF1 (F'/F) is summed backward from a depth that is doubled until the    */
/*    value is stable; the sign of F_l follows from the signs of the          */
/*    denominators (F_L > 0 at large L).                                      */
/*  - CF2 ((G'+iF')/(G+iF)) is rewritten so that the large leading term       */
/*    i(1 - eta/rho) cancels analytically: with beta_n = rho - eta + i n and   */
/*    c_n = rho^2 - 2 eta rho - l(l+1) + i rho (2n-1), the tails               */
/*    v_n = (c_n + beta_n v_{n+1}) / (beta_n - i + v_{n+1}) give              */
/*    (G'+iF')/(G+iF) = (1 + i v_1) / rho.                                    */
/* ------------------------------------------------------------------------- */
static ld cf1_at_depth(ld eta, ld rho, int l, int Lmax, int *sign) {
  ld f = (ld)(Lmax + 1) / rho;
  int sg = 1;
  for (int L = Lmax - 1; L >= l; --L) {
    const ld Lp = (ld)(L + 1);
    const ld S = Lp / rho + eta / Lp;
    const ld R2 = 1.0L + eta * eta / (Lp * Lp);
    const ld den = S + f;
    if (den < 0) sg = -sg;
    f = S - R2 / den;
  }
  *sign = sg;
  return f;
}

static int cf1(ld eta, ld rho, int l, ld *f, int *sign) {
  const ld Ltp = sqrtl(rho * rho + 2.0L * fabsl(eta) * rho);
  int extra = 2 * (int)Ltp + 60;
  ld prev = cf1_at_depth(eta, rho, l, l + extra, sign);
  for (int it = 0; it < 20; ++it) {
    extra *= 2;
    int sg;
    const ld cur = cf1_at_depth(eta, rho, l, l + extra, &sg);
    if (fabsl(cur - prev) <= CF_TOL * fabsl(cur)) {
      *f = cur;
      *sign = sg;
      return 0;
    }
    prev = cur;
  }
  return -1;
}

static cld cf2_at_depth(ld eta, ld rho, int l, long N) {
  const ld L2 = (ld)l * (l + 1);
  const ld cre = rho * rho - 2.0L * eta * rho - L2;
  /* tail estimate: fixed point of the last map, v^2 - i v - c = 0 */
  const cld cN = cre + I * rho * (ld)(2 * (N + 1) - 1);
  cld v = (I + csqrtl(-1.0L + 4.0L * cN)) / 2.0L;
  for (long n = N; n >= 1; --n) {
    const cld c = cre + I * rho * (ld)(2 * n - 1);
    const cld beta = (rho - eta) + I * (ld)n;
    v = (c + beta * v) / (beta - I + v);
  }
  return (1.0L + I * v) / rho;
}

static int cf2(ld eta, ld rho, int l, ld *p, ld *q) {
  long N = 32;
  cld prev = cf2_at_depth(eta, rho, l, N);
  while (N < CF_MAXDEPTH) {
    N *= 2;
    const cld cur = cf2_at_depth(eta, rho, l, N);
    if (cabsl(cur - prev) <= CF_TOL * cabsl(cur)) {
      *p = creall(cur);
      *q = cimagl(cur);
      return 0;
    }
    prev = cur;
  }
  return -1;
}

/* F, F', G, G' (derivatives w.r.t. rho) at rho; returns -1 if a series or
   continued fraction did not converge. */
static int coulomb_fg(ld eta, ld rho, int l, ld out[4]) {
  const ld L2 = (ld)l * (l + 1);
  /* outer turning point rho_tp = eta + sqrt(eta^2 + l(l+1)), written without
     cancellation for eta < 0 */
  ld rtp;
  if (L2 == 0)
    rtp = eta > 0 ? 2.0L * eta : 0.0L;
  else
    rtp = eta <= 0 ? L2 / (sqrtl(eta * eta + L2) - eta) : eta + sqrtl(eta * eta + L2);
  const ld rm = rho >= rtp ? rho : rtp;
  ld p, q, fm;
  int sg;
  if (cf2(eta, rm, l, &p, &q) || cf1(eta, rm, l, &fm, &sg)) return -1;
  ld F = (ld)sg / sqrtl((fm - p) * (fm - p) / q + q);
  ld Fp = fm * F;
  ld G = (fm - p) * F / q;
  ld Gp = p * G - q * F;
  if (rm > rho) {
    /* inside the turning point G grows inward: integrate it from rm to rho,
       then F from CF1 at rho and the Wronskian F'G - FG' = 1 */
    ld g = G, gp = Gp;
    if (taylor_inward(1.0L * -eta, 1.0L, L2, rm, rho, &g, &gp, 0)) return -1;
    ld f;
    if (cf1(eta, rho, l, &f, &sg)) return -1;
    G = g;
    Gp = gp;
    F = 1.0L / (f * G - Gp);
    Fp = f * F;
  }
  out[0] = F;
  out[1] = Fp;
  out[2] = G;
  out[3] = Gp;
  return 0;
}
/* note: in the rho variable the Coulomb equation reads
   u'' = (l(l+1)/rho^2 + 2 eta/rho - 1) u, i.e. the radial ODE above with
   z -> -eta and eps -> 1, which is how taylor_inward is called. */

/* ------------------------------------------------------------------------- */
/* Closed channels.  The decaying solution is W_{nu,l+1/2}(2 kappa r),         */
/* nu = z/kappa.  Continuing CF2 to k = i kappa (rho = i kappa r, eta = i nu)  */
/* makes the v-recursion real: with b_n = kappa r - nu + n and                 */
/* c_n = 2 z r - kappa^2 r^2 - l(l+1) - kappa r (2n-1),                        */
/* w_n = (b_n w_{n+1} - c_n) / (b_n - 1 + w_{n+1}) and W'/W = (1 - w_1)/r.     */
/* The backward recursion is stable only where b_1 > 0, i.e. r > (nu-1)/kappa; */
/* it is evaluated at rs = max(a, (nu+2)/kappa) and the solution is carried    */
/* inward to a with Taylor steps (W grows inward beyond the turning point and  */
/* oscillates inside it, so inward integration is stable).                    */
/* ------------------------------------------------------------------------- */
static ld closed_cf_at_depth(ld z, ld kap, ld r, int l, long N) {
  const ld nu = z / kap, L2 = (ld)l * (l + 1);
  const ld base = 2.0L * z * r - kap * kap * r * r - L2;
  const ld cN = base - kap * r * (ld)(2 * (N + 1) - 1);
  const ld disc = 1.0L - 4.0L * cN;
  ld w = disc > 0 ? (1.0L + sqrtl(disc)) / 2.0L : 0.0L;
  for (long n = N; n >= 1; --n) {
    const ld c = base - kap * r * (ld)(2 * n - 1);
    const ld b = kap * r - nu + (ld)n;
    w = (b * w - c) / (b - 1.0L + w);
  }
  return (1.0L - w) / r;
}

static int closed_logderiv_at(ld z, ld kap, ld r, int l, ld *L) {
  long N = 32;
  ld prev = closed_cf_at_depth(z, kap, r, l, N);
  while (N < CF_MAXDEPTH) {
    N *= 2;
    const ld cur = closed_cf_at_depth(z, kap, r, l, N);
    if (fabsl(cur - prev) <= CF_TOL * fabsl(cur) + 1e-300L) {
      *L = cur;
      return 0;
    }
    prev = cur;
  }
  return -1;
}

/* (W, W') at r = a up to a common positive or negative factor */
static int closed_uw(ld z, ld eps, ld a, int l, ld *u, ld *up) {
  const ld kap = sqrtl(-eps), nu = z / kap;
  const ld rs = fmaxl(a, (nu + 2.0L) / kap);
  ld L;
  if (closed_logderiv_at(z, kap, rs, l, &L)) return -1;
  ld U = 1.0L, Up = L;
  if (rs > a && taylor_inward(z, eps, (ld)l * (l + 1), rs, a, &U, &Up, 1)) return -1;
  *u = U;
  *up = Up;
  return 0;
}

/* channel functions at r = a */
static int channel_fn(ld z, ld eps, ld a, int l, ld out[4]) {
  if (eps > 0) {
    const ld k = sqrtl(eps), eta = -z / k, rho = k * a;
    ld fg[4];
    if (coulomb_fg(eta, rho, l, fg)) return -1;
    const ld sk = sqrtl(k);
    out[0] = fg[0] / sk; /* s  */
    out[1] = fg[1] * sk; /* s' (d/dr = k d/drho) */
    out[2] = fg[2] / sk; /* c  */
    out[3] = fg[3] * sk; /* c' */
    return 0;
  }
  ld u, up;
  if (closed_uw(z, eps, a, l, &u, &up)) return -1;
  ld nrm = sqrtl(u * u + a * a * up * up);
  if (u < 0 || (u == 0 && up < 0)) nrm = -nrm;
  out[0] = 0;
  out[1] = 0;
  out[2] = u / nrm;
  out[3] = up / nrm;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Dense linear algebra (long double, plain Gaussian elimination).            */
/* ------------------------------------------------------------------------- */
/* LU with partial pivoting in place, row-major n x n; piv[i] = row swapped in */
static int lu_factor(ld *A, int n, int *piv) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    ld best = fabsl(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r)
      if (fabsl(A[(size_t)r * n + c]) > best) {
        best = fabsl(A[(size_t)r * n + c]);
        p = r;
      }
    piv[c] = p;
    if (best == 0) return -1;
    if (p != c)
      for (int j = 0; j < n; ++j) {
        ld t = A[(size_t)c * n + j];
        A[(size_t)c * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = t;
      }
    const ld inv = 1.0L / A[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      const ld m = A[(size_t)r * n + c] * inv;
      A[(size_t)r * n + c] = m;
      if (m != 0)
        for (int j = c + 1; j < n; ++j) A[(size_t)r * n + j] -= m * A[(size_t)c * n + j];
    }
  }
  return 0;
}

/* solve A x = b (trans = 0) or A^T x = b (trans = 1) with the LU above */
static void lu_solve(const ld *LU, int n, const int *piv, ld *x, int trans) {
  if (!trans) {
    for (int c = 0; c < n; ++c)
      if (piv[c] != c) {
        ld t = x[c];
        x[c] = x[piv[c]];
        x[piv[c]] = t;
      }
    for (int r = 0; r < n; ++r)
      for (int j = 0; j < r; ++j) x[r] -= LU[(size_t)r * n + j] * x[j];
    for (int r = n - 1; r >= 0; --r) {
      for (int j = r + 1; j < n; ++j) x[r] -= LU[(size_t)r * n + j] * x[j];
      x[r] /= LU[(size_t)r * n + r];
    }
  } else {
    /* A = P^T L U  ->  A^T = U^T L^T P */
    for (int r = 0; r < n; ++r) {
      for (int j = 0; j < r; ++j) x[r] -= LU[(size_t)j * n + r] * x[j];
      x[r] /= LU[(size_t)r * n + r];
    }
    for (int r = n - 1; r >= 0; --r)
      for (int j = r + 1; j < n; ++j) x[r] -= LU[(size_t)j * n + r] * x[j];
    for (int c = n - 1; c >= 0; --c)
      if (piv[c] != c) {
        ld t = x[c];
        x[c] = x[piv[c]];
        x[piv[c]] = t;
      }
  }
}

/* Hager's 1-norm estimate of ||A^-1||_1 (Hager 1984, with Higham's 1988
   refinements as used in LAPACK xLACON) times ||A||_1. */
static ld cond1_estimate(const ld *A, const ld *LU, int n, const int *piv) {
  ld anorm = 0;
  for (int j = 0; j < n; ++j) {
    ld s = 0;
    for (int i = 0; i < n; ++i) s += fabsl(A[(size_t)i * n + j]);
    if (s > anorm) anorm = s;
  }
  ld *x = (ld *)malloc(sizeof(ld) * n), *y = (ld *)malloc(sizeof(ld) * n);
  for (int i = 0; i < n; ++i) x[i] = 1.0L / n;
  ld est = 0;
  int jlast = -1;
  for (int it = 0; it < 5; ++it) {
    memcpy(y, x, sizeof(ld) * n);
    lu_solve(LU, n, piv, y, 0);
    ld ny = 0;
    for (int i = 0; i < n; ++i) ny += fabsl(y[i]);
    if (it > 0 && ny <= est) break;
    est = ny;
    for (int i = 0; i < n; ++i) y[i] = y[i] >= 0 ? 1.0L : -1.0L;
    lu_solve(LU, n, piv, y, 1);
    int j = 0;
    for (int i = 1; i < n; ++i)
      if (fabsl(y[i]) > fabsl(y[j])) j = i;
    if (j == jlast) break;
    jlast = j;
    for (int i = 0; i < n; ++i) x[i] = 0;
    x[j] = 1;
  }
  /* alternative vector x_i = (-1)^i (1 + i/(n-1)) */
  for (int i = 0; i < n; ++i) x[i] = (i % 2 ? -1.0L : 1.0L) * (1.0L + (n > 1 ? (ld)i / (n - 1) : 0));
  lu_solve(LU, n, piv, x, 0);
  ld alt = 0;
  for (int i = 0; i < n; ++i) alt += fabsl(x[i]);
  alt = 2.0L * alt / (3.0L * n);
  if (alt > est) est = alt;
  free(x);
  free(y);
  return anorm * est;
}

/* ------------------------------------------------------------------------- */
/* Matching, eq. (match): F(a) = R (a F'(a) - b F(a)), with F_ij = s_i d_ij +  */
/* c_i K_ij on open rows and e_i X_ij on closed rows.  Writing C_i = c_i (open) */
/* or e_i (closed) and Y = [K; X] gives A Y = B with                          */
/*   A_im = d_im C_i - R_im (a C'_m - b C_m)                                   */
/*   B_ij = R_{i,o_j} (a s'_{o_j} - b s_{o_j}) - d_{i,o_j} s_{o_j}             */
/* ------------------------------------------------------------------------- */
static int open_list(const rmo_pw *pw, double E, int *idx);

static int32_t solve_K_one(const rmo_pw *pw, double E, const double *R, const double *fg, double *K,
                           double *cond) {
  const int n = pw->nchan;
  const ld a = pw->a, b = pw->b;
  int *open_idx = (int *)malloc(sizeof(int) * (n + 1));
  const int no = open_list(pw, E, open_idx);
  for (long t = 0; t < (long)n * n; ++t) K[t] = 0.0;
  if (cond) *cond = 0;
  if (no == 0) {
    free(open_idx);
    return 0;
  }
  ld *A = (ld *)malloc(sizeof(ld) * (size_t)n * n);
  ld *LU = (ld *)malloc(sizeof(ld) * (size_t)n * n);
  ld *Y = (ld *)malloc(sizeof(ld) * (size_t)n * no);
  int *piv = (int *)malloc(sizeof(int) * n);
  for (int i = 0; i < n; ++i)
    for (int m = 0; m < n; ++m) {
      const ld Cm = fg[4 * m + 2], Cpm = fg[4 * m + 3];
      A[(size_t)i * n + m] = (i == m ? (ld)fg[4 * i + 2] : 0.0L) - (ld)R[(size_t)i * n + m] * (a * Cpm - b * Cm);
    }
  memcpy(LU, A, sizeof(ld) * (size_t)n * n);
  int32_t st = 0;
  if (lu_factor(LU, n, piv)) {
    st = RMO_PT_SINGULAR;
  } else {
    ld *col = (ld *)malloc(sizeof(ld) * n);
    for (int j = 0; j < no; ++j) {
      const int oj = open_idx[j];
      const ld s = fg[4 * oj + 0], sp = fg[4 * oj + 1];
      for (int i = 0; i < n; ++i) col[i] = (ld)R[(size_t)i * n + oj] * (a * sp - b * s) - (i == oj ? s : 0.0L);
      lu_solve(LU, n, piv, col, 0);
      for (int i = 0; i < n; ++i) Y[(size_t)i * no + j] = col[i];
    }
    free(col);
    for (int i = 0; i < no; ++i)
      for (int j = 0; j < no; ++j) K[(size_t)i * n + j] = (double)Y[(size_t)open_idx[i] * no + j];
    if (cond) *cond = (double)cond1_estimate(A, LU, n, piv);
  }
  free(A);
  free(LU);
  free(Y);
  free(piv);
  free(open_idx);
  return st;
}

/* ------------------------------------------------------------------------- */
/* S = (1 + iK)(1 - iK)^-1 by complex Gaussian elimination, T = S - 1,         */
/* Omega_pq = (g/2) sum_{i in p, j in q, open} |T_ij|^2.                       */
/* ------------------------------------------------------------------------- */
static int32_t s_and_omega_one(const rmo_pw *pw, const double *K, int no, const int *open_idx,
                               double *omega, double *S) {
  const int n = pw->nchan, nt = pw->ntarget;
  for (long t = 0; t < (long)nt * nt; ++t) omega[t] = 0.0;
  if (S)
    for (long t = 0; t < 2L * n * n; ++t) S[t] = 0.0;
  if (no == 0) return 0;
  /* M = (1 - iK), augmented with (1 + iK)^T so that solving M^T X^T = (1+iK)^T
     gives X = (1 + iK) M^-1 */
  cld *Mt = (cld *)malloc(sizeof(cld) * (size_t)no * no);
  cld *rhs = (cld *)malloc(sizeof(cld) * (size_t)no * no);
  for (int i = 0; i < no; ++i)
    for (int j = 0; j < no; ++j) {
      const ld kij = K[(size_t)i * n + j], kji = K[(size_t)j * n + i];
      Mt[(size_t)i * no + j] = (i == j ? 1.0L : 0.0L) - I * kji;  /* (1 - iK)^T */
      rhs[(size_t)i * no + j] = (i == j ? 1.0L : 0.0L) + I * kji; /* (1 + iK)^T */
      (void)kij;
    }
  /* Gaussian elimination with partial pivoting on Mt, applied to rhs columns */
  int32_t st = 0;
  for (int c = 0; c < no && !st; ++c) {
    int p = c;
    ld best = cabsl(Mt[(size_t)c * no + c]);
    for (int r = c + 1; r < no; ++r)
      if (cabsl(Mt[(size_t)r * no + c]) > best) {
        best = cabsl(Mt[(size_t)r * no + c]);
        p = r;
      }
    if (best == 0) {
      st = RMO_PT_SINGULAR;
      break;
    }
    if (p != c)
      for (int j = 0; j < no; ++j) {
        cld t = Mt[(size_t)c * no + j];
        Mt[(size_t)c * no + j] = Mt[(size_t)p * no + j];
        Mt[(size_t)p * no + j] = t;
        t = rhs[(size_t)c * no + j];
        rhs[(size_t)c * no + j] = rhs[(size_t)p * no + j];
        rhs[(size_t)p * no + j] = t;
      }
    for (int r = c + 1; r < no; ++r) {
      const cld m = Mt[(size_t)r * no + c] / Mt[(size_t)c * no + c];
      if (m == 0) continue;
      for (int j = c; j < no; ++j) Mt[(size_t)r * no + j] -= m * Mt[(size_t)c * no + j];
      for (int j = 0; j < no; ++j) rhs[(size_t)r * no + j] -= m * rhs[(size_t)c * no + j];
    }
  }
  if (!st) {
    for (int r = no - 1; r >= 0; --r)
      for (int j = 0; j < no; ++j) {
        cld acc = rhs[(size_t)r * no + j];
        for (int q = r + 1; q < no; ++q) acc -= Mt[(size_t)r * no + q] * rhs[(size_t)q * no + j];
        rhs[(size_t)r * no + j] = acc / Mt[(size_t)r * no + r];
      }
    /* rhs now holds X^T with X = S */
    const ld half_g = 0.5L * (ld)pw->g;
    ld *om = (ld *)calloc((size_t)nt * nt, sizeof(ld));
    for (int i = 0; i < no; ++i)
      for (int j = 0; j < no; ++j) {
        const cld Sij = rhs[(size_t)j * no + i];
        const cld Tij = Sij - (i == j ? 1.0L : 0.0L);
        const ld t2 = creall(Tij) * creall(Tij) + cimagl(Tij) * cimagl(Tij);
        om[(size_t)pw->target[open_idx[i]] * nt + pw->target[open_idx[j]]] += half_g * t2;
        if (S) {
          S[2 * ((size_t)i * n + j) + 0] = (double)creall(Sij);
          S[2 * ((size_t)i * n + j) + 1] = (double)cimagl(Sij);
        }
      }
    for (long t = 0; t < (long)nt * nt; ++t) omega[t] = (double)om[t];
    free(om);
  }
  free(Mt);
  free(rhs);
  return st;
}

/* ------------------------------------------------------------------------- */
/* Per-energy drivers                                                         */
/* ------------------------------------------------------------------------- */
static int32_t asym_one(const rmo_pw *pw, double E, double thr_guard, double *fg, int8_t *open,
                        int32_t *nopen) {
  const int n = pw->nchan;
  int32_t st = 0;
  int no = 0;
  for (int i = 0; i < n; ++i) {
    const ld eps = (ld)E - (ld)pw->e_thr[i];
    double *o = fg + 4 * i;
    open[i] = eps > 0;
    if (eps > 0) no++;
    if (fabsl(eps) < (ld)thr_guard) {
      st |= RMO_PT_THRESHOLD;
      o[0] = o[1] = o[2] = o[3] = nan_value();
      continue;
    }
    ld v[4];
    if (channel_fn((ld)pw->z, eps, (ld)pw->a, pw->l[i], v)) {
      st |= RMO_PT_NOCONV;
      o[0] = o[1] = o[2] = o[3] = nan_value();
      continue;
    }
    for (int t = 0; t < 4; ++t) o[t] = (double)v[t];
  }
  *nopen = no;
  return st;
}

static void fill_nan(double *x, long count) {
  for (long t = 0; t < count; ++t) x[t] = nan_value();
}

static int all_finite(const double *x, long count) {
  for (long t = 0; t < count; ++t)
    if (!isfinite(x[t])) return 0;
  return 1;
}

static void set_threads(int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int rmo_form_R(const rmo_pw *pw, const double *E, int32_t ne, double *R, int32_t *status,
               int32_t nthreads) {
  const long nn = (long)pw->nchan * pw->nchan;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) status[e] = form_R_one(pw, E[e], R + e * nn);
  return 0;
}

int rmo_asymptotic(const rmo_pw *pw, const double *E, int32_t ne, double thr_guard, double *fg,
                   int8_t *open, int32_t *nopen, int32_t *status, int32_t nthreads) {
  const int n = pw->nchan;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e)
    status[e] = asym_one(pw, E[e], thr_guard, fg + (long)e * n * 4, open + (long)e * n, nopen + e);
  return 0;
}

int rmo_solve_K(const rmo_pw *pw, const double *E, int32_t ne, const double *R, const double *fg,
                double thr_guard, double *K, double *cond, int32_t *status, int32_t nthreads) {
  const int n = pw->nchan;
  const long nn = (long)n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    int32_t st = 0;
    for (int k = 0; k < pw->npole; ++k)
      if (pw->Ek[k] == E[e]) st |= RMO_PT_POLE;
    for (int i = 0; i < n; ++i)
      if (fabs(E[e] - pw->e_thr[i]) < thr_guard) st |= RMO_PT_THRESHOLD;
    if (!all_finite(R + e * nn, nn) || !all_finite(fg + (long)e * n * 4, 4L * n)) st |= RMO_PT_NONFINITE;
    if (st) {
      fill_nan(K + e * nn, nn);
      if (cond) cond[e] = nan_value();
    } else {
      st = solve_K_one(pw, E[e], R + e * nn, fg + (long)e * n * 4, K + e * nn, cond ? cond + e : NULL);
      if (st) fill_nan(K + e * nn, nn);
    }
    status[e] = st;
  }
  return 0;
}

static int open_list(const rmo_pw *pw, double E, int *idx) {
  int no = 0;
  for (int i = 0; i < pw->nchan; ++i)
    if ((ld)E - (ld)pw->e_thr[i] > 0) idx[no++] = i;
  return no;
}

int rmo_collision_strengths(const rmo_pw *pw, const double *E, int32_t ne, const double *K,
                            double thr_guard, double *omega, double *S, int32_t *status,
                            int32_t nthreads) {
  const int n = pw->nchan, nt = pw->ntarget;
  const long nn = (long)n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    int *idx = (int *)malloc(sizeof(int) * (n + 1));
    const int no = open_list(pw, E[e], idx);
    int32_t st = 0;
    for (int i = 0; i < n; ++i)
      if (fabs(E[e] - pw->e_thr[i]) < thr_guard) st |= RMO_PT_THRESHOLD;
    for (int i = 0; i < no && !st; ++i)
      for (int j = 0; j < no; ++j)
        if (!isfinite(K[e * nn + (long)i * n + j])) st |= RMO_PT_NONFINITE;
    if (!st) st = s_and_omega_one(pw, K + e * nn, no, idx, omega + (long)e * nt * nt, S ? S + 2 * e * nn : NULL);
    if (st) {
      fill_nan(omega + (long)e * nt * nt, (long)nt * nt);
      if (S) fill_nan(S + 2 * e * nn, 2 * nn);
    }
    status[e] = st;
    free(idx);
  }
  return 0;
}

int rmo_run(const rmo_pw *pw, const double *E, int32_t ne, double thr_guard, double *omega,
            double *K, double *S, double *cond, int32_t *status, int32_t nthreads) {
  const int n = pw->nchan, nt = pw->ntarget;
  const long nn = (long)n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    double *R = (double *)malloc(sizeof(double) * nn);
    double *fg = (double *)malloc(sizeof(double) * 4 * n);
    double *Kl = K ? K + e * nn : (double *)malloc(sizeof(double) * nn);
    int8_t *op = (int8_t *)malloc(n);
    int *idx = (int *)malloc(sizeof(int) * (n + 1));
    int32_t no = 0;
    int32_t st = form_R_one(pw, E[e], R);
    st |= asym_one(pw, E[e], thr_guard, fg, op, &no);
    if (!st && (!all_finite(R, nn) || !all_finite(fg, 4L * n))) st |= RMO_PT_NONFINITE;
    if (!st) st = solve_K_one(pw, E[e], R, fg, Kl, cond ? cond + e : NULL);
    if (!st) {
      const int no2 = open_list(pw, E[e], idx);
      st = s_and_omega_one(pw, Kl, no2, idx, omega + (long)e * nt * nt, S ? S + 2 * e * nn : NULL);
    }
    if (st) {
      fill_nan(Kl, nn);
      fill_nan(omega + (long)e * nt * nt, (long)nt * nt);
      if (S) fill_nan(S + 2 * e * nn, 2 * nn);
      if (cond) cond[e] = nan_value();
    }
    status[e] = st;
    if (!K) free(Kl);
    free(R);
    free(fg);
    free(op);
    free(idx);
  }
  return 0;
}

int rmo_coulomb(double eta, double rho, int32_t l, double out[4]) {
  ld v[4];
  if (coulomb_fg(eta, rho, l, v)) return -1;
  for (int t = 0; t < 4; ++t) out[t] = (double)v[t];
  return 0;
}

int rmo_closed_logderiv(double z, double eps, double r, int32_t l, double *L) {
  ld u, up;
  if (closed_uw(z, eps, r, l, &u, &up)) return -1;
  *L = (double)(up / u);
  return 0;
}

int rmo_channel(double z, double eps, double a, int32_t l, double out[4]) {
  ld v[4];
  if (channel_fn(z, eps, a, l, v)) return -1;
  for (int t = 0; t < 4; ++t) out[t] = (double)v[t];
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Long-range multipole coupling and Numerov propagation between r0 = a and   */
/* the asymptotic radius r1 (section "Overview": eq. (radial) with the        */
/* coupling U_nm, and the propagation of the coupled radial functions by a    */
/* Numerov method between the inner-region boundary and r1).                  */
/*                                                                            */
/* Reading of the garbled eq. (radial), in Rydberg units:                     */
/*   F'' = Q(r) F,  Q = diag(l_i(l_i+1)/r^2 - 2z/r - eps_i) + 2 U(r),          */
/*   U_ij(r) = sum_{lam=1..lamax} cf[lam-1][i][j] r^-(lam+1)                   */
/* (cf: the multipole coefficients of the H.DAT symmetry record, symmetric).  */
/*                                                                            */
/* Solution columns, ordered as the unknowns of the matching: the decaying    */
/* solution e_j of every closed channel j, the irregular c_j of every open    */
/* channel, then the regular s_j of every open channel.  At r1 each column    */
/* takes the value and derivative of its uncoupled analytic function in its   */
/* own channel (U is neglected beyond r1); its value at r1 - h comes from the */
/* Taylor series of the coupled equations about r1.                           */
/* Numerov inward with Z = T Y, T = 1 - (h^2/12) Q:                           */
/*   Z_{k-1} = (12 - 10 T_k) Y_k - Z_{k+1},  Y_k = T_k^-1 Z_k,                 */
/* on r_k = a + k h (k = npts-1 .. -1, h = (r1 - a)/(npts - 1)).  Every        */
/* `stab` steps the columns are recombined so that the closed rows of the     */
/* newest Z are the identity on the closed columns and zero on the others:    */
/* adding decaying solutions to any column leaves K unchanged, and it stops   */
/* the inward-growing closed components from swamping the open columns.       */
/* At r0: Y_0 and Y'_0 = [(2 Z_1 - Y_1) - (2 Z_-1 - Y_-1)] / (2h) (the O(h^4)  */
/* derivative that goes with Numerov).                                        */
/* ------------------------------------------------------------------------- */

/* Q(r) of one energy into q (n x n), eps[i] = E - e_i */
static void coupled_Q(const rmo_pw *pw, const rmo_coupling *cp, const ld *eps, ld r, ld *q) {
  const int n = pw->nchan;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      ld u = 0;
      ld rp = 1.0L / (r * r);
      for (int lam = 1; lam <= cp->lamax; ++lam) {
        u += (ld)cp->cf[((size_t)(lam - 1) * n + i) * n + j] * rp;
        rp /= r;
      }
      q[(size_t)i * n + j] = 2.0L * u;
    }
  for (int i = 0; i < n; ++i) {
    const ld L2 = (ld)pw->l[i] * (pw->l[i] + 1);
    q[(size_t)i * n + i] += L2 / (r * r) - 2.0L * (ld)pw->z / r - eps[i];
  }
}

/* Y = T^-1 Z for T = 1 - (h^2/12) Q (n x n), m columns */
static int numerov_solve(const ld *q, ld h, int n, int m, const ld *Z, ld *Y, ld *T, int *piv) {
  for (long t = 0; t < (long)n * n; ++t) T[t] = -(h * h / 12.0L) * q[t];
  for (int i = 0; i < n; ++i) T[(size_t)i * n + i] += 1.0L;
  if (lu_factor(T, n, piv)) return -1;
  ld *col = (ld *)malloc(sizeof(ld) * n);
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < n; ++i) col[i] = Z[(size_t)i * m + j];
    lu_solve(T, n, piv, col, 0);
    for (int i = 0; i < n; ++i) Y[(size_t)i * m + j] = col[i];
  }
  free(col);
  return 0;
}

/* Z = T Y */
static void numerov_T(const ld *q, ld h, int n, int m, const ld *Y, ld *Z) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      ld acc = Y[(size_t)i * m + j];
      for (int k = 0; k < n; ++k) acc -= (h * h / 12.0L) * q[(size_t)i * n + k] * Y[(size_t)k * m + j];
      Z[(size_t)i * m + j] = acc;
    }
}

/* column recombination of the state pair (Zn newest, Zo older); closed rows cr[0..nc) */
static int stabilise(int n, int m, int nc, const int *cr, ld *Zn, ld *Zo) {
  if (nc == 0) return 0;
  ld *G = (ld *)malloc(sizeof(ld) * (size_t)nc * nc);
  int *piv = (int *)malloc(sizeof(int) * nc);
  ld *col = (ld *)malloc(sizeof(ld) * nc);
  ld *tmp = (ld *)malloc(sizeof(ld) * (size_t)n * nc);
  int bad = 0;
  for (int a = 0; a < nc; ++a)
    for (int b = 0; b < nc; ++b) G[(size_t)a * nc + b] = Zn[(size_t)cr[a] * m + b];
  if (lu_factor(G, nc, piv)) bad = 1;
  for (int s = 0; s < 2 && !bad; ++s) {
    ld *Z = s == 0 ? Zn : Zo;
    /* closed columns: Z_E <- Z_E G^-1, row by row (G^T x = row^T) */
    for (int i = 0; i < n; ++i) {
      for (int b = 0; b < nc; ++b) col[b] = Z[(size_t)i * m + b];
      lu_solve(G, nc, piv, col, 1);
      for (int b = 0; b < nc; ++b) tmp[(size_t)i * nc + b] = col[b];
    }
    for (int i = 0; i < n; ++i)
      for (int b = 0; b < nc; ++b) Z[(size_t)i * m + b] = tmp[(size_t)i * nc + b];
  }
  if (!bad) {
    /* the other columns: X <- X - Z_E alpha, alpha = closed rows of the newest X */
    ld *alpha = (ld *)malloc(sizeof(ld) * (size_t)nc * m);
    for (int a = 0; a < nc; ++a)
      for (int j = nc; j < m; ++j) alpha[(size_t)a * m + j] = Zn[(size_t)cr[a] * m + j];
    for (int s = 0; s < 2; ++s) {
      ld *Z = s == 0 ? Zn : Zo;
      for (int i = 0; i < n; ++i)
        for (int j = nc; j < m; ++j) {
          ld acc = Z[(size_t)i * m + j];
          for (int a = 0; a < nc; ++a) acc -= Z[(size_t)i * m + a] * alpha[(size_t)a * m + j];
          Z[(size_t)i * m + j] = acc;
        }
    }
    free(alpha);
  }
  free(G);
  free(piv);
  free(col);
  free(tmp);
  return bad ? -1 : 0;
}

/* value and derivative at r1 of the uncoupled function of column type kind
   (0 = e, closed; 1 = c; 2 = s) in channel i */
static int start_values(const rmo_pw *pw, int i, ld eps, ld r1, int kind, ld *v, ld *dv) {
  ld f[4];  /* channel_fn: open (s, s', c, c'), closed (0, 0, e, e') */
  if (channel_fn(pw->z, eps, r1, pw->l[i], f)) return -1;
  *v = f[kind == 2 ? 0 : 2];
  *dv = f[kind == 2 ? 1 : 3];
  return 0;
}

/* Y(r1 - h) of the coupled solutions with Y(r1) = Y1, Y'(r1) = dY1 (n x m),
   from the Taylor series of Y'' = Q Y about r1: with Q(r1 + x) = sum_p q_p x^p
   and Y = sum_j c_j x^j, (j+2)(j+1) c_{j+2} = sum_{p<=j} q_p c_{j-p}. */
static void taylor_start(const rmo_pw *pw, const rmo_coupling *cp, const ld *eps, ld r1, ld h, int m,
                         const ld *Y1, const ld *dY1, ld *Y0) {
  const int n = pw->nchan;
  enum { JT = 40 };
  const size_t nm = (size_t)n * m, nn = (size_t)n * n;
  ld *c = (ld *)calloc((JT + 2) * nm, sizeof(ld)), *q = (ld *)calloc((JT + 1) * nn, sizeof(ld));
  /* q_p: (r1 + x)^-k = r1^-k sum_p (-1)^p C(k+p-1, p) (x/r1)^p */
  for (int p = 0; p <= JT; ++p) {
    ld sgn = (p % 2) ? -1.0L : 1.0L;
    ld *qp = q + p * nn;
    for (int i = 0; i < n; ++i) {
      const ld L2 = (ld)pw->l[i] * (pw->l[i] + 1);
      ld d = L2 * powl(r1, -2.0L - p) * (ld)(p + 1) * sgn - 2.0L * (ld)pw->z * powl(r1, -1.0L - p) * sgn;
      if (p == 0) d -= eps[i];
      qp[(size_t)i * n + i] += d;
    }
    for (int lam = 1; lam <= cp->lamax; ++lam) {
      /* C(lam + p, p) */
      ld binom = 1.0L;
      for (int t = 1; t <= p; ++t) binom = binom * (ld)(lam + t) / (ld)t;
      const ld w = 2.0L * binom * sgn * powl(r1, -(ld)(lam + 1) - p);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) qp[(size_t)i * n + j] += w * (ld)cp->cf[((size_t)(lam - 1) * n + i) * n + j];
    }
  }
  memcpy(c, Y1, sizeof(ld) * nm);
  memcpy(c + nm, dY1, sizeof(ld) * nm);
  for (int j = 0; j + 2 <= JT + 1; ++j) {
    ld *out = c + (j + 2) * nm;
    for (int p = 0; p <= j; ++p) {
      const ld *qp = q + p * nn, *cj = c + (j - p) * nm;
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
          const ld v = qp[(size_t)i * n + k];
          if (v == 0) continue;
          for (int t = 0; t < m; ++t) out[(size_t)i * m + t] += v * cj[(size_t)k * m + t];
        }
    }
    for (size_t t = 0; t < nm; ++t) out[t] /= (ld)(j + 2) * (j + 1);
  }
  for (size_t t = 0; t < nm; ++t) {
    ld acc = 0, xp = 1.0L;
    for (int j = 0; j <= JT + 1; ++j) {
      acc += c[j * nm + t] * xp;
      xp *= -h;
    }
    Y0[t] = acc;
  }
  free(c);
  free(q);
}

/* one energy: phi, dphi [n][2n] (columns: closed e, open c, open s; rest 0) */
static int32_t propagate_one(const rmo_pw *pw, const rmo_coupling *cp, double E, double thr_guard, double *phi,
                             double *dphi, int8_t *open, int32_t *nopen) {
  const int n = pw->nchan, N = cp->npts;
  const ld a = pw->a, r1 = cp->r1, h = (r1 - a) / (ld)(N - 1);
  int32_t st = 0;
  ld *eps = (ld *)malloc(sizeof(ld) * n);
  int *col_ch = (int *)malloc(sizeof(int) * 2 * n), *col_kind = (int *)malloc(sizeof(int) * 2 * n);
  int *cr = (int *)malloc(sizeof(int) * n);
  int nc = 0, no = 0;
  for (int i = 0; i < n; ++i) {
    eps[i] = (ld)E - (ld)pw->e_thr[i];
    open[i] = eps[i] > 0;
    if (fabsl(eps[i]) < (ld)thr_guard) st |= RMO_PT_THRESHOLD;
    if (eps[i] > 0) no++;
    else cr[nc++] = i;
  }
  *nopen = no;
  /* columns: closed e (ascending), open c, open s */
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (!(eps[i] > 0)) col_ch[m] = i, col_kind[m++] = 0;
  for (int i = 0; i < n; ++i)
    if (eps[i] > 0) col_ch[m] = i, col_kind[m++] = 1;
  for (int i = 0; i < n; ++i)
    if (eps[i] > 0) col_ch[m] = i, col_kind[m++] = 2;
  for (long t = 0; t < 2L * n * n; ++t) phi[t] = dphi[t] = 0.0;
  if (st) goto done;
  {
    const size_t nm = (size_t)n * m;
    ld *Zp = (ld *)calloc(nm, sizeof(ld)), *Zc = (ld *)calloc(nm, sizeof(ld)), *Zn = (ld *)malloc(sizeof(ld) * nm);
    ld *Y = (ld *)malloc(sizeof(ld) * nm), *q = (ld *)malloc(sizeof(ld) * (size_t)n * n);
    ld *T = (ld *)malloc(sizeof(ld) * (size_t)n * n);
    ld *Z1 = (ld *)malloc(sizeof(ld) * nm), *Y1 = (ld *)malloc(sizeof(ld) * nm), *Y0 = (ld *)malloc(sizeof(ld) * nm);
    int *piv = (int *)malloc(sizeof(int) * n);
    /* Y at r_{N-1} = r1: each column its uncoupled function (value and
       derivative); at r_{N-2} the coupled solutions through those data */
    ld *Ya = (ld *)calloc(nm, sizeof(ld)), *dYa = (ld *)calloc(nm, sizeof(ld)), *Yb = (ld *)calloc(nm, sizeof(ld));
    for (int j = 0; j < m && !st; ++j) {
      ld v, dv;
      if (start_values(pw, col_ch[j], eps[col_ch[j]], r1, col_kind[j], &v, &dv)) st |= RMO_PT_NOCONV;
      Ya[(size_t)col_ch[j] * m + j] = v;
      dYa[(size_t)col_ch[j] * m + j] = dv;
    }
    if (!st) taylor_start(pw, cp, eps, r1, h, m, Ya, dYa, Yb);
    if (!st) {
      coupled_Q(pw, cp, eps, a + (ld)(N - 1) * h, q);
      numerov_T(q, h, n, m, Ya, Zp);
      coupled_Q(pw, cp, eps, a + (ld)(N - 2) * h, q);
      numerov_T(q, h, n, m, Yb, Zc);
      /* step s computes Z_{k-1}, k = N-1-s, from Z_{k+1} (Zp) and Z_k (Zc);
         the last step (k = 0) gives Z_{-1} */
      for (int s = 1; s <= N - 1 && !st; ++s) {
        const int k = N - 1 - s;
        coupled_Q(pw, cp, eps, a + (ld)k * h, q);
        if (numerov_solve(q, h, n, m, Zc, Y, T, piv)) {
          st |= RMO_PT_SINGULAR;
          break;
        }
        if (k == 1) memcpy(Y1, Y, sizeof(ld) * nm);
        if (k == 0) memcpy(Y0, Y, sizeof(ld) * nm);
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < m; ++j) {
            ld qy = 0;
            for (int t = 0; t < n; ++t) qy += q[(size_t)i * n + t] * Y[(size_t)t * m + j];
            Zn[(size_t)i * m + j] = 2.0L * Y[(size_t)i * m + j] + (10.0L * h * h / 12.0L) * qy - Zp[(size_t)i * m + j];
          }
        ld *tmp = Zp;
        Zp = Zc;
        Zc = Zn;
        Zn = tmp;
        /* now Zp = Z_k, Zc = Z_{k-1}; recombinations stop once Z_1 is formed
           (the last three points feed the derivative at r0) */
        if (s % cp->stab == 0 && s <= N - 3 && stabilise(n, m, nc, cr, Zc, Zp)) st |= RMO_PT_SINGULAR;
        if (k - 1 == 1) memcpy(Z1, Zc, sizeof(ld) * nm);
      }
      if (!st) {
        /* Zc = Z_{-1}; Y_{-1} = T_{-1}^-1 Z_{-1} */
        coupled_Q(pw, cp, eps, a - h, q);
        if (numerov_solve(q, h, n, m, Zc, Y, T, piv)) st |= RMO_PT_SINGULAR;
        for (int i = 0; i < n && !st; ++i)
          for (int j = 0; j < m; ++j) {
            const size_t t = (size_t)i * m + j;
            phi[(size_t)i * 2 * n + j] = (double)Y0[t];
            dphi[(size_t)i * 2 * n + j] =
                (double)(((2.0L * Z1[t] - Y1[t]) - (2.0L * Zc[t] - Y[t])) / (2.0L * h));
          }
      }
    }
    free(Zp);
    free(Zc);
    free(Zn);
    free(Y);
    free(q);
    free(T);
    free(Z1);
    free(Y1);
    free(Y0);
    free(piv);
    free(Ya);
    free(dYa);
    free(Yb);
  }
done:
  if (st) {
    fill_nan(phi, 2L * n * n);
    fill_nan(dphi, 2L * n * n);
  }
  free(eps);
  free(col_ch);
  free(col_kind);
  free(cr);
  return st;
}

/* Matching, eq. (match), with the propagated solution matrices at r0 = a:    */
/*   F = S + Phi [K; X],  Phi = [closed e | open c] columns,                  */
/*   (Phi - R (a Phi' - b Phi)) [X; K] = R (a S' - b S) - S                   */
/* (with U = 0 the matrices are diagonal and this is the plain matching).     */
static int32_t solve_K_coupled_one(const rmo_pw *pw, double E, const double *R, const double *phi,
                                   const double *dphi, double *K, double *cond) {
  const int n = pw->nchan;
  const ld a = pw->a, b = pw->b;
  int *open_idx = (int *)malloc(sizeof(int) * (n + 1));
  const int no = open_list(pw, E, open_idx), nc = n - no;
  for (long t = 0; t < (long)n * n; ++t) K[t] = 0.0;
  if (cond) *cond = 0;
  if (no == 0) {
    free(open_idx);
    return 0;
  }
  ld *A = (ld *)malloc(sizeof(ld) * (size_t)n * n), *LU = (ld *)malloc(sizeof(ld) * (size_t)n * n);
  ld *B = (ld *)malloc(sizeof(ld) * (size_t)n * no);
  int *piv = (int *)malloc(sizeof(int) * n);
  const int ld2 = 2 * n;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      ld acc = 0;
      for (int t = 0; t < n; ++t)
        acc += (ld)R[(size_t)i * n + t] * (a * (ld)dphi[(size_t)t * ld2 + j] - b * (ld)phi[(size_t)t * ld2 + j]);
      A[(size_t)i * n + j] = (ld)phi[(size_t)i * ld2 + j] - acc;
    }
    for (int j = 0; j < no; ++j) {
      ld acc = 0;
      for (int t = 0; t < n; ++t)
        acc += (ld)R[(size_t)i * n + t] *
               (a * (ld)dphi[(size_t)t * ld2 + n + j] - b * (ld)phi[(size_t)t * ld2 + n + j]);
      B[(size_t)i * no + j] = acc - (ld)phi[(size_t)i * ld2 + n + j];
    }
  }
  memcpy(LU, A, sizeof(ld) * (size_t)n * n);
  int32_t st = 0;
  if (lu_factor(LU, n, piv)) {
    st = RMO_PT_SINGULAR;
  } else {
    ld *col = (ld *)malloc(sizeof(ld) * n);
    for (int j = 0; j < no; ++j) {
      for (int i = 0; i < n; ++i) col[i] = B[(size_t)i * no + j];
      lu_solve(LU, n, piv, col, 0);
      for (int i = 0; i < no; ++i) K[(size_t)i * n + j] = (double)col[nc + i];  /* rows of the c columns */
    }
    free(col);
    if (cond) *cond = (double)cond1_estimate(A, LU, n, piv);
  }
  free(A);
  free(LU);
  free(B);
  free(piv);
  free(open_idx);
  return st;
}

static int coupling_ok(const rmo_pw *pw, const rmo_coupling *cp) {
  return cp && cp->lamax >= 0 && (cp->lamax == 0 || cp->cf) && cp->npts >= 4 && cp->stab >= 1 && cp->r1 > pw->a;
}

int rmo_propagate(const rmo_pw *pw, const rmo_coupling *cp, const double *E, int32_t ne, double thr_guard,
                  double *phi, double *dphi, int8_t *open, int32_t *nopen, int32_t *status, int32_t nthreads) {
  if (!coupling_ok(pw, cp)) return -1;
  const int n = pw->nchan;
  const long per = 2L * n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e)
    status[e] = propagate_one(pw, cp, E[e], thr_guard, phi + e * per, dphi + e * per, open + (long)e * n, nopen + e);
  return 0;
}

int rmo_solve_K_coupled(const rmo_pw *pw, const double *E, int32_t ne, const double *R, const double *phi,
                        const double *dphi, double *K, double *cond, int32_t *status, int32_t nthreads) {
  const int n = pw->nchan;
  const long nn = (long)n * n, per = 2L * n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    int32_t st = 0;
    if (!all_finite(R + e * nn, nn) || !all_finite(phi + e * per, per) || !all_finite(dphi + e * per, per))
      st |= RMO_PT_NONFINITE;
    if (!st) st = solve_K_coupled_one(pw, E[e], R + e * nn, phi + e * per, dphi + e * per, K + e * nn,
                                      cond ? cond + e : NULL);
    if (st) {
      fill_nan(K + e * nn, nn);
      if (cond) cond[e] = nan_value();
    }
    status[e] = st;
  }
  return 0;
}

int rmo_run_coupled(const rmo_pw *pw, const rmo_coupling *cp, const double *E, int32_t ne, double thr_guard,
                    double *omega, double *K, double *cond, int32_t *status, int32_t nthreads) {
  if (!coupling_ok(pw, cp)) return -1;
  const int n = pw->nchan, nt = pw->ntarget;
  const long nn = (long)n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    double *R = (double *)malloc(sizeof(double) * nn);
    double *phi = (double *)malloc(sizeof(double) * 2 * nn), *dphi = (double *)malloc(sizeof(double) * 2 * nn);
    double *Kl = K ? K + e * nn : (double *)malloc(sizeof(double) * nn);
    int8_t *op = (int8_t *)malloc(n);
    int *idx = (int *)malloc(sizeof(int) * (n + 1));
    int32_t no = 0;
    int32_t st = form_R_one(pw, E[e], R);
    st |= propagate_one(pw, cp, E[e], thr_guard, phi, dphi, op, &no);
    if (!st && (!all_finite(R, nn) || !all_finite(phi, 2 * nn) || !all_finite(dphi, 2 * nn))) st |= RMO_PT_NONFINITE;
    if (!st) st = solve_K_coupled_one(pw, E[e], R, phi, dphi, Kl, cond ? cond + e : NULL);
    if (!st) {
      const int no2 = open_list(pw, E[e], idx);
      st = s_and_omega_one(pw, Kl, no2, idx, omega + (long)e * nt * nt, NULL);
    }
    if (st) {
      fill_nan(Kl, nn);
      fill_nan(omega + (long)e * nt * nt, (long)nt * nt);
      if (cond) cond[e] = nan_value();
    }
    status[e] = st;
    if (!K) free(Kl);
    free(R);
    free(phi);
    free(dphi);
    free(op);
    free(idx);
  }
  return 0;
}
