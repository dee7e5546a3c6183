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
 *   propagate         eq. (radial) with the multipole coupling, Numerov from r1 to a
 *   mqdt              stgf MQDT variables: unphysical K, coarse/fine mesh
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

/* ------------------------------------------------------------------------- */
/* Multichannel quantum-defect operation (section "Code Structure", stgf      */
/* namelist, MQDT variables: iqdt = 1 treats every channel as open and works   */
/* with the unphysical K; imode = -1 solves fully on a coarse mesh and by      */
/* interpolation on the fine mesh; ieq < 0 updates the unphysical K at every   */
/* |ieq|-th mesh point; iomsw = 1 and fnumin omit closed channels whose        */
/* effective quantum number is below max(fnumin, l + 0.1)).                    */
/*                                                                            */
/* The paper names these options but leaves the functions to its references;  */
/* the reading written here:                                                  */
/*  - member channels: open (eps > 0) or closed with nu = z/kappa >=           */
/*    max(fnumin, l + 0.1); the others are eliminated exactly as in the        */
/*    physical K (decaying function).  Decided in double arithmetic.           */
/*  - a closed member channel carries the pair (f, g) of Coulomb functions     */
/*    analytic in energy: f = N A^(1/2) u, u the regular solution with         */
/*    u ~ r^(l+1) at the origin, N = (2 pi z)^(1/2) (2z)^l / (2l+1)!,          */
/*    A = prod_{p=1..l} (1 + p^2 eps / z^2); g = -e / W(f, e) + f cot(pi nu)   */
/*    with e the decaying solution and W(x, y) = x y' - x' y.  Then            */
/*    W(f, g) = -1, the decaying solution is f cos(pi nu) - g sin(pi nu), and  */
/*    (f, g) join (s, c) of the open channel smoothly at the threshold         */
/*    (s = f / (1 - exp(-2 pi z / k))^(1/2) above it).                         */
/*  - unphysical K: eq. (match) with every member channel treated as open:    */
/*    F = f + g Kun on members (s, c for open members), e X on the others.     */
/*  - fine mesh (iqdt = 1: the unphysical S is interpolated, not K, whose     */
/*    poles no polynomial follows): at the coarse points M^-1 = (1 - i Kun)^-1 */
/*    (so S = 2 M^-1 - 1); its real and imaginary parts X, Y are interpolated  */
/*    elementwise in energy (Lagrange, the four nearest coarse energies of the */
/*    same member set); the unphysical K of the fine point is Y X^-1,          */
/*    symmetrised, and                                                         */
/*    K = Kun_oo - Kun_oc (Kun_cc + tan(pi nu))^-1 Kun_co.                     */
/* ------------------------------------------------------------------------- */

/* Taylor steps of u'' = (L2/r^2 - 2z/r - eps) u outward from r0 to r1 (the   */
/* series of taylor_inward with h > 0). */
static int taylor_outward(ld z, ld eps, ld L2, ld r0, ld r1, ld *u, ld *up) {
  ld r = r0, U = *u, Up = *up;
  long steps = 0;
  enum { NT = 400 };
  ld d[NT + 3];
  while (r < r1) {
    ld kl = sqrtl(fabsl(eps + 2.0L * z / r - L2 / (r * r))) + 1e-3L;
    ld h = fminl(0.5L * r, 1.5L / kl);
    if (r + h > r1) h = r1 - r;
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
    r += h;
    if (++steps > 50000000L) return -1;
  }
  *u = U;
  *up = Up;
  return 0;
}

/* f = N A^(1/2) u and f' at r = a (eps < 0, nu > l so that A > 0).  u starts  */
/* from its power series u = r^(l+1) sum_p c_p r^p about the origin,           */
/* p (p + 2l + 1) c_p = -2z c_(p-1) - eps c_(p-2), c_0 = 1, at a small r0.     */
static int mqdt_regular(ld z, ld eps, ld a, int l, ld *f, ld *fp) {
  ld r0 = 0.25L * a;
  if (0.25L / z < r0) r0 = 0.25L / z;
  if (0.25L / sqrtl(fabsl(eps)) < r0) r0 = 0.25L / sqrtl(fabsl(eps));
  ld cm2 = 0.0L, cm1 = 1.0L, rp = 1.0L;
  ld U = 1.0L, Up = (ld)(l + 1) / r0; /* u / r0^(l+1) and u' / r0^(l+1) */
  for (int p = 1; p < 2000; ++p) {
    const ld c = (-2.0L * z * cm1 - eps * cm2) / ((ld)p * (ld)(p + 2 * l + 1));
    rp *= r0;
    const ld tu = c * rp, tp = c * (ld)(p + l + 1) * rp / r0;
    U += tu;
    Up += tp;
    cm2 = cm1;
    cm1 = c;
    if (fabsl(tu) < 1e-24L * fabsl(U) && fabsl(tp) < 1e-24L * fabsl(Up) && p > 4) break;
  }
  if (taylor_outward(z, eps, (ld)l * (l + 1), r0, a, &U, &Up)) return -1;
  ld logA = 0.0L;
  for (int p = 1; p <= l; ++p) {
    const ld t = 1.0L + (ld)p * p * eps / (z * z);
    if (t <= 0) return -1;
    logA += logl(t);
  }
  const ld pi = 3.141592653589793238462643383279502884L;
  const ld logN = 0.5L * logl(2.0L * pi * z) + (ld)l * logl(2.0L * z) - lgammal((ld)(2 * l + 2));
  const ld scale = expl(logN + 0.5L * logA + (ld)(l + 1) * logl(r0));
  *f = scale * U;
  *fp = scale * Up;
  return 0;
}

/* sin(pi x), cos(pi x) with x reduced modulo 2 first (exact) */
static void sincos_pi(ld x, ld *s, ld *c) {
  const ld pi = 3.141592653589793238462643383279502884L;
  const ld y = fmodl(x, 2.0L);
  *s = sinl(pi * y);
  *c = cosl(pi * y);
}

/* member decision in double arithmetic: open, or closed with
   nu >= max(fnumin, l + 0.1), i.e. eps >= -z^2 / numin^2 */
static int mqdt_member(double z, double eps, int l, double fnumin) {
  if (eps > 0) return 1;
  const double numin = fnumin > l + 0.1 ? fnumin : l + 0.1;
  return eps >= -(z * z) / (numin * numin);
}

/* Channel functions of the unphysical K at r = a: open -> (s, s', c, c'),
   closed member -> (f, f', g, g'), other closed -> (0, 0, e, e').  Returns
   1 for a member channel, 0 otherwise, -1 on failure. */
static int mqdt_channel_fn(ld z, double eps_d, ld a, int l, double fnumin, ld out[4]) {
  const ld eps = (ld)eps_d;
  if (eps_d > 0) return channel_fn(z, eps, a, l, out) ? -1 : 1;
  if (!mqdt_member((double)z, eps_d, l, fnumin)) return channel_fn(z, eps, a, l, out) ? -1 : 0;
  ld e, ep, f, fp;
  if (closed_uw(z, eps, a, l, &e, &ep)) return -1;
  if (mqdt_regular(z, eps, a, l, &f, &fp)) return -1;
  const ld W = f * ep - fp * e;
  ld s, c;
  sincos_pi(z / sqrtl(-eps), &s, &c);
  const ld cot = c / s;
  out[0] = f;
  out[1] = fp;
  out[2] = -e / W + f * cot;
  out[3] = -ep / W + fp * cot;
  /* at an integer nu (a bound state of the Coulomb potential) g is 0 x infinity */
  if (!isfinite((double)out[2]) || !isfinite((double)out[3])) return -1;
  return 1;
}

/* 1 if a closed member channel's effective quantum number is within 1e-6 of
   an integer in sin(pi nu), where the pair's g cancels to fewer than ten
   digits: such energies are not used as coarse points. */
static int mqdt_near_integer(const rmo_pw *pw, double E, double fnumin) {
  for (int i = 0; i < pw->nchan; ++i) {
    const double eps = E - pw->e_thr[i];
    if (eps > 0 || !mqdt_member(pw->z, eps, pw->l[i], fnumin)) continue;
    ld s, c;
    sincos_pi((ld)pw->z / sqrtl(-(ld)eps), &s, &c);
    if (fabsl(s) < 1e-6L) return 1;
  }
  return 0;
}

int rmo_mqdt_channel(double z, double eps, double a, int32_t l, double fnumin, double out[4]) {
  ld v[4];
  const int m = mqdt_channel_fn((ld)z, eps, (ld)a, l, fnumin, v);
  if (m < 0) return -1;
  for (int t = 0; t < 4; ++t) out[t] = (double)v[t];
  return m;
}

/* Member channels of energy E in ascending order; returns their count. */
static int mqdt_members(const rmo_pw *pw, double E, double fnumin, int *idx) {
  int m = 0;
  for (int i = 0; i < pw->nchan; ++i)
    if (mqdt_member(pw->z, E - pw->e_thr[i], pw->l[i], fnumin)) idx[m++] = i;
  return m;
}

static int32_t mqdt_flags(const rmo_pw *pw, double E, double thr_guard) {
  int32_t st = 0;
  for (int k = 0; k < pw->npole; ++k)
    if (pw->Ek[k] == E) st |= RMO_PT_POLE;
  for (int i = 0; i < pw->nchan; ++i)
    if (fabs(E - pw->e_thr[i]) < thr_guard) st |= RMO_PT_THRESHOLD;
  return st;
}

/* Unphysical K at one energy: Ku (row stride n), leading ns x ns block over
   the member channels in ascending order. */
static int32_t unphysical_one(const rmo_pw *pw, double E, double fnumin, double thr_guard, double *Ku,
                              int *ns_out, double *cond) {
  const int n = pw->nchan;
  const ld a = pw->a, b = pw->b;
  for (long t = 0; t < (long)n * n; ++t) Ku[t] = 0.0;
  int *mem = (int *)malloc(sizeof(int) * (n + 1));
  const int ns = mqdt_members(pw, E, fnumin, mem);
  *ns_out = ns;
  int32_t st = mqdt_flags(pw, E, thr_guard);
  double *R = (double *)malloc(sizeof(double) * (size_t)n * n);
  ld *fg = (ld *)malloc(sizeof(ld) * 4 * n);
  if (!st) st |= form_R_one(pw, E, R);
  for (int i = 0; i < n && !st; ++i)
    if (mqdt_channel_fn((ld)pw->z, E - pw->e_thr[i], a, pw->l[i], fnumin, fg + 4 * i) < 0) st |= RMO_PT_NOCONV;
  if (!st && ns > 0) {
    /* A_im = d_im C_i - R_im (a C'_m - b C_m), C = g (members) or e (others);
       B_ij = R_{i,m_j} (a f'_{m_j} - b f_{m_j}) - d_{i,m_j} f_{m_j} */
    ld *A = (ld *)malloc(sizeof(ld) * (size_t)n * n);
    ld *A0 = (ld *)malloc(sizeof(ld) * (size_t)n * n);
    ld *col = (ld *)malloc(sizeof(ld) * n);
    int *piv = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m)
        A[(size_t)i * n + m] = (i == m ? fg[4 * i + 2] : 0.0L) -
                               (ld)R[(size_t)i * n + m] * (a * fg[4 * m + 3] - b * fg[4 * m + 2]);
    memcpy(A0, A, sizeof(ld) * (size_t)n * n);
    if (lu_factor(A, n, piv)) {
      st |= RMO_PT_SINGULAR;
    } else {
      if (cond) *cond = (double)cond1_estimate(A0, A, n, piv);
      for (int j = 0; j < ns; ++j) {
        const int mj = mem[j];
        for (int i = 0; i < n; ++i)
          col[i] = (ld)R[(size_t)i * n + mj] * (a * fg[4 * mj + 1] - b * fg[4 * mj + 0]) - (i == mj ? fg[4 * mj] : 0.0L);
        lu_solve(A, n, piv, col, 0);
        for (int i = 0; i < ns; ++i) Ku[(size_t)i * n + j] = (double)col[mem[i]];
      }
    }
    free(A);
    free(A0);
    free(col);
    free(piv);
  }
  if (st) fill_nan(Ku, (long)n * n);
  free(R);
  free(fg);
  free(mem);
  return st;
}

int rmo_unphysical_K(const rmo_pw *pw, const double *E, int32_t ne, double fnumin, double thr_guard, double *Ku,
                     int32_t *nmember, double *cond, int32_t *status, int32_t nthreads) {
  const long nn = (long)pw->nchan * pw->nchan;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    int ns = 0;
    double c = 0.0;
    status[e] = unphysical_one(pw, E[e], fnumin, thr_guard, Ku + e * nn, &ns, &c);
    nmember[e] = ns;
    if (cond) cond[e] = c;
  }
  return 0;
}

/* Physical K from the unphysical one at energy E (members as in Ku):
   K = Ku_oo - Ku_oc (Ku_cc + diag tan(pi nu_c))^-1 Ku_co, open channels in
   ascending order (row stride n). */
static int32_t mqdt_eliminate(const rmo_pw *pw, double E, double fnumin, const ld *Ku, int ns, double *K) {
  const int n = pw->nchan;
  int *mem = (int *)malloc(sizeof(int) * (n + 1));
  int *oi = (int *)malloc(sizeof(int) * (n + 1)), *ci = (int *)malloc(sizeof(int) * (n + 1));
  const int m = mqdt_members(pw, E, fnumin, mem);
  int no = 0, nc = 0;
  for (int t = 0; t < m; ++t) {
    if (E - pw->e_thr[mem[t]] > 0) oi[no++] = t; /* positions within the member list */
    else ci[nc++] = t;
  }
  for (long t = 0; t < (long)n * n; ++t) K[t] = 0.0;
  int32_t st = 0;
  if (m != ns) st = RMO_PT_NOCONV;
  if (!st && no > 0) {
    ld *Mc = (ld *)malloc(sizeof(ld) * ((size_t)nc * nc + 1));
    ld *X = (ld *)malloc(sizeof(ld) * ((size_t)nc * no + 1));
    ld *col = (ld *)malloc(sizeof(ld) * (nc + 1));
    int *piv = (int *)malloc(sizeof(int) * (nc + 1));
    for (int i = 0; i < nc; ++i) {
      for (int j = 0; j < nc; ++j) Mc[(size_t)i * nc + j] = Ku[(size_t)ci[i] * n + ci[j]];
      const int ch = mem[ci[i]];
      ld s, c;
      sincos_pi((ld)pw->z / sqrtl(-((ld)E - (ld)pw->e_thr[ch])), &s, &c);
      Mc[(size_t)i * nc + i] += s / c;
    }
    if (nc > 0 && lu_factor(Mc, nc, piv)) {
      st = RMO_PT_SINGULAR;
    } else {
      for (int j = 0; j < no; ++j) {
        for (int i = 0; i < nc; ++i) col[i] = Ku[(size_t)ci[i] * n + oi[j]];
        if (nc > 0) lu_solve(Mc, nc, piv, col, 0);
        for (int i = 0; i < nc; ++i) X[(size_t)i * no + j] = col[i];
      }
      for (int i = 0; i < no; ++i)
        for (int j = 0; j < no; ++j) {
          ld v = Ku[(size_t)oi[i] * n + oi[j]];
          for (int k = 0; k < nc; ++k) v -= Ku[(size_t)oi[i] * n + ci[k]] * X[(size_t)k * no + j];
          K[(size_t)i * n + j] = (double)v;
        }
    }
    free(Mc);
    free(X);
    free(col);
    free(piv);
  }
  free(mem);
  free(oi);
  free(ci);
  return st;
}

int rmo_mqdt_eliminate(const rmo_pw *pw, const double *E, int32_t ne, double fnumin, const double *Ku,
                       const int32_t *nmember, double *K, int32_t *status, int32_t nthreads) {
  const int n = pw->nchan;
  const long nn = (long)n * n;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (ne > 1)
  for (int e = 0; e < ne; ++e) {
    ld *Kl = (ld *)malloc(sizeof(ld) * nn);
    for (long t = 0; t < nn; ++t) Kl[t] = Ku[e * nn + t];
    status[e] = mqdt_eliminate(pw, E[e], fnumin, Kl, nmember[e], K + e * nn);
    if (status[e]) fill_nan(K + e * nn, nn);
    free(Kl);
  }
  return 0;
}

/* Omega at energy E from the interpolated X + iY = (1 - i Ku)^-1 over the
   members (row stride n), eliminating the closed members in S form: with the
   unphysical S = 2(X + iY) - 1 and the decaying combination of the pair,
   S = S_oo + S_oc (e^{-2 pi i nu} - S_cc)^-1 S_co, then
   Omega_pq = (g/2) sum |S_ij - d_ij|^2 over open i in p, j in q. */
static int32_t mqdt_s_eliminate(const rmo_pw *pw, double E, double fnumin, const ld *X, const ld *Y, int ns,
                                double *omega) {
  const int n = pw->nchan, nt = pw->ntarget;
  int *mem = (int *)malloc(sizeof(int) * (n + 1));
  int *oi = (int *)malloc(sizeof(int) * (n + 1)), *ci = (int *)malloc(sizeof(int) * (n + 1));
  const int m = mqdt_members(pw, E, fnumin, mem);
  int no = 0, nc = 0;
  for (int t = 0; t < m; ++t) {
    if (E - pw->e_thr[mem[t]] > 0) oi[no++] = t;
    else ci[nc++] = t;
  }
  for (long t = 0; t < (long)nt * nt; ++t) omega[t] = 0.0;
  int32_t st = m != ns ? RMO_PT_NOCONV : 0;
  if (!st && no > 0) {
#define SU(a, b) (2.0L * (X[(size_t)(a) * n + (b)] + I * Y[(size_t)(a) * n + (b)]) - ((a) == (b) ? 1.0L : 0.0L))
    cld *C = (cld *)malloc(sizeof(cld) * ((size_t)nc * nc + 1));
    cld *Z = (cld *)malloc(sizeof(cld) * ((size_t)nc * no + 1));
    for (int k = 0; k < nc; ++k) {
      ld sn, cs;
      sincos_pi(2.0L * (ld)pw->z / sqrtl(-((ld)E - (ld)pw->e_thr[mem[ci[k]]])), &sn, &cs);
      for (int l = 0; l < nc; ++l) C[(size_t)k * nc + l] = (k == l ? cs - I * sn : 0.0L) - SU(ci[k], ci[l]);
      for (int j = 0; j < no; ++j) Z[(size_t)k * no + j] = SU(ci[k], oi[j]);
    }
    /* Gaussian elimination with partial pivoting on C, applied to Z */
    for (int c = 0; c < nc && !st; ++c) {
      int p = c;
      for (int r = c + 1; r < nc; ++r)
        if (cabsl(C[(size_t)r * nc + c]) > cabsl(C[(size_t)p * nc + c])) p = r;
      if (cabsl(C[(size_t)p * nc + c]) == 0) {
        st = RMO_PT_SINGULAR;
        break;
      }
      if (p != c) {
        for (int j = 0; j < nc; ++j) {
          const cld t = C[(size_t)c * nc + j];
          C[(size_t)c * nc + j] = C[(size_t)p * nc + j];
          C[(size_t)p * nc + j] = t;
        }
        for (int j = 0; j < no; ++j) {
          const cld t = Z[(size_t)c * no + j];
          Z[(size_t)c * no + j] = Z[(size_t)p * no + j];
          Z[(size_t)p * no + j] = t;
        }
      }
      for (int r = c + 1; r < nc; ++r) {
        const cld f = C[(size_t)r * nc + c] / C[(size_t)c * nc + c];
        for (int j = c; j < nc; ++j) C[(size_t)r * nc + j] -= f * C[(size_t)c * nc + j];
        for (int j = 0; j < no; ++j) Z[(size_t)r * no + j] -= f * Z[(size_t)c * no + j];
      }
    }
    if (!st) {
      for (int r = nc - 1; r >= 0; --r)
        for (int j = 0; j < no; ++j) {
          cld acc = Z[(size_t)r * no + j];
          for (int q = r + 1; q < nc; ++q) acc -= C[(size_t)r * nc + q] * Z[(size_t)q * no + j];
          Z[(size_t)r * no + j] = acc / C[(size_t)r * nc + r];
        }
      const ld half_g = 0.5L * (ld)pw->g;
      ld *om = (ld *)calloc((size_t)nt * nt, sizeof(ld));
      for (int i = 0; i < no; ++i)
        for (int j = 0; j < no; ++j) {
          cld Sij = SU(oi[i], oi[j]);
          for (int k = 0; k < nc; ++k) Sij += SU(oi[i], ci[k]) * Z[(size_t)k * no + j];
          const cld T = Sij - (i == j ? 1.0L : 0.0L);
          om[(size_t)pw->target[mem[oi[i]]] * nt + pw->target[mem[oi[j]]]] +=
              half_g * (creall(T) * creall(T) + cimagl(T) * cimagl(T));
        }
      for (long t = 0; t < (long)nt * nt; ++t) omega[t] = (double)om[t];
      free(om);
    }
#undef SU
    free(C);
    free(Z);
  }
  free(mem);
  free(oi);
  free(ci);
  return st;
}

/* (1 - i K)^-1 of the leading m x m block of K (row stride n) by complex
   Gauss-Jordan elimination with partial pivoting; X, Y (row stride n) get its
   real and imaginary parts.  Returns -1 for a zero pivot. */
static int mqdt_minv(const double *K, int n, int m, ld *X, ld *Y) {
  cld *A = (cld *)malloc(sizeof(cld) * ((size_t)m * m + 1));
  cld *B = (cld *)malloc(sizeof(cld) * ((size_t)m * m + 1));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      A[(size_t)i * m + j] = (i == j ? 1.0L : 0.0L) - I * (ld)K[(size_t)i * n + j];
      B[(size_t)i * m + j] = i == j ? 1.0L : 0.0L;
    }
  int bad = 0;
  for (int c = 0; c < m && !bad; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r)
      if (cabsl(A[(size_t)r * m + c]) > cabsl(A[(size_t)p * m + c])) p = r;
    if (cabsl(A[(size_t)p * m + c]) == 0) {
      bad = 1;
      break;
    }
    for (int j = 0; j < m; ++j) {
      cld t = A[(size_t)c * m + j];
      A[(size_t)c * m + j] = A[(size_t)p * m + j];
      A[(size_t)p * m + j] = t;
      t = B[(size_t)c * m + j];
      B[(size_t)c * m + j] = B[(size_t)p * m + j];
      B[(size_t)p * m + j] = t;
    }
    const cld d = A[(size_t)c * m + c];
    for (int j = 0; j < m; ++j) {
      A[(size_t)c * m + j] /= d;
      B[(size_t)c * m + j] /= d;
    }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const cld f = A[(size_t)r * m + c];
      if (f == 0) continue;
      for (int j = 0; j < m; ++j) {
        A[(size_t)r * m + j] -= f * A[(size_t)c * m + j];
        B[(size_t)r * m + j] -= f * B[(size_t)c * m + j];
      }
    }
  }
  for (int i = 0; i < m && !bad; ++i)
    for (int j = 0; j < m; ++j) {
      X[(size_t)i * n + j] = creall(B[(size_t)i * m + j]);
      Y[(size_t)i * n + j] = cimagl(B[(size_t)i * m + j]);
    }
  free(A);
  free(B);
  return bad ? -1 : 0;
}

/* Coarse/fine operation over an ascending mesh E[0..ne).  The mesh splits into
   runs with the same member set (it only grows with E).  In each run the
   coarse points are every ieq-th point from the run's first and the run's
   last point, minus points flagged at a threshold or a pole; a run with
   unflagged points but no unflagged coarse point is solved fully.  Points where
   a closed member's |sin(pi nu)| < 1e-6 are never coarse (g cancels there);
   a run left without a coarse point is flagged RMO_PT_NOCONV.  Each fine
   point takes the Lagrange interpolant of Re and Im of (1 - i Kun)^-1 through
   the four coarse points of its run around it (window start: the coarse point
   before the last coarse point at or below it, clamped to the run's coarse
   list; all of them if fewer than four), its unphysical K is Y X^-1 of the
   interpolated parts X, Y, and the closed members are eliminated (iqdt = 1;
   with iqdt = 2 the unphysical K itself is interpolated).  With qetest > 0 a
   point within qetest z^2 of the last point of its run that was evaluated at
   its own energy takes the interpolant at that energy (tan(pi nu) stays its
   own).  coarse[e] (may be NULL) is set to 1 at coarse points. */
int rmo_mqdt_run(const rmo_pw *pw, const double *E, int32_t ne, int32_t ieq, int32_t iqdt, int32_t sform,
                 double fnumin, double qetest, double thr_guard, double *omega, double *K, int8_t *coarse,
                 int32_t *status, int32_t nthreads) {
  if (ieq < 1 || pw->z <= 0 || (iqdt != 1 && iqdt != 2) || (sform && iqdt != 1) || !(qetest >= 0)) return -1;
  for (int e = 1; e < ne; ++e)
    if (!(E[e] > E[e - 1])) return -1;
  const int n = pw->nchan, nt = pw->ntarget;
  const long nn = (long)n * n;
  int *ns = (int *)malloc(sizeof(int) * (ne + 1));
  int *flag = (int *)malloc(sizeof(int) * (ne + 1));
  int *isc = (int *)calloc(ne + 1, sizeof(int));
  int *avoid = (int *)calloc(ne + 1, sizeof(int));
  int *mem = (int *)malloc(sizeof(int) * (n + 1));
  for (int e = 0; e < ne; ++e) {
    ns[e] = mqdt_members(pw, E[e], fnumin, mem);
    flag[e] = mqdt_flags(pw, E[e], thr_guard);
    avoid[e] = mqdt_near_integer(pw, E[e], fnumin);
  }
  free(mem);
  for (int s0 = 0; s0 < ne;) {
    int s1 = s0 + 1;
    while (s1 < ne && ns[s1] == ns[s0]) ++s1;
    int any = 0;
    for (int j = s0; j < s1; ++j)
      if (((j - s0) % ieq == 0 || j == s1 - 1) && !flag[j] && !avoid[j]) isc[j] = 1, any = 1;
    if (!any)
      for (int j = s0; j < s1; ++j)
        if (!flag[j] && !avoid[j]) isc[j] = 1;
    s0 = s1;
  }
  free(avoid);
  if (coarse)
    for (int e = 0; e < ne; ++e) coarse[e] = (int8_t)isc[e];
  /* energy at which each point's interpolant is evaluated (qetest): walking
     each run in order, a point within qetest z^2 of the last point evaluated
     at its own energy reuses that energy; coarse points are their own */
  double *Ev = (double *)malloc(sizeof(double) * (ne + 1));
  {
    const double tol = qetest * pw->z * pw->z;
    double last = 0.0;
    int have = 0;
    for (int e = 0; e < ne; ++e) {
      if (e == 0 || ns[e] != ns[e - 1]) have = 0;
      if (!isc[e] && have && fabs(E[e] - last) <= tol) {
        Ev[e] = last;
      } else {
        Ev[e] = E[e];
        if (!flag[e]) last = E[e], have = 1;
      }
    }
  }
  /* unphysical K at the coarse points */
  double *Kc = (double *)malloc(sizeof(double) * (size_t)ne * nn);
  ld *Xc = (ld *)calloc((size_t)ne * nn + 1, sizeof(ld)), *Yc = (ld *)calloc((size_t)ne * nn + 1, sizeof(ld));
  int32_t *stc = (int32_t *)calloc(ne + 1, sizeof(int32_t));
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < ne; ++e) {
    int m = 0;
    if (!isc[e]) continue;
    stc[e] = unphysical_one(pw, E[e], fnumin, thr_guard, Kc + e * nn, &m, NULL);
    if (!stc[e] && mqdt_minv(Kc + e * nn, n, m, Xc + e * nn, Yc + e * nn)) stc[e] = RMO_PT_SINGULAR;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int e = 0; e < ne; ++e) {
    double *Kl = K ? K + e * nn : (double *)malloc(sizeof(double) * nn);
    int32_t st = flag[e];
    if (!st) {
      /* the run of e and its coarse points */
      int s0 = e, s1 = e + 1;
      while (s0 > 0 && ns[s0 - 1] == ns[e]) --s0;
      while (s1 < ne && ns[s1] == ns[e]) ++s1;
      int *cl = (int *)malloc(sizeof(int) * (s1 - s0 + 1));
      int m = 0, k = 0;
      for (int j = s0; j < s1; ++j)
        if (isc[j]) cl[m++] = j;
      for (int q = 0; q < m; ++q)
        if (cl[q] <= e) k = q;
      if (m == 0) st |= RMO_PT_NOCONV; /* a run without a usable coarse point */
      const int w = m < 4 ? m : 4;
      int st0 = k - 1;
      if (st0 > m - w) st0 = m - w;
      if (st0 < 0) st0 = 0;
      ld *Xi = (ld *)calloc(nn, sizeof(ld)), *Yi = (ld *)calloc(nn, sizeof(ld)), *Ki = (ld *)calloc(nn, sizeof(ld));
      for (int q = st0; q < st0 + w; ++q) {
        ld wt = 1.0L;
        for (int r = st0; r < st0 + w; ++r)
          if (r != q) wt *= ((ld)Ev[e] - (ld)E[cl[r]]) / ((ld)E[cl[q]] - (ld)E[cl[r]]);
        st |= stc[cl[q]];
        for (long t = 0; t < nn; ++t) {
          Xi[t] += wt * Xc[(size_t)cl[q] * nn + t];
          Yi[t] += wt * Yc[(size_t)cl[q] * nn + t];
          Ki[t] += wt * (ld)Kc[(size_t)cl[q] * nn + t]; /* iqdt = 2 */
        }
      }
      if (!st && sform) {
        /* Omega from the S form; K is not formed */
        for (long t = 0; t < nn; ++t) Kl[t] = 0.0;
        st = mqdt_s_eliminate(pw, E[e], fnumin, Xi, Yi, ns[e], omega + (long)e * nt * nt);
        if (!st) {
          status[e] = 0;
          free(Xi);
          free(Yi);
          free(Ki);
          free(cl);
          if (!K) free(Kl);
          continue;
        }
      }
      if (!st && iqdt == 1) {
        /* Ku = Y X^-1: Z = X^-1 Y column by column, Ku = Z^T (X, Y symmetric) */
        const int m = ns[e];
        ld *LU = (ld *)malloc(sizeof(ld) * ((size_t)m * m + 1));
        ld *col = (ld *)malloc(sizeof(ld) * (m + 1));
        int *piv = (int *)malloc(sizeof(int) * (m + 1));
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < m; ++j) LU[(size_t)i * m + j] = Xi[(size_t)i * n + j];
        if (m > 0 && lu_factor(LU, m, piv)) {
          st = RMO_PT_SINGULAR;
        } else {
          for (int j = 0; j < m; ++j) {
            for (int i = 0; i < m; ++i) col[i] = Yi[(size_t)i * n + j];
            if (m > 0) lu_solve(LU, m, piv, col, 0);
            for (int i = 0; i < m; ++i) Ki[(size_t)j * n + i] = col[i];
          }
          /* symmetrised: the interpolated X, Y keep Y X^-1 symmetric only up
             to the interpolation error */
          for (int i = 0; i < m; ++i)
            for (int j = 0; j < i; ++j) {
              const ld v = 0.5L * (Ki[(size_t)i * n + j] + Ki[(size_t)j * n + i]);
              Ki[(size_t)i * n + j] = v;
              Ki[(size_t)j * n + i] = v;
            }
        }
        free(LU);
        free(col);
        free(piv);
      }
      if (!st) st = mqdt_eliminate(pw, E[e], fnumin, Ki, ns[e], Kl);
      if (!st) {
        int *idx = (int *)malloc(sizeof(int) * (n + 1));
        const int no = open_list(pw, E[e], idx);
        st = s_and_omega_one(pw, Kl, no, idx, omega + (long)e * nt * nt, NULL);
        free(idx);
      }
      free(Xi);
      free(Yi);
      free(Ki);
      free(cl);
    }
    if (st) {
      fill_nan(Kl, nn);
      fill_nan(omega + (long)e * nt * nt, (long)nt * nt);
    }
    status[e] = st;
    if (!K) free(Kl);
  }
  free(Kc);
  free(Xc);
  free(Yc);
  free(Ev);
  free(stc);
  free(ns);
  free(flag);
  free(isc);
  return 0;
}
