// k_asym.hip -- channel split and asymptotic functions at r = a, FP64.
//
// PSTGF paper, section "Overview": eps_i = E - e_i decides whether channel i is
// open (eps_i > 0) or closed; beyond the boundary the open-channel solutions
// are Coulomb functions (charged target) and the closed-channel ones decay
// exponentially (Glossary, "Closed").  With the multipole potentials dropped
// the outer equation is F'' + (eps - l(l+1)/r^2 + 2z/r) F = 0 and the functions
// are evaluated directly at r = a.
//
// Open channel (k = sqrt(eps), eta = -z/k, rho = k a): Steed's method
// (Barnett, Feng, Steed & Goldfarb, Comput. Phys. Commun. 8 (1974) 377):
//   CF1  f = F'/F from the downward ratio recurrence in L, evaluated backward;
//        the sign of F_l is the product of the signs of the denominators.
//   CF2  (G' + iF')/(G + iF) = (1 + i v_1)/rho where
//        v_n = (c_n + beta_n v_{n+1}) / (beta_n - i + v_{n+1}),
//        beta_n = rho - eta + i n,  c_n = rho^2 - 2 eta rho - l(l+1) + i rho (2n-1).
//        This is the usual CF2 with its leading term i(1 - eta/rho) cancelled
//        analytically, which keeps full precision for eta -> -infinity near
//        thresholds.  The depth is twice the count at which the plain CF2,
//        run forward with modified Lentz, stops changing, and the recursion is
//        started from the fixed point of its last map.
//   Inside the turning point rho_tp = eta + sqrt(eta^2 + l(l+1)) the CF2 value
//   is taken at rho_tp and G is carried inward with Taylor steps (it grows
//   inward there); F then follows from CF1 at rho and the Wronskian.
//
// Closed channel (kappa = sqrt(-eps), nu = z/kappa): the decaying solution is
// W_{nu,l+1/2}(2 kappa r).  CF2 continued to k = i kappa becomes the real
// recursion w_n = (b_n w_{n+1} - c_n)/(b_n - 1 + w_{n+1}),
//   b_n = kappa r - nu + n,  c_n = 2 z r - kappa^2 r^2 - l(l+1) - kappa r (2n-1),
// with W'/W = (1 - w_1)/r.  It is stable only where b_1 > 0, so it is taken at
// r_s = max(a, (nu + 2)/kappa) and (W, W') are carried inward to a with Taylor
// steps.  Output is the direction (e, e') = (W, W')/sqrt(W^2 + a^2 W'^2), e >= 0.
//
// Quantum-defect mode (stgf MQDT variables iqdt = 1, iomsw = 1, fnumin): a
// closed channel with nu >= max(fnumin, l + 0.1) is treated as open with the
// Coulomb pair analytic in energy,
//   f = N A^(1/2) u,  N = (2 pi z)^(1/2) (2z)^l / (2l+1)!,
//   A = prod_{p=1..l} (1 + p^2 eps / z^2),
//   g = -e / W(f, e) + f cot(pi nu),   W(x, y) = x y' - x' y,
// with u the regular solution normalised as r^(l+1) at the origin (its power
// series about 0 at a small r0, then Taylor steps outward to a) and e the
// decaying solution above.  W(f, g) = -1 as for (s, c); the decaying solution
// is f cos(pi nu) - g sin(pi nu), and (f, g) continue (s, c) across the
// threshold.
#include "rm.h"
#include "rm_internal.h"

namespace rm {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return cmk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return cmk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return cmk((a.re + a.im * r) / den, (a.im - a.re * r) / den);
  }
  const double r = b.re / b.im, den = b.re * r + b.im;
  return cmk((a.re * r + a.im) / den, (a.im * r - a.re) / den);
}
__device__ __forceinline__ double cabs2(cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cplx csqrt_(cplx z) {
  const double m = hypot(z.re, z.im);
  double re = sqrt(0.5 * (m + z.re));
  double im = sqrt(0.5 * fmax(m - z.re, 0.0));
  if (z.im < 0) im = -im;
  return cmk(re, im);
}

constexpr long CF_CAP = 1L << 21;

// Plain CF2 forward with modified Lentz, only to find how deep it must go.
__device__ long cf2_depth(double eta, double rho, int l) {
  const cplx ai = cmk(-l, eta), bi = cmk(l + 1, eta);
  const double tiny = 1e-300;
  cplx f = cmk(tiny, 0), C = f, D = cmk(0, 0);
  for (long k = 1; k < CF_CAP; ++k) {
    const cplx an = (ai + cmk(k - 1, 0)) * (bi + cmk(k - 1, 0));
    const cplx bn = cmk(2 * (rho - eta), 2.0 * k);
    D = bn + an * D;
    if (D.re == 0 && D.im == 0) D = cmk(tiny, 0);
    C = bn + cdiv(an, C);
    if (C.re == 0 && C.im == 0) C = cmk(tiny, 0);
    D = cdiv(cmk(1, 0), D);
    const cplx del = C * D;
    f = f * del;
    if (fabs(del.re - 1.0) + fabs(del.im) < 1e-16) return k;
  }
  return -1;
}

// (G' + iF')/(G + iF) at rho by the cancellation-free backward recursion.
__device__ bool cf2_value(double eta, double rho, int l, double &p, double &q) {
  const long kc = cf2_depth(eta, rho, l);
  if (kc < 0) return false;
  const long N = 2 * kc + 16;
  const double L2 = (double)l * (l + 1);
  const double cre = rho * rho - 2.0 * eta * rho - L2;
  const cplx cN = cmk(cre, rho * (double)(2 * N + 1));
  cplx v = cdiv(cmk(0, 1) + csqrt_(cmk(4.0 * cN.re - 1.0, 4.0 * cN.im)), cmk(2, 0));
  for (long n = N; n >= 1; --n) {
    const cplx c = cmk(cre, rho * (double)(2 * n - 1));
    const cplx beta = cmk(rho - eta, (double)n);
    v = cdiv(c + beta * v, beta - cmk(0, 1) + v);
  }
  // (1 + i v)/rho
  p = (1.0 - v.im) / rho;
  q = v.re / rho;
  return true;
}

// 1/m for the CF1 recursion (no division for its coefficients while m < INV_INT_N).
constexpr int INV_INT_N = 1024;
struct InvInts {
  double v[INV_INT_N];
  constexpr InvInts() : v() {
    for (int m = 1; m < INV_INT_N; ++m) v[m] = 1.0 / (double)m;
  }
};
__constant__ constexpr InvInts kInvInts{};

__device__ double cf1_eval(double eta, double rho, int l, int Lmax, int &sign) {
  const double irho = 1.0 / rho;
  double f = (double)(Lmax + 1) * irho;
  int sg = 1;
  for (int L = Lmax - 1; L >= l; --L) {
    const double Lp = (double)(L + 1);
    const double iLp = L + 1 < INV_INT_N ? kInvInts.v[L + 1] : 1.0 / Lp;
    const double S = Lp * irho + eta * iLp;
    const double den = S + f;
    if (den < 0) sg = -sg;
    const double ei = eta * iLp;
    f = S - (1.0 + ei * ei) / den;
  }
  sign = sg;
  return f;
}

__device__ bool cf1_value(double eta, double rho, int l, double &f, int &sign) {
  const int extra = 2 * (int)sqrt(rho * rho + 2.0 * fabs(eta) * rho) + 80;
  int s2;
  f = cf1_eval(eta, rho, l, l + extra, sign);
  const double f2 = cf1_eval(eta, rho, l, l + extra + 64, s2);
  return fabs(f - f2) <= 1e-14 * fabs(f) + 1e-300 && s2 == sign;
}

// 1/((n + 1)(n + 2)) for the Taylor recurrence below (no division per term).
constexpr int TAYLOR_MAX = 240;
struct InvPairs {
  double v[TAYLOR_MAX];
  constexpr InvPairs() : v() {
    for (int n = 0; n < TAYLOR_MAX; ++n) v[n] = 1.0 / ((double)(n + 1) * (double)(n + 2));
  }
};
__constant__ constexpr InvPairs kInvPairs{};

// Taylor steps of u'' = (L2/r^2 - 2 zz/r - ee) u from r0 inward to r1.  Terms are
// carried as d_n = c_n h^n through the four-term recurrence obtained from
// (r0 + x)^2 u'' = (L2 - 2 zz (r0 + x) - ee (r0 + x)^2) u.
__device__ bool taylor_in(double zz, double ee, double L2, double r0, double r1, double &u, double &up,
                          bool renorm) {
  double r = r0;
  long steps = 0;
  while (r > r1) {
    const double kl = sqrt(fabs(ee + 2.0 * zz / r - L2 / (r * r))) + 1e-3;
    double h = -fmin(0.4 * r, 1.2 / kl);
    if (r + h < r1) h = r1 - r;
    const double A = L2 - 2.0 * zz * r - ee * r * r;
    const double B = -(2.0 * zz + 2.0 * ee * r);
    const double C = -ee;
    const double h2 = h * h, h3 = h2 * h, h4 = h2 * h2, irr = 1.0 / (r * r);
    double dm2 = 0.0, dm1 = 0.0, d0 = u, d1 = up * h;
    double su = d0 + d1, sd = d1;
    int small = 0, nn;
    for (nn = 0; nn < TAYLOR_MAX; ++nn) {
      const double dn = ((A - (double)nn * (nn - 1)) * d0 * h2 - 2.0 * r * (double)nn * (nn + 1) * d1 * h +
                         B * dm1 * h3 + C * dm2 * h4) *
                        irr * kInvPairs.v[nn];
      su += dn;
      sd += (double)(nn + 2) * dn;
      dm2 = dm1;
      dm1 = d0;
      d0 = d1;
      d1 = dn;
      if (fabs(dn) < 1e-18 * (fabs(su) + fabs(sd))) {
        if (++small >= 3) break;
      } else {
        small = 0;
      }
    }
    if (nn >= TAYLOR_MAX) return false;
    u = su;
    up = sd / h;
    if (renorm) {
      const double sc = 1.0 / fmax(fabs(u), fabs(up));
      u *= sc;
      up *= sc;
    }
    r += h;
    if (++steps > (1L << 20)) return false;
  }
  return true;
}

// open channel: s, s', c, c' (d/dr)
__device__ bool open_fn(double z, double eps, double a, int l, double out[4]) {
  const double k = sqrt(eps), eta = -z / k, rho = k * a;
  const double L2 = (double)l * (l + 1);
  double rtp;
  if (L2 == 0.0)
    rtp = eta > 0 ? 2.0 * eta : 0.0;
  else
    rtp = eta <= 0 ? L2 / (sqrt(eta * eta + L2) - eta) : eta + sqrt(eta * eta + L2);
  const double rm = rho >= rtp ? rho : rtp;
  double p, q, fm;
  int sg;
  if (!cf2_value(eta, rm, l, p, q)) return false;
  if (!cf1_value(eta, rm, l, fm, sg)) return false;
  double F = (double)sg / sqrt((fm - p) * (fm - p) / q + q);
  double Fp = fm * F;
  double G = (fm - p) * F / q;
  double Gp = p * G - q * F;
  if (rm > rho) {
    // in rho the equation is u'' = (L2/rho^2 + 2 eta/rho - 1) u
    if (!taylor_in(-eta, 1.0, L2, rm, rho, G, Gp, false)) return false;
    double f;
    if (!cf1_value(eta, rho, l, f, sg)) return false;
    F = 1.0 / (f * G - Gp);
    Fp = f * F;
  }
  const double sk = sqrt(k);
  out[0] = F / sk;
  out[1] = Fp * sk;
  out[2] = G / sk;
  out[3] = Gp * sk;
  return true;
}

// closed channel: plain real CF (Y form) forward with Lentz for the depth
__device__ long closed_depth(double z, double kap, double r, int l) {
  const double nu = z / kap;
  const double tiny = 1e-300;
  double f = tiny, C = f, D = 0.0;
  for (long n = 1; n < CF_CAP; ++n) {
    const double an = -((double)(n - 1 - l) - nu) * ((double)(n + l) - nu);
    const double bn = 2.0 * (kap * r - nu + (double)n);
    D = bn + an * D;
    if (D == 0) D = tiny;
    C = bn + an / C;
    if (C == 0) C = tiny;
    D = 1.0 / D;
    const double del = C * D;
    f *= del;
    if (fabs(del - 1.0) < 1e-16) return n;
  }
  return -1;
}

__device__ bool closed_fn(double z, double eps, double a, int l, double out[4]) {
  const double kap = sqrt(-eps), nu = z / kap;
  const double L2 = (double)l * (l + 1);
  const double rs = fmax(a, (nu + 2.0) / kap);
  const long kc = closed_depth(z, kap, rs, l);
  if (kc < 0) return false;
  const long N = 2 * kc + 16;
  const double base = 2.0 * z * rs - kap * kap * rs * rs - L2;
  const double cN = base - kap * rs * (double)(2 * N + 1);
  const double disc = 1.0 - 4.0 * cN;
  double w = disc > 0 ? 0.5 * (1.0 + sqrt(disc)) : 0.0;
  for (long n = N; n >= 1; --n) {
    const double c = base - kap * rs * (double)(2 * n - 1);
    const double b = kap * rs - nu + (double)n;
    w = (b * w - c) / (b - 1.0 + w);
  }
  double u = 1.0, up = (1.0 - w) / rs;
  if (rs > a && !taylor_in(z, eps, L2, rs, a, u, up, true)) return false;
  double nrm = sqrt(u * u + a * a * up * up);
  if (u < 0 || (u == 0 && up < 0)) nrm = -nrm;
  out[0] = 0.0;
  out[1] = 0.0;
  out[2] = u / nrm;
  out[3] = up / nrm;
  return true;
}

// Taylor steps as in taylor_in, outward from r0 to r1; (u, u') are rescaled
// when they grow past 1e150 and the log of the scale is added to lsc.
__device__ bool taylor_out(double zz, double ee, double L2, double r0, double r1, double &u, double &up,
                           double &lsc) {
  double r = r0;
  long steps = 0;
  while (r < r1) {
    const double kl = sqrt(fabs(ee + 2.0 * zz / r - L2 / (r * r))) + 1e-3;
    double h = fmin(0.4 * r, 1.2 / kl);
    if (r + h > r1) h = r1 - r;
    const double A = L2 - 2.0 * zz * r - ee * r * r;
    const double B = -(2.0 * zz + 2.0 * ee * r);
    const double C = -ee;
    const double h2 = h * h, h3 = h2 * h, h4 = h2 * h2, irr = 1.0 / (r * r);
    double dm2 = 0.0, dm1 = 0.0, d0 = u, d1 = up * h;
    double su = d0 + d1, sd = d1;
    int small = 0, nn;
    for (nn = 0; nn < TAYLOR_MAX; ++nn) {
      const double dn = ((A - (double)nn * (nn - 1)) * d0 * h2 - 2.0 * r * (double)nn * (nn + 1) * d1 * h +
                         B * dm1 * h3 + C * dm2 * h4) *
                        irr * kInvPairs.v[nn];
      su += dn;
      sd += (double)(nn + 2) * dn;
      dm2 = dm1;
      dm1 = d0;
      d0 = d1;
      d1 = dn;
      if (fabs(dn) < 1e-18 * (fabs(su) + fabs(sd))) {
        if (++small >= 3) break;
      } else {
        small = 0;
      }
    }
    if (nn >= TAYLOR_MAX) return false;
    u = su;
    up = sd / h;
    const double big = fmax(fabs(u), fabs(up));
    if (big > 1e150) {
      u /= big;
      up /= big;
      lsc += log(big);
    }
    r += h;
    if (++steps > (1L << 20)) return false;
  }
  return true;
}

// f = N A^(1/2) u and f' at r = a for a closed member channel (nu > l, A > 0).
// u / r0^(l+1) = sum_p c_p r0^p with p (p + 2l + 1) c_p = -2z c_(p-1) - eps c_(p-2).
__device__ bool regular_fn(double z, double eps, double a, int l, double &f, double &fp) {
  const double r0 = fmin(0.5 * a, fmin(0.5 / z, 0.5 / sqrt(-eps)));
  double cm2 = 0.0, cm1 = 1.0, rp = 1.0;
  double U = 1.0, Up = (double)(l + 1) / r0;
  for (int p = 1; p < 400; ++p) {
    const double c = (-2.0 * z * cm1 - eps * cm2) / ((double)p * (double)(p + 2 * l + 1));
    rp *= r0;
    const double tu = c * rp, tp = c * (double)(p + l + 1) * rp / r0;
    U += tu;
    Up += tp;
    cm2 = cm1;
    cm1 = c;
    if (p > 4 && fabs(tu) < 1e-18 * fabs(U) && fabs(tp) < 1e-18 * fabs(Up)) break;
  }
  double lsc = 0.0;
  if (!taylor_out(z, eps, (double)l * (l + 1), r0, a, U, Up, lsc)) return false;
  double logA = 0.0;
  for (int p = 1; p <= l; ++p) logA += log1p((double)p * p * eps / (z * z));
  const double logN = 0.5 * log(2.0 * M_PI * z) + (double)l * log(2.0 * z) - lgamma((double)(2 * l + 2));
  const double sc = exp(logN + 0.5 * logA + (double)(l + 1) * log(r0) + lsc);
  f = sc * U;
  fp = sc * Up;
  return isfinite(f) && isfinite(fp) && f != 0.0;
}

// closed member channel of the unphysical K: f, f', g, g'
__device__ bool mqdt_closed_fn(double z, double eps, double a, int l, double out[4]) {
  double ed[4];
  if (!closed_fn(z, eps, a, l, ed)) return false;
  double f, fp;
  if (!regular_fn(z, eps, a, l, f, fp)) return false;
  const double e = ed[2], ep = ed[3];
  const double iw = 1.0 / (f * ep - fp * e);
  const double nu = z / sqrt(-eps);
  const double cot = cospi(nu) / sinpi(nu);
  out[0] = f;
  out[1] = fp;
  out[2] = -e * iw + f * cot;
  out[3] = -ep * iw + fp * cot;
  return isfinite(out[2]) && isfinite(out[3]);
}

__global__ void k_asym(const DevPW *__restrict__ tab, const int *__restrict__ pwi, const double *__restrict__ E,
                       long ldo, double thr_guard, int mqdt, double fnumin, double *__restrict__ fg,
                       int *__restrict__ status) {
  const int e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const double eps = E[e] - p.ethr[i];
  double out[4];
  int bad = 0;
  if (fabs(eps) < thr_guard) {
    bad = RM_PT_THRESHOLD;
  } else {
    // at the boundary a, or at r1 for a wave whose coupled functions are propagated from there
    const double r = p.lamax ? p.r1 : p.a;
    const bool ok = eps > 0                                          ? open_fn(p.z, eps, r, p.l[i], out)
                    : (mqdt && mqdt_member(p.z, eps, p.l[i], fnumin)) ? mqdt_closed_fn(p.z, eps, r, p.l[i], out)
                                                                      : closed_fn(p.z, eps, r, p.l[i], out);
    if (!ok) bad = RM_PT_NOCONV;
  }
  double *o = fg + ((size_t)e * ldo + i) * 4;
  if (bad) {
    const double nan = __builtin_nan("");
    o[0] = o[1] = o[2] = o[3] = nan;
    atomicOr(status + e, bad);
  } else {
    o[0] = out[0];
    o[1] = out[1];
    o[2] = out[2];
    o[3] = out[3];
  }
}

void launch_asym(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E, double thr_guard,
                 double *fg, int *status) {
  dim3 grid((L.nmax + 63) / 64, L.ne);
  hipLaunchKernelGGL(k_asym, grid, dim3(64), 0, s, tab, pwi, E, L.ldo, thr_guard, L.mqdt, L.fnumin, fg, status);
}

// Open-channel list per energy in ascending channel order (one workgroup per
// energy, block-wide exclusive scan of per-thread counts).
__global__ __launch_bounds__(256) void k_openlist(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                  const double *__restrict__ E, int *__restrict__ nopen,
                                                  int *__restrict__ openidx, int *__restrict__ openpos,
                                                  int *__restrict__ colpos, int8_t *__restrict__ openflag, long ld,
                                                  int mqdt, double fnumin) {
  __shared__ int cnt[256];
  const int e = blockIdx.x, t = threadIdx.x;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n;
  const double *ethr = p.ethr;
  const double Ev = E[e];
  const int per = (n + 255) / 256;
  const int c0 = t * per, c1 = min(n, c0 + per);
  int c = 0;
  // "open" here: open, or (quantum-defect mode) a closed member channel
  auto is_open = [&](int i) { return Ev - ethr[i] > 0.0 || (mqdt && mqdt_member(p.z, Ev - ethr[i], p.l[i], fnumin)); };
  for (int i = c0; i < c1; ++i) c += is_open(i);
  cnt[t] = c;
  __syncthreads();
  // Hillis-Steele inclusive scan
  for (int off = 1; off < 256; off <<= 1) {
    const int v = t >= off ? cnt[t - off] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  int pos = cnt[t] - c;
  const int nc = n - cnt[255];  // closed channels take the first columns of A
  for (int i = c0; i < c1; ++i) {
    const bool op = is_open(i);
    openflag[(size_t)e * ld + i] = op ? 1 : 0;
    openpos[(size_t)e * ld + i] = op ? pos : -1;
    colpos[(size_t)e * ld + i] = op ? nc + pos : i - pos;
    if (op) openidx[(size_t)e * ld + pos++] = i;
  }
  if (t == 255) nopen[e] = cnt[255];
}

void launch_openlist(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E, int *nopen,
                     int *openidx, int *openpos, int *colpos, int8_t *openflag) {
  hipLaunchKernelGGL(k_openlist, dim3(L.ne), dim3(256), 0, s, tab, pwi, E, nopen, openidx, openpos, colpos, openflag,
                     L.ldo, L.mqdt, L.fnumin);
}

}  // namespace rm
