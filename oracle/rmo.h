/*
 * rmo.h -- FP64 CPU oracle for the outer-region R-matrix energy loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP library.
 *
 * Everything is computed in long double (x87 80-bit) and returned as double.
 * Physics follows the PSTGF paper (Fernandez-Menchero et al.):
 *   - R-matrix at the boundary:       section "Overview", eq. (rmatrix)
 *   - open/closed channel split:      section "Overview", text after eq. (radial)
 *   - asymptotic functions at r = a:  section "Overview" (Coulomb functions for
 *                                     open channels) and the Glossary (closed
 *                                     channels decay exponentially)
 *   - matching condition:             section "Overview", eq. (match)
 *   - T-matrix and collision strength: Glossary items "Transitions matrix" and
 *                                     "Collision strength"
 * Conventions the paper leaves open are fixed as follows (one reading each):
 *   outer equation   F'' + (eps - l(l+1)/r^2 + 2z/r) F = 0   (Rydberg units, U = 0)
 *   open channel     s = F_l(eta,ka)/sqrt(k), c = G_l(eta,ka)/sqrt(k), eta = -z/k,
 *                    primes are d/dr, so s'c - sc' = 1 (unit Wronskian in r)
 *   closed channel   direction of (W, dW/dr) for W = W_{z/kappa, l+1/2}(2 kappa r),
 *                    normalised so that e^2 + (a e')^2 = 1 and e >= 0
 *   K convention     F ~ s + c K on open channels, open channels in ascending order
 *   S                S = (1 + iK)(1 - iK)^-1, T = S - 1
 *   Omega            Omega_pq = (g/2) sum_{i in p, j in q, both open} |T_ij|^2
 */
#ifndef RMO_H
#define RMO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* per-energy status bits (same meaning as the library's) */
#define RMO_PT_POLE 1
#define RMO_PT_THRESHOLD 2
#define RMO_PT_NOCONV 4
#define RMO_PT_SINGULAR 8
#define RMO_PT_NONFINITE 16

typedef struct {
  int32_t nchan, npole, ntarget;
  double a, b, z, g;
  const double *e_thr;   /* [nchan] channel threshold energies (Ry) */
  const int32_t *l;      /* [nchan] channel angular momentum */
  const int32_t *target; /* [nchan] target index in [0, ntarget) */
  const double *Ek;      /* [npole] R-matrix poles (Ry) */
  const double *w;       /* [npole*nchan] w[k*nchan + i] = w_ik */
} rmo_pw;

/* R_ij(E) = (1/2a) sum_k w_ik w_jk / (E_k - E), full n x n per energy. */
int rmo_form_R(const rmo_pw *pw, const double *E, int32_t ne, double *R, int32_t *status,
               int32_t nthreads);

/* fg[e][i][0..3] = (s, s', c, c') for open channels, (0, 0, e, e') for closed
   ones; open[e][i] = 1/0; nopen[e] = number of open channels. */
int rmo_asymptotic(const rmo_pw *pw, const double *E, int32_t ne, double thr_guard, double *fg,
                   int8_t *open, int32_t *nopen, int32_t *status, int32_t nthreads);

/* K[e] (row stride n, leading nopen x nopen block) from R and fg; cond[e] is a
   1-norm condition estimate of the matching matrix (may be NULL). */
int rmo_solve_K(const rmo_pw *pw, const double *E, int32_t ne, const double *R, const double *fg,
                double thr_guard, double *K, double *cond, int32_t *status, int32_t nthreads);

/* Omega[e] (ntarget x ntarget) and optionally S[e] (n x n complex, interleaved
   re/im, leading nopen x nopen block) from K. */
int rmo_collision_strengths(const rmo_pw *pw, const double *E, int32_t ne, const double *K,
                            double thr_guard, double *omega, double *S, int32_t *status,
                            int32_t nthreads);

/* All stages for each energy without storing intermediate R for all energies.
   Any of K, S, cond may be NULL. */
int rmo_run(const rmo_pw *pw, const double *E, int32_t ne, double thr_guard, double *omega,
            double *K, double *S, double *cond, int32_t *status, int32_t nthreads);

/* Long-range multipole coupling of one partial wave and the Numerov grid of
   the propagation between r0 = a and r1 (section "Overview": eq. (radial) with
   U_nm; the propagation of the coupled radial functions between the boundary
   and the asymptotic radius; mzpts grid points). */
typedef struct {
  int32_t lamax;    /* multipole orders 1..lamax (0: no coupling) */
  const double *cf; /* [lamax][nchan][nchan], U_ij(r) = sum_lam cf[lam-1][i][j] r^-(lam+1) */
  double r1;        /* asymptotic radius, > a */
  int32_t npts;     /* grid points from a to r1 inclusive */
  int32_t stab;     /* Numerov steps between recombinations of the closed columns */
} rmo_coupling;

/* Solution matrices at r0 = a after propagation from r1: phi, dphi
   [ne][n][2n], columns: decaying solutions of the closed channels (ascending),
   irregular solutions of the open channels, regular solutions of the open
   channels; the rest zero.  Returns -1 for an invalid coupling. */
int rmo_propagate(const rmo_pw *pw, const rmo_coupling *cp, const double *E, int32_t ne, double thr_guard,
                  double *phi, double *dphi, int8_t *open, int32_t *nopen, int32_t *status, int32_t nthreads);
/* K from R and the propagated matrices (eq. (match)). */
int rmo_solve_K_coupled(const rmo_pw *pw, const double *E, int32_t ne, const double *R, const double *phi,
                        const double *dphi, double *K, double *cond, int32_t *status, int32_t nthreads);
/* R -> propagation -> K -> Omega for each energy. */
int rmo_run_coupled(const rmo_pw *pw, const rmo_coupling *cp, const double *E, int32_t ne, double thr_guard,
                    double *omega, double *K, double *cond, int32_t *status, int32_t nthreads);

/* Multichannel quantum-defect operation (section "Code Structure", stgf
   namelist MQDT variables iqdt = 1, imode = -1, ieq < 0, fnumin, iomsw = 1).
   A channel is a member at energy E if it is open or closed with effective
   quantum number nu = z/sqrt(e_i - E) >= max(fnumin, l_i + 0.1).
   Unphysical K over the member channels (ascending, leading nmember x nmember
   block of each n x n matrix): eq. (match) with every member treated as open,
   closed members carrying the energy-analytic Coulomb pair (f, g).  cond (may
   be NULL): 1-norm condition estimate of the matching matrix. */
int rmo_unphysical_K(const rmo_pw *pw, const double *E, int32_t ne, double fnumin, double thr_guard, double *Ku,
                     int32_t *nmember, double *cond, int32_t *status, int32_t nthreads);
/* Physical K from the unphysical one at the same energies:
   K = Ku_oo - Ku_oc (Ku_cc + tan(pi nu_c))^-1 Ku_co. */
int rmo_mqdt_eliminate(const rmo_pw *pw, const double *E, int32_t ne, double fnumin, const double *Ku,
                       const int32_t *nmember, double *K, int32_t *status, int32_t nthreads);
/* Coarse/fine operation on an ascending mesh: unphysical K at every ieq-th
   point of each run of equal member set (and the run's last point), Lagrange
   interpolation (four nearest coarse points of the run) of the unphysical S
   (iqdt = 1, through (1 - i Ku)^-1) or K (iqdt = 2) elsewhere, the
   interpolant reused within qetest z^2 (qetest, z-scaled Ry), then K and
   Omega at every point.  coarse (may be NULL) marks the coarse points.
   Returns -1 for ieq < 1, iqdt not 1 or 2, qetest < 0, z <= 0 or a mesh that
   is not ascending. */
int rmo_mqdt_run(const rmo_pw *pw, const double *E, int32_t ne, int32_t ieq, int32_t iqdt, int32_t sform,
                 double fnumin, double qetest, double thr_guard, double *omega, double *K, int8_t *coarse,
                 int32_t *status, int32_t nthreads);
/* (sform = 1, iqdt = 1: Omega from the elimination in S form,
   S = S_oo + S_oc (e^{-2 pi i nu} - S_cc)^-1 S_co of the interpolated
   unphysical S; K is not formed and left zero.) */
/* Channel functions of the unphysical K at r = a: (s, s', c, c') open,
   (f, f', g, g') closed member, (0, 0, e, e') otherwise; returns 1 for a
   member, 0 otherwise, -1 on failure. */
int rmo_mqdt_channel(double z, double eps, double a, int32_t l, double fnumin, double out[4]);
/* Special functions, exposed for pinning against independent references. */
/* F, dF/drho, G, dG/drho of the Coulomb functions F_l(eta, rho), G_l(eta, rho). */
int rmo_coulomb(double eta, double rho, int32_t l, double out[4]);
/* Closed channel: d/dr log W_{z/kappa, l+1/2}(2 kappa r) at r, kappa = sqrt(-eps). */
int rmo_closed_logderiv(double z, double eps, double r, int32_t l, double *L);
/* Channel functions at r = a: open -> (s, s', c, c'); closed -> (0, 0, e, e'). */
int rmo_channel(double z, double eps, double a, int32_t l, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
