/*
 * rm.h -- C ABI of librm, an MI355X (gfx950) implementation of the outer-region
 * energy loop of the R-matrix method for electron-impact excitation described in
 * "PSTGF: time-independent R-Matrix atomic electron-impact code"
 * (Fernandez-Menchero, Conroy, Ballance, Badnell, Mitnik, Gorczyca, Seaton).
 *
 * For one partial wave (the paper's "Overview" section: target thresholds e_i,
 * channel angular momenta l_i, R-matrix poles E_k and surface amplitudes w_ik)
 * and every incident energy E the library computes, on the GPU:
 *
 *   1. the boundary R-matrix, eq. (rmatrix):
 *        R_ij(E) = 1/(2a) sum_k w_ik w_jk / (E_k - E)
 *   2. the channel split eps_i = E - e_i (open iff eps_i > 0, text after
 *      eq. (radial)) and the asymptotic functions at r = a: Coulomb functions
 *      for open channels (section "Overview": the asymptotic form is a Coulomb
 *      function for a charged target) and the exponentially decaying Whittaker
 *      function for closed channels (Glossary, "Closed");
 *   3. the open-open K-matrix from the matching condition, eq. (match);
 *   4. S = (1 + iK)(1 - iK)^-1, T = S - 1 and the partial collision strengths
 *      Omega (Glossary, "Transitions matrix", "Collision strength").
 *
 * Conventions (the paper leaves them to its references; one reading each):
 *   - units: energies in Rydberg, lengths in bohr, k = sqrt(eps);
 *   - outer equation F'' + (eps - l(l+1)/r^2 + 2z/r) F = 0 with the multipole
 *     potentials dropped, so the outer solution is exactly Coulombic and the
 *     asymptotic functions are evaluated at r = a;
 *   - open channel:  s = F_l(eta,ka)/sqrt(k), c = G_l(eta,ka)/sqrt(k), eta = -z/k,
 *     primes are d/dr (unit Wronskian s'c - sc' = 1);
 *   - closed channel: the direction (e, e') of (W, dW/dr) for
 *     W = W_{z/kappa, l+1/2}(2 kappa r), kappa = sqrt(-eps), with
 *     e^2 + (a e')^2 = 1 and e >= 0 (K does not depend on this scale);
 *   - K: F ~ s + c K on open channels, open channels in ascending channel order;
 *   - Omega_pq = (g/2) sum_{i in p, j in q, both open} |T_ij|^2 with g the
 *     partial wave's statistical weight.
 *
 * Layout: row-major C arrays; every output buffer is caller-allocated with the
 * size stated at each call.  Pointers to energies and outputs are host memory
 * unless rm_opts.device_ptrs = 1, in which case they are device memory of the
 * context's GPU and the work is ordered on rm_opts.stream.  No exception crosses
 * this interface; every call returns an rm_status.
 *
 * Threading: a context may be used from one thread at a time, except that
 * rm_submit and rm_poll may be called from any single thread while the
 * context's serving worker threads run the admitted work.
 */
#ifndef RM_H
#define RM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rm_ctx rm_ctx;
typedef int32_t rm_status;

/* call status: negative = error, 0 = OK, positive = informational */
#define RM_OK 0
#define RM_PENDING 1
#define RM_E_ARG (-1)      /* bad argument (null pointer, size, layout) */
#define RM_E_NOMEM (-2)    /* host allocation (or thread start) failed or the HBM budget is exceeded */
#define RM_E_DEVICE (-3)   /* a HIP call failed; rm_last_error() has the text */
#define RM_E_NOTFOUND (-4) /* unknown partial-wave id or ticket */
#define RM_E_BUSY (-5)     /* serving admission queue full */
#define RM_E_IO (-6)       /* a file could not be opened, read, parsed or written */

/* Largest channel count of a partial wave (one matching-matrix row is staged
   on chip during assembly). */
#define RM_MAX_CHANNELS 16384

/* per-energy status bits; a flagged energy never fails its call, its outputs
   are NaN (R is NaN only for RM_PT_POLE) */
#define RM_PT_POLE 1        /* E equals a pole E_k exactly */
#define RM_PT_THRESHOLD 2   /* |E - e_i| < thr_guard for some channel */
#define RM_PT_NOCONV 4      /* an asymptotic series or continued fraction hit its cap */
#define RM_PT_SINGULAR 8    /* exact zero pivot in a factorisation */
#define RM_PT_NONFINITE 16  /* a non-finite value reached K or Omega */

typedef enum {
  RM_FP64 = 0,       /* R contraction on FP64 MFMA */
  RM_FP32_SPLIT = 1  /* FP32 MFMA with FP32 accumulation for |E_k - E| >= split_delta,
                        the remaining poles added in FP64 */
} rm_precision;

typedef struct {
  rm_precision prec;
  double split_delta; /* Ry; width of the FP64 window in RM_FP32_SPLIT (default 0.05) */
  double thr_guard;   /* Ry; energies this close to a threshold are flagged (default 1e-10) */
  void *stream;       /* hipStream_t used when device_ptrs = 1; NULL = the null stream */
  int32_t device_ptrs;/* 1: E and outputs are device pointers */
} rm_opts;

/* Fills *o with the defaults above. */
void rm_opts_default(rm_opts *o);

/* ---------------------------------------------------------------- context */
/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the device
   memory the context holds at once (resident partial waves plus workspaces);
   0 means 90% of the device's free memory.  Every HIP stream the context makes
   has the default priority: those of the direct calls (some made on first use)
   and one for each of its two serving worker threads (rm_submit). */
rm_status rm_create(int device, size_t hbm_budget_bytes, rm_ctx **out);
rm_status rm_destroy(rm_ctx *ctx);
/* Text of the last error on this context (never NULL; "" if none).  ctx =
   NULL: why the calling thread's last failed rm_create failed (the HIP call and
   HIP's text, e.g. no device), "null context" if none has failed. */
const char *rm_last_error(const rm_ctx *ctx);

/* ----------------------------------------------------------- partial waves */
/* The logical content of one partial wave's H.DAT symmetry record (PSTGF paper,
   section "Input files", H.DAT table: VALUE = Ek, WMAT = w written pole by pole,
   L2P = l, NCONAT expanded to a channel -> target map). */
typedef struct {
  int32_t nchan;        /* 1 <= n <= RM_MAX_CHANNELS channels */
  int32_t npole;        /* M >= 1 poles */
  int32_t ntarget;      /* targets; target[i] in [0, ntarget) */
  double a;             /* R-matrix box radius (bohr) */
  double b;             /* logarithmic-derivative constant of eq. (match); usually 0 */
  double z;             /* residual charge Z - N_e (>= 0) */
  double g;             /* statistical weight of the partial wave (1 for synthetic data) */
  const double *e_thr;  /* [nchan] channel threshold energies (Ry) */
  const int32_t *l;     /* [nchan] channel angular momenta, 0 <= l <= 200 */
  const int32_t *target;/* [nchan] target index of each channel */
  const double *Ek;     /* [npole] poles (Ry), ascending */
  const double *w;      /* [npole*nchan] surface amplitudes, w[k*nchan + i] = w_ik */
} rm_pw_desc;

/* Copies the partial wave to the device (host pointers; the caller keeps
   ownership).  W and E_k stay resident in HBM in the library's tile-padded
   layouts (FP64 and an FP32 copy) until rm_pw_release.  Returns RM_E_NOMEM if
   the HBM budget would be exceeded, RM_E_ARG for inconsistent sizes or unsorted
   poles. */
rm_status rm_pw_upload(rm_ctx *ctx, const rm_pw_desc *desc, int32_t *pw_id);
rm_status rm_pw_release(rm_ctx *ctx, int32_t pw_id);
/* Device bytes a partial wave of this shape occupies when resident (a wave
   uploaded with rm_pw_upload_coupled adds 16 lamax npad^2 bytes for its
   multipole coefficients, npad = nchan rounded up to 64). */
size_t rm_pw_footprint(int32_t nchan, int32_t npole);
/* Upper bound of the device workspace a chunk of ne energies of a partial wave
   of this shape needs (a chunk mixing waves needs it for its largest member);
   0 for invalid sizes.  With rm_pw_footprint this sizes hbm_budget_bytes.  A
   chunk holding a coupled wave adds 80 npad^2 bytes per energy (the five
   propagation matrices of its largest coupled wave). */
size_t rm_work_footprint(int32_t nchan, int32_t npole, int32_t ntarget, int32_t ne);

/* ------------------------------------------- long-range multipole coupling */
/* Largest channel count and multipole order of a coupled partial wave. */
#define RM_PROP_MAX_CHANNELS 128
#define RM_PROP_MAX_LAMAX 8

/* rm_pw_upload for a partial wave whose outer-region channels are coupled by
   the long-range multipole potentials (PSTGF paper, section "Overview", eq.
   (radial) with the potentials U kept, and the H.DAT CF record of the "Input
   files" table).  In Rydberg units the radial functions obey
     F'' = [diag(l(l+1)/r^2 - 2z/r - eps) + 2 U(r)] F,
     U_ij(r) = sum_{lam=1..lamax} cf[lam-1][i][j] r^-(lam+1),
   between a and the asymptotic radius r1 > a, where the uncoupled functions
   are taken as exact.  For such a wave the fused calls integrate the solution
   matrix inward from r1 to a by the Numerov method (rm_set_propagation gives
   the grid) and match it to R there; rm_asymptotic reports the functions at r1.
   cf: host [lamax][nchan][nchan] doubles (copied).  RM_E_ARG for nchan >
   RM_PROP_MAX_CHANNELS, lamax outside [1, RM_PROP_MAX_LAMAX], r1 <= a or a
   non-finite coefficient; otherwise as rm_pw_upload. */
rm_status rm_pw_upload_coupled(rm_ctx *ctx, const rm_pw_desc *desc, int32_t lamax, const double *cf, double r1,
                               int32_t *pw_id);
/* The Numerov grid of every coupled wave: npts >= 4 equally spaced points from
   a to r1 (default 3201, the paper's mzpts) and a recombination of the
   solution columns every `stab` >= 1 steps (default 64), which keeps the
   closed-channel solutions independent as they grow inward.  Applies to runs
   started after the call. */
rm_status rm_set_propagation(rm_ctx *ctx, int32_t npts, int32_t stab);
/* The propagated solution matrices of a coupled wave at r = a: phi and dphi
   [ne][n][2n] doubles, row i = channel, columns the decaying solution of every
   closed channel (channel order), then the irregular and then the regular
   solution of every open channel (channel order); columns past n + nopen are
   zero.  Each column starts at r1 as its channel's uncoupled function (value
   and derivative); the closed columns are recombined as they grow, so only
   their span is defined.  status: [ne] (RM_PT_THRESHOLD, RM_PT_NOCONV,
   RM_PT_SINGULAR), NaN rows for a failed energy.  RM_E_ARG for a wave without
   coupling. */
rm_status rm_propagate(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts,
                       double *phi, double *dphi, int32_t *status);

/* ------------------------------------------- quantum-defect operation */
/* Multichannel quantum-defect operation, section "Code Structure", stgf
   namelist, MQDT variables (iqdt = 1: every member channel treated as open,
   unphysical K; imode = -1: full solution on a coarse mesh, interpolation on
   the fine one; ieq < 0: the unphysical K updated at every |ieq|-th mesh
   point; iomsw = 1 with fnumin: closed channels with effective quantum
   number nu = z / sqrt(e_i - E) below max(fnumin, l_i + 0.1) are omitted,
   i.e. eliminated with their decaying function as in the physical K).

   Member channels at E: open, or closed with nu >= max(fnumin, l_i + 0.1).
   A closed member carries the Coulomb pair analytic in energy
     f = N A^(1/2) u,  N = (2 pi z)^(1/2) (2z)^l / (2l+1)!,
     A = prod_{p=1..l} (1 + p^2 eps / z^2),
     g = -e / W(f, e) + f cot(pi nu),
   u the regular solution with u ~ r^(l+1) at the origin, e the decaying
   solution, W(x, y) = x y' - x' y; (f, g) continue the open-channel (s, c)
   across the threshold, W(f, g) = W(s, c) = -1, and the decaying solution is
   f cos(pi nu) - g sin(pi nu), so that
     K = Ku_oo - Ku_oc (Ku_cc + tan(pi nu_c))^-1 Ku_co.
   The choice of (f, g), the member rule's decision in double arithmetic and
   the interpolation (below) are readings of the paper, which names the
   options but defers the functions to its references.  The pair loses
   accuracy where a is deep in the classically forbidden region of a member
   channel (a > 2 nu^2 / z): choose fnumin >= sqrt(z a / 2) or so.

   Only waves without a long-range coupling and with z > 0 are accepted
   (RM_E_ARG otherwise, as for fnumin < 0). */

/* Unphysical K over the member channels at each energy (eq. (match) with
   every member treated as open).  Ku: [ne][n][n], leading nmember[e] x
   nmember[e] block set (members in ascending channel order), the rest zero;
   nmember: [ne]; status: [ne] as rm_run (flagged energies: Ku NaN). */
rm_status rm_mqdt_unphysical_K(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, double fnumin,
                               const rm_opts *opts, double *Ku, int32_t *nmember, int32_t *status);

/* Coarse/fine operation on a strictly ascending mesh E[0..ne).  The mesh
   splits into runs of equal member set (the set grows with E).  In each run
   the coarse points are every ieq-th point from its first and its last
   point, leaving out points flagged at a threshold or a pole and points where
   a closed member has |sin(pi nu)| < 1e-6 (there g cancels); a run whose
   candidates all fail that has every remaining point coarse, and a run with
   none is flagged RM_PT_NOCONV.  At coarse points the unphysical K is
   computed in full and kept as X + iY = (1 - i Ku)^-1 = (1 + S_u)/2 (iqdt = 1:
   the unphysical S is interpolated, not K, which has poles where an
   eigenphase passes pi/2).  Each point takes the elementwise Lagrange
   interpolant of X and Y through the four coarse points of its run around it
   (the window starts at the coarse point before the last one at or below it,
   clamped to the run; all of them if fewer than four).  With K requested (or
   iqdt = 2, or more than 48 closed members at some point) it recovers
   Ku = Y X^-1 (a batched LU of the member count; symmetrised, as the
   interpolant keeps it symmetric only to the interpolation error; iqdt = 2
   interpolates Ku itself), eliminates its closed members as above (a second
   batched LU), and S, T and Omega follow as in rm_run.  Without K (K = NULL,
   iqdt = 1) the closed members are eliminated from the interpolated
   unphysical S_u = 2(X + iY) - 1 itself,
     S = S_u,oo + S_u,oc (e^{-2 pi i nu} - S_u,cc)^-1 S_u,co,
   and Omega follows from |S - 1|^2: no K is formed, the cost per point is
   O(n_o^2 n_c), and the two routes agree to the interpolation error.  At coarse
   points the result is the physical one (up to rounding).  Outputs as rm_run
   (omega [ne][nt][nt], K [ne][n][n] or NULL, status [ne]); coarse [ne] int8
   (may be NULL) marks the coarse points.  A point inherits the flags of the
   coarse points it is interpolated from.  ieq < 1, iqdt not 1 or 2, qetest < 0
   or a mesh that is not strictly ascending: RM_E_ARG (mq = NULL: the
   defaults).  The call allocates device temporaries (3 ncoarse n^2 doubles)
   and returns after its work is complete. */
typedef struct {
  int32_t ieq;   /* coarse step: the unphysical matrix is computed at every ieq-th point of each run (the
                    paper's |ieq| with ieq < 0); >= 1 */
  int32_t iqdt;  /* 1: interpolate the unphysical S (default); 2: interpolate the unphysical K itself
                    (one LU less per point, valid only where Ku has no pole between coarse points) */
  double fnumin; /* closed channels with nu < max(fnumin, l + 0.1) are omitted (eliminated directly) */
  double qetest; /* z-scaled Ry (E / z^2): a point within qetest of the last point of its run that was
                    evaluated at its own energy takes that point's interpolant (its tan(pi nu) stays its
                    own); 0 re-interpolates at every point */
} rm_mqdt_opts;

/* ieq = 1 (every point coarse: the direct result), iqdt = 1, fnumin = 0, qetest = 1e-7. */
void rm_mqdt_opts_default(rm_mqdt_opts *o);

rm_status rm_run_mqdt(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_mqdt_opts *mq,
                      const rm_opts *opts, double *omega, double *K, int8_t *coarse, int32_t *status);

/* ---------------------------------------------------------- staged calls */
/* Stage 1, eq. (rmatrix).  R: [ne][n][n] doubles (full symmetric matrices);
   status: [ne] int32 (RM_PT_POLE only). */
rm_status rm_form_R(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts,
                    double *R, int32_t *status);

/* Stage 2, channel split and asymptotic functions at r = a.
   fg: [ne][n][4] doubles, (s, s', c, c') for open channels and (0, 0, e, e')
   for closed ones; open: [ne][n] int8 (1 = open); nopen: [ne] int32;
   status: [ne] (RM_PT_THRESHOLD, RM_PT_NOCONV). */
rm_status rm_asymptotic(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts,
                        double *fg, int8_t *open, int32_t *nopen, int32_t *status);

/* Stage 3, eq. (match): from R [ne][n][n] and fg [ne][n][4] (as produced by the
   two calls above, or by any other source), the K-matrix K: [ne][n][n] with the
   leading nopen x nopen block filled (row stride n) and the rest zero.  K is
   returned as solved: it is symmetric up to the rounding of the solve.
   RM_E_ARG for a coupled wave (its matching needs the propagated solutions:
   use rm_run). */
rm_status rm_solve_K(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const double *R,
                     const double *fg, const rm_opts *opts, double *K, int32_t *status);

/* Stage 4, Glossary ("Transitions matrix", "Collision strength"): from K
   [ne][n][n] (leading nopen x nopen block, symmetrised as (K + K^T)/2), the
   collision strengths omega: [ne][ntarget][ntarget] and, if S != NULL,
   S = (1 + iK)(1 - iK)^-1: [ne][n][n][2] (re, im; leading nopen x nopen block).
   (1 - iK)^-1 comes from a complex symmetric factorisation of 1 - iK itself,
   so the result keeps the conditioning of 1 - iK. */
rm_status rm_collision_strengths(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne,
                                 const double *K, const rm_opts *opts, double *omega, double *S,
                                 int32_t *status);

/* All four stages fused for a block of energies: omega [ne][nt][nt]; K as in
   rm_solve_K or NULL; status [ne].  Runs the same kernels as the staged calls. */
rm_status rm_run(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts,
                 double *omega, double *K, int32_t *status);

/* --------------------------------------------------------- without allocation */
/* Bytes of the device array rm_run_noalloc works in (each GPU the library runs
   on holds one until the process ends). */
#define RM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
/* rm_run for callers that cannot allocate device memory (code under stream
   capture, tight serving loops, harnesses that forbid allocation): the same
   kernels and results as rm_run, with the whole chunk workspace carved from a
   fixed device array of RM_NOALLOC_SCRATCH_BYTES instead of allocated.  The
   call performs no hipMalloc, hipFree or other allocation (rm_create set up its
   host staging and resolved the array's address).  E, omega, K (or NULL) and
   status are device pointers (opts->device_ptrs must be 1; RM_E_ARG
   otherwise); the work is ordered on opts->stream (or the context's stream)
   and the call returns once it is queued.  Energies run in chunks as large as
   the array allows; a partial wave one energy of which needs more workspace
   than the array (about 2500 channels and up) is refused with RM_E_NOMEM and a
   message giving the bytes needed.  Calls on one context are serialised; calls
   from different contexts on one GPU share its array and race, and the array
   keeps whatever the last call left in it. */
rm_status rm_run_noalloc(rm_ctx *ctx, int32_t pw, const double *E, int32_t ne, const rm_opts *opts,
                         double *omega, double *K, int32_t *status);

/* ------------------------------------------------------------------ batching */
/* One partial wave's block of energies in a batch; outputs as in rm_run. */
typedef struct {
  int32_t pw_id;
  const double *E;   /* [ne], host or device as opts->device_ptrs says */
  int32_t ne;
  double *omega;     /* [ne][nt][nt] of this partial wave */
  double *K;         /* [ne][n][n] or NULL */
  int32_t *status;   /* [ne] */
} rm_batch_item;

/* Many partial waves of different sizes in one call.  Energies are drawn from
   every item in turn into chunks, so each chunk mixes partial waves: one
   persistent launch computes the R matrices of all of them (tasks ordered by
   cost, largest first) and the K solve and Omega run batched over the mixed
   sizes.  Results equal those of rm_run on each item alone. */
rm_status rm_run_batch(rm_ctx *ctx, const rm_batch_item *items, int32_t nitems, const rm_opts *opts);

/* Graph mode (on by default): rm_run, rm_run_batch, rm_run_sum and the
   serving workers launch each chunk's kernels as HIP graphs, one per stage
   group (asymptotics, d(E), R contraction, near-pole correction, K solve,
   S/Omega, packing of Omega, packing of K).  A group is captured from the
   stream the first time a chunk of its shape (sizes, workspace, task queues,
   options) runs on a stream and replayed while the shape repeats, so a run of
   equal chunks issues at most eight graph launches per chunk instead of
   hundreds of kernel launches.  The graphs hold kernel nodes only.  Results
   are the same in both modes.  rm_graph_stats returns how many group graphs
   were captured and replayed since the context was created. */
rm_status rm_set_graph(rm_ctx *ctx, int32_t on);
rm_status rm_graph_stats(rm_ctx *ctx, int64_t *captures, int64_t *replays);

/* Sum over partial waves of one collision problem (PSTGF paper, Glossary,
   "Collision strength", and section "Overview", the outer loop over partial
   waves: the collision strength is the sum of the partial ones):
     omega[e][p][q] = sum over w = 0 .. npw-1 of Omega^(pw_ids[w])_pq(E[e]),
   added in the order of pw_ids, so the result does not depend on scheduling.
   status[e] is the OR of the waves' status bits (a flagged wave makes the sum
   NaN).  All waves must have the same ntarget (RM_E_ARG otherwise).  order
   chooses how (wave, energy) points fill the chunks: RM_ORDER_WAVE runs the
   waves one after the other; RM_ORDER_PERMUTED gives every chunk a slice of
   consecutive energies of every wave (the permuted (J pi, E) assignment of
   section "Computational details", which spreads the slow energies).  Results
   do not depend on it.
   omega [ne][nt][nt] and status [ne] are host or device memory as
   opts->device_ptrs says; the call returns when the sum is complete. */
#define RM_ORDER_WAVE 0
#define RM_ORDER_PERMUTED 1
rm_status rm_run_sum(rm_ctx *ctx, const int32_t *pw_ids, int32_t npw, const double *E, int32_t ne, int32_t order,
                     const rm_opts *opts, double *omega, int32_t *status);

/* ------------------------------------------------------------ tile autotuner */
/* Tile shapes of the R contraction, eq. (rmatrix) (section "Overview"), formed
   in output tiles padded to multiples of 16 as in section "CUDA optimisations
   for PSTGF" (matrices padded with zeros to 32/64 boundaries).  A shape is a
   square output tile of `tile` channels per side computed for up to `energies`
   energies at once; each precision has rm_tile_count(prec) shapes (shape 0 is
   the default).  Channel counts fall into RM_NBUCKET size buckets
   (rm_tile_bucket), and a context uses one shape per (precision, bucket).
   Every shape sums each R element over the poles in the same order, so the
   choice changes the speed and never the results. */
#define RM_NBUCKET 4
/* Bucket of a channel count (0 .. RM_NBUCKET-1). */
int32_t rm_tile_bucket(int32_t nchan);
/* Number of shapes of precision prec (RM_FP64 or RM_FP32_SPLIT); 0 if prec is invalid. */
int32_t rm_tile_count(int32_t prec);
/* Tile side (channels) and energies per task of a shape.  RM_E_ARG for an
   invalid prec or shape. */
rm_status rm_tile_shape(int32_t prec, int32_t shape, int32_t *tile, int32_t *energies);
/* The shape the context uses for (prec, bucket), and setting it (takes effect
   for calls planned afterwards). */
rm_status rm_get_tile(rm_ctx *ctx, int32_t prec, int32_t bucket, int32_t *shape);
rm_status rm_set_tile(rm_ctx *ctx, int32_t prec, int32_t bucket, int32_t shape);
/* Autotuner: times the R contraction (the d(E) vector and the persistent
   contraction launch) of every shape of prec on each resident partial wave
   pw_ids[0 .. npw) for the host energies E (the first ne, at most 256 and at
   most what the HBM budget allows; reps timed runs after one warmup, the
   minimum counts), sums the times of the waves of each bucket, and makes the
   fastest shape the context's choice for every bucket that holds one of the
   waves (a shape other than shape 0 must be at least 3% faster than shape 0:
   a chunk launches the contraction once per shape it uses).  ms (NULL or
   [npw][rm_tile_count(prec)]) receives the times.
   If cache_path is not NULL the choices are also written there (JSON, one
   entry per tuned bucket, with the device architecture and compute-unit count)
   for rm_tune_load.  Synchronous; RM_E_NOTFOUND for an unknown wave, RM_E_ARG
   for bad sizes, RM_E_DEVICE if the file cannot be written. */
rm_status rm_tune(rm_ctx *ctx, int32_t prec, const int32_t *pw_ids, int32_t npw, const double *E, int32_t ne,
                  int32_t reps, const char *cache_path, double *ms);
/* Loads the choices of a cache written by rm_tune.  RM_E_NOTFOUND if the file
   cannot be read; RM_E_ARG (nothing changed) if it is malformed, names a shape
   or bucket out of range, or was made on a device of another architecture or
   compute-unit count. */
rm_status rm_tune_load(rm_ctx *ctx, const char *cache_path);

/* ------------------------------------------------------------------ serving */
typedef struct {
  int32_t pw_id;
  const double *E;   /* host; copied by rm_submit */
  int32_t ne;
  rm_opts opts;      /* device_ptrs must be 0 and stream NULL */
  double *omega;     /* host [ne][nt][nt]; must stay valid until rm_poll returns RM_OK */
  double *K;         /* host [ne][n][n] or NULL */
  int32_t *status;   /* host [ne] */
} rm_request;

typedef struct {
  int64_t t_arrive_ns, t_admit_ns, t_start_ns, t_done_ns; /* CLOCK_MONOTONIC */
  int32_t nblocks;   /* energy chunks the request was split into */
} rm_req_stats;

/* Non-blocking: copies E, queues the request and returns a ticket.  The
   scheduler admits (partial wave, energy chunk) items while the HBM budget and
   the in-flight slots allow, so requests that arrive while others run are
   interleaved with them on the device.  RM_E_BUSY if the queue is full. */
rm_status rm_submit(rm_ctx *ctx, const rm_request *req, uint64_t *ticket);
/* RM_OK (done; outputs written, ticket retired), RM_PENDING, or the error of
   one of the request's chunks (ticket retired): RM_E_NOMEM when one energy's
   workspace exceeds the HBM budget or a host allocation in the worker failed,
   RM_E_NOTFOUND when its partial wave was released, RM_E_DEVICE when a HIP call
   failed.  The outputs of a failed chunk's energies are not valid.  st may be
   NULL. */
rm_status rm_poll(rm_ctx *ctx, uint64_t ticket, rm_req_stats *st);
/* Blocks until every submitted request is done. */
rm_status rm_drain(rm_ctx *ctx);

/* ---------------------------------------------------------------- profiling */
/* Stage timing: while enabled, every launch of the named stage is bracketed by
   HIP events on the stream it runs on.  Stages: "rform" (R contraction kernel,
   either precision), "nearpole" (FP64 window correction), "asym" (channel split
   and asymptotic functions), "ksolve" (matching assembly, LU, back
   substitution), "somega" (S, T and Omega), "chunk" (one chunk's whole
   pipeline).  rm_prof_read synchronises the recorded events and returns the
   summed milliseconds, the launch count and the energies those launches
   covered, then clears the records of that stage. */
rm_status rm_prof_enable(rm_ctx *ctx, int32_t on);
rm_status rm_prof_read(rm_ctx *ctx, const char *stage, double *total_ms, int64_t *launches,
                       int64_t *energies);
/* Per-chunk records, in issue order (the single-GPU view of the load balance
   of section "Computational details": how evenly the work of the (partial
   wave, energy) points is spread over the launches).  Up to cap records are
   returned and cleared: GPU milliseconds of the chunk's pipeline, its model
   flops (per energy n(n+1)M + (2/3)n^3 + n^2 n_o + 4 n_o^3), the mean open
   fraction n_o/n of its energies and its energy count; *count = records
   returned. */
rm_status rm_prof_chunks(rm_ctx *ctx, int64_t cap, double *ms, double *model_flops, double *open_frac,
                         int64_t *energies, int64_t *count);

/* ------------------------------------------------------------ file boundary */
/* Readers of the inner-region output and the writer of the results, for the
   layouts of the paper's section "Input files" (H.DAT, sizeH.dat) and section
   "Output files" (OMEGA).  Host code; no device is used.  Errors return
   RM_E_IO (rm_hdat_error has the text) or RM_E_ARG for bad arguments. */

/* H.DAT / H.DAT000 target records: NELC, NZ, LRANG2, LAMAX, NAST, RA, BSTO. */
typedef struct {
  int32_t nelc, nz, lrang2, lamax, nast;
  double ra, bsto;
} rm_hdat_target;
/* Symmetry record 1: LRGL2 (L or 2J), NSPN2 (2S+1, or 0 in J coupling),
   NPTY2 (parity), NCHAN, MNP2 (poles), MORE2. */
typedef struct {
  int32_t lrgl2, nspn2, npty2, nchan, mnp2, more2;
} rm_hdat_sym;
typedef struct rm_hdat rm_hdat;

/* Opens an H.DAT or H.DAT000 file (Fortran unformatted sequential, either byte
   order) and reads its target records (ENAT, LAT, ISAT, COEFF and the Buttle
   records); the symmetries follow with rm_hdat_next.  *out is set (and must be
   closed) even on error, so that rm_hdat_error can be read. */
rm_status rm_hdat_open(const char *path, rm_hdat **out);
/* Frees the handle; h = NULL is a no-op (RM_OK).  The other rm_hdat_* calls,
   rm_sizeh_read and rm_omega_write return RM_E_ARG for a NULL handle, path or
   required output. */
rm_status rm_hdat_close(rm_hdat *h);
const char *rm_hdat_error(const rm_hdat *h);
/* Target records; enat [nast] (Ry), lat [nast] (L or 2J), isat [nast] (2S+1
   or 0) may be NULL. */
rm_status rm_hdat_target_info(const rm_hdat *h, rm_hdat_target *t, double *enat, int32_t *lat, int32_t *isat);
/* Continues with the symmetries of another file of the same run (H.DATXXX,
   XXX != 000: symmetry records only). */
rm_status rm_hdat_attach(rm_hdat *h, const char *path);
/* Reads the next symmetry (records NCONAT, L2P, CF, VALUE, WMAT) into the
   handle; RM_E_NOTFOUND after the last one. */
rm_status rm_hdat_next(rm_hdat *h, rm_hdat_sym *sym);
/* Copies the current symmetry's arrays (any may be NULL): nconat [nast]
   channels per target, l2p [nchan], cf [lamax][nchan][nchan] multipole
   coefficients (CF(I,N,M) with I fastest, M = multipole order), value [mnp2]
   poles, wmat [mnp2][nchan] amplitudes (pole-major, as rm_pw_desc.w). */
rm_status rm_hdat_arrays(const rm_hdat *h, int32_t *nconat, int32_t *l2p, double *cf, double *value, double *wmat);
/* A descriptor of the current symmetry for rm_pw_upload, pointing into the
   handle (valid until the next rm_hdat_next or rm_hdat_close): channels
   ordered by target as NCONAT says, channel threshold = ENAT(target) -
   ENAT(1), l = L2P, a = RA, b = BSTO, z = NZ - NELC, g = (2S+1)(2L+1) or
   2J+1. */
rm_status rm_hdat_pw_desc(const rm_hdat *h, rm_pw_desc *desc);

/* sizeH.dat (kind 0: NCHAN, NCON, MNP2, 2S+1, L, parity) or sizeBP.dat (kind 1:
   NCHAN, NCON, MNP2, 2J, parity; s = 0), one row per partial wave, read with
   the fixed columns of their Fortran formats.  Up to cap rows are stored;
   *count is the number of rows in the file.  A field that is not an integer,
   or a line longer than 1023 characters: RM_E_IO, *count the rows before it. */
typedef struct {
  int32_t nchan, ncon, mnp2, s, l, ipi;
} rm_sizeh_row;
rm_status rm_sizeh_read(const char *path, int32_t kind, int32_t cap, rm_sizeh_row *rows, int32_t *count);

/* OMEGA (formatted = 1, one record per line) or OMEGAU (formatted = 0,
   Fortran unformatted sequential records): NZ NEL; NLEV MXE NOMWRT; (S(I) L(I),
   I = 1..NLEV); ELEV; then per energy E(J) and the collision strengths of the
   stored transitions.  omega [ne][nlev][nlev] (e.g. Omega summed over partial
   waves); the transitions are the upper triangle (with the diagonal if elastic
   = 1), row-wise for nomwrt > 0 and column-wise for nomwrt < 0, the first
   |nomwrt| of them (the written NOMWRT is the count stored, with the sign).
   E and elev are divided by z^2 (z = NZ - NEL) for an ion, as the file holds
   z-scaled Rydberg energies. */
rm_status rm_omega_write(const char *path, int32_t formatted, int32_t nz, int32_t nel, int32_t nlev,
                         const int32_t *S, const int32_t *L, const double *elev, int32_t ne, const double *E,
                         const double *omega, int32_t nomwrt, int32_t elastic);

#ifdef __cplusplus
}
#endif
#endif /* RM_H */
