// rm_internal.h -- internal declarations of librm (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rm {

// Output tile of the R contraction and of the batched GEMMs (rows x cols).
constexpr int TILE = 64;
// Poles one wave stages per step of the R contraction (FP64 and FP32): the same
// bytes per slice row.
constexpr int KW64 = 16;
constexpr int KW32 = 32;
// Pole-dimension padding of resident amplitudes (a multiple of both).
constexpr int MALIGN = 64;
// Energies per batch: chunks take energies from their partial waves in batches
// of EB.
constexpr int EB = 4;
// Tile shapes of the R contraction: one wave computes a 16 tm x 16 tm lower-
// triangle tile for up to eb energies of one partial wave per task.  Entry 0 is
// the default; the tile autotuner picks one entry per (precision, size bucket).
struct RTile {
  int tm, eb;
};
constexpr int NRT32 = 3, NRT64 = 2, NRTMAX = 3;
constexpr RTile kRTile32[NRT32] = {{2, 4}, {4, 2}, {1, 8}};
constexpr RTile kRTile64[NRT64] = {{2, 4}, {1, 8}};
inline RTile rtile(int split, int shape) { return split ? kRTile32[shape] : kRTile64[shape]; }
inline int nrtile(int split) { return split ? NRT32 : NRT64; }
// Size buckets of the autotuner: bucket b holds channel counts up to kBucketMaxN[b].
constexpr int NBUCKET = 4;
constexpr int kBucketMaxN[NBUCKET] = {64, 192, 512, 1 << 30};
inline int size_bucket(int n) {
  int b = 0;
  while (b + 1 < NBUCKET && n > kBucketMaxN[b]) ++b;
  return b;
}
// Panel width of the blocked LU (one register-resident panel) and the outer
// block: two panels are factored, then the trailing matrix is updated once
// with a rank-NBU product.
constexpr int NB = 32;
constexpr int NBU = 2 * NB;
// Net row permutation of one outer block's interchanges, per energy: [0] the
// number of rows outside the block that receive a row, then NBU source rows of
// the block's rows, NBU source rows of those outside rows and their NBU indices.
constexpr int BPERM = 1 + 3 * NBU;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// A partial wave resident in HBM.  Amplitudes are stored pole-major with the
// channel dimension padded to TILE and the pole dimension padded to MALIGN, the
// padding filled with zeros so every tile load is in bounds and contributes 0.
// The struct is plain data: a chunk's partial waves are copied to the device as
// a table, and every kernel reads its energy's entry through a per-energy slot
// index, so one launch can serve energies of several partial waves.
struct DevPW {
  int n = 0, M = 0, nt = 0;
  int npad = 0, Mpad = 0;
  double a = 0, b = 0, z = 0, g = 1;
  double *W64 = nullptr;  // [Mpad][npad]
  float *W32 = nullptr;   // [Mpad][npad]
  double *Ek = nullptr;   // [Mpad], padding = +1e300
  double *ethr = nullptr; // [n]
  int *l = nullptr;       // [n]
  int *target = nullptr;  // [n]
  int *tptr = nullptr;    // [nt + 1] channels of target p are tch[tptr[p] .. tptr[p+1])
  int *tch = nullptr;     // [n]
  // long-range multipole coupling (Numerov propagation between a and r1);
  // lamax = 0 for a wave without one
  int lamax = 0;
  double r1 = 0;
  double *cft = nullptr;  // [lamax][npad][npad] transposed multipole coefficients, zero padded
  double *cfm = nullptr;  // the same in MFMA-fragment order (cfm_index)
  size_t bytes = 0;
};
// Largest channel count of a partial wave with a coupling (the propagation
// keeps a 64-column panel of every solution matrix on chip).
constexpr int PROP_MAXN = 128;
// Matrices of the propagation workspace per energy: two Numerov states, the
// record 2 Z_1 - Y_1, phi and dphi.
constexpr int PROP_NMAT = 5;
// Position of A_lam[i][j] (padded, nb = npad / 64 blocks) in the fragment-major
// copy: per multipole, per (row block, column block) tile, per k-step of 4
// columns, per 32-row half (wr) and 16-row quarter (hh), one 64-lane operand
// with lane = 16 (j % 4) + i % 16, i.e. a wave's MFMA A-operand of one k-step
// is 64 consecutive doubles.
inline size_t cfm_index(int lam, int i, int j, int nb) {
  const int rb = i / 64, kb = j / 64, ir = i % 64, jc = j % 64;
  const int wr = ir / 32, hh = (ir / 16) % 2, kq = jc / 4, lane = 16 * (jc % 4) + ir % 16;
  return (((((size_t)lam * nb + rb) * nb + kb) * 16 + kq) * 2 + wr) * 128 + (size_t)hh * 64 + lane;
}

// Strides of one chunk of energies.  Every per-energy block is laid out for the
// largest partial wave in the chunk.
struct Lay {
  int ne = 0;
  int nmax = 0, npadmax = 0, Mpadmax = 0, ntmax = 0;
  long ldD = 0;                 // d(E) rows: Mpadmax
  long ldaug = 0, roff = 0, sA = 0;  // [A | B]: ldaug = 2 npadmax, B at column roff = npadmax
  long ldk = 0, sK = 0;         // K, gre and gim: ldk = npadmax, sK = nmax * ldk
  long ldo = 0;                 // per-channel arrays (fg has 4 per channel): nmax
  long sOm = 0;                 // Omega: ntmax * ntmax per energy
  int npadc = 0;                // largest npad of the chunk's coupled waves (0: none)
  int lamc = 0;                 // largest multipole order of the chunk's coupled waves
  long zrb = 0, sZ = 0;         // propagation matrices (tiled): zrb = npadc / 64 row blocks, sZ = 2 npadc^2
  // quantum-defect mode of the channel split and the asymptotic functions:
  // closed channels with nu >= max(fnumin, l + 0.1) are treated as open
  // (unphysical K); 0 for the physical path
  int mqdt = 0;
  double fnumin = 0;
};

// Internal flag of the quantum-defect mesh scan: a closed member's effective
// quantum number is within 1e-6 of an integer in sin(pi nu).
constexpr int MQDT_NEAR_INT = 1 << 30;

// Member channel of the unphysical K (stgf MQDT variables iomsw = 1, fnumin):
// open, or closed with effective quantum number nu = z / sqrt(-eps) >=
// max(fnumin, l + 0.1), i.e. eps >= -z^2 / numin^2.  Decided in double.
__host__ __device__ inline bool mqdt_member(double z, double eps, int l, double fnumin) {
  if (eps > 0) return true;
  const double numin = fnumin > l + 0.1 ? fnumin : l + 0.1;
  return eps >= -(z * z) / (numin * numin);
}

// One task of the R contraction: energies [e0, e0 + m) (m <= the tile shape's eb,
// one partial wave, table slot `slot`) times one lower-triangle tile of the shape.
struct RTask {
  int slot, e0, m, tile;
};

// The R contraction's task list is split into NQ queues, one per XCD (a
// workgroup starts with the queue of the XCD it runs on).  Queue q holds tasks [start[q],
// start[q + 1]); a queue keeps all energy batches of a tile together, so the
// workgroups of one XCD stream the same amplitude rows through its L2.
constexpr int NQ = 8;
struct RQueues {
  int start[NQ + 1];
};

// Per-chunk device workspace.
struct Work {
  int cap_e = 0, cap_n = 0, cap_npad = 0, cap_M = 0, cap_nt = 0, cap_tab = 0, cap_tasks = 0, cap_npc = 0;
  size_t bytes = 0;
  double *E = nullptr;       // [cap_e]
  int *pwi = nullptr;        // [cap_e] table slot of each energy
  DevPW *tab = nullptr;      // [cap_tab]
  RTask *tasks = nullptr;    // [cap_tasks]
  int *counter = nullptr;    // [NRTMAX][NQ] queue heads of the persistent R contraction, per tile shape
  double *D64 = nullptr;     // [cap_e][ldD]
  float *D32 = nullptr;      // [cap_e][ldD]
  int *win = nullptr;        // [cap_e][2] near-pole window [lo, hi)
  int *status = nullptr;     // [cap_e]
  int *nopen = nullptr;      // [cap_e]
  int *openidx = nullptr;    // [cap_e][ldo]
  int *openpos = nullptr;    // [cap_e][ldo] position in the open list or -1
  int *colpos = nullptr;     // [cap_e][ldo] column of each channel in the matching matrix (closed first)
  int8_t *openflag = nullptr;// [cap_e][ldo]
  double *fg = nullptr;      // [cap_e][ldo][4]
  double *aug = nullptr;     // [cap_e][nmax][ldaug]
  double *Kw = nullptr;      // [cap_e][nmax][ldk]
  double *gre = nullptr;     // [cap_e][nmax][ldk] real part of G = C^-1 (S/Omega stage)
  double *gim = nullptr;     // [cap_e][nmax][ldk] imaginary part of G
  int *dims = nullptr;       // [cap_e][2] per-energy (rows, rhs) for batched LU
  int *ipiv = nullptr;       // [cap_e][ldo] LU row interchanges
  int *bperm = nullptr;      // [cap_e][BPERM] net permutation of the current LU block
  double *linv = nullptr;    // [cap_e][NBU][NBU] inverse of the current diagonal block (LU and S/Omega)
  double *omega = nullptr;   // [cap_e][ntmax][ntmax]
  double *pack = nullptr;    // packed outputs, [cap_e][nmax][nmax] doubles
  long *pack_off = nullptr;  // [cap_e + 1] offsets of each energy's packed block
  double *S = nullptr;       // [cap_e][nmax][nmax][2], allocated on demand
  double *pz = nullptr;      // [cap_e][PROP_NMAT][sZ] propagation matrices (chunks with coupled waves)
};

// ---- kernel launchers (all asynchronous on `s`).  tab/pwi are device pointers.
void launch_dvec(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E, int split,
                 double delta, double *D64, float *D32, int *win, int *status);
// Persistent R contraction over the tasks of q (tile shape `shape` of the
// precision); ncu = compute units of the device (the grid is the number of
// workgroups that fit at once); counter: NQ ints of this shape.
void launch_rform(hipStream_t s, const Lay &L, int split, int shape, const DevPW *tab, const RTask *tasks,
                  const RQueues &q, int *counter, int ncu, const double *D64, const float *D32, double *R);
void launch_nearpole(hipStream_t s, const Lay &L, int maxtiles, const DevPW *tab, const int *pwi, const double *E,
                     const int *win, double *R);
void launch_nanfill_R(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *status, double *R);
void launch_openlist(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E, int *nopen,
                     int *openidx, int *openpos, int *colpos, int8_t *openflag);
void launch_asym(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E, double thr_guard,
                 double *fg, int *status);
// p[0 .. n) = v.
void launch_fill_int(hipStream_t s, int *p, int n, int v);
void launch_setdims(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen, int *dims);
// Assembles [A | B] in place over R; A's columns are ordered closed channels
// first, then open channels (both ascending), as colpos says.
void launch_build(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *fg,
                  const int *nopen, const int *openidx, const int *colpos, double *aug);
// Batched LU with partial pivoting of [A | B] per energy (dims[2e] = rows of the
// square A in columns [0, rows), dims[2e+1] = right-hand sides in columns
// [roff, roff + rhs)), then back substitution: on return the right-hand-side
// columns hold A^-1 B.  Exact zero pivots set RM_PT_SINGULAR.  bperm (ne * BPERM
// ints) and linv (ne * NBU * NBU doubles) are scratch.  With tail = 1 only the
// last rhs rows of the solution are formed (the back substitution stops there).
void launch_lu_solve(hipStream_t s, int ne, int maxrows, int maxrhs, const int *dims, double *aug,
                     long ldaug, long strideA, long roff, int *ipiv, long ldp, int *bperm, double *linv, int tail,
                     int *status);
// Back substitution alone: the right-hand sides of [U | Y] become U^-1 Y (U in
// the upper triangle of each block of rows).
void launch_backsub(hipStream_t s, int ne, int maxrows, int maxrhs, const int *dims, double *aug, long ldaug,
                    long strideA, long roff, int tail);
// S/Omega stage, set-up: M = 1 - i (K + K^T)/2 in aug (real part in columns [0,
// no), imaginary part at roff), G = 0 in gre/gim; dims = {no, no}.
void launch_zs_setup(hipStream_t s, const Lay &L, const int *nopen, const double *Kw, double *aug, double *gre,
                     double *gim, int *dims);
// Complex symmetric Cholesky M = C C^T (no pivoting) with G = C^-1 carried
// along, then M^-1 = G^T G over the planes of aug (both triangles).  A zero
// pivot sets RM_PT_SINGULAR.  zinv is scratch of ne * NBU * NBU doubles.
void launch_zs_inverse(hipStream_t s, const Lay &L, const int *dims, double *aug, double *gre, double *gim,
                       double *zinv, int *status);
// Numerov propagation of the coupled energies of the chunk from r1 to a (npts
// points, recombination every `stab` steps); fg holds their functions at r1.
void launch_prop(hipStream_t s, const Lay &L, int npts, int stab, const DevPW *tab, const int *pwi, const double *E,
                 const double *fg, const int *nopen, const int *openidx, const int *colpos, double *pz, int *status);
// [A | B] of the coupled energies' matching from R (in aug) and phi / dphi,
// written over their R (gre and gim serve as staging).
void launch_prop_assemble(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen,
                          const double *pz, double *aug, double *gre, double *gim);
// Row-major copy of phi (q = 3) or dphi (q = 4) of the coupled energies.
void launch_prop_gather(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen,
                        const int *status, const double *pz, int q, double *out, long ldo, long so);
// K = the last nopen rows of the solution (the open channels, ascending), as
// solved, zero past nopen; dims = {nopen, nopen}.
void launch_mqdt_count(hipStream_t s, const DevPW *pw, const double *E, int ne, double fnumin, double thr_guard,
                       int *nmem, int *flag);
void launch_mqdt_setup(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                       double thr_guard, int *syspos, int *spos, double *tanv, int *dims, int *nsys, int *status);
void launch_mqdt_build(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *syspos,
                       const int *spos, const double *tanv, const int *nopen, const int *nsys, const double *Ku,
                       const int *status, int *dims, double *aug);
void launch_mqdt_interp(hipStream_t s, const Lay &L, int mode, const DevPW *tab, const int *pwi, const int *spos,
                        const int *nsys, const double *Xc, const double *Yc, const int *cidx, const double *cw,
                        const int *status, int *dims, double *aug, double *Kw);
void launch_mqdt_take(hipStream_t s, const Lay &L, const int *nsys, const double *aug, double *Kw);
void launch_mqdt_gather(hipStream_t s, const Lay &L, const int *nsys, const int *nopen, const double *aug,
                        double *Kw, int *dims);
void launch_gatherK(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen,
                    const double *aug, double *Kw, int *dims);
void launch_omega(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *openpos,
                  const int *nopen, const double *X, const double *Y, double *omega, double *S);
void launch_finalize(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, int *status, double *omega,
                     double *K, double *S);
void launch_check_inputs(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                         double thr, const double *R, const double *fg, const double *K, const int *nopen,
                         int *status);
// sum[e][p][q] = sum over w (ascending) of om[w][e][p][q]; sst[e] = OR of st[w][e].
void launch_sum_waves(hipStream_t s, int npw, int ne, int nt, const double *om, const int32_t *st, double *sum,
                      int32_t *sst);
// Packs each energy's leading nt x nt Omega block (what = 0) or n x n K block
// (what = 1) contiguously at pack + off[e].
void launch_pack(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, int what, const double *src,
                 const long *off, double *pack);

}  // namespace rm
