// rm_internal.h -- internal declarations of librm (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rm {

// Output tile of the R contraction and of the batched GEMMs (rows x cols).
constexpr int TILE = 64;
// Poles staged per LDS buffer in the R contraction (FP64 path; FP32 stages twice as many).
constexpr int KC64 = 32;
constexpr int KC32 = 64;
// Energies that share one staged amplitude panel in the R contraction.
constexpr int EB = 4;
// Panel width of the blocked LU.
constexpr int NB = 32;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// A partial wave resident in HBM.  Amplitudes are stored pole-major with the
// channel dimension padded to TILE and the pole dimension padded to KC32, the
// padding filled with zeros so every tile load is in bounds and contributes 0.
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
  size_t bytes = 0;
};

// Per-chunk device workspace (E_c energies of one partial wave).
struct Work {
  int cap_e = 0, cap_n = 0, cap_npad = 0, cap_M = 0, cap_nt = 0;
  size_t bytes = 0;
  double *E = nullptr;       // [cap_e]
  double *D64 = nullptr;     // [cap_e][Mpad]
  float *D32 = nullptr;      // [cap_e][Mpad]
  int *win = nullptr;        // [cap_e][2] near-pole window [lo, hi)
  int *status = nullptr;     // [cap_e]
  int *nopen = nullptr;      // [cap_e]
  int *openidx = nullptr;    // [cap_e][cap_n]
  int *openpos = nullptr;    // [cap_e][cap_n] position in the open list or -1
  int8_t *openflag = nullptr;// [cap_e][cap_n]
  double *fg = nullptr;      // [cap_e][cap_n][4]
  double *aug = nullptr;     // [cap_e][cap_n][ldaug]
  double *Kw = nullptr;      // [cap_e][ldk][ldk]
  double *XK = nullptr;      // [cap_e][ldk][ldk]
  int *dims = nullptr;       // [cap_e][2] per-energy (rows, rhs) for batched LU
  int *ipiv = nullptr;       // [cap_e][cap_n] LU row interchanges
  double *omega = nullptr;   // [cap_e][cap_nt][cap_nt]
  double *S = nullptr;       // [cap_e][cap_n][cap_n][2], allocated on demand
};

// ---- kernel launchers (all asynchronous on `s`) ----
void launch_dvec(hipStream_t s, const DevPW &pw, const double *E, int ne, int split, double delta,
                 double *D64, float *D32, int *win, int *status);
void launch_rform(hipStream_t s, const DevPW &pw, int ne, int split, const double *D64,
                  const float *D32, double *R, long ldr, long strideR);
void launch_nearpole(hipStream_t s, const DevPW &pw, const double *E, int ne, const int *win,
                     double *R, long ldr, long strideR);
void launch_nanfill_R(hipStream_t s, int ne, int n, const int *status, double *R, long ldr, long strideR);
void launch_openlist(hipStream_t s, const DevPW &pw, const double *E, int ne, int *nopen,
                     int *openidx, int *openpos, int8_t *openflag, long ld);
void launch_asym(hipStream_t s, const DevPW &pw, const double *E, int ne, double thr_guard,
                 double *fg, int *status);
void launch_build(hipStream_t s, const DevPW &pw, int ne, const double *fg, const int *nopen,
                  const int *openidx, long ldo, double *aug, long ldaug, long strideA, long roff);
// Batched LU with partial pivoting of [A | B] per energy (dims[2e] = rows of the
// square A in columns [0, rows), dims[2e+1] = right-hand sides in columns
// [roff, roff + rhs)), then back substitution: on return the right-hand-side
// columns hold A^-1 B.  Exact zero pivots set RM_PT_SINGULAR.
void launch_lu_solve(hipStream_t s, int ne, int maxrows, int maxrhs, const int *dims, double *aug,
                     long ldaug, long strideA, long roff, int *ipiv, long ldp, int *status);
// C[e] = A[e] B[e] for square no x no blocks, no = nopen[e]
void launch_gemm_sq(hipStream_t s, int ne, int maxn, const int *nopen, const double *A, long lda, long sA,
                    const double *B, long ldb, long sB, double *C, long ldc, long sC);
void launch_gatherK(hipStream_t s, int ne, int n, const int *nopen, const int *openidx, long ldo,
                    const double *aug, long ldaug, long strideA, long roff, double *Kw, long ldk,
                    long strideK);
void launch_formP(hipStream_t s, int ne, int maxno, const int *nopen, const double *Kw, long ldk,
                  long strideK, double *aug, long ldaug, long strideA, long roff, int *dims);
void launch_omega(hipStream_t s, const DevPW &pw, int ne, const int *openpos, long ldo, const int *nopen,
                  const double *X, long ldx, long sX, const double *XK, long ldxk, long sXK, double *omega,
                  double *S);
void launch_finalize(hipStream_t s, int ne, int n, int nt, int *status, double *omega, double *K, long ldk,
                     long strideK, double *S);

}  // namespace rm
