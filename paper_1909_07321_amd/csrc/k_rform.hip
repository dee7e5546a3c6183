// k_rform.hip -- boundary R-matrix, eq. (rmatrix) of the PSTGF paper:
//   R_ij(E) = 1/(2a) sum_k w_ik w_jk / (E_k - E)
// for a batch of energies, as the symmetric contraction W diag(d(E)) W^T on
// MFMA, plus the FP64 near-pole correction of the split-precision mode.
#include <algorithm>

#include "k_common.h"
#include "rm.h"
#include "rm_internal.h"

namespace rm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// d_k(E) = 1/(2a (E_k - E)).  FP64 mode stores it in FP64.  Split mode stores
// it rounded to FP32 and zero where |E_k - E| < delta (those poles are added
// back in FP64 by k_nearpole).  The predicate is evaluated on the rounded
// difference fl(E_k - E), which is monotone in E_k, so the masked poles form
// one contiguous window [lo, hi) of the ascending pole list.
// ---------------------------------------------------------------------------
__global__ void k_dvec(const DevPW *__restrict__ tab, const int *__restrict__ pwi, const double *__restrict__ E,
                       long ldD, int split, double delta, double *__restrict__ D64, float *__restrict__ D32) {
  const int e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.Mpad) return;
  const double Ev = E[e];
  double d = 0.0;
  if (k < p.M) {
    const double diff = p.Ek[k] - Ev;
    d = diff != 0.0 ? (0.5 / p.a) / diff : 0.0;  // exact pole: flagged, value unused
    if (split && fabs(diff) < delta) d = 0.0;
  }
  if (split)
    D32[(size_t)e * ldD + k] = (float)d;
  else
    D64[(size_t)e * ldD + k] = d;
}

// Window [lo, hi) of poles with |fl(E_k - E)| < delta, and the pole flag.
__global__ void k_window(const DevPW *__restrict__ tab, const int *__restrict__ pwi, const double *__restrict__ E,
                         int ne, double delta, int *__restrict__ win, int *__restrict__ status) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const DevPW &p = tab[pwi[e]];
  const double *Ek = p.Ek;
  const int M = p.M;
  const double Ev = E[e];
  // first k with fl(E_k - E) > -delta
  int lo = 0, hi = M;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Ek[mid] - Ev > -delta) hi = mid; else lo = mid + 1;
  }
  const int wlo = lo;
  lo = wlo; hi = M;
  // first k with fl(E_k - E) >= delta
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Ek[mid] - Ev >= delta) hi = mid; else lo = mid + 1;
  }
  win[2 * e] = wlo;
  win[2 * e + 1] = lo;
  // exact pole: first k with E_k >= E
  lo = 0; hi = M;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Ek[mid] >= Ev) hi = mid; else lo = mid + 1;
  }
  if (lo < M && Ek[lo] == Ev) atomicOr(status + e, RM_PT_POLE);
}

void launch_dvec(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E, int split,
                 double delta, double *D64, float *D32, int *win, int *status) {
  dim3 grid((L.Mpadmax + 255) / 256, L.ne);
  hipLaunchKernelGGL(k_dvec, grid, dim3(256), 0, s, tab, pwi, E, L.ldD, split, delta, D64, D32);
  hipLaunchKernelGGL(k_window, dim3((L.ne + 127) / 128), dim3(128), 0, s, tab, pwi, E, L.ne,
                     split ? delta : 0.0, win, status);
}

// ---------------------------------------------------------------------------
// Contraction kernel.  Every wave works on its own: a task is one lower-
// triangle RTW x RTW tile (bi, bj), bi >= bj, RTW = 16 TM, of one partial wave
// for up to EB energies of that wave.  Per stage of KW poles the wave copies
// the KW x RTW slices of W for the tile's rows i and columns j (one slice on a
// diagonal tile) into its own LDS region, then forms its TM x TM MFMA 16x16x4
// blocks per energy, scaling the A fragment by d_k(E) in registers; on a
// diagonal tile the blocks above the diagonal are skipped.  No workgroup
// barrier is involved: the next stage's slices are loaded into registers while
// the current one is multiplied, and a wave's own LDS accesses are ordered.
// MFMA operand layout (16x16x4): lane l holds A[l%16][l/16] and B[l/16][l%16];
// the result rows are given by MfmaRow.  The FP32 slices rotate odd rows by 16
// elements so that the two k-rows read by one 32-lane half fall on distinct
// banks.  The tile shapes (TM, EB) are the choices of the tile autotuner; every
// shape sums each R element over k in the same order, so they give identical
// results.
// ---------------------------------------------------------------------------
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Result element v of lane l (kk = l/16) sits in row 4*kk + v for the FP32
// 16x16x4 MFMA but in row 4*v + kk for the FP64 one; the column is l%16 in both.
template <typename T> struct MfmaRow;
template <> struct MfmaRow<float> {
  static __device__ __forceinline__ int row(int kk, int v) { return 4 * kk + v; }
};
template <> struct MfmaRow<double> {
  static __device__ __forceinline__ int row(int kk, int v) { return 4 * v + kk; }
};

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };

__device__ __forceinline__ void tri_tile(int t, int &bi, int &bj) {
  int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  bi = r;
  bj = t - r * (r + 1) / 2;
}

template <typename T> __device__ __forceinline__ const T *amplitudes(const DevPW &p);
template <> __device__ __forceinline__ const double *amplitudes<double>(const DevPW &p) { return p.W64; }
template <> __device__ __forceinline__ const float *amplitudes<float>(const DevPW &p) { return p.W32; }


// One wave's LDS region.  The FP32 kernels keep one pole's scale factors of all
// energies together (one wide LDS read per step serves every energy); the FP64
// kernels keep each energy's factors together, which measured faster there.
template <typename T, int KW, int EB, int RTW> struct WaveLds {
  static constexpr bool DT = sizeof(T) == 4;
  T a[KW][RTW];
  T b[KW][RTW];
  T d[DT ? KW : EB][DT ? EB : KW];
  __device__ __forceinline__ T &dk(int e, int k) { return DT ? d[k][e] : d[e][k]; }
};

// One task: the tile with rows [i0, i0 + RTW) and columns [j0, j0 + RTW) for
// energies [e0, e0 + me).  DIAG: i0 == j0.
template <typename T, int KW, int EB, int TM, bool DIAG>
__device__ __forceinline__ void rform_task(const T *__restrict__ W, int ldw, int Mpad, int n, int i0, int j0,
                                           const T *__restrict__ D, long ldD, int e0, int me,
                                           double *__restrict__ R, long ldr, long strideR,
                                           WaveLds<T, KW, EB, 16 * TM> &sm) {
  typedef typename Vec4<T>::type V4;
  constexpr int RTW = 16 * TM;
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, ii = lane & 15;
  constexpr int VEC = 16 / sizeof(T);            // elements per 16-byte load
  constexpr int PER_ROW = RTW / VEC;             // vectors per slice row
  constexpr int NVEC = KW * PER_ROW / 64;        // vectors per lane per slice
  constexpr int ND = (EB * KW + 63) / 64;        // scale factors per lane per stage
  constexpr int ROT = sizeof(T) == 4 ? 16 : 0;   // odd-row rotation of the FP32 slices
  static_assert(NVEC * 64 == KW * PER_ROW, "stage shape");
  typedef T TV __attribute__((ext_vector_type(VEC)));

  // fragment column of 16-block m in the slice rows (row ks + kk is rotated when kk is odd)
  int col[TM];
#pragma unroll
  for (int m = 0; m < TM; ++m) col[m] = (16 * m + ii + ROT * (kk & 1)) & (RTW - 1);

  V4 acc[EB][TM * TM];
#pragma unroll
  for (int e = 0; e < EB; ++e)
#pragma unroll
    for (int m = 0; m < TM * TM; ++m) acc[e][m] = V4{0, 0, 0, 0};

  TV ra[NVEC], rb[NVEC];
  T rd[ND];
  const GlobalPtr<TV> Wg = (GlobalPtr<TV>)W;  // ldw and the tile offsets are multiples of VEC
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < NVEC; ++r) {
      const int idx = lane + 64 * r;
      const int row = idx / PER_ROW, c = (idx % PER_ROW) * VEC;
      ra[r] = Wg[((size_t)(k0 + row) * ldw + i0 + c) / VEC];
      if (!DIAG) rb[r] = Wg[((size_t)(k0 + row) * ldw + j0 + c) / VEC];
    }
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int idx = lane + 64 * r;
      const int e = idx / KW, k = idx % KW;
      rd[r] = (idx < EB * KW && e < me) ? D[(size_t)(e0 + e) * ldD + k0 + k] : T(0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int r = 0; r < NVEC; ++r) {
      const int idx = lane + 64 * r;
      const int row = idx / PER_ROW, c = (idx % PER_ROW) * VEC;
      const int scol = (c + ROT * (row & 1)) & (RTW - 1);
      *reinterpret_cast<TV *>(&sm.a[row][scol]) = ra[r];
      if (!DIAG) *reinterpret_cast<TV *>(&sm.b[row][scol]) = rb[r];
    }
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int idx = lane + 64 * r;
      if (idx < EB * KW) sm.dk(idx / KW, idx % KW) = rd[r];
    }
  };

  const int nstage = Mpad / KW;
  gload(0);
  for (int st = 0; st < nstage; ++st) {
    sstore();
    if (st + 1 < nstage) gload((st + 1) * KW);
    // fragments of step ks + 4 are read from LDS while step ks is multiplied
    T a[TM], b[TM], d[EB];
#pragma unroll
    for (int m = 0; m < TM; ++m) {
      a[m] = sm.a[kk][col[m]];
      b[m] = DIAG ? a[m] : sm.b[kk][col[m]];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) d[e] = sm.dk(e, kk);
#pragma unroll
    for (int ks = 0; ks < KW; ks += 4) {
      T na[TM], nb[TM], nd[EB];
      if (ks + 4 < KW) {
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          na[m] = sm.a[ks + 4 + kk][col[m]];
          nb[m] = DIAG ? na[m] : sm.b[ks + 4 + kk][col[m]];
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) nd[e] = sm.dk(e, ks + 4 + kk);
      }
#pragma unroll
      for (int e = 0; e < EB; ++e)
#pragma unroll
        for (int mr = 0; mr < TM; ++mr) {
          const T x = a[mr] * d[e];
#pragma unroll
          for (int mc = 0; mc < TM; ++mc)
            if (!DIAG || mc <= mr) acc[e][mr * TM + mc] = mfma16(x, b[mc], acc[e][mr * TM + mc]);
        }
      if (ks + 4 < KW) {
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          a[m] = na[m];
          b[m] = nb[m];
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) d[e] = nd[e];
      }
    }
  }

  // epilogue: lower-triangle elements are written to (i, j) and mirrored to (j, i)
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    if (e >= me) break;
    double *Re = R + (size_t)(e0 + e) * strideR;
#pragma unroll
    for (int mr = 0; mr < TM; ++mr)
#pragma unroll
      for (int mc = 0; mc < TM; ++mc) {
        if (DIAG && mc > mr) continue;
        const int j = j0 + 16 * mc + ii;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 16 * mr + MfmaRow<T>::row(kk, v);
          if (i < n && j < n && i >= j) {
            const double val = (double)acc[e][mr * TM + mc][v];
            Re[(size_t)i * ldr + j] = val;
            Re[(size_t)j * ldr + i] = val;
          }
        }
      }
  }
}

// Persistent: every wave takes tasks from the queue of its XCD until it is
// empty, then from the other queues in turn.  Each energy's sums run over k in
// ascending order whatever wave takes the task, so results do not depend on
// scheduling.
template <typename T, int KW, int EB, int TM>
__device__ __forceinline__ void rform_wave(const DevPW *__restrict__ tab, const RTask *__restrict__ tasks,
                                           const RQueues &qs, int *__restrict__ counter, const T *__restrict__ D,
                                           long ldD, double *__restrict__ R, long ldr, long strideR,
                                           WaveLds<T, KW, EB, 16 * TM> &sm) {
  const int lane = threadIdx.x & 63;
  // start with the queue of the XCD this wave runs on (hardware register
  // XCC_ID, bits [3:0])
  int q = __builtin_amdgcn_s_getreg((3 << 11) | 20) & (NQ - 1), tried = 0;
  for (;;) {
    int task = -1;
    if (lane == 0) {
      while (tried < NQ) {
        const int len = qs.start[q + 1] - qs.start[q];
        const int idx = len > 0 ? atomicAdd(counter + q, 1) : len;
        if (idx < len) {
          task = qs.start[q] + idx;
          break;
        }
        q = (q + 1) % NQ;
        ++tried;
      }
    }
    task = __shfl(task, 0);
    if (task < 0) return;
    const RTask tk = tasks[task];
    const DevPW &p = tab[tk.slot];
    const T *__restrict__ W = amplitudes<T>(p);
    int bi, bj;
    tri_tile(tk.tile, bi, bj);
    if (bi == bj)
      rform_task<T, KW, EB, TM, true>(W, p.npad, p.Mpad, p.n, bi * 16 * TM, bj * 16 * TM, D, ldD, tk.e0, tk.m, R,
                                      ldr, strideR, sm);
    else
      rform_task<T, KW, EB, TM, false>(W, p.npad, p.Mpad, p.n, bi * 16 * TM, bj * 16 * TM, D, ldD, tk.e0, tk.m, R,
                                       ldr, strideR, sm);
  }
}

// Four independent waves per workgroup; OCC workgroups per CU (launch bound).
template <int TM, int EB, int OCC>
__global__ __launch_bounds__(256, OCC) void k_rform_f32(const DevPW *__restrict__ tab, const RTask *__restrict__ tasks,
                                                        const RQueues qs, int *__restrict__ counter,
                                                        const float *__restrict__ D, long ldD,
                                                        double *__restrict__ R, long ldr, long strideR) {
  __shared__ WaveLds<float, KW32, EB, 16 * TM> sm[4];
  rform_wave<float, KW32, EB, TM>(tab, tasks, qs, counter, D, ldD, R, ldr, strideR, sm[threadIdx.x >> 6]);
}

template <int TM, int EB, int OCC>
__global__ __launch_bounds__(256, OCC) void k_rform_f64(const DevPW *__restrict__ tab, const RTask *__restrict__ tasks,
                                                        const RQueues qs, int *__restrict__ counter,
                                                        const double *__restrict__ D, long ldD,
                                                        double *__restrict__ R, long ldr, long strideR) {
  __shared__ WaveLds<double, KW64, EB, 16 * TM> sm[4];
  rform_wave<double, KW64, EB, TM>(tab, tasks, qs, counter, D, ldD, R, ldr, strideR, sm[threadIdx.x >> 6]);
}

__global__ void k_reset(int *__restrict__ counter) {
  if (threadIdx.x < NQ) counter[threadIdx.x] = 0;
}

namespace {
typedef void (*RformF32)(const DevPW *, const RTask *, const RQueues, int *, const float *, long, double *, long,
                         long);
typedef void (*RformF64)(const DevPW *, const RTask *, const RQueues, int *, const double *, long, double *, long,
                         long);
// Kernel of each tile shape; the order is that of kRTile32 / kRTile64.
const RformF32 kF32[NRT32] = {k_rform_f32<2, 4, 3>, k_rform_f32<4, 2, 2>, k_rform_f32<1, 8, 3>};
const RformF64 kF64[NRT64] = {k_rform_f64<2, 4, 2>, k_rform_f64<1, 8, 2>};
}  // namespace

void launch_rform(hipStream_t s, const Lay &L, int split, int shape, const DevPW *tab, const RTask *tasks,
                  const RQueues &qs, int *counter, int nworkgroups, const double *D64, const float *D32,
                  double *R) {
  const int ntasks = qs.start[NQ] - qs.start[0];
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, counter);
  // persistent grid: as many workgroups as can be resident at once
  static int occ[2][NRT32 > NRT64 ? NRT32 : NRT64] = {};
  int &oc = occ[split ? 1 : 0][shape];
  if (!oc) {
    int b = 0;
    if (split)
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kF32[shape], 256, 0);
    else
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kF64[shape], 256, 0);
    oc = std::max(1, b);
  }
  const dim3 grid(std::max(1, std::min(ntasks, oc * nworkgroups)));
  if (split)
    hipLaunchKernelGGL(kF32[shape], grid, dim3(256), 0, s, tab, tasks, qs, counter, D32, L.ldD, R, L.ldaug, L.sA);
  else
    hipLaunchKernelGGL(kF64[shape], grid, dim3(256), 0, s, tab, tasks, qs, counter, D64, L.ldD, R, L.ldaug, L.sA);
}

// ---------------------------------------------------------------------------
// Near-pole correction of the split mode: R += 1/(2a) W[:, lo:hi] diag(1/(E_k - E))
// W[:, lo:hi]^T in FP64, one workgroup per (lower tile, NP_E consecutive
// energies).  The window is short (|E_k - E| < delta), so fragments are read
// straight from HBM/L2; the k loop is unrolled so that several steps' loads are
// in flight together.
// ---------------------------------------------------------------------------
constexpr int NP_E = 4;
__global__ __launch_bounds__(256) void k_nearpole(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                  const double *__restrict__ E, const int *__restrict__ win, int ne,
                                                  double *__restrict__ R, long ldr, long strideR) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  for (int q = 0; q < NP_E; ++q) {
    const int e = blockIdx.y * NP_E + q;
    if (e >= ne) return;
    const int lo = win[2 * e], hi = win[2 * e + 1];
    if (lo >= hi) continue;
    const DevPW &p = tab[pwi[e]];
    const int ntl = p.npad / TILE;
    if ((int)blockIdx.x >= ntl * (ntl + 1) / 2) continue;
    const GlobalPtr<double> W = (GlobalPtr<double>)p.W64;
    const GlobalPtr<double> Ek = (GlobalPtr<double>)p.Ek;
    const int ldw = p.npad, n = p.n;
    const double inv2a = 0.5 / p.a;
    int bi, bj;
    tri_tile(blockIdx.x, bi, bj);
    const int i0 = bi * TILE + wr * 32, j0 = bj * TILE + wc * 32;
    const double Ev = E[e];
    d4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = d4{0, 0, 0, 0};
#pragma unroll 4
    for (int k = lo; k < hi; k += 4) {
      const int kr = k + kk;
      double d = 0.0, a0 = 0, a1 = 0, b0 = 0, b1 = 0;
      if (kr < hi) {
        const double diff = Ek[kr] - Ev;
        d = diff != 0.0 ? inv2a / diff : 0.0;
        const size_t row = (size_t)kr * ldw;
        a0 = W[row + i0 + ii];
        a1 = W[row + i0 + 16 + ii];
        b0 = W[row + j0 + ii];
        b1 = W[row + j0 + 16 + ii];
      }
      const double x0 = a0 * d, x1 = a1 * d;
      acc[0] = mfma16(x0, b0, acc[0]);
      acc[1] = mfma16(x0, b1, acc[1]);
      acc[2] = mfma16(x1, b0, acc[2]);
      acc[3] = mfma16(x1, b1, acc[3]);
    }
    double *Re = R + (size_t)e * strideR;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int j = j0 + (m & 1) * 16 + ii;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + (m >> 1) * 16 + 4 * v + kk;
        if (i < n && j < n && i >= j) {
          const double val = Re[(size_t)i * ldr + j] + acc[m][v];
          Re[(size_t)i * ldr + j] = val;
          Re[(size_t)j * ldr + i] = val;
        }
      }
    }
  }
}

void launch_nearpole(hipStream_t s, const Lay &L, int maxtiles, const DevPW *tab, const int *pwi, const double *E,
                     const int *win, double *R) {
  dim3 grid(maxtiles, (L.ne + NP_E - 1) / NP_E);
  hipLaunchKernelGGL(k_nearpole, grid, dim3(256), 0, s, tab, pwi, E, win, L.ne, R, L.ldaug, L.sA);
}

__global__ void k_nanfill_R(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                            const int *__restrict__ status, double *__restrict__ R, long ldr, long strideR) {
  const int e = blockIdx.y;
  if (!(status[e] & RM_PT_POLE)) return;
  const int n = tab[pwi[e]].n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)n * n; t += (long)gridDim.x * blockDim.x)
    R[(size_t)e * strideR + (t / n) * ldr + t % n] = __builtin_nan("");
}

void launch_nanfill_R(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *status, double *R) {
  hipLaunchKernelGGL(k_nanfill_R, dim3(64, L.ne), dim3(256), 0, s, tab, pwi, status, R, L.ldaug, L.sA);
}

}  // namespace rm
