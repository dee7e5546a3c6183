// k_linalg.hip -- matching, K solve and S/Omega, FP64 on the GPU.
//
// Matching (PSTGF paper, eq. (match)): with the asymptotic form F_ij = s_i d_ij +
// c_i K_ij on open rows and e_i X_ij on closed rows, F(a) = R (a F'(a) - b F(a))
// becomes A Y = B with C_i = c_i (open) or e_i (closed) and
//   A_im = d_im C_i - R_im (a C'_m - b C_m)
//   B_ij = R_{i,o_j} (a s'_{o_j} - b s_{o_j}) - d_{i,o_j} s_{o_j}
// and K = Y restricted to the open rows.  The unknowns (columns of A, rows of
// Y) are ordered closed channels first, then open ones, so K is the last nopen
// rows of Y and the back substitution can stop there.  A Y = B is solved by a
// batched, blocked, right-looking LU with partial pivoting applied to [A | B]
// followed by a blocked back substitution.
//
// S and Omega (Glossary): S = (1 + iK)(1 - iK)^-1 = 2 M^-1 - 1 with M = 1 - iK,
// formed from a complex symmetric Cholesky factorisation of M (section "S and
// Omega from K" below):
//   T = S - 1 = 2 (M^-1 - 1),  |T_ij|^2 = 4 |(M^-1)_ij - d_ij|^2
//   Omega_pq = (g/2) sum_{i in p, j in q, both open} |T_ij|^2
//
// Augmented layout per energy: rows [0, rows), A in columns [0, rows), the
// right-hand sides in columns [roff, roff + rhs), row stride ldaug.
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "k_common.h"
#include "rm.h"
#include "rm_internal.h"

namespace rm {

// ---------------------------------------------------------------------------
// Assembly of [A | B] in place over R, one workgroup per (row, energy): the row
// of R is staged in LDS, then B's row (open columns of R) and A's row (every
// column, moved to the channel's column in A) are written.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_build(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                               const double *__restrict__ fg, const int *__restrict__ nopen,
                                               const int *__restrict__ openidx, const int *__restrict__ colpos,
                                               long ldo, double *__restrict__ aug, long ldaug, long strideA,
                                               long roff) {
  extern __shared__ double rrow[];
  const int i = blockIdx.x, e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n;
  if (i >= n || p.lamax) return;  // coupled waves: assembled from the propagated solutions
  const double a = p.a, b = p.b;
  double *row = aug + (size_t)e * strideA + (size_t)i * ldaug;
  const double *f = fg + (size_t)e * ldo * 4;
  for (int m = threadIdx.x; m < n; m += 256) rrow[m] = row[m];
  __syncthreads();
  const int no = nopen[e];
  const int *oi = openidx + (size_t)e * ldo;
  for (int j = threadIdx.x; j < no; j += 256) {
    const int oj = oi[j];
    const double s = f[4 * oj], sp = f[4 * oj + 1];
    row[roff + j] = rrow[oj] * (a * sp - b * s) - (i == oj ? s : 0.0);
  }
  const int *cp = colpos + (size_t)e * ldo;
  for (int m = threadIdx.x; m < n; m += 256) {
    const double lam = a * f[4 * m + 3] - b * f[4 * m + 2];
    double v = -rrow[m] * lam;
    if (i == m) v += f[4 * m + 2];
    row[cp[m]] = v;
  }
}

void launch_build(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *fg,
                  const int *nopen, const int *openidx, const int *colpos, double *aug) {
  hipLaunchKernelGGL(k_build, dim3(L.nmax, L.ne), dim3(256), sizeof(double) * L.nmax, s, tab, pwi, fg, nopen, openidx,
                     colpos, L.ldo, aug, L.ldaug, L.sA, L.roff);
}

// ---------------------------------------------------------------------------
// LU building blocks.  dims[2e] = rows, dims[2e+1] = rhs.  Virtual column v of
// the part right of the panel maps to a real column: v < rows - c0 -> c0 + v,
// otherwise roff + (v - (rows - c0)).
// ---------------------------------------------------------------------------
__device__ __forceinline__ long vcol(int v, int rows, int c0, long roff) {
  return v < rows - c0 ? (long)(c0 + v) : roff + (v - (rows - c0));
}

// Panel factorisation: columns [j0, j0 + jb) over rows [j0, rows).  Row
// interchanges are applied here only to the panel's own columns and recorded in
// ipiv; k_lu_trsm applies them to every column right of the panel.  One
// workgroup per energy: each thread owns rows t, t + PANEL_T, ...; the pivot
// search reduces within each wave by shuffles and across waves in LDS (ties go
// to the smaller row, so the choice is deterministic), and the pivot row's panel
// segment is staged in LDS for the rank-1 update.
constexpr int PANEL_T = 512;
__global__ __launch_bounds__(PANEL_T) void k_lu_panel(int j0, const int *__restrict__ dims,
                                                      double *__restrict__ aug, long ldaug, long strideA,
                                                      int *__restrict__ ipiv, long ldp,
                                                      int *__restrict__ status) {
  const int e = blockIdx.x;
  const int rows = dims[2 * e];
  if (j0 >= rows) return;
  const int jb = min(NB, rows - j0);
  double *A = aug + (size_t)e * strideA;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  __shared__ double wv[PANEL_T / 64];
  __shared__ int wi[PANEL_T / 64];
  __shared__ int spiv;
  __shared__ double prow[NB];
  for (int c = j0; c < j0 + jb; ++c) {
    double best = -1.0;
    int bidx = rows;
    for (int r = c + t; r < rows; r += PANEL_T) {
      const double v = fabs(A[(size_t)r * ldaug + c]);
      if (v > best) { best = v; bidx = r; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bidx, off);
      if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
    }
    if (lane == 0) { wv[wid] = best; wi[wid] = bidx; }
    __syncthreads();
    if (t == 0) {
      double bv = wv[0];
      int bi = wi[0];
      for (int w = 1; w < PANEL_T / 64; ++w)
        if (wv[w] > bv || (wv[w] == bv && wi[w] < bi)) { bv = wv[w]; bi = wi[w]; }
      if (!(bv > 0.0) || bi >= rows) {
        atomicOr(status + e, RM_PT_SINGULAR);
        bi = c;
      }
      spiv = bi;
      ipiv[(size_t)e * ldp + c] = bi;
    }
    __syncthreads();
    const int p = spiv;
    if (t < jb) {
      const int col = j0 + t;
      const double pv = A[(size_t)p * ldaug + col];
      if (p != c) {
        A[(size_t)p * ldaug + col] = A[(size_t)c * ldaug + col];
        A[(size_t)c * ldaug + col] = pv;
      }
      prow[t] = pv;
    }
    __syncthreads();
    const double piv = prow[c - j0];
    const double inv = piv != 0.0 ? 1.0 / piv : 0.0;
    for (int r = c + 1 + t; r < rows; r += PANEL_T) {
      double *row = A + (size_t)r * ldaug;
      const double m = row[c] * inv;
      row[c] = m;
      for (int q = c + 1; q < j0 + jb; ++q) row[q] -= m * prow[q - j0];
    }
    __syncthreads();
  }
}

// Register-resident panel factorisation, the same algorithm as k_lu_panel for
// panels of at most RPT * PREG_T rows: the panel is read from memory once, each
// thread keeps rows t, t + PREG_T, ... (all NB columns) in registers, the pivot
// row and the row it replaces are exchanged through LDS, and the factored panel
// is written back once.
constexpr int PREG_T = 512;
template <int RPT>
__global__ __launch_bounds__(PREG_T) void k_lu_panel_reg(int j0, const int *__restrict__ dims,
                                                         double *__restrict__ aug, long ldaug, long strideA,
                                                         int *__restrict__ ipiv, long ldp,
                                                         int *__restrict__ status) {
  const int e = blockIdx.x;
  const int rows = dims[2 * e];
  if (j0 >= rows) return;
  const int jb = min(NB, rows - j0);
  const int m = rows - j0;  // panel height; rows below are relative to j0
  double *P = aug + (size_t)e * strideA + (size_t)j0 * ldaug + j0;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  __shared__ double wv[PREG_T / 64];
  __shared__ int wi[PREG_T / 64];
  __shared__ int spiv;
  __shared__ double prow[NB], crow[NB];
  double v[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + PREG_T * q;
    if (r < m) {
      const double2 *src = reinterpret_cast<const double2 *>(P + (size_t)r * ldaug);
#pragma unroll
      for (int c = 0; c < NB / 2; ++c) {
        const double2 x = src[c];
        v[q][2 * c] = x.x;
        v[q][2 * c + 1] = x.y;
      }
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) v[q][c] = 0.0;
    }
  }
  static_for([&](auto cI) {
    constexpr int c = decltype(cI)::value;
    if (c >= jb) return;  // uniform over the workgroup
    double best = -1.0;
    int bidx = m;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = t + PREG_T * q;
      if (r >= c && r < m) {
        const double a = fabs(v[q][c]);
        if (a > best) { best = a; bidx = r; }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bidx, off);
      if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
    }
    if (lane == 0) { wv[wid] = best; wi[wid] = bidx; }
    __syncthreads();
    if (t == 0) {
      double bv = wv[0];
      int bi = wi[0];
      for (int w = 1; w < PREG_T / 64; ++w)
        if (wv[w] > bv || (wv[w] == bv && wi[w] < bi)) { bv = wv[w]; bi = wi[w]; }
      if (!(bv > 0.0) || bi >= m) {
        atomicOr(status + e, RM_PT_SINGULAR);
        bi = c;
      }
      spiv = bi;
      ipiv[(size_t)e * ldp + j0 + c] = j0 + bi;
    }
    __syncthreads();
    const int p = spiv;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = t + PREG_T * q;
      if (r == p) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) prow[cc] = v[q][cc];
      }
      if (r == c) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) crow[cc] = v[q][cc];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = t + PREG_T * q;
      if (r == c) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) v[q][cc] = prow[cc];
      } else if (r == p) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) v[q][cc] = crow[cc];
      }
    }
    const double piv = prow[c];
    const double inv = piv != 0.0 ? 1.0 / piv : 0.0;
    double l[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = t + PREG_T * q;
      const bool below = r > c && r < m;
      l[q] = below ? v[q][c] * inv : 0.0;
      if (below) v[q][c] = l[q];
    }
#pragma unroll
    for (int cc = c + 1; cc < NB; ++cc) {
      const double pr = cc < jb ? prow[cc] : 0.0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) v[q][cc] -= l[q] * pr;
    }
    __syncthreads();
  }, std::make_integer_sequence<int, NB>{});
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + PREG_T * q;
    if (r < m) {
      double2 *dst = reinterpret_cast<double2 *>(P + (size_t)r * ldaug);
#pragma unroll
      for (int c = 0; c < NB / 2; ++c) dst[c] = double2{v[q][2 * c], v[q][2 * c + 1]};
    }
  }
}

// Number of trailing "virtual" columns right of a block that ends at column c0:
// the remaining columns of A, then (if with_rhs) the right-hand sides, at most
// vlimit in all.
// Virtual column v of a trailing block whose A part is acols wide.
__device__ __forceinline__ long vcol2(int v, int acols, int c0, long roff) {
  return v < acols ? (long)(c0 + v) : roff + (v - acols);
}

__device__ __forceinline__ int trailing_cols(int rows, int rhs, int c0, int with_rhs, int vlimit) {
  return min(vlimit, (rows - c0) + (with_rhs ? rhs : 0));
}

// After the panels of an outer block [p0, p0 + jb) are factored: the second
// panel's interchanges (rows >= p0 + NB) are applied to the first panel's
// columns, so that the block's L21 rows line up with the trailing rows, and the
// net permutation of all jb interchanges is written to bperm: the source row of
// each block row, and every row outside the block that receives another row,
// with its source.  One wave per energy: lane 0 applies the transpositions in
// order; the outside rows are found by a wave-wide compare.
__global__ __launch_bounds__(64) void k_lu_blockperm(int p0, const int *__restrict__ dims, double *__restrict__ aug,
                                                     long ldaug, long strideA, const int *__restrict__ ipiv, long ldp,
                                                     int *__restrict__ bperm, double *__restrict__ linv) {
  const int e = blockIdx.x;
  const int rows = dims[2 * e];
  if (p0 >= rows) return;
  const int jb = min(NBU, rows - p0);
  const int lane = threadIdx.x;
  double *A = aug + (size_t)e * strideA;
  const int *pv = ipiv + (size_t)e * ldp + p0;
  if (jb > NB && lane < NB) {
    const long col = p0 + lane;
    for (int r = NB; r < jb; ++r) {
      const int p = pv[r];
      if (p != p0 + r) {
        const double x = A[(size_t)p * ldaug + col];
        A[(size_t)p * ldaug + col] = A[(size_t)(p0 + r) * ldaug + col];
        A[(size_t)(p0 + r) * ldaug + col] = x;
      }
    }
  }
  __shared__ int src[2 * NBU], pos[NBU];
  for (int r = lane; r < jb; r += 64) src[r] = p0 + r;
  __syncthreads();
  int nout = 0;
  for (int r = 0; r < jb; ++r) {
    const int p = pv[r];
    int sp;
    if (p < p0 + jb) {
      sp = p - p0;
    } else {
      const bool hit = lane < nout && pos[lane] == p;
      const unsigned long long m = __ballot(hit);
      if (m) {
        sp = NBU + __ffsll((long long)m) - 1;
      } else {
        sp = NBU + nout;
        if (lane == 0) {
          pos[nout] = p;
          src[sp] = p;
        }
        ++nout;
      }
    }
    __syncthreads();
    if (lane == 0 && sp != r) {
      const int a = src[r];
      src[r] = src[sp];
      src[sp] = a;
    }
    __syncthreads();
  }
  int *out = bperm + (size_t)e * BPERM;
  if (lane == 0) out[0] = nout;
  for (int r = lane; r < NBU; r += 64) {
    out[1 + r] = r < jb ? src[r] : 0;
    out[1 + NBU + r] = r < nout ? src[NBU + r] : 0;
    out[1 + 2 * NBU + r] = r < nout ? pos[r] : 0;
  }
  // Inverse of the unit lower L11 (identity beyond jb): lane j computes column j
  // by forward substitution, X[i][j] = -sum_{j <= k < i} L[i][k] X[k][j].
  __shared__ double sl[NBU][NBU + 1];
  __syncthreads();
  for (int idx = lane; idx < NBU * NBU; idx += 64) {
    const int r = idx / NBU, c = idx % NBU;
    sl[r][c] = (r < jb && c < r) ? A[(size_t)(p0 + r) * ldaug + p0 + c] : 0.0;
  }
  __syncthreads();
  double *Li = linv + (size_t)e * NBU * NBU;
  const int j = lane;
  double xc[NBU];
  static_for([&](auto iI) {
    constexpr int i = decltype(iI)::value;
    double acc = i == j ? 1.0 : 0.0;
    static_for([&](auto kI) {
      constexpr int k = decltype(kI)::value;
      if constexpr (k < i) acc -= sl[i][k] * xc[k];
    }, std::make_integer_sequence<int, NBU>{});
    xc[i] = i < j ? 0.0 : acc;
  }, std::make_integer_sequence<int, NBU>{});
  static_for([&](auto iI) {
    constexpr int i = decltype(iI)::value;
    Li[(size_t)i * NBU + j] = xc[i];
  }, std::make_integer_sequence<int, NBU>{});
}

// Triangular solve for the trailing columns of an outer block, U12 = L11^-1 P A12,
// as a product with the block's explicit inverse (k_lu_blockinv) on FP64 MFMA.
// Each workgroup owns 64 trailing columns at a time: it gathers their block
// rows from the source rows of the net permutation and loads the rows that
// move out of the block (every load of a tile before any of its stores),
// writes the moved rows, then forms the 64 x 64 product.  The loads of the
// next tile (other columns, untouched by this tile's stores) are issued before
// this tile is multiplied and have completed, in every thread, before the
// next tile's first store.
constexpr int TRSM_G = 8;
__global__ __launch_bounds__(256) void k_lu_trsm_inv(int p0, const int *__restrict__ dims, double *__restrict__ aug,
                                                     long ldaug, long strideA, long roff,
                                                     const int *__restrict__ bperm, const double *__restrict__ linv,
                                                     int tiles_n, int ne) {
  constexpr int KB = NBU;
  constexpr int NY = KB * TILE / 256;      // gathered and moved elements per thread
  __shared__ double sL[KB][Pitch<KB>::A];  // sL[i][k] = Linv[i][k]
  __shared__ double sX[KB][PB];            // sX[k][j] = (P A12)[k][v0 + j]
  __shared__ int sp[1 + 3 * KB];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  const int jt = t % TILE, kt = t / TILE;  // this thread's column and first row of a tile (rows kt + 4q)
  // an item is a group of TRSM_G column tiles of one energy: L11^-1 and the
  // permutation are staged once for the group
  for_items(ne, (tiles_n + TRSM_G - 1) / TRSM_G, [&](int e, int grp) {
    const int rows = dims[2 * e], rhs = dims[2 * e + 1];
    if (p0 >= rows) return;
    const int jb = min(KB, rows - p0);
    const int c0 = p0 + jb;
    const int ncols = (rows - c0) + rhs;
    const int vfirst = grp * TRSM_G * TILE;
    if (vfirst >= ncols) return;
    const int ntile = min(TRSM_G, (ncols - vfirst + TILE - 1) / TILE);
    double *A = aug + (size_t)e * strideA;
    const int *pm = bperm + (size_t)e * BPERM;
    const double *Li = linv + (size_t)e * KB * KB;
    for (int idx = t; idx < 1 + 3 * KB; idx += 256) sp[idx] = pm[idx];
    for (int idx = t; idx < KB * KB; idx += 256) sL[idx / KB][idx % KB] = Li[idx];
    __syncthreads();
    const int nout = sp[0];
    double xv[NY], yv[NY];
    auto load = [&](int v0) {
      const bool ok = v0 + jt < ncols;
      const long col = ok ? vcol(v0 + jt, rows, c0, roff) : 0;
#pragma unroll
      for (int q = 0; q < NY; ++q) {
        const int k = kt + 4 * q;
        xv[q] = (ok && k < jb) ? A[(size_t)sp[1 + k] * ldaug + col] : 0.0;
        yv[q] = (ok && k < nout) ? A[(size_t)sp[1 + KB + k] * ldaug + col] : 0.0;
      }
    };
    load(vfirst);
    // every load of a tile completes before any store of that tile: the moved
    // rows' destinations are gather sources of the same columns
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int g = 0; g < ntile; ++g) {
      const int v0 = vfirst + g * TILE;
      {
        const bool ok = v0 + jt < ncols;
        const long col = ok ? vcol(v0 + jt, rows, c0, roff) : 0;
#pragma unroll
        for (int q = 0; q < NY; ++q) {
          const int k = kt + 4 * q;
          sX[k][jt] = xv[q];
          if (ok && k < nout) A[(size_t)sp[1 + 2 * KB + k] * ldaug + col] = yv[q];
        }
      }
      __syncthreads();
      if (g + 1 < ntile) load(v0 + TILE);
      d4 acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = d4{0, 0, 0, 0};
      mfma_slab<KB>(sL, sX, acc, wr, wc, kk, ii);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = v0 + wc * 32 + (q & 1) * 16 + ii;
        if (v >= ncols) continue;
        const long col = vcol(v, rows, c0, roff);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = wr * 32 + (q >> 1) * 16 + 4 * r + kk;
          if (i < jb) A[(size_t)(p0 + i) * ldaug + col] = acc[q][r];
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of the next tile have completed
      __syncthreads();                // and LDS is reused by the next tile
    }
  });
}

// For trailing columns of the block of kb rows starting at p0 (columns [p0 +
// jb, ...) as in trailing_cols): apply the block's row interchanges in order,
// then U12 = L11^-1 A12 on rows [p0, p0 + jb).  One thread per column; the
// column's block rows are kept in LDS (its own slot).
template <int KB, int T>
__global__ __launch_bounds__(T) void k_lu_trsm(int p0, const int *__restrict__ dims, double *__restrict__ aug,
                                               long ldaug, long strideA, long roff, const int *__restrict__ ipiv,
                                               long ldp, int with_rhs, int vlimit) {
  const int e = blockIdx.y;
  const int rows = dims[2 * e], rhs = dims[2 * e + 1];
  if (p0 >= rows) return;
  const int jb = min(KB, rows - p0);
  const int c0 = p0 + jb;
  const int ncols = trailing_cols(rows, rhs, c0, with_rhs, vlimit);
  if ((int)(blockIdx.x * T) >= ncols) return;
  double *A = aug + (size_t)e * strideA;
  __shared__ double L[KB][KB + 1];
  __shared__ double sx[KB][T];
  __shared__ int piv[KB];
  const int t = threadIdx.x;
  for (int idx = t; idx < jb * jb; idx += T) {
    const int r = idx / jb, c = idx % jb;
    L[r][c] = A[(size_t)(p0 + r) * ldaug + p0 + c];
  }
  if (t < jb) piv[t] = ipiv[(size_t)e * ldp + p0 + t];
  __syncthreads();
  const int v = blockIdx.x * T + t;
  if (v < ncols) {
    const long col = vcol(v, rows, c0, roff);
    for (int r = 0; r < jb; ++r) {
      const int p = piv[r];
      const double x = A[(size_t)p * ldaug + col];
      if (p != p0 + r) A[(size_t)p * ldaug + col] = A[(size_t)(p0 + r) * ldaug + col];
      sx[r][t] = x;  // row p0 + r after the interchange; later interchanges of
                     // this block only touch rows > p0 + r, so it stays in LDS
    }
    for (int r = 1; r < jb; ++r) {
      double acc = sx[r][t];
      for (int c = 0; c < r; ++c) acc -= L[r][c] * sx[c][t];
      sx[r][t] = acc;
    }
    for (int r = 0; r < jb; ++r) A[(size_t)(p0 + r) * ldaug + col] = sx[r][t];
  }
}

// Memory column of virtual column v of a trailing block: the A part (acols
// wide, from column c0), then the right-hand sides from column roff.
struct ColMap {
  int acols, c0;
  long roff;
  __device__ __forceinline__ long operator()(int v) const { return v < acols ? (long)(c0 + v) : roff + (v - acols); }
};

// Tiles of C loaded ahead by the streaming updates.
#ifndef UPD_DEPTH
#define UPD_DEPTH 1
#endif
// Rows of U for the streaming updates: row k of a block of jb rows that starts
// at Ub (rows past jb read as 0).
struct RowsU {
  const double *Ub;
  long ld;
  int jb;
  __device__ __forceinline__ double operator()(int k, long col) const { return k < jb ? Ub[(long)k * ld + col] : 0.0; }
};

// C (64 rows x G column tiles) -= Lb (64 x KB) * U (KB x columns), one column
// tile at a time, with sL holding -Lb: the MFMAs accumulate onto the loaded C
// values.  The C values of the next two tiles and the U slab of the next tile
// are loaded into registers while the current tile is multiplied, so three
// tiles of C are in flight per workgroup.  Cb points at row 0 of the C block
// (row stride ld); C and U are addressed through the column map cm, and
// u(k, col) reads row k of U at memory column col.
template <int KB, int G, int DEPTH = UPD_DEPTH, typename UL>
__device__ __forceinline__ void rowblock_update(const double (*sL)[Pitch<KB>::A], double (*sU)[PB], int mrem,
                                                int vbeg, int ncols, ColMap cm, double *Cb, UL u, long ld) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  constexpr int NU = KB * TILE / 256;
  // U slab: this thread stages column ju, rows ku0 + 4q
  const int ju = t % TILE, ku0 = t / TILE;
  // C: rows wr*32 + h*16 + 4v + kk (h, v) and columns wc*32 + c*16 + ii (c)
  long rowoff[8];
  bool rok[8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = wr * 32 + h * 16 + 4 * v + kk;
      rok[h * 4 + v] = i < mrem;
      rowoff[h * 4 + v] = (long)i * ld;
    }
  auto loadU = [&](int v0, double (&dst)[NU]) {
    const int v = v0 + ju;
    const bool ok = v < ncols;
    const long col = ok ? cm(v) : 0;
#pragma unroll
    for (int q = 0; q < NU; ++q) {
      const int k = ku0 + 4 * q;
      dst[q] = ok ? u(k, col) : 0.0;
    }
  };
  auto cols = [&](int v0, long (&col)[2], bool (&cok)[2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int v = v0 + wc * 32 + c * 16 + ii;
      cok[c] = v < ncols;
      col[c] = cok[c] ? cm(v) : 0;
    }
  };
  auto loadC = [&](int v0, double (&dst)[16]) {
    long col[2];
    bool cok[2];
    cols(v0, col, cok);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          dst[(h * 2 + c) * 4 + v] = (rok[h * 4 + v] && cok[c]) ? Cb[rowoff[h * 4 + v] + col[c]] : 0.0;
  };
  const int ntile = min(G, (ncols - vbeg + TILE - 1) / TILE);
  double nu[NU], ca[16], cb[16];
  if (ntile > 0) {
    loadU(vbeg, nu);
    loadC(vbeg, ca);
  }
  if (DEPTH > 1 && ntile > 1) loadC(vbeg + TILE, cb);
  // tile g: its C values are in cur, which then receives tile g + DEPTH
  auto step = [&](int g, double (&cur)[16]) {
    const int v0 = vbeg + g * TILE;
#pragma unroll
    for (int q = 0; q < NU; ++q) sU[ku0 + 4 * q][ju] = nu[q];
    __syncthreads();
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{cur[4 * q], cur[4 * q + 1], cur[4 * q + 2], cur[4 * q + 3]};
    if (g + 1 < ntile) loadU(v0 + TILE, nu);
    if (g + DEPTH < ntile) loadC(v0 + DEPTH * TILE, cur);
    mfma_slab<KB, 4>(sL, sU, acc, wr, wc, kk, ii);
    long col[2];
    bool cok[2];
    cols(v0, col, cok);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (rok[h * 4 + v] && cok[c]) Cb[rowoff[h * 4 + v] + col[c]] = acc[h * 2 + c][v];
    __syncthreads();
  };
  for (int g = 0; g < ntile; g += DEPTH) {
    step(g, ca);
    if (DEPTH > 1 && g + 1 < ntile) step(g + 1, cb);
  }
}

// Column tiles per workgroup of the streaming updates.
// (a compile-time knob; 16 and 32 measured slower than 64 at 1500 channels)
#ifndef RM_UPD_G
#define RM_UPD_G 64
#endif
constexpr int UPD_G = RM_UPD_G;

// Trailing update A22 -= L21 U12 for the block of kb columns starting at p0:
// rows [c0, rows) with c0 = p0 + jb, trailing columns as in trailing_cols.
// Items: (energy, column group of UPD_G tiles, 64-row block), FP64 MFMA.
template <int KB>
__global__ __launch_bounds__(256, 2) void k_lu_update(int p0, const int *__restrict__ dims, double *__restrict__ aug,
                                                   long ldaug, long strideA, long roff, int tiles_m, int groups,
                                                   int ne, int with_rhs, int vlimit, int lower) {
  __shared__ double sL[TILE][Pitch<KB>::A];  // sL[i][k] = -L21[r0 + i][k]
  __shared__ double sU[KB][PB];              // sU[k][j] = U12[k][v0 + j]
  for_items(ne, tiles_m * groups, [&](int e, int it) {
    const int tmi = it % tiles_m, g = it / tiles_m;
    const int rows = dims[2 * e], rhs = dims[2 * e + 1];
    if (p0 >= rows) return;
    const int jb = min(KB, rows - p0);
    const int c0 = p0 + jb;
    const int m = rows - c0;
    const int r0 = tmi * TILE, vbeg = g * UPD_G * TILE;
    // with lower set only the columns up to this row block's diagonal tile
    // (the update is symmetric and its upper part is never read)
    const int acols = lower ? min(m, r0 + TILE) : m;
    const int ncols = min(vlimit, acols + (with_rhs ? rhs : 0));
    if (r0 >= m || vbeg >= ncols) return;
    double *A = aug + (size_t)e * strideA;
    for (int idx = threadIdx.x; idx < KB * TILE; idx += 256) {
      const int i = idx / KB, k = idx % KB;
      sL[i][k] = (r0 + i < m && k < jb) ? -A[(size_t)(c0 + r0 + i) * ldaug + p0 + k] : 0.0;
    }
    rowblock_update<KB, UPD_G>(sL, sU, m - r0, vbeg, ncols, ColMap{acols, c0, roff}, A + (size_t)(c0 + r0) * ldaug,
                               RowsU{A + (size_t)p0 * ldaug, ldaug, jb}, ldaug);
  });
}

// Back substitution, diagonal block: Y_b = U_bb^-1 B_b for the right-hand sides,
// one thread per right-hand side with its column in registers and U_bb in LDS
// (column-oriented: each solved entry is eliminated from the rows above it).
// A workgroup of BS_T threads (several waves share one staged U_bb) takes BS_G
// groups of BS_T right-hand sides per item.
constexpr int BS_T = 256, BS_G = 1;
template <int KB, int T>
__global__ __launch_bounds__(T) void k_bs_block(int j0, const int *__restrict__ dims, double *__restrict__ aug,
                                                long ldaug, long strideA, long roff, int tiles, int ne, int tail) {
  __shared__ double U[KB][KB];
  const int t = threadIdx.x;
  // an item is a group of BS_G column tiles of one energy: U_bb is staged once
  for_items(ne, (tiles + BS_G - 1) / BS_G, [&](int e, int grp) {
    const int rows = dims[2 * e], rhs = dims[2 * e + 1];
    if (j0 >= rows || grp * BS_G * T >= rhs) return;
    if (tail && j0 + KB <= rows - rhs) return;  // block above the rows that are needed
    const int jb = min(KB, rows - j0);
    double *A = aug + (size_t)e * strideA;
    for (int idx = t; idx < KB * KB; idx += T) {
      const int r = idx / KB, c = idx % KB;
      U[r][c] = (r < jb && c < jb) ? A[(size_t)(j0 + r) * ldaug + j0 + c] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int g = 0; g < BS_G; ++g) {
      const int q = (grp * BS_G + g) * T + t;
      if (q < rhs) {
        const long col = roff + q;
        double x[KB];
        static_for([&](auto rI) {
          constexpr int r = decltype(rI)::value;
          x[r] = r < jb ? A[(size_t)(j0 + r) * ldaug + col] : 0.0;
        }, std::make_integer_sequence<int, KB>{});
        static_for([&](auto rI) {
          constexpr int r = KB - 1 - decltype(rI)::value;
          const double d = U[r][r];
          x[r] = d != 0.0 ? x[r] / d : 0.0;
          static_for([&](auto iI) {
            constexpr int i = decltype(iI)::value;
            if constexpr (i < r) x[i] -= U[i][r] * x[r];
          }, std::make_integer_sequence<int, KB>{});
        }, std::make_integer_sequence<int, KB>{});
        static_for([&](auto rI) {
          constexpr int r = decltype(rI)::value;
          if (r < jb) A[(size_t)(j0 + r) * ldaug + col] = x[r];
        }, std::make_integer_sequence<int, KB>{});
      }
    }
    __syncthreads();  // U is reused by the next item
  });
}

// Back substitution, update above the block: B[0:j0] -= U[0:j0, j0:j0+jb] Y_b.
// Items: (energy, group of UPD_G right-hand-side tiles, 64-row block).
template <int KB>
__global__ __launch_bounds__(256, 2) void k_bs_update(int j0, const int *__restrict__ dims, double *__restrict__ aug,
                                                   long ldaug, long strideA, long roff, int tiles_m, int groups,
                                                   int ne, int tail) {
  __shared__ double sU[TILE][Pitch<KB>::A];  // sU[i][k] = -U[r0 + i][j0 + k]
  __shared__ double sY[KB][PB];              // sY[k][j] = Y[j0 + k][q0 + j]
  for_items(ne, tiles_m * groups, [&](int e, int it) {
    const int tmi = it % tiles_m, g = it / tiles_m;
    const int rows = dims[2 * e], rhs = dims[2 * e + 1];
    if (j0 >= rows || j0 == 0) return;
    const int jb = min(KB, rows - j0);
    const int r0 = tmi * TILE, qbeg = g * UPD_G * TILE;
    if (r0 >= j0 || qbeg >= rhs) return;
    if (tail && r0 + TILE <= rows - rhs) return;  // rows above the ones that are needed
    double *A = aug + (size_t)e * strideA;
    for (int idx = threadIdx.x; idx < KB * TILE; idx += 256) {
      const int i = idx / KB, k = idx % KB;
      sU[i][k] = (r0 + i < j0 && k < jb) ? -A[(size_t)(r0 + i) * ldaug + j0 + k] : 0.0;
    }
    rowblock_update<KB, UPD_G>(sU, sY, j0 - r0, qbeg, rhs, ColMap{0, 0, roff}, A + (size_t)r0 * ldaug,
                               RowsU{A + (size_t)j0 * ldaug, ldaug, jb}, ldaug);
  });
}

namespace {
void launch_panel(hipStream_t s, int ne, int j0, int h, const int *dims, double *aug, long ldaug, long strideA,
                  int *ipiv, long ldp, int *status) {
  if (h <= PREG_T)
    hipLaunchKernelGGL(k_lu_panel_reg<1>, dim3(ne), dim3(PREG_T), 0, s, j0, dims, aug, ldaug, strideA, ipiv, ldp,
                       status);
  else if (h <= 2 * PREG_T)
    hipLaunchKernelGGL(k_lu_panel_reg<2>, dim3(ne), dim3(PREG_T), 0, s, j0, dims, aug, ldaug, strideA, ipiv, ldp,
                       status);
  else if (h <= 3 * PREG_T)
    hipLaunchKernelGGL(k_lu_panel_reg<3>, dim3(ne), dim3(PREG_T), 0, s, j0, dims, aug, ldaug, strideA, ipiv, ldp,
                       status);
  else
    hipLaunchKernelGGL(k_lu_panel, dim3(ne), dim3(PANEL_T), 0, s, j0, dims, aug, ldaug, strideA, ipiv, ldp,
                       status);
}
}  // namespace

void launch_backsub(hipStream_t s, int ne, int maxrows, int maxrhs, const int *dims, double *aug, long ldaug,
                    long strideA, long roff, int tail);

// Outer blocks of NBU = 2 NB columns: factor the first panel, bring the second
// panel up to date (interchanges, triangular solve, rank-NB update), factor it,
// align the first panel's rows with its interchanges, then one triangular solve
// and one rank-NBU update for everything right of the block.
void launch_lu_solve(hipStream_t s, int ne, int maxrows, int maxrhs, const int *dims, double *aug,
                     long ldaug, long strideA, long roff, int *ipiv, long ldp, int *bperm, double *linv, int tail,
                     int *status) {
  constexpr int T32 = 128, T64 = 64;
  for (int j0 = 0; j0 < maxrows; j0 += NBU) {
    launch_panel(s, ne, j0, maxrows - j0, dims, aug, ldaug, strideA, ipiv, ldp, status);
    const int p1 = j0 + NB;
    if (p1 < maxrows) {
      // second panel's columns [p1, p1 + NB): no right-hand sides
      hipLaunchKernelGGL((k_lu_trsm<NB, T32>), dim3((NB + T32 - 1) / T32, ne), dim3(T32), 0, s, j0, dims, aug,
                         ldaug, strideA, roff, ipiv, ldp, 0, NB);
      const int tm = (maxrows - p1 + TILE - 1) / TILE;
      hipLaunchKernelGGL(k_lu_update<NB>, dim3(persist_grid(k_lu_update<NB>, 256, ne, tm)), dim3(256), 0, s, j0,
                         dims, aug, ldaug, strideA, roff, tm, 1, ne, 0, NB, 0);
      launch_panel(s, ne, p1, maxrows - p1, dims, aug, ldaug, strideA, ipiv, ldp, status);
    }
    hipLaunchKernelGGL(k_lu_blockperm, dim3(ne), dim3(64), 0, s, j0, dims, aug, ldaug, strideA, ipiv, ldp, bperm,
                       linv);
    const int c0 = std::min(maxrows, j0 + NBU);
    const int ncols = (maxrows - c0) + maxrhs;
    if (ncols <= 0) continue;
    const int tn = (ncols + TILE - 1) / TILE;
    hipLaunchKernelGGL(k_lu_trsm_inv, dim3(persist_grid(k_lu_trsm_inv, 256, ne, (tn + TRSM_G - 1) / TRSM_G)),
                       dim3(256), 0, s, j0, dims, aug, ldaug, strideA, roff, bperm, linv, tn, ne);
    const int m = maxrows - c0;
    if (m <= 0) continue;
    const int tm = (m + TILE - 1) / TILE, gr = (ncols + UPD_G * TILE - 1) / (UPD_G * TILE);
    hipLaunchKernelGGL(k_lu_update<NBU>, dim3(persist_grid(k_lu_update<NBU>, 256, ne, (long)tm * gr)), dim3(256), 0,
                       s, j0, dims, aug, ldaug, strideA, roff, tm, gr, ne, 1, 1 << 30, 0);
  }
  launch_backsub(s, ne, maxrows, maxrhs, dims, aug, ldaug, strideA, roff, tail);
}

// Blocked back substitution with the upper triangle of [A | B] (blocks of NBU
// rows from the bottom).
void launch_backsub(hipStream_t s, int ne, int maxrows, int maxrhs, const int *dims, double *aug, long ldaug,
                    long strideA, long roff, int tail) {
  if (maxrhs <= 0) return;
  for (int j0 = (maxrows - 1) / NBU * NBU; j0 >= 0; j0 -= NBU) {
    const int tb = (maxrhs + BS_T - 1) / BS_T;
    hipLaunchKernelGGL((k_bs_block<NBU, BS_T>),
                       dim3(persist_grid(k_bs_block<NBU, BS_T>, BS_T, ne, (tb + BS_G - 1) / BS_G)), dim3(BS_T), 0, s,
                       j0, dims, aug, ldaug, strideA, roff, tb, ne, tail);
    if (j0 == 0) break;
    const int tm = (j0 + TILE - 1) / TILE, gr = (maxrhs + UPD_G * TILE - 1) / (UPD_G * TILE);
    hipLaunchKernelGGL(k_bs_update<NBU>, dim3(persist_grid(k_bs_update<NBU>, 256, ne, (long)tm * gr)), dim3(256), 0,
                       s, j0, dims, aug, ldaug, strideA, roff, tm, gr, ne, tail);
  }
}

// ---------------------------------------------------------------------------
// S and Omega from K (Glossary, "Transitions matrix" and "Collision
// strength").  With M = 1 - iK,
//   S = (1 + iK) M^-1 = 2 M^-1 - 1,   T = S - 1 = 2 (M^-1 - 1),
//   |T_ij|^2 = 4 |(M^-1)_ij - d_ij|^2.
// K is real symmetric, so M is complex symmetric with Hermitian part 1: every
// leading block of M and of its Schur complements has Hermitian part >= 1, so
// M = C C^T (complex symmetric Cholesky, no pivoting) exists and every pivot
// has real part >= 1.  G = C^-1 is formed by forward substitution carried
// along the factorisation (identity right-hand sides), and M^-1 = G^T G.  No
// product K K is formed, so the result keeps the conditioning of M itself,
// max_lambda |1 - i lambda| over the eigenvalues lambda of K.
//
// Complex matrices are held as two real planes.  Per energy: M, then C, then
// M^-1 in aug (real part in columns [0, no), imaginary part in columns [roff,
// roff + no)); G in the planes gre and gim (row stride ldg).  The factorisation
// runs in complex blocks of ZB = 32 columns.  A complex product with a 32-wide
// inner dimension is a real product with a 64-wide one,
//   [Pr | Pi] [[Qr, Qi], [-Qi, Qr]] = [Re PQ | Im PQ],
//   [[Pr, -Pi], [Pi, Pr]] [Qr; Qi]  = [Re PQ; Im PQ],
// so the block solves are the 64 x 64 x 64 MFMA slabs of the LU, and the
// trailing update of each plane is a real rank-64 streaming update.
// ---------------------------------------------------------------------------
constexpr int ZB = NB;
constexpr int ZK = 2 * ZB;  // real inner dimension of a complex block product

// M = 1 - i (K + K^T)/2 on the leading no x no block (both triangles) and G = 0
// there; dims = {no, no}.  One pair of mirrored 32 x 32 tiles per workgroup, the
// transposed tile staged in LDS so that every access is row-contiguous.
__global__ __launch_bounds__(256) void k_zs_setup(const int *__restrict__ nopen, const double *__restrict__ Kw,
                                                  long ldk, long strideK, double *__restrict__ aug, long ldaug,
                                                  long strideA, long roff, double *__restrict__ gre,
                                                  double *__restrict__ gim, long ldg, long strideG,
                                                  int *__restrict__ dims) {
  const int e = blockIdx.y;
  const int no = nopen[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dims[2 * e] = no;
    dims[2 * e + 1] = no;
  }
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= (int)blockIdx.x) ++ti;
  const int tj = blockIdx.x - ti * (ti + 1) / 2;  // tile pair (ti, tj), ti >= tj
  const int i0 = ti * 32, j0 = tj * 32;
  if (i0 >= no) return;
  __shared__ double t1[32][33], t2[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double *K = Kw + (size_t)e * strideK;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx, i2 = j0 + r, j2 = i0 + tx;
    t1[r][tx] = (i < no && j < no) ? K[(size_t)i * ldk + j] : 0.0;
    t2[r][tx] = (i2 < no && j2 < no) ? K[(size_t)i2 * ldk + j2] : 0.0;
  }
  __syncthreads();
  double *A = aug + (size_t)e * strideA;
  double *Gr = gre + (size_t)e * strideG, *Gi = gim + (size_t)e * strideG;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx, i2 = j0 + r, j2 = i0 + tx;
    if (i < no && j < no) {
      A[(size_t)i * ldaug + j] = i == j ? 1.0 : 0.0;
      A[(size_t)i * ldaug + roff + j] = -0.5 * (t1[r][tx] + t2[tx][r]);
      Gr[(size_t)i * ldg + j] = 0.0;
      Gi[(size_t)i * ldg + j] = 0.0;
    }
    if (ti != tj && i2 < no && j2 < no) {
      A[(size_t)i2 * ldaug + j2] = 0.0;
      A[(size_t)i2 * ldaug + roff + j2] = -0.5 * (t2[r][tx] + t1[tx][r]);
      Gr[(size_t)i2 * ldg + j2] = 0.0;
      Gi[(size_t)i2 * ldg + j2] = 0.0;
    }
  }
}

// Diagonal block [j0, j0 + jb): unblocked complex symmetric Cholesky of M11 in
// LDS, C11 written back to the lower part of the planes, and L = C11^-1 (lower)
// both to G's diagonal block and, as the real 64 x 64 matrix
// Z = [[Lr, -Li], [Li, Lr]] (zero outside jb), to zinv for the block solves.
// A pivot of zero modulus (possible only for non-finite input) sets
// RM_PT_SINGULAR and is replaced by 1.
__global__ __launch_bounds__(256) void k_zs_diag(int j0, const int *__restrict__ dims, double *__restrict__ aug,
                                                 long ldaug, long strideA, long roff, double *__restrict__ gre,
                                                 double *__restrict__ gim, long ldg, long strideG,
                                                 double *__restrict__ zinv, int *__restrict__ status) {
  const int e = blockIdx.x;
  const int rows = dims[2 * e];
  if (j0 >= rows) return;
  const int jb = min(ZB, rows - j0);
  double *Ar = aug + (size_t)e * strideA + (size_t)j0 * ldaug + j0;
  double *Ai = Ar + roff;
  __shared__ double cr[ZB][ZB + 1], ci[ZB][ZB + 1], xr[ZB][ZB + 1], xi[ZB][ZB + 1];
  const int t = threadIdx.x;
  for (int idx = t; idx < ZB * ZB; idx += 256) {
    const int i = idx / ZB, k = idx % ZB;
    const bool in = i < jb && k <= i;
    cr[i][k] = in ? Ar[(size_t)i * ldaug + k] : (i == k ? 1.0 : 0.0);
    ci[i][k] = in ? Ai[(size_t)i * ldaug + k] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < jb; ++j) {
    if (t == 0) {
      // principal square root of the pivot x + iy (x >= 1 in exact arithmetic)
      double x = cr[j][j], y = ci[j][j];
      const double r = hypot(x, y);
      if (!(r > 0.0) || !isfinite(r)) {
        atomicOr(status + e, RM_PT_SINGULAR);
        x = 1.0;
        y = 0.0;
      }
      double u, v;
      if (x >= 0.0) {
        u = sqrt(0.5 * (hypot(x, y) + x));
        v = y / (2.0 * u);
      } else {
        v = copysign(sqrt(0.5 * (hypot(x, y) - x)), y);
        u = y / (2.0 * v);
      }
      cr[j][j] = u;
      ci[j][j] = v;
    }
    __syncthreads();
    // column below the pivot: c_ij = m_ij / c_jj
    const double dr = cr[j][j], di = ci[j][j], den = 1.0 / (dr * dr + di * di);
    for (int i = j + 1 + t; i < jb; i += 256) {
      const double ar = cr[i][j], ai = ci[i][j];
      cr[i][j] = (ar * dr + ai * di) * den;
      ci[i][j] = (ai * dr - ar * di) * den;
    }
    __syncthreads();
    // m_ik -= c_ij c_kj (lower part of the trailing block)
    const int c = jb - 1 - j;
    for (int idx = t; idx < c * c; idx += 256) {
      const int i = j + 1 + idx / c, k = j + 1 + idx % c;
      if (k <= i) {
        const double pr = cr[i][j] * cr[k][j] - ci[i][j] * ci[k][j];
        const double pi = cr[i][j] * ci[k][j] + ci[i][j] * cr[k][j];
        cr[i][k] -= pr;
        ci[i][k] -= pi;
      }
    }
    __syncthreads();
  }
  for (int idx = t; idx < jb * jb; idx += 256) {
    const int i = idx / jb, k = idx % jb;
    if (k <= i) {
      Ar[(size_t)i * ldaug + k] = cr[i][k];
      Ai[(size_t)i * ldaug + k] = ci[i][k];
    }
  }
  // lane j of wave 0: column j of C11^-1 by forward substitution, into LDS
  if (t < ZB) {
    const int j = t;
    for (int i = 0; i < ZB; ++i) {
      double sr = i == j ? 1.0 : 0.0, si = 0.0;
      for (int k = j; k < i; ++k) {
        const double pr = cr[i][k], pi = ci[i][k], qr = xr[k][j], qi = xi[k][j];
        sr -= pr * qr - pi * qi;
        si -= pr * qi + pi * qr;
      }
      const double dr = cr[i][i], di = ci[i][i], den = 1.0 / (dr * dr + di * di);
      xr[i][j] = i < j ? 0.0 : (sr * dr + si * di) * den;
      xi[i][j] = i < j ? 0.0 : (si * dr - sr * di) * den;
    }
  }
  __syncthreads();
  double *Gr = gre + (size_t)e * strideG + (size_t)j0 * ldg + j0;
  double *Gi = gim + (size_t)e * strideG + (size_t)j0 * ldg + j0;
  double *Z = zinv + (size_t)e * ZK * ZK;
  for (int idx = t; idx < ZB * ZB; idx += 256) {
    const int i = idx / ZB, j = idx % ZB;
    const bool in = i < jb && j < jb;
    const double lr = in ? xr[i][j] : 0.0, li = in ? xi[i][j] : 0.0;
    if (in) {
      Gr[(size_t)i * ldg + j] = lr;
      Gi[(size_t)i * ldg + j] = li;
    }
    Z[(size_t)i * ZK + j] = lr;
    Z[(size_t)i * ZK + ZB + j] = -li;
    Z[(size_t)(ZB + i) * ZK + j] = li;
    Z[(size_t)(ZB + i) * ZK + ZB + j] = lr;
  }
}

// Panel below the diagonal block: C21 = M21 C11^-T, one 64-row tile per item,
// as the real product [M21r | M21i] Z^T = [C21r | C21i].  C21 is written to the
// lower part of the planes and transposed into the upper part (rows [j0, j0 +
// jb)), where the trailing update reads it as U.
__global__ __launch_bounds__(256) void k_zs_panel(int j0, const int *__restrict__ dims, double *__restrict__ aug,
                                                  long ldaug, long strideA, long roff,
                                                  const double *__restrict__ zinv, int tiles_m, int ne) {
  __shared__ double sA[TILE][Pitch<ZK>::A];  // sA[i][k] = [M21r | M21i][r0 + i][k]
  __shared__ double sB[ZK][PB];              // sB[k][j] = Z[j][k]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  for_items(ne, tiles_m, [&](int e, int tile) {
    const int rows = dims[2 * e];
    if (j0 >= rows) return;
    const int jb = min(ZB, rows - j0);
    const int c0 = j0 + jb, m = rows - c0, r0 = tile * TILE;
    if (r0 >= m) return;
    double *A = aug + (size_t)e * strideA;
    const double *Z = zinv + (size_t)e * ZK * ZK;
    for (int idx = t; idx < ZK * TILE; idx += 256) {
      const int i = idx / ZK, k = idx % ZK, kc = k & (ZB - 1);
      sA[i][k] = (r0 + i < m && kc < jb) ? A[(size_t)(c0 + r0 + i) * ldaug + (k < ZB ? 0 : roff) + j0 + kc] : 0.0;
    }
    for (int idx = t; idx < ZK * ZK; idx += 256) sB[idx / ZK][idx % ZK] = Z[(idx % ZK) * ZK + idx / ZK];
    __syncthreads();
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0, 0, 0, 0};
    mfma_slab<ZK>(sA, sB, acc, wr, wc, kk, ii);
    // output column j: real part (j < ZB) or imaginary part (j >= ZB) of column j0 + (j mod ZB)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = wc * 32 + (q & 1) * 16 + ii, jc = j & (ZB - 1);
      if (jc >= jb) continue;
      const long off = j < ZB ? 0 : roff;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wr * 32 + (q >> 1) * 16 + 4 * v + kk;
        if (r0 + i < m) {
          A[(size_t)(c0 + r0 + i) * ldaug + off + j0 + jc] = acc[q][v];
          A[(size_t)(j0 + jc) * ldaug + off + c0 + r0 + i] = acc[q][v];
        }
      }
    }
    __syncthreads();
  });
}

// Right-hand sides of the diagonal block left of it: G1 = C11^-1 B1 on G's rows
// [j0, j0 + jb), columns [0, j0) (the diagonal block itself was written by
// k_zs_diag), as the real product Z [B1r; B1i] = [G1r; G1i], one 64-column
// tile per item, in place.
__global__ __launch_bounds__(256) void k_zs_rhs(int j0, const int *__restrict__ dims, double *__restrict__ gre,
                                                double *__restrict__ gim, long ldg, long strideG,
                                                const double *__restrict__ zinv, int tiles_n, int ne) {
  __shared__ double sL[ZK][Pitch<ZK>::A];  // sL[i][k] = Z[i][k]
  __shared__ double sX[ZK][PB];            // sX[k][j] = [B1r; B1i][k][q0 + j]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  for_items(ne, tiles_n, [&](int e, int tile) {
    const int rows = dims[2 * e];
    if (j0 >= rows) return;
    const int jb = min(ZB, rows - j0);
    const int q0 = tile * TILE;
    if (q0 >= j0) return;
    double *Gr = gre + (size_t)e * strideG + (size_t)j0 * ldg;
    double *Gi = gim + (size_t)e * strideG + (size_t)j0 * ldg;
    const double *Z = zinv + (size_t)e * ZK * ZK;
    for (int idx = t; idx < ZK * ZK; idx += 256) sL[idx / ZK][idx % ZK] = Z[idx];
    for (int idx = t; idx < ZK * TILE; idx += 256) {
      const int k = idx / TILE, j = idx % TILE, kc = k & (ZB - 1);
      sX[k][j] = (kc < jb && q0 + j < j0) ? (k < ZB ? Gr : Gi)[(size_t)kc * ldg + q0 + j] : 0.0;
    }
    __syncthreads();
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0, 0, 0, 0};
    mfma_slab<ZK>(sL, sX, acc, wr, wc, kk, ii);
    // output row i: real part (i < ZB) or imaginary part (i >= ZB) of row j0 + (i mod ZB)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = q0 + wc * 32 + (q & 1) * 16 + ii;
      if (j >= j0) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wr * 32 + (q >> 1) * 16 + 4 * v + kk, ic = i & (ZB - 1);
        if (ic < jb) (i < ZB ? Gr : Gi)[(size_t)ic * ldg + j] = acc[q][v];
      }
    }
    __syncthreads();
  });
}

// U of the complex trailing update, stacked [Ur; Ui]: rows k < ZB from the
// real plane, rows ZB + k from the imaginary one (rows past jb read as 0).
struct ZRowsU {
  const double *re, *im;
  long ld;
  int jb;
  __device__ __forceinline__ double operator()(int k, long col) const {
    const int kc = k & (ZB - 1);
    return kc < jb ? (k < ZB ? re : im)[(long)kc * ld + col] : 0.0;
  }
};

// Trailing update after the complex block [j0, j0 + jb), with c0 = j0 + jb:
//   region 0: M22 -= C21 C21^T on rows [c0, rows), columns up to each row
//             block's diagonal tile (the lower part; U = C21^T from the upper
//             part of the planes);
//   region 1: B2 -= C21 G1 on G's rows [c0, rows), columns [0, c0).
// Each plane is a real rank-64 update with the stacked U [Ur; Ui] and sL holding
// [-C21r | C21i] (real plane) or [-C21i | -C21r] (imaginary plane).
// Items: (energy, region x plane x column group, 64-row block).
__global__ __launch_bounds__(256, 2) void k_zs_update(int j0, const int *__restrict__ dims, double *__restrict__ aug,
                                                   long ldaug, long strideA, long roff, double *__restrict__ gre,
                                                   double *__restrict__ gim, long ldg, long strideG, int tiles_m,
                                                   int groups, int ne) {
  __shared__ double sL[TILE][Pitch<ZK>::A];
  __shared__ double sU[ZK][PB];
  for_items(ne, tiles_m * groups * 4, [&](int e, int it) {
    const int tmi = it % tiles_m, rest = it / tiles_m;
    const int g = rest % groups, kind = rest / groups;
    const int plane = kind & 1, region = kind >> 1;
    const int rows = dims[2 * e];
    if (j0 >= rows) return;
    const int jb = min(ZB, rows - j0);
    const int c0 = j0 + jb, m = rows - c0, r0 = tmi * TILE, vbeg = g * UPD_G * TILE;
    if (r0 >= m) return;
    const int ncols = region == 0 ? min(m, r0 + TILE) : c0;
    if (vbeg >= ncols) return;
    double *A = aug + (size_t)e * strideA;
    for (int idx = threadIdx.x; idx < ZK * TILE; idx += 256) {
      const int i = idx / ZK, k = idx % ZK, kc = k & (ZB - 1);
      double x = 0.0;
      if (r0 + i < m && kc < jb) {
        const double *c = A + (size_t)(c0 + r0 + i) * ldaug + j0 + kc;
        if (plane == 0)
          x = k < ZB ? -c[0] : c[roff];
        else
          x = k < ZB ? -c[roff] : -c[0];
      }
      sL[i][k] = x;
    }
    if (region == 0) {
      const double *U = A + (size_t)j0 * ldaug;
      rowblock_update<ZK, UPD_G>(sL, sU, m - r0, vbeg, ncols, ColMap{ncols, c0, 0},
                                 A + (size_t)(c0 + r0) * ldaug + (plane ? roff : 0), ZRowsU{U, U + roff, ldaug, jb},
                                 ldaug);
    } else {
      double *Gr = gre + (size_t)e * strideG, *Gi = gim + (size_t)e * strideG;
      rowblock_update<ZK, UPD_G>(sL, sU, m - r0, vbeg, ncols, ColMap{ncols, 0, 0},
                                 (plane ? Gi : Gr) + (size_t)(c0 + r0) * ldg,
                                 ZRowsU{Gr + (size_t)j0 * ldg, Gi + (size_t)j0 * ldg, ldg, jb}, ldg);
    }
  });
}

void launch_zs_factor(hipStream_t s, int ne, int maxrows, const int *dims, double *aug, long ldaug, long strideA,
                      long roff, double *gre, double *gim, long ldg, long strideG, double *zinv, int *status) {
  for (int j0 = 0; j0 < maxrows; j0 += ZB) {
    hipLaunchKernelGGL(k_zs_diag, dim3(ne), dim3(256), 0, s, j0, dims, aug, ldaug, strideA, roff, gre, gim, ldg,
                       strideG, zinv, status);
    const int c0 = std::min(maxrows, j0 + ZB), m = maxrows - c0;
    if (m > 0) {
      const int tm = (m + TILE - 1) / TILE;
      hipLaunchKernelGGL(k_zs_panel, dim3(persist_grid(k_zs_panel, 256, ne, tm)), dim3(256), 0, s, j0, dims, aug,
                         ldaug, strideA, roff, zinv, tm, ne);
    }
    if (j0 > 0) {
      const int tn = (j0 + TILE - 1) / TILE;
      hipLaunchKernelGGL(k_zs_rhs, dim3(persist_grid(k_zs_rhs, 256, ne, tn)), dim3(256), 0, s, j0, dims, gre, gim,
                         ldg, strideG, zinv, tn, ne);
    }
    if (m > 0) {
      const int tm = (m + TILE - 1) / TILE, gr = (std::max(m, c0) + UPD_G * TILE - 1) / (UPD_G * TILE);
      hipLaunchKernelGGL(k_zs_update, dim3(persist_grid(k_zs_update, 256, ne, (long)tm * gr * 4)), dim3(256), 0, s,
                         j0, dims, aug, ldaug, strideA, roff, gre, gim, ldg, strideG, tm, gr, ne);
    }
  }
}

// M^-1 = G^T G (complex, G lower triangular) in 128 x 128 output tiles of the
// lower triangle, mirrored, written over the planes of aug:
//   Re = Gr^T Gr - Gi^T Gi,   Im = Gr^T Gi + Gi^T Gr.
// Eight waves per workgroup, each owning a 64 x 32 block of both parts; K slabs
// of 16 are staged through LDS with the next slab loaded into registers while
// the current one is multiplied.  Because G_ki = 0 for k < i, a tile of rows
// [r0, r0 + 128) sums over k >= r0 only.
__global__ __launch_bounds__(512, 1) void k_zs_gtg(const int *__restrict__ dims, const double *__restrict__ gre,
                                                   const double *__restrict__ gim, long ldg, long strideG,
                                                   double *__restrict__ aug, long ldaug, long strideA, long roff,
                                                   int tiles_n, int ne) {
  constexpr int BT = 2 * TILE, GK = 16, NT = 512;
  constexpr int NL = BT * GK / NT;  // slab elements per thread and operand
  __shared__ double sar[BT][Pitch<GK>::A], sai[BT][Pitch<GK>::A];  // [i][k] = G[k0 + k][r0 + i]
  __shared__ double sbr[GK][BT], sbi[GK][BT];                      // [k][j] = G[k0 + k][q0 + j]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // 2 x 4 waves: rows wr*64, columns wc*32
  const int kk = lane >> 4, ii = lane & 15;
  for_items(ne, tiles_n * tiles_n, [&](int e, int it) {
    const int n = dims[2 * e];
    const int tm = it / tiles_n, tn = it % tiles_n;
    const int r0 = tm * BT, q0 = tn * BT;
    if (r0 >= n || q0 >= n || tn > tm) return;
    const double *Gr = gre + (size_t)e * strideG, *Gi = gim + (size_t)e * strideG;
    double ar[NL], ai[NL], br[NL], bi[NL];
    auto gload = [&](int k0) {
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int idx = t + NT * q;
        const int c = idx % BT, k = k0 + idx / BT;
        const bool kin = k < n;
        const size_t ra = (size_t)k * ldg + r0 + c, rb = (size_t)k * ldg + q0 + c;
        const bool aok = kin && r0 + c < n, bok = kin && q0 + c < n;
        ar[q] = aok ? Gr[ra] : 0.0;
        ai[q] = aok ? Gi[ra] : 0.0;
        br[q] = bok ? Gr[rb] : 0.0;
        bi[q] = bok ? Gi[rb] : 0.0;
      }
    };
    d4 accr[8], acci[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      accr[q] = d4{0, 0, 0, 0};
      acci[q] = d4{0, 0, 0, 0};
    }
    gload(r0);
    for (int k0 = r0; k0 < n; k0 += GK) {
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int idx = t + NT * q;
        sar[idx % BT][idx / BT] = ar[q];
        sai[idx % BT][idx / BT] = ai[q];
        sbr[idx / BT][idx % BT] = br[q];
        sbi[idx / BT][idx % BT] = bi[q];
      }
      __syncthreads();
      if (k0 + GK < n) gload(k0 + GK);
#pragma unroll
      for (int ks = 0; ks < GK; ks += 4) {
        double xr[4], xi[4], yr[2], yi[2];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          xr[m] = sar[wr * 64 + m * 16 + ii][ks + kk];
          xi[m] = sai[wr * 64 + m * 16 + ii][ks + kk];
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          yr[m] = sbr[ks + kk][wc * 32 + m * 16 + ii];
          yi[m] = sbi[ks + kk][wc * 32 + m * 16 + ii];
        }
        // the two products of each accumulator are issued 16 MFMAs apart
#pragma unroll
        for (int mr = 0; mr < 4; ++mr)
#pragma unroll
          for (int mc = 0; mc < 2; ++mc) {
            accr[mr * 2 + mc] = mfma64(xr[mr], yr[mc], accr[mr * 2 + mc]);
            acci[mr * 2 + mc] = mfma64(xr[mr], yi[mc], acci[mr * 2 + mc]);
          }
#pragma unroll
        for (int mr = 0; mr < 4; ++mr)
#pragma unroll
          for (int mc = 0; mc < 2; ++mc) {
            accr[mr * 2 + mc] = mfma64(-xi[mr], yi[mc], accr[mr * 2 + mc]);
            acci[mr * 2 + mc] = mfma64(xi[mr], yr[mc], acci[mr * 2 + mc]);
          }
      }
      __syncthreads();
    }
    double *A = aug + (size_t)e * strideA;
#pragma unroll
    for (int mr = 0; mr < 4; ++mr)
#pragma unroll
      for (int mc = 0; mc < 2; ++mc) {
        const int j = q0 + wc * 32 + mc * 16 + ii;
        if (j >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = r0 + wr * 64 + mr * 16 + 4 * v + kk;
          if (i < n) {
            const double xr = accr[mr * 2 + mc][v], xi = acci[mr * 2 + mc][v];
            A[(size_t)i * ldaug + j] = xr;
            A[(size_t)i * ldaug + roff + j] = xi;
            if (tm != tn) {
              A[(size_t)j * ldaug + i] = xr;
              A[(size_t)j * ldaug + roff + i] = xi;
            }
          }
        }
      }
  });
}

void launch_zs_setup(hipStream_t s, const Lay &L, const int *nopen, const double *Kw, double *aug, double *gre,
                     double *gim, int *dims) {
  const int nt32 = (L.nmax + 31) / 32;
  hipLaunchKernelGGL(k_zs_setup, dim3(nt32 * (nt32 + 1) / 2, L.ne), dim3(256), 0, s, nopen, Kw, L.ldk, L.sK, aug,
                     L.ldaug, L.sA, L.roff, gre, gim, L.ldk, L.sK, dims);
}

void launch_zs_inverse(hipStream_t s, const Lay &L, const int *dims, double *aug, double *gre, double *gim,
                       double *zinv, int *status) {
  if (L.nmax <= 0) return;
  launch_zs_factor(s, L.ne, L.nmax, dims, aug, L.ldaug, L.sA, L.roff, gre, gim, L.ldk, L.sK, zinv, status);
  const int tn = (L.nmax + 2 * TILE - 1) / (2 * TILE);
  hipLaunchKernelGGL(k_zs_gtg, dim3(persist_grid(k_zs_gtg, 512, L.ne, (long)tn * tn)), dim3(512), 0, s, dims, gre,
                     gim, L.ldk, L.sK, aug, L.ldaug, L.sA, L.roff, tn, L.ne);
}

// ---------------------------------------------------------------------------
// K gather, collision strengths
// ---------------------------------------------------------------------------
// K from the solution: the last nopen rows of Y (the open unknowns) as solved
// (not symmetrised; the S/Omega stage symmetrises its own copy), with zeros for
// i or j in [nopen, n); also dims = {nopen, nopen} for the S/Omega stage.
__global__ __launch_bounds__(256) void k_gatherK(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                 const int *__restrict__ nopen, const double *__restrict__ aug,
                                                 long ldaug, long strideA, long roff, double *__restrict__ Kw, long ldk,
                                                 long strideK, int *__restrict__ dims) {
  const int e = blockIdx.y, i = blockIdx.x;
  const int n = tab[pwi[e]].n, no = nopen[e];
  if (i == 0 && threadIdx.x == 0) {
    dims[2 * e] = no;
    dims[2 * e + 1] = no;
  }
  if (i >= n) return;
  const double *Y = aug + (size_t)e * strideA + (size_t)(n - no + i) * ldaug + roff;
  double *K = Kw + (size_t)e * strideK + (size_t)i * ldk;
  for (int j = threadIdx.x; j < n; j += 256) K[j] = (i < no && j < no) ? Y[j] : 0.0;
}

void launch_gatherK(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen,
                    const double *aug, double *Kw, int *dims) {
  hipLaunchKernelGGL(k_gatherK, dim3(L.nmax, L.ne), dim3(256), 0, s, tab, pwi, nopen, aug, L.ldaug, L.sA, L.roff, Kw,
                     L.ldk, L.sK, dims);
}


// Omega_pq for one energy and one target row p per wave; lanes stride over q.
// |T_ij|^2 = 4 |(M^-1)_ij - d_ij|^2 with the real and imaginary parts of M^-1 in
// X and Y.  Each entry sums its channel pairs in a fixed order (no atomics), so
// results do not depend on scheduling.
__global__ __launch_bounds__(64) void k_omega(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                              const int *__restrict__ openpos, long ldo,
                                              const double *__restrict__ X, const double *__restrict__ Y, long ldx,
                                              long sX, double *__restrict__ omega, int ntmax) {
  const int pt = blockIdx.x, e = blockIdx.y;
  const DevPW &pw = tab[pwi[e]];
  const int nt = pw.nt;
  if (pt >= nt) return;
  const double half_g = 0.5 * pw.g;
  const int *tptr = pw.tptr, *tch = pw.tch;
  const int *pos = openpos + (size_t)e * ldo;
  const double *Xe = X + (size_t)e * sX;
  const double *Ye = Y + (size_t)e * sX;
  for (int q = threadIdx.x; q < nt; q += 64) {
    double acc = 0.0;
    for (int a = tptr[pt]; a < tptr[pt + 1]; ++a) {
      const int i = pos[tch[a]];
      if (i < 0) continue;
      for (int b = tptr[q]; b < tptr[q + 1]; ++b) {
        const int j = pos[tch[b]];
        if (j < 0) continue;
        const double x = Xe[(size_t)i * ldx + j] - (i == j ? 1.0 : 0.0), y = Ye[(size_t)i * ldx + j];
        acc += 4.0 * (x * x + y * y);
      }
    }
    omega[((size_t)e * ntmax + pt) * ntmax + q] = half_g * acc;
  }
}

// S = 2 M^-1 - 1 on the leading no x no block, zero elsewhere
__global__ void k_smatrix(const DevPW *__restrict__ tab, const int *__restrict__ pwi, const int *__restrict__ nopen,
                          const double *__restrict__ X, const double *__restrict__ Y, long ldx, long sX,
                          double *__restrict__ S, int nmax) {
  const int e = blockIdx.z, i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = tab[pwi[e]].n;
  if (i >= n || j >= n) return;
  const int no = nopen[e];
  double re = 0.0, im = 0.0;
  if (i < no && j < no) {
    re = 2.0 * X[(size_t)e * sX + (size_t)i * ldx + j] - (i == j ? 1.0 : 0.0);
    im = 2.0 * Y[(size_t)e * sX + (size_t)i * ldx + j];
  }
  double *o = S + (((size_t)e * nmax + i) * nmax + j) * 2;
  o[0] = re;
  o[1] = im;
}

void launch_omega(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *openpos,
                  const int *nopen, const double *X, const double *Y, double *omega, double *S) {
  hipLaunchKernelGGL(k_omega, dim3(L.ntmax, L.ne), dim3(64), 0, s, tab, pwi, openpos, L.ldo, X, Y, L.ldaug, L.sA,
                     omega, L.ntmax);
  if (S)
    hipLaunchKernelGGL(k_smatrix, dim3((L.nmax + 63) / 64, L.nmax, L.ne), dim3(64), 0, s, tab, pwi, nopen, X, Y,
                       L.ldaug, L.sA, S, L.nmax);
}

// Flag non-finite results and overwrite the outputs of flagged energies with NaN.
__global__ __launch_bounds__(256) void k_finalize(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                  int *__restrict__ status, double *__restrict__ omega, int ntmax,
                                                  double *__restrict__ K, long ldk, long strideK,
                                                  double *__restrict__ S, int nmax) {
  const int e = blockIdx.x;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n, nt = p.nt;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  if (omega)
    for (int t = threadIdx.x; t < nt * nt; t += 256)
      if (!isfinite(omega[(size_t)e * ntmax * ntmax + (t / nt) * ntmax + t % nt])) mine = 1;
  if (mine) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0 && bad) status[e] |= RM_PT_NONFINITE;
  __syncthreads();
  if (status[e] == 0) return;
  const double nan = __builtin_nan("");
  if (omega)
    for (int t = threadIdx.x; t < nt * nt; t += 256) omega[(size_t)e * ntmax * ntmax + (t / nt) * ntmax + t % nt] = nan;
  if (K)
    for (long t = threadIdx.x; t < (long)n * n; t += 256) K[(size_t)e * strideK + (t / n) * ldk + t % n] = nan;
  if (S)
    for (long t = threadIdx.x; t < (long)n * n; t += 256) {
      double *o = S + (((size_t)e * nmax + t / n) * nmax + t % n) * 2;
      o[0] = nan;
      o[1] = nan;
    }
}

void launch_finalize(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, int *status, double *omega,
                     double *K, double *S) {
  hipLaunchKernelGGL(k_finalize, dim3(L.ne), dim3(256), 0, s, tab, pwi, status, omega, L.ntmax, K, L.ldk, L.sK, S,
                     L.nmax);
}

// p[0 .. n) = v (a fill kernel: stream-captured graphs keep no memset nodes).
__global__ void k_fill_int(int *__restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_int(hipStream_t s, int *p, int n, int v) {
  if (n > 0) hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

__global__ void k_setdims(const DevPW *__restrict__ tab, const int *__restrict__ pwi, int ne,
                          const int *__restrict__ nopen, int *__restrict__ dims) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  dims[2 * e] = tab[pwi[e]].n;
  dims[2 * e + 1] = nopen[e];
}

void launch_setdims(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen, int *dims) {
  hipLaunchKernelGGL(k_setdims, dim3((L.ne + 127) / 128), dim3(128), 0, s, tab, pwi, L.ne, nopen, dims);
}

// Flags of the staged calls that take R, fg or K from the caller: energies within
// thr of a threshold, and non-finite inputs.
__global__ __launch_bounds__(256) void k_check_inputs(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                      const double *__restrict__ E, double thr,
                                                      const double *__restrict__ R, long ldr, long strideR,
                                                      const double *__restrict__ fg, long ldo,
                                                      const double *__restrict__ K, long ldk, long strideK,
                                                      const int *__restrict__ nopen, int *__restrict__ status) {
  const int e = blockIdx.x;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n;
  __shared__ int flags;
  if (threadIdx.x == 0) flags = 0;
  __syncthreads();
  int f = 0;
  const double Ev = E[e];
  for (int i = threadIdx.x; i < n; i += 256)
    if (fabs(Ev - p.ethr[i]) < thr) f |= RM_PT_THRESHOLD;
  if (R)
    for (long t = threadIdx.x; t < (long)n * n; t += 256)
      if (!isfinite(R[(size_t)e * strideR + (t / n) * ldr + t % n])) f |= RM_PT_NONFINITE;
  if (fg)
    for (long t = threadIdx.x; t < 4L * n; t += 256)
      if (!isfinite(fg[(size_t)e * ldo * 4 + t])) f |= RM_PT_NONFINITE;
  if (K) {
    const int no = nopen[e];
    for (long t = threadIdx.x; t < (long)no * no; t += 256)
      if (!isfinite(K[(size_t)e * strideK + (t / no) * ldk + t % no])) f |= RM_PT_NONFINITE;
  }
  if (f) atomicOr(&flags, f);
  __syncthreads();
  if (threadIdx.x == 0 && flags) atomicOr(status + e, flags);
}

void launch_check_inputs(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                         double thr, const double *R, const double *fg, const double *K, const int *nopen,
                         int *status) {
  hipLaunchKernelGGL(k_check_inputs, dim3(L.ne), dim3(256), 0, s, tab, pwi, E, thr, R, L.ldaug, L.sA, fg, L.ldo, K,
                     L.ldk, L.sK, nopen, status);
}

// Sum over partial waves: one thread per (energy, p, q) element, waves added in
// ascending order.
__global__ void k_sum_waves(int npw, long per, int ne, const double *__restrict__ om, const int32_t *__restrict__ st,
                            double *__restrict__ sum, int32_t *__restrict__ sst) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < per) {
    double acc = 0.0;
    for (int w = 0; w < npw; ++w) acc += om[(size_t)w * per + idx];
    sum[idx] = acc;
  }
  if (idx < ne) {
    int32_t f = 0;
    for (int w = 0; w < npw; ++w) f |= st[(size_t)w * ne + idx];
    sst[idx] = f;
  }
}

void launch_sum_waves(hipStream_t s, int npw, int ne, int nt, const double *om, const int32_t *st, double *sum,
                      int32_t *sst) {
  const long per = (long)ne * nt * nt;
  const long n = std::max<long>(per, ne);
  hipLaunchKernelGGL(k_sum_waves, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, npw, per, ne, om, st, sum, sst);
}

// Output packing: energy e's leading block goes to pack + off[e], row-major.
__global__ void k_pack(const DevPW *__restrict__ tab, const int *__restrict__ pwi, int what,
                       const double *__restrict__ src, long ld, long stride, const long *__restrict__ off,
                       double *__restrict__ pack) {
  const int e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  const int w = what == 0 ? p.nt : p.n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)w * w; t += (long)gridDim.x * blockDim.x)
    pack[off[e] + t] = src[(size_t)e * stride + (t / w) * ld + t % w];
}

void launch_pack(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, int what, const double *src,
                 const long *off, double *pack) {
  const long ld = what == 0 ? L.ntmax : L.ldk;
  const long stride = what == 0 ? L.sOm : L.sK;
  hipLaunchKernelGGL(k_pack, dim3(32, L.ne), dim3(256), 0, s, tab, pwi, what, src, ld, stride, off, pack);
}

}  // namespace rm
