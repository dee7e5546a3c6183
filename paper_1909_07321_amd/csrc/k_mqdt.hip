// k_mqdt.hip -- multichannel quantum-defect operation on the fine mesh.
//
// PSTGF paper, section "Code Structure", stgf namelist, MQDT variables: with
// iqdt = 1 every member channel is treated as open and the unphysical K is
// computed on a coarse mesh (every |ieq|-th point, imode = -1); the fine mesh
// is solved by interpolation.  A member channel is open or closed with
// effective quantum number nu >= max(fnumin, l + 0.1) (iomsw = 1).  Closed
// member channels carry the energy-analytic Coulomb pair (f, g) whose
// decaying combination is f cos(pi nu) - g sin(pi nu) (k_asym.hip), so at a
// fine energy the closed members are eliminated by
//   K = Ku_oo - Ku_oc (Ku_cc + tan(pi nu))^-1 Ku_co.
// Between coarse points the unphysical S is interpolated by default (iqdt = 1),
// not the unphysical K, which has poles (an eigenphase through pi/2; iqdt = 2
// interpolates K itself and skips the recovery): the coarse step keeps
// X + iY = (1 - i Ku)^-1 = (1 + S)/2 (bounded), the fine step interpolates X
// and Y elementwise and recovers Ku = Y X^-1 by one batched LU of the member
// count with the full back substitution (k_mqdt_interp, k_mqdt_take).
// K is then the tail of the solution of one linear system of the member
// count m = n_c + n_o, unknowns ordered [X (closed members) | K (open)]:
//   [ Ku_cc + tan(pi nu)  0 ] [X]   [Ku_co]
//   [ Ku_oc               1 ] [K] = [Ku_oo],
// which the batched LU with its tail back substitution solves unchanged
// (k_linalg.hip): K is the last n_o rows, as in the physical path.
#include "k_common.h"
#include "k_mqdt.h"
#include "rm.h"

namespace rm {

// Member count and flags (threshold, pole) of every energy of a mesh: one
// thread per energy.  Poles are ascending, so a pole equal to E is found by
// bisection.  MQDT_NEAR_INT is added to the flags where a closed member's
// |sin(pi nu)| < 1e-6 (its g cancels there; the host does not take such a
// point as a coarse point).
__global__ void k_mqdt_count(const double *__restrict__ ethr, const int *__restrict__ l,
                             const double *__restrict__ Ek, int n, int M, double z, const double *__restrict__ E,
                             int ne, double fnumin, double thr_guard, int *__restrict__ nmem, int *__restrict__ flag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double Ev = E[e];
  int m = 0, st = 0;
  for (int i = 0; i < n; ++i) {
    const double eps = Ev - ethr[i];
    const bool mem = mqdt_member(z, eps, l[i], fnumin);
    m += mem;
    if (fabs(eps) < thr_guard) st |= RM_PT_THRESHOLD;
    if (mem && eps < 0 && fabs(sinpi(z / sqrt(-eps))) < 1e-6) st |= MQDT_NEAR_INT;
  }
  int lo = 0, hi = M;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Ek[mid] < Ev) lo = mid + 1;
    else hi = mid;
  }
  if (lo < M && Ek[lo] == Ev) st |= RM_PT_POLE;
  nmem[e] = m;
  flag[e] = st;
}

void launch_mqdt_count(hipStream_t s, const DevPW *pw, const double *E, int ne, double fnumin, double thr_guard,
                       int *nmem, int *flag) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(k_mqdt_count, dim3((ne + 127) / 128), dim3(128), 0, s, pw->ethr, pw->l, pw->Ek, pw->n, pw->M,
                     pw->z, E, ne, fnumin, thr_guard, nmem, flag);
}

// Per energy of a chunk (one workgroup): each member channel's row and column
// in the system above (syspos: closed members first, then open channels, each
// in ascending channel order; -1 for other channels), its index in the
// unphysical K (spos: ascending over the members), tan(pi nu) of closed
// members, dims = {m, n_o}, nsys = m; threshold and pole flags are or-ed into
// status.  The three counts are scanned together, packed 21 bits apiece.
__global__ __launch_bounds__(256) void k_mqdt_setup(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                    const double *__restrict__ E, long ldo, double fnumin,
                                                    double thr_guard, int *__restrict__ syspos,
                                                    int *__restrict__ spos, double *__restrict__ tanv,
                                                    int *__restrict__ dims, int *__restrict__ nsys,
                                                    int *__restrict__ status, int *__restrict__ clist,
                                                    int *__restrict__ olist, int *__restrict__ cch) {
  __shared__ long long cnt[256];
  __shared__ int flag;
  const int e = blockIdx.x, t = threadIdx.x;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n;
  const double Ev = E[e], z = p.z;
  const int per = (n + 255) / 256;
  const int c0 = min(n, t * per), c1 = min(n, c0 + per);
  constexpr long long ONE_O = 1LL << 21, ONE_M = 1LL << 42, MASK = (1LL << 21) - 1;
  long long c = 0;
  int st = 0;
  for (int i = c0; i < c1; ++i) {
    const double eps = Ev - p.ethr[i];
    if (mqdt_member(z, eps, p.l[i], fnumin)) c += (eps > 0 ? ONE_O : 1LL) + ONE_M;
    if (fabs(eps) < thr_guard) st |= RM_PT_THRESHOLD;
  }
  if (t == 0) {
    flag = 0;
    int lo = 0, hi = p.M;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (p.Ek[mid] < Ev) lo = mid + 1;
      else hi = mid;
    }
    if (lo < p.M && p.Ek[lo] == Ev) st |= RM_PT_POLE;
  }
  cnt[t] = c;
  __syncthreads();
  if (st) atomicOr(&flag, st);
  for (int off = 1; off < 256; off <<= 1) {
    const long long v = t >= off ? cnt[t - off] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  const long long tot = cnt[255], mine = cnt[t] - c;
  const int ncm = (int)(tot & MASK), nop = (int)((tot >> 21) & MASK), nm = (int)(tot >> 42);
  int pc = (int)(mine & MASK), po = (int)((mine >> 21) & MASK), pm = (int)(mine >> 42);
  int *sp = syspos + (size_t)e * ldo, *mp = spos + (size_t)e * ldo;
  double *tv = tanv + (size_t)e * ldo;
  for (int i = c0; i < c1; ++i) {
    const double eps = Ev - p.ethr[i];
    if (!mqdt_member(z, eps, p.l[i], fnumin)) {
      sp[i] = -1;
      mp[i] = -1;
      tv[i] = 0.0;
      continue;
    }
    if (clist) {
      if (eps > 0) {
        olist[(size_t)e * ldo + po] = pm;
      } else {
        clist[(size_t)e * ldo + pc] = pm;
        cch[(size_t)e * ldo + pc] = i;
      }
    }
    mp[i] = pm++;
    if (eps > 0) {
      sp[i] = ncm + po++;
      tv[i] = 0.0;
    } else {
      sp[i] = pc++;
      const double nu = z / sqrt(-eps);
      tv[i] = sinpi(nu) / cospi(nu);
    }
  }
  __syncthreads();
  if (t == 0) {
    dims[2 * e] = nm;
    dims[2 * e + 1] = nop;
    nsys[e] = nm;
    if (flag) status[e] |= flag;
  }
}

void launch_mqdt_setup_lists(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                             double thr_guard, int *syspos, int *spos, double *tanv, int *dims, int *nsys, int *status,
                             int *clist, int *olist, int *cch) {
  hipLaunchKernelGGL(k_mqdt_setup, dim3(L.ne), dim3(256), 0, s, tab, pwi, E, L.ldo, L.fnumin, thr_guard, syspos, spos,
                     tanv, dims, nsys, status, clist, olist, cch);
}

void launch_mqdt_setup(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                       double thr_guard, int *syspos, int *spos, double *tanv, int *dims, int *nsys, int *status) {
  launch_mqdt_setup_lists(s, L, tab, pwi, E, thr_guard, syspos, spos, tanv, dims, nsys, status, nullptr, nullptr,
                          nullptr);
}

// ---------------------------------------------------------------------------
// Elimination in S form (Omega only).  With the unphysical S = 2(X + iY) - 1 of
// the interpolated X + iY = (1 - i Ku)^-1 and the decaying combination
// f cos(pi nu) - g sin(pi nu) of a closed member, the open-channel S is
//   S = S_oo + S_oc (e^{-2 pi i nu} - S_cc)^-1 S_co,
// and Omega follows from |S - 1|^2 (the S/Omega stage's k_omega, fed with
// (S + 1)/2).  clist / olist: member positions of the closed / open members
// in ascending order; cch: the closed members' channels.

// X + iY at (member row r, member column c) interpolated over the energy's
// coarse points
struct Interp {
  const double *xq[4], *yq[4];
  double wq[4];
  long n;
  __device__ __forceinline__ void at(int r, int c, double &x, double &y) const {
    x = 0.0;
    y = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t o = (size_t)r * n + c;
      x += wq[q] * xq[q][o];
      y += wq[q] * yq[q][o];
    }
  }
};

__device__ __forceinline__ Interp make_interp(const double *Xc, const double *Yc, const int *cidx, const double *cw,
                                              int e, int n) {
  Interp I;
  I.n = n;
  const size_t nn = (size_t)n * n;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = cidx[4 * e + q];
    I.wq[q] = c >= 0 ? cw[4 * e + q] : 0.0;
    I.xq[q] = Xc + (c >= 0 ? c : 0) * nn;
    I.yq[q] = Yc + (c >= 0 ? c : 0) * nn;
  }
  return I;
}

// W = (e^{-2 pi i nu} - S_cc)^-1, n_c <= MQDT_SMAX, one workgroup per energy:
// in-place Gauss-Jordan with partial pivoting on the complex matrix in LDS,
// the row interchanges undone on the columns at the end.  W [e][SMAX][SMAX]
// as two planes.
__global__ __launch_bounds__(256) void k_mqdt_sinv(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                   const double *__restrict__ E, const int *__restrict__ nsys,
                                                   const int *__restrict__ nopen, const int *__restrict__ clist,
                                                   const int *__restrict__ cch, long ldo,
                                                   const double *__restrict__ Xc, const double *__restrict__ Yc,
                                                   const int *__restrict__ cidx, const double *__restrict__ cw,
                                                   const int *__restrict__ status, double *__restrict__ Wr,
                                                   double *__restrict__ Wi) {
  constexpr int SM = MQDT_SMAX;
  __shared__ double Ar[SM][SM + 1], Ai[SM][SM + 1];
  __shared__ int perm[SM], piv_s;
  const int e = blockIdx.x, t = threadIdx.x;
  const int nc = nsys[e] - nopen[e];
  if (status[e] || nc <= 0 || nc > SM) return;
  const DevPW &p = tab[pwi[e]];
  const Interp I = make_interp(Xc, Yc, cidx, cw, e, p.n);
  const int *cl = clist + (size_t)e * ldo;
  for (int idx = t; idx < nc * nc; idx += 256) {
    const int k = idx / nc, l = idx % nc;
    double x, y;
    I.at(cl[k], cl[l], x, y);
    double re = -(2.0 * x - (k == l ? 1.0 : 0.0)), im = -2.0 * y;
    if (k == l) {
      const double nu = p.z / sqrt(p.ethr[cch[(size_t)e * ldo + k]] - E[e]);
      re += cospi(2.0 * nu);
      im -= sinpi(2.0 * nu);
    }
    Ar[k][l] = re;
    Ai[k][l] = im;
  }
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    if (t == 0) {
      int pr = c;
      double best = Ar[c][c] * Ar[c][c] + Ai[c][c] * Ai[c][c];
      for (int r = c + 1; r < nc; ++r) {
        const double v = Ar[r][c] * Ar[r][c] + Ai[r][c] * Ai[r][c];
        if (v > best) best = v, pr = r;
      }
      piv_s = pr;
      perm[c] = pr;
    }
    __syncthreads();
    const int pr = piv_s;
    if (pr != c)
      for (int j = t; j < nc; j += 256) {
        double a = Ar[c][j], b = Ai[c][j];
        Ar[c][j] = Ar[pr][j];
        Ai[c][j] = Ai[pr][j];
        Ar[pr][j] = a;
        Ai[pr][j] = b;
      }
    __syncthreads();
    // 1 / pivot, then row c scaled with the pivot entry replaced by 1
    const double pr_ = Ar[c][c], pi_ = Ai[c][c];
    const double d = pr_ * pr_ + pi_ * pi_;
    const double ir = pr_ / d, ii = -pi_ / d;
    __syncthreads();
    for (int j = t; j < nc; j += 256) {
      const double a = j == c ? 1.0 : Ar[c][j], b = j == c ? 0.0 : Ai[c][j];
      Ar[c][j] = a * ir - b * ii;
      Ai[c][j] = a * ii + b * ir;
    }
    __syncthreads();
    // other rows: row r -= f row c with f = A[r][c] (its column-c entry becomes -f / pivot)
    for (int idx = t; idx < nc * nc; idx += 256) {
      const int r = idx / nc, j = idx % nc;
      if (r == c) continue;
      const double fr = Ar[r][c], fi = Ai[r][c];
      if (j == c) continue;
      const double ar = Ar[c][j], ai = Ai[c][j];
      Ar[r][j] -= fr * ar - fi * ai;
      Ai[r][j] -= fr * ai + fi * ar;
    }
    __syncthreads();
    for (int r = t; r < nc; r += 256) {
      if (r == c) continue;
      const double fr = Ar[r][c], fi = Ai[r][c];
      // the column of the inverse: -f * (1 / pivot) = -f * A[c][c] (already 1/pivot)
      const double cr = Ar[c][c], ci = Ai[c][c];
      Ar[r][c] = -(fr * cr - fi * ci);
      Ai[r][c] = -(fr * ci + fi * cr);
    }
    __syncthreads();
  }
  // undo the interchanges on the columns, last first
  for (int c = nc - 1; c >= 0; --c) {
    const int pr = perm[c];
    if (pr != c)
      for (int r = t; r < nc; r += 256) {
        double a = Ar[r][c], b = Ai[r][c];
        Ar[r][c] = Ar[r][pr];
        Ai[r][c] = Ai[r][pr];
        Ar[r][pr] = a;
        Ai[r][pr] = b;
      }
    __syncthreads();
  }
  double *wr = Wr + (size_t)e * SM * SM, *wi = Wi + (size_t)e * SM * SM;
  for (int idx = t; idx < nc * nc; idx += 256) {
    const int k = idx / nc, l = idx % nc;
    wr[k * SM + l] = Ar[k][l];
    wi[k * SM + l] = Ai[k][l];
  }
}

// Z = W S_co, stored as Zt [e][n][SMAX] (open position major) in two planes;
// one thread per open position.
__global__ __launch_bounds__(256) void k_mqdt_sz(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                 const int *__restrict__ nsys, const int *__restrict__ nopen,
                                                 const int *__restrict__ clist, const int *__restrict__ olist,
                                                 long ldo, const double *__restrict__ Xc,
                                                 const double *__restrict__ Yc, const int *__restrict__ cidx,
                                                 const double *__restrict__ cw, const int *__restrict__ status,
                                                 const double *__restrict__ Wr, const double *__restrict__ Wi,
                                                 double *__restrict__ Zr, double *__restrict__ Zi, long ldz) {
  constexpr int SM = MQDT_SMAX, KB = 16;
  const int e = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  const int no = nopen[e], nc = nsys[e] - no;
  if (status[e] || j >= no || nc <= 0 || nc > SM) return;
  const DevPW &p = tab[pwi[e]];
  const Interp I = make_interp(Xc, Yc, cidx, cw, e, p.n);
  const int *cl = clist + (size_t)e * ldo;
  const int oj = olist[(size_t)e * ldo + j];
  const double *wr = Wr + (size_t)e * SM * SM, *wi = Wi + (size_t)e * SM * SM;
  double *zr = Zr + ((size_t)e * ldz + j) * SM, *zi = Zi + ((size_t)e * ldz + j) * SM;
  for (int k0 = 0; k0 < nc; k0 += KB) {
    double ar[KB], ai[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) ar[k] = ai[k] = 0.0;
    for (int l = 0; l < nc; ++l) {
      double x, y;
      I.at(cl[l], oj, x, y);
      const double sr = 2.0 * x, si = 2.0 * y;  // S_co: off the diagonal
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (k0 + k >= nc) break;
        const double vr = wr[(k0 + k) * SM + l], vi = wi[(k0 + k) * SM + l];
        ar[k] += vr * sr - vi * si;
        ai[k] += vr * si + vi * sr;
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
      if (k0 + k < nc) {
        zr[k0 + k] = ar[k];
        zi[k0 + k] = ai[k];
      }
  }
}

// S = S_oo + S_oc Z for open row i (one workgroup per (i, energy)), written as
// (S + 1)/2 over the planes the S/Omega stage leaves for k_omega: real part in
// columns [0, n_o), imaginary part from column roff, row i.
__global__ __launch_bounds__(256) void k_mqdt_som(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                  const int *__restrict__ nsys, const int *__restrict__ nopen,
                                                  const int *__restrict__ clist, const int *__restrict__ olist,
                                                  long ldo, const double *__restrict__ Xc,
                                                  const double *__restrict__ Yc, const int *__restrict__ cidx,
                                                  const double *__restrict__ cw, const int *__restrict__ status,
                                                  const double *__restrict__ Zr, const double *__restrict__ Zi,
                                                  long ldz, double *__restrict__ aug, long ldaug, long strideA,
                                                  long roff) {
  constexpr int SM = MQDT_SMAX;
  __shared__ double br[SM], bi[SM];
  const int i = blockIdx.x, e = blockIdx.y, t = threadIdx.x;
  const int no = nopen[e], nc = nsys[e] - no;
  if (status[e] || i >= no || nc > SM) return;
  const DevPW &p = tab[pwi[e]];
  const Interp I = make_interp(Xc, Yc, cidx, cw, e, p.n);
  const int *cl = clist + (size_t)e * ldo, *ol = olist + (size_t)e * ldo;
  const int oi = ol[i];
  for (int k = t; k < nc; k += 256) {
    double x, y;
    I.at(oi, cl[k], x, y);
    br[k] = 2.0 * x;  // S_oc: off the diagonal
    bi[k] = 2.0 * y;
  }
  __syncthreads();
  double *row = aug + (size_t)e * strideA + (size_t)i * ldaug;
  for (int j = t; j < no; j += 256) {
    double x, y;
    I.at(oi, ol[j], x, y);
    double sr = 2.0 * x - (i == j ? 1.0 : 0.0), si = 2.0 * y;
    const double *zr = Zr + ((size_t)e * ldz + j) * SM, *zi = Zi + ((size_t)e * ldz + j) * SM;
    for (int k = 0; k < nc; ++k) {
      sr += br[k] * zr[k] - bi[k] * zi[k];
      si += br[k] * zi[k] + bi[k] * zr[k];
    }
    row[j] = 0.5 * (sr + (i == j ? 1.0 : 0.0));
    row[roff + j] = 0.5 * si;
  }
}

void launch_mqdt_sform(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                       const int *nsys, const int *nopen, const int *clist, const int *olist, const int *cch,
                       const double *Xc, const double *Yc, const int *cidx, const double *cw, const int *status,
                       double *Wr, double *Wi, double *Zr, double *Zi, double *aug) {
  hipLaunchKernelGGL(k_mqdt_sinv, dim3(L.ne), dim3(256), 0, s, tab, pwi, E, nsys, nopen, clist, cch, L.ldo, Xc, Yc,
                     cidx, cw, status, Wr, Wi);
  hipLaunchKernelGGL(k_mqdt_sz, dim3((L.nmax + 255) / 256, L.ne), dim3(256), 0, s, tab, pwi, nsys, nopen, clist,
                     olist, L.ldo, Xc, Yc, cidx, cw, status, Wr, Wi, Zr, Zi, (long)L.nmax);
  hipLaunchKernelGGL(k_mqdt_som, dim3(L.nmax, L.ne), dim3(256), 0, s, tab, pwi, nsys, nopen, clist, olist, L.ldo, Xc,
                     Yc, cidx, cw, status, Zr, Zi, (long)L.nmax, aug, L.ldaug, L.sA, L.roff);
}

// One workgroup per (member channel i, energy): row spos[i] of the energy's
// unphysical K (Ku, row stride ldk, energy stride sK, members in ascending
// order), written as row syspos[i] of the system and of its right-hand sides;
// dims = {m, n_o}.  An energy already flagged (threshold, pole, or a coarse
// point it depends on) gets the identity system instead, so that the solve
// adds no flags of its own; its outputs are NaN from the flag.
__global__ __launch_bounds__(256) void k_mqdt_build(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                    const int *__restrict__ syspos, const int *__restrict__ spos,
                                                    const double *__restrict__ tanv, const int *__restrict__ nopen,
                                                    const int *__restrict__ nsys, long ldo,
                                                    const double *__restrict__ Ku, long ldk, long sK,
                                                    const int *__restrict__ status, int *__restrict__ dims,
                                                    double *__restrict__ aug, long ldaug, long strideA, long roff) {
  const int i = blockIdx.x, e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n;
  if (i == 0 && threadIdx.x == 0) {
    dims[2 * e] = nsys[e];
    dims[2 * e + 1] = nopen[e];
  }
  if (i >= n) return;
  const int *sp = syspos + (size_t)e * ldo, *mp = spos + (size_t)e * ldo;
  const int ri = sp[i];
  if (ri < 0) return;
  const int ncm = nsys[e] - nopen[e];
  const bool iopen = ri >= ncm;
  const double ti = tanv[(size_t)e * ldo + i];
  const double *krow = Ku + (size_t)e * sK + (size_t)mp[i] * ldk;
  double *row = aug + (size_t)e * strideA + (size_t)ri * ldaug;
  if (status[e]) {
    for (int j = threadIdx.x; j < n; j += 256) {
      const int rj = sp[j];
      if (rj < 0) continue;
      row[rj] = i == j ? 1.0 : 0.0;
      if (rj >= ncm) row[roff + (rj - ncm)] = 0.0;
    }
    return;
  }
  for (int j = threadIdx.x; j < n; j += 256) {
    const int rj = sp[j];
    if (rj < 0) continue;
    const double v = krow[mp[j]];
    const bool jopen = rj >= ncm;
    if (jopen) {
      row[roff + (rj - ncm)] = v;
      row[rj] = (iopen && i == j) ? 1.0 : 0.0;
    } else {
      row[rj] = (!iopen && i == j) ? v + ti : v;
    }
  }
}

void launch_mqdt_build(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *syspos,
                       const int *spos, const double *tanv, const int *nopen, const int *nsys, const double *Ku,
                       const int *status, int *dims, double *aug) {
  hipLaunchKernelGGL(k_mqdt_build, dim3(L.nmax, L.ne), dim3(256), 0, s, tab, pwi, syspos, spos, tanv, nopen, nsys,
                     L.ldo, Ku, L.ldk, L.sK, status, dims, aug, L.ldaug, L.sA, L.roff);
}

// One workgroup per (member channel i, energy): row spos[i] of the
// interpolated planes over the energy's coarse points (cidx < 0: unused),
// X(E) = sum_q w_q X(E_q).  Mode 1 (the unphysical S): X and Y written as
// [X | Y] (X in columns 0..m, Y from column roff), dims = {m, m}; a flagged
// energy gets [1 | 0].  Mode 2 (the unphysical K itself, in Xc): the row
// written into the K workspace; a flagged energy gets 0.  Coarse planes are
// [q][n][n], members in ascending order.
__global__ __launch_bounds__(256) void k_mqdt_interp(int mode, const DevPW *__restrict__ tab,
                                                     const int *__restrict__ pwi, const int *__restrict__ spos,
                                                     const int *__restrict__ nsys, long ldo,
                                                     const double *__restrict__ Xc, const double *__restrict__ Yc,
                                                     const int *__restrict__ cidx, const double *__restrict__ cw,
                                                     const int *__restrict__ status, int *__restrict__ dims,
                                                     double *__restrict__ aug, long ldaug, long strideA, long roff,
                                                     double *__restrict__ Kw, long ldk, long strideK) {
  const int i = blockIdx.x, e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  const int n = p.n, m = nsys[e];
  if (mode == 1 && i == 0 && threadIdx.x == 0) {
    dims[2 * e] = m;
    dims[2 * e + 1] = m;
  }
  if (i >= n) return;
  const int *mp = spos + (size_t)e * ldo;
  const int pi = mp[i];
  if (pi < 0) return;
  if (mode == 2) {
    double *krow = Kw + (size_t)e * strideK + (size_t)pi * ldk;
    const size_t nn = (size_t)n * n;
    const double *kq[4];
    double wq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = cidx[4 * e + q];
      wq[q] = (c >= 0 && !status[e]) ? cw[4 * e + q] : 0.0;
      kq[q] = Xc + (c >= 0 ? c : 0) * nn + (size_t)pi * n;
    }
    for (int q = threadIdx.x; q < m; q += 256) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) v += wq[c] * kq[c][q];
      krow[q] = v;
    }
    return;
  }
  double *row = aug + (size_t)e * strideA + (size_t)pi * ldaug;
  if (status[e]) {
    for (int q = threadIdx.x; q < m; q += 256) {
      row[q] = q == pi ? 1.0 : 0.0;
      row[roff + q] = 0.0;
    }
    return;
  }
  const size_t nn = (size_t)n * n;
  const double *xq[4], *yq[4];
  double wq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = cidx[4 * e + q];
    wq[q] = c >= 0 ? cw[4 * e + q] : 0.0;
    const size_t off = (c >= 0 ? c : 0) * nn + (size_t)pi * n;
    xq[q] = Xc + off;
    yq[q] = Yc + off;
  }
  for (int q = threadIdx.x; q < m; q += 256) {
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x += wq[c] * xq[c][q];
      y += wq[c] * yq[c][q];
    }
    row[q] = x;
    row[roff + q] = y;
  }
}

void launch_mqdt_interp(hipStream_t s, const Lay &L, int mode, const DevPW *tab, const int *pwi, const int *spos,
                        const int *nsys, const double *Xc, const double *Yc, const int *cidx, const double *cw,
                        const int *status, int *dims, double *aug, double *Kw) {
  hipLaunchKernelGGL(k_mqdt_interp, dim3(L.nmax, L.ne), dim3(256), 0, s, mode, tab, pwi, spos, nsys, L.ldo, Xc, Yc,
                     cidx, cw, status, dims, aug, L.ldaug, L.sA, L.roff, Kw, L.ldk, L.sK);
}

// Ku = (Z + Z^T) / 2 for the solution Z = X^-1 Y in the right-hand-side
// columns of the member block (X and Y symmetric, so Z^T = Y X^-1; the
// interpolated X, Y keep it symmetric only up to the interpolation error, and
// the unphysical K is symmetric), into the K workspace.
__global__ __launch_bounds__(256) void k_mqdt_take(const int *__restrict__ nsys, const double *__restrict__ aug,
                                                   long ldaug, long strideA, long roff, double *__restrict__ Kw,
                                                   long ldk, long strideK) {
  const int e = blockIdx.y, p = blockIdx.x;
  const int m = nsys[e];
  if (p >= m) return;
  const double *Z = aug + (size_t)e * strideA + roff;
  double *K = Kw + (size_t)e * strideK + (size_t)p * ldk;
  for (int q = threadIdx.x; q < m; q += 256) K[q] = 0.5 * (Z[(size_t)q * ldaug + p] + Z[(size_t)p * ldaug + q]);
}

void launch_mqdt_take(hipStream_t s, const Lay &L, const int *nsys, const double *aug, double *Kw) {
  hipLaunchKernelGGL(k_mqdt_take, dim3(L.nmax, L.ne), dim3(256), 0, s, nsys, aug, L.ldaug, L.sA, L.roff, Kw, L.ldk,
                     L.sK);
}

// K = the last n_o rows of the system's solution (rows m - n_o .. m), into the
// K workspace, and dims = {n_o, n_o} for the S/Omega stage.
__global__ __launch_bounds__(256) void k_mqdt_gather(const int *__restrict__ nsys, const int *__restrict__ nopen,
                                                     const double *__restrict__ aug, long ldaug, long strideA,
                                                     long roff, double *__restrict__ Kw, long ldk, long strideK,
                                                     int *__restrict__ dims, int nmax) {
  const int e = blockIdx.y, i = blockIdx.x;
  const int no = nopen[e], m = nsys[e];
  if (i == 0 && threadIdx.x == 0) {
    dims[2 * e] = no;
    dims[2 * e + 1] = no;
  }
  if (i >= nmax) return;
  const double *Y = aug + (size_t)e * strideA + (size_t)(m - no + (i < no ? i : 0)) * ldaug + roff;
  double *K = Kw + (size_t)e * strideK + (size_t)i * ldk;
  for (int j = threadIdx.x; j < nmax; j += 256) K[j] = (i < no && j < no) ? Y[j] : 0.0;
}

void launch_mqdt_gather(hipStream_t s, const Lay &L, const int *nsys, const int *nopen, const double *aug,
                        double *Kw, int *dims) {
  hipLaunchKernelGGL(k_mqdt_gather, dim3(L.nmax, L.ne), dim3(256), 0, s, nsys, nopen, aug, L.ldaug, L.sA, L.roff,
                     Kw, L.ldk, L.sK, dims, L.nmax);
}

}  // namespace rm
