// k_prop.hip -- outer-region propagation with the long-range multipole
// coupling (PSTGF paper, section "Overview": eq. (radial) with U_nm, whose
// coupled radial functions are carried by a Numerov method between the
// inner-region boundary r0 = a and the asymptotic radius r1), FP64.
//
// Equations (Rydberg units): F'' = Q F with Q = diag(l(l+1)/r^2 - 2z/r - eps)
// + 2U and U(r) = sum_lam r^-(lam+1) A_lam (A_lam: the multipole coefficients).
// The solution columns of one energy -- the decaying solution of every closed
// channel, the irregular and the regular solution of every open channel, in
// the column order of the matching unknowns -- start at r1 with the value and
// derivative of their uncoupled analytic function; the second point comes
// from the Taylor series of the coupled equations about r1.  Inward Numerov in
// Z = T Y, T = 1 - (h^2/12) Q:
//   Z_{k-1} = 2 Y_k + (10 h^2/12) Q_k Y_k - Z_{k+1},   Y_k = T_k^-1 Z_k,
// where T = D - (h^2/6) U with D = diag(1 - (h^2/12) Q_diag), so that
// Y = (1 + P + P^2) D^-1 Z with P = (h^2/6) D^-1 U: the neglected P^3 is below
// 1e-18 for the multipole strengths and steps of these grids (|h^2 U / 6| ~
// 1e-7).  In the recurrence U Y is taken as U W + U P W (W = D^-1 Z), whose
// products the series already forms: the dropped U P^2 W is O(h^4 U^3) and
// enters Z_{k-1} with the factor 10 h^2/12.  Every `stab` steps the columns are recombined (closed rows of the
// newest Z made the identity on the closed columns and zero elsewhere), which
// adds decaying solutions to the columns and leaves K unchanged.  At r0 the
// derivative is [(2 Z_1 - Y_1) - (2 Z_-1 - Y_-1)] / (2h).
//
// Per energy the workspace holds five n x 2n matrices (rows and columns padded
// to multiples of 64): the two Numerov states (the newer one after step s is
// matrix s % 2), the record 2 Z_1 - Y_1, and the results Y_0 (phi) and Y'_0
// (dphi); until the last recombination the three serve as its scratch.  They
// are stored by 64 x 64 tiles, column panel-major, each tile in the order in
// which the stepping kernel's threads hold it (value y of thread t at
// 256 y + t), so that its loads and stores are whole-wave contiguous.
#include <type_traits>

#include "k_common.h"
#include "rm.h"
#include "rm_internal.h"

namespace rm {

namespace {

constexpr int JT = 20;  // Taylor orders of the second start point

__device__ __forceinline__ double *pmat(double *pz, long sZ, int e, int q) {
  return pz + ((size_t)e * PROP_NMAT + q) * sZ;
}

// Offset of element (i, j) of a propagation matrix with zrb row blocks: in
// the tile of row block i / 64 and column panel j / 64, thread
// t = 64 (2 wr + wc) + 16 kk + ii holds it as value y = 4 q + v, where the
// tile row is 32 wr + 16 (q >> 1) + 4 v + kk and the tile column 32 wc +
// 16 (q & 1) + ii (the MFMA 16 x 16 accumulator layout).
__device__ __forceinline__ size_t zoff(int i, int j, long zrb) {
  const int ir = i & 63, jc = j & 63;
  const int t = ((ir >> 5) * 2 + (jc >> 5)) * 64 + (ir & 3) * 16 + (jc & 15);
  const int y = (((ir >> 4) & 1) * 2 + ((jc >> 4) & 1)) * 4 + ((ir >> 2) & 3);
  return (((size_t)(j >> 6) * zrb + (i >> 6)) * 16 + y) * 256 + t;
}

}  // namespace

// Start values: one workgroup per (column, energy), one thread per row.
// fg holds the uncoupled functions at r1 (the asymptotic stage evaluates a
// coupled wave there).  Writes Z_{N-1} to matrix 1 and Z_{N-2} to matrix 0,
// zero in the padding rows and in the columns of the energy's last panel past
// its m = n + nopen.
__global__ __launch_bounds__(PROP_MAXN) void k_prop_start(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                          const double *__restrict__ E, const double *__restrict__ fg,
                                                          const int *__restrict__ nopen,
                                                          const int *__restrict__ openidx,
                                                          const int *__restrict__ colpos, long ldo,
                                                          double *__restrict__ pz, long zrb, long sZ, int npts) {
  const int j = blockIdx.x, e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  if (p.lamax == 0) return;
  const int n = p.n, no = nopen[e], nc = n - no, m = n + no;
  if (j >= (m + TILE - 1) / TILE * TILE) return;
  const int i = threadIdx.x;
  double *Z0 = pmat(pz, sZ, e, 0), *Z1 = pmat(pz, sZ, e, 1);
  if (j >= m) {
    if (i < p.npad) Z0[zoff(i, j, zrb)] = Z1[zoff(i, j, zrb)] = 0.0;
    return;
  }
  __shared__ int ch_s;
  __shared__ double c[JT + 2][PROP_MAXN], g[8][PROP_MAXN], y[PROP_MAXN];
  const int *cp = colpos + (size_t)e * ldo;
  if (j < nc) {
    if (i < n && cp[i] == j) ch_s = i;   // the closed channel of column j
  } else if (i == 0) {
    ch_s = openidx[(size_t)e * ldo + (j < n ? j - nc : j - n)];
  }
  __syncthreads();
  const int ch = ch_s;
  const double *f = fg + ((size_t)e * ldo + ch) * 4;
  const bool reg = j >= n;   // regular (s) column of an open channel
  const double v = reg ? f[0] : f[2], dv = reg ? f[1] : f[3];
  const double r1 = p.r1, h = (p.r1 - p.a) / (npts - 1), Ev = E[e];
  const int L = p.lamax, npad = p.npad;
  const double eps_i = i < n ? Ev - p.ethr[i] : 0.0;
  const double L2 = i < n ? (double)p.l[i] * (p.l[i] + 1) : 0.0;
  for (int t = 0; t < JT + 2; ++t) c[t][i] = 0.0;
  if (i == ch) {
    c[0][i] = v;
    c[1][i] = dv;
  }
  __syncthreads();
  // Taylor coefficients of Q(r1 + x) = sum_p (D_p + 2 U_p) x^p:
  //   D_p = l(l+1) (p+1) (-1)^p r1^-(p+2) - 2z (-1)^p r1^-(p+1) - [p = 0] eps
  //   U_p = sum_lam C(lam+p, p) (-1)^p r1^-(lam+1+p) A_lam
  for (int jt = 0; jt < JT; ++jt) {
    // g_lam = sum_{p <= jt} C(lam+p, p) (-1)^p r1^-(lam+1+p) c_{jt-p}
    for (int lam = 1; lam <= L; ++lam) {
      double acc = 0.0, w = pow(r1, -(double)(lam + 1));
      for (int pp = 0; pp <= jt; ++pp) {
        acc += w * c[jt - pp][i];
        w *= -(double)(lam + pp + 1) / ((double)(pp + 1) * r1);
      }
      g[lam - 1][i] = acc;
    }
    __syncthreads();
    double sum = 0.0;
    if (i < n) {
      double rp2 = 1.0 / (r1 * r1), rp1 = 1.0 / r1, sg = 1.0;
      for (int pp = 0; pp <= jt; ++pp) {
        double d = L2 * rp2 * (pp + 1) * sg - 2.0 * p.z * rp1 * sg;
        if (pp == 0) d -= eps_i;
        sum += d * c[jt - pp][i];
        rp2 /= r1;
        rp1 /= r1;
        sg = -sg;
      }
      for (int lam = 0; lam < L; ++lam) {
        const double *At = p.cft + (size_t)lam * npad * npad + i;  // A^T: row k of A^T is read across threads
        double u = 0.0;
        for (int k = 0; k < n; ++k) u += At[(size_t)k * npad] * g[lam][k];
        sum += 2.0 * u;
      }
    }
    c[jt + 2][i] = sum / ((double)(jt + 2) * (jt + 1));
    __syncthreads();
  }
  // Y at r1 - h, then Z = T Y at both points
  double yb = 0.0, xp = 1.0;
  for (int t = 0; t < JT + 2; ++t) {
    yb += c[t][i] * xp;
    xp *= -h;
  }
  for (int side = 0; side < 2; ++side) {
    const double r = side == 0 ? r1 : r1 - h;
    const double yi = side == 0 ? c[0][i] : yb;
    y[i] = i < n ? yi : 0.0;
    __syncthreads();
    if (i < n) {
      double u = 0.0;
      for (int lam = 0; lam < L; ++lam) {
        const double *At = p.cft + (size_t)lam * npad * npad + i;
        const double w = pow(r, -(double)(lam + 2));
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += At[(size_t)k * npad] * y[k];
        u += w * s;
      }
      const double qy = (L2 / (r * r) - 2.0 * p.z / r - eps_i) * yi + 2.0 * u;
      (side == 0 ? Z1 : Z0)[zoff(i, j, zrb)] = yi - (h * h / 12.0) * qy;
    } else if (i < p.npad) {
      (side == 0 ? Z1 : Z0)[zoff(i, j, zrb)] = 0.0;   // padding rows stay zero through the recurrence
    }
    __syncthreads();
  }
}

// Steps s = s0 .. s1 of the recurrence (step s takes Z_k, k = npts-1-s, to
// Z_{k-1}) for one 64-column panel per item: two coupling products per step
// (U W and U P W).  The workgroup has 4 waves per 64-row block of the panel
// (NRB blocks); each wave holds a 32 x 32 block in the MFMA accumulator
// layout, 16 values per thread.  A coupling product stages X (all rows of the
// panel) in LDS once and reads U's MFMA operands straight from the
// fragment-major multipole matrices (L2-resident, shared by every energy of
// the wave), combining them with the step's powers of r in registers; the
// operands of k-step q + 2 (q + 1 for LB = 8) are requested before the MFMAs
// of k-step q.  The
// rows' D^-1 and Q_diag of the step sit in LDS (two copies, alternating with
// the step's parity).  LB >= the largest lamax of the launch's waves (a
// multipole count bucket: 2, 4 or 8).
template <int NRB, int LB>
__global__ __launch_bounds__(256 * NRB) void k_numerov(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                       const double *__restrict__ E, const int *__restrict__ nopen,
                                                       double *__restrict__ pz, long zrb, long sZ, int npts, int s0,
                                                       int s1, int npanel, int ne) {
  constexpr int ROWS = NRB * TILE;
  __shared__ double sX[ROWS][PB];
  __shared__ double sdi[2][ROWS], sqd[2][ROWS];
  // The lane indices are re-derived at every step from an opaque copy of the
  // thread index, so that the compiler recomputes the few address operations
  // of a step instead of holding every LDS and global address of the step in
  // registers across the loop.
  int t = threadIdx.x, rb = 0, wr = 0, wc = 0, kk = 0, ii = 0;
  auto relane = [&]() {
    int tq = threadIdx.x;
    asm volatile("" : "+v"(tq));
    t = tq;
    rb = tq >> 8;
    wr = (tq >> 7) & 1;
    wc = (tq >> 6) & 1;
    kk = (tq >> 4) & 3;
    ii = tq & 15;
  };
  relane();
  // value y = 4 q + v of this thread: row 64 rb + 32 wr + 16 (q>>1) + 4 v + kk,
  // panel column 32 wc + 16 (q&1) + ii (accumulator register v of MFMA block q)
  auto rowof = [&](int y) { return rb * TILE + wr * 32 + ((y >> 3) & 1) * 16 + 4 * (y & 3) + kk; };
  auto colof = [&](int y) { return wc * 32 + ((y >> 2) & 1) * 16 + ii; };
  for_items(ne, npanel, [&](int e, int panel) {
    const DevPW &p = tab[pwi[e]];
    if (p.lamax == 0 || p.n > ROWS || (NRB > 1 && p.n <= ROWS - TILE)) return;
    const int n = p.n, m = n + nopen[e];
    if (panel * TILE >= m) return;
    const double a = p.a, h = (p.r1 - p.a) / (npts - 1), h2 = h * h, Ev = E[e], z = p.z;
    const int L = p.lamax;
    const GlobalPtr<double> cfm = (GlobalPtr<double>)p.cfm;
    const size_t lstride = (size_t)p.npad * p.npad;  // one multipole matrix
    // this thread's row of the diagonal terms (padding rows: D = 1, Q = 0)
    const double l2t = t < n ? (double)p.l[t] * (p.l[t] + 1) : 0.0, ept = t < n ? Ev - p.ethr[t] : 0.0;
    // this thread's values of the item's panel: value y at [256 y] of its row block's tile
    const size_t pbase = (size_t)panel * zrb * 4096;
    size_t pofs = pbase + (size_t)rb * 4096 + (t & 255);
    auto load = [&](GlobalPtr<double> M, double(&dst)[16]) {
#pragma unroll
      for (int y = 0; y < 16; ++y) dst[y] = M[pofs + 256 * y];
    };
    auto store = [&](GlobalMut<double> M, const double(&src)[16]) {
#pragma unroll
      for (int y = 0; y < 16; ++y) M[pofs + 256 * y] = src[y];
    };
    // acc = U(r) X for the X the threads hold (all rows of the panel), with
    // U's MFMA operands combined from the multipole matrices in registers:
    // a = sum_lam w_lam A_lam.  stage = false: sX already holds X.
    auto couple = [&](const double(&w)[LB], const double(&X)[16], d4(&acc)[4], bool stage = true) {
      __syncthreads();  // the previous product has finished reading sX
      if (stage) {
#pragma unroll
        for (int y = 0; y < 16; ++y) sX[rowof(y)][colof(y)] = X[y];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = d4{0, 0, 0, 0};
      __syncthreads();
      // this wave's operands: row block rb, 32-row half wr, one 64-lane fragment per k-step
      const GlobalPtr<double> Ab = cfm + (size_t)rb * NRB * 4096 + (size_t)wr * 128 + (t & 63);
      constexpr int NF = LB * 2, RING = LB >= 8 ? 2 : 3;  // k-steps of operands in registers
      double fr[RING][NF];
      auto fetch = [&](int kb, int kq, double(&d)[NF]) {
        const GlobalPtr<double> f = Ab + ((size_t)kb * 16 + kq) * 256;
#pragma unroll
        for (int lam = 0; lam < LB; ++lam) {
          // past the wave's own L the last matrix is read again (weight 0)
          const size_t o = (size_t)(lam < L ? lam : L - 1) * lstride;
          d[2 * lam] = f[o];
          d[2 * lam + 1] = f[o + 64];
        }
      };
#pragma unroll 1
      for (int kb = 0; kb < NRB; ++kb) {
#pragma unroll
        for (int kq = 0; kq < RING - 1; ++kq) fetch(kb, kq, fr[kq]);
#pragma unroll
        for (int kq = 0; kq < 16; ++kq) {
          if (kq + RING - 1 < 16) fetch(kb, kq + RING - 1, fr[(kq + RING - 1) % RING]);
          const double b0 = sX[kb * TILE + 4 * kq + kk][wc * 32 + ii], b1 = sX[kb * TILE + 4 * kq + kk][wc * 32 + 16 + ii];
          const double(&d)[NF] = fr[kq % RING];
          double a0 = 0.0, a1 = 0.0;
#pragma unroll
          for (int lam = 0; lam < LB; ++lam) {
            a0 += w[lam] * d[2 * lam];
            a1 += w[lam] * d[2 * lam + 1];
          }
          acc[0] = mfma64(a0, b0, acc[0]);
          acc[1] = mfma64(a0, b1, acc[1]);
          acc[2] = mfma64(a1, b0, acc[2]);
          acc[3] = mfma64(a1, b1, acc[3]);
        }
      }
    };
    auto accv = [](const d4(&acc)[4], int y) { return acc[y >> 2][y & 3]; };
    double Y[16];
    d4 acc[4];
    // KEEP: the two states of this thread's values stay in registers over the
    // segment (Zk = Z_k, Zp = Z_{k+1}), the stores keeping memory current for
    // the recombination, the next segment and the outputs; otherwise (the
    // 512-thread instances with more than two multipoles, whose operand ring
    // leaves no room) they are read back each step
    constexpr bool KEEP = NRB == 1 || LB <= 2;
    double Zk[16], Zp[16];
    if constexpr (KEEP) {
      load((GlobalPtr<double>)pmat(pz, sZ, e, (s0 + 1) & 1), Zk);
      load((GlobalPtr<double>)pmat(pz, sZ, e, s0 & 1), Zp);
    }
    // step s (k = npts-1-s): Y_k = T_k^-1 Z_k, then Z_{k-1}; the extra pass
    // k = -1 after the last step gives Y_{-1} and the derivative at r0
    const int s_last = s1 == npts - 1 ? npts : s1;
    for (int s = s0; s <= s_last; ++s) {
      const int k = npts - 1 - s, par = s & 1;
      const double r = a + k * h;
      relane();
      pofs = pbase + (size_t)rb * 4096 + (t & 255);
      const GlobalMut<double> Mold = (GlobalMut<double>)pmat(pz, sZ, e, par);
      const GlobalPtr<double> Mnew = (GlobalPtr<double>)pmat(pz, sZ, e, (s + 1) & 1);
      if constexpr (!KEEP) load(Mnew, Zk);
      double w[LB];  // r^-(lam+1) of multipole lam = 1, 2, ..., L; 0 past L
      w[0] = 1.0 / (r * r);
#pragma unroll
      for (int lam = 1; lam < LB; ++lam) w[lam] = w[lam - 1] / r;
#pragma unroll
      for (int lam = 1; lam < LB; ++lam)
        if (lam >= L) w[lam] = 0.0;
      if (t < ROWS) {
        const double q = l2t / (r * r) - 2.0 * z / r - ept;
        sqd[par][t] = t < n ? q : 0.0;
        sdi[par][t] = t < n ? 1.0 / (1.0 - (h2 / 12.0) * q) : 1.0;
      }
      __syncthreads();
      // Y = W + P W + P^2 W with W = D^-1 Z and P = (h^2/6) D^-1 U: the
      // registers carry W, then W + P W while P W is the next product's X
#pragma unroll
      for (int y = 0; y < 16; ++y) Y[y] = Zk[y] * sdi[par][rowof(y)];
      couple(w, Y, acc);
      __syncthreads();  // every wave has read sX
#pragma unroll
      for (int y = 0; y < 16; ++y) {
        const double pw = (h2 / 6.0) * sdi[par][rowof(y)] * accv(acc, y);
        sX[rowof(y)][colof(y)] = pw;
        Y[y] += pw;
      }
      couple(w, Y, acc, false);
#pragma unroll
      for (int y = 0; y < 16; ++y) Y[y] += (h2 / 6.0) * sdi[par][rowof(y)] * accv(acc, y);
      if (k == 1) {  // record 2 Z_1 - Y_1
        const GlobalMut<double> R2 = (GlobalMut<double>)pmat(pz, sZ, e, 2);
#pragma unroll
        for (int y = 0; y < 16; ++y) R2[pofs + 256 * y] = 2.0 * (KEEP ? Zk[y] : Mnew[pofs + 256 * y]) - Y[y];
      }
      if (k == 0) store((GlobalMut<double>)pmat(pz, sZ, e, 3), Y);
      if (k >= 0) {
        // Z_{k-1} = 2 Y + (10 h^2/12) (Q_diag Y + 2 U Y) - Z_{k+1}, over Z_{k+1},
        // with U Y = U W + U (P W) + U (P^2 W) taken as its first two terms: U W
        // is recovered from this thread's P W (still in sX) as (6/h^2) D P W and
        // U (P W) is the accumulator; the dropped term is O(h^4 U^3) and enters
        // Z with the factor 10 h^2/12 (a relative 1e-18 on these grids)
        if constexpr (!KEEP) load(Mold, Zp);
#pragma unroll
        for (int y = 0; y < 16; ++y) {
          const double q = sqd[par][rowof(y)];
          const double uw = (6.0 / h2) * (1.0 - (h2 / 12.0) * q) * sX[rowof(y)][colof(y)];
          const double qy = q * Y[y] + 2.0 * (uw + accv(acc, y));
          const double zn = 2.0 * Y[y] + (10.0 * h2 / 12.0) * qy - Zp[y];
          Mold[pofs + 256 * y] = zn;
          if constexpr (KEEP) {
            Zp[y] = Zk[y];
            Zk[y] = zn;
          }
        }
      } else {
        // k = -1: Zk is Z_{-1}; dphi = [(2 Z_1 - Y_1) - (2 Z_-1 - Y_-1)] / (2h)
        const GlobalPtr<double> R2 = (GlobalPtr<double>)pmat(pz, sZ, e, 2);
        const GlobalMut<double> D = (GlobalMut<double>)pmat(pz, sZ, e, 4);
#pragma unroll
        for (int y = 0; y < 16; ++y) {
          const size_t o = pofs + 256 * y;
          D[o] = (R2[o] - (2.0 * (KEEP ? Zk[y] : Mnew[o]) - Y[y])) / (2.0 * h);
        }
      }
    }
    __syncthreads();  // sX and the row terms are reused by the next item
  });
}

// Recombination of the two Numerov states after step s (the newer is matrix
// s % 2): with E the closed columns of a state, G the closed rows of the newer
// state's closed columns and alpha its closed rows of the other columns, every
// state's closed columns become E' = E G^-1 and its other columns X - E' alpha.
// Three launches: k_prop_stab_inv forms G^-1 (Gauss-Jordan with partial
// pivoting in LDS, one workgroup per energy) and writes [G^-1 | alpha] on the
// first n_c rows of matrix 4; k_prop_stab_mm<1> forms E' of both states into
// matrices 2 and 3; k_prop_stab_mm<2> writes both states' new columns.  The
// products run on FP64 MFMA over 64 x 64 tiles of the tiled layout.
__global__ __launch_bounds__(256) void k_prop_stab_inv(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                       const int *__restrict__ nopen, const int *__restrict__ colpos,
                                                       long ldo, double *__restrict__ pz, long zrb, long sZ, int s,
                                                       int *__restrict__ status) {
  const int e = blockIdx.x;
  const DevPW &p = tab[pwi[e]];
  if (p.lamax == 0) return;
  const int n = p.n, no = nopen[e], nc = n - no, m = n + no;
  if (nc == 0) return;
  __shared__ double G[PROP_MAXN][PROP_MAXN + 1];
  __shared__ int cr[PROP_MAXN], sw[PROP_MAXN], piv_s;
  const int t = threadIdx.x;
  const int *cp = colpos + (size_t)e * ldo;
  for (int i = t; i < n; i += 256)
    if (cp[i] < nc) cr[cp[i]] = i;
  __syncthreads();
  const double *Nw = pmat(pz, sZ, e, s & 1);
  double *H = pmat(pz, sZ, e, 4);
  for (int idx = t; idx < nc * nc; idx += 256) G[idx / nc][idx % nc] = Nw[zoff(cr[idx / nc], idx % nc, zrb)];
  for (int idx = t; idx < nc * (m - nc); idx += 256) {
    const int r = idx / (m - nc), j = nc + idx % (m - nc);
    H[zoff(r, j, zrb)] = Nw[zoff(cr[r], j, zrb)];
  }
  __syncthreads();
  // G <- G^-1 in place (row interchanges undone as column swaps at the end)
  for (int c = 0; c < nc; ++c) {
    if (t == 0) {
      int pr = c;
      double best = fabs(G[c][c]);
      for (int r = c + 1; r < nc; ++r)
        if (fabs(G[r][c]) > best) {
          best = fabs(G[r][c]);
          pr = r;
        }
      if (!(best > 0.0)) atomicOr(status + e, RM_PT_SINGULAR);
      piv_s = pr;
      sw[c] = pr;
    }
    __syncthreads();
    const int pr = piv_s;
    if (pr != c)
      for (int q = t; q < nc; q += 256) {
        const double tmp = G[c][q];
        G[c][q] = G[pr][q];
        G[pr][q] = tmp;
      }
    __syncthreads();
    double d = G[c][c];
    if (!(fabs(d) > 0.0)) d = 1.0;
    __syncthreads();
    if (t == 0) G[c][c] = 1.0;
    __syncthreads();
    for (int q = t; q < nc; q += 256) G[c][q] /= d;
    __syncthreads();
    for (int idx = t; idx < nc * nc; idx += 256) {
      const int r = idx / nc, q = idx % nc;
      if (r == c) continue;
      const double f = G[r][c];
      if (q != c) G[r][q] -= f * G[c][q];
    }
    __syncthreads();
    for (int r = t; r < nc; r += 256)
      if (r != c) G[r][c] = -G[r][c] * G[c][c];
    __syncthreads();
  }
  for (int c = nc - 1; c >= 0; --c) {
    const int pr = sw[c];
    if (pr != c)
      for (int r = t; r < nc; r += 256) {
        const double tmp = G[r][c];
        G[r][c] = G[r][pr];
        G[r][pr] = tmp;
      }
    __syncthreads();
  }
  for (int idx = t; idx < nc * nc; idx += 256) H[zoff(idx / nc, idx % nc, zrb)] = G[idx / nc][idx % nc];
}

// One 64 x 64 output tile per item (energy, state, row block, column panel):
//   PH = 1: E'(rb, c) = sum_kb E(rb, kb) G^-1(kb, c) for the closed columns, into
//           matrix 2 (newer state) or 3 (older);
//   PH = 2: state(rb, c) = E' where j < n_c, X - E' alpha where j >= n_c.
// A tile of the tiled layout is one contiguous block of 4096 doubles, staged
// into LDS with whole-wave loads; the output is stored in the MFMA
// accumulator layout, which is the tile's own order.
template <int PH>
__global__ __launch_bounds__(256) void k_prop_stab_mm(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                      const int *__restrict__ nopen, double *__restrict__ pz,
                                                      long zrb, long sZ, int s, int npanel, int ne) {
  __shared__ double sA[TILE][Pitch<TILE>::A];
  __shared__ double sB[TILE][PB];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  // element of this thread's value y in a tile (the layout of zoff)
  auto tr = [&](int y) { return wr * 32 + ((y >> 3) & 1) * 16 + 4 * (y & 3) + kk; };
  auto tc = [&](int y) { return wc * 32 + ((y >> 2) & 1) * 16 + ii; };
  const int nrb = (int)zrb;
  for_items(ne, 2 * nrb * npanel, [&](int e, int it) {
    const DevPW &p = tab[pwi[e]];
    if (p.lamax == 0) return;
    const int n = p.n, no = nopen[e], nc = n - no, m = n + no;
    const int st = it % 2, rb = (it / 2) % nrb, pc = it / (2 * nrb);
    if (nc == 0 || rb * TILE >= n) return;
    const int ncol = PH == 1 ? nc : m;  // output columns
    if (pc * TILE >= ncol) return;
    double *S = pmat(pz, sZ, e, st == 0 ? (s & 1) : ((s + 1) & 1));   // the state
    double *Ep = pmat(pz, sZ, e, 2 + st);                              // its E'
    const double *H = pmat(pz, sZ, e, 4);                              // [G^-1 | alpha]
    const double *Asrc = PH == 1 ? S : Ep;
    auto tile = [&](auto *M, int r, int c) { return M + (((size_t)c * zrb + r) * 16) * 256; };
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0, 0, 0, 0};
    for (int kb = 0; kb * TILE < nc; ++kb) {
      __syncthreads();
      const double *At = tile(Asrc, rb, kb), *Bt = tile(H, kb, pc);
#pragma unroll
      for (int y = 0; y < 16; ++y) {
        const int i = tr(y), j = tc(y);
        // A: rows of the state, its closed columns k < n_c
        sA[i][j] = kb * TILE + j < nc ? At[y * 256 + t] : 0.0;
        // B: G^-1 (PH 1, columns < n_c) or alpha (PH 2, columns in [n_c, m)), closed rows only
        const int jg = pc * TILE + j;
        const bool bok = kb * TILE + i < nc && (PH == 1 ? jg < nc : (jg >= nc && jg < m));
        sB[i][j] = bok ? Bt[y * 256 + t] : 0.0;
      }
      __syncthreads();
      mfma_slab<TILE>(sA, sB, acc, wr, wc, kk, ii);
    }
    if (PH == 1) {
      double *O = tile(Ep, rb, pc);
#pragma unroll
      for (int y = 0; y < 16; ++y) O[y * 256 + t] = acc[y >> 2][y & 3];
    } else {
      double *O = tile(S, rb, pc);
      const double *Et = tile(Ep, rb, pc);
#pragma unroll
      for (int y = 0; y < 16; ++y) {
        const int jg = pc * TILE + tc(y);
        O[y * 256 + t] = jg < nc ? Et[y * 256 + t] : O[y * 256 + t] - acc[y >> 2][y & 3];
      }
    }
  });
}

// Matching with the propagated matrices (eq. (match)): for each 64 x 64 tile of
// R Lambda, Lambda = a dphi - b phi over the columns [Phi | S], A = Phi -
// (R Lambda)_Phi to gre and B = (R Lambda)_S - S to gim (R is read from aug,
// so the results wait there until k_prop_copy moves them).
__global__ __launch_bounds__(256) void k_prop_assemble(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                       const int *__restrict__ nopen, const double *__restrict__ pz,
                                                       long zrb, long sZ, const double *__restrict__ aug, long ldaug,
                                                       long strideA, double *__restrict__ gre,
                                                       double *__restrict__ gim, long ldk, long strideK, int tiles_m,
                                                       int tiles_n, int ne) {
  __shared__ double sA[TILE][Pitch<TILE>::A];
  __shared__ double sB[TILE][PB];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int kk = lane >> 4, ii = lane & 15;
  for_items(ne, tiles_m * tiles_n, [&](int e, int it) {
    const DevPW &p = tab[pwi[e]];
    if (p.lamax == 0) return;
    const int n = p.n, m = n + nopen[e];
    const int r0 = (it / tiles_n) * TILE, q0 = (it % tiles_n) * TILE;
    if (r0 >= n || q0 >= m) return;
    const double a = p.a, b = p.b;
    const double *R = aug + (size_t)e * strideA;
    const double *PHI = pmat(const_cast<double *>(pz), sZ, e, 3), *DPHI = pmat(const_cast<double *>(pz), sZ, e, 4);
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += TILE) {
      __syncthreads();
      for (int idx = t; idx < TILE * TILE; idx += 256) {
        const int i = idx / TILE, k = idx % TILE;
        sA[i][k] = (r0 + i < n && k0 + k < n) ? R[(size_t)(r0 + i) * ldaug + k0 + k] : 0.0;
        const int kb = idx / TILE, j = idx % TILE;
        sB[kb][j] = (k0 + kb < n && q0 + j < m)
                        ? a * DPHI[zoff(k0 + kb, q0 + j, zrb)] - b * PHI[zoff(k0 + kb, q0 + j, zrb)]
                        : 0.0;
      }
      __syncthreads();
      mfma_slab<TILE>(sA, sB, acc, wr, wc, kk, ii);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = q0 + wc * 32 + (q & 1) * 16 + ii;
      if (j >= m) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = r0 + wr * 32 + (q >> 1) * 16 + 4 * v + kk;
        if (i >= n) continue;
        const double ph = PHI[zoff(i, j, zrb)];
        if (j < n)
          gre[(size_t)e * strideK + (size_t)i * ldk + j] = ph - acc[q][v];
        else
          gim[(size_t)e * strideK + (size_t)i * ldk + (j - n)] = acc[q][v] - ph;
      }
    }
    __syncthreads();
  });
}

// [A | B] of the coupled energies from gre / gim into aug (one row per workgroup)
__global__ __launch_bounds__(256) void k_prop_copy(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                   const int *__restrict__ nopen, const double *__restrict__ gre,
                                                   const double *__restrict__ gim, long ldk, long strideK,
                                                   double *__restrict__ aug, long ldaug, long strideA, long roff) {
  const int i = blockIdx.x, e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  if (p.lamax == 0 || i >= p.n) return;
  const int n = p.n, no = nopen[e];
  double *row = aug + (size_t)e * strideA + (size_t)i * ldaug;
  for (int j = threadIdx.x; j < n; j += 256) row[j] = gre[(size_t)e * strideK + (size_t)i * ldk + j];
  for (int j = threadIdx.x; j < no; j += 256) row[roff + j] = gim[(size_t)e * strideK + (size_t)i * ldk + j];
}

// phi (q = 3) or dphi (q = 4) of the coupled energies into row-major
// [n][ldo] blocks (ldo >= 2n): columns past m zero, NaN for a failed energy.
// One workgroup per (row, energy).
__global__ __launch_bounds__(256) void k_prop_gather(const DevPW *__restrict__ tab, const int *__restrict__ pwi,
                                                     const int *__restrict__ nopen, const int *__restrict__ status,
                                                     const double *__restrict__ pz, long zrb, long sZ, int q,
                                                     double *__restrict__ out, long ldo, long so) {
  const int i = blockIdx.x, e = blockIdx.y;
  const DevPW &p = tab[pwi[e]];
  if (p.lamax == 0 || i >= p.n) return;
  const int n = p.n, m = n + nopen[e];
  const bool bad = status[e] != 0;
  const double *M = pmat(const_cast<double *>(pz), sZ, e, q);
  double *row = out + (size_t)e * so + (size_t)i * ldo;
  for (int j = threadIdx.x; j < 2 * n; j += 256)
    row[j] = bad ? __builtin_nan("") : j < m ? M[zoff(i, j, zrb)] : 0.0;
}

void launch_prop_gather(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen,
                        const int *status, const double *pz, int q, double *out, long ldo, long so) {
  if (!L.npadc) return;
  hipLaunchKernelGGL(k_prop_gather, dim3(L.npadc, L.ne), dim3(256), 0, s, tab, pwi, nopen, status, pz, L.zrb, L.sZ, q,
                     out, ldo, so);
}

namespace {

template <int NRB, int LB>
void step_one(hipStream_t s, const DevPW *tab, const int *pwi, const double *E, const int *nopen,
              double *pz, long zrb, long sZ, int npts, int s0, int s1, int npanel, int ne) {
  hipLaunchKernelGGL((k_numerov<NRB, LB>), dim3(persist_grid(k_numerov<NRB, LB>, 256 * NRB, ne, npanel)),
                     dim3(256 * NRB), 0, s, tab, pwi, E, nopen, pz, zrb, sZ, npts, s0, s1, npanel, ne);
}

// k_numerov with NRB row blocks for waves of up to lamc multipoles
void step_launch(hipStream_t s, int nrb, int lamc, const DevPW *tab, const int *pwi, const double *E,
                 const int *nopen, double *pz, long zrb, long sZ, int npts, int s0, int s1, int npanel, int ne) {
  const int lb = lamc <= 2 ? 2 : lamc <= 4 ? 4 : 8;
  auto go = [&](auto nrb_c, auto lb_c) {
    step_one<decltype(nrb_c)::value, decltype(lb_c)::value>(s, tab, pwi, E, nopen, pz, zrb, sZ, npts, s0, s1, npanel,
                                                             ne);
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  if (nrb == 1) {
    if (lb == 2) go(I1{}, I2{});
    else if (lb == 4) go(I1{}, I4{});
    else go(I1{}, I8{});
  } else {
    if (lb == 2) go(I2{}, I2{});
    else if (lb == 4) go(I2{}, I4{});
    else go(I2{}, I8{});
  }
}

}  // namespace

void launch_prop(hipStream_t s, const Lay &L, int npts, int stab, const DevPW *tab, const int *pwi, const double *E,
                 const double *fg, const int *nopen, const int *openidx, const int *colpos, double *pz, int *status) {
  if (!L.npadc) return;
  const int ncol = 2 * L.npadc, npanel = ncol / TILE;
  hipLaunchKernelGGL(k_prop_start, dim3(ncol, L.ne), dim3(PROP_MAXN), 0, s, tab, pwi, E, fg, nopen, openidx, colpos,
                     L.ldo, pz, L.zrb, L.sZ, npts);
  for (int s0 = 1; s0 <= npts - 1;) {
    const int s1 = std::min(npts - 1, (s0 - 1) / stab * stab + stab);
    // every energy is stepped by the instance whose row blocks match its padded channels
    step_launch(s, 1, L.lamc, tab, pwi, E, nopen, pz, L.zrb, L.sZ, npts, s0, s1, npanel, L.ne);
    if (L.npadc > TILE)
      step_launch(s, 2, L.lamc, tab, pwi, E, nopen, pz, L.zrb, L.sZ, npts, s0, s1, npanel, L.ne);
    if (s1 % stab == 0 && s1 <= npts - 3) {
      hipLaunchKernelGGL(k_prop_stab_inv, dim3(L.ne), dim3(256), 0, s, tab, pwi, nopen, colpos, L.ldo, pz, L.zrb,
                         L.sZ, s1, status);
      const int items = 2 * (int)L.zrb * npanel;
      hipLaunchKernelGGL(k_prop_stab_mm<1>, dim3(persist_grid(k_prop_stab_mm<1>, 256, L.ne, items)), dim3(256), 0, s,
                         tab, pwi, nopen, pz, L.zrb, L.sZ, s1, npanel, L.ne);
      hipLaunchKernelGGL(k_prop_stab_mm<2>, dim3(persist_grid(k_prop_stab_mm<2>, 256, L.ne, items)), dim3(256), 0, s,
                         tab, pwi, nopen, pz, L.zrb, L.sZ, s1, npanel, L.ne);
    }
    s0 = s1 + 1;
  }
}

void launch_prop_assemble(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const int *nopen,
                          const double *pz, double *aug, double *gre, double *gim) {
  if (!L.npadc) return;
  const int tm = L.npadc / TILE, tn = 2 * L.npadc / TILE;
  hipLaunchKernelGGL(k_prop_assemble, dim3(persist_grid(k_prop_assemble, 256, L.ne, (long)tm * tn)), dim3(256), 0, s,
                     tab, pwi, nopen, pz, L.zrb, L.sZ, aug, L.ldaug, L.sA, gre, gim, L.ldk, L.sK, tm, tn, L.ne);
  hipLaunchKernelGGL(k_prop_copy, dim3(L.npadc, L.ne), dim3(256), 0, s, tab, pwi, nopen, gre, gim, L.ldk, L.sK, aug,
                     L.ldaug, L.sA, L.roff);
}

}  // namespace rm
