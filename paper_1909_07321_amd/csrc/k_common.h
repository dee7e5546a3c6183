// k_common.h -- device helpers shared by the batched FP64 kernels (linear
// algebra of the K and S/Omega stages, the outer-region propagation).
#ifndef K_COMMON_H
#define K_COMMON_H
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "rm_internal.h"

namespace rm {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Calls f(std::integral_constant<int, I>) for I = 0, 1, ...: a loop whose index
// is a compile-time constant in every iteration, so register arrays indexed by
// it stay in registers.
template <typename F, int... I>
__device__ __forceinline__ void static_for(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

// LDS slabs of the 64 x 64 FP64 MFMA tiles.  LDS serves 64-bit reads sixteen
// lanes at a time from 32 four-byte banks.  The A operand is staged as it lies
// in memory, [row][k], with an odd pitch K + 1: the sixteen lanes of a fragment
// read take sixteen rows at one k, which an odd pitch spreads over all banks
// (a pitch of 64 would put them on one bank pair).  The B operand is staged
// [k][col]: sixteen lanes read sixteen consecutive columns, conflict-free at
// pitch TILE.  Staging stores are row-contiguous.
constexpr int PB = TILE;
template <int K> struct Pitch { static constexpr int A = K + 1; };

// Persistent distribution of per-energy work items: energy e belongs to XCD
// e % NQ (workgroup b runs on XCD b % NQ), and the items of an XCD's energies go
// round-robin to its workgroups, so the items of one energy share one L2 and no
// workgroup is launched for an item that turns out to be empty.  f(e, r) runs
// item r of energy e; its early returns must be uniform over the workgroup.
template <typename F>
__device__ __forceinline__ void for_items(int ne, int ipe, F &&f) {
  const int x = blockIdx.x % NQ, l = blockIdx.x / NQ, nl = gridDim.x / NQ;
  const int nex = ne > x ? (ne - x + NQ - 1) / NQ : 0;
  const long total = (long)nex * ipe;
  for (long u = l; u < total; u += nl) f(x + NQ * (int)(u / ipe), (int)(u % ipe));
}

// Global-memory views of a pointer read from a table: loads through them are
// global loads, which count only against vmcnt (a generic pointer gives flat
// loads, which also count against lgkmcnt, so every wait for an LDS read would
// wait for outstanding memory loads as well).
template <typename T> using GlobalPtr = const T __attribute__((address_space(1))) *;
template <typename T> using GlobalMut = T __attribute__((address_space(1))) *;

// acc += A_slab (64 x K) * B_slab (K x 64): every wave owns a 32 x 32 quarter.
// UNROLL bounds how many k-steps' fragments are read ahead (registers).
template <int K, int UNROLL = K / 4>
__device__ __forceinline__ void mfma_slab(const double (*sA)[Pitch<K>::A], const double (*sB)[PB], d4 (&acc)[4],
                                          int wr, int wc, int kk, int ii) {
#pragma unroll UNROLL
  for (int ks = 0; ks < K; ks += 4) {
    const double a0 = sA[wr * 32 + ii][ks + kk], a1 = sA[wr * 32 + 16 + ii][ks + kk];
    const double b0 = sB[ks + kk][wc * 32 + ii], b1 = sB[ks + kk][wc * 32 + 16 + ii];
    acc[0] = mfma64(a0, b0, acc[0]);
    acc[1] = mfma64(a0, b1, acc[1]);
    acc[2] = mfma64(a1, b0, acc[2]);
    acc[3] = mfma64(a1, b1, acc[3]);
  }
}

// Grid of a persistent for_items launch: enough workgroups to fill every CU at
// the kernel's occupancy, and no more than there are items per XCD.
template <typename K>
inline int persist_grid(K kernel, int threads, int ne, long ipe) {
  static std::mutex mu;
  static std::map<const void *, int> occ;
  static int ncu = 0;
  int oc;
  {
    std::lock_guard<std::mutex> g(mu);
    if (!ncu) {
      int dev = 0;
      (void)hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    }
    auto it = occ.find((const void *)kernel);
    if (it == occ.end()) {
      int b = 0;
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, threads, 0);
      it = occ.emplace((const void *)kernel, std::max(1, b)).first;
    }
    oc = it->second;
  }
  const long per_xcd = (long)((ne + NQ - 1) / NQ) * ipe;
  const long lim = (long)oc * std::max(1, ncu / NQ);
  return NQ * (int)std::max(1L, std::min(per_xcd, lim));
}

}  // namespace rm
#endif
