// a3 -- batched triangular solves X = U^{-1} L^{-1} P B with the factors of a2.
//
// One workgroup (4 waves) owns one box and one 64-column tile of the
// right-hand sides.  Forward: for each LU panel r (rows [s, s+RB)),
//     C = B[perm[s:s+RB], tile] - L[s:s+RB, 0:s] Y[0:s, tile]   (MFMA tile GEMM)
//     Y[s:s+RB, tile] = Linv_r C                                (stored inverse)
// Backward runs the panels in reverse with U and Uinv.  The k loops read L/U
// rows straight from global memory and stage the Y/X rows in LDS.
//
// Workgroup -> (box, tile) mapping is XCD-aware: consecutive workgroup ids are
// dealt round-robin to the 8 XCDs, so all tiles of one box are given ids that
// land on the same XCD and share that XCD's L2 for the L/U reads.
#include "common.h"
#include "kernels.h"

namespace hps {

constexpr int kTsThreads = 256;
constexpr int kTsWaves = 4;
constexpr int kTsLd = 64 + 8;

template <typename T>
struct TsSmem {
  T stage[32 * kTsLd];
  T ctile[64 * kTsLd];
};

__device__ inline bool map_box_tile(int nbox, int ntile, int& box, int& tile) {
  const int id = blockIdx.x;
  const int xcd = id & 7, slot = id >> 3;
  const int lb = slot / ntile;
  tile = slot - lb * ntile;
  box = xcd + 8 * lb;
  return box < nbox;
}

template <typename T, int RB>
__device__ void ts_fwd_step(const Geom& g, const T* LU, const int* perm, const T* Linv, const T* B, T* Y, int c0,
                            int s, TsSmem<T>& sm) {
  constexpr int NRT = RB / 16;
  constexpr int CT = NRT;  // (RB=64: 4 row tiles x 4 col tiles per wave) (RB=32: 2 x 2)
  const int N = g.n_pad, ldx = g.ldx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rtile = wave % NRT, cgrp = wave / NRT;
  const int col0 = cgrp * CT * 16;
  typename Mfma<T>::acc acc[1][CT];
  auto bptr = [&](int, int rr) -> T* { return const_cast<T*>(B) + (size_t)perm[s + rtile * 16 + rr] * ldx + c0 + col0; };
  acc_load<T, 1, CT>(acc, bptr);
  if (s > 0) {
    auto arow = [&](int) -> const T* { return LU + (size_t)perm[s + rtile * 16 + (lane & 15)] * N; };
    auto brow = [&](int k) -> const T* { return Y + (size_t)k * ldx + c0; };
    wg_gemm_sub<T, kTsWaves, 1, CT, 32>(acc, arow, brow, 0, s, sm.stage, kTsLd, col0, 64);
  }
  auto crow = [&](int, int rr) -> T* { return sm.ctile + (rtile * 16 + rr) * kTsLd + col0; };
  acc_store<T, 1, CT>(acc, crow);
  __syncthreads();
  typename Mfma<T>::acc out[1][CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) out[0][ct] = Mfma<T>::zero();
  auto arow2 = [&](int) -> const T* { return Linv + (rtile * 16 + (lane & 15)) * 64; };
  wg_gemm_lds_add<T, 1, CT>(out, arow2, sm.ctile, kTsLd, RB, col0);
  auto yrow = [&](int, int rr) -> T* { return Y + (size_t)(s + rtile * 16 + rr) * ldx + c0 + col0; };
  acc_store<T, 1, CT>(out, yrow);
  __syncthreads();
}

template <typename T, int RB>
__device__ void ts_bwd_step(const Geom& g, const T* LU, const int* perm, const T* Uinv, T* X, int c0, int s,
                            TsSmem<T>& sm) {
  constexpr int NRT = RB / 16;
  constexpr int CT = NRT;
  const int N = g.n_pad, ldx = g.ldx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rtile = wave % NRT, cgrp = wave / NRT;
  const int col0 = cgrp * CT * 16;
  typename Mfma<T>::acc acc[1][CT];
  auto xrow = [&](int, int rr) -> T* { return X + (size_t)(s + rtile * 16 + rr) * ldx + c0 + col0; };
  acc_load<T, 1, CT>(acc, xrow);
  if (s + RB < N) {
    auto arow = [&](int) -> const T* { return LU + (size_t)perm[s + rtile * 16 + (lane & 15)] * N; };
    auto brow = [&](int k) -> const T* { return X + (size_t)k * ldx + c0; };
    wg_gemm_sub<T, kTsWaves, 1, CT, 32>(acc, arow, brow, s + RB, N, sm.stage, kTsLd, col0, 64);
  }
  auto crow = [&](int, int rr) -> T* { return sm.ctile + (rtile * 16 + rr) * kTsLd + col0; };
  acc_store<T, 1, CT>(acc, crow);
  __syncthreads();
  typename Mfma<T>::acc out[1][CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) out[0][ct] = Mfma<T>::zero();
  auto arow2 = [&](int) -> const T* { return Uinv + (rtile * 16 + (lane & 15)) * 64; };
  wg_gemm_lds_add<T, 1, CT>(out, arow2, sm.ctile, kTsLd, RB, col0);
  acc_store<T, 1, CT>(out, xrow);
  __syncthreads();
}

// X[box] = A_ii^{-1} B[box] for the boxes with active[box] != 0 (all if active is null).
template <typename T>
__global__ __launch_bounds__(kTsThreads) void getrs_kernel(Geom g, const T* LU_all, const int* perm_all,
                                                          const T* dinv_all, const T* B_all, T* X_all, int nbox,
                                                          int ntile, const int* active) {
  __shared__ TsSmem<T> sm;
  int box, tile;
  if (!map_box_tile(nbox, ntile, box, tile)) return;
  if (active && active[box] == 0) return;
  const int N = g.n_pad;
  const T* LU = LU_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  const T* dinv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64;
  const T* B = B_all + (size_t)box * N * g.ldx;
  T* X = X_all + (size_t)box * N * g.ldx;
  const int c0 = tile * 64;
  for (int r = 0; r < g.npanel; r++) {
    const int s = r * kPanel;
    const T* Linv = dinv + (size_t)(2 * r) * 64 * 64;
    if (N - s >= 64) ts_fwd_step<T, 64>(g, LU, perm, Linv, B, X, c0, s, sm);
    else ts_fwd_step<T, 32>(g, LU, perm, Linv, B, X, c0, s, sm);
  }
  for (int r = g.npanel - 1; r >= 0; r--) {
    const int s = r * kPanel;
    const T* Uinv = dinv + (size_t)(2 * r + 1) * 64 * 64;
    if (N - s >= 64) ts_bwd_step<T, 64>(g, LU, perm, Uinv, X, c0, s, sm);
    else ts_bwd_step<T, 32>(g, LU, perm, Uinv, X, c0, s, sm);
  }
}

template <typename T>
hipError_t getrs_dispatch(const Geom& g, const T* LU, const int* perm, const T* dinv, const T* B, T* X, int nbox,
                          const int* active, hipStream_t st) {
  const int ntile = g.ldx / 64;
  const int grid = 8 * ((nbox + 7) / 8) * ntile;
  hipLaunchKernelGGL((getrs_kernel<T>), dim3(grid), dim3(kTsThreads), 0, st, g, LU, perm, dinv, B, X, nbox, ntile,
                     active);
  return hipGetLastError();
}

template hipError_t getrs_dispatch<float>(const Geom&, const float*, const int*, const float*, const float*, float*,
                                          int, const int*, hipStream_t);
template hipError_t getrs_dispatch<double>(const Geom&, const double*, const int*, const double*, const double*,
                                           double*, int, const int*, hipStream_t);

}  // namespace hps
