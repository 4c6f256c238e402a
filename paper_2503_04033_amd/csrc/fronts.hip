// Factorization and solves of the interface system T u = rhs on the GPU by nested
// dissection over the box grid, with dense frontal matrices (paper Sec. 3.1 and Sec. 3.3:
// T is block-sparse with one m^2 x m^2 block per pair of faces of a box, and its sparse
// factorization dominates the build stage; the paper hands it to a multifrontal CPU
// solver).  A front of the dissection tree holds the faces its two halves share (the
// separator P, eliminated here) and the faces on its outer boundary (B, passed up):
//
//   F = [[A_PP, A_PB], [A_BP, A_BB]]   assembled from the two halves' Schur complements
//                                      (for a single box: its DtN map T^tau);
//   partial LU with row pivoting inside P:  P_r A_PP = L11 U11,  L21 = A_BP U11^{-1},
//   U12 = L11^{-1} P_r A_PB,  S = A_BB - L21 U12 (the Schur complement passed up).
//
// The partial LU is the leaf LU of lu.hip run over the first n_piv columns with pivots
// restricted to the first n_piv rows; S is left in the trailing block of F.  The solve
// runs the forward substitution up the tree and the backward one down.
#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/hps_leaf.h"
#include "common.h"
#include "kernels.h"

namespace hps {

// F = 0 with ones on the diagonal at positions [d0, d1) and [d2, d3) (padding rows of
// the separator and boundary blocks), for nfront fronts of n x n.
__global__ void front_init_kernel(int nfront, int n, int d0, int d1, int d2, int d3, double* F) {
  const size_t per = (size_t)n * n;
  const size_t total = per * nfront;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t k = e % per;
    const int i = (int)(k / n), j = (int)(k % n);
    double v = 0.0;
    if (i == j && ((i >= d0 && i < d1) || (i >= d2 && i < d3))) v = 1.0;
    F[e] = v;
  }
}

// dst[t.d + i * t.ld_d + j] += src[t.s + i * t.ld_s + j] for 0 <= i, j < bm; one workgroup
// per task.  Tasks of one launch write disjoint blocks.
__global__ __launch_bounds__(256) void block_add_kernel(int ntask, const int64_t* tasks, int bm, double* dst,
                                                        const double* src) {
  const int64_t* t = tasks + (size_t)blockIdx.x * 4;
  const int64_t d = t[0], s = t[1], ldd = t[2], lds = t[3];
  for (int e = threadIdx.x; e < bm * bm; e += blockDim.x) {
    const int i = e / bm, j = e - i * bm;
    dst[d + i * ldd + j] += src[s + i * lds + j];
  }
}

// Segments of len doubles: dst[t.d + i] = src[t.s + i] (mode 0), += (mode 1) or -= (mode
// -1); one workgroup per task.
__global__ __launch_bounds__(256) void segment_kernel(int ntask, const int64_t* tasks, int len, double* dst,
                                                      const double* src, int mode) {
  const int64_t* t = tasks + (size_t)blockIdx.x * 2;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const double v = src[t[1] + i];
    dst[t[0] + i] = mode == 0 ? v : (mode > 0 ? dst[t[0] + i] + v : dst[t[0] + i] - v);
  }
}

// One vector per front through the partial factorization (the rows below n_piv never
// move: perm[i] = i there).  vec: [nfront][n] FP64.
//  mode 0 (upward): on entry r in unknown order.  Leaves y = L11^{-1} P_r r_P in
//         positions [0, n_piv) and r_B - L21 y in [n_piv, n).
//  mode 1 (downward): on entry y in [0, n_piv) (as mode 0 left it) and u_B in [n_piv, n).
//         Leaves u_P = U11^{-1} (y - U12 u_B) in [0, n_piv), in unknown order.
// The transposed system (T^T = U^T L^T, for adjoint solves):
//  mode 2 (upward): on entry r in unknown order.  Leaves z = U11^{-T} r_P in positions
//         [0, n_piv) and r_B - U12^T z in [n_piv, n).
//  mode 3 (downward): on entry z in [0, n_piv) and lam_B in [n_piv, n).  Leaves lam_P =
//         P_r^T L11^{-T} (z - L21^T lam_B) in [0, n_piv), in unknown order.
__global__ __launch_bounds__(kVecThreads) void front_solve_kernel(int n, int n_piv, const double* F_all,
                                                                  const int* perm_all, const double* dinv_all,
                                                                  double* vec_all, int mode) {
  extern __shared__ double vs[];  // [n], then 64 of scratch
  double* tmp = vs + n;
  const int f = blockIdx.x;
  const double* F = F_all + (size_t)f * n * n;
  const int* perm = perm_all + (size_t)f * n;
  const int npanel = (n + kPanel - 1) / kPanel;
  const double* dinv = dinv_all + (size_t)f * npanel * 2 * 64 * 64;
  double* vec = vec_all + (size_t)f * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) vs[i] = (mode == 0 && i < n_piv) ? vec[perm[i]] : vec[i];
  __syncthreads();
  auto row = [&](int j) { return F + (size_t)perm[j] * n; };
  auto prow = [&](int j) { return F + (size_t)j * n; };  // rows past n_piv never move
  const int np = n_piv / kPanel;
  if (mode == 0) {
    for (int bk = 0; bk < np; bk++) {
      const int s = bk * kPanel;
      vec_block_inverse<double>(vs, tmp, dinv + (size_t)(2 * bk) * 64 * 64, s, kPanel, false);
      vec_rows_update<double>(vs, s + kPanel, n, s, kPanel, row);
    }
  } else if (mode == 1) {
    for (int c0 = n_piv; c0 < n; c0 += kPanel)  // y - U12 u_B, 64 columns at a time
      vec_rows_update<double>(vs, 0, n_piv, c0, (n - c0) < kPanel ? (n - c0) : kPanel, row);
    for (int bk = np - 1; bk >= 0; bk--) {
      const int s = bk * kPanel;
      vec_block_inverse<double>(vs, tmp, dinv + (size_t)(2 * bk + 1) * 64 * 64, s, kPanel, false);
      vec_rows_update<double>(vs, 0, s, s, kPanel, row);
    }
  } else if (mode == 2) {
    for (int bk = 0; bk < np; bk++) {
      const int s = bk * kPanel;
      vec_block_inverse<double>(vs, tmp, dinv + (size_t)(2 * bk + 1) * 64 * 64, s, kPanel, true);
      vec_cols_update<double>(vs, s, kPanel, s + kPanel, n, row);
    }
  } else {
    for (int r0 = n_piv; r0 < n; r0 += kPanel)  // z - L21^T lam_B, 64 rows at a time
      vec_cols_update<double>(vs, r0, (n - r0) < kPanel ? (n - r0) : kPanel, 0, n_piv, prow);
    for (int bk = np - 1; bk >= 0; bk--) {
      const int s = bk * kPanel;
      vec_block_inverse<double>(vs, tmp, dinv + (size_t)(2 * bk) * 64 * 64, s, kPanel, true);
      vec_cols_update<double>(vs, s, kPanel, 0, s, row);
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) vec[(mode == 3 && i < n_piv) ? perm[i] : i] = vs[i];
}

}  // namespace hps

struct hps_front_plan_s {
  hps::Geom g;
  int n_piv;
  std::vector<int> ops;
};

namespace {

void sched_trsm_f(std::vector<int>& ops, int r0, int r1, int cA, int cB) {
  if (r1 - r0 <= hps::kLuRowsMax) {
    ops.insert(ops.end(), {hps::kOpRows, r0, r1, cA, cB, 0, 0, 0});
    return;
  }
  const int mid = r0 + ((r1 - r0) / 2 + 63) / 64 * 64;
  sched_trsm_f(ops, r0, mid, cA, cB);
  ops.insert(ops.end(), {hps::kOpGemm, mid, r1, cA, cB, r0, mid, 0});
  sched_trsm_f(ops, mid, r1, cA, cB);
}

// the recursive column split of the leaf LU (see abi.hip), over columns [c0, c1) of an
// n-row matrix
void sched_lu_f(std::vector<int>& ops, int c0, int c1, int n) {
  if (c1 - c0 <= 64) {
    ops.insert(ops.end(), {hps::kOpPanel, c0, c1 - c0, 0, 0, 0, 0, 0});
    return;
  }
  const int mid = c0 + ((c1 - c0) / 2 + 63) / 64 * 64;
  sched_lu_f(ops, c0, mid, n);
  sched_trsm_f(ops, c0, mid, mid, c1);
  ops.insert(ops.end(), {hps::kOpGemm, mid, n, mid, c1, c0, mid, 0});
  sched_lu_f(ops, mid, c1, n);
}

bool bad_tasks(int ntask, const void* tasks) { return ntask < 0 || (ntask > 0 && !tasks); }

}  // namespace

extern "C" {

hps_status hps_front_plan_create(hps_front_plan* out, int32_t n, int32_t n_piv) {
  if (!out || n < 64 || n > 12288 || n % 32 != 0 || n_piv < 64 || n_piv > n || n_piv % 64 != 0) return HPS_EINVAL;
  hps_front_plan_s* pl = new (std::nothrow) hps_front_plan_s();
  if (!pl) return HPS_ENOMEM;
  hps::Geom& g = pl->g;
  g = hps::Geom{};
  g.n = n;
  g.n_pad = n;
  g.npanel = (n + hps::kPanel - 1) / hps::kPanel;
  pl->n_piv = n_piv;
  // the vector solves keep one vector of n doubles in LDS (beyond 64 KB for n > 8128); the
  // kernel attribute is process-wide, so it is set for the largest front every time
  const int shm = (int)(sizeof(double) * (12288 + 64));
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&hps::front_solve_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, shm) != hipSuccess) {
    delete pl;
    return HPS_EDEVICE;
  }
  sched_lu_f(pl->ops, 0, n_piv, n);
  if (n_piv < n) {
    sched_trsm_f(pl->ops, 0, n_piv, n_piv, n);
    pl->ops.insert(pl->ops.end(), {hps::kOpGemm, n_piv, n, n_piv, n, 0, n_piv, 0});
  }
  *out = pl;
  return HPS_OK;
}

hps_status hps_front_plan_destroy(hps_front_plan pl) {
  if (!pl) return HPS_EINVAL;
  delete pl;
  return HPS_OK;
}

size_t hps_front_dinv_elems(hps_front_plan pl) {
  return pl ? (size_t)pl->g.npanel * 2 * 64 * 64 : 0;
}

hps_status hps_front_init(int32_t nfront, int32_t n, int32_t d0, int32_t d1, int32_t d2, int32_t d3, double* F,
                          hipStream_t st) {
  if (nfront < 0 || n <= 0 || (nfront > 0 && !F)) return HPS_EINVAL;
  if (nfront == 0) return HPS_OK;
  const size_t total = (size_t)nfront * n * n;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(hps::front_init_kernel, dim3(blocks), dim3(256), 0, st, nfront, n, d0, d1, d2, d3, F);
  return hipGetLastError() == hipSuccess ? HPS_OK : HPS_EDEVICE;
}

hps_status hps_front_block_add(int32_t ntask, const int64_t* tasks, int32_t bm, double* dst, const double* src,
                               hipStream_t st) {
  if (bad_tasks(ntask, tasks) || bm <= 0 || (ntask > 0 && (!dst || !src))) return HPS_EINVAL;
  if (ntask == 0) return HPS_OK;
  hipLaunchKernelGGL(hps::block_add_kernel, dim3(ntask), dim3(256), 0, st, ntask, tasks, bm, dst, src);
  return hipGetLastError() == hipSuccess ? HPS_OK : HPS_EDEVICE;
}

hps_status hps_front_segments(int32_t ntask, const int64_t* tasks, int32_t len, double* dst, const double* src,
                              int32_t add, hipStream_t st) {
  if (bad_tasks(ntask, tasks) || len <= 0 || add < -1 || add > 1 || (ntask > 0 && (!dst || !src))) return HPS_EINVAL;
  if (ntask == 0) return HPS_OK;
  hipLaunchKernelGGL(hps::segment_kernel, dim3(ntask), dim3(256), 0, st, ntask, tasks, len, dst, src, (int)add);
  return hipGetLastError() == hipSuccess ? HPS_OK : HPS_EDEVICE;
}

hps_status hps_front_factor(hps_front_plan pl, int32_t nfront, double* F, int32_t* perm, double* dinv,
                            int32_t* info, hipStream_t st) {
  if (!pl || nfront < 0 || nfront > 65535) return HPS_EINVAL;
  if (nfront == 0) return HPS_OK;
  if (!F || !perm || !dinv || !info) return HPS_EINVAL;
  const hipError_t e = hps::getrf_run<double>(pl->g, pl->ops, F, perm, dinv, info, nfront, st, nullptr, pl->n_piv);
  return e == hipSuccess ? HPS_OK : HPS_EDEVICE;
}

hps_status hps_front_solve(hps_front_plan pl, int32_t nfront, const double* F, const int32_t* perm,
                           const double* dinv, double* vec, int32_t mode, hipStream_t st) {
  if (!pl || nfront < 0 || nfront > 65535 || mode < 0 || mode > 3) return HPS_EINVAL;
  if (nfront == 0) return HPS_OK;
  if (!F || !perm || !dinv || !vec) return HPS_EINVAL;
  const int n = pl->g.n_pad;
  const size_t shm = sizeof(double) * ((size_t)n + 64);
  hipLaunchKernelGGL(hps::front_solve_kernel, dim3(nfront), dim3(hps::kVecThreads), shm, st, n, pl->n_piv, F, perm,
                     dinv, vec, (int)mode);
  return hipGetLastError() == hipSuccess ? HPS_OK : HPS_EDEVICE;
}

}  // extern "C"
