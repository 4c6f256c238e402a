// a2 -- batched dense LU with partial pivoting of the interior blocks A_ii.
//
// The paper factors every box's interior block A_ii (Alg. 1, "form the local
// solution operator"; A_ii is block diagonal over boxes, Sec. 2.2).  Here one
// workgroup factors one box, left-looking with 64-wide panels:
//
//   for each panel P = columns [j0, j0+W):
//     U part   rows at positions < j0 : blocked forward substitution with the
//              unit-lower L of earlier panels, each 64-row step a tile GEMM
//              (MFMA) followed by a product with the stored inverse of that
//              panel's diagonal L block;
//     L part   rows at positions >= j0: A[pos, P] -= L[pos, 0:j0] U[0:j0, P]
//              (MFMA tile GEMM, rows independent);
//     panel    partial pivoting column by column on register-resident
//              sub-panels of SP columns (left-looking inside the panel);
//     inverses of the panel's diagonal L and U blocks for the solves.
//
// Left-looking reads L once per panel and writes only the panel, which halves
// the HBM traffic of a right-looking update.  Rows are never moved: perm[pos]
// names the physical row at position pos (row gathers are contiguous reads in
// row-major storage).  Pivot rule: largest modulus among the rows not yet
// pivoted, ties to the lowest current position; after each sub-panel the chosen
// pivots take the next positions in order and the remaining rows keep their
// relative order.
#include "common.h"
#include "kernels.h"

namespace hps {

constexpr int kLuThreads = 512;
constexpr int kLuWaves = kLuThreads / 64;
constexpr int kLdsLd = 64 + 8;  // padded row length of LDS tiles

template <typename T>
struct LuSmem {
  T tile[64 * kLdsLd];   // GEMM B staging / C tile / diagonal block
  union {
    T ub[64 * 16];       // U part of the current sub-panel (<= 64 rows x SP)
    T inv[64 * 65];      // diagonal-block inverses: strictly lower = L^{-1}, upper = U^{-1}
  };
  T prow[16];            // pivot row of the current column
  T red_v[kLuWaves];
  int red_s[kLuWaves];
  int cnt[32 * kLuWaves];
};

// A operand rows for the LU GEMMs: position -> physical row pointer.
template <typename T>
struct PermRows {
  const T* A;
  const int* perm;
  int lda;
  __device__ const T* operator()(int pos) const { return A + (size_t)perm[pos] * lda; }
};

// One 64-row step of the U part of panel [j0, j0+W): positions [s, s+64).
template <typename T, int W>
__device__ __attribute__((noinline)) void lu_upart_step(const Geom& g, T* A, const int* perm, const T* dinv, int j0, int r, LuSmem<T>& sm) {
  constexpr int CT = W / 32;               // 4 row tiles x 2 column groups over 8 waves
  constexpr int RT = 1;
  const int lda = g.n_pad;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rtile = wave & 3, cgrp = wave >> 2;
  const int s = r * kPanel;
  const int col0 = cgrp * CT * 16;
  PermRows<T> rows{A, perm, lda};
  typename Mfma<T>::acc acc[RT][CT];
  auto rowptr = [&](int, int rr) -> T* { return A + (size_t)perm[s + rtile * 16 + rr] * lda + j0 + col0; };
  acc_load<T, RT, CT>(acc, rowptr);
  if (s > 0) {
    auto arow = [&](int) -> const T* { return rows(s + rtile * 16 + (lane & 15)); };
    auto brow = [&](int k) -> const T* { return rows(k) + j0; };
    wg_gemm_sub<T, kLuWaves, RT, CT, 32>(acc, arow, brow, 0, s, sm.tile, kLdsLd, col0, W);
  }
  __syncthreads();
  // C tile -> LDS, then U rows = Linv_r * C
  auto ldsrow = [&](int, int rr) -> T* { return sm.tile + (rtile * 16 + rr) * kLdsLd + col0; };
  acc_store<T, RT, CT>(acc, ldsrow);
  __syncthreads();
  typename Mfma<T>::acc out[RT][CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) out[0][ct] = Mfma<T>::zero();
  const T* Linv = dinv + (size_t)(2 * r) * 64 * 64;
  auto arow2 = [&](int) -> const T* { return Linv + (rtile * 16 + (lane & 15)) * 64; };
  wg_gemm_lds_add<T, RT, CT>(out, arow2, sm.tile, kLdsLd, 64, col0);
  acc_store<T, RT, CT>(out, rowptr);
  __syncthreads();
}

// L part of panel [j0, j0+W): positions [j0, n_pad).
template <typename T, int W>
__device__ __attribute__((noinline)) void lu_lpart(const Geom& g, T* A, const int* perm, int j0, LuSmem<T>& sm) {
  constexpr int CT = W / 16;
  constexpr int RT = sizeof(T) == 4 ? 2 : 1;
  constexpr int GROUP = kLuWaves * RT * 16;
  const int N = g.n_pad, lda = N;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  PermRows<T> rows{A, perm, lda};
  for (int gs = j0; gs < N; gs += GROUP) {
    const int wrow = gs + wave * RT * 16;
    typename Mfma<T>::acc acc[RT][CT];
    auto rowptr = [&](int rt, int rr) -> T* {
      int pos = wrow + rt * 16 + rr;
      return pos < N ? A + (size_t)perm[pos] * lda + j0 : nullptr;
    };
    acc_load<T, RT, CT>(acc, rowptr);
    auto arow = [&](int rt) -> const T* {
      int pos = wrow + rt * 16 + (lane & 15);
      return pos < N ? rows(pos) : nullptr;
    };
    auto brow = [&](int k) -> const T* { return rows(k) + j0; };
    wg_gemm_sub<T, kLuWaves, RT, CT, 32>(acc, arow, brow, 0, j0, sm.tile, kLdsLd, 0, W);
    acc_store<T, RT, CT>(acc, rowptr);
  }
  __syncthreads();
}

// Pivoted factorization of the panel columns [j0, j0+W) for positions >= j0.
template <typename T, int ROWS, int SP, int W>
__device__ __attribute__((noinline)) void lu_panel(const Geom& g, T* A, int* perm, int j0, LuSmem<T>& sm, int& info) {
  const int N = g.n_pad, lda = N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = 0; q < W / SP; q++) {
    const int c0 = j0 + q * SP;
    const int npv = c0 - j0;
    // (a) U part of this sub-panel: rows pivoted earlier in the panel,
    //     U = L11^{-1} A[piv rows, c0:c0+SP) with L11 unit lower (npv x npv).
    if (npv > 0) {
      for (int e = tid; e < npv * npv; e += kLuThreads) {
        int i = e / npv, k = e - i * npv;
        sm.tile[i * kLdsLd + k] = A[(size_t)perm[j0 + i] * lda + j0 + k];
      }
      for (int e = tid; e < npv * SP; e += kLuThreads) {
        int i = e / SP, c = e - i * SP;
        sm.ub[i * SP + c] = A[(size_t)perm[j0 + i] * lda + c0 + c];
      }
      __syncthreads();
      if (tid < SP) {
        for (int i = 1; i < npv; i++) {
          T s = sm.ub[i * SP + tid];
          for (int k = 0; k < i; k++) s -= sm.tile[i * kLdsLd + k] * sm.ub[k * SP + tid];
          sm.ub[i * SP + tid] = s;
        }
      }
      __syncthreads();
      for (int e = tid; e < npv * SP; e += kLuThreads) {
        int i = e / SP, c = e - i * SP;
        A[(size_t)perm[j0 + i] * lda + c0 + c] = sm.ub[i * SP + c];
      }
    }
    // (b) candidates: slot s = tid + 512 r sits at position c0 + s.
    const int nrem = N - c0;
    T v[ROWS][SP];
    int phys[ROWS];
    bool done[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const int s = tid + kLuThreads * r;
      const bool valid = s < nrem;
      done[r] = !valid;
      phys[r] = valid ? perm[c0 + s] : 0;
      if (valid) {
        const T* row = A + (size_t)phys[r] * lda;
#pragma unroll
        for (int c = 0; c < SP; c++) v[r][c] = row[c0 + c];
        for (int k = 0; k < npv; k++) {
          const T lk = row[j0 + k];
#pragma unroll
          for (int c = 0; c < SP; c++) v[r][c] -= lk * sm.ub[k * SP + c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < SP; c++) v[r][c] = T(0);
      }
    }
    int pivslot[SP];
    // (c) pivoting, one column at a time
#pragma unroll
    for (int c = 0; c < SP; c++) {
      T best = T(-1);
      int bslot = 0x7fffffff;
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (!done[r]) {
          T a = fabs(v[r][c]);
          if (a != a) a = T(INFINITY);  // a NaN is taken as the pivot and flagged below
          const int s = tid + kLuThreads * r;
          if (a > best || (a == best && s < bslot)) { best = a; bslot = s; }
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        T ob = __shfl_xor(best, off);
        int os = __shfl_xor(bslot, off);
        if (ob > best || (ob == best && os < bslot)) { best = ob; bslot = os; }
      }
      if (lane == 0) { sm.red_v[wave] = best; sm.red_s[wave] = bslot; }
      __syncthreads();
      best = sm.red_v[0];
      bslot = sm.red_s[0];
#pragma unroll
      for (int w = 1; w < kLuWaves; w++) {
        T ob = sm.red_v[w];
        int os = sm.red_s[w];
        if (ob > best || (ob == best && os < bslot)) { best = ob; bslot = os; }
      }
      const int ps = bslot;
      pivslot[c] = ps;
      if ((ps & (kLuThreads - 1)) == tid) {
#pragma unroll
        for (int r = 0; r < ROWS; r++) {
          if (r == ps / kLuThreads) {
#pragma unroll
            for (int cc = 0; cc < SP; cc++) sm.prow[cc] = v[r][cc];
            done[r] = true;
          }
        }
      }
      __syncthreads();
      const T pv = sm.prow[c];
      if (!(pv != T(0) && isfinite(pv)) && info == 0) info = c0 + c + 1;
      const T inv = pv != T(0) ? T(1) / pv : T(0);
      T pr[SP];
#pragma unroll
      for (int cc = 0; cc < SP; cc++) pr[cc] = sm.prow[cc];
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (!done[r]) {
          const T l = v[r][c] * inv;
          v[r][c] = l;
#pragma unroll
          for (int cc = c + 1; cc < SP; cc++) v[r][cc] -= l * pr[cc];
        }
      }
    }
    // (d) write the sub-panel back (every slot's row keeps its physical place)
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const int s = tid + kLuThreads * r;
      if (s < nrem) {
        T* row = A + (size_t)phys[r] * lda;
#pragma unroll
        for (int c = 0; c < SP; c++) row[c0 + c] = v[r][c];
      }
    }
    // (e) new order of positions [c0, N): the SP pivots, then the rest in slot order
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int pre[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const int s = tid + kLuThreads * r;
      const bool keep = (s < nrem) && !done[r];
      const unsigned long long mask = __ballot(keep);
      pre[r] = __popcll(mask & lt);
      if (lane == 0) sm.cnt[r * kLuWaves + wave] = __popcll(mask);
    }
    __syncthreads();
    int base = c0 + SP;
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const int s = tid + kLuThreads * r;
      int before = 0, tot = 0;
      for (int w = 0; w < kLuWaves; w++) {
        const int cw = sm.cnt[r * kLuWaves + w];
        tot += cw;
        if (w < wave) before += cw;
      }
      if (s < nrem && !done[r]) perm[base + before + pre[r]] = phys[r];
      base += tot;
    }
#pragma unroll
    for (int c = 0; c < SP; c++) {
      const int ps = pivslot[c];
      if ((ps & (kLuThreads - 1)) == tid) {
#pragma unroll
        for (int r = 0; r < ROWS; r++)
          if (r == ps / kLuThreads) perm[c0 + c] = phys[r];
      }
    }
    __syncthreads();
  }
}

// Inverses of the panel's diagonal blocks: Linv (unit lower) and Uinv (upper),
// W x W, stored row-major with stride 64 (entries beyond W are left unset).
template <typename T, int W>
__device__ __attribute__((noinline)) void lu_diag_inverses(const Geom& g, const T* A, const int* perm, T* dinv_panel, LuSmem<T>& sm) {
  const int lda = g.n_pad;
  const int tid = threadIdx.x;
  for (int e = tid; e < W * W; e += kLuThreads) {
    int i = e / W, k = e - i * W;
    sm.tile[i * kLdsLd + k] = A[(size_t)perm[i] * lda + k];
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int j = lane;
  if (wave == 0 && lane < W) {
    // column j of L^{-1} (rows > j; unit diagonal implied)
    for (int i = j + 1; i < W; i++) {
      T s = -sm.tile[i * kLdsLd + j];
      for (int k = j + 1; k < i; k++) s -= sm.tile[i * kLdsLd + k] * sm.inv[k * 65 + j];
      sm.inv[i * 65 + j] = s;
    }
  } else if (wave == 1 && lane < W) {
    // column j of U^{-1} (rows <= j)
    for (int i = j; i >= 0; i--) {
      T s = (i == j) ? T(1) : T(0);
      for (int k = i + 1; k <= j; k++) s -= sm.tile[i * kLdsLd + k] * sm.inv[k * 65 + j];
      sm.inv[i * 65 + j] = s / sm.tile[i * kLdsLd + i];
    }
  }
  __syncthreads();
  T* Linv = dinv_panel;
  T* Uinv = dinv_panel + 64 * 64;
  for (int e = tid; e < W * W; e += kLuThreads) {
    int i = e / W, k = e - i * W;
    const T x = sm.inv[i * 65 + k];
    Linv[i * 64 + k] = i > k ? x : (i == k ? T(1) : T(0));
    Uinv[i * 64 + k] = i <= k ? x : T(0);
  }
  __syncthreads();
}

template <typename T, int ROWS, int SP>
__global__ __launch_bounds__(kLuThreads, 4) void getrf_kernel(Geom g, T* A_all, int* perm_all, T* dinv_all,
                                                               int* info_all, int nbox) {
  __shared__ LuSmem<T> sm;
  const int box = blockIdx.x;
  if (box >= nbox) return;
  const int N = g.n_pad;
  T* A = A_all + (size_t)box * N * N;
  int* perm = perm_all + (size_t)box * N;
  T* dinv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64;
  for (int i = threadIdx.x; i < N; i += kLuThreads) perm[i] = i;
  __syncthreads();
  int info = 0;
  for (int P = 0; P < g.npanel; P++) {
    const int j0 = P * kPanel;
    const int W = (N - j0) < kPanel ? (N - j0) : kPanel;
    if (W == 64) {
      for (int r = 0; r < P; r++) lu_upart_step<T, 64>(g, A, perm, dinv, j0, r, sm);
      if (P > 0) lu_lpart<T, 64>(g, A, perm, j0, sm);
      lu_panel<T, ROWS, SP, 64>(g, A, perm, j0, sm, info);
      lu_diag_inverses<T, 64>(g, A + j0, perm + j0, dinv + (size_t)P * 2 * 64 * 64, sm);
    } else {
      for (int r = 0; r < P; r++) lu_upart_step<T, 32>(g, A, perm, dinv, j0, r, sm);
      if (P > 0) lu_lpart<T, 32>(g, A, perm, j0, sm);
      lu_panel<T, ROWS, SP, 32>(g, A, perm, j0, sm, info);
      lu_diag_inverses<T, 32>(g, A + j0, perm + j0, dinv + (size_t)P * 2 * 64 * 64, sm);
    }
  }
  // first failing column over the workgroup (every thread tracked the same pivots)
  if (threadIdx.x == 0) info_all[box] = info;
}

template <typename T, int ROWS, int SP>
static hipError_t launch_getrf(const Geom& g, T* A, int* perm, T* dinv, int* info, int nbox, hipStream_t st) {
  hipLaunchKernelGGL((getrf_kernel<T, ROWS, SP>), dim3(nbox), dim3(kLuThreads), 0, st, g, A, perm, dinv, info, nbox);
  return hipGetLastError();
}

template <typename T>
hipError_t getrf_dispatch(const Geom& g, T* A, int* perm, T* dinv, int* info, int nbox, hipStream_t st) {
  const int rows = (g.n_pad + kLuThreads - 1) / kLuThreads;
  constexpr bool f32 = sizeof(T) == 4;
  constexpr int SP = f32 ? 8 : 4;
  if (rows <= 1) return launch_getrf<T, 1, SP>(g, A, perm, dinv, info, nbox, st);
  if (rows <= 2) return launch_getrf<T, 2, SP>(g, A, perm, dinv, info, nbox, st);
  if (rows <= 4) return launch_getrf<T, 4, SP>(g, A, perm, dinv, info, nbox, st);
  if (rows <= 6) return launch_getrf<T, 6, SP>(g, A, perm, dinv, info, nbox, st);
  if (rows <= 8) return launch_getrf<T, 8, SP>(g, A, perm, dinv, info, nbox, st);
  if (rows <= 12) return launch_getrf<T, 12, SP>(g, A, perm, dinv, info, nbox, st);
  return hipErrorInvalidValue;
}

template hipError_t getrf_dispatch<float>(const Geom&, float*, int*, float*, int*, int, hipStream_t);
template hipError_t getrf_dispatch<double>(const Geom&, double*, int*, double*, int*, int, hipStream_t);

}  // namespace hps
