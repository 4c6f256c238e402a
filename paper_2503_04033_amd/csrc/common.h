// Device-side building blocks shared by the leaf-box kernels (gfx950 / CDNA4).
//
// Storage conventions (see include/hps_leaf.h):
//   * per-box matrices are row-major with padded leading dimension;
//   * the LU factors keep rows where they were assembled and carry the row
//     permutation as an index vector perm[position] = physical row, so pivoting
//     never moves data (a row gather in row-major storage is a contiguous read);
//   * n_pad is a multiple of 32, LU panels are 64 wide (the last may be 32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hps {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;
constexpr int kPanel = 64;  // LU panel width == row block of the triangular solves

// ---------------------------------------------------------------------------
// MFMA 16x16x4 wrappers.  Operand layout (both precisions): lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  Accumulator layout differs:
//   f32: lane l holds C[4*(l/16)+i][l%16], i = 0..3
//   f64: lane l holds C[(l/16)+4*i][l%16], i = 0..3
// ---------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<float> {
  typedef f4 acc;
  __device__ static inline acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <> struct Mfma<double> {
  typedef d4 acc;
  __device__ static inline acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

// Four consecutive elements (16-byte aligned for float, 2x16 for double).
template <typename T> struct Vec4;
template <> struct Vec4<float> {
  __device__ static inline void load(const float* p, float v[4]) {
    f4 x = *reinterpret_cast<const f4*>(p);
    v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
  }
};
template <> struct Vec4<double> {
  __device__ static inline void load(const double* p, double v[4]) {
    d2 x = *reinterpret_cast<const d2*>(p);
    d2 y = *reinterpret_cast<const d2*>(p + 2);
    v[0] = x[0]; v[1] = x[1]; v[2] = y[0]; v[3] = y[1];
  }
};

// ---------------------------------------------------------------------------
// Geometry of one plan, passed to kernels by value.
// ---------------------------------------------------------------------------
struct Geom {
  int p, m, n, nb, n_pad, nrhs, ldx, npanel;
  double s2[3];    // (2/h_a)^2: scale of the second derivative along axis a
  double s1[3];    // 2/h_a: scale of the first derivative
  double kappa2;   // kappa^2
  const double* D;     // [p][p] Gauss-Lobatto differentiation matrix on [-1,1]
  const double* D2;    // [p][p] D*D
};

__device__ inline int panel_start(int r) { return r * kPanel; }
__device__ inline int panel_width(const Geom& g, int r) {
  int s = r * kPanel;
  return (g.n_pad - s) < kPanel ? (g.n_pad - s) : kPanel;
}

// ---------------------------------------------------------------------------
// Workgroup tile GEMM:  acc -= A[rows, k0:k1) * B[k0:k1, cols)
//
// The workgroup has NW waves; wave w owns rows [w*RT*16, (w+1)*RT*16) of the
// tile and all CT*16 columns.  A rows are read straight from global memory:
// for a 16-wide k chunk, lane l reads the 4 consecutive elements
// A[row0 + l%16][kc + 4*(l/16) .. +3] and MFMA step t uses element t, i.e. the
// instruction's k slot g = l/16 stands for k = kc + 4g + t (the matching B
// element is B[kc + 4g + t][col]).  B rows are staged in LDS in chunks of KC
// rows shared by all waves.  arow(rt) returns the row pointer of this lane's
// A row in row tile rt (nullptr for rows beyond the tile -> treated as zero);
// brow(k) the pointer to B[k][col0].
// ---------------------------------------------------------------------------
template <typename T, int NW, int RT, int CT, int KC, typename ARow, typename BRow>
__device__ inline void wg_gemm_sub(typename Mfma<T>::acc (&acc)[RT][CT], ARow arow, BRow brow, int k0, int k1,
                                   T* lds_b, int ldb, int col0, int W) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int c16 = lane & 15;
  const T* ap[RT];
#pragma unroll
  for (int rt = 0; rt < RT; rt++) ap[rt] = arow(rt);
  for (int kb = k0; kb < k1; kb += KC) {
    const int kc_n = (k1 - kb) < KC ? (k1 - kb) : KC;  // multiple of 16
    __syncthreads();
    // stage B[kb:kb+kc_n, 0:W) -> lds_b[kk][c]
    for (int e = tid; e < kc_n * W; e += NW * 64) {
      int kk = e / W, c = e - kk * W;
      lds_b[kk * ldb + c] = brow(kb + kk)[c];
    }
    __syncthreads();
    for (int kc = 0; kc < kc_n; kc += 16) {
      T a[RT][4];
#pragma unroll
      for (int rt = 0; rt < RT; rt++) {
        if (ap[rt]) {
          Vec4<T>::load(ap[rt] + kb + kc + 4 * g, a[rt]);
        } else {
          a[rt][0] = a[rt][1] = a[rt][2] = a[rt][3] = T(0);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; t++) {
        T bv[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ct++) bv[ct] = lds_b[(kc + 4 * g + t) * ldb + col0 + ct * 16 + c16];
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
          for (int ct = 0; ct < CT; ct++) acc[rt][ct] = Mfma<T>::op(-a[rt][t], bv[ct], acc[rt][ct]);
      }
    }
  }
}

// acc += A[rows, 0:K) * C[0:K, col0 + cols) with A rows from global memory
// (row pointer per lane as in wg_gemm_sub) and C already resident in LDS.
template <typename T, int RT, int CT, typename ARow>
__device__ inline void wg_gemm_lds_add(typename Mfma<T>::acc (&acc)[RT][CT], ARow arow, const T* lds_c, int ldc,
                                       int K, int col0) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int c16 = lane & 15;
  const T* ap[RT];
#pragma unroll
  for (int rt = 0; rt < RT; rt++) ap[rt] = arow(rt);
  for (int kc = 0; kc < K; kc += 16) {
    T a[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; rt++) Vec4<T>::load(ap[rt] + kc + 4 * g, a[rt]);
#pragma unroll
    for (int t = 0; t < 4; t++) {
      T bv[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ct++) bv[ct] = lds_c[(kc + 4 * g + t) * ldc + col0 + ct * 16 + c16];
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) acc[rt][ct] = Mfma<T>::op(a[rt][t], bv[ct], acc[rt][ct]);
    }
  }
}

// Load / store an accumulator tile: element (r, c) of row tile rt, column tile
// ct lives at rowptr(rt, r)[ct*16 + c] with r the tile-local row.
template <typename T, int RT, int CT, typename RowPtr>
__device__ inline void acc_load(typename Mfma<T>::acc (&acc)[RT][CT], RowPtr rowptr) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const T* p = rowptr(rt, Mfma<T>::row(lane, i));
        acc[rt][ct][i] = p ? p[ct * 16 + (lane & 15)] : T(0);
      }
}

template <typename T, int RT, int CT, typename RowPtr>
__device__ inline void acc_store(const typename Mfma<T>::acc (&acc)[RT][CT], RowPtr rowptr) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        T* p = rowptr(rt, Mfma<T>::row(lane, i));
        if (p) p[ct * 16 + (lane & 15)] = acc[rt][ct][i];
      }
}

}  // namespace hps
