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
// schedules of the triangular solves: one launch per 64-row block row, or one launch
// per sweep with every block row of a (box, column tile) in one workgroup
constexpr int kTrsmRows = 0, kTrsmSweep = 1;

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
// One FP64 vector in LDS against a stored factor (the one-vector-per-matrix solves:
// interior solves, adjoint solves, interface fronts), one 1024-thread workgroup per
// matrix.  Row updates use 16 lanes per row and keep 8 rows in flight per 16-lane group
// (512 row reads outstanding per workgroup), so that a single workgroup per matrix is
// not held to a few GB/s by memory latency.
// ---------------------------------------------------------------------------
constexpr int kVecThreads = 1024;

// v[j] -= sum_{c < w} A_j[c] v[c0 + c] for rows j in [j0, j1), A_j = rowptr(j) + c0, w <= 64.
// The rows updated lie outside [c0, c0 + w).
template <typename T, typename RowPtr>
__device__ inline void vec_rows_update(double* v, int j0, int j1, int c0, int w, RowPtr rowptr) {
  constexpr int RB = 8;
  const int lane16 = threadIdx.x & 15, grp = threadIdx.x >> 4, ngrp = blockDim.x >> 4;
  double xv[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int c = lane16 + 16 * q;
    xv[q] = c < w ? v[c0 + c] : 0.0;
  }
  for (int jb = j0 + grp * RB; jb < j1; jb += ngrp * RB) {
    T a[RB][4];
#pragma unroll
    for (int r = 0; r < RB; r++) {
      const bool ok = jb + r < j1;
      const T* row = ok ? rowptr(jb + r) + c0 : nullptr;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int c = lane16 + 16 * q;
        a[r][q] = (ok && c < w) ? row[c] : T(0);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; r++) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 4; q++) acc += (double)a[r][q] * xv[q];
      for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
      if (lane16 == 0 && jb + r < j1) v[jb + r] -= acc;
    }
  }
  __syncthreads();
}

// v[c] -= sum_{i < w} A_{r0+i}[c] v[r0 + i] for columns c in [c0, c1), A_i = rowptr(i)
// (the transposed update: consecutive threads read consecutive columns of a row).
template <typename T, typename RowPtr>
__device__ inline void vec_cols_update(double* v, int r0, int w, int c0, int c1, RowPtr rowptr) {
  for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < w; i += 8) {
#pragma unroll
      for (int u = 0; u < 8; u++)
        if (i + u < w) acc[u] += (double)rowptr(r0 + i + u)[c] * v[r0 + i + u];
    }
    v[c] -= ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  __syncthreads();
}

// v[s + t] = sum_{k < w} Inv[t][k] v[s + k] (or Inv[k][t] when trans) for t < w, Inv a
// stored 64 x 64 block (row stride 64): 16 lanes per output, 1024 threads.
template <typename T>
__device__ inline void vec_block_inverse(double* v, double* tmp, const T* Inv, int s, int w, bool trans) {
  const int lane16 = threadIdx.x & 15, t = threadIdx.x >> 4;
  if (t < w) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int k = lane16 + 16 * q;
      if (k < w) acc += (double)(trans ? Inv[k * 64 + t] : Inv[t * 64 + k]) * v[s + k];
    }
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (lane16 == 0) tmp[t] = acc;
  }
  __syncthreads();
  if ((int)threadIdx.x < w) v[s + threadIdx.x] = tmp[threadIdx.x];
  __syncthreads();
}

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
  const double* D2z;   // [p][p] s2[2] D*D
  const int* coords;   // [n] interior node -> ii | jj << 8 | kk << 16
  // Right-hand-side columns inside the solves (B, Y, the FP32 residual) are kept in 16-column
  // groups in an internal order; X and everything outside the solves use the natural one.
  const int* gmap;     // [ldx/16] internal group -> natural group
  const int* ginv;     // [ldx/16] natural group -> internal group
};

// internal position of natural right-hand-side column c, and back
__device__ inline int rhs_icol(const Geom& g, int c) { return g.ginv[c >> 4] * 16 + (c & 15); }
__device__ inline int rhs_ncol(const Geom& g, int ic) { return g.gmap[ic >> 4] * 16 + (ic & 15); }

// Schedule record kinds for the recursive LU and solves (record = {kind, a1..a7}):
//   kOpPanel {c0, w}                 factor columns [c0, c0+w) (w <= 64)
//   kOpGemm  {m0, m1, n0, n1, k0, k1} rows [m0,m1) x cols [n0,n1) -= F[., k0:k1] X[k0:k1, .]
//   kOpRows  {r0, r1, cA, cB}         rows [r0, r1) := L[r0:r1, r0:r1]^-1 rows on columns [cA, cB),
//                                     left-looking 64-row blocks (r1 - r0 <= kLuRowsMax)
constexpr int kOpPanel = 0, kOpGemm = 2, kOpRows = 3;
constexpr int kLuRowsMax = 256;

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

// ---------------------------------------------------------------------------
// Pipelined workgroup tile GEMM:  acc -= A[rows, k0:k1) * B[k0:k1, tile cols)
//
// GM x GN waves; wave (wm, wn) owns rows [wm*WRT*16, +WRT*16) and columns
// [wn*WCT*16, +WCT*16) of the MT x NT tile.  Both operands are staged through
// double-buffered LDS in chunks of KC: while the MFMAs of chunk c read LDS, the
// 16-byte global loads of chunks c+1 .. c+PF sit in staging registers (PF sets)
// and chunk c+1 is written to the other buffer afterwards, so each chunk costs
// one barrier and a global load has PF chunks of math to arrive.  A fragments are read as 4 consecutive
// k values per lane (the MFMA k slot g = lane/16 stands for k = 4g + t, t the
// step); B fragments are the matching rows.
//   arow(r): pointer to A row r of the tile (r in [0, MT)), nullptr -> zeros;
//   brow(k): pointer to B[k][tile col 0]; bcols: valid tile columns (rest zero).
//   (k1 - k0) % KC == 0.  smem: SMEM elements.
// ---------------------------------------------------------------------------
template <typename T, int WRT, int WCT, int GM, int GN, int KC, int PF = 1>
struct TileGemm {
  static constexpr int KCHUNK = KC;
  static constexpr int MT = GM * WRT * 16;
  static constexpr int NT = GN * WCT * 16;
  static constexpr int NTHR = GM * GN * 64;
  static constexpr int VEC = 16 / sizeof(T);  // elements per 16-byte load
  static constexpr int LDA = KC + VEC;        // padded LDS row lengths
  static constexpr int LDB = NT + VEC;
  static constexpr int ABUF = MT * LDA, BBUF = KC * LDB;
  static constexpr int SMEM = 2 * (ABUF + BBUF);
  static constexpr int ALOADS = MT * KC / (NTHR * VEC);
  static constexpr int BLOADS = KC * NT / (NTHR * VEC);
  static_assert(ALOADS >= 1 && MT * KC == ALOADS * NTHR * VEC, "A chunk must split evenly");
  static_assert(BLOADS >= 1 && KC * NT == BLOADS * NTHR * VEC, "B chunk must split evenly");
  typedef typename Mfma<T>::acc acc_t;
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));

  struct NoHook {
    __device__ void operator()(int) const {}
  };

  // after_chunk(c) runs after the MFMAs of chunk c (every wave, uniform): a caller can
  // fold acc into a second accumulator there without restarting the pipeline.
  template <typename ARow, typename BRow, typename Hook = NoHook>
  __device__ static void run(acc_t (&acc)[WRT][WCT], ARow arow, BRow brow, int bcols, int k0, int k1, T* smem,
                             Hook after_chunk = Hook()) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave % GM, wn = wave / GM;
    const int g = lane >> 4, c16 = lane & 15;
    const int nchunk = (k1 - k0) / KC;
    if (nchunk <= 0) return;
    // per-thread A staging rows (fixed over the k loop)
    const T* asrc[ALOADS];
#pragma unroll
    for (int q = 0; q < ALOADS; q++) {
      const int e = (tid + q * NTHR) * VEC;
      asrc[q] = arow(e / KC);
      if (asrc[q]) asrc[q] += e % KC;
    }
    vec_t ast[PF][ALOADS], bst[PF][BLOADS];
    auto gload = [&](int kb, int set) {
#pragma unroll
      for (int q = 0; q < ALOADS; q++) {
        if (asrc[q]) {
          ast[set][q] = *reinterpret_cast<const vec_t*>(asrc[q] + kb);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; v++) ast[set][q][v] = T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < BLOADS; q++) {
        const int e = (tid + q * NTHR) * VEC;
        const int kk = e / NT, c = e - kk * NT;
        if (c < bcols) {
          bst[set][q] = *reinterpret_cast<const vec_t*>(brow(kb + kk) + c);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; v++) bst[set][q][v] = T(0);
        }
      }
    };
    auto lstore = [&](T* buf, int set) {
#pragma unroll
      for (int q = 0; q < ALOADS; q++) {
        const int e = (tid + q * NTHR) * VEC;
        *reinterpret_cast<vec_t*>(buf + (e / KC) * LDA + e % KC) = ast[set][q];
      }
      T* bb = buf + ABUF;
#pragma unroll
      for (int q = 0; q < BLOADS; q++) {
        const int e = (tid + q * NTHR) * VEC;
        const int kk = e / NT, c = e - kk * NT;
        *reinterpret_cast<vec_t*>(bb + kk * LDB + c) = bst[set][q];
      }
    };
    auto compute = [&](const T* buf) {
      const T* as = buf;
      const T* bs = buf + ABUF;
#pragma unroll
      for (int s = 0; s < KC / 16; s++) {
        T a[WRT][4];
#pragma unroll
        for (int rt = 0; rt < WRT; rt++) Vec4<T>::load(as + ((wm * WRT + rt) * 16 + c16) * LDA + 16 * s + 4 * g, a[rt]);
#pragma unroll
        for (int t = 0; t < 4; t++) {
          T bv[WCT];
#pragma unroll
          for (int ct = 0; ct < WCT; ct++) bv[ct] = bs[(16 * s + 4 * g + t) * LDB + (wn * WCT + ct) * 16 + c16];
#pragma unroll
          for (int rt = 0; rt < WRT; rt++)
#pragma unroll
            for (int ct = 0; ct < WCT; ct++) acc[rt][ct] = Mfma<T>::op(-a[rt][t], bv[ct], acc[rt][ct]);
        }
      }
    };
    // Chunk c lives in staging set c % PF; the loop is unrolled by PF so the sets are
    // static.  Loads are issued unconditionally (past the end they reread the last
    // chunk) so that the compiler's wait counts keep PF chunks in flight.
#pragma unroll
    for (int j = 0; j < PF; j++) gload(k0 + (j < nchunk ? j : nchunk - 1) * KC, j);
    __syncthreads();  // previous users of smem are done
    lstore(smem, 0);
    int c0 = 0;
    for (; c0 + PF <= nchunk; c0 += PF) {
#pragma unroll
      for (int j = 0; j < PF; j++) {
        const int c = c0 + j;
        T* cur = smem + (c & 1) * (ABUF + BBUF);
        T* nxt = smem + ((c + 1) & 1) * (ABUF + BBUF);
        __syncthreads();
        const int cl = c + PF < nchunk ? c + PF : nchunk - 1;
        gload(k0 + cl * KC, j);  // set j held chunk c, already in LDS
        compute(cur);
        after_chunk(c);
        if (c + 1 < nchunk) lstore(nxt, (j + 1) % PF);
      }
    }
#pragma unroll
    for (int j = 0; j + 1 < PF; j++) {  // the last nchunk % PF chunks: nothing left to load
      const int c = c0 + j;
      if (c < nchunk) {
        T* cur = smem + (c & 1) * (ABUF + BBUF);
        T* nxt = smem + ((c + 1) & 1) * (ABUF + BBUF);
        __syncthreads();
        compute(cur);
        after_chunk(c);
        if (c + 1 < nchunk) lstore(nxt, (j + 1) % PF);
      }
    }
  }
};

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
