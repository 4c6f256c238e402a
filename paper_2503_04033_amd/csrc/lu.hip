// a2 + a3 -- batched dense LU with partial pivoting of the interior blocks A_ii
// and the triangular solves X = U^{-1} L^{-1} P B with its factors.
//
// The paper factors every box's interior block A_ii and solves with it (Alg. 1,
// the per-box solution operator; Alg. 2, the per-box interior load solve; A_ii is
// block diagonal over boxes, Sec. 2.2).  The factorization is a recursive column
// split, the solves are block rows:
//
//   lu(c0, c1):  if c1 - c0 <= 64: pivoted panel factorization
//                else: lu(c0, mid); U12 = L11^{-1} A12 (triangular solve: up to
//                256 rows left-looking 64-row blocks, above that split again with
//                a tile GEMM between the halves); A22 -= L21 U12 (tile GEMM on
//                MFMA); lu(mid, c1)
//   solve:       L Y = P B and U X = Y as left-looking 64-row block rows: a tile
//                GEMM over the finished rows, then a product with the stored
//                64 x 64 inverse of the diagonal block
//
// so nearly all flops are MFMA tile GEMMs.  The recursion depends only on the
// matrix size, so the host unrolls it into an op list once per plan and launches
// one kernel per op over all boxes of a chunk: a GEMM kernel (many workgroups per
// box, each one output tile, XCD-aware placement so a box's tiles share one L2),
// a block-row solve kernel, and a panel kernel (one workgroup per box, sub-panels
// in registers, workgroup-wide pivot search).  Each kernel gets its own register
// budget and occupancy.
//
// Rows are never moved: perm[pos] names the physical row at position pos (a
// row gather in row-major storage is a contiguous read).  Pivot rule: largest
// modulus among the rows not yet pivoted, ties to the lowest current position;
// after each sub-panel the chosen pivots take the next positions in order and
// the remaining rows keep their relative order.
#include <type_traits>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace hps {

constexpr int kLuThreads = 512;
constexpr int kLuWaves = kLuThreads / 64;

// Columns of a panel held in registers at a time: the widest of 32, 16, 8, 4 whose
// ROWS x CW block takes at most 96 VGPRs with 512 threads (one workgroup per CU keeps the
// rest of the 256-register budget for the L values and the pivot row in flight), 48 with
// 1024 threads (128 registers per thread).
template <typename T, int ROWS, int NT = 512>
struct PanelChunk {
  static constexpr int B = NT >= 1024 ? 48 : 96;
  static constexpr int regs(int cw) { return ROWS * cw * (int)(sizeof(T) / 4); }
  static constexpr int CW = regs(32) <= B ? 32 : (regs(16) <= B ? 16 : (regs(8) <= B ? 8 : 4));
};

// f(std::integral_constant<int, I>) for I = B .. E-1, expanded at compile time (indices into
// register arrays stay static however long the body is).
template <int B, int E, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// LDS of the panel kernel.  M = L11^{-1} and Nn = U11^{-1} of the panel's growing
// diagonal block (positions [j0, j0+npv)), kept up to date after every chunk, so the U
// rows of the earlier pivots in a new chunk are one parallel product and the
// diagonal-block inverses needed by the solves come out at the end for free.
template <typename T, int CW, int NWV>
struct LuSmem {
  T M[64 * 65];
  T Nn[64 * 65];
  T ub[64 * CW];           // U rows of the earlier pivots in the chunk columns (npv x CW)
  T stg[64 * CW];          // their raw values; later Z = Nn * ub
  T lq[CW * 64];           // the chunk's pivot rows' L values in earlier columns (CW x npv)
  T t1[CW * 64];           // lq * M
  T uq[CW * CW];           // inverse of the chunk pivots' CW x CW upper block
  T PR[CW * CW];           // the chunk's pivot rows in the chunk columns (L left, U on and right)
  T wrow[2][NWV][CW];
  T wval[2][NWV];
  int wslot[2][NWV];
  int pphys[64];           // physical row of the panel's k-th pivot
  int cnt[24 * NWV];  // per (row slot r < 24, wave): rows that stay candidates
};

// DPP lane moves (GFX9 encodings: row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143).  A lane whose source lies outside its row of 16, or whose row
// ROWS leaves out, gets `id`.
template <int CTRL, int ROWS = 0xf>
__device__ inline int dpp_move(int id, int v) {
  return __builtin_amdgcn_update_dpp(id, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ inline float dpp_move(float id, float v) {
  return __int_as_float(dpp_move<CTRL, ROWS>(__float_as_int(id), __float_as_int(v)));
}
template <int CTRL, int ROWS = 0xf>
__device__ inline double dpp_move(double id, double v) {
  const long long a = __double_as_longlong(id), b = __double_as_longlong(v);
  const int lo = dpp_move<CTRL, ROWS>((int)a, (int)b);
  const int hi = dpp_move<CTRL, ROWS>((int)(a >> 32), (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Reduction with an associative, commutative op (identity id) over the first row of 16
// lanes (WAVE false) or over the whole wave, returned in every lane.  Every lane must be
// active.
template <bool WAVE, typename V, typename Op>
__device__ inline V dpp_reduce(V v, V id, Op op) {
  v = op(v, dpp_move<0x111>(id, v));
  v = op(v, dpp_move<0x112>(id, v));
  v = op(v, dpp_move<0x114>(id, v));
  v = op(v, dpp_move<0x118>(id, v));  // lane 15 of each row: the row's result
  if constexpr (WAVE) {
    v = op(v, dpp_move<0x142, 0xa>(id, v));  // lanes 31 and 63: two rows each
    v = op(v, dpp_move<0x143, 0xc>(id, v));  // lane 63: all four rows
  }
  return lane_value(v, WAVE ? 63 : 15);
}

// The pivot candidate of the lanes (of row 0, or of the wave): the largest modulus, the
// lowest slot among the lanes that hold it (an empty candidate has modulus -1 and slot
// 0x7fffffff).  Returned in every lane.
template <bool WAVE, typename T>
__device__ inline void argmax_lanes(T& best, int& slot) {
  // (fmax: the moduli hold no NaN, a NaN entry having been taken as infinity)
  const T m = dpp_reduce<WAVE>(best, T(-INFINITY), [](T a, T b) { return fmax(a, b); });
  slot = dpp_reduce<WAVE>(best == m ? slot : 0x7fffffff, 0x7fffffff, [](int a, int b) { return a < b ? a : b; });
  best = m;
}

template <typename T> struct Store4;
template <> struct Store4<float> {
  __device__ static inline void store(float* p, const float* v) {
    *reinterpret_cast<f4*>(p) = f4{v[0], v[1], v[2], v[3]};
  }
};
template <> struct Store4<double> {
  __device__ static inline void store(double* p, const double* v) {
    *reinterpret_cast<d2*>(p) = d2{v[0], v[1]};
    *reinterpret_cast<d2*>(p + 2) = d2{v[2], v[3]};
  }
};

// Pivoted factorization of panel columns [j0, j0+W) for positions >= j0.  Thread t
// owns the rows at positions j0 + t + 512 r (r < ROWS) of the panel's start for the
// whole panel, so a row is read and written by one thread only.  The columns go in
// chunks of CW held in registers (left-looking between chunks, right-looking inside
// one).  Per chunk (columns [cb, cb+CW), npv = cb - j0 pivots chosen before):
//   (a) U rows of the earlier pivots in the chunk: ub = M * A[pivots, chunk)
//   (b) candidate rows: v -= L[row, j0:cb) * ub, the L values read as whole
//       128-byte lines
//   (c) per column: per-wave best candidate (modulus, lowest position on ties) and
//       its row to LDS, one barrier, every thread picks the winner; candidates are
//       scaled and updated in registers
//   (d) write back, (e) extend M and Nn with the chunk's pivots (block triangular
//       inverses)
// Candidates never change their relative order, so "lowest position" is the lowest
// starting slot.  Rows at positions >= pivot_end are eliminated like the others but never
// become pivots (a partial factorization whose trailing block is a Schur complement).  At the end the pivots take positions j0.. in order and the other
// rows follow in their previous order; M and Nn go to dinv_panel as Linv / Uinv.
template <typename T, int ROWS, int CW, int W, int NT>
__device__ __attribute__((always_inline)) inline void lu_panel(const Geom& g, T* A, int* perm, int j0, int pivot_end,
                                                               LuSmem<T, CW, NT / 64>& sm, int& info, T* dinv_panel) {
  static_assert(W % CW == 0 && CW % 4 == 0, "chunks tile the panel");
  constexpr int LB = CW < 16 ? CW : 16;  // L values loaded per step of (b)
  const int N = g.n_pad, lda = N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nrem = N - j0;
  int phys[ROWS];
  // -1: candidate, >= 0: index of the pivot it became, -2: no row, -3: a row at or past
  // pivot_end (updated like a candidate, never chosen as a pivot)
  int pk[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    const int s = tid + NT * r;
    phys[r] = s < nrem ? perm[j0 + s] : 0;
    pk[r] = s < nrem ? (j0 + s < pivot_end ? -1 : -3) : -2;
  }
  for (int h = 0; h < W / CW; h++) {
    const int cb = j0 + h * CW;
    const int npv = h * CW;
    // every slot loads (a slot with no row reads row phys = 0 and is never used): loads
    // outside branches are waited for once, not one row at a time
    T v[ROWS][CW];
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      const T* row = A + (size_t)phys[r] * lda + cb;
#pragma unroll
      for (int c = 0; c < CW; c += 4) Vec4<T>::load(row + c, v[r] + c);
    }
    if (npv > 0) {
      // (a)
#pragma unroll
      for (int r = 0; r < ROWS; r++)
        if (pk[r] >= 0)
#pragma unroll
          for (int c = 0; c < CW; c++) sm.stg[pk[r] * CW + c] = v[r][c];
      __syncthreads();
      for (int e = tid; e < npv * CW; e += NT) {
        const int k = e / CW, c = e - k * CW;
        T s = T(0);
        for (int i = 0; i <= k; i++) s += sm.M[k * 65 + i] * sm.stg[i * CW + c];
        sm.ub[e] = s;
        A[(size_t)sm.pphys[k] * lda + cb + c] = s;
      }
      __syncthreads();
      // (b)
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (pk[r] != -1 && pk[r] != -3) continue;
        const T* row = A + (size_t)phys[r] * lda + j0;
        for (int k0 = 0; k0 < npv; k0 += LB) {
          T lb[LB];
#pragma unroll
          for (int u = 0; u < LB; u += 4) Vec4<T>::load(row + k0 + u, lb + u);
#pragma unroll
          for (int u = 0; u < LB; u++)
#pragma unroll
            for (int c = 0; c < CW; c++) v[r][c] -= lb[u] * sm.ub[(k0 + u) * CW + c];
        }
      }
    }
    // (c)
    static_for<0, CW>([&](auto ic) __attribute__((always_inline)) {
      constexpr int c = decltype(ic)::value;
      T best = T(-1);
      int bslot = 0x7fffffff;
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (pk[r] == -1) {
          T a = fabs(v[r][c]);
          if (a != a) a = T(INFINITY);  // a NaN is taken as the pivot and flagged below
          const int s = tid + NT * r;
          if (a > best || (a == best && s < bslot)) { best = a; bslot = s; }
        }
      }
      argmax_lanes<true>(best, bslot);  // the wave's candidate, in every lane
      const int buf = c & 1;
      if (bslot == 0x7fffffff) {
        if (lane == 0) { sm.wval[buf][wave] = T(-1); sm.wslot[buf][wave] = bslot; }
      } else if ((bslot & (NT - 1)) == tid) {
        sm.wval[buf][wave] = best;
        sm.wslot[buf][wave] = bslot;
#pragma unroll
        for (int r = 0; r < ROWS; r++)
          if (r == bslot / NT)
#pragma unroll
            for (int cc = 0; cc < CW; cc++) sm.wrow[buf][wave][cc] = v[r][cc];
      }
      __syncthreads();
      // the waves' candidates: lane l of each row reads wave l % (NT / 64), one LDS round trip
      static_assert(16 % (NT / 64) == 0, "a row of 16 lanes holds every wave's candidate");
      best = sm.wval[buf][lane % (NT / 64)];
      bslot = sm.wslot[buf][lane % (NT / 64)];
      argmax_lanes<false>(best, bslot);
      const int wbest = bslot == 0x7fffffff ? 0 : (bslot & (NT - 1)) >> 6;  // the winner's wave
      const T* pr = sm.wrow[buf][wbest];
      if ((bslot & (NT - 1)) == tid) {
#pragma unroll
        for (int r = 0; r < ROWS; r++)
          if (r == bslot / NT) {
            pk[r] = npv + c;
            sm.pphys[npv + c] = phys[r];
          }
      }
      if (tid < CW) sm.PR[c * CW + tid] = pr[tid];
      const T pv = pr[c];
      if (!(pv != T(0) && isfinite(pv)) && info == 0) info = cb + c + 1;
      const T inv = pv != T(0) ? T(1) / pv : T(0);
#pragma unroll
      for (int r = 0; r < ROWS; r++) {
        if (pk[r] == -1 || pk[r] == -3) {
          const T l = v[r][c] * inv;
          v[r][c] = l;
#pragma unroll
          for (int cc = c + 1; cc < CW; cc++) v[r][cc] -= l * pr[cc];
        }
      }
    });
    // (d) candidates and this chunk's pivots; earlier pivots got their U rows in (a)
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
      if (pk[r] == -1 || pk[r] == -3 || pk[r] >= npv) {
        T* row = A + (size_t)phys[r] * lda + cb;
#pragma unroll
        for (int c = 0; c < CW; c += 4) Store4<T>::store(row + c, v[r] + c);
      }
    }
    __syncthreads();
    // (e) M <- [[M, 0], [-Lq^{-1} lq M, Lq^{-1}]],  Nn <- [[Nn, -Nn ub Uq^{-1}], [0, Uq^{-1}]]
    for (int e = tid; e < CW * npv; e += NT) {
      const int i = e / npv, k = e - i * npv;
      sm.lq[i * 64 + k] = A[(size_t)sm.pphys[npv + i] * lda + j0 + k];
    }
    __syncthreads();
    for (int e = tid; e < CW * npv; e += NT) {
      const int i = e / npv, j = e - i * npv;
      T s = T(0);
      for (int k = j; k < npv; k++) s += sm.lq[i * 64 + k] * sm.M[k * 65 + j];
      sm.t1[i * 64 + j] = s;
    }
    for (int e = tid; e < npv * CW; e += NT) {
      const int r = e / CW, c = e - r * CW;
      T s = T(0);
      for (int i = r; i < npv; i++) s += sm.Nn[r * 65 + i] * sm.ub[i * CW + c];
      sm.stg[e] = s;
    }
    __syncthreads();
    if (tid < npv + CW) {
      const int j = tid;
      T x[CW];
      static_for<0, CW>([&](auto ii) __attribute__((always_inline)) {
        constexpr int i = decltype(ii)::value;
        T s = j < npv ? -sm.t1[i * 64 + j] : (j - npv == i ? T(1) : T(0));
#pragma unroll
        for (int r = 0; r < i; r++) s -= sm.PR[i * CW + r] * x[r];
        x[i] = s;
        sm.M[(npv + i) * 65 + j] = s;
      });
    } else if (tid >= 64 && tid < 64 + CW) {
      const int j = tid - 64;
      T y[CW];
      static_for<0, CW>([&](auto ii) __attribute__((always_inline)) {
        constexpr int i = CW - 1 - decltype(ii)::value;
        T s = (i == j) ? T(1) : T(0);
#pragma unroll
        for (int k = i + 1; k < CW; k++) s -= sm.PR[i * CW + k] * y[k];
        y[i] = s / sm.PR[i * CW + i];
      });
#pragma unroll
      for (int i = 0; i < CW; i++) sm.uq[i * CW + j] = i <= j ? y[i] : T(0);
    }
    __syncthreads();
    for (int e = tid; e < (npv + CW) * CW; e += NT) {
      const int r = e / CW, j = e - r * CW;
      T s;
      if (r < npv) {
        s = T(0);
#pragma unroll
        for (int i = 0; i < CW; i++) s -= sm.stg[r * CW + i] * sm.uq[i * CW + j];
      } else {
        s = sm.uq[(r - npv) * CW + j];
      }
      sm.Nn[r * 65 + npv + j] = s;
    }
    __syncthreads();
  }
  // new position order: the W pivots, then the other rows in their previous order
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int pre[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    const unsigned long long mask = __ballot(pk[r] == -1 || pk[r] == -3);
    pre[r] = __popcll(mask & lt);
    if (lane == 0) sm.cnt[r * (NT / 64) + wave] = __popcll(mask);
  }
  __syncthreads();
  int base = j0 + W;
#pragma unroll
  for (int r = 0; r < ROWS; r++) {
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < (NT / 64); w++) {
      const int cw = sm.cnt[r * (NT / 64) + w];
      tot += cw;
      if (w < wave) before += cw;
    }
    if (pk[r] == -1 || pk[r] == -3) perm[base + before + pre[r]] = phys[r];
    base += tot;
  }
  if (tid < W) perm[j0 + tid] = sm.pphys[tid];
  T* Linv = dinv_panel;
  T* Uinv = dinv_panel + 64 * 64;
  for (int e = tid; e < W * W; e += NT) {
    const int i = e / W, k = e - i * W;
    Linv[i * 64 + k] = i > k ? sm.M[i * 65 + k] : (i == k ? T(1) : T(0));
    Uinv[i * 64 + k] = i <= k ? sm.Nn[i * 65 + k] : T(0);
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__device__ inline bool map_box_tile(int nbox, int ntile, int& box, int& tile) {
  // consecutive workgroup ids go round-robin to the 8 XCDs: give all tiles of a
  // box ids on one XCD so they share its L2.  Fewer than 8 boxes (the large interface
  // fronts): a box's tiles spread over every XCD instead.
  const int id = blockIdx.x;
  if (nbox < 8) {
    box = id / ntile;
    tile = id - box * ntile;
    return box < nbox;
  }
  const int xcd = id & 7, slot = id >> 3;
  const int lb = slot / ntile;
  tile = slot - lb * ntile;
  box = xcd + 8 * lb;
  return box < nbox;
}

__global__ void lu_init_kernel(int N, int* perm_all, int* info, int nbox) {
  const int box = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
    perm_all[(size_t)box * N + i] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) info[box] = 0;
}

template <typename T, int ROWS, int CW, int W, int NT>
__global__ __launch_bounds__(NT, NT >= 1024 ? 1 : 2) void lu_panel_kernel(Geom g, T* A_all, int* perm_all, T* dinv_all,
                                                                           int* info_all, int nbox, int c0,
                                                                           int pivot_end) {
  __shared__ LuSmem<T, CW, NT / 64> sm;
  const int box = blockIdx.x;
  if (box >= nbox) return;
  const int N = g.n_pad;
  T* A = A_all + (size_t)box * N * N;
  int* perm = perm_all + (size_t)box * N;
  T* dp = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64 + (size_t)(c0 / kPanel) * 2 * 64 * 64;
  int info = 0;
  lu_panel<T, ROWS, CW, W, NT>(g, A, perm, c0, pivot_end, sm, info, dp);
  if (threadIdx.x == 0 && info != 0 && info_all[box] == 0) info_all[box] = info;
}

template <typename T> struct GemmCfg;
// 64 x 64 workgroup tiles, 4 waves of 32 x 32, K chunks of 16 with two chunks in
// flight: the best shape measured for every update size in the recursion on gfx950
// (more resident workgroups per CU outweigh the smaller operand reuse; the second
// staging set hides the global-load latency behind one more chunk of MFMAs).
template <> struct GemmCfg<float> { typedef TileGemm<float, 2, 2, 2, 2, 16, 2> G; };
template <> struct GemmCfg<double> { typedef TileGemm<double, 2, 2, 2, 2, 16, 2> G; };

// C[row(pos)][n] -= sum_k F[perm[pos]][k] * B[row(k)][n] for pos in [m0,m1),
// n in [n0,n1), k in [k0,k1).  F is the factor (ld n_pad, rows via perm); B and
// C are the target X: the factor itself (PERM, rows via perm) or a right-hand
// side block (rows direct, ld ldx).  Row and k ranges never overlap within one
// op, so reads and writes are disjoint.
template <typename T, bool PERM>
__global__ __launch_bounds__(256, 4) void gemm_op_kernel(Geom g, const T* F_all, const int* perm_all, T* X_all,
                                                         int ld, size_t xstride, int m0, int m1, int n0, int n1,
                                                         int k0, int k1, int nbox, int ntm, int ntn,
                                                         const int* active) {
  typedef typename GemmCfg<T>::G G;
  constexpr int WRT = G::MT / (2 * 16), WCT = G::NT / (2 * 16);
  __shared__ T smem[G::SMEM];
  int box, tile;
  if (!map_box_tile(nbox, ntm * ntn, box, tile)) return;
  if (active && active[box] == 0) return;
  const int N = g.n_pad;
  const T* F = F_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  T* X = X_all + (size_t)box * xstride;
  const int tm = tile / ntn, tn = tile - tm * ntn;
  const int mt = m0 + tm * G::MT, nt = n0 + tn * G::NT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave % 2, wn = wave / 2;
  typename G::acc_t acc[WRT][WCT];
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int ct = 0; ct < WCT; ct++) acc[rt][ct] = Mfma<T>::zero();
  auto arow = [&](int r) -> const T* {
    const int pos = mt + r;
    return pos < m1 ? F + (size_t)perm[pos] * N : nullptr;
  };
  // B rows through perm: the K range of perm is staged in LDS once, so that no global
  // load of a row index sits in front of each row load of the K loop
  extern __shared__ int kperm[];  // [k1 - k0] when PERM
  if (PERM) {
    for (int i = threadIdx.x; i < k1 - k0; i += blockDim.x) kperm[i] = perm[k0 + i];
    __syncthreads();
  }
  auto brow = [&](int k) -> const T* { return X + (size_t)(PERM ? kperm[k - k0] : k) * ld + nt; };
  const int bcols = (n1 - nt) < G::NT ? (n1 - nt) : G::NT;
  G::run(acc, arow, brow, bcols, k0, k1, smem);
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int pos = mt + (wm * WRT + rt) * 16 + Mfma<T>::row(lane, i);
      if (pos < m1) {
        T* row = X + (size_t)(PERM ? perm[pos] : pos) * ld + nt + wn * WCT * 16 + (lane & 15);
#pragma unroll
        for (int ct = 0; ct < WCT; ct++)
          if (nt + (wn * WCT + ct) * 16 < n1) row[ct * 16] += acc[rt][ct][i];
      }
    }
}

// Row stride (elements) of a 64 x 64 block in LDS that is multiplied by a stored
// diagonal-block inverse (the last step of every 64-row block of a triangular solve).
constexpr int kLeafLd = 64 + 4;


// One block row of the solves, left-looking: Z = R_j - F[j rows][k range] Y[k range]
// over the finished rows, then Y_j = Inv_j Z with the stored inverse of the diagonal
// block.  Forward (L, unit diagonal): R_j = B[perm[s + i]], k in [0, s).  Backward (U):
// R_j = Y_j itself, k in [s + w, N).  One 64 x 64 output tile per workgroup: the K loop
// is the tile GEMM, the 64 x 64 x 64 inverse product reads Z from LDS.
constexpr int kTrsmSeg = 512;
constexpr int kTrsmSegAbove = 4096;

template <typename T, bool UPPER, bool SEG>
__device__ __attribute__((always_inline)) inline void solve_block_row(const Geom& g, const T* F, const int* perm,
                                                                      const T* Inv, const T* B, T* Y, double* Xb,
                                                                      int xmode, int s, int w, int nt, int ks,
                                                                      int bdirect, const T* Y0, T* smem) {
  typedef typename GemmCfg<T>::G G;
  static_assert(G::MT == 64 && G::NT == 64, "one 64 x 64 tile per workgroup");
  static_assert(G::SMEM >= 64 * kLeafLd, "Z must fit the GEMM staging buffer");
  constexpr int WRT = 2, WCT = 2;
  const int N = g.n_pad, ld = g.ldx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave % 2, wn = wave / 2;
  const int g4 = lane >> 4, c16 = lane & 15;
  // Forward sweep: rows of the tile above ks (a multiple of 64) are exactly zero, so a
  // block row that ends there is stored as zeros and the K range starts at ks.
  if (!UPPER && s + w <= ks) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = wave * 16 + Mfma<T>::row(lane, i);
        if (r < w) Y[(size_t)(s + r) * ld + nt + ct * 16 + c16] = T(0);
      }
    return;
  }
  // acc = -F Y first, R_j added once at the end: every rounding of the K loop is relative
  // to the running sum of products, not to R_j (this matters where the two cancel)
  typename G::acc_t acc[WRT][WCT];
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int ct = 0; ct < WCT; ct++) acc[rt][ct] = Mfma<T>::zero();
  auto arow = [&](int r) -> const T* { return r < w ? F + (size_t)perm[s + r] * N : nullptr; };
  auto brow = [&](int k) -> const T* { return Y + (size_t)k * ld + nt; };
  // With SEG (FP32, long K) the running sum `part` is folded into acc every
  // kTrsmSeg values of k, so that no accumulator adds more than kTrsmSeg products in
  // sequence; the fold runs inside the K loop and keeps its pipeline going.
  const int k0 = UPPER ? s + w : ks, k1 = UPPER ? N : s;
  if constexpr (!SEG) {
    G::run(acc, arow, brow, 64, k0, k1, smem);
  } else {
    typename G::acc_t part[WRT][WCT];
#pragma unroll
    for (int rt = 0; rt < WRT; rt++)
#pragma unroll
      for (int ct = 0; ct < WCT; ct++) part[rt][ct] = Mfma<T>::zero();
    const int nchunk = (k1 - k0) / G::KCHUNK;
    auto fold = [&](int c) {
      if ((c + 1) % (kTrsmSeg / G::KCHUNK) == 0 || c + 1 == nchunk) {
#pragma unroll
        for (int rt = 0; rt < WRT; rt++)
#pragma unroll
          for (int ct = 0; ct < WCT; ct++) {
            acc[rt][ct] += part[rt][ct];
            part[rt][ct] = Mfma<T>::zero();
          }
      }
    };
    G::run(part, arow, brow, 64, k0, k1, smem, fold);
  }
  __syncthreads();  // every wave is done with the staging buffer
  T* zs = smem;     // Z [64][kLeafLd]
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = (wm * WRT + rt) * 16 + Mfma<T>::row(lane, i);
      const T* rr =
          r < w ? (UPPER ? Y + (size_t)(s + r) * ld : B + (size_t)(bdirect ? s + r : perm[s + r]) * ld) + nt : nullptr;
#pragma unroll
      for (int ct = 0; ct < WCT; ct++) {
        const int c = (wn * WCT + ct) * 16 + c16;
        zs[r * kLeafLd + c] = rr ? rr[c] + acc[rt][ct][i] : T(0);
      }
    }
  // Y_j = Inv_j Z: the wave's 16 rows of the inverse (columns past w zeroed) times all 64
  // columns of Z, the inverse read one 16-column chunk ahead; for X += Y (xmode 2) the
  // old X is loaded first, in flight during the product
  const T* irow = Inv + (wave * 16 + c16) * 64 + 4 * g4;
  T ia[4];
  Vec4<T>::load(irow, ia);
  // X += Y (xmode 2) or X = Y0 + Y (xmode 3): the old X or Y0 is loaded now
  const bool xadd = Xb && (xmode == 2 || xmode == 3);
  double xo[4][4];
  if (xadd) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = wave * 16 + Mfma<T>::row(lane, i);
        xo[ct][i] = r >= w ? 0.0
                    : xmode == 2 ? Xb[(size_t)(s + r) * ld + g.gmap[(nt >> 4) + ct] * 16 + c16]
                                 : (double)Y0[(size_t)(s + r) * ld + nt + ct * 16 + c16];
      }
  }
  __syncthreads();
  typename Mfma<T>::acc out[4];
#pragma unroll
  for (int ct = 0; ct < 4; ct++) out[ct] = Mfma<T>::zero();
#pragma unroll
  for (int kc = 0; kc < 4; kc++) {
    T ib[4];
    if (kc + 1 < 4) Vec4<T>::load(irow + (kc + 1) * 16, ib);
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int k = kc * 16 + 4 * g4 + t;
      const T a = k < w ? ia[t] : T(0);
      const T* zr = zs + k * kLeafLd + c16;
#pragma unroll
      for (int ct = 0; ct < 4; ct++) out[ct] = Mfma<T>::op(a, zr[ct * 16], out[ct]);
    }
    if (kc + 1 < 4)
#pragma unroll
      for (int t = 0; t < 4; t++) ia[t] = ib[t];
  }
  // the finished rows; the backward sweep may also write them to the FP64 X (xmode 1:
  // X = Y, 2: X += Y, 3: X = Y0 + Y)
#pragma unroll
  for (int ct = 0; ct < 4; ct++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = wave * 16 + Mfma<T>::row(lane, i);
      if (r < w) {
        Y[(size_t)(s + r) * ld + nt + ct * 16 + c16] = out[ct][i];
        // X is in the natural column order
        const size_t ex = (size_t)(s + r) * ld + g.gmap[(nt >> 4) + ct] * 16 + c16;
        if (Xb) Xb[ex] = xadd ? xo[ct][i] + (double)out[ct][i] : (double)out[ct][i];
      }
    }
}

// ---------------------------------------------------------------------------
// 128-row block rows (FP32 solves): twice the rows per launch, so the finished rows Y of
// a tile are read once per 128 rows instead of per 64 and a sweep takes half the launches.
// The 128 x 64 output tile is the tile GEMM with the four waves stacked (32 rows x 64
// columns each); the 128 x 128 diagonal block is applied as its two stored 64 x 64
// inverses and the coupling block between them:
//   forward (L):  Y0 = Linv0 Z0;  Z1 -= L10 Y0;  Y1 = Linv1 Z1
//   backward (U): Y1 = Uinv1 Z1;  Z0 -= U01 Y1;  Y0 = Uinv0 Z0
// ---------------------------------------------------------------------------
constexpr int kBlockRows = 128;
template <typename T> struct GemmCfg128;
template <> struct GemmCfg128<float> { typedef TileGemm<float, 2, 4, 4, 1, 16, 2> G; };
template <> struct GemmCfg128<double> { typedef TileGemm<double, 2, 4, 4, 1, 16, 2> G; };
template <typename T>
constexpr int smem128() {
  return GemmCfg128<T>::G::SMEM > kBlockRows * kLeafLd ? GemmCfg128<T>::G::SMEM : kBlockRows * kLeafLd;
}

// out = Inv Z for one 64-row half: wave w forms rows [16w, 16w + 16) x 64 columns; Inv is a
// stored 64 x 64 inverse (row stride 64), Z the LDS rows [z0, z0 + 64) (stride kLeafLd),
// k < wk (the half's width; LDS rows past it hold zeros).
template <typename T>
__device__ inline void half_inverse(const T* Inv, const T* zs, int z0, int wk, typename Mfma<T>::acc (&out)[4]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g4 = lane >> 4, c16 = lane & 15;
  const T* irow = Inv + (wave * 16 + c16) * 64 + 4 * g4;
  T ia[4];
  Vec4<T>::load(irow, ia);
#pragma unroll
  for (int ct = 0; ct < 4; ct++) out[ct] = Mfma<T>::zero();
#pragma unroll
  for (int kc = 0; kc < 4; kc++) {
    T ib[4];
    if (kc + 1 < 4) Vec4<T>::load(irow + (kc + 1) * 16, ib);
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int k = kc * 16 + 4 * g4 + t;
      const T a = k < wk ? ia[t] : T(0);
      const T* zr = zs + (z0 + k) * kLeafLd + c16;
#pragma unroll
      for (int ct = 0; ct < 4; ct++) out[ct] = Mfma<T>::op(a, zr[ct * 16], out[ct]);
    }
    if (kc + 1 < 4)
#pragma unroll
      for (int t = 0; t < 4; t++) ia[t] = ib[t];
  }
}

// cor = -C Yh for one 64-row half: C rows from the factor (rowp(r) + c0, r < wr, k < wk),
// Yh the LDS rows [y0, y0 + 64); wave w forms rows [16w, 16w + 16).
template <typename T, typename RowP>
__device__ inline void half_couple(RowP rowp, int wr, int c0, int wk, const T* zs, int y0,
                                   typename Mfma<T>::acc (&cor)[4]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g4 = lane >> 4, c16 = lane & 15;
  const int r = wave * 16 + c16;
  const T* arow = r < wr ? rowp(r) + c0 : nullptr;
#pragma unroll
  for (int ct = 0; ct < 4; ct++) cor[ct] = Mfma<T>::zero();
#pragma unroll
  for (int kc = 0; kc < 4; kc++) {
    T a[4];
    if (arow && kc * 16 + 4 * g4 < wk) Vec4<T>::load(arow + kc * 16 + 4 * g4, a);  // never past column c0 + wk
    else a[0] = a[1] = a[2] = a[3] = T(0);
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int k = kc * 16 + 4 * g4 + t;
      const T av = k < wk ? -a[t] : T(0);
      const T* yr = zs + (y0 + k) * kLeafLd + c16;
#pragma unroll
      for (int ct = 0; ct < 4; ct++) cor[ct] = Mfma<T>::op(av, yr[ct * 16], cor[ct]);
    }
  }
}

template <typename T, bool UPPER, bool SEG>
__device__ __attribute__((always_inline)) inline void solve_block_row128(
    const Geom& g, const T* F, const int* perm, const T* Inv0, const T* Inv1, const T* B, T* Y, double* Xb, int xmode,
    int s, int w, int nt, int ks, int bdirect, const T* Y0, T* smem) {
  typedef typename GemmCfg128<T>::G G;
  static_assert(G::MT == 128 && G::NT == 64, "one 128 x 64 tile per workgroup");
  constexpr int WRT = 2, WCT = 4;
  const int N = g.n_pad, ld = g.ldx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, c16 = lane & 15;
  if (!UPPER && s + w <= ks) {  // every row of this block row of the tile is zero
    for (int e = threadIdx.x; e < w * 64; e += blockDim.x) Y[(size_t)(s + e / 64) * ld + nt + (e & 63)] = T(0);
    return;
  }
  typename G::acc_t acc[WRT][WCT];
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int ct = 0; ct < WCT; ct++) acc[rt][ct] = Mfma<T>::zero();
  auto arow = [&](int r) -> const T* { return r < w ? F + (size_t)perm[s + r] * N : nullptr; };
  auto brow = [&](int k) -> const T* { return Y + (size_t)k * ld + nt; };
  const int k0 = UPPER ? s + w : ks, k1 = UPPER ? N : s;
  if constexpr (!SEG) {
    G::run(acc, arow, brow, 64, k0, k1, smem);
  } else {
    typename G::acc_t part[WRT][WCT];
#pragma unroll
    for (int rt = 0; rt < WRT; rt++)
#pragma unroll
      for (int ct = 0; ct < WCT; ct++) part[rt][ct] = Mfma<T>::zero();
    const int nchunk = (k1 - k0) / G::KCHUNK;
    auto fold = [&](int c) {
      if ((c + 1) % (kTrsmSeg / G::KCHUNK) == 0 || c + 1 == nchunk) {
#pragma unroll
        for (int rt = 0; rt < WRT; rt++)
#pragma unroll
          for (int ct = 0; ct < WCT; ct++) {
            acc[rt][ct] += part[rt][ct];
            part[rt][ct] = Mfma<T>::zero();
          }
      }
    };
    G::run(part, arow, brow, 64, k0, k1, smem, fold);
  }
  __syncthreads();  // every wave is done with the staging buffer
  T* zs = smem;     // Z [128][kLeafLd]; rows past w hold zeros
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = wave * 32 + rt * 16 + Mfma<T>::row(lane, i);
      const T* rr =
          r < w ? (UPPER ? Y + (size_t)(s + r) * ld : B + (size_t)(bdirect ? s + r : perm[s + r]) * ld) + nt : nullptr;
#pragma unroll
      for (int ct = 0; ct < WCT; ct++) {
        const int c = ct * 16 + c16;
        zs[r * kLeafLd + c] = rr ? rr[c] + acc[rt][ct][i] : T(0);
      }
    }
  __syncthreads();
  const int w0 = w < 64 ? w : 64, w1 = w - w0;
  // rows [h0, h0 + wk) of the block: Y, and for the backward sweep X (1: X = Y, 2: X += Y,
  // 3: X = Y0 + Y; X in the natural column order)
  auto store = [&](typename Mfma<T>::acc (&out)[4], int h0, int wk) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = wave * 16 + Mfma<T>::row(lane, i);
        if (r < wk) {
          const size_t row = (size_t)(s + h0 + r) * ld;
          Y[row + nt + ct * 16 + c16] = out[ct][i];
          if (Xb) {
            const size_t ex = row + g.gmap[(nt >> 4) + ct] * 16 + c16;
            const double old = xmode == 2 ? Xb[ex] : (xmode == 3 ? (double)Y0[row + nt + ct * 16 + c16] : 0.0);
            Xb[ex] = old + (double)out[ct][i];
          }
        }
      }
  };
  // the finished half back into LDS (rows [z0, z0 + wk)), where the coupling reads it
  auto to_lds = [&](typename Mfma<T>::acc (&out)[4], int z0, int wk) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = wave * 16 + Mfma<T>::row(lane, i);
        if (r < wk) zs[(z0 + r) * kLeafLd + ct * 16 + c16] = out[ct][i];
      }
  };
  auto add_lds = [&](typename Mfma<T>::acc (&cor)[4], int z0, int wk) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int r = wave * 16 + Mfma<T>::row(lane, i);
        if (r < wk) zs[(z0 + r) * kLeafLd + ct * 16 + c16] += cor[ct][i];
      }
  };
  typename Mfma<T>::acc out[4], cor[4];
  if (!UPPER) {
    half_inverse<T>(Inv0, zs, 0, w0, out);
    store(out, 0, w0);
    if (w1 > 0) {
      __syncthreads();  // every wave has read Z0
      to_lds(out, 0, w0);
      __syncthreads();
      half_couple<T>([&](int r) { return F + (size_t)perm[s + 64 + r] * N; }, w1, s, w0, zs, 0, cor);
      add_lds(cor, 64, w1);
      __syncthreads();
      half_inverse<T>(Inv1, zs, 64, w1, out);
      store(out, 64, w1);
    }
  } else {
    if (w1 > 0) {
      half_inverse<T>(Inv1, zs, 64, w1, out);
      store(out, 64, w1);
      __syncthreads();  // every wave has read Z1
      to_lds(out, 64, w1);
      __syncthreads();
      half_couple<T>([&](int r) { return F + (size_t)perm[s + r] * N; }, w0, s + 64, w1, zs, 64, cor);
      add_lds(cor, 0, w0);
      __syncthreads();
    }
    half_inverse<T>(Inv0, zs, 0, w0, out);
    store(out, 0, w0);
  }
}

template <typename T, bool UPPER, bool SEG, int OCC>
__global__ __launch_bounds__(256, OCC) void trsm_row128_kernel(Geom g, const T* F_all, const int* perm_all,
                                                             const T* dinv_all, const T* B_all, T* Y_all, int s,
                                                             int w, int nbox, int ntn, const int* active,
                                                             double* X_all, int xmode, const int* kstart, int bdirect,
                                                             const T* Y0_all) {
  __shared__ T smem[smem128<T>()];
  int box, tn;
  if (!map_box_tile(nbox, ntn, box, tn)) return;
  if (active && active[box] == 0) return;
  const int N = g.n_pad;
  const size_t xs = (size_t)N * g.ldx;
  const T* Inv0 = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64 + (size_t)(s / kPanel) * 2 * 64 * 64 +
                  (UPPER ? 64 * 64 : 0);
  solve_block_row128<T, UPPER, SEG>(g, F_all + (size_t)box * N * N, perm_all + (size_t)box * N, Inv0,
                                    Inv0 + 2 * 64 * 64, B_all + (size_t)box * xs, Y_all + (size_t)box * xs,
                                    X_all ? X_all + (size_t)box * xs : nullptr, xmode, s, w, tn * 64,
                                    kstart ? kstart[(size_t)box * ntn + tn] : 0, bdirect,
                                    Y0_all ? Y0_all + (size_t)box * xs : nullptr, smem);
}

// One block row per launch: workgroup (box, 64-column tile).  OCC: waves per SIMD the
// register allocation must allow (workgroups resident per CU, LDS permitting).
template <typename T, bool UPPER, bool SEG, int OCC>
__global__ __launch_bounds__(256, OCC) void trsm_row_kernel(Geom g, const T* F_all, const int* perm_all,
                                                          const T* dinv_all, const T* B_all, T* Y_all, int s, int w,
                                                          int nbox, int ntn, const int* active, double* X_all,
                                                          int xmode, const int* kstart, int bdirect, const T* Y0_all) {
  typedef typename GemmCfg<T>::G G;
  __shared__ T smem[G::SMEM];
  int box, tn;
  if (!map_box_tile(nbox, ntn, box, tn)) return;
  if (active && active[box] == 0) return;
  const int N = g.n_pad;
  const size_t xs = (size_t)N * g.ldx;
  const T* Inv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64 + (size_t)(s / kPanel) * 2 * 64 * 64 +
                 (UPPER ? 64 * 64 : 0);
  solve_block_row<T, UPPER, SEG>(g, F_all + (size_t)box * N * N, perm_all + (size_t)box * N, Inv,
                                 B_all + (size_t)box * xs, Y_all + (size_t)box * xs,
                                 X_all ? X_all + (size_t)box * xs : nullptr, xmode, s, w, tn * 64,
                                 kstart ? kstart[(size_t)box * ntn + tn] : 0, bdirect,
                                 Y0_all ? Y0_all + (size_t)box * xs : nullptr, smem);
}

// Short triangular solves of the LU recursion (rows [r0, r1), r1 - r0 <= kLuRowsMax, of
// the U block right of a factored panel): one launch per 64-row block s, left-looking like
// the block rows of the solves but on the factor itself, rows through perm:
//   Z = A[perm[s + i]][cols] - L[s + i, r0:s) U[r0:s, cols],  U_s = Linv_s Z  (in place).
// The K loop is the tile GEMM (the K range of perm staged in LDS), the leaf product reads
// Z from LDS; the short GEMMs and separate leaf launches of a deeper recursion go away.
template <typename T>
__global__ __launch_bounds__(256, 4) void lu_rows_kernel(Geom g, T* A_all, const int* perm_all, const T* dinv_all,
                                                         int r0, int s, int w, int cA, int cB, int nbox, int ntn) {
  typedef typename GemmCfg<T>::G G;
  static_assert(G::MT == 64 && G::NT == 64, "one 64 x 64 tile per workgroup");
  static_assert(G::SMEM >= 64 * kLeafLd, "Z must fit the GEMM staging buffer");
  constexpr int WRT = 2, WCT = 2;
  __shared__ T smem[G::SMEM];
  __shared__ int kperm[kLuRowsMax];
  int box, tn;
  if (!map_box_tile(nbox, ntn, box, tn)) return;
  const int N = g.n_pad;
  T* A = A_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  const T* Inv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64 + (size_t)(s / kPanel) * 2 * 64 * 64;
  const int nt = cA + tn * 64;
  const int bcols = (cB - nt) < 64 ? (cB - nt) : 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave % 2, wn = wave / 2;
  const int g4 = lane >> 4, c16 = lane & 15;
  for (int i = threadIdx.x; i < s - r0; i += blockDim.x) kperm[i] = perm[r0 + i];
  __syncthreads();
  typename G::acc_t acc[WRT][WCT];
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int ct = 0; ct < WCT; ct++) acc[rt][ct] = Mfma<T>::zero();
  auto arow = [&](int r) -> const T* { return r < w ? A + (size_t)perm[s + r] * N : nullptr; };
  auto brow = [&](int k) -> const T* { return A + (size_t)kperm[k - r0] * N + nt; };
  G::run(acc, arow, brow, bcols, r0, s, smem);
  __syncthreads();  // every wave is done with the staging buffer
  T* zs = smem;     // Z [64][kLeafLd]
#pragma unroll
  for (int rt = 0; rt < WRT; rt++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = (wm * WRT + rt) * 16 + Mfma<T>::row(lane, i);
      const T* rr = r < w ? A + (size_t)perm[s + r] * N + nt : nullptr;
#pragma unroll
      for (int ct = 0; ct < WCT; ct++) {
        const int c = (wn * WCT + ct) * 16 + c16;
        zs[r * kLeafLd + c] = (rr && c < bcols) ? rr[c] + acc[rt][ct][i] : T(0);
      }
    }
  const T* irow = Inv + (wave * 16 + c16) * 64 + 4 * g4;
  T ia[4];
  Vec4<T>::load(irow, ia);
  __syncthreads();
  typename Mfma<T>::acc out[4];
#pragma unroll
  for (int ct = 0; ct < 4; ct++) out[ct] = Mfma<T>::zero();
#pragma unroll
  for (int kc = 0; kc < 4; kc++) {
    T ib[4];
    if (kc + 1 < 4) Vec4<T>::load(irow + (kc + 1) * 16, ib);
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int k = kc * 16 + 4 * g4 + t;
      const T a = k < w ? ia[t] : T(0);
      const T* zr = zs + k * kLeafLd + c16;
#pragma unroll
      for (int ct = 0; ct < 4; ct++) out[ct] = Mfma<T>::op(a, zr[ct * 16], out[ct]);
    }
    if (kc + 1 < 4)
#pragma unroll
      for (int t = 0; t < 4; t++) ia[t] = ib[t];
  }
#pragma unroll
  for (int ct = 0; ct < 4; ct++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = wave * 16 + Mfma<T>::row(lane, i);
      const int c = ct * 16 + c16;
      if (r < w && c < bcols) A[(size_t)perm[s + r] * N + nt + c] = out[ct][i];
    }
}

// One whole triangular sweep per workgroup: the right-hand-side columns of a box are
// independent, so the workgroup of (box, 64-column tile) runs every block row of its
// tile in order (top down for L, bottom up for U) with no other workgroup involved.
// One launch per sweep: no drain between block rows, and the epilogue of one block row
// overlaps the K loops of the other workgroups resident on the CU.  The block row just
// stored is the first or last K chunk of the next one; the barrier after the stores
// makes it visible to every wave of the workgroup (one CU, one vector L1).
template <typename T, bool UPPER, bool SEG, int OCC>
__global__ __launch_bounds__(256, OCC) void trsm_sweep_kernel(Geom g, const T* F_all, const int* perm_all,
                                                            const T* dinv_all, const T* B_all, T* Y_all, int nbox,
                                                            int ntn, const int* active, double* X_all, int xmode,
                                                            const int* kstart, int bdirect, const T* Y0_all) {
  typedef typename GemmCfg<T>::G G;
  __shared__ T smem[G::SMEM];
  int box, tn;
  if (!map_box_tile(nbox, ntn, box, tn)) return;
  if (active && active[box] == 0) return;
  const int N = g.n_pad;
  const size_t xs = (size_t)N * g.ldx;
  const T* F = F_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  const T* dinv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64 + (UPPER ? 64 * 64 : 0);
  T* Y = Y_all + (size_t)box * xs;
  const T* B = B_all + (size_t)box * xs;
  double* Xb = X_all ? X_all + (size_t)box * xs : nullptr;
  const T* Y0 = Y0_all ? Y0_all + (size_t)box * xs : nullptr;
  const int nblk = (N + kPanel - 1) / kPanel;
  const int ks = kstart ? kstart[(size_t)box * ntn + tn] : 0;
#pragma unroll 1
  for (int q = 0; q < nblk; q++) {
    const int jb = UPPER ? nblk - 1 - q : q;
    const int s = jb * kPanel, w = (N - s) < kPanel ? (N - s) : kPanel;
    solve_block_row<T, UPPER, SEG>(g, F, perm, dinv + (size_t)jb * 2 * 64 * 64, B, Y, Xb, xmode, s, w, tn * 64, ks,
                                   bdirect, Y0, smem);
    __syncthreads();  // Y_j stored before the next block row loads it
  }
}


// The 128-row schedule of trsm_sweep_kernel: one workgroup per (box, 64-column tile) runs
// every 128-row block row of its tile.
template <typename T, bool UPPER, bool SEG, int OCC>
__global__ __launch_bounds__(256, OCC) void trsm_sweep128_kernel(Geom g, const T* F_all, const int* perm_all,
                                                               const T* dinv_all, const T* B_all, T* Y_all, int nbox,
                                                               int ntn, const int* active, double* X_all, int xmode,
                                                               const int* kstart, int bdirect, const T* Y0_all) {
  __shared__ T smem[smem128<T>()];
  int box, tn;
  if (!map_box_tile(nbox, ntn, box, tn)) return;
  if (active && active[box] == 0) return;
  const int N = g.n_pad;
  const size_t xs = (size_t)N * g.ldx;
  const T* F = F_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  const T* dinv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64 + (UPPER ? 64 * 64 : 0);
  T* Y = Y_all + (size_t)box * xs;
  const T* B = B_all + (size_t)box * xs;
  double* Xb = X_all ? X_all + (size_t)box * xs : nullptr;
  const T* Y0 = Y0_all ? Y0_all + (size_t)box * xs : nullptr;
  const int nblk = (N + kBlockRows - 1) / kBlockRows;
  const int ks = kstart ? kstart[(size_t)box * ntn + tn] : 0;
#pragma unroll 1
  for (int q = 0; q < nblk; q++) {
    int s, w;
    sweep_block(N, kBlockRows, UPPER, q, s, w);
    const T* Inv0 = dinv + (size_t)(s / kPanel) * 2 * 64 * 64;
    solve_block_row128<T, UPPER, SEG>(g, F, perm, Inv0, Inv0 + 2 * 64 * 64, B, Y, Xb, xmode, s, w, tn * 64, ks,
                                      bdirect, Y0, smem);
    __syncthreads();  // Y_j stored before the next block row loads it
  }
}

// ---------------------------------------------------------------------------
// host-side sequencing
// ---------------------------------------------------------------------------
static int grid_for(int nbox, int ntile) { return (nbox < 8 ? nbox : 8 * ((nbox + 7) / 8)) * ntile; }

// algorithmic flops of one schedule record over nbox boxes (for the profiler)
static double gemm_flops(const int* op, int nbox) {
  return 2.0 * (op[2] - op[1]) * (double)(op[4] - op[3]) * (op[6] - op[5]) * nbox;
}

template <typename T, bool PERM>
static hipError_t launch_gemm(const Geom& g, const T* F, const int* perm, T* X, int ld, size_t xstride, const int* op,
                              int nbox, const int* active, hipStream_t st) {
  typedef typename GemmCfg<T>::G G;
  const int m0 = op[1], m1 = op[2], n0 = op[3], n1 = op[4], k0 = op[5], k1 = op[6];
  const int ntm = (m1 - m0 + G::MT - 1) / G::MT, ntn = (n1 - n0 + G::NT - 1) / G::NT;
  const size_t shm = PERM ? sizeof(int) * (size_t)(k1 - k0) : 0;
  hipLaunchKernelGGL((gemm_op_kernel<T, PERM>), dim3(grid_for(nbox, ntm * ntn)), dim3(256), shm, st, g, F, perm, X,
                     ld, xstride, m0, m1, n0, n1, k0, k1, nbox, ntm, ntn, active);
  return hipGetLastError();
}


template <typename T, int ROWS, int NT>
static hipError_t launch_panel(const Geom& g, T* A, int* perm, T* dinv, int* info, int nbox, int c0, int w,
                               int pivot_end, hipStream_t st) {
  constexpr int CW = PanelChunk<T, ROWS, NT>::CW;
  if (w == 64)
    hipLaunchKernelGGL((lu_panel_kernel<T, ROWS, CW, 64, NT>), dim3(nbox), dim3(NT), 0, st, g, A, perm, dinv, info,
                       nbox, c0, pivot_end);
  else
    hipLaunchKernelGGL((lu_panel_kernel<T, ROWS, (CW < 32 ? CW : 32), 32, NT>), dim3(nbox), dim3(NT), 0, st, g, A,
                       perm, dinv, info, nbox, c0, pivot_end);
  return hipGetLastError();
}

template <typename T, int ROWS, int NT = kLuThreads>
static hipError_t run_lu(const Geom& g, const std::vector<int>& ops, T* A, int* perm, T* dinv, int* info, int nbox,
                         hipStream_t st, Profiler* prof, int pivot_end) {
  const int N = g.n_pad;
  hipLaunchKernelGGL(lu_init_kernel, dim3((N + 255) / 256, nbox), dim3(256), 0, st, N, perm, info, nbox);
  hipError_t e = hipGetLastError();
  for (size_t q = 0; q + 8 <= ops.size() && e == hipSuccess; q += 8) {
    const int* op = ops.data() + q;
    if (op[0] == kOpPanel) {
      ProfScope ps(prof, Profiler::kLuPanel, 0.0, st);
      e = launch_panel<T, ROWS, NT>(g, A, perm, dinv, info, nbox, op[1], op[2], pivot_end, st);
    } else if (op[0] == kOpRows) {
      const int r0 = op[1], r1 = op[2], cA = op[3], cB = op[4], ntn = (cB - cA + 63) / 64;
      for (int s = r0; s < r1 && e == hipSuccess; s += kPanel) {
        const int w = (r1 - s) < kPanel ? (r1 - s) : kPanel;
        ProfScope ps(prof, Profiler::kLuLeaf, (2.0 * w * (s - r0) + (double)w * w) * (cB - cA) * nbox, st);
        hipLaunchKernelGGL((lu_rows_kernel<T>), dim3(grid_for(nbox, ntn)), dim3(256), 0, st, g, A, perm, dinv, r0,
                           s, w, cA, cB, nbox, ntn);
        e = hipGetLastError();
      }
    } else {
      ProfScope ps(prof, Profiler::kLuGemm, gemm_flops(op, nbox), st);
      e = launch_gemm<T, true>(g, A, perm, A, N, (size_t)N * N, op, nbox, nullptr, st);
    }
  }
  return e;
}

template <typename T>
hipError_t getrf_run(const Geom& g, const std::vector<int>& ops, T* A, int* perm, T* dinv, int* info, int nbox,
                     hipStream_t st, Profiler* prof, int pivot_end, int panel_threads) {
  const int rows = (g.n_pad + kLuThreads - 1) / kLuThreads;
  const int pe = pivot_end < 0 ? g.n_pad : pivot_end;
  // 1024-thread panels (four waves per SIMD to hide the latency of each pivot step): FP32,
  // 2049..3072 rows (three rows per thread); bitwise the 512-thread result
  if constexpr (sizeof(T) == 4)
    if (panel_threads == 1024 && g.n_pad > 2048 && g.n_pad <= 3072)
      return run_lu<T, 3, 1024>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if (rows <= 1) return run_lu<T, 1>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if (rows <= 2) return run_lu<T, 2>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if (rows <= 4) return run_lu<T, 4>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if (rows <= 6) return run_lu<T, 6>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if (rows <= 8) return run_lu<T, 8>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if (rows <= 12) return run_lu<T, 12>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  if constexpr (sizeof(T) == 8) {  // interface fronts (FP64 only) up to 12288 rows
    if (rows <= 16) return run_lu<T, 16>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
    if (rows <= 20) return run_lu<T, 20>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
    if (rows <= 24) return run_lu<T, 24>(g, ops, A, perm, dinv, info, nbox, st, prof, pe);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool UPPER, bool SEG, int OCC>
static hipError_t launch_sweep(const Geom& g, const T* F, const int* perm, const T* dinv, const T* B, T* Y, int nbox,
                               const int* active, hipStream_t st, double* X, int xmode, int sched,
                               const int* kstart, int bdirect, const T* Y0) {
  const int ntn = g.ldx / 64, N = g.n_pad;
  constexpr bool R128 = solve_block_rows<T>() == kBlockRows;
  if (sched == kTrsmSweep) {
    if constexpr (R128)
      hipLaunchKernelGGL((trsm_sweep128_kernel<T, UPPER, SEG, OCC>), dim3(grid_for(nbox, ntn)), dim3(256), 0, st, g,
                         F, perm, dinv, B, Y, nbox, ntn, active, X, xmode, kstart, bdirect, Y0);
    else
      hipLaunchKernelGGL((trsm_sweep_kernel<T, UPPER, SEG, OCC>), dim3(grid_for(nbox, ntn)), dim3(256), 0, st, g, F,
                         perm, dinv, B, Y, nbox, ntn, active, X, xmode, kstart, bdirect, Y0);
    return hipGetLastError();
  }
  constexpr int BR = solve_block_rows<T>();
  const int nblk = (N + BR - 1) / BR;
  for (int q = 0; q < nblk; q++) {
    int s, w;
    sweep_block(N, BR, UPPER, q, s, w);
    if constexpr (R128)
      hipLaunchKernelGGL((trsm_row128_kernel<T, UPPER, SEG, OCC>), dim3(grid_for(nbox, ntn)), dim3(256), 0, st, g,
                         F, perm, dinv, B, Y, s, w, nbox, ntn, active, X, xmode, kstart, bdirect, Y0);
    else
      hipLaunchKernelGGL((trsm_row_kernel<T, UPPER, SEG, OCC>), dim3(grid_for(nbox, ntn)), dim3(256), 0, st, g, F,
                         perm, dinv, B, Y, s, w, nbox, ntn, active, X, xmode, kstart, bdirect, Y0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// FP32: segmented sums for long K (accuracy at p >= 19), and the occupancy the kernels are
// built for (4, 6 or 8 waves per SIMD; the 64 x 64 tile's 18.5 KB of LDS allows 8
// workgroups per CU).  FP64: 4 (its 34.5 KB of LDS allows 4).
template <typename T, bool UPPER>
static hipError_t dispatch_sweep(const Geom& g, const T* F, const int* perm, const T* dinv, const T* B, T* Y,
                                 int nbox, const int* active, hipStream_t st, double* X, int xmode, int sched,
                                 int waves, const int* kstart, int bdirect, const T* Y0) {
#define HPS_SWEEP(SEG, OCC) \
  launch_sweep<T, UPPER, SEG, OCC>(g, F, perm, dinv, B, Y, nbox, active, st, X, xmode, sched, kstart, bdirect, Y0)
  if constexpr (sizeof(T) == 4) {
    if (g.n_pad > kTrsmSegAbove) return HPS_SWEEP(true, 4);
    if (waves == 8) return HPS_SWEEP(false, 8);
    if (waves == 6) return HPS_SWEEP(false, 6);
  }
  return HPS_SWEEP(false, 4);
#undef HPS_SWEEP
}

// X = A^{-1} B for every active box: the forward sweep L Y = P B reads the rows of B
// through perm, the backward sweep U X = Y works in place in Y (B and Y must not alias).
// sched: kTrsmRows (one launch per block row) or kTrsmSweep (one launch per sweep);
// waves: FP32 occupancy target (see dispatch_sweep).  kstart (may be null): per (box,
// 64-column tile), a multiple of 64 above which every row of P B is zero (the forward
// sweep skips those rows).  sf: the flops the profiler records (see SolveFlops).
template <typename T>
hipError_t getrs_run(const Geom& g, const T* F, const int* perm, const T* dinv, const T* B, T* Y, int nbox,
                     const int* active, hipStream_t st, Profiler* prof, double* X, int xmode, int sched, int waves,
                     const int* kstart, int bdirect, const T* Y0, const SolveFlops* sf) {
  const int nlaunch = sched == kTrsmSweep ? 1 : (g.n_pad + solve_block_rows<T>() - 1) / solve_block_rows<T>();
  const double alg = sf ? sf->alg : 0.0;
  hipError_t e;
  {
    ProfScope ps(prof, Profiler::kSolveFwd, alg, st, nlaunch, sf ? sf->fwd_exec : 0.0);
    e = dispatch_sweep<T, false>(g, F, perm, dinv, B, Y, nbox, active, st, nullptr, 0, sched, waves, kstart, bdirect,
                                 nullptr);
  }
  if (e != hipSuccess) return e;
  {
    ProfScope ps(prof, Profiler::kSolveBwd, alg, st, nlaunch, sf ? sf->bwd_exec : 0.0);
    e = dispatch_sweep<T, true>(g, F, perm, dinv, Y, Y, nbox, active, st, xmode ? X : nullptr, xmode, sched, waves,
                                nullptr, 0, Y0);
  }
  return e;
}
template hipError_t getrf_run<float>(const Geom&, const std::vector<int>&, float*, int*, float*, int*, int, hipStream_t,
                                     Profiler*, int, int);
template hipError_t getrf_run<double>(const Geom&, const std::vector<int>&, double*, int*, double*, int*, int,
                                      hipStream_t, Profiler*, int, int);
template hipError_t getrs_run<float>(const Geom&, const float*,
                                     const int*, const float*, const float*, float*, int, const int*, hipStream_t,
                                     Profiler*, double*, int, int, int, const int*, int, const float*,
                                     const SolveFlops*);
template hipError_t getrs_run<double>(const Geom&, const double*,
                                      const int*, const double*, const double*, double*, int, const int*,
                                      hipStream_t, Profiler*, double*, int, int, int, const int*, int,
                                      const double*, const SolveFlops*);

}  // namespace hps
