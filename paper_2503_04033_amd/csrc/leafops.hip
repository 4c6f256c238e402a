// Bandwidth-bound leaf kernels: operator assembly (a1), right-hand sides, the
// FP64 residual of the refinement loop (a3), DtN assembly and loads (a4), the
// interface block reduction, reconstruction (a5), adjoint helpers (a6), nodes.
//
// Local numbering: interior node (ii, jj, kk) in [0, m)^3 (grid index = +1)
// has index ii + m jj + m^2 kk; face a = 2*axis + side holds m^2 nodes indexed
// by the tangential interior coordinates, lower axis fastest.
#include "common.h"
#include "kernels.h"

namespace hps {

// ----------------------------------------------------------------------------
// atomics on non-negative doubles: their bit patterns order like unsigned ints
// ----------------------------------------------------------------------------
__device__ inline void atomic_max_nonneg(double* addr, double v) {
  if (!(v >= 0.0)) v = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf (flags the box)
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ----------------------------------------------------------------------------
// fills (kernels rather than hipMemsetAsync so that the sequence can be captured)
// ----------------------------------------------------------------------------
__global__ void fill_zero_kernel(unsigned int* p, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  size_t nw = bytes / 4;
  int grid = (int)((nw + 255) / 256 < 65536 ? (nw + 255) / 256 : 65536);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, st, (unsigned int*)p, nw);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_int(int* p, int value, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  int grid = (int)((count + 255) / 256 < 65536 ? (count + 255) / 256 : 65536);
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// node coordinates (Sec. 2.1): x = origin + h (t + 1) / 2
// ----------------------------------------------------------------------------
__global__ void nodes_kernel(Geom g, const double* t, double h0, double h1, double h2, int nbox,
                             const double* origin, double* xi, double* xb) {
  const int box = blockIdx.y;
  const int m = g.m, mm = m * m;
  const double* o = origin + 3 * box;
  const double h[3] = {h0, h1, h2};
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.n + g.nb; e += gridDim.x * blockDim.x) {
    int c[3];
    if (e < g.n) {
      c[0] = e % m + 1;
      c[1] = (e / m) % m + 1;
      c[2] = e / mm + 1;
      double* out = xi + ((size_t)box * g.n + e) * 3;
      for (int a = 0; a < 3; a++) out[a] = o[a] + 0.5 * h[a] * (t[c[a]] + 1.0);
    } else {
      const int f = e - g.n;
      const int a = f / mm, q = f % mm, axis = a >> 1, side = a & 1;
      const int t0 = axis == 0 ? 1 : 0, t1 = axis == 2 ? 1 : 2;
      c[axis] = side ? g.p - 1 : 0;
      c[t0] = q % m + 1;
      c[t1] = q / m + 1;
      double* out = xb + ((size_t)box * g.nb + f) * 3;
      for (int d = 0; d < 3; d++) out[d] = o[d] + 0.5 * h[d] * (t[c[d]] + 1.0);
    }
  }
}

hipError_t launch_nodes(const Geom& g, const double* t, const double* h, int nbox, const double* origin, double* xi,
                        double* xb, hipStream_t st) {
  dim3 grid((g.n + g.nb + 255) / 256, nbox);
  hipLaunchKernelGGL(nodes_kernel, grid, dim3(256), 0, st, g, t, h[0], h[1], h[2], nbox, origin, xi, xb);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// a1: A_ii = -(Dxx + Dyy + Dzz) - kappa^2 diag(b) on interior nodes, identity border.
// One workgroup writes one row; each thread writes 4 consecutive columns.
// ----------------------------------------------------------------------------
template <typename T> struct Store4;
template <> struct Store4<float> {
  __device__ static void st(float* p, const double v[4]) { *reinterpret_cast<f4*>(p) = f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]}; }
};
template <> struct Store4<double> {
  __device__ static void st(double* p, const double v[4]) {
    *reinterpret_cast<d2*>(p) = d2{v[0], v[1]};
    *reinterpret_cast<d2*>(p + 2) = d2{v[2], v[3]};
  }
};

// A_ii has 3m - 2 nonzeros per row (the three D2 lines through the node; the identity
// on the padding rows), so each workgroup first writes zero rows with 16-byte stores and,
// after one barrier, the nonzeros of its rows.
constexpr int kOperatorRows = 8;

template <typename T>
__global__ __launch_bounds__(256) void operators_kernel(Geom g, int nbox, const double* b, T* A_all, double* anorm) {
  const int box = blockIdx.y;
  const int N = g.n_pad, n = g.n, m = g.m, mm = m * m, p = g.p;
  T* A = A_all + (size_t)box * N * N;
  const int r0 = blockIdx.x * kOperatorRows;
  const int nr = (N - r0) < kOperatorRows ? (N - r0) : kOperatorRows;
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  const int q4 = N / 4;
  for (int e = threadIdx.x; e < nr * q4; e += blockDim.x) {
    const int rr = e / q4, c = (e - rr * q4) * 4;
    Store4<T>::st(A + (size_t)(r0 + rr) * N + c, zero);
  }
  __syncthreads();
  const double* D2 = g.D2;
  for (int e = threadIdx.x; e < nr * 3 * m; e += blockDim.x) {
    const int rr = e / (3 * m), t = e - rr * 3 * m, line = t / m, q = t - line * m;
    const int r = r0 + rr;
    if (r >= n) {
      if (t == 0) A[(size_t)r * N + r] = T(1);
      continue;
    }
    const int cd = g.coords[r];
    const int ii = cd & 255, jj = (cd >> 8) & 255, kk = cd >> 16;
    int col;
    double v;
    if (line == 0) {  // x-line, carries the whole diagonal
      col = r - ii + q;
      v = -g.s2[0] * D2[(ii + 1) * p + q + 1];
      if (q == ii)
        v += -g.s2[1] * D2[(jj + 1) * p + jj + 1] - g.s2[2] * D2[(kk + 1) * p + kk + 1] -
             g.kappa2 * b[(size_t)box * n + r];
    } else if (line == 1) {
      if (q == jj) continue;
      col = r + m * (q - jj);
      v = -g.s2[1] * D2[(jj + 1) * p + q + 1];
    } else {
      if (q == kk) continue;
      col = r + mm * (q - kk);
      v = -g.s2[2] * D2[(kk + 1) * p + q + 1];
    }
    A[(size_t)r * N + col] = (T)v;
  }
  if ((int)threadIdx.x < nr && r0 + (int)threadIdx.x < n) {  // exact |row| sum of A_ii (FP64)
    const int r = r0 + threadIdx.x;
    const int cd = g.coords[r];
    const int ii = cd & 255, jj = (cd >> 8) & 255, kk = cd >> 16;
    double sum = 0.0;
    for (int q = 0; q < m; q++) {
      if (q != ii) sum += g.s2[0] * fabs(D2[(ii + 1) * p + q + 1]);
      if (q != jj) sum += g.s2[1] * fabs(D2[(jj + 1) * p + q + 1]);
      if (q != kk) sum += g.s2[2] * fabs(D2[(kk + 1) * p + q + 1]);
    }
    const double d = -(g.s2[0] * D2[(ii + 1) * p + ii + 1] + g.s2[1] * D2[(jj + 1) * p + jj + 1] +
                       g.s2[2] * D2[(kk + 1) * p + kk + 1]) - g.kappa2 * b[(size_t)box * n + r];
    atomic_max_nonneg(anorm + box, sum + fabs(d));
  }
}

template <typename T>
hipError_t launch_operators(const Geom& g, int nbox, const double* b, T* A, double* anorm, hipStream_t st) {
  hipError_t e = launch_fill_zero(anorm, sizeof(double) * nbox, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((operators_kernel<T>), dim3((g.n_pad + kOperatorRows - 1) / kOperatorRows, nbox), dim3(256), 0, st, g, nbox,
                     b, A, anorm);
  return hipGetLastError();
}
template hipError_t launch_operators<float>(const Geom&, int, const double*, float*, double*, hipStream_t);
template hipError_t launch_operators<double>(const Geom&, int, const double*, double*, double*, hipStream_t);

// ----------------------------------------------------------------------------
// B = [A_ib | f_i | 0] (rows >= n are zero).  A_ib (Sec. 2.2) couples interior
// node (ii,jj,kk) to the two face nodes at the ends of each of its three lines:
// entry -(2/h_a)^2 D2[c+1][e], c the node's coordinate along axis a, e = 0 or p-1.
// ----------------------------------------------------------------------------
__device__ inline double aib_entry(const Geom& g, int ii, int jj, int kk, int col) {
  const int m = g.m, mm = m * m;
  const int a = col / mm, q = col - a * mm;
  const int axis = a >> 1, side = a & 1;
  int along, tq;
  if (axis == 0) { along = ii; tq = jj + m * kk; }
  else if (axis == 1) { along = jj; tq = ii + m * kk; }
  else { along = kk; tq = ii + m * jj; }
  if (tq != q) return 0.0;
  return -g.s2[axis] * g.D2[(along + 1) * g.p + (side ? g.p - 1 : 0)];
}

// B has at most 7 nonzeros per row (A_ib: the two face nodes at the ends of each of the
// node's three lines; the load f): zero rows with 16-byte stores, then the nonzeros.
template <typename T>
__global__ __launch_bounds__(256) void rhs_kernel(Geom g, int nbox, const double* f, T* B_all, double* maxb,
                                                  double* maxbf, const double* fsc) {
  const int box = blockIdx.y;
  const int N = g.n_pad, ldx = g.ldx, n = g.n, m = g.m, mm = m * m, p = g.p;
  T* B = B_all + (size_t)box * N * ldx;
  const int r0 = blockIdx.x * kOperatorRows;
  const int nr = (N - r0) < kOperatorRows ? (N - r0) : kOperatorRows;
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  const int q4 = ldx / 4;
  for (int e = threadIdx.x; e < nr * q4; e += blockDim.x) {
    const int rr = e / q4, c = (e - rr * q4) * 4;
    Store4<T>::st(B + (size_t)(r0 + rr) * ldx + c, zero);
  }
  __syncthreads();
  double mx = 0.0, mxf = 0.0;
  for (int e = threadIdx.x; e < nr * 7; e += blockDim.x) {
    const int rr = e / 7, t = e - rr * 7, r = r0 + rr;
    if (r >= n) continue;
    double v;
    int col;
    if (t == 6) {
      if (!f) continue;
      v = f[(size_t)box * n + r] * (fsc ? 1.0 / fsc[box] : 1.0);  // (a power of two: exact)
      col = g.nb;
    } else {
      const int cd = g.coords[r];
      const int ii = cd & 255, jj = (cd >> 8) & 255, kk = cd >> 16;
      const int axis = t >> 1, side = t & 1;
      const int along = axis == 0 ? ii : (axis == 1 ? jj : kk);
      const int tq = axis == 0 ? jj + m * kk : (axis == 1 ? ii + m * kk : ii + m * jj);
      col = t * mm + tq;
      v = -g.s2[axis] * g.D2[(along + 1) * p + (side ? p - 1 : 0)];
    }
    B[(size_t)r * ldx + rhs_icol(g, col)] = (T)v;
    mx = fmax(mx, fabs(v));
    if (t == 6) mxf = fmax(mxf, fabs(v));
  }
  mx = wave_max(mx);
  mxf = wave_max(mxf);
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(maxb + box, mx);
    if (maxbf) atomic_max_nonneg(maxbf + box, mxf);
  }
}

template <typename T>
hipError_t launch_rhs(const Geom& g, int nbox, const double* f, T* B, double* maxb, hipStream_t st, double* fst,
                      const double* fsc) {
  hipError_t e = launch_fill_zero(maxb, sizeof(double) * nbox, st);
  if (e == hipSuccess && fst) e = launch_fill_zero(fst, sizeof(double) * nbox, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((rhs_kernel<T>), dim3((g.n_pad + kOperatorRows - 1) / kOperatorRows, nbox), dim3(256), 0, st, g, nbox, f, B,
                     maxb, fst, fsc);
  return hipGetLastError();
}
template hipError_t launch_rhs<float>(const Geom&, int, const double*, float*, double*, hipStream_t, double*,
                                      const double*);
template hipError_t launch_rhs<double>(const Geom&, int, const double*, double*, double*, hipStream_t, double*,
                                       const double*);

// Load-column scale of the FP32 solves: per box the power of two s with
// 1 <= max|f| / s < 2 (1 when f is zero or not finite).  The FP32 right-hand side and the
// refinement carry f / s, so a load far below FP32's range (a source's far field) is
// resolved like any other column; dividing by a power of two is exact, so loads inside
// the range give bitwise the same X.
__global__ __launch_bounds__(256) void fscale_kernel(int n, int nbox, const double* f, double* fsc) {
  __shared__ double wm[4];
  const int box = blockIdx.x;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(f[(size_t)box * n + i]));
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    int ex = 0;
    (void)frexp(mx, &ex);
    fsc[box] = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, ex - 1) : 1.0;
  }
}

hipError_t launch_fscale(const Geom& g, int nbox, const double* f, double* fsc, hipStream_t st) {
  hipLaunchKernelGGL(fscale_kernel, dim3(nbox), dim3(256), 0, st, g.n, nbox, f, fsc);
  return hipGetLastError();
}

// X's load column (natural column nb) back from f / s to f: X[:, nb] *= s.
__global__ __launch_bounds__(256) void funscale_kernel(Geom g, int nbox, double* X_all, const double* fsc) {
  const int box = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.n_pad) return;
  X_all[((size_t)box * g.n_pad + r) * g.ldx + g.nb] *= fsc[box];
}

hipError_t launch_funscale(const Geom& g, int nbox, double* X, const double* fsc, hipStream_t st) {
  hipLaunchKernelGGL(funscale_kernel, dim3((g.n_pad + 255) / 256, nbox), dim3(256), 0, st, g, nbox, X, fsc);
  return hipGetLastError();
}

// First pivoted row at which each 64-column tile of B = [A_ib | f] (columns in the
// solves' internal order, see Geom) can be nonzero.
// Column c < n_b belongs to face node c; its nonzeros in A_ib sit on the m interior
// nodes of the grid line through that node normal to its face (the D2 coupling along
// the line, Sec. 2.1), so after the row permutation its first nonzero is at
// min over the line of pos[node], pos = perm^-1.  The f column counts as dense when f
// is given; padding columns are zero.  The forward sweep L Y = P B leaves every row
// of Y above this one exactly zero for the tile.  Rounded down to a multiple of 64.
// One workgroup per box; pos lives in LDS.
constexpr int kMaxPad = 5888;  // n_pad at p = 20 is 5856

__global__ __launch_bounds__(256) void rhs_first_row_kernel(Geom g, int nbox, const int* perm_all, int has_f, int ntn,
                                                            int* kstart, int* pos_out) {
  __shared__ int pos[kMaxPad];
  __shared__ int tmin[64];
  const int box = blockIdx.x;
  const int N = g.n_pad, m = g.m, mm = m * m;
  const int* perm = perm_all + (size_t)box * N;
  for (int k = threadIdx.x; k < N; k += blockDim.x) pos[perm[k]] = k;
  for (int t = threadIdx.x; t < ntn; t += blockDim.x) tmin[t] = N;
  __syncthreads();
  for (int ic = threadIdx.x; ic < ntn * 64; ic += blockDim.x) {  // internal column order
    const int c = rhs_ncol(g, ic);
    int v = N;
    if (c < g.nb) {
      const int axis = c / (2 * mm), tq = c % mm;
      const int t0 = tq % m, t1 = tq / m;
      const int base = axis == 0 ? m * t0 + mm * t1 : (axis == 1 ? t0 + mm * t1 : t0 + m * t1);
      const int stride = axis == 0 ? 1 : (axis == 1 ? m : mm);
      for (int l = 0; l < m; l++) v = min(v, pos[base + l * stride]);
    } else if (c == g.nb && has_f) {
      v = 0;
    }
    atomicMin(&tmin[ic >> 6], v);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ntn; t += blockDim.x) kstart[(size_t)box * ntn + t] = tmin[t] / 64 * 64;
  if (pos_out)
    for (int k = threadIdx.x; k < N; k += blockDim.x) pos_out[(size_t)box * N + k] = pos[k];
}

hipError_t launch_rhs_first_row(const Geom& g, int nbox, const int* perm, int has_f, int* kstart, int* pos,
                                hipStream_t st) {
  const int ntn = g.ldx / 64;
  if (g.n_pad > kMaxPad || ntn > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rhs_first_row_kernel, dim3(nbox), dim3(256), 0, st, g, nbox, perm, has_f, ntn, kstart, pos);
  return hipGetLastError();
}

// The FP32 first solution Y (internal column order) as the FP64 X (natural order), for the
// boxes that need no correction.  One workgroup per (row, box).
__global__ __launch_bounds__(256) void x_from_y_kernel(Geom g, const float* Y_all, double* X_all,
                                                       const int* active) {
  const int box = blockIdx.y, row = blockIdx.x;
  if (active[box] != 0) return;
  const size_t base = ((size_t)box * g.n_pad + row) * g.ldx;
  for (int c = threadIdx.x; c < g.ldx; c += blockDim.x) X_all[base + c] = (double)Y_all[base + rhs_icol(g, c)];
}

hipError_t launch_x_from_y(const Geom& g, int nbox, const float* Y, double* X, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(x_from_y_kernel, dim3(g.n_pad, nbox), dim3(256), 0, st, g, Y, X, active);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// FP64 residual R = B - A_ii X through the tensor structure of A_ii (never a
// dense FP64 A_ii): -A_ii X = s2x D2 X (along x) + s2y (along y) + s2z (along z)
// + kappa^2 b X.  One workgroup per (box, CW-column chunk) stages the chunk
// X[0:n, c0:c0+CW) in LDS (read from HBM once) and forms every output from LDS;
// R goes to FP32 for the correction solve (R32 may be null), max|R| and max|X|
// per box feed the stopping test.
// ----------------------------------------------------------------------------
constexpr int kResThreads = 512;

__device__ inline bool map_box_chunk(int nbox, int nchunk, int& box, int& chunk) {
  const int id = blockIdx.x;
  const int xcd = id & 7, slot = id >> 3;
  const int lb = slot / nchunk;
  chunk = slot - lb * nchunk;
  box = xcd + 8 * lb;
  return box < nbox;
}

template <int CW, typename TX>
__global__ __launch_bounds__(kResThreads) void residual_kernel(Geom g, int nbox, const double* b, const double* f,
                                                               const TX* X_all, float* R32_all, const int* pos_all,
                                                               double* maxr, double* maxx, const int* active,
                                                               double* fst, const double* fsc) {
  extern __shared__ double xs[];  // [n][CW] then D2 interior block [m][m] and its two boundary columns
  int box, chunk;
  if (!map_box_chunk(nbox, g.ldx / CW, box, chunk)) return;
  if (active && active[box] == 0) return;
  const int m = g.m, mm = m * m, n = g.n, ldx = g.ldx, p = g.p;
  double* d2s = xs + (size_t)n * CW;   // D2[i+1][j+1]
  double* d2e = d2s + mm;              // D2[i+1][0] and D2[i+1][p-1]
  const int c0 = chunk * CW;
  const TX* X = X_all + (size_t)box * g.n_pad * ldx;
  const int* pos = pos_all ? pos_all + (size_t)box * g.n_pad : nullptr;
  for (int e = threadIdx.x; e < n * CW; e += kResThreads) {  // an FP32 X: internal column order
    const int node = e / CW, c = e - node * CW;
    xs[e] = (double)X[(size_t)node * ldx + (sizeof(TX) == 4 ? rhs_icol(g, c0 + c) : c0 + c)];
  }
  for (int e = threadIdx.x; e < mm; e += kResThreads) d2s[e] = g.D2[(e / m + 1) * p + e % m + 1];
  for (int e = threadIdx.x; e < 2 * m; e += kResThreads) d2e[e] = g.D2[(e % m + 1) * p + (e < m ? 0 : p - 1)];
  __syncthreads();
  // this thread's column and its A_ib face node (if any)
  const int c = threadIdx.x % CW;
  const int col = c0 + c;
  int axis = -1, qq = 0, side = 0;
  if (col < g.nb) {
    const int a = col / mm;
    qq = col - a * mm;
    axis = a >> 1;
    side = a & 1;
  }
  const bool fcol = (col == g.nb) && f;
  const double s2a = axis >= 0 ? g.s2[axis] : 0.0;
  double mr = 0.0, mxv = 0.0;
  const double* bb = b + (size_t)box * n;
  float* R32 = R32_all ? R32_all + (size_t)box * g.n_pad * ldx : nullptr;
  for (int node = threadIdx.x / CW; node < n; node += kResThreads / CW) {
    const int cd = g.coords[node];
    const int ii = cd & 255, jj = (cd >> 8) & 255, kk = cd >> 16;
    const double* xl = xs + (size_t)(node - ii) * CW + c;       // x-line: stride CW
    const double* yl = xs + (size_t)(node - m * jj) * CW + c;   // y-line: stride m*CW
    const double* zl = xs + (size_t)(node - mm * kk) * CW + c;  // z-line: stride mm*CW
    const double* dx = d2s + ii * m;
    const double* dy = d2s + jj * m;
    const double* dz = d2s + kk * m;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int q = 0; q < m; q++) {
      ax += dx[q] * xl[q * CW];
      ay += dy[q] * yl[q * m * CW];
      az += dz[q] * zl[q * mm * CW];
    }
    const double xv = xs[(size_t)node * CW + c];
    double bv = 0.0;
    if (axis == 0) {
      if (jj + m * kk == qq) bv = -s2a * d2e[side * m + ii];
    } else if (axis == 1) {
      if (ii + m * kk == qq) bv = -s2a * d2e[side * m + jj];
    } else if (axis == 2) {
      if (ii + m * jj == qq) bv = -s2a * d2e[side * m + kk];
    } else if (fcol) {
      bv = f[(size_t)box * n + node] * (fsc ? 1.0 / fsc[box] : 1.0);
    }
    const double r = bv + g.s2[0] * ax + g.s2[1] * ay + g.s2[2] * az + g.kappa2 * bb[node] * xv;
    if (R32) R32[(size_t)(pos ? pos[node] : node) * ldx + rhs_icol(g, col)] = (float)r;
    mr = fmax(mr, fabs(r));
    mxv = fmax(mxv, fabs(xv));
  }
  double mrf = fcol ? mr : 0.0, mxf = fcol ? mxv : 0.0;  // the load column alone
  mr = wave_max(mr);
  mxv = wave_max(mxv);
  mrf = wave_max(mrf);
  mxf = wave_max(mxf);
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(maxr + box, mr);
    atomic_max_nonneg(maxx + box, mxv);
    if (fst) {
      atomic_max_nonneg(fst + nbox + box, mrf);
      atomic_max_nonneg(fst + 2 * nbox + box, mxf);
    }
  }
}

// Residual for boxes with m <= 16 interior nodes per direction.  One workgroup of
// 64 CB NW threads per (box, CB columns); NW waves share a column, each owning a run of
// H = ceil(m / NW) output slabs.  For a fixed column the z-slab kk of X is an m x m
// matrix S[ii][jj]; its x- and y-derivative terms are D2i S and S D2i^T, both written as
// 16x16x4 FP64 MFMA chains into one 16x16 accumulator (rows ii, columns jj, zero
// padded), by the wave that owns slab kk.  The z-derivative couples slabs: as each slab
// q arrives every wave adds D2i[kk][q] X[.., q] to its accumulators of its slabs kk
// (VALU).
// Column blocks run in the solves' internal column order (the order of the FP32 X and of
// R32), so the CB columns of a block are one contiguous row segment of X and of R32 and
// the blocks that share a 128-byte line are neighbours in the launch.  X is read once, in
// two-element row segments (8 or 16 bytes, so that most threads of the workgroup load)
// held PD slabs deep in registers (the bytes in flight that keep a CU streaming), then
// converted into one of two LDS slab buffers; b (and f, in the block
// that holds the load column) is staged in LDS once.  R32 may be null (check only: max
// |R| and max |X| per box); otherwise it is written through LDS in row segments of CB
// floats.
constexpr int kRmLd = 17;                // row stride of a 16x16 slab tile in LDS
constexpr int kRmTile = 16 * kRmLd + 4;  // doubles per tile plane

// A value known to be equal in all lanes, moved to scalar registers.
__device__ inline double wave_uniform(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)bits);
  const int hi = __builtin_amdgcn_readfirstlane((int)(bits >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int M, int NW, int CB, typename TX, bool HASF>
__global__ __launch_bounds__(64 * CB * NW, 4) void residual_mfma_kernel(Geom g, int nbox, int ncb, const double* b,
                                                                       const double* f, const TX* X_all,
                                                                       float* R32_all, const int* pos_all,
                                                                       double* maxr, double* maxx,
                                                                       const int* active, double* fst,
                                                                       const double* fsc) {
  constexpr int m = M, mm = M * M;
  constexpr int kRmThreads = 64 * CB * NW;
  constexpr int H = (M + NW - 1) / NW;        // output slabs per wave
  constexpr int VX = 2;                       // X elements per load (8 or 16 bytes)
  constexpr int XT = CB / VX;                 // loads per row of the column block
  constexpr int NX = mm * XT;                 // loads per slab
  constexpr int NTK = (NX + kRmThreads - 1) / kRmThreads;  // loads per thread and slab
  // slabs in flight: as deep as the registers left by the accumulators allow (no spills)
  constexpr int PD0 = NTK > 1 ? 2 : (sizeof(TX) == 4 ? (M == 15 ? 4 : 8) : (M == 15 ? 2 : 4));
  constexpr int PD = PD0 < M ? PD0 : M;
  constexpr int BUF = CB * kRmTile;           // one slab buffer
  static_assert(CB % VX == 0 && 16 % CB == 0, "a column block is whole load segments of one 16-column group");
  static_assert(4 * mm * CB <= 2 * BUF * 2, "output staging must fit the slab buffers");
  using V = TX __attribute__((ext_vector_type(VX)));
  __shared__ double sm[2 * BUF];
  __shared__ double sb[M * M * M];             // kappa^2 b of the box
  __shared__ double sf[HASF ? M * M * M : 1];  // f of the box (the launch of the load column's block)
  __shared__ double te[2 * 16];                // D2[i+1][0] and D2[i+1][p-1]
  // Two launches: every column block except, when f is given, the one that holds the load
  // column; then that block alone (one workgroup per box, f staged in LDS), so the first
  // launch needs no LDS for f and more of its workgroups fit on a CU.
  int box, cb;
  const int fcb = rhs_icol(g, g.nb) / CB;
  if constexpr (HASF) {
    box = blockIdx.x;
    cb = fcb;
    if (box >= nbox) return;
  } else {
    if (!map_box_chunk(nbox, ncb, box, cb)) return;
    if (f && cb == fcb) return;
  }
  const int p = g.p, ldx = g.ldx;
  // the wave index in a scalar register: everything derived from it (column, run of slabs,
  // the column's face) stays scalar and its branches are scalar branches
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wc = w % CB, part = w / CB;  // column within the block, run of slabs
  const int c0 = cb * CB;                // first internal column of the block
  const int col = rhs_ncol(g, c0 + wc);  // this wave's natural column
  const int lr = lane >> 4, lc = lane & 15;
  // the FP32 X is the solves' buffer (internal column order); an FP64 X has the natural order
  const TX* X = X_all + (size_t)box * g.n_pad * ldx + (sizeof(TX) == 4 ? c0 : rhs_ncol(g, c0));
  const int* pos = pos_all ? pos_all + (size_t)box * g.n_pad : nullptr;
  const double* bb = b + (size_t)box * g.n;
  // (the column-map loads above and this one are in flight together)
  if (active && active[box] == 0) return;
  // Load task t = threadIdx.x + s * threads (t < NX) of a slab: row t / XT, elements
  // VX (t % XT) ..+VX-1 of the block; xo = offset in the slab, lo = LDS slot of its first
  // element (tile [ii][jj] of plane VX (t % XT)).  Loads and LDS stores are branch-free
  // (a load under a branch costs the wait for every load in flight): threads without a
  // task reload row 0 of the slab (a cached line) and store into column 16 of a tile,
  // which no reader touches.
  int xo[NTK], lo[NTK];
#pragma unroll
  for (int s = 0; s < NTK; s++) {
    const int t = threadIdx.x + s * kRmThreads;
    const int r = t / XT, h = t % XT;
    xo[s] = t < NX ? r * ldx + h * VX : 0;
    lo[s] = t < NX ? (h * VX) * kRmTile + (r % m) * kRmLd + r / m : (lane & 15) * kRmLd + 16;
  }
  V pf[PD][NTK];
  auto fetch = [&](int q, int slot) {
    const TX* Xq = X + (size_t)q * mm * ldx;
#pragma unroll
    for (int s = 0; s < NTK; s++) pf[slot][s] = *reinterpret_cast<const V*>(Xq + xo[s]);
  };
  auto stash = [&](int buf, int slot) {
#pragma unroll
    for (int s = 0; s < NTK; s++)
#pragma unroll
      for (int e = 0; e < VX; e++) sm[buf * BUF + lo[s] + e * kRmTile] = (double)pf[slot][s][e];
  };
  // The global loads of b, f and the operator tables are issued together and branch-free
  // (one wait, not one per loop trip), ahead of the slab loads; their values go to LDS
  // after the slab loads are on their way.
  constexpr int NB = (M * M * M + kRmThreads - 1) / kRmThreads;
  static_assert(2 * M <= kRmThreads, "one table entry per thread");
  double rb[NB], rf[HASF ? NB : 1];
#pragma unroll
  for (int k = 0; k < NB; k++) {
    const int e = threadIdx.x + k * kRmThreads, ec = e < m * mm ? e : 0;
    rb[k] = bb[ec];
    if constexpr (HASF) rf[k] = f[(size_t)box * g.n + ec];
  }
  const double finv = (HASF && fsc) ? 1.0 / fsc[box] : 1.0;  // (a power of two: exact)
  const int e0 = threadIdx.x;
  const double re = g.D2[e0 < 2 * m ? (e0 % m + 1) * p + (e0 < m ? 0 : p - 1) : 0];
  // MFMA operand of both derivative terms, kept in registers: lane (lr, lc) holds, for k
  // chunk kb, s2x D2[lc+1][lr+4kb+1] (zero outside m x m).  It is the A operand of the
  // x term D2i S and, with the ratio s2y / s2x moved onto S, the B operand of the y term
  // S D2i^T.
  double dreg[4];
#pragma unroll
  for (int kb = 0; kb < 4; kb++) {
    const bool in = lc < m && lr + 4 * kb < m;
    const double v = g.D2[in ? (lc + 1) * p + lr + 4 * kb + 1 : 0];
    dreg[kb] = in ? g.s2[0] * v : 0.0;
  }
  // (the slab loads stay behind these in issue order, so the wait for the values above
  // does not also wait for the slabs)
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < PD; q++) fetch(q, q);
  for (int e = threadIdx.x; e < 2 * BUF; e += kRmThreads) sm[e] = 0.0;
#pragma unroll
  for (int k = 0; k < NB; k++) {
    const int e = threadIdx.x + k * kRmThreads;
    if (e < m * mm) {
      sb[e] = g.kappa2 * rb[k];
      if constexpr (HASF) sf[e] = rf[k] * finv;
    }
  }
  if (e0 < 2 * m) te[e0] = re;
  // This wave's column of [A_ib | f].  A_ib column col is nonzero on the normal line of
  // face node (la, lb); bit i of emask marks this lane's node (lr + 4i, lc) on it, whose
  // entry is -s2[axis] D2[t+1][edge] with t the node's coordinate along the axis.
  int axis = -1, side = 0, la = 0, lb = 0;
  if (col < g.nb) {
    const int a = col / mm, qq = col - a * mm;
    axis = a >> 1;
    side = a & 1;
    la = qq % m;
    lb = qq / m;
  }
  const bool fcol = HASF && col == g.nb;
  int emask = 0, inb = 0;  // inb: bit i marks node (lr + 4i, lc) inside the m x m slab
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int ii = lr + 4 * i;
    bool on = false;
    if (ii < m && lc < m) {
      inb |= 1 << i;
      if (axis == 0) on = lc == la;
      else if (axis == 1) on = ii == la;
      else if (axis == 2) on = ii == la && lc == lb;
    }
    emask |= on ? (1 << i) : 0;
  }
  // (selects, not g.s2[axis]: a per-lane index into the argument block is a vector load,
  // whose wait would also wait for the slab loads above)
  const double s2a = axis == 0 ? -g.s2[0] : (axis == 1 ? -g.s2[1] : (axis == 2 ? -g.s2[2] : 0.0));
  const double ry = g.s2[1] / g.s2[0];
  __syncthreads();  // zero fill and tables done
  stash(0, 0);
  d4 acc[H];
#pragma unroll
  for (int k = 0; k < H; k++) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
  double mxv = 0.0;
#pragma unroll
  for (int q = 0; q < m; q++) {
    __builtin_amdgcn_sched_barrier(0);  // keep each slab's work (and its registers) in place
    __syncthreads();                    // slab q visible; the other buffer is free
    if (q + PD < m) fetch(q + PD, q % PD);
    const double* S = sm + (q & 1) * BUF;
    const double* Sc = S + wc * kRmTile;
    double bx[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) bx[kb] = Sc[(lr + 4 * kb) * kRmLd + lc];
#pragma unroll
    for (int pt = 0; pt < NW; pt++) {
      if (part != pt) continue;  // wave-uniform: one static copy per run of slabs
      if (q >= pt * H && q < (pt + 1) * H) {
        // x- and y-derivative terms of slab q, the diagonal term and the load column
        double ay[4];
#pragma unroll
        for (int kb = 0; kb < 4; kb++) ay[kb] = ry * Sc[lc * kRmLd + lr + 4 * kb];
        d4 a = acc[q - pt * H];
#pragma unroll
        for (int kb = 0; kb < 4; kb++) a = __builtin_amdgcn_mfma_f64_16x16x4f64(dreg[kb], bx[kb], a, 0, 0, 0);
#pragma unroll
        for (int kb = 0; kb < 4; kb++) a = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[kb], dreg[kb], a, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          // (lanes outside the m x m slab hold X = 0: any node of the box serves there)
          const int node = q * mm + ((inb >> i) & 1 ? lr + 4 * i + m * lc : 0);
          a[i] += sb[node] * bx[i];
        }
        if constexpr (HASF) {
          if (fcol) {
#pragma unroll
            for (int i = 0; i < 4; i++)
              if ((inb >> i) & 1) a[i] += sf[q * mm + lr + 4 * i + m * lc];
          }
        }
        acc[q - pt * H] = a;
#pragma unroll
        for (int i = 0; i < 4; i++) mxv = fmax(mxv, fabs(bx[i]));
      }
      // z-derivative: slab q feeds this wave's slabs kk (coefficients s2z D2i[kk][q]
      // through the scalar cache: their address is the same in every lane)
#pragma unroll
      for (int k = 0; k < H; k++) {
        const int kk = pt * H + k;
        if (kk < m) {
          const double cz = g.D2z[(kk + 1) * p + q + 1];
#pragma unroll
          for (int i = 0; i < 4; i++) acc[k][i] += cz * bx[i];
        }
      }
    }
    if (q + 1 < m) stash((q + 1) & 1, (q + 1) % PD);
  }
  // A_ib column: -s2[axis] D2[t+1][edge] on the normal line of face node (la, lb), t the
  // node's coordinate along the axis
#pragma unroll
  for (int pt = 0; pt < NW; pt++) {
    if (part != pt) continue;
#pragma unroll
    for (int k = 0; k < H; k++) {
      const int kk = pt * H + k;
      if (kk < m) {
        const bool eslab = axis == 2 || kk == lb;
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const double ev = te[side * m + (axis == 0 ? (lr + 4 * i < m ? lr + 4 * i : 0) : (axis == 1 ? lc % m : kk))];
          acc[k][i] += (eslab && ((emask >> i) & 1)) ? s2a * ev : 0.0;
        }
      }
    }
  }
  // max |R| (entries outside the m x m tile are exactly zero), then R32 through LDS,
  // four slabs at a time
  double mr = 0.0;
#pragma unroll
  for (int k = 0; k < H; k++)
#pragma unroll
    for (int i = 0; i < 4; i++) mr = fmax(mr, fabs(acc[k][i]));
  if (R32_all) {
    float* O = reinterpret_cast<float*>(sm);  // [4 slabs][m^2 rows][CB]
    float* R32 = R32_all + (size_t)box * g.n_pad * ldx + c0;
#pragma unroll
    for (int k0 = 0; k0 < m; k0 += 4) {
      __syncthreads();  // LDS free (slab reads or the previous group's stores done)
#pragma unroll
      for (int pt = 0; pt < NW; pt++) {
        if (part != pt) continue;
#pragma unroll
        for (int k = 0; k < H; k++) {
          const int kk = pt * H + k;
          if (kk >= k0 && kk < k0 + 4 && kk < m) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
              const int ii = lr + 4 * i;
              if (ii < m && lc < m) O[((kk - k0) * mm + ii + m * lc) * CB + wc] = (float)acc[k][i];
            }
          }
        }
      }
      __syncthreads();
      // row segments of OV floats; the R32 rows (pos) come from L2, issued together
      constexpr int OV = CB < 4 ? CB : 4;
      constexpr int VO = CB / OV;
      constexpr int NR = (4 * mm * VO + kRmThreads - 1) / kRmThreads;
      using FO = float __attribute__((ext_vector_type(OV)));
      const int nk = (m - k0) < 4 ? (m - k0) : 4;
      int prow[NR];
#pragma unroll
      for (int j = 0; j < NR; j++) {
        const int t = threadIdx.x + j * kRmThreads, row = t / VO;
        const int node = k0 * mm + (t < nk * mm * VO ? row : 0);
        prow[j] = pos ? pos[node] : node;
      }
#pragma unroll
      for (int j = 0; j < NR; j++) {
        const int t = threadIdx.x + j * kRmThreads;
        if (t < nk * mm * VO) {
          const int row = t / VO, h = t % VO;  // row = (slab - k0) * m^2 + r
          const FO v = *reinterpret_cast<const FO*>(O + row * CB + OV * h);
          *reinterpret_cast<FO*>(R32 + (size_t)prow[j] * ldx + OV * h) = v;
        }
      }
    }
  }
  mr = wave_max(mr);
  mxv = wave_max(mxv);
  if (lane == 0) {
    atomic_max_nonneg(maxr + box, mr);
    atomic_max_nonneg(maxx + box, mxv);
    if constexpr (HASF) {
      if (fcol && fst) {  // the load column alone (this wave's column)
        atomic_max_nonneg(fst + nbox + box, mr);
        atomic_max_nonneg(fst + 2 * nbox + box, mxv);
      }
    }
  }
}

// Kernel attributes are set once per plan (outside any stream capture).
hipError_t residual_prepare(const Geom& g) {
  const size_t shm4 = ((size_t)g.n * 4 + g.m * g.m + 2 * g.m) * sizeof(double);
  const size_t shm2 = ((size_t)g.n * 2 + g.m * g.m + 2 * g.m) * sizeof(double);
  const int s4 = (int)(shm4 < 160 * 1024 ? shm4 : 160 * 1024), s2 = (int)(shm2 < 160 * 1024 ? shm2 : 160 * 1024);
  const void* k[4] = {reinterpret_cast<const void*>(&residual_kernel<4, double>),
                      reinterpret_cast<const void*>(&residual_kernel<2, double>),
                      reinterpret_cast<const void*>(&residual_kernel<4, float>),
                      reinterpret_cast<const void*>(&residual_kernel<2, float>)};
  hipError_t e = hipSuccess;
  for (int i = 0; i < 4 && e == hipSuccess; i++)
    e = hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, (i % 2) ? s2 : s4);
  return e;
}

template <int NW, int CB, typename TX>
static hipError_t launch_residual_mfma(const Geom& g, int nbox, int grid_boxes, const double* b, const double* f,
                                       const TX* X, float* R32, const int* pos, double* maxr, double* maxx,
                                       const int* active, hipStream_t st, double* fst, const double* fsc) {
  // column blocks run over the internal order's 16-column groups that hold natural columns
  // 0..nb (they come first); later groups hold zeros in X and in R32 (left as the caller
  // wrote them).  With f, the load column's block runs in a second launch.
  const int ncb = 16 * ((g.nb + 1 + 15) / 16) / CB;
  const dim3 grid(grid_boxes * ncb), gridf(grid_boxes), block(64 * CB * NW);
  switch (g.m) {
#define HPS_RES_CASE(M)                                                                                          \
  case M:                                                                                                        \
    hipLaunchKernelGGL((residual_mfma_kernel<M, NW, CB, TX, false>), grid, block, 0, st, g, nbox, ncb, b, f, X,  \
                       R32, pos, maxr, maxx, active, fst, fsc);                                                  \
    if (f)                                                                                                       \
      hipLaunchKernelGGL((residual_mfma_kernel<M, NW, CB, TX, true>), gridf, block, 0, st, g, nbox, ncb, b, f,   \
                         X, R32, pos, maxr, maxx, active, fst, fsc);                                             \
    break;
    HPS_RES_CASE(4) HPS_RES_CASE(5) HPS_RES_CASE(6) HPS_RES_CASE(7) HPS_RES_CASE(8) HPS_RES_CASE(9)
    HPS_RES_CASE(10) HPS_RES_CASE(11) HPS_RES_CASE(12) HPS_RES_CASE(13) HPS_RES_CASE(14) HPS_RES_CASE(15)
    HPS_RES_CASE(16)
#undef HPS_RES_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TX>
hipError_t launch_residual(const Geom& g, int nbox, const double* b, const double* f, const TX* X, float* R32,
                           const int* pos, double* maxr, double* maxx, const int* active, hipStream_t st, int cols,
                           double* fst, const double* fsc) {
  if (!f) fst = nullptr;
  hipError_t e = launch_fill_zero(maxr, sizeof(double) * nbox, st);
  if (e == hipSuccess) e = launch_fill_zero(maxx, sizeof(double) * nbox, st);
  if (e == hipSuccess && fst) e = launch_fill_zero(fst + nbox, 2 * sizeof(double) * nbox, st);
  if (e != hipSuccess) return e;
  const int grid_boxes = 8 * ((nbox + 7) / 8);
  if (g.m >= 4 && g.m <= 16) {
    // two waves per column; 8 columns (1024 threads), 4 (512) or 2 (256) per workgroup
    if (cols == 2) return launch_residual_mfma<2, 2>(g, nbox, grid_boxes, b, f, X, R32, pos, maxr, maxx, active, st,
                                                      fst, fsc);
    if (cols == 4) return launch_residual_mfma<2, 4>(g, nbox, grid_boxes, b, f, X, R32, pos, maxr, maxx, active, st,
                                                      fst, fsc);
    return launch_residual_mfma<2, 8>(g, nbox, grid_boxes, b, f, X, R32, pos, maxr, maxx, active, st,
                                                      fst, fsc);
  } else if (((size_t)g.n * 4 + g.m * g.m + 2 * g.m) * sizeof(double) <= 96 * 1024) {
    const size_t shm = ((size_t)g.n * 4 + g.m * g.m + 2 * g.m) * sizeof(double);
    hipLaunchKernelGGL((residual_kernel<4, TX>), dim3(grid_boxes * (g.ldx / 4)), dim3(kResThreads), shm, st, g, nbox,
                       b, f, X, R32, pos, maxr, maxx, active, fst, fsc);
  } else {
    const size_t shm = ((size_t)g.n * 2 + g.m * g.m + 2 * g.m) * sizeof(double);
    hipLaunchKernelGGL((residual_kernel<2, TX>), dim3(grid_boxes * (g.ldx / 2)), dim3(kResThreads), shm, st, g, nbox,
                       b, f, X, R32, pos, maxr, maxx, active, fst, fsc);
  }
  return hipGetLastError();
}
template hipError_t launch_residual<double>(const Geom&, int, const double*, const double*, const double*, float*,
                                            const int*, double*, double*, const int*, hipStream_t, int, double*,
                                            const double*);
template hipError_t launch_residual<float>(const Geom&, int, const double*, const double*, const float*, float*,
                                           const int*, double*, double*, const int*, hipStream_t, int, double*,
                                           const double*);

// Backward error check of one refinement step; decides which boxes continue.
__global__ void ir_check_kernel(int nbox, int it, int last, double tol, const double* anorm, const double* maxb,
                                const double* maxr, const double* maxx, int* active, int* iters, double* berr,
                                const double* fst) {
  const int box = blockIdx.x * blockDim.x + threadIdx.x;
  if (box >= nbox || active[box] == 0) return;
  double be = maxr[box] / (anorm[box] * maxx[box] + maxb[box]);
  if (fst) {  // the load column on its own scale (its entries are far smaller than A_ib's)
    const double num = fst[nbox + box], den = anorm[box] * fst[2 * nbox + box] + fst[box];
    // a zero load with a zero solution has nothing to refine (0 / 0 counts as 0)
    const double bf = num != num ? num : (den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0));
    be = (bf > be || bf != bf) ? bf : be;  // (a NaN stays a NaN)
  }
  if (berr) berr[box] = be;
  if (be <= tol) {
    active[box] = 0;
    if (iters) iters[box] = it;
  } else if (last) {
    active[box] = 0;
    if (iters) iters[box] = -1 - it;  // still above tol after `it` corrections
  }
}

hipError_t launch_ir_check(int nbox, int it, int last, double tol, const double* anorm, const double* maxb,
                           const double* maxr, const double* maxx, int* active, int* iters, double* berr,
                           hipStream_t st, const double* fst) {
  hipLaunchKernelGGL(ir_check_kernel, dim3((nbox + 255) / 256), dim3(256), 0, st, nbox, it, last, tol, anorm, maxb,
                     maxr, maxx, active, iters, berr, fst);
  return hipGetLastError();
}


// ----------------------------------------------------------------------------
// a4: DtN rows and loads (Sec. 3.1 eq. t-block, Alg. 1; Alg. 2 load loop).
// Face row (face a of axis d, tangential q) is the outward normal derivative along the
// line through its node:
//   face d- row: -(2/h_d) sum_l D[0][l] u_l,    face d+ row: +(2/h_d) sum_l D[p-1][l] u_l
// so  T = A_bb - A_bi X_b  and  g = -A_bi X_f - sum_{Dirichlet faces b} T[:, b] g_dir[b].
// One workgroup per (box, block of kDtnCols columns of X) streams X one z-plane at a
// time through LDS, so every element of X is read from HBM once: the x- and y-lines of
// a plane are summed from LDS, the z-lines accumulate in registers over the planes.
// The Dirichlet and load columns of a face row are summed per column block into
// `part` [nbox][ncb][n_b]; dtn_lift_kernel adds the blocks in a fixed order.
// ----------------------------------------------------------------------------
constexpr int kDtnCols = 16;
constexpr int kDtnLd = kDtnCols + 1;       // LDS row stride (doubles)

struct DtnCtx {
  Geom g;
  double* T_vals;
  int c, box_nb;    // this lane's column (c < nb + 1 valid), n_b
  bool valid;
  // fixed per lane, loaded once (no dependent loads behind the line sums): the column's
  // face is a Dirichlet face (its entries move to the load, times gd); slot[a] = the
  // block (face a, the column's face) where T is stored, -1 where it is not; qc = the
  // column's node on its face; dend[side][e] = D[side ? p-1 : 0][e ? p-1 : 0]
  bool dir_col;
  double gd;
  int slot[6], qc;
  double dend[2][2];
};

__device__ inline void dtn_ctx_init(DtnCtx& k, const Geom& g, const double* gdir, const int* smap, double* T_vals,
                                    int c, int mm) {
  const int nb = g.nb, p = g.p;
  k.g = g;
  k.T_vals = T_vals;
  k.c = c;
  k.box_nb = nb;
  k.valid = c <= nb;
  const int cc = c < nb ? c : 0, b = cc / mm;  // (other lanes read column 0's entries, unused)
  k.qc = cc - b * mm;
  k.dir_col = smap[b * 6 + b] < 0;
  k.gd = gdir ? gdir[cc] : 0.0;
#pragma unroll
  for (int a = 0; a < 6; a++) {
    const int sa = smap[a * 6 + a], sl = smap[a * 6 + b];
    k.slot[a] = sa >= 0 ? sl : -1;
  }
  k.dend[0][0] = g.D[0];
  k.dend[0][1] = g.D[p - 1];
  k.dend[1][0] = g.D[(size_t)(p - 1) * p];
  k.dend[1][1] = g.D[(size_t)(p - 1) * p + p - 1];
}

// Value of face row (face a, tangential q) at this lane's column from the line sum
// xs_ = sum_l D[end][l+1] X[line node l][c]; returns the lane's contribution to the
// row's lift (load column or Dirichlet column), and writes T where it is stored.
__device__ inline double dtn_entry(const DtnCtx& k, int a, int q, double xs_, int mm) {
  if (!k.valid) return 0.0;
  const Geom& g = k.g;
  const int axis = a >> 1, side = a & 1;
  const double s1 = g.s1[axis];
  const int row_m = 2 * axis * mm + q, row_p = row_m + mm;
  if (k.c == k.box_nb) return side ? -s1 * xs_ : s1 * xs_;  // g = -A_bi v
  double t = side ? -s1 * xs_ : s1 * xs_;                   // -A_bi X_b
  const double sg = side ? s1 : -s1;                        // A_bb: outward derivative ends
  if (k.c == row_m) t += sg * k.dend[side][0];
  if (k.c == row_p) t += sg * k.dend[side][1];
  if (k.dir_col) return -t * k.gd;  // Dirichlet column: moves to the load
  const int sl = k.slot[a];
  if (sl >= 0) k.T_vals[(size_t)sl * mm * mm + (size_t)q * mm + k.qc] = t;
  return 0.0;
}

// Sum over the 16 lanes of a column group (lanes 16j .. 16j+15 of a wave).
__device__ inline double group16_sum(double v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <int M>
__global__ __launch_bounds__(256) void dtn_kernel(Geom g, int nbox, int ncb, const double* X_all, const double* gdir,
                                                  const int* slot_map, double* T_vals, double* part) {
  constexpr int mm = M * M;
  constexpr int ZL = (mm + 15) / 16;  // plane rows (and z-lines) per thread
  __shared__ double xs[mm * kDtnLd];
  __shared__ double dd[2][M];  // D[0][l+1] and D[p-1][l+1]: outward derivative weights
  const int box = blockIdx.y, cb = blockIdx.x;
  const int p = g.p, nb = g.nb, ldx = g.ldx;
  const int cl = threadIdx.x & 15, sub = threadIdx.x >> 4;  // column lane, row group
  DtnCtx k;
  dtn_ctx_init(k, g, gdir ? gdir + (size_t)box * nb : nullptr, slot_map + box * 36, T_vals, cb * kDtnCols + cl, mm);
  // column c < ldx for every lane (ncb * 16 <= ldx), so loads need no guard; rows past
  // the plane reread its last row
  const double* X = X_all + (size_t)box * g.n_pad * ldx + cb * kDtnCols + cl;
  double* pb = part + ((size_t)box * ncb + cb) * nb;
  const double* D0 = g.D;
  const double* D1 = g.D + (size_t)(p - 1) * p;
  for (int e = threadIdx.x; e < 2 * M; e += blockDim.x) dd[e / M][e % M] = (e < M ? D0 : D1)[e % M + 1];
  double zm[ZL], zp[ZL], pre[ZL];
#pragma unroll
  for (int u = 0; u < ZL; u++) {
    zm[u] = zp[u] = 0.0;
    const int t = min(sub + 16 * u, mm - 1);
    pre[u] = X[(size_t)t * ldx];
  }
  for (int kk = 0; kk < M; kk++) {
    __syncthreads();  // the previous plane is consumed
#pragma unroll
    for (int u = 0; u < ZL; u++) {
      const int t = sub + 16 * u;
      if (t < mm) xs[t * kDtnLd + cl] = k.valid ? pre[u] : 0.0;
    }
    __syncthreads();
    if (kk + 1 < M) {  // the next plane is in flight while this one is used
#pragma unroll
      for (int u = 0; u < ZL; u++) {
        const int t = min(sub + 16 * u, mm - 1);
        pre[u] = X[(size_t)((kk + 1) * mm + t) * ldx];
      }
    }
    // z-lines (ii, jj) = plane row zl: this thread owns zl = sub + 16 u
    const double d0 = dd[0][kk], d1 = dd[1][kk];
#pragma unroll
    for (int u = 0; u < ZL; u++) {
      const int zl = sub + 16 * u;
      if (zl < mm) {
        const double x = xs[zl * kDtnLd + cl];
        zm[u] += d0 * x;
        zp[u] += d1 * x;
      }
    }
    // x-lines (jj fixed, ii runs) and y-lines (ii fixed, jj runs) of this plane
    for (int j = sub; j < M; j += 16) {
      double xm = 0.0, xp = 0.0, ym = 0.0, yp = 0.0;
#pragma unroll 2
      for (int l = 0; l < M; l++) {
        const double a0 = dd[0][l], a1 = dd[1][l];
        const double vx = xs[(l + M * j) * kDtnLd + cl];  // node (ii = l, jj = j)
        const double vy = xs[(j + M * l) * kDtnLd + cl];  // node (ii = j, jj = l)
        xm += a0 * vx;
        xp += a1 * vx;
        ym += a0 * vy;
        yp += a1 * vy;
      }
      const int q = j + M * kk;
      const double lxm = group16_sum(dtn_entry(k, 0, q, xm, mm));
      const double lxp = group16_sum(dtn_entry(k, 1, q, xp, mm));
      const double lym = group16_sum(dtn_entry(k, 2, q, ym, mm));
      const double lyp = group16_sum(dtn_entry(k, 3, q, yp, mm));
      if (cl == 0) {
        pb[0 * mm + q] = lxm;
        pb[1 * mm + q] = lxp;
        pb[2 * mm + q] = lym;
        pb[3 * mm + q] = lyp;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < ZL; u++) {
    const int zl = sub + 16 * u;
    if (zl < mm) {
      const double lzm = group16_sum(dtn_entry(k, 4, zl, zm[u], mm));
      const double lzp = group16_sum(dtn_entry(k, 5, zl, zp[u], mm));
      if (cl == 0) {
        pb[4 * mm + zl] = lzm;
        pb[5 * mm + zl] = lzp;
      }
    }
  }
}

// gload[box][row] = sum over column blocks of part (fixed order); 0 on Dirichlet faces.
__global__ void dtn_lift_kernel(int nb, int mm, int nbox, int ncb, const int* slot_map, const double* part,
                                double* gload) {
  const int box = blockIdx.y;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nb) return;
  const int a = row / mm;
  double s = 0.0;
  if (slot_map[box * 36 + a * 6 + a] >= 0) {
    const double* pb = part + (size_t)box * ncb * nb + row;
    for (int cb = 0; cb < ncb; cb++) s += pb[(size_t)cb * nb];
  }
  gload[(size_t)box * nb + row] = s;
}

hipError_t launch_dtn(const Geom& g, int nbox, const double* X, const double* gdir, const int* slot_map,
                      double* T_vals, double* gload, double* part, hipStream_t st) {
  const int ncb = (g.nb + 1 + kDtnCols - 1) / kDtnCols;
  const dim3 grid(ncb, nbox);
  switch (g.m) {
#define HPS_DTN_CASE(M)                                                                                      case M:                                                                                                      hipLaunchKernelGGL(dtn_kernel<M>, grid, dim3(256), 0, st, g, nbox, ncb, X, gdir, slot_map, T_vals, part);     break;
    HPS_DTN_CASE(2) HPS_DTN_CASE(3) HPS_DTN_CASE(4) HPS_DTN_CASE(5) HPS_DTN_CASE(6) HPS_DTN_CASE(7)
    HPS_DTN_CASE(8) HPS_DTN_CASE(9) HPS_DTN_CASE(10) HPS_DTN_CASE(11) HPS_DTN_CASE(12) HPS_DTN_CASE(13)
    HPS_DTN_CASE(14) HPS_DTN_CASE(15) HPS_DTN_CASE(16) HPS_DTN_CASE(17) HPS_DTN_CASE(18)
#undef HPS_DTN_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dtn_lift_kernel, dim3((g.nb + 255) / 256, nbox), dim3(256), 0, st, g.nb, g.m * g.m, nbox, ncb,
                     slot_map, part, gload);
  return hipGetLastError();
}

// bytes of `part` for nbox boxes
size_t dtn_part_bytes(const Geom& g, int nbox) {
  const size_t ncb = (g.nb + 1 + kDtnCols - 1) / kDtnCols;
  return 8 * ncb * g.nb * (size_t)nbox;
}

// T_vals[dst] = T_vals[lo] + T_vals[hi] for each (dst, lo, hi) triple: the shared
// diagonal block of an internal face is the sum of its two boxes' contributions, each
// kept in a slot of its own, so that running the reduction again gives the same bits.
__global__ void reduce_kernel(int ntrip, const long long* trip, long long block_elems, double* T) {
  const int pr = blockIdx.y;
  if (pr >= ntrip) return;
  const long long dst = trip[3 * pr], lo = trip[3 * pr + 1], hi = trip[3 * pr + 2];
  double* d = T + dst * block_elems;
  const double* a = T + lo * block_elems;
  const double* b = T + hi * block_elems;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < block_elems;
       i += (long long)gridDim.x * blockDim.x)
    d[i] = a[i] + b[i];
}

hipError_t launch_reduce(int ntrip, const long long* trip, long long block_elems, double* T_vals, hipStream_t st) {
  if (ntrip == 0) return hipSuccess;
  int gx = (int)((block_elems + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(reduce_kernel, dim3(gx, ntrip), dim3(256), 0, st, ntrip, trip, block_elems, T_vals);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// a5: u_i = X_f - X_b u_b (one wave per interior node)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reconstruct_kernel(Geom g, int nbox, const double* X_all, const double* ub,
                                                          double* ui) {
  const int box = blockIdx.y;
  const int node = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (node >= g.n) return;
  const double* x = X_all + ((size_t)box * g.n_pad + node) * g.ldx;
  const double* u = ub + (size_t)box * g.nb;
  double s = 0.0;
  for (int c = lane; c < g.nb; c += 64) s += x[c] * u[c];
  s = wave_sum(s);
  if (lane == 0) ui[(size_t)box * g.n + node] = x[g.nb] - s;
}

hipError_t launch_reconstruct(const Geom& g, int nbox, const double* X, const double* ub, double* ui,
                              hipStream_t st) {
  hipLaunchKernelGGL(reconstruct_kernel, dim3((g.n + 3) / 4, nbox), dim3(256), 0, st, g, nbox, X, ub, ui);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// a6 helpers.  rhs = w - A_bi^T lam_b: node (ii,jj,kk) lies on one line per axis;
// the face rows at the ends of that line have A_bi entries -/+ (2/h) D[e][c+1].
// ----------------------------------------------------------------------------
__global__ void adjoint_rhs_kernel(Geom g, int nbox, const double* w, const double* lam, double* rhs) {
  const int box = blockIdx.y;
  const int m = g.m, mm = m * m, p = g.p;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < g.n_pad; r += gridDim.x * blockDim.x) {
    double v = 0.0;
    if (r < g.n) {
      v = w[(size_t)box * g.n + r];
      if (lam) {
        const int ii = r % m, jj = (r / m) % m, kk = r / mm;
        const int along[3] = {ii, jj, kk};
        const int tq[3] = {jj + m * kk, ii + m * kk, ii + m * jj};
        const double* lb = lam + (size_t)box * g.nb;
        for (int axis = 0; axis < 3; axis++) {
          const double lm = lb[(2 * axis) * mm + tq[axis]];
          const double lp = lb[(2 * axis + 1) * mm + tq[axis]];
          v -= -g.s1[axis] * g.D[along[axis] + 1] * lm;
          v -= g.s1[axis] * g.D[(size_t)(p - 1) * p + along[axis] + 1] * lp;
        }
      }
    }
    rhs[(size_t)box * g.n_pad + r] = v;
  }
}

hipError_t launch_adjoint_rhs(const Geom& g, int nbox, const double* w, const double* lam_b, double* rhs,
                              hipStream_t st) {
  hipLaunchKernelGGL(adjoint_rhs_kernel, dim3((g.n_pad + 255) / 256, nbox), dim3(256), 0, st, g, nbox, w, lam_b, rhs);
  return hipGetLastError();
}

// z = A_ii^{-T} rhs with P A = L U:  A^T = U^T L^T P, so solve U^T y = rhs
// (forward), L^T v = y (backward), z[perm[i]] = v[i].  One workgroup per box;
// the vector lives in LDS, the factor rows are read coalesced (row-major).
__global__ __launch_bounds__(kVecThreads) void getrs_t_kernel(Geom g, int nbox, const double* LU_all,
                                                              const int* perm_all, const double* dinv_all,
                                                              const double* rhs_all, double* z_all) {
  extern __shared__ double vec[];
  double* tmp = vec + g.n_pad;
  const int box = blockIdx.x;
  const int N = g.n_pad;
  const double* LU = LU_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  const double* dinv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64;
  for (int i = threadIdx.x; i < N; i += blockDim.x) vec[i] = rhs_all[(size_t)box * N + i];
  __syncthreads();
  auto row = [&](int j) { return LU + (size_t)perm[j] * N; };
  // U^T y = r: block b, y_b = Uinv_b^T (r_b - sum_{k<b} U_kb^T y_k); right-looking updates
  for (int bk = 0; bk < g.npanel; bk++) {
    const int s = bk * kPanel, w = (N - s) < kPanel ? (N - s) : kPanel;
    vec_block_inverse<double>(vec, tmp, dinv + (size_t)(2 * bk + 1) * 64 * 64, s, w, true);
    vec_cols_update<double>(vec, s, w, s + w, N, row);
  }
  // L^T v = y: block b from the last, v_b = Linv_b^T (y_b - sum_{k>b} L_kb^T v_k)
  for (int bk = g.npanel - 1; bk >= 0; bk--) {
    const int s = bk * kPanel, w = (N - s) < kPanel ? (N - s) : kPanel;
    vec_block_inverse<double>(vec, tmp, dinv + (size_t)(2 * bk) * 64 * 64, s, w, true);
    vec_cols_update<double>(vec, s, w, 0, s, row);
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) z_all[(size_t)box * N + perm[i]] = vec[i];
}

hipError_t launch_getrs_t(const Geom& g, int nbox, const double* LU, const int* perm, const double* dinv,
                          const double* rhs, double* z, hipStream_t st) {
  const size_t shm = sizeof(double) * (g.n_pad + 64);
  hipLaunchKernelGGL(getrs_t_kernel, dim3(nbox), dim3(kVecThreads), shm, st, g, nbox, LU, perm, dinv, rhs, z);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// a5 in solve form: u_i = A_ii^{-1} (f_i - A_ib u_b), refined in FP64.
// ----------------------------------------------------------------------------
// r = f - A_ib u_b - A_ii u for one vector per box: with the face values u_b at the
// two ends of every line, -(A_ii u + A_ib u_b) is s2x, s2y, s2z times D2 applied
// along the full x-, y- and z-lines, plus kappa^2 b u.  One workgroup per box.
__device__ inline double block_max_256(double v, double* red) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return m;
}

// rmax/umax (optional, [nbox]): max|r| and max|u| of the box; a NaN counts as +inf.  With
// f null the load is fscale * u (the Crank-Nicolson right-hand side c u^n - L u^n).
__global__ __launch_bounds__(256) void box_residual_kernel(Geom g, int nbox, const double* b, const double* f,
                                                           double fscale, const double* ub_all, const double* u_all,
                                                           double* r_all, double* rmax, double* umax) {
  extern __shared__ double us[];  // u [n], then D2 [p][p]
  __shared__ double red[4];
  const int box = blockIdx.x;
  const int m = g.m, mm = m * m, n = g.n, p = g.p;
  double* d2 = us + n;
  const double* u = u_all ? u_all + (size_t)box * n : nullptr;
  const double* ub = ub_all + (size_t)box * g.nb;
  double am = 0.0, au = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    us[i] = u ? u[i] : 0.0;
    const double a = fabs(us[i]);
    au = (a == a) ? fmax(au, a) : INFINITY;
  }
  for (int i = threadIdx.x; i < p * p; i += blockDim.x) d2[i] = g.D2[i];
  __syncthreads();
  for (int node = threadIdx.x; node < n; node += blockDim.x) {
    const int cd = g.coords[node];
    const int ii = cd & 255, jj = (cd >> 8) & 255, kk = cd >> 16;
    double lx = d2[(ii + 1) * p] * ub[0 * mm + jj + m * kk] + d2[(ii + 1) * p + p - 1] * ub[1 * mm + jj + m * kk];
    double ly = d2[(jj + 1) * p] * ub[2 * mm + ii + m * kk] + d2[(jj + 1) * p + p - 1] * ub[3 * mm + ii + m * kk];
    double lz = d2[(kk + 1) * p] * ub[4 * mm + ii + m * jj] + d2[(kk + 1) * p + p - 1] * ub[5 * mm + ii + m * jj];
    for (int l = 0; l < m; l++) {
      lx += d2[(ii + 1) * p + l + 1] * us[node - ii + l];
      ly += d2[(jj + 1) * p + l + 1] * us[node + m * (l - jj)];
      lz += d2[(kk + 1) * p + l + 1] * us[node + mm * (l - kk)];
    }
    const double fv = f ? f[(size_t)box * n + node] : (fscale != 0.0 ? fscale * us[node] : 0.0);
    const double r = fv + g.s2[0] * lx + g.s2[1] * ly + g.s2[2] * lz + g.kappa2 * b[(size_t)box * n + node] * us[node];
    r_all[(size_t)box * n + node] = r;
    const double a = fabs(r);
    am = (a == a) ? fmax(am, a) : INFINITY;
  }
  if (rmax) {
    const double v = block_max_256(am, red);
    if (threadIdx.x == 0) rmax[box] = v;
  }
  if (umax) {
    const double v = block_max_256(au, red);
    if (threadIdx.x == 0) umax[box] = v;
  }
}

// berr = max|r| / (|A_ii|_inf max|u| + max|f - A_ib u_b|) per box (NaN -> +inf)
__global__ void interior_berr_kernel(int nbox, const double* anorm, const double* r0max, const double* rmax,
                                     const double* umax, double* berr) {
  const int box = blockIdx.x * blockDim.x + threadIdx.x;
  if (box >= nbox) return;
  const double den = anorm[box] * umax[box] + r0max[box];
  double e = den > 0.0 ? rmax[box] / den : (rmax[box] > 0.0 ? INFINITY : 0.0);
  berr[box] = (e == e) ? e : INFINITY;
}

hipError_t launch_interior_berr(int nbox, const double* anorm, const double* r0max, const double* rmax,
                                const double* umax, double* berr, hipStream_t st) {
  hipLaunchKernelGGL(interior_berr_kernel, dim3((nbox + 255) / 256), dim3(256), 0, st, nbox, anorm, r0max, rmax,
                     umax, berr);
  return hipGetLastError();
}

// x = (P^T L U)^{-1} r for one vector per box with the stored factors: positions hold
// physical rows perm[pos]; each 64-block is solved with its stored diagonal inverse and
// the rows below (forward) or above (backward) are updated, 16 lanes per row.  The
// factors may be FP32; the vector is carried in FP64.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void getrs_vec_kernel(Geom g, int nbox, const T* LU_all,
                                                                const int* perm_all, const T* dinv_all,
                                                                const double* r_all, double* x_all, int accumulate) {
  extern __shared__ double vec[];  // [n_pad], then 64 of scratch
  double* tmp = vec + g.n_pad;
  const int box = blockIdx.x;
  const int N = g.n_pad, n = g.n;
  const T* LU = LU_all + (size_t)box * N * N;
  const int* perm = perm_all + (size_t)box * N;
  const T* dinv = dinv_all + (size_t)box * g.npanel * 2 * 64 * 64;
  const double* r = r_all + (size_t)box * n;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int pr = perm[i];
    vec[i] = pr < n ? r[pr] : 0.0;
  }
  __syncthreads();
  auto row = [&](int j) { return LU + (size_t)perm[j] * N; };
  for (int bk = 0; bk < g.npanel; bk++) {  // L y = P r
    const int s = bk * kPanel, w = (N - s) < kPanel ? (N - s) : kPanel;
    vec_block_inverse<T>(vec, tmp, dinv + (size_t)(2 * bk) * 64 * 64, s, w, false);
    vec_rows_update<T>(vec, s + w, N, s, w, row);
  }
  for (int bk = g.npanel - 1; bk >= 0; bk--) {  // U x = y
    const int s = bk * kPanel, w = (N - s) < kPanel ? (N - s) : kPanel;
    vec_block_inverse<T>(vec, tmp, dinv + (size_t)(2 * bk + 1) * 64 * 64, s, w, false);
    vec_rows_update<T>(vec, 0, s, s, w, row);
  }
  double* x = x_all + (size_t)box * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = accumulate ? x[i] + vec[i] : vec[i];
}

hipError_t launch_box_residual(const Geom& g, int nbox, const double* b, const double* f, const double* ub,
                               const double* u, double* r, double* rmax, double* umax, hipStream_t st,
                               double fscale) {
  const size_t shm = sizeof(double) * ((size_t)g.n + (size_t)g.p * g.p);
  hipLaunchKernelGGL(box_residual_kernel, dim3(nbox), dim3(256), shm, st, g, nbox, b, f, fscale, ub, u, r, rmax,
                     umax);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_getrs_vec(const Geom& g, int nbox, const T* LU, const int* perm, const T* dinv, const double* r,
                            double* x, int accumulate, hipStream_t st) {
  const size_t shm = sizeof(double) * (g.n_pad + 64);
  hipLaunchKernelGGL(getrs_vec_kernel<T>, dim3(nbox), dim3(kVecThreads), shm, st, g, nbox, LU, perm, dinv, r, x,
                     accumulate);
  return hipGetLastError();
}
template hipError_t launch_getrs_vec<float>(const Geom&, int, const float*, const int*, const float*, const double*,
                                            double*, int, hipStream_t);
template hipError_t launch_getrs_vec<double>(const Geom&, int, const double*, const int*, const double*,
                                             const double*, double*, int, hipStream_t);

// Outward normal derivative at the face nodes, A_bi u_i + A_bb u_b: the face rows of
// the interface equations (eq. Aentries).  One thread per line and box; both ends.
__global__ void flux_kernel(Geom g, int nbox, const double* u_all, const double* ub_all, double* flux_all) {
  const int box = blockIdx.y;
  const int m = g.m, mm = m * m, p = g.p;
  const int line = blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= 3 * mm) return;
  const int axis = line / mm, q = line % mm;
  const int t0 = q % m, t1 = q / m;
  int base, stride;
  if (axis == 0) { base = m * t0 + mm * t1; stride = 1; }
  else if (axis == 1) { base = t0 + mm * t1; stride = m; }
  else { base = t0 + m * t1; stride = mm; }
  const double* u = u_all + (size_t)box * g.n;
  const double* ub = ub_all + (size_t)box * g.nb;
  const double* D0 = g.D;                        // D[0][.]
  const double* D1 = g.D + (size_t)(p - 1) * p;  // D[p-1][.]
  const double um = ub[(2 * axis) * mm + q], up = ub[(2 * axis + 1) * mm + q];
  double dm = D0[0] * um + D0[p - 1] * up, dp = D1[0] * um + D1[p - 1] * up;
  for (int l = 0; l < m; l++) {
    const double v = u[base + l * stride];
    dm += D0[l + 1] * v;
    dp += D1[l + 1] * v;
  }
  const double s1 = g.s1[axis];
  double* flux = flux_all + (size_t)box * g.nb;
  flux[(2 * axis) * mm + q] = -s1 * dm;
  flux[(2 * axis + 1) * mm + q] = s1 * dp;
}

hipError_t launch_flux(const Geom& g, int nbox, const double* u, const double* ub, double* flux, hipStream_t st) {
  const int lines = 3 * g.m * g.m;
  hipLaunchKernelGGL(flux_kernel, dim3((lines + 255) / 256, nbox), dim3(256), 0, st, g, nbox, u, ub, flux);
  return hipGetLastError();
}

// y_b = -A_ib^T z: face node (a, q) collects +(2/h_a)^2 D2[c+1][e] z over its line.
__global__ void adjoint_yb_kernel(Geom g, int nbox, const double* z, double* yb) {
  const int box = blockIdx.y;
  const int m = g.m, mm = m * m, p = g.p;
  for (int row = blockIdx.x * blockDim.x + threadIdx.x; row < g.nb; row += gridDim.x * blockDim.x) {
    const int a = row / mm, q = row % mm, axis = a >> 1, side = a & 1;
    const int t0 = q % m, t1 = q / m;
    int base, stride;
    if (axis == 0) { base = m * t0 + mm * t1; stride = 1; }
    else if (axis == 1) { base = t0 + mm * t1; stride = m; }
    else { base = t0 + m * t1; stride = mm; }
    const int e = side ? p - 1 : 0;
    double s = 0.0;
    for (int l = 0; l < m; l++) s += g.D2[(l + 1) * p + e] * z[(size_t)box * g.n_pad + base + l * stride];
    yb[(size_t)box * g.nb + row] = g.s2[axis] * s;
  }
}

hipError_t launch_adjoint_yb(const Geom& g, int nbox, const double* z, double* yb, hipStream_t st) {
  hipLaunchKernelGGL(adjoint_yb_kernel, dim3((g.nb + 255) / 256, nbox), dim3(256), 0, st, g, nbox, z, yb);
  return hipGetLastError();
}

__global__ void compact_kernel(Geom g, int nbox, const double* in, double* out) {
  const int box = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += gridDim.x * blockDim.x)
    out[(size_t)box * g.n + i] = in[(size_t)box * g.n_pad + i];
}

hipError_t launch_compact(const Geom& g, int nbox, const double* in, double* out, hipStream_t st) {
  hipLaunchKernelGGL(compact_kernel, dim3((g.n + 255) / 256, nbox), dim3(256), 0, st, g, nbox, in, out);
  return hipGetLastError();
}

__global__ void grad_kernel(Geom g, int nbox, const double* lam, const double* u, double* grad) {
  const size_t tot = (size_t)nbox * g.n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < tot; i += (size_t)gridDim.x * blockDim.x)
    grad[i] = g.kappa2 * lam[i] * u[i];
}

hipError_t launch_grad(const Geom& g, int nbox, const double* lam, const double* u, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(grad_kernel, dim3(1024), dim3(256), 0, st, g, nbox, lam, u, grad);
  return hipGetLastError();
}

}  // namespace hps
