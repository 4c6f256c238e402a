// Host-side declarations of the kernel launchers (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"

namespace hps {

// Optional per-family kernel timing (see hps_plan_profile_enable).
struct Profiler {
  enum { kLuGemm = 0, kLuPanel, kLuLeaf, kSolveFwd, kSolveBwd, kResidual, kDtn, kOperators, kFamilies };
  struct Rec {
    int fam;
    int n;  // kernel launches between the two events
    double flops, exec;
    hipEvent_t a, b;
  };
  bool on = false;
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  long long launches[kFamilies] = {};
  double ms[kFamilies] = {};
  double flops[kFamilies] = {};
  double exec[kFamilies] = {};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void reset() {
    flush();
    for (int f = 0; f < kFamilies; f++) launches[f] = 0, ms[f] = 0.0, flops[f] = 0.0, exec[f] = 0.0;
  }
  void flush() {
    for (auto& r : pending) {
      float t = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        launches[r.fam] += r.n;
        ms[r.fam] += t;
        flops[r.fam] += r.flops;
        exec[r.fam] += r.exec;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~Profiler() {
    flush();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Brackets `launches` kernel launches of one family with events when profiling is on.
// flops: algorithmic flops of the launches; exec: flops the kernels carry out (less where
// structurally zero blocks are skipped; negative = same as flops).
struct ProfScope {
  Profiler* p;
  hipStream_t st;
  Profiler::Rec r;
  ProfScope(Profiler* prof, int fam, double flops, hipStream_t s, int launches = 1, double exec = -1.0)
      : p(prof && prof->on ? prof : nullptr), st(s) {
    if (!p) return;
    r.fam = fam;
    r.n = launches;
    r.flops = flops;
    r.exec = exec < 0.0 ? flops : exec;
    r.a = p->get();
    r.b = p->get();
    (void)hipEventRecord(r.a, st);
  }
  ~ProfScope() {
    if (!p) return;
    (void)hipEventRecord(r.b, st);
    p->pending.push_back(r);
  }
};

// lu.hip: one kernel launch per schedule record (records of 8 ints, see common.h)
// pivot_end >= 0: rows at positions >= pivot_end are never pivots (partial factorization of
// an interface front; the schedule then stops after the pivot columns and its trailing
// update); -1: every row may be a pivot.  panel_threads: 512, or 1024 where a 1024-thread
// panel kernel exists (FP32, 2049..3072 rows; elsewhere 512 is used).
template <typename T>
hipError_t getrf_run(const Geom& g, const std::vector<int>& ops, T* A, int* perm, T* dinv, int* info, int nbox,
                     hipStream_t st, Profiler* prof, int pivot_end = -1, int panel_threads = 512);
// Rows per block row of the triangular solves of getrs_run: 128 in FP32 (two 64-row LU
// panels per launch), 64 in FP64.
template <typename T>
constexpr int solve_block_rows() { return sizeof(T) == 4 ? 128 : 64; }

// Block q (in sweep order) of the block rows of a triangular sweep over N rows in blocks of
// BR: rows [s, s + w).  With 128-row blocks and N = 64 mod 128 the 64-row block is the first
// one in either direction, where its product with the rows already solved is empty: the
// forward sweep takes rows [0, 64) first and continues at 64 + 128 j (block rows stay made
// of whole 64-row diagonal blocks of the factor), the backward sweep starts at the last 64
// rows.  Otherwise the blocks start at multiples of BR.
__host__ __device__ inline void sweep_block(int N, int BR, bool upper, int q, int& s, int& w) {
  if (BR == 128 && !upper && N % 128 == 64) {
    s = q == 0 ? 0 : 64 + 128 * (q - 1);
    w = q == 0 ? 64 : 128;
    return;
  }
  const int nblk = (N + BR - 1) / BR;
  s = (upper ? nblk - 1 - q : q) * BR;
  w = (N - s) < BR ? (N - s) : BR;
}
// Flops of one solve for the profiler (set by the caller when profiling is on): algorithmic
// n_i^2 (n_b + 1) per active box and sweep, and what the kernels execute per sweep.
struct SolveFlops {
  double alg, fwd_exec, bwd_exec;
};
// xmode 1: X = Y, 2: X += Y, 3: X = Y0 + Y (FP64 X: the refinement's solution and
// corrections), written by the backward block-row launches as they finish each tile.
// bdirect: the rows of B are already in the factor's row order (else gathered via perm);
// B may then be Y itself (the solve runs in place).
template <typename T>
hipError_t getrs_run(const Geom& g, const T* F, const int* perm, const T* dinv, const T* B, T* Y, int nbox,
                     const int* active, hipStream_t st, Profiler* prof, double* X = nullptr, int xmode = 0,
                     int sched = kTrsmRows, int waves = 4, const int* kstart = nullptr, int bdirect = 0,
                     const T* Y0 = nullptr, const SolveFlops* sf = nullptr);

// leafops.hip
hipError_t launch_nodes(const Geom& g, const double* t, const double* h, int nbox, const double* origin, double* xi,
                        double* xb, hipStream_t st);
template <typename T>
hipError_t launch_operators(const Geom& g, int nbox, const double* b, T* A, double* anorm, hipStream_t st);
template <typename T>
// fst (may be null): the load column's own statistics, [3][nbox]: max|f| (written here),
// max|R| and max|X| of that column (written by launch_residual); launch_ir_check then also
// takes the load column's backward error on its own scale
// fsc (may be null): the load column's per-box scale s (launch_fscale); B then carries f / s
hipError_t launch_rhs(const Geom& g, int nbox, const double* f, T* B, double* maxb, hipStream_t st,
                      double* fst = nullptr, const double* fsc = nullptr);
// fsc[box] = the power of two s with 1 <= max|f| / s < 2 (1 for a zero load), and back:
// X[:, nb] *= s for the load column of an X that was solved for f / s
hipError_t launch_fscale(const Geom& g, int nbox, const double* f, double* fsc, hipStream_t st);
hipError_t launch_funscale(const Geom& g, int nbox, double* X, const double* fsc, hipStream_t st);
// kstart [nbox][ldx/64]: first pivoted row at which each 64-column tile of [A_ib | f]
// can be nonzero, rounded down to 64 (for the forward sweep of the first solve)
// and, if pos is given, the inverse permutation pos [nbox][n_pad] (pos[perm[k]] = k)
hipError_t launch_rhs_first_row(const Geom& g, int nbox, const int* perm, int has_f, int* kstart, int* pos,
                                hipStream_t st);
hipError_t residual_prepare(const Geom& g);
// R32 = B - A_ii X (FP64 arithmetic), max|R| and max|X| per box.  X in FP64 (natural
// column order) or FP32 (the solve buffer: internal column order).  R32 columns in the
// internal order, rows at pos[node] when pos is given (the factor's row order), else node
template <typename TX>
hipError_t launch_residual(const Geom& g, int nbox, const double* b, const double* f, const TX* X, float* R32,
                           const int* pos, double* maxr, double* maxx, const int* active, hipStream_t st,
                           int cols = 8, double* fst = nullptr, const double* fsc = nullptr);
// X = (double) Y (natural column order) for the boxes whose active flag is 0
hipError_t launch_x_from_y(const Geom& g, int nbox, const float* Y, double* X, const int* active, hipStream_t st);
hipError_t launch_ir_check(int nbox, int it, int last, double tol, const double* anorm, const double* maxb,
                           const double* maxr, const double* maxx, int* active, int* iters, double* berr,
                           hipStream_t st, const double* fst = nullptr);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_fill_int(int* p, int value, size_t count, hipStream_t st);
// a4: T and the lifted loads; part: scratch of dtn_part_bytes(g, nbox) bytes
hipError_t launch_dtn(const Geom& g, int nbox, const double* X, const double* gdir, const int* slot_map,
                      double* T_vals, double* gload, double* part, hipStream_t st);
size_t dtn_part_bytes(const Geom& g, int nbox);
hipError_t launch_reduce(int ntrip, const long long* trip, long long block_elems, double* T_vals, hipStream_t st);
hipError_t launch_reconstruct(const Geom& g, int nbox, const double* X, const double* ub, double* ui,
                              hipStream_t st);
hipError_t launch_adjoint_rhs(const Geom& g, int nbox, const double* w, const double* lam_b, double* rhs,
                              hipStream_t st);
hipError_t launch_getrs_t(const Geom& g, int nbox, const double* LU, const int* perm, const double* dinv,
                          const double* rhs, double* z, hipStream_t st);
hipError_t launch_adjoint_yb(const Geom& g, int nbox, const double* z, double* yb, hipStream_t st);
hipError_t launch_compact(const Geom& g, int nbox, const double* in, double* out, hipStream_t st);
// r = f - A_ib u_b - A_ii u per box (u null: u = 0); rmax/umax optional per-box max|r|, max|u|
// r = f - A_ii u - A_ib u_b per box (f null: fscale * u instead of f)
hipError_t launch_box_residual(const Geom& g, int nbox, const double* b, const double* f, const double* ub,
                               const double* u, double* r, double* rmax, double* umax, hipStream_t st,
                               double fscale = 0.0);
hipError_t launch_interior_berr(int nbox, const double* anorm, const double* r0max, const double* rmax,
                                const double* umax, double* berr, hipStream_t st);
template <typename T>
hipError_t launch_getrs_vec(const Geom& g, int nbox, const T* LU, const int* perm, const T* dinv, const double* r,
                            double* x, int accumulate, hipStream_t st);
hipError_t launch_flux(const Geom& g, int nbox, const double* u, const double* ub, double* flux, hipStream_t st);
hipError_t launch_grad(const Geom& g, int nbox, const double* lam, const double* u, double* grad, hipStream_t st);

}  // namespace hps
