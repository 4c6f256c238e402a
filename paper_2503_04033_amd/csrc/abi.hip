// extern "C" entry points of libhps_leaf (declared in include/hps_leaf.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hps_leaf.h"
#include "common.h"
#include "kernels.h"

struct hps_plan_s {
  hps_leaf_desc desc;
  hps::Geom g;
  int device;
  double* tables;  // device: t[p], D[p*p], D2[p*p], s2z D2[p*p]
  int* coords;     // device: interior node coordinates (packed)
  std::vector<int> lu_ops;  // LU schedule (records of 8 ints)
  std::vector<int> gmap_h;  // host copy of g.gmap (internal -> natural 16-column group)
  hps::Profiler prof;                          // optional kernel timing
  const double* t;
  int trsm_sched = hps::kTrsmRows;             // HPS_TUNE_TRSM_SCHEDULE
  int trsm_waves = 4;                          // HPS_TUNE_TRSM_WAVES
  int res_cols = 4;                            // HPS_TUNE_RESIDUAL_COLS
  int panel_threads = 1024;                    // HPS_TUNE_PANEL_THREADS
  void* scratch = nullptr;                     // this device's address of `scratch` (below)
};

namespace {

using hps::Geom;

hps_status dev(hipError_t e) { return e == hipSuccess ? HPS_OK : HPS_EDEVICE; }

#define HPS_TRY(expr)                               \
  do {                                              \
    hipError_t e__ = (expr);                        \
    if (e__ != hipSuccess) return HPS_EDEVICE;      \
  } while (0)

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


// Gauss-Lobatto points t_j = -cos(pi j/(p-1)) and the barycentric
// differentiation matrix on them (weights (-1)^j, halved at the end points),
// with the diagonal chosen so that every row sums to zero (Sec. 2.1).
void cheb_tables(int p, std::vector<double>& t, std::vector<double>& D, std::vector<double>& D2) {
  const double pi = 3.14159265358979323846;
  t.assign(p, 0.0);
  for (int j = 0; j < p; j++) t[j] = -std::cos(pi * j / (p - 1));
  std::vector<double> w(p);
  for (int j = 0; j < p; j++) w[j] = ((j % 2) ? -1.0 : 1.0) * ((j == 0 || j == p - 1) ? 0.5 : 1.0);
  D.assign((size_t)p * p, 0.0);
  for (int i = 0; i < p; i++) {
    double rowsum = 0.0;
    for (int j = 0; j < p; j++) {
      if (i == j) continue;
      const double v = (w[j] / w[i]) / (t[i] - t[j]);
      D[(size_t)i * p + j] = v;
      rowsum += v;
    }
    D[(size_t)i * p + i] = -rowsum;
  }
  D2.assign((size_t)p * p, 0.0);
  for (int i = 0; i < p; i++)
    for (int k = 0; k < p; k++) {
      const double a = D[(size_t)i * p + k];
      for (int j = 0; j < p; j++) D2[(size_t)i * p + j] += a * D[(size_t)k * p + j];
    }
}

// Recursive column-split LU unrolled into records (see lu.hip):
//   lu(c0, c1): panel if c1 - c0 <= 64, else lu(c0, mid); trsm(c0, mid | mid, c1);
//               gemm(rows [mid, N), cols [mid, c1), k [c0, mid)); lu(mid, c1)
//   trsm(r0, r1 | cA, cB): block rows if r1 - r0 <= 256, else trsm(r0, mid); gemm(rows
//               [mid, r1), cols [cA, cB), k [r0, mid)); trsm(mid, r1)
// Split points are multiples of 64 so that leaves coincide with 64-wide panels.
void sched_trsm(std::vector<int>& ops, int r0, int r1, int cA, int cB) {
  if (r1 - r0 <= hps::kLuRowsMax) {  // short: 64-row blocks, each a K loop plus the leaf product
    ops.insert(ops.end(), {hps::kOpRows, r0, r1, cA, cB, 0, 0, 0});
    return;
  }
  const int mid = r0 + (int)round_up((r1 - r0) / 2, 64);
  sched_trsm(ops, r0, mid, cA, cB);
  ops.insert(ops.end(), {hps::kOpGemm, mid, r1, cA, cB, r0, mid, 0});
  sched_trsm(ops, mid, r1, cA, cB);
}

void sched_lu(std::vector<int>& ops, int c0, int c1, int N) {
  if (c1 - c0 <= 64) {
    ops.insert(ops.end(), {hps::kOpPanel, c0, c1 - c0, 0, 0, 0, 0, 0});
    return;
  }
  const int mid = c0 + (int)round_up((c1 - c0) / 2, 64);
  sched_lu(ops, c0, mid, N);
  sched_trsm(ops, c0, mid, mid, c1);
  ops.insert(ops.end(), {hps::kOpGemm, mid, N, mid, c1, c0, mid, 0});
  sched_lu(ops, mid, c1, N);
}

struct Sizes {
  size_t a, perm, dinv, x, ws;
};

Sizes sizes_of(const hps_plan_s* pl) {
  const Geom& g = pl->g;
  const size_t es = pl->desc.precision == HPS_FP32_IR ? 4 : 8;
  Sizes s;
  s.a = es * g.n_pad * (size_t)g.n_pad;
  s.perm = 4 * (size_t)g.n_pad;
  s.dinv = es * (size_t)g.npanel * 2 * 64 * 64;
  s.x = 8 * (size_t)g.n_pad * g.ldx;
  const size_t elems = (size_t)g.n_pad * g.ldx;
  // FP32_IR: B32 (right-hand side, later the FP32 residual) and Y32; FP64: B64.
  // Plus per-box scalars, the first nonzero row of each right-hand-side tile and the
  // inverse row permutation.
  s.ws = 8 * elems + 64 + 4 * round_up(g.ldx / 64, 16) + 4 * (size_t)g.n_pad;
  return s;
}

struct WsLayout {
  void* B;      // B32 or B64
  float* Y32;
  double *maxb, *maxr, *maxx;
  int* active;
  double* fst;  // [3][nbox]: the load column's max|f|, max|R|, max|X|
  double* fsc;  // [nbox]: the load column's scale in the FP32 solves
  int* kstart;  // [nbox][ldx/64]
  int* pos;     // [nbox][n_pad]: inverse of perm
};

WsLayout ws_layout(const hps_plan_s* pl, int nbox, void* ws) {
  const Geom& g = pl->g;
  const size_t elems = (size_t)g.n_pad * g.ldx * nbox;
  char* p = static_cast<char*>(ws);
  WsLayout L;
  L.B = p;
  L.Y32 = pl->desc.precision == HPS_FP32_IR ? reinterpret_cast<float*>(p + 4 * elems) : nullptr;
  p += 8 * elems;
  L.maxb = reinterpret_cast<double*>(p);
  L.maxr = L.maxb + nbox;
  L.maxx = L.maxr + nbox;
  L.active = reinterpret_cast<int*>(L.maxx + nbox);
  L.fst = reinterpret_cast<double*>(p + 32 * (size_t)nbox);  // after active
  L.fsc = L.fst + 3 * (size_t)nbox;                            // bytes 56..64 per box
  L.kstart = reinterpret_cast<int*>(p + 64 * (size_t)nbox);
  L.pos = L.kstart + round_up(g.ldx / 64, 16) * (size_t)nbox;
  return L;
}

bool bad_plan(hps_plan p) { return p == nullptr; }

// Scratch of hps_leaf_interior_solve_noalloc: a device array of fixed size that every
// GPU the library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol): the
// device address is looked up once per device, with that device current, and kept.
constexpr size_t kNoAllocScratchBytes = HPS_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
std::vector<std::pair<int, void*>> g_scratch_addr;  // (device, address of scratch there)

// Address of `scratch` on `device`, which must be the current device.
hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  for (const auto& e : g_scratch_addr)
    if (e.first == device) {
      *out = e.second;
      return hipSuccess;
    }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr.emplace_back(device, ptr);
  *out = ptr;
  return hipSuccess;
}

// Profiling only (synchronizes the stream): the flops of one solve over nbox boxes.
// Algorithmic: n_i^2 (n_b + 1) per sweep and active box.  Executed: per 64-column tile
// and block row of w rows, (2 w K + w^2) times the tile's columns that are real right-hand
// sides, K the rows the block row's product runs over; the forward sweep of a tile with
// first nonzero row ks stores block rows that end above ks as zeros and starts K at ks.
hps::SolveFlops solve_flops(const hps_plan_s* pl, int nbox, const int* kstart_dev, const int* active_dev,
                            hipStream_t st) {
  const Geom& g = pl->g;
  const int ntn = g.ldx / 64, N = g.n_pad;
  // rows per block row of the solves (hps::solve_block_rows): 128 for FP32 plans, 64 for FP64
  const int br = pl->desc.precision == HPS_FP32_IR ? 128 : 64;
  std::vector<int> act(nbox, 1), ks;
  if (active_dev) (void)hipMemcpyAsync(act.data(), active_dev, sizeof(int) * nbox, hipMemcpyDeviceToHost, st);
  if (kstart_dev) {
    ks.resize((size_t)nbox * ntn);
    (void)hipMemcpyAsync(ks.data(), kstart_dev, sizeof(int) * ks.size(), hipMemcpyDeviceToHost, st);
  }
  (void)hipStreamSynchronize(st);
  std::vector<double> cols(ntn, 0.0);
  for (int tn = 0; tn < ntn; tn++)
    for (int q = 0; q < 4; q++) {
      const int grp = pl->gmap_h[4 * tn + q];
      cols[tn] += std::max(0, std::min(16, g.nrhs - 16 * grp));
    }
  double full = 0.0;  // executed flops of a full sweep: sum over block rows of 2 w K + w^2 = N^2
  for (int tn = 0; tn < ntn; tn++) full += (double)N * N * cols[tn];
  hps::SolveFlops f{0.0, 0.0, 0.0};
  for (int b = 0; b < nbox; b++) {
    if (!act[b]) continue;
    f.alg += (double)g.n * g.n * g.nrhs;
    f.bwd_exec += full;
    if (ks.empty()) {
      f.fwd_exec += full;
      continue;
    }
    for (int tn = 0; tn < ntn; tn++) {
      const int k0 = ks[(size_t)b * ntn + tn];
      double t = 0.0;
      for (int q = 0; q < (N + br - 1) / br; q++) {
        int s, w;
        hps::sweep_block(N, br, false, q, s, w);
        if (s + w <= k0) continue;
        t += 2.0 * w * std::max(0, s - k0) + (double)w * w;
      }
      f.fwd_exec += t * cols[tn];
    }
  }
  return f;
}

}  // namespace

extern "C" {

const char* hps_status_string(hps_status s) {
  switch (s) {
    case HPS_OK: return "ok";
    case HPS_EINVAL: return "invalid argument";
    case HPS_ENOMEM: return "out of memory";
    case HPS_EDEVICE: return "HIP runtime or launch failure";
    case HPS_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

hps_status hps_plan_create(hps_plan* out, const hps_leaf_desc* d) {
  if (!out || !d) return HPS_EINVAL;
  if (d->p < 4 || d->p > 20) return HPS_EUNSUPPORTED;
  for (int a = 0; a < 3; a++)
    if (!(d->h[a] > 0.0) || !std::isfinite(d->h[a])) return HPS_EINVAL;
  if (!std::isfinite(d->kappa)) return HPS_EINVAL;
  if (d->precision != HPS_FP64 && d->precision != HPS_FP32_IR) return HPS_EINVAL;
  if (d->precision == HPS_FP32_IR && (d->ir_max_iter < 0 || d->ir_max_iter > 8 || !(d->ir_tol >= 0.0)))
    return HPS_EINVAL;
  hps_plan_s* pl = new (std::nothrow) hps_plan_s();
  if (!pl) return HPS_ENOMEM;
  pl->desc = *d;
  Geom& g = pl->g;
  g.p = d->p;
  g.m = d->p - 2;
  g.n = g.m * g.m * g.m;
  g.nb = 6 * g.m * g.m;
  g.n_pad = (int)round_up(g.n, 32);
  g.nrhs = g.nb + 1;
  g.ldx = (int)round_up(g.nrhs, 64);
  g.npanel = (g.n_pad + hps::kPanel - 1) / hps::kPanel;
  for (int a = 0; a < 3; a++) {
    g.s1[a] = 2.0 / d->h[a];
    g.s2[a] = g.s1[a] * g.s1[a];
  }
  g.kappa2 = d->kappa * d->kappa;
  std::vector<double> t, D, D2;
  cheb_tables(g.p, t, D, D2);
  std::vector<double> all;
  all.insert(all.end(), t.begin(), t.end());
  all.insert(all.end(), D.begin(), D.end());
  all.insert(all.end(), D2.begin(), D2.end());
  for (double v : D2) all.push_back(g.s2[2] * v);  // s2z D2: the z-derivative coefficients
  if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return HPS_EDEVICE; }
  if (hipMalloc(&pl->tables, all.size() * sizeof(double)) != hipSuccess) { delete pl; return HPS_ENOMEM; }
  if (hipMemcpy(pl->tables, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(pl->tables);
    delete pl;
    return HPS_EDEVICE;
  }
  pl->t = pl->tables;
  g.D = pl->tables + g.p;
  g.D2 = pl->tables + g.p + (size_t)g.p * g.p;
  g.D2z = g.D2 + (size_t)g.p * g.p;
  const int ngrp = g.ldx / 16;
  std::vector<int> coords(g.n + 2 * (size_t)ngrp);
  for (int node = 0; node < g.n; node++)
    coords[node] = (node % g.m) | (((node / g.m) % g.m) << 8) | ((node / (g.m * g.m)) << 16);
  // Internal order of the right-hand-side columns of FP32_IR plans: 16-column groups
  // sorted by the first interior row their A_ib columns touch (the first node of the
  // face node's normal line), so that a 64-column tile of the first forward sweep holds
  // columns with alike runs of leading zero rows (see the first-row kernel).  The f
  // column counts as touching row 0.  FP64 plans solve in place in X: natural order.
  {
    const int m = g.m, mm = m * m;
    std::vector<int> first(ngrp, g.n_pad), order(ngrp);
    for (int c = 0; c < g.nb; c++) {
      const int axis = c / (2 * mm), tq = c % mm, t0 = tq % m, t1 = tq / m;
      const int base = axis == 0 ? m * t0 + mm * t1 : (axis == 1 ? t0 + mm * t1 : t0 + m * t1);
      first[c / 16] = std::min(first[c / 16], base);
    }
    first[g.nb / 16] = 0;
    for (int i = 0; i < ngrp; i++) order[i] = i;
    if (d->precision == HPS_FP32_IR)
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return first[a] < first[b]; });
    for (int i = 0; i < ngrp; i++) {
      coords[g.n + i] = order[i];
      coords[g.n + ngrp + order[i]] = i;
    }
    pl->gmap_h = order;
  }
  if (hipMalloc(&pl->coords, coords.size() * sizeof(int)) != hipSuccess) {
    (void)hipFree(pl->tables);
    delete pl;
    return HPS_ENOMEM;
  }
  if (hipMemcpy(pl->coords, coords.data(), coords.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(pl->coords);
    (void)hipFree(pl->tables);
    delete pl;
    return HPS_EDEVICE;
  }
  g.coords = pl->coords;
  g.gmap = pl->coords + g.n;
  g.ginv = pl->coords + g.n + ngrp;
  sched_lu(pl->lu_ops, 0, g.n_pad, g.n_pad);
  if (hps::residual_prepare(g) != hipSuccess) {
    (void)hipFree(pl->coords);
    (void)hipFree(pl->tables);
    delete pl;
    return HPS_EDEVICE;
  }
  // the no-allocation entry point's scratch on this device (a failed lookup only
  // disables that entry point, which then returns HPS_EDEVICE)
  if (scratch_address(pl->device, &pl->scratch) != hipSuccess) pl->scratch = nullptr;
  *out = pl;
  return HPS_OK;
}

hps_status hps_plan_destroy(hps_plan pl) {
  if (!pl) return HPS_EINVAL;
  (void)hipFree(pl->coords);
  (void)hipFree(pl->tables);
  delete pl;
  return HPS_OK;
}

hps_status hps_plan_get_info(hps_plan pl, hps_plan_info* info) {
  if (bad_plan(pl) || !info) return HPS_EINVAL;
  const Geom& g = pl->g;
  Sizes s = sizes_of(pl);
  info->m = g.m;
  info->n_i = g.n;
  info->n_b = g.nb;
  info->n_pad = g.n_pad;
  info->nrhs = g.nrhs;
  info->ldx = g.ldx;
  info->npanel = g.npanel;
  info->elem_bytes = pl->desc.precision == HPS_FP32_IR ? 4 : 8;
  info->a_bytes = s.a;
  info->perm_bytes = s.perm;
  info->dinv_bytes = s.dinv;
  info->x_bytes = s.x;
  info->ws_bytes = s.ws;
  return HPS_OK;
}

hps_status hps_leaf_nodes(hps_plan pl, int32_t nbox, const double* origin, double* xi, double* xb,
                          hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || (nbox > 0 && (!origin || !xi || !xb))) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  return dev(hps::launch_nodes(pl->g, pl->t, pl->desc.h, nbox, origin, xi, xb, st));
}

hps_status hps_leaf_operators(hps_plan pl, int32_t nbox, const double* b, void* A, double* anorm,
                              hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || nbox > 65535 || (nbox > 0 && (!b || !A || !anorm))) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  hps::ProfScope ps(&pl->prof, hps::Profiler::kOperators, 0.0, st);
  if (pl->desc.precision == HPS_FP32_IR)
    return dev(hps::launch_operators<float>(pl->g, nbox, b, static_cast<float*>(A), anorm, st));
  return dev(hps::launch_operators<double>(pl->g, nbox, b, static_cast<double*>(A), anorm, st));
}

hps_status hps_leaf_factor(hps_plan pl, int32_t nbox, void* A, int32_t* perm, void* dinv, int32_t* info,
                           hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || (nbox > 0 && (!A || !perm || !dinv || !info))) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  if (pl->desc.precision == HPS_FP32_IR)
    return dev(hps::getrf_run<float>(pl->g, pl->lu_ops, static_cast<float*>(A), perm, static_cast<float*>(dinv),
                                     info, nbox, st, &pl->prof, -1, pl->panel_threads));
  return dev(hps::getrf_run<double>(pl->g, pl->lu_ops, static_cast<double*>(A), perm, static_cast<double*>(dinv),
                                    info, nbox, st, &pl->prof));
}

hps_status hps_leaf_dtn(hps_plan pl, int32_t nbox, const void* LU, const int32_t* perm, const void* dinv,
                        const double* b, const double* anorm, const double* f, const double* g_dir,
                        const int32_t* slot_map, double* T_vals, double* gload, double* X, int32_t* ir_iters,
                        double* berr, void* ws, hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || nbox > 65535) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  if (!LU || !perm || !dinv || !b || !anorm || !slot_map || !T_vals || !gload || !X || !ws) return HPS_EINVAL;
  const Geom& g = pl->g;
  if (hps::dtn_part_bytes(g, 1) > 8 * (size_t)g.n_pad * g.ldx) return HPS_EUNSUPPORTED;  // never, for p <= 20
  WsLayout L = ws_layout(pl, nbox, ws);
  const bool ir = pl->desc.precision == HPS_FP32_IR;
  if (!ir) {
    double* B = static_cast<double*>(L.B);
    double* fst = f ? L.fst : nullptr;
    HPS_TRY(hps::launch_rhs<double>(g, nbox, f, B, L.maxb, st, fst));
    HPS_TRY(hps::launch_rhs_first_row(g, nbox, perm, f != nullptr, L.kstart, nullptr, st));
    hps::SolveFlops sf{};
    if (pl->prof.on) sf = solve_flops(pl, nbox, L.kstart, nullptr, st);
    HPS_TRY(hps::getrs_run<double>(g, static_cast<const double*>(LU), perm,
                                   static_cast<const double*>(dinv), B, X, nbox, nullptr, st, &pl->prof, nullptr, 0,
                                   pl->trsm_sched, pl->trsm_waves, L.kstart, 0, nullptr, &sf));
    if (ir_iters) HPS_TRY(hps::launch_fill_int(ir_iters, 0, nbox, st));
    if (berr) {
      HPS_TRY(hps::launch_fill_int(L.active, 1, nbox, st));
      hps::ProfScope ps(&pl->prof, hps::Profiler::kResidual, 0.0, st);
      HPS_TRY(hps::launch_residual<double>(g, nbox, b, f, X, nullptr, nullptr, L.maxr, L.maxx, nullptr, st,
                                           pl->res_cols, fst));
      HPS_TRY(hps::launch_ir_check(nbox, 0, 1, INFINITY, anorm, L.maxb, L.maxr, L.maxx, L.active, nullptr, berr,
                                   st, fst));
    }
  } else {
    float* B = static_cast<float*>(L.B);
    const float* LUf = static_cast<const float*>(LU);
    const float* Dinv = static_cast<const float*>(dinv);
    // The load column is solved and refined as f / s (s a power of two per box), so that a
    // load far below FP32's range is resolved like the other columns; X's load column is
    // scaled back after the refinement.
    double* fst = f ? L.fst : nullptr;
    double* fsc = f ? L.fsc : nullptr;
    if (fsc) HPS_TRY(hps::launch_fscale(g, nbox, f, fsc, st));
    HPS_TRY(hps::launch_rhs<float>(g, nbox, f, B, L.maxb, st, fst, fsc));
    HPS_TRY(hps::launch_rhs_first_row(g, nbox, perm, f != nullptr, L.kstart, L.pos, st));
    // First solve into Y32 only: X0 = Y32 is exact in FP32 and is read from there.  The
    // residual writes R32 in the factor's row order, so each correction runs in place in
    // B; the first correction writes X = X0 + d once, later ones X += d.
    hps::SolveFlops sf{};
    if (pl->prof.on) sf = solve_flops(pl, nbox, L.kstart, nullptr, st);
    HPS_TRY(hps::getrs_run<float>(g, LUf, perm, Dinv, B, L.Y32, nbox, nullptr, st, &pl->prof, nullptr, 0,
                                  pl->trsm_sched, pl->trsm_waves, L.kstart, 0, nullptr, &sf));
    HPS_TRY(hps::launch_fill_int(L.active, 1, nbox, st));
    const int kmax = pl->desc.ir_max_iter;
    const double tol = pl->desc.ir_tol;
    // After a correction most boxes pass the test, so the residual is first formed for the
    // test alone (no R32); the boxes still above the tolerance form it again with R32.
    for (int it = 0; it <= kmax; it++) {
      const int last = it == kmax;
      {
        hps::ProfScope ps(&pl->prof, hps::Profiler::kResidual, 0.0, st);
        if (it == 0)
          HPS_TRY(hps::launch_residual<float>(g, nbox, b, f, L.Y32, B, L.pos, L.maxr, L.maxx, L.active, st,
                                              pl->res_cols, fst, fsc));
        else
          HPS_TRY(hps::launch_residual<double>(g, nbox, b, f, X, nullptr, nullptr, L.maxr, L.maxx, L.active, st,
                                               pl->res_cols, fst, fsc));
      }
      HPS_TRY(hps::launch_ir_check(nbox, it, last, tol, anorm, L.maxb, L.maxr, L.maxx, L.active, ir_iters, berr,
                                   st, fst));
      if (it == 0) HPS_TRY(hps::launch_x_from_y(g, nbox, L.Y32, X, L.active, st));  // boxes done after 0 steps
      if (last) break;
      if (it > 0) {
        hps::ProfScope ps(&pl->prof, hps::Profiler::kResidual, 0.0, st);
        HPS_TRY(hps::launch_residual<double>(g, nbox, b, f, X, B, L.pos, L.maxr, L.maxx, L.active, st,
                                             pl->res_cols, fst, fsc));
      }
      hps::SolveFlops sfc{};
      if (pl->prof.on) sfc = solve_flops(pl, nbox, nullptr, L.active, st);
      HPS_TRY(hps::getrs_run<float>(g, LUf, perm, Dinv, B, B, nbox, L.active, st, &pl->prof, X, it == 0 ? 3 : 2,
                                    pl->trsm_sched, pl->trsm_waves, nullptr, 1, L.Y32, &sfc));
    }
    if (fsc) HPS_TRY(hps::launch_funscale(g, nbox, X, fsc, st));  // X's load column for f
  }
  hps::ProfScope ps(&pl->prof, hps::Profiler::kDtn, 0.0, st);
  // the right-hand-side region of the workspace (8 n_pad ldx bytes per box) is free again:
  // the column-block sums of the loads go there
  return dev(hps::launch_dtn(g, nbox, X, g_dir, slot_map, T_vals, gload, static_cast<double*>(L.B), st));
}

hps_status hps_interface_reduce(int32_t ntrip, const int64_t* triples, int64_t block_elems, double* T_vals,
                                hipStream_t st) {
  if (ntrip < 0 || ntrip > 65535 || block_elems <= 0 || (ntrip > 0 && (!triples || !T_vals))) return HPS_EINVAL;
  return dev(hps::launch_reduce(ntrip, reinterpret_cast<const long long*>(triples), block_elems, T_vals, st));
}

hps_status hps_leaf_reconstruct(hps_plan pl, int32_t nbox, const double* X, const double* u_b, double* u_i,
                                hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || nbox > 65535 || (nbox > 0 && (!X || !u_b || !u_i))) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  return dev(hps::launch_reconstruct(pl->g, nbox, X, u_b, u_i, st));
}

}  // extern "C"

namespace {

// Bytes of scratch an interior solve of nbox boxes uses: r [nbox][n_i], then the
// per-box maxima max|f - A_ib u_b|, max|r|, max|u|.
size_t interior_scratch_bytes(const Geom& g, int nbox) { return 8 * (size_t)nbox * (g.n + 3); }

hps_status interior_solve(hps_plan pl, int nbox, const void* LU, const int32_t* perm, const void* dinv,
                          const double* b, const double* anorm, const double* f, const double* u_b, double* u_i,
                          int steps, double* berr, double* work, hipStream_t st) {
  const Geom& g = pl->g;
  double* r = work;
  double* r0max = r + (size_t)nbox * g.n;
  double* rmax = r0max + nbox;
  double* umax = rmax + nbox;
  const bool f32 = pl->desc.precision == HPS_FP32_IR;
  for (int s = 0; s <= steps; s++) {
    // r = f - A_ib u_b - A_ii u (u = 0 first), then u += (LU)^{-1} r
    HPS_TRY(hps::launch_box_residual(g, nbox, b, f, u_b, s == 0 ? nullptr : u_i, r,
                                     (s == 0 && berr) ? r0max : nullptr, nullptr, st));
    if (f32)
      HPS_TRY(hps::launch_getrs_vec<float>(g, nbox, static_cast<const float*>(LU), perm,
                                           static_cast<const float*>(dinv), r, u_i, s > 0, st));
    else
      HPS_TRY(hps::launch_getrs_vec<double>(g, nbox, static_cast<const double*>(LU), perm,
                                            static_cast<const double*>(dinv), r, u_i, s > 0, st));
  }
  if (berr) {
    HPS_TRY(hps::launch_box_residual(g, nbox, b, f, u_b, u_i, r, rmax, umax, st));
    HPS_TRY(hps::launch_interior_berr(nbox, anorm, r0max, rmax, umax, berr, st));
  }
  return HPS_OK;
}

hps_status interior_args(hps_plan pl, int nbox, const void* LU, const int32_t* perm, const void* dinv,
                         const double* b, const double* anorm, const double* u_b, double* u_i, int steps,
                         const double* berr) {
  if (bad_plan(pl) || nbox < 0 || nbox > 65535 || steps < 0 || steps > 8) return HPS_EINVAL;
  if (nbox > 0 && (!LU || !perm || !dinv || !b || !u_b || !u_i || (berr && !anorm))) return HPS_EINVAL;
  return HPS_OK;
}

}  // namespace

extern "C" {

hps_status hps_leaf_interior_solve(hps_plan pl, int32_t nbox, const void* LU, const int32_t* perm,
                                  const void* dinv, const double* b, const double* anorm, const double* f,
                                  const double* u_b, double* u_i, int32_t steps, double* berr, void* ws,
                                  hipStream_t st) {
  const hps_status a = interior_args(pl, nbox, LU, perm, dinv, b, anorm, u_b, u_i, steps, berr);
  if (a != HPS_OK) return a;
  if (nbox == 0) return HPS_OK;
  if (!ws) return HPS_EINVAL;
  return interior_solve(pl, nbox, LU, perm, dinv, b, anorm, f, u_b, u_i, steps, berr, static_cast<double*>(ws), st);
}

hps_status hps_leaf_interior_solve_noalloc(hps_plan pl, int32_t nbox, const void* LU, const int32_t* perm,
                                          const void* dinv, const double* b, const double* anorm, const double* f,
                                          const double* u_b, double* u_i, int32_t steps, double* berr,
                                          hipStream_t st) {
  const hps_status a = interior_args(pl, nbox, LU, perm, dinv, b, anorm, u_b, u_i, steps, berr);
  if (a != HPS_OK) return a;
  if (nbox == 0) return HPS_OK;
  if (8 * (size_t)nbox * ((size_t)pl->g.n + 3) > kNoAllocScratchBytes) return HPS_EINVAL;
  if (!pl->scratch) return HPS_EDEVICE;
  return interior_solve(pl, nbox, LU, perm, dinv, b, anorm, f, u_b, u_i, steps, berr,
                        static_cast<double*>(pl->scratch), st);
}

hps_status hps_leaf_cn_rhs(hps_plan pl, int32_t nbox, const double* b, double c, const double* u_i,
                          const double* u_b, double* f, hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || nbox > 65535 || !std::isfinite(c)) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  if (!b || !u_i || !u_b || !f) return HPS_EINVAL;
  return dev(hps::launch_box_residual(pl->g, nbox, b, nullptr, u_b, u_i, f, nullptr, nullptr, st, c));
}

hps_status hps_leaf_flux(hps_plan pl, int32_t nbox, const double* u_i, const double* u_b, double* flux,
                         hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || nbox > 65535 || (nbox > 0 && (!u_i || !u_b || !flux))) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  return dev(hps::launch_flux(pl->g, nbox, u_i, u_b, flux, st));
}

hps_status hps_leaf_adjoint_solve(hps_plan pl, int32_t nbox, const void* LU, const int32_t* perm,
                                  const void* dinv, const double* b, const double* w_i, const double* lam_b,
                                  double* z, double* y_b, void* ws, hipStream_t st) {
  (void)b;
  if (bad_plan(pl) || nbox < 0 || nbox > 65535) return HPS_EINVAL;
  if (pl->desc.precision != HPS_FP64) return HPS_EUNSUPPORTED;
  if (nbox == 0) return HPS_OK;
  if (!LU || !perm || !dinv || !w_i || !z || !ws) return HPS_EINVAL;
  const Geom& g = pl->g;
  double* rhs = static_cast<double*>(ws);
  double* zt = rhs + (size_t)nbox * g.n_pad;
  HPS_TRY(hps::launch_adjoint_rhs(g, nbox, w_i, lam_b, rhs, st));
  HPS_TRY(hps::launch_getrs_t(g, nbox, static_cast<const double*>(LU), perm, static_cast<const double*>(dinv), rhs,
                              zt, st));
  HPS_TRY(hps::launch_compact(g, nbox, zt, z, st));
  if (y_b) HPS_TRY(hps::launch_adjoint_yb(g, nbox, zt, y_b, st));
  return HPS_OK;
}

hps_status hps_leaf_workspace_bytes(hps_plan pl, int32_t call, int32_t nbox, size_t* bytes) {
  if (bad_plan(pl) || nbox < 0 || !bytes) return HPS_EINVAL;
  const Geom& g = pl->g;
  const size_t nb = (size_t)nbox;
  switch (call) {
    case HPS_CALL_DTN: *bytes = nb * sizes_of(pl).ws; return HPS_OK;
    case HPS_CALL_INTERIOR_SOLVE: *bytes = 8 * nb * ((size_t)g.n + 3); return HPS_OK;
    case HPS_CALL_ADJOINT_SOLVE: *bytes = 16 * nb * (size_t)g.n_pad; return HPS_OK;
    default: return HPS_EINVAL;
  }
}

hps_status hps_plan_set_tuning(hps_plan pl, int32_t key, int32_t value) {
  if (bad_plan(pl)) return HPS_EINVAL;
  if (key == HPS_TUNE_TRSM_SCHEDULE && (value == hps::kTrsmRows || value == hps::kTrsmSweep)) {
    pl->trsm_sched = value;
    return HPS_OK;
  }
  if (key == HPS_TUNE_TRSM_WAVES && (value == 4 || value == 6 || value == 8)) {
    pl->trsm_waves = value;
    return HPS_OK;
  }
  if (key == HPS_TUNE_RESIDUAL_COLS && (value == 2 || value == 4 || value == 8)) {
    pl->res_cols = value;
    return HPS_OK;
  }
  if (key == HPS_TUNE_PANEL_THREADS && (value == 512 || value == 1024)) {
    pl->panel_threads = value;
    return HPS_OK;
  }
  return HPS_EINVAL;
}

hps_status hps_plan_get_tuning(hps_plan pl, int32_t key, int32_t* value) {
  if (bad_plan(pl) || !value) return HPS_EINVAL;
  if (key == HPS_TUNE_TRSM_SCHEDULE) {
    *value = pl->trsm_sched;
    return HPS_OK;
  }
  if (key == HPS_TUNE_TRSM_WAVES) {
    *value = pl->trsm_waves;
    return HPS_OK;
  }
  if (key == HPS_TUNE_RESIDUAL_COLS) {
    *value = pl->res_cols;
    return HPS_OK;
  }
  if (key == HPS_TUNE_PANEL_THREADS) {
    *value = pl->panel_threads;
    return HPS_OK;
  }
  return HPS_EINVAL;
}

hps_status hps_plan_profile_enable(hps_plan pl, int32_t enable) {
  if (bad_plan(pl)) return HPS_EINVAL;
  pl->prof.reset();
  pl->prof.on = enable != 0;
  return HPS_OK;
}

hps_status hps_plan_profile_read(hps_plan pl, hps_profile* out) {
  if (bad_plan(pl) || !out) return HPS_EINVAL;
  pl->prof.flush();
  for (int f = 0; f < HPS_PROFILE_FAMILIES; f++) {
    out->launches[f] = pl->prof.launches[f];
    out->ms[f] = pl->prof.ms[f];
    out->flops[f] = pl->prof.flops[f];
    out->exec_flops[f] = pl->prof.exec[f];
  }
  return HPS_OK;
}

hps_status hps_leaf_adjoint_grad(hps_plan pl, int32_t nbox, const double* lam_i, const double* u_i, double* grad,
                                 hipStream_t st) {
  if (bad_plan(pl) || nbox < 0 || (nbox > 0 && (!lam_i || !u_i || !grad))) return HPS_EINVAL;
  if (nbox == 0) return HPS_OK;
  return dev(hps::launch_grad(pl->g, nbox, lam_i, u_i, grad, st));
}

}  // extern "C"
