/*
 * hps_leaf.h -- C ABI of the MI355X (gfx950) leaf-box reduction of the
 * two-level Hierarchical Poincare-Steklov solver (Kump, Yesypenko, Martinsson,
 * "A Two-Level Direct Solver for the Hierarchical Poincare-Steklov Method").
 *
 * Problem (paper Sec. 1, eqs. bvp/bvphelmholtz): -Lap u - kappa^2 b(x) u = f on a
 * union of equal rectangular leaf boxes, u = g on the outer boundary.  Each box
 * carries p Chebyshev-Gauss-Lobatto nodes per axis (Sec. 2.1); m = p - 2 interior
 * nodes per axis; n_i = m^3 interior unknowns; n_b = 6 m^2 face unknowns (edges
 * and corners are dropped, Remark 1).
 *
 * Per box the library computes (Sec. 2.2, Sec. 3.1, Alg. 1 and Alg. 2):
 *   hps_leaf_operators   A_ii, the interior block of the collocation operator;
 *   hps_leaf_factor      P A_ii = L U with partial pivoting by rows;
 *   hps_leaf_dtn         X = A_ii^{-1} [A_ib | f_i] (FP64, optionally from an FP32
 *                        factorization refined in FP64), the DtN map
 *                        T = A_bb - A_bi X_b = A_bb + A_bi S (eq. t-block),
 *                        scattered into the block-sparse interface matrix, and
 *                        the equivalent load g = -A_bi v (v = X_f) lifted by the
 *                        Dirichlet data of boundary faces;
 *   hps_leaf_reconstruct u_i = v + S u_b = X_f - X_b u_b (last step of Alg. 2);
 *   hps_leaf_interior_solve  the same u_i from the factors, refined in FP64;
 *   hps_leaf_flux        outward normal derivatives at the faces (interface
 *                        residual for refining the interface solution);
 *   hps_leaf_adjoint_*   transposed solves for the gradient of a misfit with
 *                        respect to b (transpose of eq. factor2).
 * The sparse interface system itself is assembled and factored by the caller.
 *
 * Node numbering inside a box (all arrays below use it):
 *   interior node (i,j,k), 1 <= i,j,k <= m, has index (i-1) + m(j-1) + m^2(k-1);
 *   faces are x-, x+, y-, y+, z-, z+ (face a = 2*axis + side); a face's m^2 nodes
 *   are indexed by its two tangential axes in increasing axis order, the lower
 *   axis fastest; face node index = a*m^2 + local.
 * Box node coordinates: x = origin + h (t + 1)/2 with t_j = -cos(pi j/(p-1)).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer owned by the caller; the library
 *     never frees or keeps them.  Sizes per box come from hps_plan_get_info().
 *   - Calls enqueue work on `stream` and return without synchronizing.  The
 *     returned hps_status reports argument and launch errors only; numerical
 *     outcomes are reported per box in device arrays (info, ir_iters, berr).
 *   - The plan holds the Chebyshev tables on the device and is not thread-safe;
 *     use one plan per host thread.  Plans are tied to the device that was
 *     current at hps_plan_create().
 *   - Per-box matrices are row-major with padded leading dimensions:
 *       A / LU : [nbox][n_pad][n_pad] (FP32 in HPS_FP32_IR mode, else FP64);
 *                rows and columns n_i..n_pad-1 are an identity border.
 *       X      : [nbox][n_pad][ldx] FP64; column c < n_b is face node c,
 *                column n_b is the load column, the rest is zero padding.
 */
#ifndef HPS_LEAF_H
#define HPS_LEAF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPS_OK = 0,
  HPS_EINVAL = -1,       /* bad argument (null pointer, size out of range)      */
  HPS_ENOMEM = -2,       /* plan creation could not allocate its tables          */
  HPS_EDEVICE = -3,      /* a HIP call or kernel launch failed                   */
  HPS_EUNSUPPORTED = -4  /* p outside the compiled range                         */
} hps_status;

typedef enum { HPS_FP64 = 0, HPS_FP32_IR = 1 } hps_precision;

typedef struct {
  int32_t p;            /* Gauss-Lobatto nodes per axis per box, 4 <= p <= 20      */
  double h[3];          /* box side lengths along x, y, z (> 0)                    */
  double kappa;         /* wavenumber                                              */
  int32_t precision;    /* hps_precision                                           */
  int32_t ir_max_iter;  /* FP32_IR: max FP64 refinement steps (0..8)               */
  double ir_tol;        /* FP32_IR: stop when the normwise backward error
                           max|R| / (|A_ii|_inf max|X| + max|B|) <= ir_tol         */
} hps_leaf_desc;

typedef struct {
  int32_t m, n_i, n_b;   /* interior nodes per axis, per box, face nodes per box  */
  int32_t n_pad;         /* n_i rounded up to a multiple of 32                     */
  int32_t nrhs, ldx;     /* n_b + 1 right-hand sides; ldx = nrhs rounded to 64     */
  int32_t npanel;        /* LU panels of width <= 64                               */
  int32_t elem_bytes;    /* 4 (FP32_IR) or 8 (FP64): element size of A / LU       */
  size_t a_bytes;        /* per box: A / LU storage                                */
  size_t perm_bytes;     /* per box: row permutation (int32 [n_pad])               */
  size_t dinv_bytes;     /* per box: inverses of the diagonal LU blocks            */
  size_t x_bytes;        /* per box: X (FP64 [n_pad][ldx])                         */
  size_t ws_bytes;       /* per box: workspace of hps_leaf_dtn                     */
} hps_plan_info;

typedef struct hps_plan_s* hps_plan;

/* Create a plan: validates `desc`, builds the differentiation tables of paper
 * Sec. 2.1 in FP64 on the host and uploads them.  Returns HPS_EINVAL for bad
 * sizes, HPS_EUNSUPPORTED for p outside [4, 20], HPS_ENOMEM/HPS_EDEVICE if the
 * device tables cannot be created.  *plan is set only on success. */
hps_status hps_plan_create(hps_plan* plan, const hps_leaf_desc* desc);
hps_status hps_plan_destroy(hps_plan plan);
hps_status hps_plan_get_info(hps_plan plan, hps_plan_info* info);

/* Coordinates of the interior nodes xi [nbox][n_i][3] and face nodes
 * xb [nbox][n_b][3] of boxes with lower corners origin [nbox][3] (Sec. 2.1).
 * The caller evaluates b, f and g at these points. */
hps_status hps_leaf_nodes(hps_plan plan, int32_t nbox, const double* origin, double* xi, double* xb,
                          hipStream_t stream);

/* a1 -- collocation operator (Sec. 2.1 eq. Aentries, interior rows; Alg. 1, the
 * per-box operator step).  Writes A_ii = -(Dxx + Dyy + Dzz) - kappa^2
 * diag(b) restricted to interior nodes, rounded to the plan's element type, into
 * A [nbox][n_pad][n_pad] with an identity border, and |A_ii|_inf (FP64, exact
 * row sums) into anorm [nbox].  b: [nbox][n_i] FP64 values at interior nodes. */
hps_status hps_leaf_operators(hps_plan plan, int32_t nbox, const double* b, void* A, double* anorm,
                              hipStream_t stream);

/* a2 -- dense LU with partial pivoting of every box's A_ii, in place (Alg. 1,
 * the per-box solution-operator step; the interior block is block diagonal,
 * Sec. 2.2).  The pivot in column k is the row of largest modulus among the
 * rows not yet pivoted (lowest current position on ties).  On return, for
 * position i, row perm[i] of A holds row i of L (unit lower, below the
 * diagonal) and of U (on and above); perm [nbox][n_pad] int32.  dinv receives
 * the inverses of the diagonal 64x64 blocks of L and U (workspace reused by
 * the solves).  info[box] = 0, or k > 0 if U(k,k) (1-based) is exactly zero or
 * not finite (LAPACK convention; the factorization still completes). */
hps_status hps_leaf_factor(hps_plan plan, int32_t nbox, void* A, int32_t* perm, void* dinv, int32_t* info,
                           hipStream_t stream);

/* a3 + a4 -- interior solves and DtN assembly (Sec. 2.2 four-step solve, steps
 * 1-2; Sec. 3.1 eq. t-block; Alg. 1 and the load loop of Alg. 2).
 *   X = A_ii^{-1} [A_ib | f_i] in FP64.  FP64 plans solve with the FP64 factors.
 *   FP32_IR plans solve with the FP32 factors and refine in FP64: R = B - A_ii X
 *   is formed in FP64 through the tensor-product structure of A_ii (b is needed
 *   for that), the correction is solved in FP32 and added in FP64, until the
 *   backward error is <= ir_tol or ir_max_iter steps; ir_iters[box] = steps
 *   taken, or -1 - steps if still above ir_tol (a NaN counts as above);
 *   berr[box] = final backward error: the larger of
 *     max|R| / (|A_ii|_inf max|X| + max|B|) over every column of [A_ib | f_i] and,
 *     when f is given, the same over the load column alone (its entries are far
 *     smaller than A_ib's, so the first figure alone would not see its error).
 *   FP32_IR plans solve and refine the load column as f / s, s the power of two
 *   with 1 <= max|f| / s < 2 per box (exact; berr is taken in that scale), so that
 *   loads far below FP32's range are resolved like the other columns.
 *   T = A_bb - A_bi X_b: row block a / column block b of box t is written to
 *   T_vals + slot_map[t*36 + 6a + b] * m^4 (row-major m^2 x m^2 block) when the
 *   slot is >= 0; slot -1 drops the block (rows of boundary faces, columns of
 *   boundary faces).  g[box][n_b] = -A_bi X_f - sum over boundary faces b of
 *   T[:, b] g_dir[box][b]: the load lifted by the Dirichlet data g_dir (values on
 *   boundary faces, ignored elsewhere).  f, g_dir may be NULL (zero).
 *   ws: hps_plan_info.ws_bytes per box.  X, T_vals, g, ir_iters, berr are
 *   written; ir_iters/berr may be NULL. */
hps_status hps_leaf_dtn(hps_plan plan, int32_t nbox, const void* LU, const int32_t* perm, const void* dinv,
                        const double* b, const double* anorm, const double* f, const double* g_dir,
                        const int32_t* slot_map, double* T_vals, double* g, double* X, int32_t* ir_iters,
                        double* berr, void* ws, hipStream_t stream);

/* Deterministic reduction of duplicate interface blocks (Alg. 1, accumulation of
 * each box's DtN blocks into the interface matrix).  The diagonal block of an
 * internal face receives one contribution from each of its two boxes; each box
 * writes its contribution to a slot of its own and this call forms, for
 * q = 0..ntrip-1, T_vals[dst_q] = T_vals[lo_q] + T_vals[hi_q] (blocks of
 * block_elems doubles; triples int64 [ntrip][3] = (dst, lo, hi) block indices,
 * every dst once, no dst equal to any lo or hi).  The sources are left intact, so
 * calling it again after some boxes were recomputed gives the right sums. */
hps_status hps_interface_reduce(int32_t ntrip, const int64_t* triples, int64_t block_elems, double* T_vals,
                                hipStream_t stream);

/* a5 -- reconstruction (Sec. 2.2 step 4; Alg. 2 last loop): u_i = X_f - X_b u_b
 * for every box, with X from hps_leaf_dtn and u_b [nbox][n_b] the box's face
 * values (interface solution on internal faces, Dirichlet data on boundary
 * faces).  u_i: [nbox][n_i] FP64. */
hps_status hps_leaf_reconstruct(hps_plan plan, int32_t nbox, const double* X, const double* u_b, double* u_i,
                                hipStream_t stream);

/* a5, solve form (Sec. 2.2 step 4 with the local factors instead of X; the
 * interior solve of Alg. 2): u_i = A_ii^{-1} (f_i - A_ib u_b) for every box, with
 * the factors of hps_leaf_factor and FP64 refinement: u = (LU)^{-1} r_0, then
 * `steps` times r = f_i - A_ib u_b - A_ii u (FP64, tensor structure of the
 * operator), u += (LU)^{-1} r.  The vector solves run in FP64 arithmetic on the
 * stored (FP32 or FP64) factors; with FP32 factors each step gains about six
 * digits on well-conditioned boxes, so 2 steps reach FP64 rounding.
 * b, f_i (NULL = 0), u_i: [nbox][n_i]; u_b: [nbox][n_b]; steps in 0..8.
 * berr [nbox] (may be NULL): the final normwise backward error
 *   max|f_i - A_ib u_b - A_ii u| / (|A_ii|_inf max|u| + max|f_i - A_ib u_b|)
 * (NaN counts as +inf); anorm [nbox] (|A_ii|_inf from hps_leaf_operators) is
 * required when berr is given.  A caller compares berr with its tolerance: on
 * an ill-conditioned box FP32 factors can leave it large, and that box then
 * needs FP64 factors.  ws: at least 8 nbox (n_i + 3) bytes (one FP64 vector and
 * three scalars per box; hps_plan_info.ws_bytes per box is always enough).  Any
 * precision. */
hps_status hps_leaf_interior_solve(hps_plan plan, int32_t nbox, const void* LU, const int32_t* perm,
                                  const void* dinv, const double* b, const double* anorm, const double* f,
                                  const double* u_b, double* u_i, int32_t steps, double* berr, void* ws,
                                  hipStream_t stream);

/* Crank-Nicolson right-hand side (Sec. 4.4: the previous step is the body load of the
 * interior solves, through I + (dt/2) A): f = c u_i - (A_ii u_i + A_ib u_b) for every box,
 * with the plan's operator A = -Lap - kappa^2 diag(b) (eq. Aentries, interior rows).  For
 * u_t = nu Lap u + k^2 b' u the plan is built with kappa = 1 and b = k^2 b'/nu - 2/(nu dt),
 * and c = 4/(nu dt); then the step is A u^{n+1} = f.  b, u_i, f: [nbox][n_i]; u_b
 * [nbox][n_b] (the face values of u^n, Dirichlet data on boundary faces); FP64. */
hps_status hps_leaf_cn_rhs(hps_plan plan, int32_t nbox, const double* b, double c, const double* u_i,
                           const double* u_b, double* f, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): hps_leaf_interior_solve
 * without the ws argument.  Its scratch (8 nbox (n_i + 3) bytes) lives in a
 * device array of HPS_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends; the call allocates nothing.  Returns
 * HPS_EINVAL when 8 nbox (n_i + 3) exceeds HPS_NOALLOC_SCRATCH_BYTES (at most
 * 1526 boxes at p = 16, 718 at p = 20), HPS_EDEVICE if the array's device
 * address could not be looked up at hps_plan_create.  Every call on one GPU
 * shares the array, so calls that overlap on one GPU (two streams, two host
 * threads) race and give wrong results; order them on one stream.  Results are
 * bitwise those of hps_leaf_interior_solve. */
#define HPS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
hps_status hps_leaf_interior_solve_noalloc(hps_plan plan, int32_t nbox, const void* LU, const int32_t* perm,
                                          const void* dinv, const double* b, const double* anorm,
                                          const double* f, const double* u_b, double* u_i, int32_t steps,
                                          double* berr, hipStream_t stream);

/* Outward normal derivative at every face node of every box, flux = A_bi u_i +
 * A_bb u_b (the face rows of eq. Aentries: (2/h_a) D[p-1][.] along the normal line
 * on + faces, -(2/h_a) D[0][.] on - faces).  Summed over the two boxes of an
 * internal face it is minus the residual of the interface equations
 * T_FF u_F = rhs for the exact interiors, which the caller uses to refine u_F.
 * u_i: [nbox][n_i]; u_b, flux: [nbox][n_b], FP64. */
hps_status hps_leaf_flux(hps_plan plan, int32_t nbox, const double* u_i, const double* u_b, double* flux,
                         hipStream_t stream);

/* a6 -- adjoint solves for dJ/db (transpose of eq. factor2):
 * hps_leaf_adjoint_solve:  z = A_ii^{-T} (w_i - A_bi^T lam_b) per box and
 *   y_b = -A_ib^T z; lam_b may be NULL (zero).  Uses the FP64 factors of
 *   hps_leaf_factor: FP64 plans only (HPS_EUNSUPPORTED otherwise).
 *   w_i, z: [nbox][n_i]; lam_b, y_b: [nbox][n_b]; y_b may be NULL.
 * ws: hps_plan_info.ws_bytes per box. */
hps_status hps_leaf_adjoint_solve(hps_plan plan, int32_t nbox, const void* LU, const int32_t* perm,
                                  const void* dinv, const double* b, const double* w_i, const double* lam_b,
                                  double* z, double* y_b, void* ws, hipStream_t stream);

/* Gradient assembly: grad[box][n_i] = kappa^2 * lam_i * u_i (dA/db_n = -kappa^2
 * e_n e_n^T at interior node n). */
hps_status hps_leaf_adjoint_grad(hps_plan plan, int32_t nbox, const double* lam_i, const double* u_i,
                                 double* grad, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Interface system T u_F = rhs on the GPU (the sparse factorization that the paper
 * hands to a multifrontal CPU solver, Sec. 3.1 and Sec. 3.3; its cost dominates the
 * build stage, Sec. 4.2).  Nested dissection over the box grid with dense fronts: a
 * front holds the n_P separator unknowns its two halves share (first, padded to n_piv)
 * and the unknowns of its outer boundary (after them), F = [[A_PP, A_PB],
 * [A_BP, A_BB]], assembled by the caller from the halves' Schur complements (a single
 * box contributes its DtN blocks T^tau).  Fronts are FP64, row-major n x n, stored
 * back to back; perm [nfront][n] int32; dinv [nfront][hps_front_dinv_elems] FP64.
 * ------------------------------------------------------------------------- */
typedef struct hps_front_plan_s* hps_front_plan;

/* A plan for fronts of n rows (64 <= n <= 12288, a multiple of 32) whose first n_piv
 * rows and columns (a multiple of 64, <= n) are eliminated.  HPS_EINVAL for other
 * sizes, HPS_EDEVICE if the solve kernel's LDS limit cannot be raised. */
hps_status hps_front_plan_create(hps_front_plan* plan, int32_t n, int32_t n_piv);
hps_status hps_front_plan_destroy(hps_front_plan plan);
/* Elements of dinv per front (0 for a null plan). */
size_t hps_front_dinv_elems(hps_front_plan plan);

/* F = 0 for nfront fronts of n x n, with ones on the diagonal at positions [d0, d1)
 * and [d2, d3) (the padding of the separator and boundary blocks). */
hps_status hps_front_init(int32_t nfront, int32_t n, int32_t d0, int32_t d1, int32_t d2, int32_t d3, double* F,
                          hipStream_t stream);

/* Extend-add of bm x bm blocks: for each task t = tasks[4t .. 4t+3] = (dst offset, src
 * offset, dst row stride, src row stride), in elements, dst[d + i ld_d + j] += src[s +
 * i ld_s + j].  Tasks of one call must write disjoint blocks (the caller adds the two
 * halves of a front in two calls, so that sums have a fixed order). */
hps_status hps_front_block_add(int32_t ntask, const int64_t* tasks, int32_t bm, double* dst, const double* src,
                               hipStream_t stream);

/* Segments of len doubles: for each task (dst offset, src offset) = tasks[2t .. 2t+1],
 * dst[d + i] = src[s + i] (add = 0), dst[d + i] += src[s + i] (add = 1) or
 * dst[d + i] -= src[s + i] (add = -1).  Tasks of one call must write disjoint segments. */
hps_status hps_front_segments(int32_t ntask, const int64_t* tasks, int32_t len, double* dst, const double* src,
                              int32_t add, hipStream_t stream);

/* Partial LU of nfront fronts in place: row pivoting among the first n_piv rows (the
 * leaf LU's panel rule), P_r A_PP = L11 U11, L21 = A_BP U11^{-1}, U12 = L11^{-1} P_r A_PB,
 * and the Schur complement S = A_BB - L21 U12 in rows and columns [n_piv, n).  Rows past
 * n_piv keep their places (perm[i] = i there).  info[f] = 0, or k > 0 if the k-th pivot
 * (1-based) is zero or not finite. */
hps_status hps_front_factor(hps_front_plan plan, int32_t nfront, double* F, int32_t* perm, double* dinv,
                            int32_t* info, hipStream_t stream);

/* One vector per front, vec [nfront][n] FP64, in place.  mode 0 (upward): vec holds r
 * in unknown order; on return positions [0, n_piv) hold y = L11^{-1} P_r r_P and
 * [n_piv, n) hold r_B - L21 y.  mode 1 (downward): vec holds y (as mode 0 left it) and
 * u_B in [n_piv, n); on return [0, n_piv) holds u_P = U11^{-1}(y - U12 u_B).
 * Modes 2 and 3 do the same for the transposed system (adjoint solves): mode 2 leaves
 * z = U11^{-T} r_P in [0, n_piv) and r_B - U12^T z; mode 3 takes z and lam_B and leaves
 * lam_P = P_r^T L11^{-T}(z - L21^T lam_B) in [0, n_piv), in unknown order. */
hps_status hps_front_solve(hps_front_plan plan, int32_t nfront, const double* F, const int32_t* perm,
                           const double* dinv, double* vec, int32_t mode, hipStream_t stream);

/* Device workspace, in bytes, that one call needs for `nbox` boxes (the `ws`
 * argument; caller-owned, any alignment of at least 256 bytes):
 *   HPS_CALL_DTN             hps_leaf_dtn: nbox * hps_plan_info.ws_bytes
 *   HPS_CALL_INTERIOR_SOLVE  hps_leaf_interior_solve: 8 nbox (n_i + 3)
 *   HPS_CALL_ADJOINT_SOLVE   hps_leaf_adjoint_solve: 16 nbox n_pad
 * HPS_EINVAL for an unknown call, nbox < 0 or bytes == NULL; *bytes is set only
 * on success. */
typedef enum { HPS_CALL_DTN = 0, HPS_CALL_INTERIOR_SOLVE = 1, HPS_CALL_ADJOINT_SOLVE = 2 } hps_call;
hps_status hps_leaf_workspace_bytes(hps_plan plan, int32_t call, int32_t nbox, size_t* bytes);

/* Run-time tuning of a plan.  A knob changes how the work is scheduled, never
 * what is computed: every setting gives bitwise the same results.
 *   HPS_TUNE_TRSM_SCHEDULE: the interior solves of hps_leaf_dtn (Alg. 1, the
 *     triangular solves with the LU factors) as 0 = one launch per 64-row block
 *     row (default) or 1 = one launch per forward / backward sweep, each
 *     workgroup running every block row of its (box, 64-column) tile.
 *   HPS_TUNE_TRSM_WAVES: FP32_IR plans, p <= 18: the waves per SIMD (4, 6 or 8;
 *     default 4) the solve kernels are register-allocated for, i.e. how many of
 *     their workgroups one CU keeps resident.  FP64 plans and p >= 19 always run
 *     at 4; the value is accepted and ignored there.
 *   HPS_TUNE_RESIDUAL_COLS: the FP64 refinement residual of FP32_IR plans (the
 *     Alg. 1 solves, refined), 6 <= p <= 18: right-hand-side columns per workgroup,
 *     4 (512 threads, two workgroups per CU, default), 8 (1024 threads) or 2 (256
 *     threads, four workgroups per CU).  Other p
 *     use one kernel and ignore the value.
 *   HPS_TUNE_PANEL_THREADS: FP32_IR plans whose padded interior size is 2049..3072
 *     (p = 15, 16): threads of the pivoted panel factorization of hps_leaf_factor,
 *     512 (six rows per thread) or 1024 (default: three rows per thread, four waves
 *     per SIMD).  Other plans accept the value and use 512.
 * set: HPS_EINVAL for an unknown key or value (the plan is left unchanged);
 * get: writes the current value to *value. */
typedef enum {
  HPS_TUNE_TRSM_SCHEDULE = 0,
  HPS_TUNE_TRSM_WAVES = 1,
  HPS_TUNE_RESIDUAL_COLS = 2,
  HPS_TUNE_PANEL_THREADS = 3
} hps_tuning_key;
hps_status hps_plan_set_tuning(hps_plan plan, int32_t key, int32_t value);
hps_status hps_plan_get_tuning(hps_plan plan, int32_t key, int32_t* value);

/* Human-readable message for a status code (static storage). */
const char* hps_status_string(hps_status s);

/* Kernel timing (tracing aid, not part of the method).  While enabled, every
 * launch the plan makes (or run of consecutive launches of one family, such as
 * the block rows of one triangular sweep) is bracketed by HIP events on its
 * stream; hps_plan_profile_read synchronizes on the recorded events and
 * returns, per kernel family, the number of kernel launches, total
 * milliseconds, the algorithmic flops of those launches and the flops the
 * kernels executed.  Algorithmic: 2*M*N*K for tile GEMMs, 2*w*K*ncols + w*w*ncols
 * for the LU's short triangular solves, n_i^2 * (n_b + 1) per box and sweep for
 * the solves of hps_leaf_dtn (boxes whose refinement has already converged run
 * no correction and count nothing), 0 for bandwidth kernels.  Executed equals
 * algorithmic except for the solves, where it sums 2 w K + w^2 per 64-row block
 * row over the real right-hand-side columns of each 64-column tile on the padded
 * size n_pad, leaving out the block rows of the first forward sweep that are
 * structurally zero and skipped.  Families: 0 LU GEMM, 1 LU panel, 2 LU
 * triangular solves, 3 forward solve (L), 4 backward solve (U), 5 residual,
 * 6 DtN, 7 operators.  Enabling clears the counters.  Event recording adds
 * launch overhead and, for the solve flops, a host copy of small per-box arrays
 * with a stream synchronization per solve; leave it off in production. */
#define HPS_PROFILE_FAMILIES 8
typedef struct {
  int64_t launches[HPS_PROFILE_FAMILIES];
  double ms[HPS_PROFILE_FAMILIES];
  double flops[HPS_PROFILE_FAMILIES];
  double exec_flops[HPS_PROFILE_FAMILIES];
} hps_profile;
hps_status hps_plan_profile_enable(hps_plan plan, int32_t enable);
hps_status hps_plan_profile_read(hps_plan plan, hps_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* HPS_LEAF_H */
