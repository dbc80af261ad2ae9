/*
 * apf.h -- C ABI of the MI355X augmented-partial-factorization library.
 *
 * One sparse direct factorization of the augmented matrix K = [A, B; C, D]
 * of a 2D TM (Ez) finite-difference frequency-domain problem yields the
 * generalised scattering matrix S = C A^-1 B - D (Sec. 2 of Li, Lin and Hsu,
 * "Fast multi-channel inverse design through augmented partial
 * factorization", arXiv 2306.09257) and the gradient of an objective f(S)
 * with respect to every design-pixel permittivity (Sec. 2, Eqs. (1)-(3)).
 *
 * Discretisation (the paper leaves it to its solver package; this library
 * fixes it and documents it here):
 *   - Ez on nodes (i, j), i = 0..nx-1 along x (periodic), j = 0..ny-1 rows
 *     from the top; node index n = j*nx + i; spacing dx in both directions.
 *   - Time convention exp(-i w t).  Uniaxial PML stretching y in the top
 *     npml_top and bottom npml_bot rows: s(d) = 1 + i alpha (d/L)^m, d the
 *     distance in pixels past the PML's inner face (the half-row between the
 *     PML and the first physical row), m = pml_power,
 *     alpha = (m+1) ln(1/R0) / (2 h sqrt(eps_pml) L), h = 2 pi dx/lambda.
 *   - A (dx^2-scaled, complex symmetric):
 *       (A E)_ij = s_j (2E_ij - E_i+1,j - E_i-1,j)
 *                + (1/s_j+1/2 + 1/s_j-1/2) E_ij - E_i,j+1/s_j+1/2 - E_i,j-1/s_j-1/2
 *                - h^2 eps_ji s_j E_ij,      E = 0 beyond rows 0 and ny-1.
 *   - Channel a: phi_a(i) = exp(2 pi i a i/nx)/sqrt(nx), q_a in (0, pi) with
 *     sin^2(q_a/2) = h^2 eps_medium/4 - sin^2(pi a/nx).
 *     B[(i, src_row), a] = -2i sqrt(sin q_a) phi_a(i)   (unit-flux line source)
 *     C[b, (i, prj_row)] = sqrt(sin q_b) conj(phi_b(i)), D = 0.
 *
 * Conventions of every entry point:
 *   - Complex arrays are interleaved (re, im) float64 pairs, row-major.
 *   - Pointers named *_dev are device pointers owned by the caller; they must
 *     stay valid until the work queued on `stream` has finished.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it, except where stated.
 *   - No exceptions cross the ABI; every call returns an apf_status and, on
 *     failure, leaves a thread-local message for apf_last_error().
 *   - Calls on one handle must not overlap in time (the handle owns the
 *     factors and workspaces they share); distinct handles are independent.
 */
#ifndef APF_H
#define APF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APF_OK = 0,
  APF_EINVAL = -1,     /* bad argument or descriptor                       */
  APF_ENOMEM = -2,     /* device or host allocation failed                 */
  APF_EHIP = -3,       /* a HIP runtime call failed                        */
  APF_ESINGULAR = -4,  /* a zero or non-finite pivot appeared in a pivot block */
  APF_ENOTCONV = -5,   /* iterative refinement did not reach its tolerance */
  APF_ESTATE = -6      /* call out of order (see apf_grad / apf_factor_schur) */
} apf_status;

typedef enum {
  APF_FP64 = 0,        /* every front operation in complex FP64            */
  APF_MIXED = 1,       /* front GEMMs and sweeps on FP32 MFMA (operands
                          rounded to FP32, FP32 accumulation); pivot blocks,
                          storage, the S / gradient reductions and the
                          low-rank subtree products in FP64; no iterative
                          refinement: the result carries the FP32 rounding
                          amplified by ill-conditioned pivot blocks
                          (measured 1e-6 .. 4e-4 relative)                 */
  APF_MIXED_REFINED = 2 /* the APF_MIXED factorization, then FP64 iterative
                          refinement of the M_in forward fields A^-1 B (in
                          apf_factor_schur) and of the M_in weighted adjoint
                          fields A^-1 (C^T dF/dS) (in apf_grad): residuals
                          r - A x from the FP64 stencil, corrections by
                          full solves with the FP32-computed factors of every
                          front, S = C x and the gradient contraction in
                          FP64.  Needs apf_set_refinement before the first
                          apf_assemble; not for the batched factorization */
} apf_precision;

typedef struct apf_handle apf_handle;

/* Problem descriptor (host memory; copied by apf_create).
 * Rows: [0, npml_top) top PML | top medium eps_top | design rows
 * [design_row0, design_row1) | bottom medium eps_bot | bottom PML.
 * src_row must lie in the top medium and prj_row in the bottom medium, both
 * outside the PML and outside the design rows; the design rows must not
 * overlap the PML.  Every channel order must propagate in the medium of its
 * row.  nx >= 3. */
typedef struct {
  int32_t nx, ny;
  double dx_over_lambda;
  int32_t npml_top, npml_bot;
  double pml_R0;
  int32_t pml_power;
  double eps_top, eps_bot;
  int32_t src_row, prj_row;
  int32_t design_row0, design_row1;
  int32_t n_in, n_out;
  const int32_t *in_orders;   /* n_in channel orders a (source row)       */
  const int32_t *out_orders;  /* n_out channel orders b (projection row)  */
  int32_t leaf_size;          /* max nodes of a nested-dissection leaf; 0 = default (48) */
} apf_problem_desc;

/* Validate the descriptor and create a handle (host only, no GPU work). */
apf_status apf_create(const apf_problem_desc *desc, apf_handle **out);

/* Symbolic analysis (host only; idempotent; cached on the handle): geometric
 * nested dissection of the periodic grid, elimination tree, frontal index
 * sets, extend-add maps, level schedule and exact work counts.  The sparsity
 * of K does not depend on eps, so one analysis serves every later call
 * (Sec. 2: one partial factorization per evaluation of S). */
apf_status apf_analyze(apf_handle *h);

/* Assemble A (the 5-point operator above with the given permittivity) on
 * the GPU: its five stencil values per node, which the factorization scatters
 * into the frontal workspaces level by level (the rows of B and C are
 * generated there from the channel definitions).
 *   eps_dev: float64 [ny][nx] relative permittivity (real, nonzero and
 *   finite).  The values are checked on the GPU as they are read; since this
 *   call only enqueues work, a zero, NaN or infinite value is reported by the
 *   next apf_factor_schur (or apf_factor_schur_batched) as APF_EINVAL.
 * The first call allocates the device plan (workspaces, factor storage, task
 * lists) and synchronises `stream` once; later calls only enqueue work.
 * Requires apf_analyze. */
apf_status apf_assemble(apf_handle *h, const double *eps_dev, void *stream);

/* Numeric multifrontal partial factorization of K = [A, B; C, 0] (Sec. 2):
 * eliminates every grid unknown and writes the Schur-complement block as
 *   S_dev: complex128 [n_out][n_in],  S = C A^-1 B.
 * prec: APF_FP64, APF_MIXED or APF_MIXED_REFINED (see apf_precision); apf_grad
 * then runs in the same precision.  APF_MIXED_REFINED returns APF_ENOTCONV
 * when the refinement misses its tolerance (S is then the last iterate's,
 * and apf_grad may still run).
 * The factors are kept on the handle for apf_grad.  Synchronises `stream` at
 * the end to read the device status words: APF_EINVAL if the last assembled
 * permittivity had a zero or non-finite value, APF_ESINGULAR if a pivot block
 * met a zero or non-finite pivot (the pivot search always picks an unused row,
 * so the factorization itself stays in bounds; S is then meaningless and
 * apf_grad refuses to run).  Requires apf_assemble. */
apf_status apf_factor_schur(apf_handle *h, apf_precision prec, double *S_dev,
                            void *stream);

/* Batched partial factorization of n independent problems (different grids,
 * wavelengths and channel sets allowed): every handle must have been
 * analysed and assembled (its own apf_assemble).  The elimination-tree levels
 * of all problems (counted from the leaves) are merged, so each level of the
 * whole batch is one launch per kernel; the first call on a set of handles
 * builds the merged task lists (cached until one of the handles is
 * destroyed), and later calls with the same handles and outputs replay a
 * HIP graph captured from the first graph-mode call (no graph while
 * profiling is on for hs[0]).
 *   hs: n handle pointers (host array); S_devs: n device pointers, complex128
 *   [n_out_i][n_in_i] each.  The factors stay on each handle for apf_grad.
 *   Synchronises `stream` at the end; APF_EINVAL if a problem's permittivity
 *   had a zero or non-finite value, APF_ESINGULAR if any pivot block of the
 *   batch had a zero or non-finite pivot (either way no handle of the batch
 *   may then be used by apf_grad). */
apf_status apf_factor_schur_batched(apf_handle *const *hs, int32_t n, apf_precision prec,
                                    double *const *S_devs, void *stream);

/* Objective helper for f = sum_nm w_nm |S_nm|^2 (Sec. 2, Eq. (1) needs the
 * Wirtinger derivative dF/dS):
 *   S_dev, dfdS_dev: complex128 [n_out][n_in]; w_dev: float64 [n_out][n_in];
 *   f_dev: one float64.  Writes f and dF/dS = w * conj(S). */
apf_status apf_weighted_power(apf_handle *h, const double *S_dev,
                              const double *w_dev, double *f_dev,
                              double *dfdS_dev, void *stream);

/* The same objective as apf_weighted_power, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): no handle, no library allocation, no allocating library
 * call.  The reduction's block partials (at most 1024 doubles) live in a
 * static device array of the library, one per GPU, looked up on the first
 * call on each device (with that device current).
 *   S_dev, dfdS_dev: complex128 [n]; w_dev: float64 [n]; f_dev: one float64.
 *   Writes f = sum w |S|^2 and dF/dS = w conj(S), summed in the same order as
 *   apf_weighted_power for the same n.
 * APF_EINVAL for a null pointer or n outside [1, 2^40]; APF_EHIP if the
 * launch fails.  Every call on one GPU uses that GPU's single scratch array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller. */
apf_status apf_weighted_power_noalloc(const double *S_dev, const double *w_dev, int64_t n,
                                      double *f_dev, double *dfdS_dev, void *stream);

/* Objective helper for the beam-splitter figure of merit (Sec. 3, Eq. (5)):
 *   f = sum_nm (|S_nm|^2 - t_nm)^2,  t_nm = t1 where the output order minus
 *   the input order is +-1 (the +-1 diffraction orders; the paper's t1 is
 *   1/2), 0 elsewhere;  dF/dS = 2 (|S|^2 - t) conj(S) (the paper's df/dT).
 *   S_dev, dfdS_dev: complex128 [n_out][n_in]; f_dev: one float64.
 * Requires apf_assemble since the handle was analysed (APF_ESTATE). */
apf_status apf_splitter_fom(apf_handle *h, const double *S_dev, double t1,
                            double *f_dev, double *dfdS_dev, void *stream);

/* Objective helper for the multi-angle splitter: for input a the targets
 * T(a) are the outputs whose order differs from a's by g * delta, |g| <= gmax
 * (a supercell's diffraction orders, Sec. 3); with p = |S|^2 and mu_a the
 * mean of p over T(a),
 *   f = sum_a sum_{t in T(a)} [ -p_ta + (p_ta - mu_a)^2 ]
 * (transmit into the target orders, evenly), and
 *   dF/dS_ta = (-1 + 2 (p_ta - mu_a)) conj(S_ta) on the targets, 0 elsewhere.
 *   S_dev, dfdS_dev: complex128 [n_out][n_in]; f_dev: one float64.
 * APF_EINVAL for delta <= 0, gmax < 0 or more than 262,144 inputs;
 * APF_ESTATE before the first apf_assemble. */
apf_status apf_group_fom(apf_handle *h, const double *S_dev, int32_t delta, int32_t gmax,
                         double *f_dev, double *dfdS_dev, void *stream);

/* Ridge parameterization of the design rows (Sec. 3: edge positions as the
 * design parameters, mirror symmetry about the central plane):
 *   edges_dev: float64 [n_edges] ascending edge positions in grid units
 *     along the periodic axis (node j stands for the cell [j-1/2, j+1/2));
 *     ridges are consecutive pairs (x1, x2), (x3, x4), ...  With mirror = 1
 *     these are the first half period's edges and the period continues with
 *     nx - x_n, ..., nx - x_1 (the reflection about x = nx/2).
 *   eps_dev: float64 [ny][nx]; only the design rows are written: every design
 *     row of column j gets eps_gap + (eps_ridge - eps_gap) * (fraction of
 *     cell j covered by ridges, periodic images included).
 * Ridges are assumed disjoint (overlaps add up); edges outside the period
 * wrap.  APF_EINVAL for a null pointer, mirror not 0/1, n_edges <= 0 or an
 * odd number of edges in the period. */
apf_status apf_ridges_eps(apf_handle *h, const double *edges_dev, int32_t n_edges,
                          int32_t mirror, double eps_ridge, double eps_gap,
                          double *eps_dev, void *stream);

/* Chain rule from the permittivity gradient to the edge positions (Sec. 2:
 * dA/dp_k touches only the pixels p_k modifies): with the covered fraction
 * of the cell holding an edge changing by -1 (left edge) or +1 (right edge)
 * per unit move, and an image edge nx - x moving by -1,
 *   grad_edges[k] = sum over design rows of grad_eps at the cells of edge k
 *                   (and of its image) times -/+(eps_ridge - eps_gap).
 *   grad_eps_dev: float64 [design_row1 - design_row0][nx] (as from apf_grad);
 *   grad_edges_dev: float64 [n_edges].  Same arguments and errors as
 *   apf_ridges_eps. */
apf_status apf_ridges_grad(apf_handle *h, const double *edges_dev, int32_t n_edges,
                           int32_t mirror, double eps_ridge, double eps_gap,
                           const double *grad_eps_dev, double *grad_edges_dev,
                           void *stream);

/* The weighted adjoint source C^T dF/dS of the sweep fronts is one dense
 * product unless dF/dS has at most 32 nonzeros in every input column (and at
 * most n_out / 8): then (an objective over a few target outputs per input)
 * it is formed from compact per-column lists, the same sum without its zero
 * terms.  Telling the two apart reads the column counts back, so apf_grad
 * synchronises `stream` once before the sweeps.
 * (APF_MIXED_REFINED: the adjoint fields are refined like the forward ones,
 * the call synchronises `stream` at its end to check the residuals and
 * returns APF_ENOTCONV when they miss the tolerance; grad_dev then holds the
 * gradient of the last iterate.)
 * Gradient of a real objective f(S) with respect to the permittivity of every
 * design pixel (Sec. 2, Eq. (1) with dS/deps_k of Eq. (3), U_k = e_k and
 * Sigma_k = dA_kk/deps_k = -h^2):
 *   df/deps_k = sum_nm 2 Re(dF/dS_nm dS_nm/deps_k)
 *             = 2 h^2 Re sum_m Lam_km Y_km,
 *   Y = A^-1 B, Lam = A^-1 (C^T dF/dS)  (the M_in weighted adjoint problems).
 *   dfdS_dev: complex128 [n_out][n_in], the Wirtinger derivative dF/dS.
 *   grad_dev: float64 [design_row1 - design_row0][nx] (overwritten).
 * Uses the factors of the last apf_factor_schur (else APF_ESTATE). */
apf_status apf_grad(apf_handle *h, const double *dfdS_dev, double *grad_dev,
                    void *stream);

/* Flags of the parameter-augmented gradient. */
#define APF_AUG_SKIP_UU 1   /* do not form the U(n)^T A^-1 U(n) block of S~(n) */

/* Gradient with respect to general design parameters p_k by the
 * parameter-augmented partial factorization (Sec. 2, Eq. (4), with the matrix
 * division into N_sub sub-factorizations of Fig. 1d): dA/dp_k = U_k Sigma_k
 * U_k^T (Eq. (2)) with U_k the unit vectors of the design pixels p_k changes
 * and Sigma_k the corresponding diagonal entries of dA/dp_k.  The columns of
 * U = [U_1, ..., U_Np] are divided into n_sub groups of whole parameters;
 * sub-factorization n eliminates the grid unknowns of
 *   K~(n) = [A, [B, U(n)]; [C; U(n)^T], 0]
 * and yields C A^-1 U(n), U(n)^T A^-1 B and (unless APF_AUG_SKIP_UU)
 * U(n)^T A^-1 U(n); Eq. (3) is applied to each sub's blocks, unmerged:
 *   df/dp_k = -2 Re sum_{c in k} Sigma_c sum_nm (C A^-1 U)_nc dF/dS_nm (U^T A^-1 B)_cm.
 *   n_cols, col_pixel, col_sigma (host): the columns of U, each the design
 *     pixel (row-major index over the design rows) and its Sigma entry;
 *   n_params, param_begin (host, n_params + 1 entries, non-decreasing from 0
 *     to n_cols): the columns of parameter k are [param_begin[k],
 *     param_begin[k + 1]);
 *   n_sub: the number of sub-factorizations (>= 1), or 0 for the smallest
 *     one whose S~(n) has at most 5 nnz(A) entries (clamped to [1, n_params]);
 *     *n_sub_used (may be NULL) receives the number run;
 *   dfdS_dev: complex128 [n_out][n_in], dF/dS (from an earlier apf_factor_schur
 *     with the same permittivity); S_dev: NULL, or complex128 [n_out][n_in]
 *     receiving the first sub-factorization's C A^-1 B; dfdp_dev: float64
 *     [n_params].
 * FP64.  Requires apf_assemble; every sub-factorization refactors A, and the
 * handle then holds FP64 factors of the assembled permittivity (apf_grad may
 * follow).  Synchronises `stream`.  APF_EINVAL for bad arguments (a pixel
 * outside the design rows, a decreasing param_begin), plus the errors of
 * apf_factor_schur. */
apf_status apf_grad_augmented(apf_handle *h, int32_t n_cols, const int32_t *col_pixel,
                              const double *col_sigma, int32_t n_params, const int32_t *param_begin,
                              int32_t n_sub, int32_t flags, const double *dfdS_dev, double *S_dev,
                              double *dfdp_dev, int32_t *n_sub_used, void *stream);

/* apf_grad_augmented for the ridge parameterization of apf_ridges_eps: the
 * parameters are the n_edges free edge positions; U_k holds the pixels of
 * the cell holding edge k on every design row (and, with mirror = 1, those of
 * the cell holding its image), Sigma_k = -h^2 deps/dx_k with deps/dx_k =
 * -/+(eps_ridge - eps_gap) for a left / right edge and the opposite sign for
 * the image (which moves by -1); r_k = 2 x design rows with mirror symmetry.
 * The edges are read back from the device (the call synchronises `stream`).
 * Same arguments and errors as apf_ridges_grad and apf_grad_augmented. */
apf_status apf_ridges_grad_augmented(apf_handle *h, const double *edges_dev, int32_t n_edges,
                                     int32_t mirror, double eps_ridge, double eps_gap, int32_t n_sub,
                                     int32_t flags, const double *dfdS_dev, double *S_dev,
                                     double *dfdp_dev, int32_t *n_sub_used, void *stream);

/* Autotuner of the GEMM kernel form.  Every GEMM task list of a plan runs
 * in one of three forms: 0 the four-product complex kernel at four
 * workgroups per CU, 1 the three-product (Karatsuba) form on the deep-K
 * kernel at three workgroups per CU, 2 the four-product form on the deep-K
 * kernel (the occupancy variant).  The tile is fixed at 64 x 64 (2 x 2 MFMA
 * blocks of 16 x 16 per wave, four waves).  apf_autotune times every list in
 * every form with HIP events over `reps` runs of the work the plan does --
 * for n = 1 apf_factor_schur (FP64) and apf_grad of hs[0], for n > 1 the
 * batched factorization of hs[0..n) -- groups the lists into buckets (mean k
 * extent of a tile, log2; number of tiles, log2), picks the fastest form per
 * bucket, applies it and, if save_path is not NULL, writes the table as text.
 * apf_tuning_apply reads such a table and applies it to the same kind of
 * plan without timing (buckets missing from the table keep their form).
 * Both synchronise `stream` and reset the handle's profiling counters; the
 * timing runs overwrite the factors (assemble again before the next
 * apf_factor_schur if the permittivity changed).  A form changes only
 * rounding (the three-product form rounds differently from the others), so
 * after a batched autotune the batched and single factorizations agree to
 * rounding, not bit for bit.  Requires apf_assemble on every handle
 * (APF_ESTATE); APF_EINVAL for reps outside [1, 100] or an unreadable
 * table. */
apf_status apf_autotune(apf_handle *const *hs, int32_t n, int32_t reps, const char *save_path, void *stream);
apf_status apf_tuning_apply(apf_handle *const *hs, int32_t n, const char *path, void *stream);

/* Cap the right-hand-side chunk of the gradient sweeps (0: the default, as
 * many columns as three quarters of the free device memory hold).  The
 * sweep arrays X and V hold one row per sweep pivot and `chunk` columns each;
 * apf_grad runs the sweeps once per chunk of inputs.  For callers that must bound the
 * memory the handle takes.  Call before the first apf_assemble (else
 * APF_ESTATE); APF_EINVAL unless max_chunk is 0 or a positive multiple of 64. */
apf_status apf_set_rhs_chunk(apf_handle *h, int32_t max_chunk);

/* B/C compression (Supplement Sec. 1; this library's reading of its
 * one-sentence recipe).  The input orders a_lo..a_hi and the output orders
 * (each set consecutive) are extended by `pad` orders (pad / 2 below),
 * M' = M + pad, with window weights w_t = sin^2(pi (t + 1/2) / M'); the
 * compressed source column j on the source row is
 *   b_j(x) = sum_t w_t phi_{a'_t}(x) exp(-2 pi i t j / M'),
 * localized around x_j = j nx / M' and truncated to the nodes within half of
 * `window_wavelengths` (periodic distance), and the compressed projection rows
 * c_j are the conjugate construction on the projection row.  The
 * factorization then carries, per front, only the compressed columns whose
 * window meets its region, forms S~ = C~ A^-1 B~ (M'_C x M'_B) block by block
 * and returns S = D_C S~ D_B, the exact S of the original channels when
 * nothing is truncated and an approximation otherwise (about 1e-3 .. 1e-2 at
 * a 3-wavelength window and pad = M / 5, less for wider windows; see the
 * design notes).  apf_grad then runs Eq. (3) over the compressed channels:
 * dF/dS~ = D_C^T dF/dS D_B^T, forward fields A^-1 B~ and weighted adjoint
 * fields A^-1 C~^T dF/dS~ over the M'_B compressed columns (the exact
 * gradient of the decompressed S).  The augmented and batched entry points
 * refuse compressed handles (APF_EINVAL).  pad = -1 switches compression off
 * again.
 * Call after apf_analyze and before the first apf_assemble (else
 * APF_ESTATE); APF_EINVAL for non-consecutive orders, pad < -1, a window that
 * is not positive or narrower than the spacing nx / M' of the columns. */
apf_status apf_set_compression(apf_handle *h, int32_t pad, double window_wavelengths);

/* Whether the plan prepares the gradient sweeps (on = 1, the default) or
 * only S (on = 0): without them the factorization skips the products that
 * only the sweeps read (X12 = U^-1 U12, Z = L21 L^-1, X1B and XC1 of the
 * fronts the sweeps visit) and the handle allocates no sweep arrays;
 * apf_grad then returns APF_ESTATE, except after an APF_MIXED_REFINED
 * factorization (the refined gradient solves for the fields itself).  Call after apf_analyze and before the
 * first apf_assemble (else APF_ESTATE); APF_EINVAL unless on is 0 or 1. */
apf_status apf_set_gradient(apf_handle *h, int32_t on);

/* Enable (max_iter >= 1) or disable (0, the default) APF_MIXED_REFINED on
 * this handle: the plan then keeps the triangular inverses, L21 and
 * X12 = U^-1 U12 of every front (not only of the fronts the gradient sweeps
 * visit), two N x rc field arrays, the forward fields of the design pixels
 * (design pixels x n_in) and the channel rows of B and C; rc, the
 * refinement's right-hand-side chunk, comes from the free memory and the cap
 * of apf_set_rhs_chunk.  A refined call runs the first solve and max_iter
 * corrections per chunk and returns APF_ENOTCONV when the final residual
 * |r - A x| / |r| of some chunk exceeds tol (0 < tol < 1); the fields are then
 * the last iterate.  Call before the first apf_assemble (else APF_ESTATE);
 * APF_EINVAL for max_iter outside [0, 16] or a bad tol. */
apf_status apf_set_refinement(apf_handle *h, int32_t max_iter, double tol);

/* Symmetric route (on = 1; 0, the default, is the LU route).  The operator is
 * complex symmetric, A = A^T (Sec. 2), and the Supplement (Sec. 1) obtains
 * S from a symmetric factorization of K; this library factors each front's
 * pivot block as F11 = L D L^T (no row exchanges inside the block: U = D L^T,
 * the identity permutation) and uses the symmetry in the products: U12 =
 * L^-1 F12 = D L21^T and the sweeps' Z = L21 L^-1 = X12^T are transposes
 * instead of products, and the contribution block F22 - L21 U12, symmetric,
 * is formed on its lower 64 x 64 tiles only (the lower triangle of each
 * front's core is maintained; its upper triangle is not read).  The channel
 * panels B and C are carried apart as on the LU route, so K itself need not
 * be symmetric (one-sided channels serve).  Without row exchanges a pivot
 * block can meet a nearly vanishing diagonal pivot that partial pivoting
 * avoids, and digits are lost (on a 48000 x 160 grid with 4,559 channels:
 * S 1.0e-10 from the FP64 reference against 3.0e-13 on the LU route, the
 * smallest pivot spread 5.0e-10 against 5.3e-4): check "pivot_spread_min"
 * after a factorization.  FP64 only: apf_factor_schur
 * returns APF_EINVAL for the other precisions (with FP32 products the
 * unpivoted blocks amplify the rounding: S 3.8e-5 and gradient 1.5e-4 from
 * the FP64 values at 240 x 92, against 1.2e-6 and 8.4e-6 on the LU route);
 * APF_EINVAL with compressed channels or refinement (set either way round),
 * and from apf_factor_schur_batched, apf_autotune over several handles and
 * the augmented entry points.  Call before the first apf_assemble (else APF_ESTATE);
 * APF_EINVAL unless on is 0 or 1. */
apf_status apf_set_symmetric(apf_handle *h, int32_t on);

/* Depth of the low-rank sweep subtrees: channel-free sweep subtrees of up to
 * `levels` levels (0, 1 or 2) whose gradient comes from the b x b product
 * Wt = Y_bnd Lam_bnd^T of their root instead of the Y and Lam sweeps (the same
 * quantity, Eqs. (1)-(3), in another order of operations; cheaper where
 * b^2 < 2 p b summed over the subtree).  With 0 every sweep front runs the
 * sweeps.  The dense propagation below a root multiplies the rounding error
 * of its fields by the cancellation of both field reconstructions, which
 * depends on dF/dS; the default depth is the library's default (see the
 * design notes of the release).  Call before the first apf_assemble (else
 * APF_ESTATE); APF_EINVAL for other values. */
apf_status apf_set_lowrank(apf_handle *h, int32_t levels);

/* Per-class HIP-event timing of the handle's launches (counters reset):
 * on = 0 off, 1 every launch, 2 only the GEMM-family launches (classes
 * gemm_factor, gemm_schur, gemm_sweep; half the events of mode 1, for timed
 * runs that need only the GEMM figures).  When on, each call waits for its
 * own events at its end, so calls become synchronous.  APF_EINVAL for any
 * other value. */
apf_status apf_set_profiling(apf_handle *h, int32_t on);

/* Free the handle, its symbolic data, factors and device buffers.  Waits for
 * nothing: the caller must have synchronised the streams it used. */
apf_status apf_destroy(apf_handle *h);

/* Kernel test hook (for the kernel unit tests, not for applications): one
 * complex GEMM C = Cin +/- op(A) op(B) in the library's internal task format,
 * cut into 64 x 64 tiles and run on one kernel form (0 four-product FP64,
 * 1 three-product FP64, 2 four-product FP64 on the deep-K kernel, 3 FP32
 * MFMA, 4 four-product FP64 with the tiles of at most 32 valid rows on the
 * thin kernels, as the factorization and sweep lists run, 5 the same on
 * FP32 MFMA), so that its
 * operand layouts, triangular masks, row and column maps, Cin forms, edges
 * and k stages can be checked against a plain reference.
 * flags: the internal task flags of the tested set (transposed A, negation,
 * Cin and its column offset / own indexing / column range, external B with
 * element offset b_offset, triangular A or B, accumulation into C, k limited
 * to nlim); other flags give APF_EINVAL.  All pointers are device pointers
 * to complex128 (A, B, Cin, C) or int32 maps (browmap, crowmap, ccolmap,
 * each may be NULL); coff and nlim are the launch's column offset and
 * column (or k) limit; xcd = 1 orders the tiles for the eight XCDs.
 * The contraction flag (G_CONTRACT, 2048; with G_NO_STORE, 4096, C itself is
 * not written) also forms the gradient partials of the sweeps: for output
 * row i (C row oi through crowmap) and each 32-column group g of the tile
 * columns, part[((coff + 32 g) / 32) * pstride + auxmap[oi]] =
 * sum over the group's columns j of Re(C(i, j) aux[oi * ldc + j]), written
 * where auxmap[oi] >= 0 (aux: device complex128 rows of stride ldc; auxmap:
 * device int32; part: device float64; coff a multiple of 32); pass NULL and
 * 0 otherwise.  Allocates and synchronises `stream`. */
apf_status apf_test_gemm(int32_t form, int32_t flags, int32_t M, int32_t N, int32_t K,
                         const double *A, int32_t lda, const double *B, int32_t ldb, int64_t b_offset,
                         const double *Cin, int32_t ldcin, double *C, int32_t ldc,
                         const int32_t *browmap, const int32_t *crowmap, const int32_t *ccolmap,
                         int32_t cin_c0, int32_t cin_w, int32_t coff, int32_t nlim, int32_t xcd,
                         const double *aux, const int32_t *auxmap, double *part, int32_t pstride,
                         void *stream);

/* Kernel test hook (for the kernel unit tests, not for applications): the
 * pivot-block kernel on one p x p block F (device, complex128 row-major,
 * 1 <= p <= 128; read only): LU with partial pivoting inside the block
 * (largest modulus, ties to the lowest row), then the in-place inverses;
 * with sym = 1 the kernel's symmetric mode (apf_set_symmetric): only the
 * lower triangle of F is read (the block taken as symmetric) and step k
 * pivots on row k, so perm is the identity and U = D L^T.
 * tri_dev (device, complex128 p x p) receives L^-1 below the diagonal (unit
 * diagonal implied) and U^-1 on and above it, perm_dev (device, int32 p) the
 * row of F taken at each step, so that U^-1 L^-1 F[perm] = I; *spread (host,
 * may be NULL) the pivot spread min |u_kk| / max |u_kk|.  APF_ESINGULAR when
 * a pivot was zero or non-finite (the outputs are then undefined); the
 * kernel runs to its end either way.  Allocates and synchronises `stream`. */
apf_status apf_test_pivot_block(int32_t p, const double *F_dev, double *tri_dev, int32_t *perm_dev,
                                double *spread, int32_t sym, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *apf_last_error(void);

/* Read a named statistic of an analysed handle (host only):
 *   "refine_chunk" (right-hand-side chunk of the refined solves, -1 before
 *   the plan), "refine_residual" and "refine_residual_first" (largest final
 *   and first-solve relative residual over the chunks of the last refined
 *   call), "retained_factor_bytes" (factors kept for the refinement),
 *   "n_fronts", "n_levels", "max_front" (largest p+b), "n_factorizations"
 *   (factorizations run on the handle so far, failed ones included: a caller
 *   that keeps the factors for a later apf_grad can tell whether they were
 *   replaced meanwhile), "factor_cmacs" and
 *   "grad_cmacs" (complex multiply-adds the factorization and the gradient
 *   perform), "algo_factor_cmacs" (sum over fronts of the rank-p updates of
 *   the rectangular front, channel block included), "ws_bytes" (workspace
 *   peak), "factor_bytes", "schur_store_bytes", "n_sweep_rows",
 *   "n_sweep_fronts", "k_total";
 *   after the first apf_assemble: "rhs_chunk", "gemm_cmacs_factor",
 *   "gemm_cmacs_schur", "gemm_cmacs_sweep" (complex multiply-adds of the
 *   GEMM tasks of one call whose operands are structurally nonzero: the
 *   stored triangle of a triangular factor, no tile padding),
 *   "gemm_cmacs_k3" (the part of those three that the FP64 path runs in the
 *   three-product complex form, 6 real flops per complex multiply-add
 *   instead of 8), "gemm_cmacs_lowrank_w" (the part run by the low-rank W
 *   kernel, three-product on both paths),
 *   "gemm_cmacs_vinit" (the dense weighted-adjoint-source product's part of
 *   gemm_cmacs_sweep), "adjoint_source_sparse_k" (0 if the last apf_grad ran
 *   that dense product, else the width of the compact column lists of a
 *   dF/dS with at most 32 nonzeros per input column, at most n_out / 8),
 *   "lowrank_fronts" and "lowrank_roots" (sweep fronts served by the
 *   low-rank subtree products, and the subtrees' roots);
 *   after a successful apf_factor_schur (else APF_ESTATE; copies from the
 *   device): "pivot_spread_min" (the smallest, over the fronts, of the pivot
 *   block's min |u_kk| / max |u_kk|: a pivot block close to singular, e.g.
 *   near a resonance of the subdomain it eliminates, shows as a small value)
 *   and "pivot_spread_front" (the front it belongs to);
 *   with profiling on: "ms_<class>" and "launches_<class>", the summed
 *   HIP-event time and launch count since profiling was enabled, for the
 *   classes stencil, zero, assemble, inverse, gemm_factor, gemm_schur,
 *   gemm_sweep, contract, wpow, refine (APF_MIXED_REFINED's solves and
 *   residuals), adjoint_source (the sparse weighted adjoint source); the
 *   children's contribution blocks are added into their parents by the
 *   gemm_factor launches. */
apf_status apf_query(apf_handle *h, const char *key, double *value);

/* Structure export for host-side validation (host only, after apf_analyze).
 *   info[8]: parent (-1 for the root), height, p (pivots), b (boundary
 *   size), has_B, has_C, in_sweep, first elimination index.
 *   pivots (p entries) and boundary (b entries) receive node indices
 *   j*nx+i; either may be NULL. */
apf_status apf_front(apf_handle *h, int32_t f, int32_t info[8],
                     int32_t *pivots, int32_t *boundary);

#ifdef __cplusplus
}
#endif

#endif /* APF_H */
