// Launchers of the APF HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "apf_internal.h"

namespace apf {

hipError_t launch_zero(const ZeroRange *r, int n, hipStream_t s);
// status: ST_BAD_EPS is or-ed in for a zero or non-finite permittivity
hipError_t launch_stencil(const Phys &P, const double *eps, cplx *Aval, int *status, hipStream_t s);
hipError_t launch_scatter_A(const AsmEntry *e, int n, hipStream_t s);
hipError_t launch_assemble_panel(const PanelEntry *e, int n, hipStream_t s);
hipError_t launch_fill_int(int *p, int v, hipStream_t s);
constexpr int N_INV_VARIANTS = 6;
// kernel variant of a pivot block of size p (1 <= p <= MAX_PIVOTS), -1 beyond
int inverse_variant(int p);
// pivq (may be null): per front index, the block's pivot spread min |u_kk| / max |u_kk|;
// sym != 0: symmetric blocks, lower triangle read, no row exchanges (F11 = L D L^T)
hipError_t launch_inverse(int variant, const FrontDev *fr, const int32_t *ids, int n, int *status, double *pivq,
                          int sym, hipStream_t s);
// dst = src^T per task, rows scaled by the inverse of diag's diagonal when given
hipError_t launch_transpose_scale(const TransTask *t, int n, hipStream_t s);
// part / pstride: output of the tasks flagged G_CONTRACT, partial of design
// slot g and 32-column block b at part[b * pstride + g] (unused otherwise);
// deep: MFMA-bound deep-K task list (three-product complex form on FP64);
// nthin: the last nthin tasks are thin tiles (thin_tile_task), run by the
// thin kernels (FP64 or FP32 like the rest); the last nthin_tri of them have
// a triangular operand
hipError_t launch_gemm(const GemmTask *t, int n, int coff, int nlim, const cplx *ext, hipStream_t s,
                       bool f32 = false, double *part = nullptr, int pstride = 0, bool deep = false,
                       int nthin = 0, int nthin_tri = 0);
// kernel launches that launch_gemm makes for such a list
int gemm_kernel_launches(int n, int nthin, int nthin_tri, bool f32);
// Wt = Y_bnd Lam_bnd^T of the low-rank subtree roots: one task (b <= 64) per
// root, one workgroup per task; nlim: the chunk's width (k extent)
hipError_t launch_lowrank_w(const GemmTask *t, int n, int coff, int nlim, hipStream_t s);
// one workgroup per front of a low-rank sweep subtree (gradient + children's Wt)
hipError_t launch_wprop(const WFront *f, int n, double scale, double *grad, hipStream_t s);
hipError_t launch_row_map(int32_t *map, const int32_t *base, const int32_t *pidx, const int32_t *perm, int64_t n,
                          hipStream_t s);
hipError_t launch_sum_partials(const cplx *part, int nseg, int64_t stride, cplx *S, int64_t n, hipStream_t s);
hipError_t launch_reduce_partials(const double *part, int nblk, int64_t n, double scale, double *grad,
                                  hipStream_t s);
hipError_t launch_weighted_power(const cplx *S, const double *w, double *f, cplx *G, int64_t n, double *part,
                                 int npart, hipStream_t s);
// block partials of the weighted-power reduction for n entries (<= 1024)
int weighted_power_parts(int64_t n);

// iterative refinement of the mixed path (see kernels.hip)
hipError_t launch_channel_matrices(const ChanParams *cp_src, const ChanParams *cp_prj, cplx *Bmat, cplx *Cmat,
                                   hipStream_t s);
hipError_t launch_residual(int nx, int ny, const int32_t *elim, const cplx *Aval, const cplx *X, cplx *W, int ld,
                           int w, int rrow, const cplx *rb, int ldr, int coff, bool first, double *norm2,
                           hipStream_t s);
hipError_t launch_add_fields(cplx *X, const cplx *W, int64_t rows, int ld, int w, bool first, hipStream_t s);
hipError_t launch_gather_rows(const int32_t *erow, int64_t n, const cplx *X, int ld, int w, cplx *Y, int64_t ldy,
                              int coff, hipStream_t s);
hipError_t launch_contract_rows(const int32_t *erow, int64_t n, const cplx *Lam, int ld, int w, const cplx *Y,
                                int64_t ldy, int coff, double scale, bool first, double *grad, hipStream_t s);
hipError_t launch_copy(const CopyRange *r, int n, hipStream_t s);
hipError_t launch_fill_double(double *p, int n, double v, hipStream_t s);

// parameter-augmented factorization (Eq. (4)): unit entries of U and U^T in
// the augmented panels; Eq. (3) summed per parameter
hipError_t launch_set_one(cplx *const *p, int n, hipStream_t s);
hipError_t launch_zero_flat(cplx *p, int64_t n, hipStream_t s);   // n contiguous complex zeros
// weighted adjoint source from a column-sparse dF/dS
hipError_t launch_col_nnz(const cplx *G, int n_out, int n_in, int *nnz, int *maxnnz, hipStream_t s);
hipError_t launch_col_compact(const cplx *G, int n_out, int n_in, int K, int32_t *idx, cplx *val, hipStream_t s);
// amp[] of both panels' channel parameters (cp[0], cp[1]: n = m0 + m1 orders)
hipError_t launch_channel_amp(const ChanParams *cp, int n, hipStream_t s);
hipError_t launch_sparse_vinit(const cplx *XC, int n_out, int64_t rows, const int32_t *vmap, const int32_t *idx,
                               const cplx *val, int K, int coff, int w, cplx *V, int ldv, hipStream_t s);
// compressed channel basis on one channel row (nx x Mx, zeroed beforehand)
hipError_t launch_compress_basis(int nx, int Mx, int a0, double half_px, bool conj_all, cplx *out, hipStream_t s);
// autotuner: set or clear G_K3 on n tasks
hipError_t launch_set_k3(GemmTask *t, int n, bool on, hipStream_t s);
hipError_t launch_param_sum(const int32_t *cbeg, int np, const double *sigma, const double *v, double *dfdp,
                            hipStream_t s);

// beam-splitter workload: Eq. (5) figure of merit, ridge permittivity and
// the chain rule to the edge positions (see include/apf.h)
hipError_t launch_splitter_fom(const cplx *S, const int32_t *in_ord, const int32_t *out_ord, int n_in, int n_out,
                               double t1, double *f, cplx *G, double *part, int npart, hipStream_t s);
hipError_t launch_group_fom(const cplx *S, const int32_t *in_ord, const int32_t *out_ord, int n_in, int n_out,
                            int delta, int gmax, double *f, cplx *G, double *part, hipStream_t s);
hipError_t launch_ridges_eps(const double *edges, int n, int mirror, int nx, int row0, int nrows, double eps_ridge,
                             double eps_gap, double *eps, hipStream_t s);
hipError_t launch_ridges_grad(const double *edges, int n, int mirror, int nx, int nrows, double eps_ridge,
                              double eps_gap, const double *grad_eps, double *grad_edges, hipStream_t s);

}  // namespace apf
