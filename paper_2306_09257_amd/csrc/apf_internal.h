// Internal structures shared by the host analysis, the device plan and the
// kernels of the APF library.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/apf.h"

namespace apf {

// complex128 as two doubles (the device code uses double2 with the same layout)
struct cplx { double re, im; };

// ---------------------------------------------------------------------------
// Symbolic data (host)
// ---------------------------------------------------------------------------
struct Front {
  int parent = -1;
  int height = 0;
  int child[2] = {-1, -1};
  int nchild = 0;
  int x0 = 0, x1 = 0, y0 = 0, y1 = 0;   // region of the subtree (x periodic)
  std::vector<int> piv;                 // pivot nodes, elimination order
  std::vector<int> bnd;                 // boundary nodes, sorted by elimination index
  std::vector<int> rmap;                // boundary -> parent-local index (0..p+b of the parent)
  bool hasB = false, hasC = false, sweep = false, sfront = false;
  int64_t elim0 = 0;                    // elimination index of piv[0]
  int p() const { return (int)piv.size(); }
  int b() const { return (int)bnd.size(); }
};

struct Symbolic {
  int nx = 0, ny = 0;
  std::vector<Front> fronts;            // postorder: children before parents; root last
  std::vector<int> node_front;          // node -> front owning it as a pivot
  std::vector<int> node_local;          // node -> index among that front's pivots
  std::vector<int64_t> node_elim;       // node -> elimination index
  std::vector<std::vector<int>> levels; // fronts by height
  int64_t n_sweep_rows = 0;
  std::vector<int64_t> node_sweep_row;  // -1 if the node's front is not in the sweep set
  int64_t k_total = 0;                  // sum of p over S-fronts (has_B and has_C)
  double algo_factor_cmacs = 0, factor_cmacs = 0, grad_cmacs = 0;
  int max_front = 0;
};

struct Desc {
  int nx, ny;
  double dx_over_lambda;
  int npml_top, npml_bot;
  double pml_R0;
  int pml_power;
  double eps_top, eps_bot;
  int src_row, prj_row, design_row0, design_row1;
  int n_in, n_out;
  std::vector<int> in_orders, out_orders;
  int leaf_size;
};

// Builds the nested-dissection tree and every index set of the symbolic
// factorization.  Throws std::runtime_error on an invalid grid.
void analyze(const Desc &d, Symbolic &sym);

// ---------------------------------------------------------------------------
// Device plan structures (POD, copied to the GPU)
// ---------------------------------------------------------------------------
struct FrontDev {
  int32_t p, b, mB, mC;
  int32_t sweep_row0;      // row of the first pivot in the X/V sweep arrays, -1 if none
  int32_t pad;
  cplx *core;              // (p+b) x (p+b) row-major frontal core
  cplx *bp_piv, *bp_bnd;   // B-panel rows: p x mB and b x mB (ld mB)
  cplx *cpt_piv, *cpt_bnd; // C-panel transposed rows: p x mC and b x mC (ld mC)
  const int32_t *rmap;     // b entries: boundary -> parent-local index
  cplx *tri;               // p x p: strict lower = L^-1 (unit diagonal implied), upper = U^-1
  int32_t *perm;           // p entries: perm[k] = pivot-local row of elimination step k
  int32_t parent;
  int32_t pad2;
};

// Physical parameters the assembly kernels evaluate the operator from.
struct Phys {
  int nx, ny;
  double h2;                    // (k0 dx)^2
  int npml_top, npml_bot, pml_power;
  double alpha_top, alpha_bot;  // PML stretch amplitudes
  double eps_src, eps_prj;      // media of the source and projection rows
};

// Channel set of one panel (device memory): the source row's inputs or the
// projection row's outputs of one problem.
struct ChanParams {
  Phys P;
  const int32_t *orders;
  double *amp;             // per order: sqrt(sin q / nx) in the panel's medium (filled on the device)
  int32_t m, is_source;
};

// Row maps of the channel-panel updates that a child writes straight into
// its parent's panel: entry = parent-local row, | EXT_ADD when an earlier
// writer has stored that row already (the update adds instead of storing).
constexpr int32_t EXT_ADD = 1 << 30;
constexpr int32_t EXT_ROW_MASK = EXT_ADD - 1;

struct AsmEntry {          // one stencil entry of A: *src is added at dest
  const cplx *src;         // Aval + node*5 + direction (0 centre, 1 x-1, 2 x+1, 3 y-1, 4 y+1)
  cplx *dest;
};

struct PanelEntry {        // one source (B) or projection (C) node: a whole row of the panel, stored
  int32_t node, pad;
  cplx *dest;
  const ChanParams *cp;
};

enum GemmFlags : int32_t {
  G_TRANS_A = 1,           // A(i,k) = A[k*lda + i]
  G_NEG = 2,               // C = Cin - A*B  (else Cin + A*B)
  G_CIN = 4,               // Cin present (else treated as zero)
  G_B_COFF = 8,            // add the launch's column offset to B
  G_CIN_COFF = 16,         // add the launch's column offset to Cin
  G_B_EXT = 32,            // B is the launch's external pointer (caller buffer) plus the element
                           // offset held in the B field (a plain number, not an address)
  G_C_EXT = 64,            // C is the launch's external pointer (caller buffer)
  // triangular operands stored packed in one square array (masks apply to the
  // stored indices (r, c); zero blocks of K are skipped):
  G_A_TRI_L = 128,         // stored A: r > c entries, unit diagonal, zero above
  G_A_TRI_U = 256,         // stored A: r <= c entries, zero below
  G_B_TRI_L = 512,         // stored B: r > c entries, unit diagonal, zero above
  G_B_TRI_U = 1024,        // stored B: r <= c entries, zero below
  // gradient contraction in the epilogue: for every output row i with
  // auxmap[i] >= 0, the partial sum of Re(C(i,j) aux(i,j)) over the 32
  // columns of one wave goes to part[auxmap[i] * nblk + column / 32]
  // (aux has the layout of C)
  G_CONTRACT = 2048,
  G_NO_STORE = 4096,       // C itself is not written (only the contraction)
  G_CIN_OWN = 8192,        // Cin entry (i, j) is Cin[i*ldcin + j] (not mapped by crowmap / ccolmap)
  G_C_ACC = 16384,         // C's old value is added to every entry (as EXT_ADD for all rows)
  G_TRANS_B = 32768,       // B(k, j) = B[j*ldb + k]; browmap then maps j (low-rank W tasks only)
  G_K_LIM = 65536,         // K is limited to the launch's column limit (a right-hand-side chunk)
  G_ACC_CHUNK = 131072,    // C's old value is added when the launch's column offset is > 0
  G_K3 = 262144,           // complex products in the three-product form (launched on the deep-K kernel)
  G_C_COFF = 524288,       // add the launch's column offset to C
  // Cin covers only the global columns [cin_c0, cin_c0 + cin_w) of the
  // launch (column coff + j of the launch is Cin column coff + j - cin_c0;
  // zero outside): a compressed channel panel of one front
  G_CIN_RANGE = 1048576,
};

struct GemmTask {          // one 64 x 64 output tile of C = Cin +/- op(A) B (a 32 x 32 quadrant for W tasks)
  const cplx *A;
  const cplx *B;
  const cplx *Cin;
  cplx *C;
  const int32_t *browmap;  // if set, row k of B is B + browmap[k]*ldb
  const int32_t *crowmap;  // if set, row i of C (and of Cin) is C + (crowmap[i] & EXT_ROW_MASK)*ldc,
                           // and C's old value is added when crowmap[i] & EXT_ADD
  int32_t M, N, K;
  int32_t lda, ldb, ldcin, ldc;
  int32_t flags;
  int32_t tm, tn;
  const cplx *aux;         // G_CONTRACT: the second factor of the contraction
  const int32_t *auxmap;   // G_CONTRACT: row -> contraction slot, or -1
  const int32_t *ccolmap;  // if set, column j of C is column ccolmap[j]
  const int32_t *arowmap;  // W tasks: row i of A is A + arowmap[i]*lda
  int32_t cin_c0, cin_w;   // G_CIN_RANGE: the global columns Cin holds
};

// Tiles that the thin GEMM kernel takes: at most THIN_ROWS valid rows (the
// small separator fronts near the leaves, the leaves' products with at most
// 32 output rows, ragged last row tiles); the plan moves them to the end of
// the factorization and sweep lists.
constexpr int THIN_ROWS = 32;
inline bool thin_tile_task(const GemmTask &T) {
  return T.M > 0 && T.N > 0 && T.M - T.tm <= THIN_ROWS && !(T.flags & G_TRANS_B);
}
inline bool tri_task(const GemmTask &T) { return T.flags & (G_A_TRI_L | G_A_TRI_U | G_B_TRI_L | G_B_TRI_U); }

struct ZeroRange { cplx *ptr; int64_t n; };
struct CopyRange { const cplx *src; cplx *dst; int64_t n; };   // n contiguous complex entries
// dst (rows x cols) = src^T, dst row r scaled by 1 / diag[r * ldiag + r] when
// diag is not null (the symmetric route's U12 = D L21^T and Z = X12^T)
struct TransTask {
  const cplx *src;
  cplx *dst;
  const cplx *diag;
  int32_t lds, ldd, ldiag, rows, cols, pad;
};

// A front of a low-rank sweep subtree.  A sweep front whose subtree holds no
// channel rows has Y_piv = -X12 Y_bnd and Lam_piv[perm[k]] = -(Z^T Lam_bnd)[k]
// (no source terms), so every product of its fields over the right-hand-side
// columns follows from the b x b matrix Wt = Y_bnd Lam_bnd^T: with
// U1t = Wt Z and Qt = X12 [U1t | Wt], the matrix Rt = Y Lam^T over the
// front's rows (pivots, then boundary) is
//   Rt[j][perm[k]] = Qt[j][k],      Rt[j][p + a] = -Qt[j][p + a],
//   Rt[p + c][perm[k]] = -U1t[c][k], Rt[p + c][p + a] = Wt[c][a].
// Its diagonal at the pivots gives the gradient of the front's pixels, and
// each child's Wt is Rt restricted to the child's boundary (through the
// child's row map).  Only the subtree's root forms Wt from the sweep fields.
struct WFront {
  const cplx *Qt;         // p x (p + b)
  const cplx *Bf;         // b x (p + b): [U1t | Wt]
  const int32_t *perm;    // p pivot rows in step order
  const int32_t *gidx;    // p design-pixel indices (by pivot), or -1
  int32_t p, b;
  int32_t nch;            // children in low-rank subtrees (0..2)
  int32_t pc[2], bc[2];   // their pivot and boundary counts
  cplx *dst[2];           // their Wt (b_c x b_c, ld p_c + b_c)
  const int32_t *rmap[2]; // their boundary -> this front's local row
};

constexpr int GEMM_TILE = 64;

// Largest pivot block of one front.  The nested dissection splits longer
// separators into chains of fronts; the pivot-block kernels, the low-rank
// subtree gather and the plan builder are all sized by this one constant.
constexpr int MAX_PIVOTS = 128;

// Bits of the device status word a factorization reports through.
constexpr int ST_SINGULAR = 1;   // a pivot block met a zero or non-finite pivot
constexpr int ST_BAD_EPS = 2;    // the assembled permittivity had a zero or non-finite value

}  // namespace apf
