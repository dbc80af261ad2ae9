// C ABI of the APF library: descriptor validation, symbolic analysis, the
// device plan (buffers and per-level task arrays) and the per-call drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "apf_internal.h"
#include "kernels.h"

using namespace apf;

namespace {

thread_local std::string g_err;

apf_status fail(apf_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

}  // namespace

// the thread-local message, for entry points defined in other sources
void apf_set_error(const std::string &msg) { g_err = msg; }

namespace {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) throw HipError(std::string(#x) + ": " + hipGetErrorString(e_));            \
  } while (0)

constexpr int64_t ALIGN = 32;  // complex elements (512 bytes)
int64_t up(int64_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over one arena, for workspaces whose lifetimes are
// level intervals of the elimination tree.
struct Arena {
  std::map<int64_t, int64_t> free_;  // offset -> size
  int64_t top = 0;
  int64_t alloc(int64_t n) {
    n = up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        int64_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > n) free_[off + n] = sz - n;
        return off;
      }
    }
    int64_t off = top;
    top += n;
    return off;
  }
  void release(int64_t off, int64_t n) {
    n = up(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Host staging of a device blob of task arrays.
struct Blob {
  std::vector<char> h;
  int64_t add(const void *p, size_t bytes) {
    size_t off = (h.size() + 255) / 256 * 256;
    h.resize(off + bytes);
    if (bytes) std::memcpy(h.data() + off, p, bytes);
    return (int64_t)off;
  }
  template <class T>
  int64_t add(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

struct LevelTasks {
  // g2b: the phase-2 channel-panel updates of second children, which write
  // into the same parent rows as the first children's (g2) and run after them
  int64_t zero = -1, scat = -1, pan = -1, g1 = -1, g2 = -1, g2b = -1;
  int nzero = 0, nscat = 0, npan = 0, ng1 = 0, ng2 = 0, ng2b = 0;
  char deep1 = 0, deep2 = 0, deep2b = 0;   // lists run by the deep-K kernel (k_gemm_k3)
  int nthin1 = 0, nthin2 = 0, nthin2b = 0; // thin tiles at the end of each list (thin kernels)
  int ntri1 = 0, ntri2 = 0, ntri2b = 0;    // of which the last have a triangular operand
  // compressed channels: panel rows copied from the compressed basis, and
  // the blocks of S~ of the level's fronts, in launches whose blocks do not
  // overlap
  int64_t cpy = -1;
  int ncpy = 0;
  static constexpr int kSchurColors = 4;
  int64_t sch[kSchurColors] = {-1, -1, -1, -1};
  int nsch[kSchurColors] = {0, 0, 0, 0};
  int id1 = -1, id2 = -1, id2b = -1;       // the lists' entries in the plan's tunable-list table
  // symmetric route: U12 = D L21^T of the level's fronts, between phases 1 and 2
  int64_t utr = -1;
  int nutr = 0;
  int64_t inv[N_INV_VARIANTS];
  int ninv[N_INV_VARIANTS];
  LevelTasks() {
    for (int v = 0; v < N_INV_VARIANTS; ++v) { inv[v] = -1; ninv[v] = 0; }
  }
};

// Extra per-level work of one parameter-augmented sub-factorization (Eq. (4)
// with U divided into N_sub parts): zeroing and unit entries of the fronts'
// U / U^T panels at their panel level, then the panels' phase-1 and phase-2
// products (the latter with the blocks of S~ they add into).
struct AugLevel {
  int64_t zero = -1, one = -1, g1 = -1, g2 = -1;
  int nzero = 0, none = 0, ng1 = 0, ng2 = 0;
};

constexpr int64_t ZERO_CHUNK = 8192;   // complex elements per zeroing block
constexpr int64_t SPLIT_K = 4096;      // k rows per partial block of the split Schur product

// Per-class HIP-event timing of the launches (off unless enabled).
enum ProfClass { P_STENCIL, P_ZERO, P_ASSEMBLE, P_INVERSE, P_GEMM_FACTOR, P_GEMM_SCHUR, P_GEMM_SWEEP,
                 P_CONTRACT, P_WPOW, P_REFINE, P_VSRC, P_NCLASS };
const char *const kProfNames[P_NCLASS] = {"stencil", "zero", "assemble", "inverse", "gemm_factor",
                                          "gemm_schur", "gemm_sweep", "contract", "wpow", "refine",
                                          "adjoint_source"};
// A dF/dS with at most this many nonzeros in every input column (and at most
// an eighth of the outputs) takes the sparse weighted-adjoint-source kernel.
constexpr int kSparseG = 32;
// Levels of the low-rank sweep subtrees unless apf_set_lowrank says otherwise.
constexpr int kWMaxLevelsDefault = 1;

// A GEMM task list of a plan that the autotuner may run in another kernel
// form: 0 the four-product kernel at four workgroups per CU (k_gemm), 1 the
// three-product form on the deep-K kernel (three per CU), 2 the four-product
// form on the deep-K kernel.
struct TunableList {
  char *blob = nullptr;      // device blob holding the tasks
  int64_t off = -1;
  int n = 0;
  char *deep = nullptr;      // launch flag: 1 = the deep-K kernel
};

struct Profiler {
  bool on = false;
  int cur_tag = -1;          // tunable-list id of the launches that follow (-1: none)
  bool record = false;       // keep (tag, ms) of every timed launch in `trace`
  std::vector<std::pair<int, float>> trace;
  std::vector<int> tags;     // per mark
  std::vector<int> nkern;    // kernel launches per mark
  bool gemm_only = false;    // time only the GEMM-family launches
  static bool gemm_class(int cls) { return cls == P_GEMM_FACTOR || cls == P_GEMM_SCHUR || cls == P_GEMM_SWEEP; }
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, int>> marks;  // (class, index of the start event)
  double ms[P_NCLASS] = {0};
  int64_t count[P_NCLASS] = {0};
  size_t used = 0;
  hipEvent_t next() {
    if (used == pool.size()) {
      // timing only: no system-scope fence at each record (nothing on the
      // host reads device memory through these events)
      hipEvent_t e;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      pool.push_back(e);
    }
    return pool[used++];
  }
  // nk: kernel launches that fn makes (a GEMM list with thin tiles makes two)
  template <class Fn>
  void run(int cls, hipStream_t s, Fn &&fn, int nk = 1) {
    if (!on || (gemm_only && !gemm_class(cls))) {
      HIPCHK(fn());
      return;
    }
    size_t i0 = used;
    hipEvent_t a = next(), b = next();
    HIPCHK(hipEventRecord(a, s));
    HIPCHK(fn());
    HIPCHK(hipEventRecord(b, s));
    marks.push_back({cls, (int)i0});
    tags.push_back(cur_tag);
    nkern.push_back(nk);
  }
  void collect() {
    for (size_t i = 0; i < marks.size(); ++i) {
      const auto &m = marks[i];
      float t = 0.f;
      HIPCHK(hipEventSynchronize(pool[m.second + 1]));
      HIPCHK(hipEventElapsedTime(&t, pool[m.second], pool[m.second + 1]));
      ms[m.first] += t;
      count[m.first] += nkern[i];
      if (record) trace.push_back({tags[i], t});
    }
    marks.clear();
    tags.clear();
    nkern.clear();
    used = 0;
  }
  void reset() {
    for (int k = 0; k < P_NCLASS; ++k) { ms[k] = 0; count[k] = 0; }
    marks.clear();
    tags.clear();
    nkern.clear();
    trace.clear();
    used = 0;
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Iterative refinement of the mixed path (APF_MIXED_REFINED): a full solve
// with the factors of every front, level by level like the factorization's
// channel panels (forward: y1 = L^-1 P^T r1 and the children's updates
// r2 - L21 y1 written into the parent's front-local rows; backward:
// x1 = U^-1 y1 - X12 x2 in place, root to leaves), on right-hand-side chunks
// of rc columns held in elimination order.
struct RefineLevel {
  int64_t zero = -1, copy = -1, g1 = -1, g2 = -1, g2b = -1, bk = -1;
  int nzero = 0, ncopy = 0, ng1 = 0, ng2 = 0, ng2b = 0, nbk = 0;
};

struct Refine {
  int iters = 0;               // corrections after the first solve
  double tol = 0.0;            // bound on the final relative residual
  int rc = 0;                  // right-hand-side chunk (columns)
  int nchunks = 0;
  int64_t ss_elems = 0;
  cplx *ss = nullptr;          // retained factors of every front: tri, L21 and (non-sweep fronts) X12
  cplx *X = nullptr, *W = nullptr;      // N x rc: solution, residual / correction (elimination order)
  cplx *arena = nullptr;       // front-local right-hand-side panels and y1 blocks
  int64_t arena_elems = 0;
  cplx *Bmat = nullptr;        // nx x n_in: the source row of B
  cplx *Cmat = nullptr;        // n_out x nx: the projection row of C
  cplx *rowbuf = nullptr;      // nx x rc: C^T dF/dS of one chunk (the adjoint right-hand side)
  cplx *Ydes = nullptr;        // design pixels x n_in: refined forward fields, kept for the gradient
  int32_t *elim = nullptr;     // node -> elimination index
  double *norms = nullptr;     // per chunk: (iters + 2) squared residual norms
  char *blob = nullptr;
  std::vector<RefineLevel> lv;
  int64_t sgemm = -1, agemm = -1, erow_des = -1;
  int nsgemm = 0, nagemm = 0;
  double last_res = 0.0, last_res1 = 0.0;   // last call: final and first-solve relative residuals (max over chunks)
  template <class T>
  T *at(int64_t off) const { return off < 0 ? nullptr : reinterpret_cast<T *>(blob + off); }
};

struct Plan {
  int device = -1;
  Refine R;
  double gemm_cmacs_factor = 0, gemm_cmacs_schur = 0, gemm_cmacs_sweep = 0;
  // of those, the complex MACs the FP64 path runs in the three-product form
  // (6 real flops each instead of 8), and those of the low-rank W kernel
  // (always three-product, also on the mixed path)
  double gemm_cmacs_k3 = 0, gemm_cmacs_w = 0;
  cplx *ws = nullptr, *fs = nullptr, *sb = nullptr, *sc = nullptr, *X = nullptr, *V = nullptr, *aval = nullptr;
  int32_t *perms = nullptr;   // pivot permutation of every front, at its first elimination index
  char *blob = nullptr;
  int *status = nullptr;      // [0]: pivot status of the last factorization; [1]: permittivity check of the last assembly
  double *pivq = nullptr;     // per front: pivot spread min |u_kk| / max |u_kk| of the last factorization
  int32_t *g_nnz = nullptr;   // column-sparse dF/dS: nonzeros per input, their max, compact (row, value) lists
  int *g_max = nullptr;
  int32_t *g_idx = nullptr;
  cplx *g_val = nullptr;
  int last_sparse_k = 0;      // the last apf_grad's compact width (0: dense product)
  // compressed channels: the bases on the channel rows (nx x M'_B, nx x M'_C),
  // S~ (M'_C x M'_B), the decompression matrices D_B (M'_B x n_in) and D_C
  // (n_out x M'_C), the product S~ D_B, and the two decompression task lists
  cplx *czBt = nullptr, *czCt = nullptr, *czS = nullptr, *czDB = nullptr, *czDC = nullptr, *czT = nullptr;
  int64_t czD1 = -1, czD2 = -1;
  int nczD1 = 0, nczD2 = 0;
  // compressed gradient: dF/dS~ = D_C^T dF/dS D_B^T (M'_C x M'_B) through
  // T2 = D_C^T dF/dS (M'_C x n_in), with D_B^T stored (n_in x M'_B)
  cplx *czG = nullptr, *czT2 = nullptr, *czDBt = nullptr;
  int64_t czG1 = -1, czG2 = -1;
  int nczG1 = 0, nczG2 = 0;
  double vinit_cmacs = 0;     // complex MACs of the dense weighted-adjoint-source product
  double *part = nullptr;
  int64_t ws_elems = 0, fs_elems = 0, x_elems = 0;
  int rhs_chunk = 0;
  std::vector<LevelTasks> lv;
  int64_t vinit = -1, gidx = -1, fronts = -1, gSsplit = -1, vmap_base = -1, vmap_pidx = -1;
  bool sym = false;           // symmetric route (apf_set_symmetric)
  int64_t ztr = -1;           // symmetric route: Z = X12^T of the sweep fronts, after the factorization
  int nztr = 0;
  int64_t xc_rows = 0;        // rows of the weighted-adjoint operand store (sweep fronts with C rows)
  int64_t xc_elems = 0;       // its size: xc_rows x n_out, or the sum of p x mC of compressed panels
  cplx *xc = nullptr;         // L^-T U^-T FC1^T of those fronts, stacked front by front (ld mC)
  int ncol = 0;               // right-hand-side columns of the sweeps: n_in, or M'_B when compressed
  int32_t *vmap = nullptr;    // V row of every xc row (rebuilt from the pivot permutations per call)
  int nfronts = 0, ngSsplit = 0, nseg = 0;
  cplx *spart = nullptr;      // FP64 partial Schur blocks (nseg x n_out x n_in)
  char *chan = nullptr;       // ChanParams of the source and projection rows, then their orders
  int nvinit = 0;
  // gradient sweeps: launch t holds the Y tiles of level H - t and the
  // adjoint tiles (with the contraction) of level H - t + 1
  std::vector<int64_t> swl;
  std::vector<int> nswl, nswl_thin;   // (thin tiles at the end of each list)
  // low-rank sweep subtrees (no channel rows): instead of Y and Lam tiles,
  // launch t is followed by the Wt = Y_bnd Lam_bnd^T quadrant tasks of the
  // subtree roots of level H - t + 1 (swtb); after the sweeps, level by level
  // from the top, the U1t and Qt products (wu, wq) and the gather of the
  // children's Wt with the fronts' gradient (wp)
  std::vector<char> swl_deep;
  std::vector<int> swl_id, wu_id, wq_id;
  char vinit_deep = 1, schur_deep = 1;      // the weighted adjoint source and the Schur partials
  int vinit_id = -1, schur_id = -1;
  std::vector<TunableList> tl;               // every tunable GEMM list of the plan
  std::vector<int64_t> swtb;
  std::vector<int> nswtb;
  std::vector<int64_t> wu, wq, wp;
  std::vector<int> nwu, nwq, nwp;
  std::vector<char> wu_deep, wq_deep;
  cplx *lrW = nullptr;        // per front: Bf (b x (p+b)) and Qt (p x (p+b))
  int n_wfronts = 0, n_wroots = 0;   // fronts of low-rank sweep subtrees, their roots
  int64_t ndesign = 0;        // design pixels (contraction slots)
  int nblk = 0;               // 32-column contraction partials per pixel
  double *gpart = nullptr;    // nblk x ndesign (block-major)
  template <class T>
  T *at(int64_t off) const { return off < 0 ? nullptr : reinterpret_cast<T *>(blob + off); }
};

double g_cmacs_acc = 0;   // executed complex MACs of the tasks added (plan building only)

// Complex MACs of one tile whose operands are both structurally nonzero: a
// triangular operand contributes only its stored triangle (diagonal
// included), everything else the full k range.  This is the algorithmic work
// of the tile, not counting the zeros the MFMA tiles multiply.
double tile_cmacs(const GemmTask &t, int tm, int tn) {
  const bool tr = t.flags & G_TRANS_A;
  const int mm = std::min(GEMM_TILE, t.M - tm), nn = std::min(GEMM_TILE, t.N - tn);
  if (mm <= 0 || nn <= 0 || t.K <= 0) return 0.0;
  // nonzero k count for an index x of the triangular operand: k <= x (kind 1)
  // or k >= x (kind 2), within [0, K)
  auto cnt = [&](int kind, int x) -> double {
    if (kind == 1) return std::max(0, std::min(t.K, x + 1));
    return std::max(0, t.K - std::max(0, x));
  };
  const bool triA = t.flags & (G_A_TRI_L | G_A_TRI_U), triB = t.flags & (G_B_TRI_L | G_B_TRI_U);
  double s = 0.0;
  if (triA) {
    // stored (r, c) = (i, k) or, transposed, (k, i); L keeps r >= c, U r <= c
    const int kind = (((t.flags & G_A_TRI_L) != 0) != tr) ? 1 : 2;
    for (int i = tm; i < tm + mm; ++i) s += cnt(kind, i);
    return s * nn;
  }
  if (triB) {
    const int kind = (t.flags & G_B_TRI_L) ? 2 : 1;   // stored (k, j)
    for (int j = tn; j < tn + nn; ++j) s += cnt(kind, j);
    return s * mm;
  }
  return (double)mm * nn * t.K;
}


void add_tiles(std::vector<GemmTask> &v, const GemmTask &t) {
  if (t.M <= 0 || t.N <= 0) return;
  for (int tm = 0; tm < t.M; tm += GEMM_TILE)
    for (int tn = 0; tn < t.N; tn += GEMM_TILE) {
      GemmTask u = t;
      u.tm = tm;
      u.tn = tn;
      g_cmacs_acc += tile_cmacs(t, tm, tn);
      v.push_back(u);
    }
}

// Tiles of one large GEMM in an order that suits the 8 XCDs (each with its
// own L2): workgroup b runs on XCD b % 8, so the list interleaves eight
// queues.  The tile grid is cut into eight equal rectangular regions (the
// split of 8 into row x column groups that keeps regions squarest), one per
// XCD, so that an XCD's tiles share A row panels and B column panels; each
// region is walked in 8 x 8 sub-blocks, the tiles that run side by side.
// Queues are padded with empty tasks (M = N = 0, which the kernel skips).
constexpr int N_XCD = 8, SUB = 8;

void add_tiles_xcd(std::vector<GemmTask> &v, const GemmTask &t) {
  if (t.M <= 0 || t.N <= 0) return;
  const int nm = (t.M + GEMM_TILE - 1) / GEMM_TILE, nn = (t.N + GEMM_TILE - 1) / GEMM_TILE;
  int RB = 1, CB = 8;
  double best = 1e30;
  for (int rb : {1, 2, 4, 8}) {
    const int cb = N_XCD / rb;
    if (rb > nm || cb > nn) continue;
    const double h = (double)nm / rb, w = (double)nn / cb;
    const double score = std::max(h / w, w / h);
    if (score < best) { best = score; RB = rb; CB = cb; }
  }
  if (best == 1e30) { RB = std::min(nm, N_XCD); CB = 1; }
  std::vector<std::vector<GemmTask>> q(N_XCD);
  for (int rb = 0; rb < RB; ++rb)
    for (int cb = 0; cb < CB; ++cb) {
      std::vector<GemmTask> &qq = q[(rb * CB + cb) % N_XCD];
      const int m0 = rb * nm / RB, m1 = (rb + 1) * nm / RB, n0 = cb * nn / CB, n1 = (cb + 1) * nn / CB;
      for (int sm = m0; sm < m1; sm += SUB)
        for (int sn = n0; sn < n1; sn += SUB)
          for (int im = sm; im < std::min(m1, sm + SUB); ++im)
            for (int in = sn; in < std::min(n1, sn + SUB); ++in) {
              GemmTask u = t;
              u.tm = im * GEMM_TILE;
              u.tn = in * GEMM_TILE;
              g_cmacs_acc += tile_cmacs(t, u.tm, u.tn);
              qq.push_back(u);
            }
    }
  size_t len = 0;
  for (auto &qq : q) len = std::max(len, qq.size());
  GemmTask empty = t;
  empty.M = empty.N = 0;
  empty.tm = empty.tn = 0;
  for (size_t k = 0; k < len; ++k)
    for (int x = 0; x < N_XCD; ++x) v.push_back(k < q[x].size() ? q[x][k] : empty);
}

GemmTask gemm(const cplx *A, int lda, const cplx *B, int ldb, cplx *C, int ldc, int M, int N, int K, int flags,
              const cplx *Cin = nullptr, int ldcin = 0, const int32_t *browmap = nullptr) {
  GemmTask t{};
  t.A = A; t.B = B; t.C = C; t.Cin = Cin; t.browmap = browmap; t.crowmap = nullptr;
  t.M = M; t.N = N; t.K = K;
  t.lda = lda; t.ldb = ldb; t.ldc = ldc; t.ldcin = ldcin;
  t.flags = flags;
  return t;
}

// Offsets of one front's blocks.  Workspace (transient) sub-blocks are
// relative to the front's workspace block `ws`; fs_* are offsets in the
// persistent factor store (-1 if absent); sk is the front's first row in the
// Schur operand stores (fronts holding both channel blocks).
struct Off {
  // Transient blocks, two arena allocations that both end after the front's
  // own level.  pws: the core and the channel panels (bp, cpiv, cbnd), taken
  // at the first child's level (the children write their contribution blocks
  // into them); ws: tri, u12, l21, u1b, lc1t, taken at the front's level.
  int64_t pws = -1, pwsz = 0;
  int64_t ws = -1, core = -1, bp = -1, cpiv = -1, cbnd = -1, tri = -1, u12 = -1, l21 = -1, u1b = -1, lc1t = -1;
  int64_t fs_x12 = -1, fs_z = -1, fs_x1b = -1, xk = -1, sk = -1;
  int64_t xoff = -1;   // first element of the front's XC1 block (p x mC) in the xc store
  int64_t wsz = 0;
  // refinement: retained tri, L21 and (fronts outside the sweeps) X12
  int64_t ss_tri = -1, ss_l21 = -1, ss_x12 = -1;
};

}  // namespace

// B/C compression (Supplement Sec. 1, reading of this library): the channel
// sets are extended by `pad` orders, weighted by a Hann window, transformed
// to spatially localized columns on the channel rows and truncated to
// +-half_px; the factorization carries, per front, only the columns whose
// window meets its region, and S is recovered from S~ = C~ A^-1 B~ by two
// dense products.
struct Compress {
  int pad = -1;                          // < 0: off
  double half_px = 0.0;
  int MxB = 0, MxC = 0, a0B = 0, a0C = 0;
  std::vector<int> cB0, cB1, cC0, cC1;   // per front: column ranges of its B / C panels
};

struct apf_handle {
  Desc d;
  Compress cz;
  bool analyzed = false;
  Symbolic sym;
  Phys phys{};
  bool planned = false;
  Plan plan;
  std::vector<Off> off;
  Profiler prof;
  int state = 0;        // 0 analysed, 1 assembled, 2 factored
  bool mixed = false;   // precision of the factors held (APF_MIXED)
  int max_chunk = 0;    // cap on the right-hand-side chunk of the sweeps (0: memory decides)
  int lowrank = kWMaxLevelsDefault;  // levels of a low-rank sweep subtree (0: none)
  int64_t n_factor = 0; // factorizations run on this handle (a caller can tell whether the factors changed)
  int refine_iters = 0; // > 0: the plan keeps every front's factors for APF_MIXED_REFINED
  double refine_tol = 0.0;
  bool refined = false; // the factors held come from APF_MIXED_REFINED (apf_grad refines too)
  bool sweeps = true;   // the plan prepares the gradient sweeps (apf_set_gradient)
  bool symmetric = false;  // L D L^T pivot blocks and the products' symmetry (apf_set_symmetric)
};

// The gradient sweeps' data (X12, Z, X1B, XC1 of the sweep fronts, the X/V
// arrays) is built only when the handle wants gradients: without it, no
// front is a sweep front.
static void drop_sweeps_unless_wanted(apf_handle *H) {
  if (H->sweeps) return;
  Symbolic &S = H->sym;
  for (Front &F : S.fronts) F.sweep = false;
  S.n_sweep_rows = 0;
  std::fill(S.node_sweep_row.begin(), S.node_sweep_row.end(), -1);
}

// ---------------------------------------------------------------------------
// validation and creation
// ---------------------------------------------------------------------------
static double pml_alpha(double h, double eps, int L, int m, double R0) {
  return (m + 1) * std::log(1.0 / R0) / (2.0 * h * std::sqrt(eps) * L);
}

static bool propagates(int a, int nx, double h, double eps) {
  double s = std::sin(M_PI * a / nx);
  double rhs = h * h * eps / 4.0 - s * s;
  return rhs > 0.0 && rhs < 1.0;
}

extern "C" apf_status apf_create(const apf_problem_desc *in, apf_handle **out) {
  if (!in || !out) return fail(APF_EINVAL, "null argument");
  *out = nullptr;
  const apf_problem_desc &q = *in;
  if (q.nx < 3 || q.ny < 3) return fail(APF_EINVAL, "need nx >= 3 and ny >= 3");
  if ((int64_t)q.nx * q.ny > INT_MAX / 8) return fail(APF_EINVAL, "grid too large");
  if (!(q.dx_over_lambda > 0.0) || !std::isfinite(q.dx_over_lambda)) return fail(APF_EINVAL, "bad dx_over_lambda");
  if (q.npml_top < 0 || q.npml_bot < 0 || q.npml_top + q.npml_bot >= q.ny) return fail(APF_EINVAL, "bad PML rows");
  if ((q.npml_top > 0 || q.npml_bot > 0) && !(q.pml_R0 > 0.0 && q.pml_R0 < 1.0)) return fail(APF_EINVAL, "bad pml_R0");
  if (q.pml_power < 0 || q.pml_power > 8) return fail(APF_EINVAL, "bad pml_power");
  if (!(q.eps_top > 0.0) || !(q.eps_bot > 0.0)) return fail(APF_EINVAL, "bad background permittivity");
  const int lo = q.npml_top, hi = q.ny - q.npml_bot;  // physical rows [lo, hi)
  if (!(q.design_row0 >= lo && q.design_row0 < q.design_row1 && q.design_row1 <= hi))
    return fail(APF_EINVAL, "design rows must be non-empty and outside the PML");
  if (!(q.src_row >= lo && q.src_row < q.design_row0)) return fail(APF_EINVAL, "src_row must be in the top medium");
  if (!(q.prj_row >= q.design_row1 && q.prj_row < hi)) return fail(APF_EINVAL, "prj_row must be in the bottom medium");
  if (q.n_in < 1 || q.n_out < 1 || !q.in_orders || !q.out_orders) return fail(APF_EINVAL, "need channels");
  if (q.leaf_size < 0 || q.leaf_size > 1024) return fail(APF_EINVAL, "leaf_size must be in [0, 1024]");
  if (q.ny > 1024) return fail(APF_EINVAL, "ny > 1024 is not supported (separator length)");
  const double h = 2.0 * M_PI * q.dx_over_lambda;
  for (int k = 0; k < q.n_in; ++k)
    if (!propagates(q.in_orders[k], q.nx, h, q.eps_top)) return fail(APF_EINVAL, "input order does not propagate");
  for (int k = 0; k < q.n_out; ++k)
    if (!propagates(q.out_orders[k], q.nx, h, q.eps_bot)) return fail(APF_EINVAL, "output order does not propagate");
  apf_handle *H = new (std::nothrow) apf_handle();
  if (!H) return fail(APF_ENOMEM, "host allocation failed");
  Desc &d = H->d;
  d.nx = q.nx; d.ny = q.ny; d.dx_over_lambda = q.dx_over_lambda;
  d.npml_top = q.npml_top; d.npml_bot = q.npml_bot; d.pml_R0 = q.pml_R0; d.pml_power = q.pml_power;
  d.eps_top = q.eps_top; d.eps_bot = q.eps_bot;
  d.src_row = q.src_row; d.prj_row = q.prj_row; d.design_row0 = q.design_row0; d.design_row1 = q.design_row1;
  d.n_in = q.n_in; d.n_out = q.n_out;
  d.in_orders.assign(q.in_orders, q.in_orders + q.n_in);
  d.out_orders.assign(q.out_orders, q.out_orders + q.n_out);
  d.leaf_size = q.leaf_size;
  Phys &P = H->phys;
  P.nx = d.nx; P.ny = d.ny; P.h2 = h * h;
  P.npml_top = d.npml_top; P.npml_bot = d.npml_bot; P.pml_power = d.pml_power;
  P.alpha_top = d.npml_top > 0 ? pml_alpha(h, d.eps_top, d.npml_top, d.pml_power, d.pml_R0) : 0.0;
  P.alpha_bot = d.npml_bot > 0 ? pml_alpha(h, d.eps_bot, d.npml_bot, d.pml_power, d.pml_R0) : 0.0;
  P.eps_src = d.eps_top; P.eps_prj = d.eps_bot;
  *out = H;
  g_err.clear();
  return APF_OK;
}

static void size_plan(apf_handle *H);

extern "C" apf_status apf_analyze(apf_handle *h) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (h->analyzed) return APF_OK;
  try {
    analyze(h->d, h->sym);
    drop_sweeps_unless_wanted(h);
    size_plan(h);
  } catch (const std::bad_alloc &) {
    return fail(APF_ENOMEM, "host allocation failed in analysis");
  } catch (const std::exception &e) {
    return fail(APF_EINVAL, e.what());
  }
  h->analyzed = true;
  return APF_OK;
}

// ---------------------------------------------------------------------------
// device plan
// ---------------------------------------------------------------------------
// Memory plan (host only): workspace offsets from a lifetime-interval
// allocation over the levels, persistent factor offsets, store sizes.
static void size_plan(apf_handle *H) {
  Symbolic &S = H->sym;
  const Desc &d = H->d;
  Plan &P = H->plan;
  const int nf = (int)S.fronts.size();
  const int H_ = (int)S.levels.size() - 1;
  const int Mi = d.n_in, Mo = d.n_out;
  std::vector<Off> &o = H->off;
  o.assign(nf, Off());
  Arena ar;
  std::vector<std::vector<int>> release_at(H_ + 2);
  int64_t fs = 0, ktot = 0, xck = 0, xce = 0, ss = 0;
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    const bool cz = H->cz.pad >= 0;
    int64_t p = F.p(), b = F.b(), n = p + b;
    int64_t mB = F.hasB ? (cz ? H->cz.cB1[f] - H->cz.cB0[f] : Mi) : 0;
    int64_t mC = F.hasC ? (cz ? H->cz.cC1[f] - H->cz.cC0[f] : Mo) : 0;
    Off &q = o[f];
    int64_t w = 0;
    q.tri = w; w += up(p * p);
    if (b) { q.u12 = w; w += up(p * b); q.l21 = w; w += up(b * p); }
    if (mB && (!F.sfront || cz)) { q.u1b = w; w += up(p * mB); }
    if (mC && (!F.sfront || cz)) { q.lc1t = w; w += up(p * mC); }
    q.wsz = w;
    int64_t pw = 0;
    q.core = pw; pw += up(n * n);
    if (mB) { q.bp = pw; pw += up(n * mB); }
    if (mC) { q.cpiv = pw; q.cbnd = pw + p * mC; pw += up(n * mC); }
    q.pwsz = pw;
    if (F.sweep) {
      if (b) { q.fs_x12 = fs; fs += up(p * b); q.fs_z = fs; fs += up(b * p); }
      if (mB) { q.fs_x1b = fs; fs += up(p * mB); }
      if (mC) { q.xk = xck; xck += p; q.xoff = xce; xce += p * mC; }
    }
    if (F.sfront && !cz) { q.sk = ktot; ktot += p; }
    if (H->refine_iters > 0) {
      q.ss_tri = ss; ss += up(p * p);
      if (b) {
        q.ss_l21 = ss; ss += up(b * p);
        if (!F.sweep) { q.ss_x12 = ss; ss += up(p * b); }
      }
    }
  }
  // lifetime allocation, level by level: a front's workspace is taken at its
  // first child's level and given back after its own level
  std::vector<std::vector<int>> alloc_at(H_ + 1);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    int lp = F.height;
    for (int c = 0; c < F.nchild; ++c) lp = std::min(lp, S.fronts[F.child[c]].height);
    alloc_at[lp].push_back(f);
  }
  for (int lvl = 0; lvl <= H_; ++lvl) {
    for (int f : release_at[lvl]) {
      ar.release(o[f].ws, o[f].wsz);
      ar.release(o[f].pws, o[f].pwsz);
    }
    for (int f : alloc_at[lvl]) o[f].pws = ar.alloc(o[f].pwsz);
    for (int f : S.levels[lvl]) {
      o[f].ws = ar.alloc(o[f].wsz);
      release_at[lvl + 1].push_back(f);
    }
  }
  P.ws_elems = std::max<int64_t>(ar.top, 1);
  P.fs_elems = std::max<int64_t>(fs, 1);
  P.R.ss_elems = ss;
  P.xc_rows = xck;
  P.xc_elems = xce;
  S.k_total = ktot;
}

// Mean k extent of a GEMM task list's tiles (the k range a tile runs, as the
// kernel narrows it for triangular operands).  Lists whose tiles are deep
// enough to be MFMA-bound run on the three-product kernel.
static double mean_tile_k(const std::vector<GemmTask> &v) {
  if (v.empty()) return 0.0;
  double sum = 0.0;
  for (const GemmTask &T : v) {
    int kb = 0, ke = T.K;
    const bool ta = T.flags & G_TRANS_A;
    if (T.flags & G_A_TRI_L) { if (ta) kb = T.tm; else ke = std::min(ke, T.tm + 64); }
    if (T.flags & G_A_TRI_U) { if (ta) ke = std::min(ke, T.tm + 64); else kb = T.tm; }
    if (T.flags & G_B_TRI_L) kb = std::max(kb, T.tn);
    if (T.flags & G_B_TRI_U) ke = std::min(ke, T.tn + 64);
    sum += std::max(0, ke - kb);
  }
  return sum / (double)v.size();
}
// Threshold measured at 24000x160 and 48000x160 with the thin tiles on their
// own kernel: lists with a mean k extent of 32 or more run faster on the
// three-product kernel (fewer MFMAs) despite its lower occupancy (thresholds
// from 0 to 64 within 3 ms of each other; 96 cost 3 and 6 ms); shallower
// lists are bound by their loads and epilogues.
constexpr double kDeepMeanK = 32.0;
constexpr int kWMaxLevels = 2;   // most levels of a low-rank sweep subtree
// Flags every task of a deep list for the three-product form.  The flag is
// per task, so a task rounds the same way in any launch that holds it
// (single problems and merged batches alike).
static bool mark_deep(std::vector<GemmTask> &v) {
  if (mean_tile_k(v) < kDeepMeanK) return false;
  for (GemmTask &T : v) T.flags |= G_K3;
  return true;
}
static bool any_k3(const std::vector<GemmTask> &v) {
  for (const GemmTask &T : v)
    if (T.flags & G_K3) return true;
  return false;
}
// Moves the thin tiles of a list to its end (in their order), those with a
// triangular operand last, and returns their count (*ntri: the triangular
// ones): launch_gemm runs them on the thin kernels.  Whether a tile is thin
// depends on the tile alone, so it runs the same kernel (and rounds the same
// way) in every list that holds it, merged batches included.
static int split_thin(std::vector<GemmTask> &v, int *ntri) {
  auto it = std::stable_partition(v.begin(), v.end(), [](const GemmTask &T) { return !thin_tile_task(T); });
  auto jt = std::stable_partition(it, v.end(), [](const GemmTask &T) { return !tri_task(T); });
  *ntri = (int)(v.end() - jt);
  return (int)(v.end() - it);
}

// Device plan of the refined solves (after the main plan, whose channel
// parameters, permutations and retained factors it uses).  The chunk rc is
// taken from the free memory (two N x rc field arrays, the front-local panel
// arena, the adjoint row buffer), capped by apf_set_rhs_chunk's cap.
static void build_refine(apf_handle *H) {
  Symbolic &S = H->sym;
  const Desc &d = H->d;
  Plan &P = H->plan;
  Refine &R = P.R;
  const std::vector<Off> &o = H->off;
  const int nf = (int)S.fronts.size();
  const int H_ = (int)S.levels.size() - 1;
  const int Mi = d.n_in, Mo = d.n_out, nx = d.nx;
  const int64_t N = (int64_t)d.nx * d.ny;
  R.iters = H->refine_iters;
  R.tol = H->refine_tol;

  // element maps, channel matrices, kept forward fields
  {
    std::vector<int32_t> el(N);
    for (int64_t n = 0; n < N; ++n) el[n] = (int32_t)S.node_elim[n];
    HIPCHK(hipMalloc(&R.elim, N * sizeof(int32_t)));
    HIPCHK(hipMemcpy(R.elim, el.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMalloc(&R.Bmat, (int64_t)nx * Mi * sizeof(cplx)));
  HIPCHK(hipMalloc(&R.Cmat, (int64_t)Mo * nx * sizeof(cplx)));
  {
    const ChanParams *cp = reinterpret_cast<const ChanParams *>(P.chan);
    HIPCHK(launch_channel_matrices(cp, cp + 1, R.Bmat, R.Cmat, nullptr));
    HIPCHK(hipDeviceSynchronize());
  }
  HIPCHK(hipMalloc(&R.Ydes, std::max<int64_t>(P.ndesign * Mi, 1) * sizeof(cplx)));

  // panel level of every front: its first child's level (its own for leaves)
  std::vector<int> lp(nf);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    lp[f] = F.height;
    for (int c = 0; c < F.nchild; ++c) lp[f] = std::min(lp[f], S.fronts[F.child[c]].height);
  }
  // arena of the front-local panels ((p + b) x rc, from the panel level to the
  // own level) and y1 blocks (p x rc, at the own level)
  std::vector<int64_t> pan_off(nf), y1_off(nf);
  auto size_arena = [&](int64_t rc) -> int64_t {
    Arena ar;
    std::vector<std::vector<int>> alloc_at(H_ + 1), release_at(H_ + 2);
    for (int f = 0; f < nf; ++f) alloc_at[lp[f]].push_back(f);
    for (int lvl = 0; lvl <= H_; ++lvl) {
      for (int f : release_at[lvl]) {
        ar.release(pan_off[f], (int64_t)(S.fronts[f].p() + S.fronts[f].b()) * rc);
        ar.release(y1_off[f], (int64_t)S.fronts[f].p() * rc);
      }
      for (int f : alloc_at[lvl]) pan_off[f] = ar.alloc((int64_t)(S.fronts[f].p() + S.fronts[f].b()) * rc);
      for (int f : S.levels[lvl]) {
        y1_off[f] = ar.alloc((int64_t)S.fronts[f].p() * rc);
        release_at[lvl + 1].push_back(f);
      }
    }
    return std::max<int64_t>(ar.top, 1);
  };
  {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    const double per_col = 2.0 * N * sizeof(cplx) + (double)nx * sizeof(cplx) +
                           (double)size_arena(64) / 64.0 * sizeof(cplx);
    int64_t rc = (int64_t)(0.5 * (double)fr / per_col);
    rc = std::min<int64_t>(rc, Mi);
    if (H->max_chunk > 0) rc = std::min<int64_t>(rc, H->max_chunk);
    if (rc < Mi) rc = std::max<int64_t>(64, rc / 64 * 64);
    R.rc = (int)std::max<int64_t>(rc, 1);
  }
  const int rc = R.rc;
  R.arena_elems = size_arena(rc);
  R.nchunks = (Mi + rc - 1) / rc;
  HIPCHK(hipMalloc(&R.X, N * rc * sizeof(cplx)));
  HIPCHK(hipMalloc(&R.W, N * rc * sizeof(cplx)));
  HIPCHK(hipMalloc(&R.arena, R.arena_elems * sizeof(cplx)));
  HIPCHK(hipMalloc(&R.rowbuf, (int64_t)nx * rc * sizeof(cplx)));
  HIPCHK(hipMalloc(&R.norms, (int64_t)R.nchunks * (R.iters + 2) * sizeof(double)));

  Blob bl;
  {
    const char pad[16] = {0};
    bl.add(pad, sizeof pad);
  }
  auto PAN = [&](int f) { return R.arena + pan_off[f]; };
  auto Y1 = [&](int f) { return R.arena + y1_off[f]; };
  // integer arrays: boundary elimination rows, flagged parent rows, design
  // and projection rows (offsets; rebased once the blob is allocated)
  std::vector<int64_t> bnde_off(nf, -1), rows_off(nf, -1);
  // writers of each front's panel rows: its own pivot rows are copied from
  // the global array at its panel level (first writer); boundary rows are
  // written by the children (first writer stores, later ones add)
  std::vector<std::vector<uint8_t>> wr(nf);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    wr[f].assign(F.p() + F.b(), 0);
    for (int k = 0; k < F.p(); ++k) wr[f][k] = 1;
  }
  std::vector<int> slot_of(nf, 0);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    int order[2] = {0, 1};
    if (F.nchild == 2 && S.fronts[F.child[1]].height < S.fronts[F.child[0]].height) std::swap(order[0], order[1]);
    for (int oc = 0; oc < F.nchild; ++oc) {
      const int c = order[oc], cf = F.child[c];
      const Front &Ch = S.fronts[cf];
      slot_of[cf] = c;
      if (Ch.b() == 0) continue;
      std::vector<int32_t> rr;
      for (int r = 0; r < Ch.b(); ++r) {
        const int pr = Ch.rmap[r];
        rr.push_back(pr | (wr[f][pr] ? EXT_ADD : 0));
        wr[f][pr] = 1;
      }
      rows_off[cf] = bl.add(rr);
    }
    if (F.b()) {
      std::vector<int32_t> be(F.b());
      for (int k = 0; k < F.b(); ++k) be[k] = (int32_t)S.node_elim[F.bnd[k]];
      bnde_off[f] = bl.add(be);
    }
  }
  int64_t erow_prj = -1;
  {
    std::vector<int32_t> ep(nx), ed(P.ndesign);
    for (int i = 0; i < nx; ++i) ep[i] = (int32_t)S.node_elim[(int64_t)d.prj_row * nx + i];
    for (int y = d.design_row0; y < d.design_row1; ++y)
      for (int x = 0; x < nx; ++x)
        ed[(int64_t)(y - d.design_row0) * nx + x] = (int32_t)S.node_elim[(int64_t)y * nx + x];
    erow_prj = bl.add(ep);
    R.erow_des = bl.add(ed);
  }
  auto IP = [](int64_t off) { return reinterpret_cast<const int32_t *>((intptr_t)off); };   // rebased below

  std::vector<std::vector<ZeroRange>> zr(H_ + 1);
  std::vector<std::vector<CopyRange>> cr(H_ + 1);
  std::vector<std::vector<GemmTask>> g1(H_ + 1), g2(H_ + 1), g2b(H_ + 1), bk(H_ + 1);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    const Off &q = o[f];
    const int p = F.p(), b = F.b(), lvl = F.height;
    cplx *pan = PAN(f), *y1 = Y1(f);
    cplx *tri = P.R.ss + q.ss_tri;
    cplx *Wf = R.W + F.elim0 * rc;
    for (int64_t o0 = 0; o0 < (int64_t)p * rc; o0 += ZERO_CHUNK)
      cr[lp[f]].push_back({Wf + o0, pan + o0, std::min(ZERO_CHUNK, (int64_t)p * rc - o0)});
    bool bnd_read = false;
    for (int k = p; k < p + b; ++k) bnd_read = bnd_read || wr[f][k];
    if (bnd_read)
      for (int k = p; k < p + b;) {
        if (wr[f][k]) { ++k; continue; }
        int e = k + 1;
        while (e < p + b && !wr[f][e]) ++e;
        for (int64_t o0 = 0; o0 < (int64_t)(e - k) * rc; o0 += ZERO_CHUNK)
          zr[lp[f]].push_back({pan + (int64_t)k * rc + o0, std::min(ZERO_CHUNK, (int64_t)(e - k) * rc - o0)});
        k = e;
      }
    const int32_t *perm = P.perms + F.elim0;
    // forward: y1 = L^-1 P^T r1; T = U^-1 y1 into the global rows; the
    // parent's rows take r2 - L21 y1
    add_tiles(g1[lvl], gemm(tri, p, pan, rc, y1, rc, p, rc, p, G_A_TRI_L, nullptr, 0, perm));
    add_tiles(g2[lvl], gemm(tri, p, y1, rc, Wf, rc, p, rc, p, G_A_TRI_U));
    if (b) {
      const int par = F.parent;
      GemmTask t = gemm(P.R.ss + q.ss_l21, p, y1, rc, PAN(par), rc, b, rc, p,
                        G_NEG | (bnd_read ? G_CIN | G_CIN_OWN : 0), bnd_read ? pan + (int64_t)p * rc : nullptr, rc);
      t.crowmap = IP(rows_off[f]);
      add_tiles(slot_of[f] ? g2b[lvl] : g2[lvl], t);
      // backward: x1 = T - X12 x2, in place
      const cplx *x12 = q.ss_x12 >= 0 ? P.R.ss + q.ss_x12 : P.fs + q.fs_x12;
      add_tiles(bk[lvl], gemm(x12, b, R.W, rc, Wf, rc, p, rc, b, G_NEG | G_CIN, Wf, rc, IP(bnde_off[f])));
    }
  }
  // S columns = Cmat X[projection rows]; the adjoint rows C^T dF/dS
  std::vector<GemmTask> sg, ag;
  {
    GemmTask t = gemm(R.Cmat, nx, R.X, rc, nullptr, Mi, Mo, rc, nx, G_C_EXT | G_C_COFF | G_K3, nullptr, 0,
                      IP(erow_prj));
    add_tiles_xcd(sg, t);
    add_tiles_xcd(ag, gemm(R.Cmat, nx, nullptr, Mi, R.rowbuf, rc, nx, rc, Mo,
                           G_TRANS_A | G_B_EXT | G_B_COFF | G_K3));
  }
  R.lv.assign(H_ + 1, RefineLevel());
  for (int lvl = 0; lvl <= H_; ++lvl) {
    RefineLevel &L = R.lv[lvl];
    L.zero = bl.add(zr[lvl]); L.nzero = (int)zr[lvl].size();
    L.copy = bl.add(cr[lvl]); L.ncopy = (int)cr[lvl].size();
    L.g1 = bl.add(g1[lvl]); L.ng1 = (int)g1[lvl].size();
    L.g2 = bl.add(g2[lvl]); L.ng2 = (int)g2[lvl].size();
    L.g2b = bl.add(g2b[lvl]); L.ng2b = (int)g2b[lvl].size();
    L.bk = bl.add(bk[lvl]); L.nbk = (int)bk[lvl].size();
  }
  R.sgemm = bl.add(sg); R.nsgemm = (int)sg.size();
  R.agemm = bl.add(ag); R.nagemm = (int)ag.size();
  HIPCHK(hipMalloc(&R.blob, bl.h.size()));
  char *base = R.blob;
  auto rebase = [&](const int32_t *&ptr) {
    if (ptr) ptr = reinterpret_cast<const int32_t *>(base + (intptr_t)ptr);
  };
  for (int lvl = 0; lvl <= H_; ++lvl) {
    const RefineLevel &L = R.lv[lvl];
    for (int which = 0; which < 3; ++which) {
      const int64_t off = which == 0 ? L.g2 : (which == 1 ? L.g2b : L.bk);
      const int n = which == 0 ? L.ng2 : (which == 1 ? L.ng2b : L.nbk);
      GemmTask *t = reinterpret_cast<GemmTask *>(bl.h.data() + off);
      for (int k = 0; k < n; ++k) {
        rebase(t[k].crowmap);
        rebase(t[k].browmap);
      }
    }
  }
  {
    GemmTask *t = reinterpret_cast<GemmTask *>(bl.h.data() + R.sgemm);
    for (int k = 0; k < R.nsgemm; ++k) rebase(t[k].browmap);
  }
  HIPCHK(hipMemcpy(R.blob, bl.h.data(), bl.h.size(), hipMemcpyHostToDevice));
}

static void build_plan(apf_handle *H) {
  Symbolic &S = H->sym;
  const Desc &d = H->d;
  Plan &P = H->plan;
  const int nf = (int)S.fronts.size();
  const int H_ = (int)S.levels.size() - 1;
  const int Mi = d.n_in, Mo = d.n_out;
  HIPCHK(hipGetDevice(&P.device));
  size_plan(H);

  const std::vector<Off> &o = H->off;
  const int64_t ktot = S.k_total;
  P.ncol = H->cz.pad >= 0 ? H->cz.MxB : Mi;
  HIPCHK(hipMalloc(&P.ws, P.ws_elems * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.fs, P.fs_elems * sizeof(cplx)));
  const bool cz = H->cz.pad >= 0;
  if (cz) {
    const Compress &Z = H->cz;
    const int nx = d.nx;
    HIPCHK(hipMalloc(&P.czBt, (int64_t)nx * Z.MxB * sizeof(cplx)));
    HIPCHK(hipMalloc(&P.czCt, (int64_t)nx * Z.MxC * sizeof(cplx)));
    HIPCHK(hipMalloc(&P.czS, (int64_t)Z.MxC * Z.MxB * sizeof(cplx)));
    HIPCHK(hipMalloc(&P.czT, (int64_t)Z.MxC * Mi * sizeof(cplx)));
    HIPCHK(hipMalloc(&P.czDB, (int64_t)Z.MxB * Mi * sizeof(cplx)));
    HIPCHK(hipMalloc(&P.czDC, (int64_t)Mo * Z.MxC * sizeof(cplx)));
    HIPCHK(hipMemset(P.czBt, 0, (int64_t)nx * Z.MxB * sizeof(cplx)));
    HIPCHK(hipMemset(P.czCt, 0, (int64_t)nx * Z.MxC * sizeof(cplx)));
    HIPCHK(launch_compress_basis(nx, Z.MxB, Z.a0B, Z.half_px, false, P.czBt, nullptr));
    HIPCHK(launch_compress_basis(nx, Z.MxC, Z.a0C, Z.half_px, true, P.czCt, nullptr));
    // D_C[b][j] = gamma_b exp(-2 pi i t_b j / M'_C) / (M'_C w_tb),
    // D_B[j][a] = exp(+2 pi i t_a j / M'_B) beta_a / (M'_B w_ta), with the
    // channel normalisations beta_a = -2i sqrt(sin q_a), gamma_b = sqrt(sin q_b)
    const double h = 2.0 * M_PI * d.dx_over_lambda;
    auto sinq = [&](int a, double eps) {
      const double sa = std::sin(M_PI * a / nx), rhs = h * h * eps / 4.0 - sa * sa;
      return std::sin(2.0 * std::asin(std::sqrt(rhs)));
    };
    auto wt = [](int t, int M) { const double v = std::sin(M_PI * (t + 0.5) / M); return v * v; };
    std::vector<cplx> DB((size_t)Z.MxB * Mi), DC((size_t)Mo * Z.MxC);
    for (int a = 0; a < Mi; ++a) {
      const int t = d.in_orders[a] - Z.a0B;
      const double bmag = 2.0 * std::sqrt(sinq(d.in_orders[a], d.eps_top)) / (Z.MxB * wt(t, Z.MxB));
      for (int j = 0; j < Z.MxB; ++j) {
        const double ang = 2.0 * M_PI * (double)(((int64_t)t * j) % Z.MxB) / Z.MxB;
        // beta_a = -2i sqrt(sin q):  (cos + i sin) * (-i) * bmag
        DB[(size_t)j * Mi + a] = {bmag * std::sin(ang), -bmag * std::cos(ang)};
      }
    }
    for (int b = 0; b < Mo; ++b) {
      const int t = d.out_orders[b] - Z.a0C;
      const double g = std::sqrt(sinq(d.out_orders[b], d.eps_bot)) / (Z.MxC * wt(t, Z.MxC));
      for (int j = 0; j < Z.MxC; ++j) {
        const double ang = 2.0 * M_PI * (double)(((int64_t)t * j) % Z.MxC) / Z.MxC;
        DC[(size_t)b * Z.MxC + j] = {g * std::cos(ang), -g * std::sin(ang)};
      }
    }
    HIPCHK(hipMemcpy(P.czDB, DB.data(), DB.size() * sizeof(cplx), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(P.czDC, DC.data(), DC.size() * sizeof(cplx), hipMemcpyHostToDevice));
    if (S.n_sweep_rows > 0) {
      std::vector<cplx> DBt((size_t)Mi * Z.MxB);
      for (int j = 0; j < Z.MxB; ++j)
        for (int a = 0; a < Mi; ++a) DBt[(size_t)a * Z.MxB + j] = DB[(size_t)j * Mi + a];
      HIPCHK(hipMalloc(&P.czDBt, DBt.size() * sizeof(cplx)));
      HIPCHK(hipMalloc(&P.czT2, (int64_t)Z.MxC * Mi * sizeof(cplx)));
      HIPCHK(hipMalloc(&P.czG, (int64_t)Z.MxC * Z.MxB * sizeof(cplx)));
      HIPCHK(hipMemcpy(P.czDBt, DBt.data(), DBt.size() * sizeof(cplx), hipMemcpyHostToDevice));
    }
    HIPCHK(hipDeviceSynchronize());
  }
  if (H->refine_iters > 0) HIPCHK(hipMalloc(&P.R.ss, std::max<int64_t>(P.R.ss_elems, 1) * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.sb, std::max<int64_t>(ktot * Mi, 1) * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.sc, std::max<int64_t>(ktot * Mo, 1) * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.aval, (int64_t)d.nx * d.ny * 5 * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.perms, (int64_t)d.nx * d.ny * sizeof(int32_t)));
  HIPCHK(hipMalloc(&P.xc, std::max<int64_t>(P.xc_elems, 1) * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.vmap, std::max<int64_t>(P.xc_rows, 1) * sizeof(int32_t)));
  HIPCHK(hipMalloc(&P.status, 2 * sizeof(int)));
  HIPCHK(hipMalloc(&P.pivq, std::max<size_t>(S.fronts.size(), 1) * sizeof(double)));
  HIPCHK(hipMalloc(&P.g_nnz, (int64_t)Mi * sizeof(int32_t)));
  HIPCHK(hipMalloc(&P.g_max, sizeof(int)));
  HIPCHK(hipMalloc(&P.g_idx, (int64_t)Mi * kSparseG * sizeof(int32_t)));
  HIPCHK(hipMalloc(&P.g_val, (int64_t)Mi * kSparseG * sizeof(cplx)));
  HIPCHK(hipMalloc(&P.part, 1024 * sizeof(double)));
  HIPCHK(hipMemset(P.status, 0, 2 * sizeof(int)));

  // sweep arrays: pick the right-hand-side chunk from the free memory (three
  // quarters of it: every chunk reruns the sweeps' latency-bound bottom
  // levels, so fewer, wider chunks pay; the quarter left covers the plan's
  // later buffers and the caller's S and dF/dS)
  {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    int64_t rows = std::max<int64_t>(S.n_sweep_rows, 1);
    double budget = 0.75 * (double)fr;
    int64_t chunk = (int64_t)(budget / (2.0 * rows * sizeof(cplx)));
    chunk = std::min<int64_t>(chunk, P.ncol);
    if (H->max_chunk > 0) chunk = std::min<int64_t>(chunk, H->max_chunk);
    if (chunk < P.ncol) chunk = std::max<int64_t>(64, chunk / 64 * 64);
    P.rhs_chunk = (int)std::max<int64_t>(chunk, 1);
    P.x_elems = rows * P.rhs_chunk;
    HIPCHK(hipMalloc(&P.X, P.x_elems * sizeof(cplx)));
    HIPCHK(hipMalloc(&P.V, P.x_elems * sizeof(cplx)));
  }

  auto WS = [&](int64_t off) -> cplx * { return P.ws + off; };
  auto FSx = [&](int64_t off) -> cplx * { return P.fs + off; };

  // ---- integer arrays (first blob pass) --------------------------------------
  Blob ib;
  {
    // offset 0 is reserved so that a rebased offset is never mistaken for null
    const char pad[16] = {0};
    ib.add(pad, sizeof pad);
  }
  std::vector<int64_t> rmap_off(nf, -1), bndrow_off(nf, -1);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    if (F.b()) rmap_off[f] = ib.add(F.rmap);
    if (F.sweep && F.b()) {
      std::vector<int32_t> br(F.b());
      for (int k = 0; k < F.b(); ++k) br[k] = (int32_t)S.node_sweep_row[F.bnd[k]];
      bndrow_off[f] = ib.add(br);
    }
  }
  {
    // contraction slot of every sweep row: the design pixel (row-major over
    // the design rows) or -1
    std::vector<int32_t> gi(std::max<int64_t>(S.n_sweep_rows, 1), -1);
    for (int y = d.design_row0; y < d.design_row1; ++y)
      for (int x = 0; x < d.nx; ++x)
        if (S.node_sweep_row[(int64_t)y * d.nx + x] >= 0)
          gi[S.node_sweep_row[(int64_t)y * d.nx + x]] = (int32_t)((int64_t)(y - d.design_row0) * d.nx + x);
    P.gidx = ib.add(gi);
    P.ndesign = (int64_t)(d.design_row1 - d.design_row0) * d.nx;
    P.nblk = 2 * ((P.ncol + 63) / 64);
    HIPCHK(hipMalloc(&P.gpart, std::max<int64_t>(P.ndesign * P.nblk, 1) * sizeof(double)));
    // slots of low-rank fronts' pixels are never written: keep them zero
    HIPCHK(hipMemset(P.gpart, 0, std::max<int64_t>(P.ndesign * P.nblk, 1) * sizeof(double)));
  }
  // Low-rank sweep subtrees.  For a sweep front f without channel rows the
  // sweeps cost 2 p b M complex MACs (Y and Lam rows, M right-hand sides)
  // plus its sweep children's costs; forming Wt = Y_bnd Lam_bnd^T instead
  // costs b^2 M, after which the whole subtree is served by small dense
  // products (b^2 p + p b (p + b) per front, independent of M).  The cheaper
  // choice is taken bottom-up (fronts are in postorder); a chosen front with
  // no chosen ancestor is a subtree root.  Subtrees span at most
  // kWMaxLevels levels: the rounding error of the dense propagation grows by
  // the cancellation factor of both field reconstructions at every level,
  // where the sweeps add it once per level (24000 x 160, gradient over all
  // pixels against the plain sweeps: 1.6e-15 for one level, 8e-14 for two,
  // 4.3e-9 for three, with 1.5e-8 in the worst sixteenth of the grid).
  std::vector<char> wcov(nf, 0), wroot(nf, 0);
  std::vector<int64_t> bf_off(nf, -1), qt_off(nf, -1);
  {
    const double M = (double)Mi;
    std::vector<double> cost(nf, 0.0), dense(nf, 0.0);
    std::vector<char> pick(nf, 0);
    std::vector<int> sdepth(nf, 0);   // levels of sweep fronts below f
    for (int f = 0; f < nf; ++f) {
      const Front &F = S.fronts[f];
      if (!F.sweep) continue;
      const double p = F.p(), b = F.b();
      double direct = 2.0 * p * b * M, dsub = b * b * p + p * b * (p + b);
      // (a root forms Wt in one 64 x 64 tile: b <= 64)
      bool ok = H->lowrank > 0 && !F.hasB && !F.hasC && F.b() > 0 && F.b() <= 64;
      for (int c = 0; c < F.nchild; ++c) {
        const int ch = F.child[c];
        if (!S.fronts[ch].sweep) continue;
        direct += cost[ch];
        dsub += dense[ch];
        sdepth[f] = std::max(sdepth[f], sdepth[ch] + 1);
      }
      ok = ok && sdepth[f] < std::min(H->lowrank, kWMaxLevels);
      dense[f] = dsub;
      const double viaW = b * b * M + dsub;
      pick[f] = ok && viaW < direct;
      cost[f] = pick[f] ? viaW : direct;
    }
    // a chosen front covers its whole sweep subtree (parents come after their
    // children, so walk down from the root)
    for (int f = nf - 1; f >= 0; --f) {
      const Front &F = S.fronts[f];
      if (!F.sweep) continue;
      const bool pc = F.parent >= 0 && wcov[F.parent];
      wcov[f] = pc || pick[f];
      wroot[f] = !pc && pick[f];
    }
    int64_t wtot = 0;
    for (int f = 0; f < nf; ++f) {
      P.n_wroots += wroot[f];
      if (!wcov[f]) continue;
      ++P.n_wfronts;
      const Front &F = S.fronts[f];
      if (F.p() > MAX_PIVOTS) throw std::runtime_error("pivot block larger than MAX_PIVOTS in a low-rank sweep subtree");
      const int64_t n = F.p() + F.b();
      bf_off[f] = wtot;
      wtot += (int64_t)F.b() * n;
      qt_off[f] = wtot;
      wtot += (int64_t)F.p() * n;
    }
    HIPCHK(hipMalloc(&P.lrW, std::max<int64_t>(wtot, 1) * sizeof(cplx)));
  }
  // channel parameters of the two panels, in a small buffer of their own
  const ChanParams *cp_src, *cp_prj;
  {
    // [2 ChanParams][orders: n_in + n_out int32][amplitudes: n_in + n_out doubles]
    const size_t ord_off = 2 * sizeof(ChanParams);
    const size_t amp_off = (ord_off + (d.n_in + d.n_out) * sizeof(int32_t) + 15) / 16 * 16;
    std::vector<char> hb(amp_off + (d.n_in + d.n_out) * sizeof(double));
    HIPCHK(hipMalloc(&P.chan, hb.size()));
    ChanParams c[2];
    c[0].P = H->phys; c[0].m = d.n_in; c[0].is_source = 1;
    c[0].orders = reinterpret_cast<const int32_t *>(P.chan + ord_off);
    c[0].amp = reinterpret_cast<double *>(P.chan + amp_off);
    c[1].P = H->phys; c[1].m = d.n_out; c[1].is_source = 0;
    c[1].orders = c[0].orders + d.n_in;
    c[1].amp = c[0].amp + d.n_in;
    std::memcpy(hb.data(), c, sizeof c);
    std::memcpy(hb.data() + ord_off, d.in_orders.data(), d.n_in * sizeof(int32_t));
    std::memcpy(hb.data() + ord_off + d.n_in * sizeof(int32_t), d.out_orders.data(), d.n_out * sizeof(int32_t));
    HIPCHK(hipMemcpy(P.chan, hb.data(), hb.size(), hipMemcpyHostToDevice));
    cp_src = reinterpret_cast<const ChanParams *>(P.chan);
    cp_prj = cp_src + 1;
    // the orders' amplitude factors, once per plan (the panel assembly reads them)
    HIPCHK(launch_channel_amp(cp_src, d.n_in + d.n_out, nullptr));
    HIPCHK(hipDeviceSynchronize());
  }
  // Channel panel rows: the first writer of a row stores, later writers add.
  // The writers of a front's panel rows, in launch order: the channel
  // assembly (pivot rows on the source or projection row; at the front's
  // panel level), then its children's phase-2 panel updates ordered by
  // (child level, slot).  wrB/wrC[f][k] marks row k of front f as written;
  // rowsB/rowsC_off[c] is child c's flagged row map into its parent.
  std::vector<std::vector<uint8_t>> wrB(nf), wrC(nf);
  std::vector<int64_t> rowsB_off(nf, -1), rowsC_off(nf, -1);
  std::vector<int> slot_of(nf, 0);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    std::vector<uint8_t> &wb = wrB[f], &wc = wrC[f];
    if (F.hasB) wb.assign(F.p() + F.b(), 0);
    if (F.hasC) wc.assign(F.p() + F.b(), 0);
    for (int k = 0; k < F.p(); ++k) {
      const int y = F.piv[k] / d.nx;
      if (F.hasB && y == d.src_row) wb[k] = 1;
      if (F.hasC && y == d.prj_row) wc[k] = 1;
    }
    int order[2] = {0, 1};
    if (F.nchild == 2 && S.fronts[F.child[1]].height < S.fronts[F.child[0]].height) std::swap(order[0], order[1]);
    for (int oc = 0; oc < F.nchild; ++oc) {
      const int c = order[oc], cf = F.child[c];
      const Front &Ch = S.fronts[cf];
      slot_of[cf] = c;
      if (Ch.b() == 0) continue;
      if ((Ch.hasB && !F.hasB) || (Ch.hasC && !F.hasC)) throw std::runtime_error("child panel without parent panel");
      std::vector<int32_t> rb, rc;
      for (int r = 0; r < Ch.b(); ++r) {
        const int pr = Ch.rmap[r];
        if (Ch.hasB) {
          rb.push_back(pr | ((wb[pr] || cz) ? EXT_ADD : 0));
          wb[pr] = 1;
        }
        if (Ch.hasC) {
          rc.push_back(pr | ((wc[pr] || cz) ? EXT_ADD : 0));
          wc[pr] = 1;
        }
      }
      if (Ch.hasB) rowsB_off[cf] = ib.add(rb);
      if (Ch.hasC) rowsC_off[cf] = ib.add(rc);
    }
  }
  P.lv.assign(H_ + 1, LevelTasks());
  for (int lvl = 0; lvl <= H_; ++lvl) {
    std::vector<int32_t> inv[N_INV_VARIANTS];
    for (int f : S.levels[lvl]) {
      const Front &F = S.fronts[f];
      if (F.p() > 0) {
        const int v = inverse_variant(F.p());
        if (v < 0) throw std::runtime_error("pivot block larger than MAX_PIVOTS");
        inv[v].push_back(f);
      }
    }
    LevelTasks &L = P.lv[lvl];
    for (int v = 0; v < N_INV_VARIANTS; ++v) { L.inv[v] = ib.add(inv[v]); L.ninv[v] = (int)inv[v].size(); }
  }
  const int64_t ib_size = (int64_t)ib.h.size();

  // The task structures reference the integer arrays; both go into one blob
  // whose device base is known once it is allocated.  Reserve generously,
  // build, then upload.
  // ---- device front descriptors and tasks (second pass) ---------------------
  // the blob base is needed for pointers into it: allocate after sizing.
  std::vector<FrontDev> fd(nf);
  // temporary: compute pointers relative to a null base, fixed up below
  char *base = nullptr;
  // Sizing pass is avoided by allocating the blob at the end and rebasing the
  // int-array pointers: they are stored as offsets here and converted once
  // the base is known.
  auto ipt = [&](int64_t off) -> const int32_t * {
    return off < 0 ? nullptr : reinterpret_cast<const int32_t *>(base + off);
  };
  (void)ipt;

  // Build everything with base = nullptr, remember which fields need rebasing.
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    const Off &q = o[f];
    FrontDev &D = fd[f];
    int64_t p = F.p(), b = F.b(), n = p + b;
    D.p = (int)p; D.b = (int)b;
    D.mB = F.hasB ? (cz ? H->cz.cB1[f] - H->cz.cB0[f] : Mi) : 0;
    D.mC = F.hasC ? (cz ? H->cz.cC1[f] - H->cz.cC0[f] : Mo) : 0;
    D.sweep_row0 = F.sweep ? (int32_t)S.node_sweep_row[F.piv[0]] : -1;
    D.core = WS(q.pws + q.core);
    D.bp_piv = D.mB ? WS(q.pws + q.bp) : nullptr;
    D.bp_bnd = D.mB ? WS(q.pws + q.bp) + p * D.mB : nullptr;
    D.cpt_piv = D.mC ? WS(q.pws + q.cpiv) : nullptr;
    D.cpt_bnd = D.mC ? WS(q.pws + q.cbnd) : nullptr;
    D.tri = q.ss_tri >= 0 ? P.R.ss + q.ss_tri : WS(q.ws + q.tri);
    D.perm = P.perms + F.elim0;
    D.rmap = reinterpret_cast<const int32_t *>((intptr_t)rmap_off[f]);  // offset; rebased below
    D.parent = F.parent;
    (void)n;
  }
  // L^-1 P^T F1B and U^-T FC1^T of fronts holding both channel blocks live in
  // the Schur operand stores
  auto U1B = [&](int f) -> cplx * {
    const Off &q = o[f];
    return (S.fronts[f].sfront && !cz) ? P.sb + q.sk * Mi : WS(q.ws + q.u1b);
  };
  auto LC1T = [&](int f) -> cplx * {
    const Off &q = o[f];
    return (S.fronts[f].sfront && !cz) ? P.sc + q.sk * Mo : WS(q.ws + q.lc1t);
  };

  std::vector<std::vector<ZeroRange>> zr(H_ + 1);
  std::vector<std::vector<AsmEntry>> ae(H_ + 1);
  std::vector<std::vector<PanelEntry>> pe(H_ + 1);
  std::vector<std::vector<CopyRange>> cpyL(H_ + 1);
  std::vector<std::vector<std::vector<GemmTask>>> schL(H_ + 1);   // compressed: S~ blocks, per colour
  std::vector<std::vector<std::vector<GemmTask>>> schTiles(H_ + 1, std::vector<std::vector<GemmTask>>(LevelTasks::kSchurColors));
  std::vector<std::vector<GemmTask>> g1(H_ + 1), g2(H_ + 1), g2b(H_ + 1), swY(H_ + 1), swL(H_ + 1), swW(H_ + 1);
  const bool sym = H->symmetric;
  P.sym = sym;
  std::vector<std::vector<TransTask>> utrL(H_ + 1);
  std::vector<TransTask> ztrL;
  std::vector<std::vector<GemmTask>> wuL(H_ + 1), wqL(H_ + 1);
  std::vector<std::vector<WFront>> wpL(H_ + 1);
  std::vector<GemmTask> vinit;
  std::vector<int32_t> vmap_base(P.xc_rows), vmap_pidx(P.xc_rows);
  std::vector<int> loc((int64_t)d.nx * d.ny, -1);
  double cm_factor = 0, cm_sweep = 0, cm_wprop = 0, cm_w = 0, vinit_acc = 0;
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    const FrontDev &D = fd[f];
    const int lvl = F.height;
    // panel level: the core and the channel panels are zeroed and assembled
    // before the first child's phase-2 update writes into them
    int lp = lvl;
    for (int c = 0; c < F.nchild; ++c) lp = std::min(lp, S.fronts[F.child[c]].height);
    const int p = F.p(), b = F.b(), n = p + b, mB = D.mB, mC = D.mC;
    auto zero = [&](cplx *ptr, int64_t cnt) {
      for (int64_t o0 = 0; o0 < cnt; o0 += ZERO_CHUNK) zr[lp].push_back({ptr + o0, std::min(ZERO_CHUNK, cnt - o0)});
    };
    zero(D.core, (int64_t)n * n);
    // Channel panel rows no writer touches are zeroed: pivot rows always (the
    // phase-1 products read them), boundary rows only when some boundary row
    // is written; otherwise the phase-2 update does not read them (no Cin).
    auto zero_rows = [&](cplx *piv0, cplx *bnd0, int m, const std::vector<uint8_t> &w) {
      bool bnd_read = false;
      for (int k = p; k < n; ++k) bnd_read = bnd_read || w[k];
      for (int k = 0; k < n;) {
        if (w[k] || (k >= p && !bnd_read)) { ++k; continue; }
        int e = k + 1;
        while (e < n && e != p && !w[e]) ++e;
        zero(k < p ? piv0 + (int64_t)k * m : bnd0 + (int64_t)(k - p) * m, (int64_t)(e - k) * m);
        k = e;
      }
      return bnd_read;
    };
    bool cinB = false, cinC = false;
    if (!cz) {
      cinB = mB ? zero_rows(D.bp_piv, D.bp_bnd, mB, wrB[f]) : false;
      cinC = mC ? zero_rows(D.cpt_piv, D.cpt_bnd, mC, wrC[f]) : false;
    } else {
      // compressed panels: zeroed whole, every writer adds (the sibling
      // panels' column ranges overlap)
      if (mB) zero(D.bp_piv, (int64_t)n * mB);
      if (mC) zero(D.cpt_piv, (int64_t)n * mC);
      cinB = mB > 0;
      cinC = mC > 0;
    }
    // stencil entries owned by this front (the earlier-eliminated end of each edge)
    for (int k = 0; k < p; ++k) loc[F.piv[k]] = k;
    for (int k = 0; k < b; ++k) loc[F.bnd[k]] = p + k;
    for (int k = 0; k < p; ++k) {
      const int u = F.piv[k];
      const int x = u % d.nx, y = u / d.nx;
      const int64_t eu = S.node_elim[u];
      int nb[5] = {u, y * d.nx + (x - 1 + d.nx) % d.nx, y * d.nx + (x + 1) % d.nx, y > 0 ? u - d.nx : -1,
                   y < d.ny - 1 ? u + d.nx : -1};
      for (int dir = 0; dir < 5; ++dir) {
        const int v = nb[dir];
        if (v < 0) continue;
        if (dir > 0 && S.node_elim[v] < eu) continue;   // owned by the front of v
        const int lu = loc[u], lv = loc[v];
        if (lv < 0) throw std::runtime_error("stencil neighbour outside the front");
        const cplx *src = P.aval + (int64_t)u * 5 + dir;
        ae[lp].push_back({src, D.core + (int64_t)lu * n + lv});
        if (dir > 0) ae[lp].push_back({src, D.core + (int64_t)lv * n + lu});   // A = A^T
      }
      if (!cz) {
        if (mB && y == d.src_row) pe[lp].push_back({u, 0, D.bp_piv + (int64_t)k * mB, cp_src});
        if (mC && y == d.prj_row) pe[lp].push_back({u, 0, D.cpt_piv + (int64_t)k * mC, cp_prj});
      } else {
        const int64_t i = u % d.nx;
        if (mB && y == d.src_row)
          cpyL[lp].push_back({P.czBt + i * H->cz.MxB + H->cz.cB0[f], D.bp_piv + (int64_t)k * mB, (int64_t)mB});
        if (mC && y == d.prj_row)
          cpyL[lp].push_back({P.czCt + i * H->cz.MxC + H->cz.cC0[f], D.cpt_piv + (int64_t)k * mC, (int64_t)mC});
      }
    }
    for (int k = 0; k < p; ++k) loc[F.piv[k]] = -1;
    for (int k = 0; k < b; ++k) loc[F.bnd[k]] = -1;

    // Factorization GEMMs.  After the pivot-block kernel, tri holds L^-1
    // (strict lower, unit diagonal) and U^-1 (upper) and perm the pivot rows:
    //   phase 1: U12 = L^-1 P^T F12, U1B = L^-1 P^T F1B, L21 = F21 U^-1, LC1T = U^-T FC1^T
    //   phase 2: F22 -= L21 U12, F2B -= L21 U1B, FC2^T -= U12^T LC1T and, for the
    //            fronts the gradient sweeps visit, X12 = U^-1 U12, X1B = U^-1 U1B,
    //            Z = L21 L^-1, XC1 = L^-T LC1T.
    const Off &q = o[f];
    cplx *core = D.core, *tri = D.tri;
    cplx *F12 = core + p, *F21 = core + (int64_t)p * n, *F22 = core + (int64_t)p * n + p;
    cplx *u12 = b ? WS(q.ws + q.u12) : nullptr;
    cplx *l21 = b ? (q.ss_l21 >= 0 ? P.R.ss + q.ss_l21 : WS(q.ws + q.l21)) : nullptr;
    cplx *u1b = mB ? U1B(f) : nullptr, *lc1t = mC ? LC1T(f) : nullptr;
    const int32_t *perm = D.perm;
    g_cmacs_acc = 0;
    // Symmetric route (F11 = L D L^T, perm the identity, F12 = F21^T, only
    // the lower triangle of each core maintained): L21 = F21 U^-1 as below,
    // and U12 = L^-1 F12 = D L21^T by a transpose instead of a product; the
    // contribution F22 - L21 U12 is symmetric and formed on its lower tiles
    // only (the boundary maps keep the elimination order, so it lands in the
    // lower triangle of the parent's core).
    if (b && !sym) add_tiles(g1[lvl], gemm(tri, p, F12, n, u12, b, p, b, p, G_A_TRI_L, nullptr, 0, perm));
    if (b && sym) utrL[lvl].push_back(TransTask{l21, u12, tri, p, b, p, p, b, 0});
    if (mB) add_tiles(g1[lvl], gemm(tri, p, D.bp_piv, mB, u1b, mB, p, mB, p, G_A_TRI_L, nullptr, 0, perm));
    if (b) add_tiles(g1[lvl], gemm(F21, n, tri, p, l21, p, b, p, p, G_B_TRI_U));
    if (mC) add_tiles(g1[lvl], gemm(tri, p, D.cpt_piv, mC, lc1t, mC, p, mC, p, G_TRANS_A | G_A_TRI_U));
    // contribution blocks, written straight into the parent: the core update
    // F22 - L21 U12 is added at (rmap[r], rmap[c]) of the parent's core; the
    // channel-panel updates F2B - L21 U1B and FC2^T - U12^T LC1T go to the
    // parent's panel rows (stored or added per row).  Second children run in
    // the g2b launch, after the first children of the same level.
    if (b) {
      const FrontDev &PD = fd[F.parent];
      std::vector<GemmTask> &gp = slot_of[f] ? g2b[lvl] : g2[lvl];
      {
        GemmTask t = gemm(l21, p, u12, b, PD.core, PD.p + PD.b, b, b, p, G_NEG | G_CIN | G_CIN_OWN | G_C_ACC, F22, n);
        t.crowmap = reinterpret_cast<const int32_t *>((intptr_t)rmap_off[f]);  // rebased below
        t.ccolmap = t.crowmap;
        if (!sym) {
          add_tiles(gp, t);
        } else {
          for (int k = 1; k < b; ++k)
            if (F.rmap[k] <= F.rmap[k - 1]) throw std::runtime_error("boundary map out of elimination order");
          std::vector<GemmTask> all;
          const double acc0 = g_cmacs_acc;
          add_tiles(all, t);
          g_cmacs_acc = acc0;
          for (const GemmTask &u : all)
            if (u.tn <= u.tm) {
              g_cmacs_acc += tile_cmacs(u, u.tm, u.tn);
              gp.push_back(u);
            }
        }
      }
      if (mB) {
        cplx *dst = PD.bp_piv + (cz ? H->cz.cB0[f] - H->cz.cB0[F.parent] : 0);
        GemmTask t = gemm(l21, p, u1b, mB, dst, PD.mB, b, mB, p, G_NEG | (cinB ? G_CIN | G_CIN_OWN : 0),
                          cinB ? D.bp_bnd : nullptr, mB);
        t.crowmap = reinterpret_cast<const int32_t *>((intptr_t)rowsB_off[f]);  // rebased below
        add_tiles(gp, t);
      }
      if (mC) {
        cplx *dst = PD.cpt_piv + (cz ? H->cz.cC0[f] - H->cz.cC0[F.parent] : 0);
        GemmTask t = gemm(u12, b, lc1t, mC, dst, PD.mC, b, mC, p,
                          G_TRANS_A | G_NEG | (cinC ? G_CIN | G_CIN_OWN : 0), cinC ? D.cpt_bnd : nullptr, mC);
        t.crowmap = reinterpret_cast<const int32_t *>((intptr_t)rowsC_off[f]);  // rebased below
        add_tiles(gp, t);
      }
    }
    if (cz && F.sfront) {
      // S~[C range, B range] += LC1T^T U1B, in the first colour whose blocks
      // of this level it does not overlap
      const int r0 = H->cz.cC0[f], r1 = H->cz.cC1[f], k0 = H->cz.cB0[f], k1 = H->cz.cB1[f];
      GemmTask t = gemm(lc1t, mC, u1b, mB, P.czS + (int64_t)r0 * H->cz.MxB + k0, H->cz.MxB, mC, mB, p,
                        G_TRANS_A | G_C_ACC);
      std::vector<std::vector<GemmTask>> &cols = schL[lvl];
      int colour = -1;
      for (size_t c = 0; c < cols.size() && colour < 0; ++c) {
        bool clash = false;
        for (const GemmTask &o2 : cols[c]) {
          const int64_t off2 = o2.C - P.czS, rr0 = off2 / H->cz.MxB, kk0 = off2 % H->cz.MxB;
          if (rr0 < r1 && r0 < rr0 + o2.M && kk0 < k1 && k0 < kk0 + o2.N) { clash = true; break; }
        }
        if (!clash) colour = (int)c;
      }
      if (colour < 0) {
        cols.emplace_back();
        colour = (int)cols.size() - 1;
      }
      if (colour >= LevelTasks::kSchurColors) throw std::runtime_error("too many overlapping S~ blocks on one level");
      std::vector<GemmTask> tiles;
      add_tiles(tiles, t);
      // remember the block (one whole-block task) for the overlap test, and its tiles
      cols[colour].push_back(t);
      schTiles[lvl][colour].insert(schTiles[lvl][colour].end(), tiles.begin(), tiles.end());
    }
    if (q.ss_x12 >= 0) add_tiles(g2[lvl], gemm(tri, p, u12, b, P.R.ss + q.ss_x12, b, p, b, p, G_A_TRI_U));
    if (F.sweep) {
      if (b) add_tiles(g2[lvl], gemm(tri, p, u12, b, FSx(q.fs_x12), b, p, b, p, G_A_TRI_U));
      if (mB) add_tiles(g2[lvl], gemm(tri, p, u1b, mB, FSx(q.fs_x1b), mB, p, mB, p, G_A_TRI_U));
      if (b && !sym) add_tiles(g2[lvl], gemm(l21, p, tri, p, FSx(q.fs_z), p, b, p, p, G_B_TRI_L));
      if (b && sym) ztrL.push_back(TransTask{FSx(q.fs_x12), FSx(q.fs_z), nullptr, b, p, 0, b, p, 0});
      if (mC) add_tiles(g2[lvl], gemm(tri, p, lc1t, mC, P.xc + q.xoff, mC, p, mC, p, G_TRANS_A | G_A_TRI_L));
    }
    cm_factor += g_cmacs_acc;
    g_cmacs_acc = 0;
    // gradient sweeps (root to leaves), with F11^-1 = U^-1 L^-1 P^T:
    //   Y_f   = X1B_f - X12 Y_bnd
    //   Lam_f = P (XC1 G - Z^T Lam_bnd)      (rows scattered through perm)
    // The adjoint tiles also form the gradient partials Re(Lam Y) of their
    // design rows; fronts whose children do not take part in the sweeps do
    // not store Lam (nothing reads it).
    if (F.sweep) {
      const int ch = P.rhs_chunk;
      cplx *Xf = P.X + (int64_t)D.sweep_row0 * ch, *Vf = P.V + (int64_t)D.sweep_row0 * ch;
      const int32_t *bm = reinterpret_cast<const int32_t *>((intptr_t)bndrow_off[f]);  // rebased below
      GemmTask ty = gemm(b ? FSx(q.fs_x12) : nullptr, b, P.X, ch, Xf, ch, p, ch, b,
                         G_NEG | (mB ? G_CIN | (cz ? G_CIN_RANGE : G_CIN_COFF) : 0), mB ? FSx(q.fs_x1b) : nullptr, mB,
                         b ? bm : nullptr);
      if (cz && mB) {   // X1B holds the compressed columns [cB0, cB1) of the front
        ty.cin_c0 = H->cz.cB0[f];
        ty.cin_w = mB;
      }
      bool lam_read = false;
      for (int c = 0; c < F.nchild; ++c) lam_read = lam_read || S.fronts[F.child[c]].sweep;
      GemmTask tv = gemm(b ? FSx(q.fs_z) : nullptr, p, P.V, ch, Vf, ch, p, ch, b,
                         G_TRANS_A | G_NEG | (mC ? G_CIN : 0) | G_CONTRACT | (lam_read ? 0 : G_NO_STORE),
                         mC ? Vf : nullptr, ch, b ? bm : nullptr);
      tv.crowmap = perm;
      tv.aux = Xf;
      tv.auxmap = reinterpret_cast<const int32_t *>((intptr_t)(P.gidx + (int64_t)D.sweep_row0 * 4));  // rebased below
      if (wroot[f]) {
        // Wt = Y_bnd Lam_bnd^T over the right-hand-side columns (summed over
        // chunks): A = boundary rows of X, B = the same rows of V, both
        // k-contiguous; one task per root, written into the Wt columns of
        // the front's Bf
        if (b > 64) throw std::runtime_error("low-rank subtree root with more than 64 boundary nodes");
        GemmTask tw = gemm(P.X, ch, P.V, ch, P.lrW + bf_off[f] + p, n, b, b, ch, G_TRANS_B | G_K_LIM | G_ACC_CHUNK);
        tw.arowmap = bm;
        tw.browmap = bm;
        g_cmacs_acc += (double)b * b * ch;
        cm_w += (double)b * b * P.ncol;
        swW[lvl].push_back(tw);
      }
      if (wcov[f]) {
        // U1t = Wt Z into the first p columns of Bf; Qt = X12 [U1t | Wt]
        cplx *bf = P.lrW + bf_off[f], *qt = P.lrW + qt_off[f];
        const double acc0 = g_cmacs_acc;
        add_tiles(wuL[lvl], gemm(bf + p, n, FSx(q.fs_z), p, bf, n, b, p, b, 0));
        add_tiles(wqL[lvl], gemm(FSx(q.fs_x12), b, bf, n, qt, n, p, n, b, 0));
        cm_wprop += g_cmacs_acc - acc0;
        g_cmacs_acc = acc0;
        WFront W{};
        W.Qt = qt;
        W.Bf = bf;
        W.perm = perm;
        W.gidx = reinterpret_cast<const int32_t *>((intptr_t)(P.gidx + (int64_t)D.sweep_row0 * 4));  // rebased below
        W.p = p;
        W.b = b;
        for (int c = 0; c < F.nchild; ++c) {
          const int cf = F.child[c];
          if (!S.fronts[cf].sweep) continue;
          const int pc = S.fronts[cf].p(), bc = S.fronts[cf].b();
          W.pc[W.nch] = pc;
          W.bc[W.nch] = bc;
          W.dst[W.nch] = P.lrW + bf_off[cf] + pc;
          W.rmap[W.nch] = reinterpret_cast<const int32_t *>((intptr_t)rmap_off[cf]);  // rebased below
          ++W.nch;
        }
        wpL[lvl].push_back(W);
      } else {
        add_tiles(swY[lvl], ty);
        add_tiles(swL[lvl], tv);
      }
      if (mC)
        for (int k = 0; k < p; ++k) {   // V row of xc row xk + k: sweep_row0 + perm[k]
          vmap_base[q.xk + k] = D.sweep_row0;
          vmap_pidx[q.xk + k] = (int32_t)(F.elim0 + k);
        }
      if (mC && cz) {
        // compressed: the front's own weighted adjoint source, V rows of its
        // pivots = XC1 (p x mC) times rows [cC0, cC1) of dF/dS~ (the launch's
        // external operand, at element offset cC0 M'_B)
        GemmTask ti = gemm(P.xc + q.xoff, mC,
                           reinterpret_cast<const cplx *>((intptr_t)((int64_t)H->cz.cC0[f] * H->cz.MxB)),
                           H->cz.MxB, P.V, ch, p, ch, mC, G_B_EXT | G_B_COFF);
        ti.crowmap = P.vmap + q.xk;
        const double acc0 = g_cmacs_acc;
        add_tiles_xcd(vinit, ti);
        vinit_acc += g_cmacs_acc - acc0;
        g_cmacs_acc = acc0;
      }
    }
    cm_sweep += g_cmacs_acc * ((double)P.ncol / P.rhs_chunk);
  }
  // weighted adjoint source of every sweep front with C rows in one GEMM:
  // V[vmap[r]] = XC[r] G, rows scattered through the permutation map
  double cm_vinit = 0;
  if (cz) {
    cm_vinit = vinit_acc * ((double)P.ncol / P.rhs_chunk);
    cm_sweep += cm_vinit;
    P.vinit_cmacs = cm_vinit;
  } else if (P.xc_rows) {
    g_cmacs_acc = 0;
    GemmTask ti = gemm(P.xc, Mo, nullptr, Mi, P.V, P.rhs_chunk, (int)P.xc_rows, P.rhs_chunk, Mo, G_B_EXT | G_B_COFF);
    ti.crowmap = P.vmap;
    add_tiles_xcd(vinit, ti);
    cm_vinit = g_cmacs_acc * ((double)Mi / P.rhs_chunk);
    cm_sweep += cm_vinit;
    P.vinit_cmacs = cm_vinit;
  }
  P.gemm_cmacs_factor = cm_factor;
  P.gemm_cmacs_sweep = cm_sweep + cm_wprop;
  // S = sum over fronts holding both channel blocks of FC1 F11^-1 F1B
  //   = (U^-T FC1^T)^T (L^-1 P^T F1B) = SC^T SB,
  // split over k segments of SPLIT_K rows, each accumulated on MFMA (FP64,
  // or FP32 on the mixed path) into an FP64 partial block; one kernel sums
  // the blocks
  std::vector<GemmTask> gSsplit, czD1, czD2, czG1, czG2;
  P.nseg = cz ? 0 : (int)std::max<int64_t>(1, (ktot + SPLIT_K - 1) / SPLIT_K);
  if (!cz) HIPCHK(hipMalloc(&P.spart, (int64_t)P.nseg * Mo * Mi * sizeof(cplx)));
  g_cmacs_acc = 0;
  if (cz) {
    // S = D_C (S~ D_B)
    add_tiles_xcd(czD1, gemm(P.czS, H->cz.MxB, P.czDB, Mi, P.czT, Mi, H->cz.MxC, Mi, H->cz.MxB, G_K3));
    add_tiles_xcd(czD2, gemm(P.czDC, H->cz.MxC, P.czT, Mi, nullptr, Mi, Mo, Mi, H->cz.MxC, G_C_EXT | G_K3));
    if (P.czG) {
      // dF/dS~ = (D_C^T dF/dS) D_B^T
      add_tiles_xcd(czG1, gemm(P.czDC, H->cz.MxC, nullptr, Mi, P.czT2, Mi, H->cz.MxC, Mi, Mo,
                               G_TRANS_A | G_B_EXT | G_K3));
      add_tiles_xcd(czG2, gemm(P.czT2, Mi, P.czDBt, H->cz.MxB, P.czG, H->cz.MxB, H->cz.MxC, H->cz.MxB, Mi, G_K3));
    }
  }
  for (int g = 0; g < P.nseg; ++g) {
    const int64_t k0 = (int64_t)g * SPLIT_K;
    const int kk = (int)std::min<int64_t>(SPLIT_K, ktot - k0);
    add_tiles_xcd(gSsplit, gemm(P.sc + k0 * Mo, Mo, P.sb + k0 * Mi, Mi, P.spart + (int64_t)g * Mo * Mi, Mi, Mo, Mi,
                                std::max(kk, 0), G_TRANS_A));
  }
  P.gemm_cmacs_schur = g_cmacs_acc;

  // ---- assemble the blob ------------------------------------------------------
  Blob &bl = ib;  // continue after the integer arrays
  auto list_cmacs = [](const std::vector<GemmTask> &v) {
    double c = 0.0;
    for (const GemmTask &T : v) c += tile_cmacs(T, T.tm, T.tn);
    return c;
  };
  double cm_k3 = P.gemm_cmacs_schur + cm_vinit;   // always three-product
  for (int lvl = 0; lvl <= H_; ++lvl) {
    LevelTasks &L = P.lv[lvl];
    L.zero = bl.add(zr[lvl]); L.nzero = (int)zr[lvl].size();
    L.scat = bl.add(ae[lvl]); L.nscat = (int)ae[lvl].size();
    L.pan = bl.add(pe[lvl]); L.npan = (int)pe[lvl].size();
    L.cpy = bl.add(cpyL[lvl]); L.ncpy = (int)cpyL[lvl].size();
    for (int c = 0; c < LevelTasks::kSchurColors; ++c) {
      L.sch[c] = bl.add(schTiles[lvl][c]);
      L.nsch[c] = (int)schTiles[lvl][c].size();
    }
    L.deep1 = mark_deep(g1[lvl]);
    L.deep2 = mark_deep(g2[lvl]);
    L.deep2b = mark_deep(g2b[lvl]);
    L.nthin1 = split_thin(g1[lvl], &L.ntri1);
    L.nthin2 = split_thin(g2[lvl], &L.ntri2);
    L.nthin2b = split_thin(g2b[lvl], &L.ntri2b);
    // (tiles of a deep list that run thin take the four-product form)
    auto k3_cmacs = [&](const std::vector<GemmTask> &v, int nthin) {
      return list_cmacs(std::vector<GemmTask>(v.begin(), v.end() - nthin));
    };
    if (L.deep1) cm_k3 += k3_cmacs(g1[lvl], L.nthin1);
    if (L.deep2) cm_k3 += k3_cmacs(g2[lvl], L.nthin2);
    if (L.deep2b) cm_k3 += k3_cmacs(g2b[lvl], L.nthin2b);
    L.g1 = bl.add(g1[lvl]); L.ng1 = (int)g1[lvl].size();
    L.g2 = bl.add(g2[lvl]); L.ng2 = (int)g2[lvl].size();
    L.g2b = bl.add(g2b[lvl]); L.ng2b = (int)g2b[lvl].size();
    L.utr = bl.add(utrL[lvl]); L.nutr = (int)utrL[lvl].size();
  }
  P.ztr = bl.add(ztrL); P.nztr = (int)ztrL.size();
  P.swl.assign(H_ + 2, -1);
  P.nswl.assign(H_ + 2, 0);
  P.nswl_thin.assign(H_ + 2, 0);
  P.swl_deep.assign(H_ + 2, 0);
  for (int t = 0; t <= H_ + 1; ++t) {
    std::vector<GemmTask> m;
    if (H_ - t >= 0) m.insert(m.end(), swY[H_ - t].begin(), swY[H_ - t].end());
    if (H_ - t + 1 <= H_) m.insert(m.end(), swL[H_ - t + 1].begin(), swL[H_ - t + 1].end());
    P.swl_deep[t] = mark_deep(m);
    int ntri_sw = 0;
    P.nswl_thin[t] = split_thin(m, &ntri_sw);
    if (ntri_sw) throw std::runtime_error("triangular operand in a sweep list");
    if (P.swl_deep[t])
      cm_k3 += list_cmacs(std::vector<GemmTask>(m.begin(), m.end() - P.nswl_thin[t])) * ((double)Mi / P.rhs_chunk);
    P.swl[t] = bl.add(m);
    P.nswl[t] = (int)m.size();
  }
  P.swtb.assign(H_ + 2, -1);
  P.nswtb.assign(H_ + 2, 0);
  for (int t = 1; t <= H_ + 1; ++t) {
    P.swtb[t] = bl.add(swW[H_ - t + 1]);
    P.nswtb[t] = (int)swW[H_ - t + 1].size();
  }
  P.wu.assign(H_ + 1, -1); P.wq.assign(H_ + 1, -1); P.wp.assign(H_ + 1, -1);
  P.nwu.assign(H_ + 1, 0); P.nwq.assign(H_ + 1, 0); P.nwp.assign(H_ + 1, 0);
  P.wu_deep.assign(H_ + 1, 0); P.wq_deep.assign(H_ + 1, 0);
  for (int l = 0; l <= H_; ++l) {
    P.wu_deep[l] = mark_deep(wuL[l]);
    P.wq_deep[l] = mark_deep(wqL[l]);
    if (P.wu_deep[l]) cm_k3 += list_cmacs(wuL[l]);
    if (P.wq_deep[l]) cm_k3 += list_cmacs(wqL[l]);
    P.wu[l] = bl.add(wuL[l]); P.nwu[l] = (int)wuL[l].size();
    P.wq[l] = bl.add(wqL[l]); P.nwq[l] = (int)wqL[l].size();
    P.wp[l] = bl.add(wpL[l]); P.nwp[l] = (int)wpL[l].size();
  }
  // the Schur partials and the weighted adjoint source are K_total / M_out
  // deep: always the three-product form
  for (GemmTask &T : gSsplit) T.flags |= G_K3;
  for (GemmTask &T : vinit) T.flags |= G_K3;
  P.gemm_cmacs_k3 = cm_k3 + cm_w;
  P.gemm_cmacs_w = cm_w;
  P.gSsplit = bl.add(gSsplit); P.ngSsplit = (int)gSsplit.size();
  P.czD1 = bl.add(czD1); P.nczD1 = (int)czD1.size();
  P.czD2 = bl.add(czD2); P.nczD2 = (int)czD2.size();
  P.czG1 = bl.add(czG1); P.nczG1 = (int)czG1.size();
  P.czG2 = bl.add(czG2); P.nczG2 = (int)czG2.size();
  P.vinit = bl.add(vinit); P.nvinit = (int)vinit.size();
  P.vmap_base = bl.add(vmap_base);
  P.vmap_pidx = bl.add(vmap_pidx);
  P.fronts = bl.add(fd);
  P.nfronts = nf;
  HIPCHK(hipMalloc(&P.blob, bl.h.size()));
  base = P.blob;
  {
    auto reg = [&](int64_t off, int n, char *deep) -> int {
      if (n <= 0) return -1;
      P.tl.push_back({P.blob, off, n, deep});
      return (int)P.tl.size() - 1;
    };
    for (LevelTasks &L : P.lv) {
      L.id1 = reg(L.g1, L.ng1, &L.deep1);
      L.id2 = reg(L.g2, L.ng2, &L.deep2);
      L.id2b = reg(L.g2b, L.ng2b, &L.deep2b);
    }
    P.swl_id.assign(P.swl.size(), -1);
    for (size_t t = 0; t < P.swl.size(); ++t) P.swl_id[t] = reg(P.swl[t], P.nswl[t], &P.swl_deep[t]);
    P.vinit_id = reg(P.vinit, P.nvinit, &P.vinit_deep);
    P.schur_id = reg(P.gSsplit, P.ngSsplit, &P.schur_deep);
    P.wu_id.assign(P.wu.size(), -1);
    P.wq_id.assign(P.wq.size(), -1);
    for (size_t l = 0; l < P.wu.size(); ++l) {
      P.wu_id[l] = reg(P.wu[l], P.nwu[l], &P.wu_deep[l]);
      P.wq_id[l] = reg(P.wq[l], P.nwq[l], &P.wq_deep[l]);
    }
  }
  // rebase the pointers into the integer section
  auto rebase = [&](const int32_t *&ptr) {
    if (ptr) ptr = reinterpret_cast<const int32_t *>(base + (intptr_t)ptr);
  };
  {
    FrontDev *fdv = reinterpret_cast<FrontDev *>(bl.h.data() + P.fronts);
    for (int f = 0; f < nf; ++f) {
      if (rmap_off[f] >= 0) rebase(fdv[f].rmap);
      else fdv[f].rmap = nullptr;
    }
    // (an empty list and the next one can share an offset: take each list's
    // own count, never look the count up by offset)
    for (int lvl = 0; lvl <= H_; ++lvl)
      for (int which = 0; which < 2; ++which) {
        const LevelTasks &L = P.lv[lvl];
        GemmTask *t = reinterpret_cast<GemmTask *>(bl.h.data() + (which ? L.g2b : L.g2));
        const int n = which ? L.ng2b : L.ng2;
        for (int k = 0; k < n; ++k) {
          rebase(t[k].crowmap);
          rebase(t[k].ccolmap);
        }
      }
    for (size_t l = 0; l < P.swl.size(); ++l) {
      GemmTask *t = reinterpret_cast<GemmTask *>(bl.h.data() + P.swl[l]);
      for (int k = 0; k < P.nswl[l]; ++k) {
        rebase(t[k].browmap);
        rebase(t[k].auxmap);
      }
      if (P.nswtb[l] > 0) {
        GemmTask *w = reinterpret_cast<GemmTask *>(bl.h.data() + P.swtb[l]);
        for (int k = 0; k < P.nswtb[l]; ++k) {
          rebase(w[k].browmap);
          rebase(w[k].arowmap);
        }
      }
    }
    for (int l = 0; l <= H_; ++l) {
      WFront *wf = reinterpret_cast<WFront *>(bl.h.data() + P.wp[l]);
      for (int k = 0; k < P.nwp[l]; ++k) {
        rebase(wf[k].gidx);
        for (int c = 0; c < wf[k].nch; ++c) rebase(wf[k].rmap[c]);
      }
    }
  }
  (void)ib_size;
  HIPCHK(hipMemcpy(P.blob, bl.h.data(), bl.h.size(), hipMemcpyHostToDevice));
  if (H->refine_iters > 0) build_refine(H);
  H->planned = true;
}

static void free_plan(Plan &P) {
  const Refine &R = P.R;
  void *ptrs[] = {P.ws, P.fs, P.sb, P.sc, P.X, P.V, P.aval, P.blob, P.status, P.pivq, P.part, P.perms, P.chan, P.spart,
                  P.xc, P.vmap, P.gpart, P.lrW, P.g_nnz, P.g_max, P.g_idx, P.g_val, P.czBt, P.czCt, P.czS,
                  P.czDB, P.czDC, P.czT, P.czG, P.czT2, P.czDBt, R.ss, R.X, R.W, R.arena, R.Bmat, R.Cmat, R.rowbuf, R.Ydes,
                  R.elim, R.norms, R.blob};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  P = Plan();
}

template <class F>
static apf_status guarded(F &&fn) {
  try {
    return fn();
  } catch (const HipError &e) {
    return fail(APF_EHIP, e.what());
  } catch (const std::bad_alloc &) {
    return fail(APF_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(APF_EINVAL, e.what());
  }
}

extern "C" apf_status apf_assemble(apf_handle *h, const double *eps_dev, void *stream) {
  if (!h || !eps_dev) return fail(APF_EINVAL, "null argument");
  if (!h->analyzed) return fail(APF_ESTATE, "apf_analyze has not run");
  return guarded([&]() -> apf_status {
    hipStream_t s = (hipStream_t)stream;
    if (!h->planned) {
      try {
        build_plan(h);
      } catch (...) {
        free_plan(h->plan);
        throw;
      }
    }
    Profiler &pr = h->prof;
    HIPCHK(launch_fill_int(h->plan.status + 1, 0, s));
    pr.run(P_STENCIL, s, [&] { return launch_stencil(h->phys, eps_dev, h->plan.aval, h->plan.status + 1, s); });
    if (pr.on) pr.collect();
    h->state = 1;
    return APF_OK;
  });
}

// The level loop of the numeric factorization (leaves to root): zero the
// level's workspaces, scatter A, generate the channel rows, extend-add the
// children (two slots: siblings never share a launch), factor the pivot
// blocks, then the two GEMM phases.  `blob` holds the task arrays that `lv`
// indexes; `fr` the front descriptors.
static void run_levels(const std::vector<LevelTasks> &lv, char *blob, const FrontDev *fr, int *status,
                       Profiler &pr, hipStream_t s, bool f32, const std::vector<AugLevel> *aug = nullptr,
                       char *ablob = nullptr, double *pivq = nullptr, bool sym = false) {
  auto at = [&](int64_t off) -> char * { return off < 0 ? nullptr : blob + off; };
  auto aat = [&](int64_t off) -> char * { return off < 0 ? nullptr : ablob + off; };
  for (size_t lvl = 0; lvl < lv.size(); ++lvl) {
    const LevelTasks &L = lv[lvl];
    const AugLevel *A = (aug && lvl < aug->size()) ? &(*aug)[lvl] : nullptr;
    pr.run(P_ZERO, s, [&] { return launch_zero((const ZeroRange *)at(L.zero), L.nzero, s); });
    if (A) {
      pr.run(P_ZERO, s, [&] {
        hipError_t e = launch_zero((const ZeroRange *)aat(A->zero), A->nzero, s);
        if (e == hipSuccess) e = launch_set_one((cplx *const *)aat(A->one), A->none, s);
        return e;
      });
    }
    pr.run(P_ASSEMBLE, s, [&] {
      hipError_t e = launch_scatter_A((const AsmEntry *)at(L.scat), L.nscat, s);
      if (e == hipSuccess) e = launch_assemble_panel((const PanelEntry *)at(L.pan), L.npan, s);
      if (e == hipSuccess) e = launch_copy((const CopyRange *)at(L.cpy), L.ncpy, s);
      return e;
    });
    pr.run(P_INVERSE, s, [&] {
      hipError_t e = hipSuccess;
      for (int v = 0; v < N_INV_VARIANTS && e == hipSuccess; ++v)
        e = launch_inverse(v, fr, (const int32_t *)at(L.inv[v]), L.ninv[v], status, pivq, sym ? 1 : 0, s);
      return e;
    });
    // (empty task lists launch nothing and are not counted)
    for (int g = 0; g < 3; ++g) {
      const int64_t off = g == 0 ? L.g1 : (g == 1 ? L.g2 : L.g2b);
      const int n = g == 0 ? L.ng1 : (g == 1 ? L.ng2 : L.ng2b);
      const bool deep = (g == 0 ? L.deep1 : (g == 1 ? L.deep2 : L.deep2b)) != 0;
      const int nthin = g == 0 ? L.nthin1 : (g == 1 ? L.nthin2 : L.nthin2b);
      const int ntri = g == 0 ? L.ntri1 : (g == 1 ? L.ntri2 : L.ntri2b);
      pr.cur_tag = g == 0 ? L.id1 : (g == 1 ? L.id2 : L.id2b);
      if (n > 0)
        pr.run(P_GEMM_FACTOR, s, [&] {
          return launch_gemm((const GemmTask *)at(off), n, 0, INT_MAX, nullptr, s, f32, nullptr, 0, deep, nthin,
                             ntri);
        }, gemm_kernel_launches(n, nthin, ntri, f32));
      pr.cur_tag = -1;
      if (g == 0 && L.nutr > 0)
        pr.run(P_GEMM_FACTOR, s, [&] { return launch_transpose_scale((const TransTask *)at(L.utr), L.nutr, s); });
      // the augmented panels' products after the main phase 1 (their inputs)
      // and phase 2 (no dependence either way)
      if (A && g < 2) {
        const int64_t ao = g == 0 ? A->g1 : A->g2;
        const int an = g == 0 ? A->ng1 : A->ng2;
        if (an > 0)
          pr.run(P_GEMM_FACTOR, s, [&] { return launch_gemm((const GemmTask *)aat(ao), an, 0, INT_MAX, nullptr, s, f32); });
      }
    }
    // compressed channels: the level's blocks of S~, one launch per colour
    for (int c = 0; c < LevelTasks::kSchurColors; ++c)
      if (L.nsch[c] > 0)
        pr.run(P_GEMM_SCHUR, s, [&] { return launch_gemm((const GemmTask *)at(L.sch[c]), L.nsch[c], 0, INT_MAX, nullptr, s, f32); });
  }
}

// The channel-by-channel Schur block S = SC^T SB: partial products over k
// segments (FP64 MFMA, or FP32 MFMA on the mixed path) summed in FP64.
static void enqueue_schur(const Plan &P, bool f32, double *S_dev, Profiler &pr, hipStream_t s, int Mo, int Mi) {
  // k split into segments of SPLIT_K rows: shorter, more numerous tasks than
  // one K_total-deep tile each, summed in FP64 afterwards
  pr.cur_tag = P.schur_id;
  pr.run(P_GEMM_SCHUR, s, [&] {
    hipError_t e = launch_gemm(P.at<GemmTask>(P.gSsplit), P.ngSsplit, 0, INT_MAX, nullptr, s, f32, nullptr, 0,
                               P.schur_deep != 0);
    if (e == hipSuccess)
      e = launch_sum_partials(P.spart, P.nseg, (int64_t)Mo * Mi, reinterpret_cast<cplx *>(S_dev), (int64_t)Mo * Mi, s);
    return e;
  });
  pr.cur_tag = -1;
}

// One refined solve of the chunk's right-hand sides, in place on R.W:
// forward through the fronts' local panels (leaves to root), then back
// substitution (root to leaves).  FP32 MFMA with the mixed factors.
static void refine_solve(const Plan &P, int w, Profiler &pr, hipStream_t s) {
  const Refine &R = P.R;
  pr.run(P_REFINE, s, [&] {
    hipError_t e = hipSuccess;
    for (size_t lvl = 0; lvl < R.lv.size() && e == hipSuccess; ++lvl) {
      const RefineLevel &L = R.lv[lvl];
      e = launch_zero(R.at<ZeroRange>(L.zero), L.nzero, s);
      if (e == hipSuccess) e = launch_copy(R.at<CopyRange>(L.copy), L.ncopy, s);
      if (e == hipSuccess) e = launch_gemm(R.at<GemmTask>(L.g1), L.ng1, 0, w, nullptr, s, true);
      if (e == hipSuccess) e = launch_gemm(R.at<GemmTask>(L.g2), L.ng2, 0, w, nullptr, s, true);
      if (e == hipSuccess) e = launch_gemm(R.at<GemmTask>(L.g2b), L.ng2b, 0, w, nullptr, s, true);
    }
    for (int lvl = (int)R.lv.size() - 1; lvl >= 0 && e == hipSuccess; --lvl)
      e = launch_gemm(R.at<GemmTask>(R.lv[lvl].bk), R.lv[lvl].nbk, 0, w, nullptr, s, true);
    return e;
  });
}

// Refined fields of one right-hand-side chunk (w columns), into R.X:
//   X = solve(r); then `iters` times: W = r - A X (FP64), X += solve(W);
// finally the residual once more for the convergence check.  r is zero
// except on grid row rrow (entries rb[i * ldr + coff + j]).  Squared norms:
// slot 0 |r|^2, slot k the residual after k solves.
static void refine_fields(apf_handle *h, int rrow, const cplx *rb, int ldr, int coff, int w, int chunk,
                          hipStream_t s) {
  Plan &P = h->plan;
  Refine &R = P.R;
  Profiler &pr = h->prof;
  const int nx = h->d.nx, ny = h->d.ny;
  const int64_t N = (int64_t)nx * ny;
  double *nrm = R.norms + (int64_t)chunk * (R.iters + 2);
  auto residual = [&](bool first, int slot) {
    pr.run(P_REFINE, s, [&] {
      return launch_residual(nx, ny, R.elim, P.aval, R.X, R.W, R.rc, w, rrow, rb, ldr, coff, first, nrm + slot, s);
    });
  };
  residual(true, 0);
  refine_solve(P, w, pr, s);
  pr.run(P_REFINE, s, [&] { return launch_add_fields(R.X, R.W, N, R.rc, w, true, s); });
  for (int it = 1; it <= R.iters; ++it) {
    residual(false, it);
    refine_solve(P, w, pr, s);
    pr.run(P_REFINE, s, [&] { return launch_add_fields(R.X, R.W, N, R.rc, w, false, s); });
  }
  residual(false, R.iters + 1);
}

static std::string sci(double v) {
  char b[32];
  std::snprintf(b, sizeof b, "%.3e", v);
  return b;
}

// Largest final and first relative residual over the chunks of the last
// refined call (after the stream was synchronised).
static void refine_residuals(Refine &R) {
  std::vector<double> v((size_t)R.nchunks * (R.iters + 2));
  HIPCHK(hipMemcpy(v.data(), R.norms, v.size() * sizeof(double), hipMemcpyDeviceToHost));
  R.last_res = R.last_res1 = 0.0;
  for (int c = 0; c < R.nchunks; ++c) {
    const double *n = v.data() + (size_t)c * (R.iters + 2);
    if (!(n[0] > 0.0)) continue;
    R.last_res = std::max(R.last_res, std::sqrt(n[R.iters + 1] / n[0]));
    R.last_res1 = std::max(R.last_res1, std::sqrt(n[1] / n[0]));
  }
}

extern "C" apf_status apf_factor_schur(apf_handle *h, apf_precision prec, double *S_dev, void *stream) {
  if (!h || !S_dev) return fail(APF_EINVAL, "null argument");
  if (prec != APF_FP64 && prec != APF_MIXED && prec != APF_MIXED_REFINED) return fail(APF_EINVAL, "unknown precision");
  if (h->state < 1) return fail(APF_ESTATE, "apf_assemble has not run");
  if (h->symmetric && prec != APF_FP64) return fail(APF_EINVAL, "the symmetric route runs in FP64 only");
  const bool refine = prec == APF_MIXED_REFINED;
  if (refine && h->refine_iters <= 0)
    return fail(APF_ESTATE, "APF_MIXED_REFINED needs apf_set_refinement before the first apf_assemble");
  if (refine && h->cz.pad >= 0) return fail(APF_EINVAL, "APF_MIXED_REFINED does not combine with compressed channels");
  return guarded([&]() -> apf_status {
    hipStream_t s = (hipStream_t)stream;
    Plan &P = h->plan;
    Profiler &pr = h->prof;
    const bool f32 = prec != APF_FP64;
    const int Mi = h->d.n_in;
    HIPCHK(launch_fill_int(P.status, 0, s));
    const bool cz = h->cz.pad >= 0;
    if (cz) HIPCHK(launch_zero_flat(P.czS, (int64_t)h->cz.MxC * h->cz.MxB, s));
    run_levels(P.lv, P.blob, P.at<FrontDev>(P.fronts), P.status, pr, s, f32, nullptr, nullptr, P.pivq, P.sym);
    if (P.nztr > 0)
      pr.run(P_GEMM_FACTOR, s, [&] { return launch_transpose_scale(P.at<TransTask>(P.ztr), P.nztr, s); });
    if (cz) {
      // decompression: S = D_C (S~ D_B), FP64
      pr.run(P_GEMM_SCHUR, s, [&] {
        hipError_t e = launch_gemm(P.at<GemmTask>(P.czD1), P.nczD1, 0, INT_MAX, nullptr, s, false, nullptr, 0, true);
        if (e == hipSuccess)
          e = launch_gemm(P.at<GemmTask>(P.czD2), P.nczD2, 0, INT_MAX, reinterpret_cast<const cplx *>(S_dev), s,
                          false, nullptr, 0, true);
        return e;
      });
    } else if (!refine) {
      enqueue_schur(P, f32, S_dev, pr, s, h->d.n_out, Mi);
    } else {
      // S from refined forward fields, chunk by chunk; their design rows are
      // kept for apf_grad
      Refine &R = P.R;
      HIPCHK(launch_fill_double(R.norms, R.nchunks * (R.iters + 2), 0.0, s));
      for (int c = 0; c < R.nchunks; ++c) {
        const int m0 = c * R.rc, w = std::min(R.rc, Mi - m0);
        refine_fields(h, h->d.src_row, R.Bmat, Mi, m0, w, c, s);
        pr.run(P_GEMM_SCHUR, s, [&] {
          return launch_gemm(R.at<GemmTask>(R.sgemm), R.nsgemm, m0, w, reinterpret_cast<const cplx *>(S_dev), s,
                             false, nullptr, 0, true);
        });
        pr.run(P_REFINE, s, [&] {
          return launch_gather_rows(R.at<int32_t>(R.erow_des), P.ndesign, R.X, R.rc, w, R.Ydes, Mi, m0, s);
        });
      }
    }
    int st[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(st, P.status, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (pr.on) pr.collect();
    ++h->n_factor;
    if (st[1] & ST_BAD_EPS) {
      h->state = 0;
      return fail(APF_EINVAL, "the permittivity has a zero or non-finite value");
    }
    if (st[0]) {
      h->state = 0;
      return fail(APF_ESINGULAR, "zero or non-finite pivot in a pivot block");
    }
    h->state = 2;
    h->mixed = f32;
    h->refined = refine;
    if (refine) {
      refine_residuals(P.R);
      if (!(P.R.last_res <= P.R.tol))
        return fail(APF_ENOTCONV, "refinement of the forward fields ended at relative residual " +
                                      sci(P.R.last_res) + " (first solve " + sci(P.R.last_res1) + ")");
    }
    return APF_OK;
  });
}

// ---------------------------------------------------------------------------
// Batched factorization of several independent problems: the level lists of
// every handle are concatenated (level = height above the leaves), so each
// level of the whole batch is one launch per kernel; repeated calls with the
// same handles and outputs replay a captured HIP graph of that sequence.
// ---------------------------------------------------------------------------
namespace {

struct BatchPlan {
  std::vector<apf_handle *> hs;
  std::vector<LevelTasks> lv;
  char *blob = nullptr;
  int64_t fronts = -1;
  int *status = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;       // private stream the graph is captured on
  std::vector<double *> graph_S;   // outputs the graph was captured with
  bool graph_f32 = false;          // and its precision
  std::vector<TunableList> tl;     // the merged factorization lists
  ~BatchPlan() {
    if (cap) (void)hipStreamDestroy(cap);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (blob) (void)hipFree(blob);
    if (status) (void)hipFree(status);
  }
};

std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchPlan>> g_batches;

template <class T>
std::vector<T> fetch(const char *blob, int64_t off, int n) {
  std::vector<T> v(n);
  if (n) HIPCHK(hipMemcpy(v.data(), blob + off, n * sizeof(T), hipMemcpyDeviceToHost));
  return v;
}

std::unique_ptr<BatchPlan> build_batch(const std::vector<apf_handle *> &hs) {
  auto B = std::make_unique<BatchPlan>();
  B->hs = hs;
  size_t nl = 0;
  for (apf_handle *h : hs) nl = std::max(nl, h->plan.lv.size());
  Blob bl;
  {
    const char pad[16] = {0};
    bl.add(pad, sizeof pad);
  }
  std::vector<FrontDev> fd;
  std::vector<int> base(hs.size());
  for (size_t i = 0; i < hs.size(); ++i) {
    const Plan &P = hs[i]->plan;
    base[i] = (int)fd.size();
    std::vector<FrontDev> f = fetch<FrontDev>(P.blob, P.fronts, P.nfronts);
    for (FrontDev &x : f)
      if (x.parent >= 0) x.parent += base[i];
    fd.insert(fd.end(), f.begin(), f.end());
  }
  B->lv.assign(nl, LevelTasks());
  for (size_t lvl = 0; lvl < nl; ++lvl) {
    std::vector<ZeroRange> zr;
    std::vector<AsmEntry> ae;
    std::vector<PanelEntry> pe;
    std::vector<int32_t> inv[N_INV_VARIANTS];
    std::vector<GemmTask> g1, g2, g2b;
    for (size_t i = 0; i < hs.size(); ++i) {
      const Plan &P = hs[i]->plan;
      if (lvl >= P.lv.size()) continue;
      const LevelTasks &L = P.lv[lvl];
      auto z = fetch<ZeroRange>(P.blob, L.zero, L.nzero); zr.insert(zr.end(), z.begin(), z.end());
      auto a = fetch<AsmEntry>(P.blob, L.scat, L.nscat); ae.insert(ae.end(), a.begin(), a.end());
      auto pp = fetch<PanelEntry>(P.blob, L.pan, L.npan); pe.insert(pe.end(), pp.begin(), pp.end());
      for (int v = 0; v < N_INV_VARIANTS; ++v)
        for (int32_t k : fetch<int32_t>(P.blob, L.inv[v], L.ninv[v])) inv[v].push_back(k + base[i]);
      auto t1 = fetch<GemmTask>(P.blob, L.g1, L.ng1); g1.insert(g1.end(), t1.begin(), t1.end());
      auto t2 = fetch<GemmTask>(P.blob, L.g2, L.ng2); g2.insert(g2.end(), t2.begin(), t2.end());
      auto t3 = fetch<GemmTask>(P.blob, L.g2b, L.ng2b); g2b.insert(g2b.end(), t3.begin(), t3.end());
    }
    LevelTasks &L = B->lv[lvl];
    L.zero = bl.add(zr); L.nzero = (int)zr.size();
    L.scat = bl.add(ae); L.nscat = (int)ae.size();
    L.pan = bl.add(pe); L.npan = (int)pe.size();
    for (int v = 0; v < N_INV_VARIANTS; ++v) { L.inv[v] = bl.add(inv[v]); L.ninv[v] = (int)inv[v].size(); }
    L.nthin1 = split_thin(g1, &L.ntri1);
    L.nthin2 = split_thin(g2, &L.ntri2);
    L.nthin2b = split_thin(g2b, &L.ntri2b);
    L.g1 = bl.add(g1); L.ng1 = (int)g1.size();
    L.g2 = bl.add(g2); L.ng2 = (int)g2.size();
    L.g2b = bl.add(g2b); L.ng2b = (int)g2b.size();
    L.deep1 = any_k3(g1);
    L.deep2 = any_k3(g2);
    L.deep2b = any_k3(g2b);
  }
  B->fronts = bl.add(fd);
  HIPCHK(hipMalloc(&B->blob, bl.h.size()));
  for (LevelTasks &L : B->lv) {
    auto reg = [&](int64_t off, int n, char *deep) -> int {
      if (n <= 0) return -1;
      B->tl.push_back({B->blob, off, n, deep});
      return (int)B->tl.size() - 1;
    };
    L.id1 = reg(L.g1, L.ng1, &L.deep1);
    L.id2 = reg(L.g2, L.ng2, &L.deep2);
    L.id2b = reg(L.g2b, L.ng2b, &L.deep2b);
  }
  HIPCHK(hipMemcpy(B->blob, bl.h.data(), bl.h.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMalloc(&B->status, sizeof(int)));
  return B;
}

void enqueue_batch(BatchPlan &B, double *const *S_devs, Profiler &pr, hipStream_t s, bool f32) {
  HIPCHK(launch_fill_int(B.status, 0, s));
  run_levels(B.lv, B.blob, reinterpret_cast<const FrontDev *>(B.blob + B.fronts), B.status, pr, s, f32);
  for (size_t i = 0; i < B.hs.size(); ++i)
    enqueue_schur(B.hs[i]->plan, f32, S_devs[i], pr, s, B.hs[i]->d.n_out, B.hs[i]->d.n_in);
}

void forget_batches_of(apf_handle *h) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batches.erase(std::remove_if(g_batches.begin(), g_batches.end(),
                                 [&](const std::unique_ptr<BatchPlan> &b) {
                                   return std::find(b->hs.begin(), b->hs.end(), h) != b->hs.end();
                                 }),
                  g_batches.end());
}

}  // namespace

extern "C" apf_status apf_factor_schur_batched(apf_handle *const *hs, int32_t n, apf_precision prec,
                                               double *const *S_devs, void *stream) {
  if (!hs || !S_devs || n < 1) return fail(APF_EINVAL, "need at least one handle and output");
  if (prec == APF_MIXED_REFINED) return fail(APF_EINVAL, "the batched factorization has no refined precision");
  if (prec != APF_FP64 && prec != APF_MIXED) return fail(APF_EINVAL, "unknown precision");
  const bool f32 = prec == APF_MIXED;
  std::vector<apf_handle *> v(hs, hs + n);
  for (int i = 0; i < n; ++i) {
    if (!hs[i] || !S_devs[i]) return fail(APF_EINVAL, "null handle or output");
    if (hs[i]->state < 1) return fail(APF_ESTATE, "apf_assemble has not run on every handle");
    if (hs[i]->cz.pad >= 0) return fail(APF_EINVAL, "compressed channels are not batched");
    if (hs[i]->symmetric) return fail(APF_EINVAL, "the symmetric route is not batched");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(APF_EINVAL, "a handle appears twice in the batch");
  }
  return guarded([&]() -> apf_status {
    hipStream_t s = (hipStream_t)stream;
    BatchPlan *B = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_batch_mu);
      for (auto &b : g_batches)
        if (b->hs == v) B = b.get();
      if (!B) {
        g_batches.push_back(build_batch(v));
        B = g_batches.back().get();
      }
    }
    Profiler &pr = hs[0]->prof;
    const std::vector<double *> Sv(S_devs, S_devs + n);
    if (pr.on) {
      enqueue_batch(*B, S_devs, pr, s, f32);   // timed launches are not captured
    } else {
      if (!B->exec || B->graph_S != Sv || B->graph_f32 != f32) {
        if (B->exec) { HIPCHK(hipGraphExecDestroy(B->exec)); B->exec = nullptr; }
        if (B->graph) { HIPCHK(hipGraphDestroy(B->graph)); B->graph = nullptr; }
        // capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph is then launched on `s`
        if (!B->cap) HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
        try {
          enqueue_batch(*B, S_devs, pr, B->cap, f32);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(B->cap, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIPCHK(hipStreamEndCapture(B->cap, &B->graph));
        HIPCHK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
        B->graph_S = Sv;
        B->graph_f32 = f32;
      }
      HIPCHK(hipGraphLaunch(B->exec, s));
    }
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, B->status, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (pr.on) pr.collect();
    int bad_eps = -1;
    for (int i = 0; i < n && bad_eps < 0; ++i) {
      int e = 0;
      HIPCHK(hipMemcpy(&e, hs[i]->plan.status + 1, sizeof(int), hipMemcpyDeviceToHost));
      if (e & ST_BAD_EPS) bad_eps = i;
    }
    for (int i = 0; i < n; ++i) {
      hs[i]->state = (st || bad_eps >= 0) ? 0 : 2;
      hs[i]->mixed = f32;
      hs[i]->refined = false;
      ++hs[i]->n_factor;
    }
    if (bad_eps >= 0)
      return fail(APF_EINVAL, "the permittivity of problem " + std::to_string(bad_eps) +
                                  " of the batch has a zero or non-finite value");
    if (st) return fail(APF_ESINGULAR, "zero or non-finite pivot in a pivot block of the batch");
    return APF_OK;
  });
}

extern "C" apf_status apf_weighted_power(apf_handle *h, const double *S_dev, const double *w_dev, double *f_dev,
                                         double *dfdS_dev, void *stream) {
  if (!h || !S_dev || !w_dev || !f_dev || !dfdS_dev) return fail(APF_EINVAL, "null argument");
  if (!h->planned) return fail(APF_ESTATE, "apf_assemble has not run");
  return guarded([&]() -> apf_status {
    int64_t n = (int64_t)h->d.n_in * h->d.n_out;
    int npart = weighted_power_parts(n);
    hipStream_t s = (hipStream_t)stream;
    Profiler &pr = h->prof;
    pr.run(P_WPOW, s, [&] {
      return launch_weighted_power(reinterpret_cast<const cplx *>(S_dev), w_dev, f_dev,
                                   reinterpret_cast<cplx *>(dfdS_dev), n, h->plan.part, npart, s);
    });
    if (pr.on) pr.collect();
    return APF_OK;
  });
}

extern "C" apf_status apf_splitter_fom(apf_handle *h, const double *S_dev, double t1, double *f_dev,
                                       double *dfdS_dev, void *stream) {
  if (!h || !S_dev || !f_dev || !dfdS_dev) return fail(APF_EINVAL, "null argument");
  if (!h->planned) return fail(APF_ESTATE, "apf_assemble has not run");
  return guarded([&]() -> apf_status {
    const int Mi = h->d.n_in, Mo = h->d.n_out;
    const int64_t n = (int64_t)Mi * Mo;
    const int npart = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipStream_t s = (hipStream_t)stream;
    const int32_t *in_ord = reinterpret_cast<const int32_t *>(h->plan.chan + 2 * sizeof(ChanParams));
    Profiler &pr = h->prof;
    pr.run(P_WPOW, s, [&] {
      return launch_splitter_fom(reinterpret_cast<const cplx *>(S_dev), in_ord, in_ord + Mi, Mi, Mo, t1, f_dev,
                                 reinterpret_cast<cplx *>(dfdS_dev), h->plan.part, npart, s);
    });
    if (pr.on) pr.collect();
    return APF_OK;
  });
}

extern "C" apf_status apf_group_fom(apf_handle *h, const double *S_dev, int32_t delta, int32_t gmax, double *f_dev,
                                    double *dfdS_dev, void *stream) {
  if (!h || !S_dev || !f_dev || !dfdS_dev) return fail(APF_EINVAL, "null argument");
  if (delta <= 0 || gmax < 0) return fail(APF_EINVAL, "delta must be positive and gmax non-negative");
  if (!h->planned) return fail(APF_ESTATE, "apf_assemble has not run");
  return guarded([&]() -> apf_status {
    const int Mi = h->d.n_in, Mo = h->d.n_out;
    if ((Mi + 255) / 256 > 1024) return fail(APF_EINVAL, "more than 262,144 inputs");
    hipStream_t s = (hipStream_t)stream;
    const int32_t *in_ord = reinterpret_cast<const int32_t *>(h->plan.chan + 2 * sizeof(ChanParams));
    Profiler &pr = h->prof;
    pr.run(P_WPOW, s, [&] {
      return launch_group_fom(reinterpret_cast<const cplx *>(S_dev), in_ord, in_ord + Mi, Mi, Mo, delta, gmax,
                              f_dev, reinterpret_cast<cplx *>(dfdS_dev), h->plan.part, s);
    });
    if (pr.on) pr.collect();
    return APF_OK;
  });
}

static apf_status check_ridges(apf_handle *h, const double *edges_dev, int32_t n_edges, int32_t mirror) {
  if (!h || !edges_dev) return fail(APF_EINVAL, "null argument");
  if (mirror != 0 && mirror != 1) return fail(APF_EINVAL, "mirror must be 0 or 1");
  if (n_edges <= 0 || ((mirror ? 2 * (int64_t)n_edges : n_edges) % 2) != 0)
    return fail(APF_EINVAL, "the edges of the period must form pairs");
  if (h->d.design_row1 <= h->d.design_row0) return fail(APF_EINVAL, "no design rows");
  return APF_OK;
}

extern "C" apf_status apf_ridges_eps(apf_handle *h, const double *edges_dev, int32_t n_edges, int32_t mirror,
                                     double eps_ridge, double eps_gap, double *eps_dev, void *stream) {
  if (apf_status st = check_ridges(h, edges_dev, n_edges, mirror)) return st;
  if (!eps_dev) return fail(APF_EINVAL, "null argument");
  return guarded([&]() -> apf_status {
    HIPCHK(launch_ridges_eps(edges_dev, n_edges, mirror, h->d.nx, h->d.design_row0,
                             h->d.design_row1 - h->d.design_row0, eps_ridge, eps_gap, eps_dev, (hipStream_t)stream));
    return APF_OK;
  });
}

extern "C" apf_status apf_ridges_grad(apf_handle *h, const double *edges_dev, int32_t n_edges, int32_t mirror,
                                      double eps_ridge, double eps_gap, const double *grad_eps_dev,
                                      double *grad_edges_dev, void *stream) {
  if (apf_status st = check_ridges(h, edges_dev, n_edges, mirror)) return st;
  if (!grad_eps_dev || !grad_edges_dev) return fail(APF_EINVAL, "null argument");
  return guarded([&]() -> apf_status {
    HIPCHK(launch_ridges_grad(edges_dev, n_edges, mirror, h->d.nx, h->d.design_row1 - h->d.design_row0, eps_ridge,
                              eps_gap, grad_eps_dev, grad_edges_dev, (hipStream_t)stream));
    return APF_OK;
  });
}

extern "C" apf_status apf_grad(apf_handle *h, const double *dfdS_dev, double *grad_dev, void *stream) {
  if (!h || !dfdS_dev || !grad_dev) return fail(APF_EINVAL, "null argument");
  if (h->state != 2) return fail(APF_ESTATE, "apf_factor_schur has not run since the last assembly");
  // (the refined gradient runs its own full solves, not the sweeps)
  if (!h->sweeps && !h->refined)
    return fail(APF_ESTATE, "the handle prepares no gradient sweeps (apf_set_gradient)");
  return guarded([&]() -> apf_status {
    hipStream_t s = (hipStream_t)stream;
    Plan &P = h->plan;
    const int Mi = h->d.n_in, ch = P.rhs_chunk, ncol = P.ncol;
    const bool cz = h->cz.pad >= 0;
    const cplx *G = reinterpret_cast<const cplx *>(dfdS_dev);
    const double two_h2 = 2.0 * h->phys.h2;
    Profiler &pr = h->prof;
    if (h->refined) {
      // refined weighted adjoint fields, contracted with the refined forward
      // fields the factorization kept
      Refine &R = P.R;
      HIPCHK(launch_fill_double(R.norms, R.nchunks * (R.iters + 2), 0.0, s));
      for (int c = 0; c < R.nchunks; ++c) {
        const int m0 = c * R.rc, w = std::min(R.rc, Mi - m0);
        pr.run(P_REFINE, s, [&] {
          return launch_gemm(R.at<GemmTask>(R.agemm), R.nagemm, m0, w, G, s, false, nullptr, 0, true);
        });
        refine_fields(h, h->d.prj_row, R.rowbuf, R.rc, 0, w, c, s);
        pr.run(P_CONTRACT, s, [&] {
          return launch_contract_rows(R.at<int32_t>(R.erow_des), P.ndesign, R.X, R.rc, w, R.Ydes, Mi, m0, two_h2,
                                      c == 0, grad_dev, s);
        });
      }
      HIPCHK(hipStreamSynchronize(s));
      if (pr.on) pr.collect();
      refine_residuals(R);
      if (!(R.last_res <= R.tol))
        return fail(APF_ENOTCONV, "refinement of the adjoint fields ended at relative residual " +
                                      sci(R.last_res) + " (first solve " + sci(R.last_res1) + ")");
      return APF_OK;
    }
    HIPCHK(launch_row_map(P.vmap, P.at<int32_t>(P.vmap_base), P.at<int32_t>(P.vmap_pidx), P.perms, P.xc_rows, s));
    const bool f32 = h->mixed;
    if (cz) {
      // Eq. (3) over the compressed channels: S = D_C S~ D_B, so the
      // derivative with respect to S~ is D_C^T dF/dS D_B^T (FP64)
      pr.run(P_VSRC, s, [&] {
        hipError_t e = launch_gemm(P.at<GemmTask>(P.czG1), P.nczG1, 0, INT_MAX, G, s, false, nullptr, 0, true);
        if (e == hipSuccess)
          e = launch_gemm(P.at<GemmTask>(P.czG2), P.nczG2, 0, INT_MAX, nullptr, s, false, nullptr, 0, true);
        return e;
      });
      G = P.czG;
    }
    // a dF/dS with few nonzeros per input column (a few target orders per
    // input) forms the weighted adjoint source from compact column lists
    int K = 0;
    if (P.nvinit > 0 && !cz) {
      const int Mo = h->d.n_out;
      int mx = 0;
      HIPCHK(launch_fill_int(P.g_max, 0, s));
      HIPCHK(launch_col_nnz(G, Mo, Mi, P.g_nnz, P.g_max, s));
      HIPCHK(hipMemcpyAsync(&mx, P.g_max, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (mx <= kSparseG && 8 * mx <= Mo) {
        K = std::max(mx, 1);
        HIPCHK(launch_col_compact(G, Mo, Mi, K, P.g_idx, P.g_val, s));
      }
    }
    P.last_sparse_k = K;
    for (int m0 = 0; m0 < ncol; m0 += ch) {
      const int w = std::min(ch, ncol - m0);
      if (P.nvinit > 0 && K > 0) {
        pr.run(P_VSRC, s, [&] {
          return launch_sparse_vinit(P.xc, h->d.n_out, P.xc_rows, P.vmap, P.g_idx, P.g_val, K, m0, w, P.V, ch, s);
        });
      } else if (P.nvinit > 0) {
        pr.cur_tag = P.vinit_id;
        pr.run(P_GEMM_SWEEP, s, [&] { return launch_gemm(P.at<GemmTask>(P.vinit), P.nvinit, m0, w, G, s, f32, nullptr, 0, P.vinit_deep != 0); });
        pr.cur_tag = -1;
      }
      for (size_t t = 0; t < P.swl.size(); ++t) {
        pr.cur_tag = P.swl_id[t];
        if (P.nswl[t] > 0)
          pr.run(P_GEMM_SWEEP, s, [&] {
            return launch_gemm(P.at<GemmTask>(P.swl[t]), P.nswl[t], m0, w, nullptr, s, f32, P.gpart, (int)P.ndesign,
                               P.swl_deep[t] != 0, P.nswl_thin[t]);
          }, gemm_kernel_launches(P.nswl[t], P.nswl_thin[t], 0, f32));
        pr.cur_tag = -1;
        if (P.nswtb[t] > 0)
          pr.run(P_GEMM_SWEEP, s, [&] { return launch_lowrank_w(P.at<GemmTask>(P.swtb[t]), P.nswtb[t], m0, w, s); });
      }
    }
    pr.run(P_CONTRACT, s, [&] {
      return launch_reduce_partials(P.gpart, P.nblk, P.ndesign, two_h2, grad_dev, s);
    });
    // low-rank sweep subtrees, from the top: U1t, Qt, then the gradient of
    // the level's fronts and their children's Wt.  These products stay FP64
    // on the mixed path too: a front's gradient is the diagonal of Qt, far
    // smaller than the entries of Wt that form it, so FP32 rounding of U1t
    // and Qt would swamp it.
    for (int l = (int)P.wp.size() - 1; l >= 0; --l) {
      if (P.nwp[l] == 0) continue;
      pr.cur_tag = P.wu_id[l];
      if (P.nwu[l] > 0)
        pr.run(P_GEMM_SWEEP, s, [&] {
          return launch_gemm(P.at<GemmTask>(P.wu[l]), P.nwu[l], 0, INT_MAX, nullptr, s, false, nullptr, 0, P.wu_deep[l] != 0);
        });
      pr.cur_tag = P.wq_id[l];
      if (P.nwq[l] > 0)
        pr.run(P_GEMM_SWEEP, s, [&] {
          return launch_gemm(P.at<GemmTask>(P.wq[l]), P.nwq[l], 0, INT_MAX, nullptr, s, false, nullptr, 0, P.wq_deep[l] != 0);
        });
      pr.cur_tag = -1;
      pr.run(P_CONTRACT, s, [&] { return launch_wprop(P.at<WFront>(P.wp[l]), P.nwp[l], two_h2, grad_dev, s); });
    }
    if (h->prof.on) h->prof.collect();
    return APF_OK;
  });
}

// ---------------------------------------------------------------------------
// Parameter-augmented partial factorization (Sec. 2, Eq. (4) and the N_sub
// division of U): every sub-factorization eliminates the grid unknowns of
//   K~(n) = [A, [B, U(n)]; [C; U(n)^T], 0]
// and reads the blocks C A^-1 U(n), U(n)^T A^-1 B (and, unless skipped,
// U(n)^T A^-1 U(n)) of its Schur complement; Eq. (3) is applied to each
// sub's blocks without merging them.  A column of U is the unit vector of one
// design pixel (Eq. (2): dA/dp_k is diagonal on the pixels p_k modifies), so
// a front carries the columns of the pixels in its subtree: with the columns
// sorted by the pixels' elimination index these are one contiguous range per
// front, nested in the parent's range.
// ---------------------------------------------------------------------------
namespace {

struct AugBuffers {                 // grow-only device buffers of the augmented route
  cplx *arena = nullptr; int64_t arena_elems = 0;
  cplx *blocks = nullptr; int64_t block_elems = 0;
  double *misc = nullptr; int64_t misc_elems = 0;   // v, partials, sigma
  char *blob = nullptr; int64_t blob_bytes = 0;
};

template <class T>
void grow(T *&p, int64_t &have, int64_t need) {
  if (need <= have) return;
  if (p) HIPCHK(hipFree(p));
  p = nullptr;
  have = 0;
  HIPCHK(hipMalloc(&p, need * sizeof(T)));
  have = need;
}

std::mutex g_aug_mu;
std::map<apf_handle *, AugBuffers> g_aug;

void forget_aug_of(apf_handle *h) {
  std::lock_guard<std::mutex> lk(g_aug_mu);
  auto it = g_aug.find(h);
  if (it == g_aug.end()) return;
  AugBuffers &B = it->second;
  if (B.arena) (void)hipFree(B.arena);
  if (B.blocks) (void)hipFree(B.blocks);
  if (B.misc) (void)hipFree(B.misc);
  if (B.blob) (void)hipFree(B.blob);
  g_aug.erase(it);
}

struct AugSubPlan {
  std::vector<AugLevel> lv;
  int64_t cg = -1;            // Eq. (3) contraction tasks
  int ncg = 0;
  int r = 0;                  // columns of U(n)
};

}  // namespace

static apf_status augmented_grad(apf_handle *h, int32_t n_cols, const int32_t *col_pixel, const double *col_sigma,
                                 int32_t n_params, const int32_t *param_begin, int32_t n_sub, int32_t flags,
                                 const double *dfdS_dev, double *S_dev, double *dfdp_dev, hipStream_t s,
                                 int32_t *n_sub_used) {
  if (h->symmetric) return fail(APF_EINVAL, "the augmented route runs on the LU route's factor lists");
  Symbolic &S = h->sym;
  const Desc &d = h->d;
  Plan &P = h->plan;
  const std::vector<Off> &o = h->off;
  const int nf = (int)S.fronts.size();
  const int H_ = (int)S.levels.size() - 1;
  const int Mi = d.n_in, Mo = d.n_out;
  const bool uu = !(flags & APF_AUG_SKIP_UU);
  const int64_t ndes = P.ndesign;
  for (int c = 0; c < n_cols; ++c)
    if (col_pixel[c] < 0 || col_pixel[c] >= ndes) return fail(APF_EINVAL, "column pixel outside the design rows");
  if (param_begin[0] != 0 || param_begin[n_params] != n_cols)
    return fail(APF_EINVAL, "param_begin must run from 0 to n_cols");
  for (int k = 0; k < n_params; ++k)
    if (param_begin[k + 1] < param_begin[k]) return fail(APF_EINVAL, "param_begin must not decrease");
  // N_sub: given, or the smallest division whose S~(n) has at most five
  // times as many entries as A has nonzeros
  int nsub = n_sub;
  if (nsub == 0) {
    const double nnzA = 5.0 * d.nx * d.ny;
    nsub = 1;
    while (nsub < n_params) {
      const double r = std::ceil((double)n_cols / nsub);
      if ((Mi + r) * (Mo + r) <= 5.0 * nnzA) break;
      ++nsub;
    }
  }
  nsub = std::max(1, std::min(nsub, std::max(1, n_params)));
  *n_sub_used = nsub;
  // parameters split into nsub consecutive groups of about equal column counts
  std::vector<int> pgrp(nsub + 1, n_params);
  pgrp[0] = 0;
  {
    int k = 0;
    for (int g = 1; g < nsub; ++g) {
      const int64_t target = (int64_t)n_cols * g / nsub;
      while (k < n_params && param_begin[k] < target) ++k;
      pgrp[g] = std::max(pgrp[g - 1], k);
    }
  }
  // subtree elimination ranges [lo, elim0 + p) (postorder: contiguous)
  std::vector<int64_t> lo(nf);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    lo[f] = F.elim0;
    for (int c = 0; c < F.nchild; ++c) lo[f] = std::min(lo[f], lo[F.child[c]]);
  }
  std::vector<int> lp(nf);
  for (int f = 0; f < nf; ++f) {
    const Front &F = S.fronts[f];
    lp[f] = F.height;
    for (int c = 0; c < F.nchild; ++c) lp[f] = std::min(lp[f], S.fronts[F.child[c]].height);
  }
  auto WS = [&](int64_t off) { return P.ws + off; };

  // pass 1: each sub's columns (sorted by elimination index), per-front
  // column ranges, arena layout and block sizes
  struct SubLayout {
    int r = 0;
    std::vector<std::pair<int64_t, int>> col;   // (elimination index, input column)
    std::vector<int> c0, c1;
    std::vector<int64_t> pan, own;
    int64_t scu = 0, sub = 0, suu = 0;
  };
  std::vector<SubLayout> lay(nsub);
  int64_t arena_max = 1, block_max = 1;
  for (int n = 0; n < nsub; ++n) {
    SubLayout &Y = lay[n];
    const int c_beg = param_begin[pgrp[n]], c_end = param_begin[pgrp[n + 1]];
    const int r = c_end - c_beg;
    Y.r = r;
    if (r == 0) continue;
    Y.col.resize(r);
    for (int c = 0; c < r; ++c) {
      const int64_t px = col_pixel[c_beg + c];
      const int64_t node = (int64_t)(d.design_row0 + px / d.nx) * d.nx + px % d.nx;
      Y.col[c] = {S.node_elim[node], c_beg + c};
    }
    std::stable_sort(Y.col.begin(), Y.col.end(),
                     [](const std::pair<int64_t, int> &x, const std::pair<int64_t, int> &y) { return x.first < y.first; });
    std::vector<int64_t> ce(r);
    for (int c = 0; c < r; ++c) ce[c] = Y.col[c].first;
    Y.c0.assign(nf, 0);
    Y.c1.assign(nf, 0);
    for (int f = 0; f < nf; ++f) {
      const Front &F = S.fronts[f];
      Y.c0[f] = (int)(std::lower_bound(ce.begin(), ce.end(), lo[f]) - ce.begin());
      Y.c1[f] = (int)(std::lower_bound(ce.begin(), ce.end(), F.elim0 + F.p()) - ce.begin());
    }
    // blocks: S_CU (Mo x r), S_UB (r x Mi), S_UU (r x r)
    Y.scu = 0;
    Y.sub = up((int64_t)Mo * r);
    Y.suu = Y.sub + up((int64_t)r * Mi);
    block_max = std::max<int64_t>(block_max, Y.suu + (uu ? up((int64_t)r * r) : 0));
    // arena: U and U^T panels ((p + b) x r_f each, panel level to own level),
    // U1U and LCU (p x r_f each, own level)
    Arena ar;
    Y.pan.assign(nf, -1);
    Y.own.assign(nf, -1);
    std::vector<std::vector<int>> alloc_at(H_ + 1), rel_at(H_ + 2);
    for (int f = 0; f < nf; ++f)
      if (Y.c1[f] > Y.c0[f]) alloc_at[lp[f]].push_back(f);
    for (int lvl = 0; lvl <= H_; ++lvl) {
      for (int f : rel_at[lvl]) {
        const int64_t rf = Y.c1[f] - Y.c0[f];
        ar.release(Y.pan[f], 2 * (int64_t)(S.fronts[f].p() + S.fronts[f].b()) * rf);
        ar.release(Y.own[f], 2 * (int64_t)S.fronts[f].p() * rf);
      }
      for (int f : alloc_at[lvl])
        Y.pan[f] = ar.alloc(2 * (int64_t)(S.fronts[f].p() + S.fronts[f].b()) * (Y.c1[f] - Y.c0[f]));
      for (int f : S.levels[lvl])
        if (Y.c1[f] > Y.c0[f]) {
          Y.own[f] = ar.alloc(2 * (int64_t)S.fronts[f].p() * (Y.c1[f] - Y.c0[f]));
          rel_at[lvl + 1].push_back(f);
        }
    }
    arena_max = std::max<int64_t>(arena_max, ar.top);
  }
  const int nblk = 2 * ((Mi + 63) / 64);
  AugBuffers *B;
  {
    std::lock_guard<std::mutex> lk(g_aug_mu);
    B = &g_aug[h];
  }
  grow(B->arena, B->arena_elems, arena_max);
  grow(B->blocks, B->block_elems, block_max);
  grow(B->misc, B->misc_elems, (int64_t)n_cols + (int64_t)nblk * n_cols + n_cols);
  double *v = B->misc, *part = v + n_cols, *sig = part + (int64_t)nblk * n_cols;

  // pass 2: task lists with device pointers; the integer arrays (row maps,
  // contraction slots, parameter ranges) are blob offsets rebased below
  Blob bl;
  {
    const char pad[16] = {0};
    bl.add(pad, sizeof pad);
  }
  auto IP = [](int64_t off) { return reinterpret_cast<const int32_t *>((intptr_t)off); };
  std::vector<AugSubPlan> subs(nsub);
  for (int n = 0; n < nsub; ++n) {
    AugSubPlan &SP = subs[n];
    const SubLayout &Y = lay[n];
    const int r = Y.r;
    SP.r = r;
    SP.lv.assign(H_ + 1, AugLevel());
    if (r == 0) continue;
    cplx *const AR = B->arena, *const BK = B->blocks;
    std::vector<std::vector<ZeroRange>> zr(H_ + 1);
    std::vector<std::vector<cplx *>> ones(H_ + 1);
    std::vector<std::vector<GemmTask>> g1(H_ + 1), g2(H_ + 1);
    for (int f = 0; f < nf; ++f) {
      const int c0 = Y.c0[f], rf = Y.c1[f] - c0;
      if (rf == 0) continue;
      const Front &F = S.fronts[f];
      const Off &q = o[f];
      const int p = F.p(), b = F.b(), lvl = F.height, nn = p + b;
      cplx *UP = AR + Y.pan[f], *UCT = UP + (int64_t)nn * rf, *U1U = AR + Y.own[f], *LCU = U1U + (int64_t)p * rf;
      for (int64_t o0 = 0; o0 < 2 * (int64_t)nn * rf; o0 += ZERO_CHUNK)
        zr[lp[f]].push_back({UP + o0, std::min(ZERO_CHUNK, 2 * (int64_t)nn * rf - o0)});
      for (int c = c0; c < c0 + rf; ++c) {
        const int64_t e = Y.col[c].first;
        if (e >= F.elim0 && e < F.elim0 + p) {
          ones[lp[f]].push_back(UP + (e - F.elim0) * rf + (c - c0));
          ones[lp[f]].push_back(UCT + (e - F.elim0) * rf + (c - c0));
        }
      }
      cplx *tri = q.ss_tri >= 0 ? P.R.ss + q.ss_tri : WS(q.ws + q.tri);
      const int32_t *perm = P.perms + F.elim0;
      // phase 1: U1U = L^-1 P^T U_piv, LCU = U^-T (U^T)_piv^T
      add_tiles(g1[lvl], gemm(tri, p, UP, rf, U1U, rf, p, rf, p, G_A_TRI_L, nullptr, 0, perm));
      add_tiles(g1[lvl], gemm(tri, p, UCT, rf, LCU, rf, p, rf, p, G_TRANS_A | G_A_TRI_U));
      // phase 2: the parent's panels (its column range holds this front's
      // at offset c0 - c0_parent; siblings hold disjoint columns, so every
      // write adds to the zeroed panel), then the blocks of S~
      if (b) {
        const int par = F.parent, rp = Y.c1[par] - Y.c0[par];
        const Front &PF = S.fronts[par];
        cplx *pUP = AR + Y.pan[par], *pUCT = pUP + (int64_t)(PF.p() + PF.b()) * rp;
        const int32_t *rm = IP(bl.add(F.rmap));
        cplx *l21 = q.ss_l21 >= 0 ? P.R.ss + q.ss_l21 : WS(q.ws + q.l21);
        cplx *u12 = WS(q.ws + q.u12);
        GemmTask t = gemm(l21, p, U1U, rf, pUP + (c0 - Y.c0[par]), rp, b, rf, p, G_NEG | G_CIN | G_CIN_OWN | G_C_ACC,
                          UP + (int64_t)p * rf, rf);
        t.crowmap = rm;
        add_tiles(g2[lvl], t);
        GemmTask t2 = gemm(u12, b, LCU, rf, pUCT + (c0 - Y.c0[par]), rp, b, rf, p,
                           G_TRANS_A | G_NEG | G_CIN | G_CIN_OWN | G_C_ACC, UCT + (int64_t)p * rf, rf);
        t2.crowmap = rm;
        add_tiles(g2[lvl], t2);
      }
      if (F.hasC) {
        const cplx *lc1t = F.sfront ? P.sc + q.sk * Mo : WS(q.ws + q.lc1t);
        add_tiles(g2[lvl], gemm(lc1t, Mo, U1U, rf, BK + Y.scu + c0, r, Mo, rf, p, G_TRANS_A | G_C_ACC));
      }
      if (F.hasB) {
        const cplx *u1b = F.sfront ? P.sb + q.sk * Mi : WS(q.ws + q.u1b);
        add_tiles(g2[lvl], gemm(LCU, rf, u1b, Mi, BK + Y.sub + (int64_t)c0 * Mi, Mi, rf, Mi, p, G_TRANS_A | G_C_ACC));
      }
      if (uu)
        add_tiles(g2[lvl], gemm(LCU, rf, U1U, rf, BK + Y.suu + (int64_t)c0 * r + c0, r, rf, rf, p,
                                G_TRANS_A | G_C_ACC));
    }
    // Eq. (3) on this sub's blocks: v_c = sum_m ((C A^-1 U)^T dF/dS)_cm (U^T A^-1 B)_cm,
    // the contraction partials of column c going to its input index
    std::vector<int32_t> slot(r);
    for (int c = 0; c < r; ++c) slot[c] = Y.col[c].second;
    std::vector<GemmTask> cg;
    {
      GemmTask t = gemm(BK + Y.scu, r, nullptr, Mi, BK + Y.sub, Mi, r, Mi, Mo,
                        G_TRANS_A | G_B_EXT | G_CONTRACT | G_NO_STORE);
      t.aux = BK + Y.sub;
      t.auxmap = IP(bl.add(slot));
      add_tiles(cg, t);
    }
    for (int lvl = 0; lvl <= H_; ++lvl) {
      AugLevel &L = SP.lv[lvl];
      L.zero = bl.add(zr[lvl]); L.nzero = (int)zr[lvl].size();
      L.one = bl.add(ones[lvl]); L.none = (int)ones[lvl].size();
      L.g1 = bl.add(g1[lvl]); L.ng1 = (int)g1[lvl].size();
      L.g2 = bl.add(g2[lvl]); L.ng2 = (int)g2[lvl].size();
    }
    SP.cg = bl.add(cg); SP.ncg = (int)cg.size();
  }
  const int64_t cbeg_off = bl.add(param_begin, (size_t)(n_params + 1) * sizeof(int32_t));
  grow(B->blob, B->blob_bytes, (int64_t)bl.h.size());
  char *base = B->blob;
  auto rb_i = [&](const int32_t *&ptr) {
    if (ptr) ptr = reinterpret_cast<const int32_t *>(base + (intptr_t)ptr);
  };
  for (int n = 0; n < nsub; ++n) {
    AugSubPlan &SP = subs[n];
    if (SP.r == 0) continue;
    for (AugLevel &L : SP.lv) {
      GemmTask *t = reinterpret_cast<GemmTask *>(bl.h.data() + L.g2);
      for (int k = 0; k < L.ng2; ++k) rb_i(t[k].crowmap);
    }
    GemmTask *t = reinterpret_cast<GemmTask *>(bl.h.data() + SP.cg);
    for (int k = 0; k < SP.ncg; ++k) rb_i(t[k].auxmap);
  }
  HIPCHK(hipMemcpy(B->blob, bl.h.data(), bl.h.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(sig, col_sigma, (size_t)n_cols * sizeof(double), hipMemcpyHostToDevice));

  Profiler &pr = h->prof;
  const cplx *G = reinterpret_cast<const cplx *>(dfdS_dev);
  HIPCHK(launch_fill_int(P.status, 0, s));
  for (int n = 0; n < nsub; ++n) {
    const AugSubPlan &SP = subs[n];
    HIPCHK(launch_zero_flat(B->blocks, block_max, s));
    run_levels(P.lv, P.blob, P.at<FrontDev>(P.fronts), P.status, pr, s, false, &SP.lv, B->blob, P.pivq);
    if (n == 0 && S_dev) enqueue_schur(P, false, S_dev, pr, s, Mo, Mi);
    if (SP.ncg > 0)
      pr.run(P_CONTRACT, s, [&] {
        return launch_gemm(reinterpret_cast<const GemmTask *>(B->blob + SP.cg), SP.ncg, 0, INT_MAX, G, s, false, part,
                           n_cols, false);
      });
  }
  pr.run(P_CONTRACT, s, [&] {
    hipError_t e = launch_reduce_partials(part, nblk, n_cols, 1.0, v, s);
    if (e == hipSuccess)
      e = launch_param_sum(reinterpret_cast<const int32_t *>(B->blob + cbeg_off), n_params, sig, v, dfdp_dev, s);
    return e;
  });
  int st[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(st, P.status, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (pr.on) pr.collect();
  h->n_factor += nsub;
  if (st[1] & ST_BAD_EPS) {
    h->state = 0;
    return fail(APF_EINVAL, "the permittivity has a zero or non-finite value");
  }
  if (st[0]) {
    h->state = 0;
    return fail(APF_ESINGULAR, "zero or non-finite pivot in a pivot block");
  }
  h->state = 2;
  h->mixed = false;
  h->refined = false;
  return APF_OK;
}

extern "C" apf_status apf_grad_augmented(apf_handle *h, int32_t n_cols, const int32_t *col_pixel,
                                         const double *col_sigma, int32_t n_params, const int32_t *param_begin,
                                         int32_t n_sub, int32_t flags, const double *dfdS_dev, double *S_dev,
                                         double *dfdp_dev, int32_t *n_sub_used, void *stream) {
  if (!h || !col_pixel || !col_sigma || !param_begin || !dfdS_dev || !dfdp_dev)
    return fail(APF_EINVAL, "null argument");
  if (n_cols < 1 || n_params < 1) return fail(APF_EINVAL, "need at least one column and one parameter");
  if (n_sub < 0) return fail(APF_EINVAL, "n_sub must be >= 0");
  if (flags & ~APF_AUG_SKIP_UU) return fail(APF_EINVAL, "unknown flags");
  if (h->state < 1) return fail(APF_ESTATE, "apf_assemble has not run");
  if (h->cz.pad >= 0) return fail(APF_EINVAL, "the augmented route runs on uncompressed channel panels");
  int32_t used = 0;
  apf_status st = guarded([&]() -> apf_status {
    return augmented_grad(h, n_cols, col_pixel, col_sigma, n_params, param_begin, n_sub, flags, dfdS_dev, S_dev,
                          dfdp_dev, (hipStream_t)stream, &used);
  });
  if (n_sub_used) *n_sub_used = used;
  return st;
}

extern "C" apf_status apf_ridges_grad_augmented(apf_handle *h, const double *edges_dev, int32_t n_edges,
                                                int32_t mirror, double eps_ridge, double eps_gap, int32_t n_sub,
                                                int32_t flags, const double *dfdS_dev, double *S_dev,
                                                double *dfdp_dev, int32_t *n_sub_used, void *stream) {
  if (apf_status st = check_ridges(h, edges_dev, n_edges, mirror)) return st;
  if (!dfdS_dev || !dfdp_dev) return fail(APF_EINVAL, "null argument");
  if (h->state < 1) return fail(APF_ESTATE, "apf_assemble has not run");
  if (h->cz.pad >= 0) return fail(APF_EINVAL, "the augmented route runs on uncompressed channel panels");
  return guarded([&]() -> apf_status {
    // U_k: the pixels of the cells holding edge k (and its mirror image) on
    // every design row, with Sigma = dA/dp = -h^2 deps/dp: -/+(eps_ridge -
    // eps_gap) for a left / right edge, the image moving by -1
    std::vector<double> e(n_edges);
    HIPCHK(hipMemcpyAsync(e.data(), edges_dev, n_edges * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    const int nx = h->d.nx, nrows = h->d.design_row1 - h->d.design_row0, nfull = mirror ? 2 * n_edges : n_edges;
    const double de = eps_ridge - eps_gap, h2 = h->phys.h2;
    auto cell = [&](double x) { int c = (int)std::floor(x + 0.5) % nx; return c < 0 ? c + nx : c; };
    auto edge = [&](int q) { return (!mirror || q < n_edges) ? e[q] : (double)nx - e[2 * n_edges - 1 - q]; };
    std::vector<int32_t> pix, pbeg(1, 0);
    std::vector<double> sig;
    for (int k = 0; k < n_edges; ++k) {
      const int ck = cell(e[k]);
      double sk = k % 2 == 0 ? -de : de;
      int ci = -1;
      double si = 0.0;
      if (mirror) {
        const int q = nfull - 1 - k;
        ci = cell(edge(q));
        si = -(q % 2 == 0 ? -de : de);
        if (ci == ck) { sk += si; ci = -1; }
      }
      for (int rr = 0; rr < nrows; ++rr) {
        pix.push_back(rr * nx + ck);
        sig.push_back(-h2 * sk);
        if (ci >= 0) {
          pix.push_back(rr * nx + ci);
          sig.push_back(-h2 * si);
        }
      }
      pbeg.push_back((int32_t)pix.size());
    }
    int32_t used = 0;
    apf_status st = augmented_grad(h, (int32_t)pix.size(), pix.data(), sig.data(), n_edges, pbeg.data(), n_sub, flags,
                                   dfdS_dev, S_dev, dfdp_dev, (hipStream_t)stream, &used);
    if (n_sub_used) *n_sub_used = used;
    return st;
  });
}

// ---------------------------------------------------------------------------
// Autotuner: the kernel form of every tunable GEMM list (four-product at four
// workgroups per CU, three-product or four-product on the deep-K kernel at
// three), decided per bucket of lists (mean k extent of a tile, number of
// tiles) from HIP-event times of the actual launches, saved as a text table.
// ---------------------------------------------------------------------------
namespace {

constexpr int kTuneForms = 3;

// bucket of a list: (log2 of mean tile k over 16, rounded; log2 of the tile count)
std::pair<int, int> tune_bucket(const TunableList &t) {
  std::vector<GemmTask> v = fetch<GemmTask>(t.blob, t.off, t.n);
  const double mk = std::max(1.0, mean_tile_k(v));
  const int kb = std::max(0, std::min(9, (int)std::lround(std::log2(mk / 16.0))));
  const int tb = std::max(0, std::min(20, (int)std::floor(std::log2((double)std::max(1, t.n)))));
  return {kb, tb};
}

void set_form(TunableList &t, int form, hipStream_t s) {
  *t.deep = form != 0;
  HIPCHK(launch_set_k3(reinterpret_cast<GemmTask *>(t.blob + t.off), t.n, form == 1, s));
}

struct TuneRow { double ms[kTuneForms] = {0, 0, 0}; int lists = 0; int form = -1; };

std::string table_text(const std::map<std::pair<int, int>, TuneRow> &tab) {
  std::string out = "# APF GEMM autotune table: bucket (kb = round(log2(mean tile k / 16)), tb = floor(log2(tiles)))\n"
                    "# -> form (0 four-product k_gemm, 1 three-product k_gemm_k3, 2 four-product k_gemm_k3)\n"
                    "# kb tb form ms_form0 ms_form1 ms_form2 lists\n";
  char b[256];
  for (const auto &kv : tab) {
    std::snprintf(b, sizeof b, "%d %d %d %.4f %.4f %.4f %d\n", kv.first.first, kv.first.second, kv.second.form,
                  kv.second.ms[0], kv.second.ms[1], kv.second.ms[2], kv.second.lists);
    out += b;
  }
  return out;
}

}  // namespace

// The lists an autotune call works on, and the work that runs them: the
// single plan (factorization, Schur product, gradient sweeps) for n = 1, the
// merged batch plan (factorization levels) for n > 1.
static apf_status autotune_impl(apf_handle *const *hs, int32_t n, int32_t reps, const char *load_path,
                                const char *save_path, hipStream_t s) {
  std::vector<TunableList> *tl = nullptr;
  BatchPlan *B = nullptr;
  if (n == 1) {
    tl = &hs[0]->plan.tl;
  } else {
    for (int i = 0; i < n; ++i)
      if (hs[i]->symmetric) return fail(APF_EINVAL, "the symmetric route is not batched");
    std::vector<apf_handle *> v(hs, hs + n);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto &b : g_batches)
      if (b->hs == v) B = b.get();
    if (!B) {
      g_batches.push_back(build_batch(v));
      B = g_batches.back().get();
    }
    tl = &B->tl;
  }
  std::vector<std::pair<int, int>> bucket(tl->size());
  for (size_t i = 0; i < tl->size(); ++i) bucket[i] = tune_bucket((*tl)[i]);
  std::map<std::pair<int, int>, TuneRow> tab;
  if (load_path) {
    FILE *f = std::fopen(load_path, "r");
    if (!f) return fail(APF_EINVAL, std::string("cannot open ") + load_path);
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
      if (line[0] == '#') continue;
      int kb, tb, form, lists;
      double a, b, c;
      if (std::sscanf(line, "%d %d %d %lf %lf %lf %d", &kb, &tb, &form, &a, &b, &c, &lists) == 7 && form >= 0 &&
          form < kTuneForms) {
        TuneRow r;
        r.ms[0] = a; r.ms[1] = b; r.ms[2] = c; r.lists = lists; r.form = form;
        tab[{kb, tb}] = r;
      }
    }
    std::fclose(f);
  } else {
    // time every list in every form over `reps` runs of the work
    Profiler &pr = hs[0]->prof;
    const bool was_on = pr.on, was_gemm = pr.gemm_only;
    std::vector<double *> Ss(n, nullptr);
    double *G = nullptr, *grad = nullptr;
    auto cleanup = [&] {
      for (double *p : Ss) if (p) (void)hipFree(p);
      if (G) (void)hipFree(G);
      if (grad) (void)hipFree(grad);
      pr.on = was_on; pr.gemm_only = was_gemm; pr.record = false; pr.reset();
    };
    try {
      for (int i = 0; i < n; ++i)
        HIPCHK(hipMalloc(&Ss[i], (int64_t)hs[i]->d.n_out * hs[i]->d.n_in * 2 * sizeof(double)));
      if (n == 1) {
        HIPCHK(hipMalloc(&G, (int64_t)hs[0]->d.n_out * hs[0]->d.n_in * 2 * sizeof(double)));
        HIPCHK(hipMemset(G, 0, (int64_t)hs[0]->d.n_out * hs[0]->d.n_in * 2 * sizeof(double)));
        HIPCHK(hipMalloc(&grad, std::max<int64_t>(hs[0]->plan.ndesign, 1) * sizeof(double)));
      }
      std::vector<std::vector<double>> t(kTuneForms, std::vector<double>(tl->size(), 0.0));
      auto work = [&]() -> apf_status {
        if (n == 1) {
          apf_status st = apf_factor_schur(hs[0], APF_FP64, Ss[0], s);
          if (st == APF_OK) st = apf_grad(hs[0], G, grad, s);
          return st;
        }
        return apf_factor_schur_batched(hs, n, APF_FP64, Ss.data(), s);
      };
      for (int form = 0; form < kTuneForms; ++form) {
        for (TunableList &l : *tl) set_form(l, form, s);
        HIPCHK(hipStreamSynchronize(s));
        pr.reset();
        pr.on = true; pr.gemm_only = true; pr.record = false;   // eager launches (no graph replay)
        apf_status st = work();                         // warm-up
        if (st != APF_OK) { cleanup(); return st; }
        pr.reset();
        pr.on = true; pr.gemm_only = true; pr.record = true;
        for (int r = 0; r < reps; ++r) {
          st = work();
          if (st != APF_OK) { cleanup(); return st; }
        }
        for (const auto &e : pr.trace)
          if (e.first >= 0 && e.first < (int)tl->size()) t[form][e.first] += e.second / reps;
        pr.record = false;
        pr.reset();
      }
      for (size_t i = 0; i < tl->size(); ++i) {
        TuneRow &r = tab[bucket[i]];
        for (int form = 0; form < kTuneForms; ++form) r.ms[form] += t[form][i];
        ++r.lists;
      }
      for (auto &kv : tab) {
        int best = 0;
        for (int form = 1; form < kTuneForms; ++form)
          if (kv.second.ms[form] < kv.second.ms[best]) best = form;
        kv.second.form = best;
      }
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
  }
  // apply: lists in a bucket of the table take its form; others keep theirs
  for (size_t i = 0; i < tl->size(); ++i) {
    auto it = tab.find(bucket[i]);
    if (it != tab.end() && it->second.form >= 0) set_form((*tl)[i], it->second.form, s);
  }
  HIPCHK(hipStreamSynchronize(s));
  if (B) {
    // the captured graph launches the kernels the old forms chose
    if (B->exec) { HIPCHK(hipGraphExecDestroy(B->exec)); B->exec = nullptr; }
    if (B->graph) { HIPCHK(hipGraphDestroy(B->graph)); B->graph = nullptr; }
  } else {
    forget_batches_of(hs[0]);   // merged plans copied the old task flags
  }
  if (save_path) {
    FILE *f = std::fopen(save_path, "w");
    if (!f) return fail(APF_EINVAL, std::string("cannot write ") + save_path);
    const std::string txt = table_text(tab);
    std::fputs(txt.c_str(), f);
    std::fclose(f);
  }
  return APF_OK;
}

extern "C" apf_status apf_autotune(apf_handle *const *hs, int32_t n, int32_t reps, const char *save_path,
                                   void *stream) {
  if (!hs || n < 1) return fail(APF_EINVAL, "need at least one handle");
  if (reps < 1 || reps > 100) return fail(APF_EINVAL, "reps must be in [1, 100]");
  for (int i = 0; i < n; ++i) {
    if (!hs[i]) return fail(APF_EINVAL, "null handle");
    if (hs[i]->state < 1) return fail(APF_ESTATE, "apf_assemble has not run on every handle");
  }
  return guarded([&]() { return autotune_impl(hs, n, reps, nullptr, save_path, (hipStream_t)stream); });
}

extern "C" apf_status apf_tuning_apply(apf_handle *const *hs, int32_t n, const char *path, void *stream) {
  if (!hs || n < 1 || !path) return fail(APF_EINVAL, "need handles and a table path");
  for (int i = 0; i < n; ++i) {
    if (!hs[i]) return fail(APF_EINVAL, "null handle");
    if (!hs[i]->planned) return fail(APF_ESTATE, "apf_assemble has not run on every handle");
  }
  return guarded([&]() { return autotune_impl(hs, n, 1, path, nullptr, (hipStream_t)stream); });
}

extern "C" apf_status apf_set_rhs_chunk(apf_handle *h, int32_t max_chunk) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (max_chunk < 0 || (max_chunk > 0 && max_chunk % 64 != 0))
    return fail(APF_EINVAL, "the chunk cap must be 0 or a positive multiple of 64");
  if (h->planned) return fail(APF_ESTATE, "the sweep arrays are already sized (apf_assemble has run)");
  h->max_chunk = max_chunk;
  return APF_OK;
}

extern "C" apf_status apf_set_symmetric(apf_handle *h, int32_t on) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (on != 0 && on != 1) return fail(APF_EINVAL, "on must be 0 or 1");
  if (h->planned) return fail(APF_ESTATE, "the plan is already built (apf_assemble has run)");
  if (on && h->cz.pad >= 0) return fail(APF_EINVAL, "the symmetric route does not combine with compressed channels");
  if (on && h->refine_iters > 0) return fail(APF_EINVAL, "the symmetric route does not combine with refinement");
  h->symmetric = on != 0;
  return APF_OK;
}

extern "C" apf_status apf_set_lowrank(apf_handle *h, int32_t levels) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (levels < 0 || levels > kWMaxLevels) return fail(APF_EINVAL, "low-rank subtree levels must be 0, 1 or 2");
  if (h->planned) return fail(APF_ESTATE, "the sweep plan is already built (apf_assemble has run)");
  h->lowrank = levels;
  return APF_OK;
}

extern "C" apf_status apf_set_compression(apf_handle *h, int32_t pad, double window_wavelengths) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (!h->analyzed) return fail(APF_ESTATE, "apf_analyze has not run");
  if (h->planned) return fail(APF_ESTATE, "the plan is already built (apf_assemble has run)");
  if (pad < -1) return fail(APF_EINVAL, "pad must be >= 0 (or -1 to switch compression off)");
  if (pad >= 0 && h->symmetric) return fail(APF_EINVAL, "compressed channels do not combine with the symmetric route");
  const Desc &d = h->d;
  return guarded([&]() -> apf_status {
    if (pad < 0) {
      // back to full channel panels and the gradient sweeps
      h->cz = Compress();
      size_plan(h);
      return APF_OK;
    }
    if (!(window_wavelengths > 0.0) || !std::isfinite(window_wavelengths))
      return fail(APF_EINVAL, "the window must be a positive number of wavelengths");
    for (int k = 1; k < d.n_in; ++k)
      if (d.in_orders[k] != d.in_orders[k - 1] + 1) return fail(APF_EINVAL, "input orders must be consecutive");
    for (int k = 1; k < d.n_out; ++k)
      if (d.out_orders[k] != d.out_orders[k - 1] + 1) return fail(APF_EINVAL, "output orders must be consecutive");
    Compress Z;
    Z.pad = pad;
    Z.half_px = 0.5 * window_wavelengths / d.dx_over_lambda;
    Z.MxB = d.n_in + pad;
    Z.MxC = d.n_out + pad;
    Z.a0B = d.in_orders[0] - pad / 2;
    Z.a0C = d.out_orders[0] - pad / 2;
    // every node must lie in some column's window
    if ((double)d.nx / std::min(Z.MxB, Z.MxC) > 2.0 * Z.half_px)
      return fail(APF_EINVAL, "the window is narrower than the spacing of the compressed columns");
    Symbolic &S = h->sym;
    // per front: the columns whose window meets the front's region (x0..x1,
    // periodic), one margin column each side; a range that would wrap is the
    // whole set.  A parent's region holds its children's, so its range does.
    const int nf = (int)S.fronts.size();
    auto range = [&](const Front &F, int Mx, int &c0, int &c1) {
      const double lo = (F.x0 - Z.half_px) * Mx / (double)d.nx, hi = (F.x1 - 1 + Z.half_px) * Mx / (double)d.nx;
      c0 = (int)std::ceil(lo) - 1;
      c1 = (int)std::floor(hi) + 2;   // exclusive
      if (c0 < 0 || c1 > Mx || F.x1 - F.x0 >= d.nx - 1) { c0 = 0; c1 = Mx; }
    };
    Z.cB0.assign(nf, 0); Z.cB1.assign(nf, 0); Z.cC0.assign(nf, 0); Z.cC1.assign(nf, 0);
    for (int f = 0; f < nf; ++f) {
      const Front &F = S.fronts[f];
      if (F.hasB) range(F, Z.MxB, Z.cB0[f], Z.cB1[f]);
      if (F.hasC) range(F, Z.MxC, Z.cC0[f], Z.cC1[f]);
    }
    for (int f = 0; f < nf; ++f) {   // nesting (guaranteed by the regions; checked)
      const Front &F = S.fronts[f];
      if (F.parent < 0) continue;
      if (F.hasB && (Z.cB0[f] < Z.cB0[F.parent] || Z.cB1[f] > Z.cB1[F.parent]))
        throw std::runtime_error("compressed column ranges do not nest");
      if (F.hasC && (Z.cC0[f] < Z.cC0[F.parent] || Z.cC1[f] > Z.cC1[F.parent]))
        throw std::runtime_error("compressed column ranges do not nest");
    }
    h->cz = std::move(Z);
    size_plan(h);
    return APF_OK;
  });
}

extern "C" apf_status apf_set_gradient(apf_handle *h, int32_t on) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (on != 0 && on != 1) return fail(APF_EINVAL, "on must be 0 or 1");
  if (!h->analyzed) return fail(APF_ESTATE, "apf_analyze has not run");
  if (h->planned) return fail(APF_ESTATE, "the plan is already built (apf_assemble has run)");
  if (h->sweeps == (on != 0)) return APF_OK;
  return guarded([&]() -> apf_status {
    h->sweeps = on != 0;
    // the analysis marks the sweep fronts; the tree (and any compressed
    // column ranges over it) is the same on every run
    analyze(h->d, h->sym);
    drop_sweeps_unless_wanted(h);
    size_plan(h);
    return APF_OK;
  });
}

extern "C" apf_status apf_set_refinement(apf_handle *h, int32_t max_iter, double tol) {
  if (!h) return fail(APF_EINVAL, "null handle");
  if (max_iter < 0 || max_iter > 16) return fail(APF_EINVAL, "max_iter must be in [0, 16]");
  if (max_iter > 0 && !(tol > 0.0 && tol < 1.0)) return fail(APF_EINVAL, "tol must be in (0, 1)");
  if (h->planned) return fail(APF_ESTATE, "the plan is already built (apf_assemble has run)");
  if (max_iter > 0 && h->symmetric) return fail(APF_EINVAL, "refinement does not combine with the symmetric route");
  h->refine_iters = max_iter;
  h->refine_tol = max_iter > 0 ? tol : 0.0;
  if (h->analyzed) size_plan(h);   // the retained-factor offsets depend on it
  return APF_OK;
}

extern "C" apf_status apf_set_profiling(apf_handle *h, int32_t on) {
  if (!h) return fail(APF_EINVAL, "null handle");
  return guarded([&]() -> apf_status {
    if (on < 0 || on > 2) return fail(APF_EINVAL, "profiling mode must be 0, 1 or 2");
    h->prof.reset();
    h->prof.on = on != 0;
    h->prof.gemm_only = on == 2;
    return APF_OK;
  });
}

extern "C" apf_status apf_destroy(apf_handle *h) {
  if (!h) return APF_OK;
  forget_batches_of(h);
  forget_aug_of(h);
  free_plan(h->plan);
  delete h;
  return APF_OK;
}

extern "C" const char *apf_last_error(void) { return g_err.c_str(); }

extern "C" apf_status apf_query(apf_handle *h, const char *key, double *value) {
  if (!h || !key || !value) return fail(APF_EINVAL, "null argument");
  if (!h->analyzed) return fail(APF_ESTATE, "apf_analyze has not run");
  const Symbolic &S = h->sym;
  std::string k(key);
  if (k == "n_fronts") *value = (double)S.fronts.size();
  else if (k == "n_levels") *value = (double)S.levels.size();
  else if (k == "max_front") *value = S.max_front;
  else if (k == "factor_cmacs") *value = S.factor_cmacs;
  else if (k == "grad_cmacs") *value = S.grad_cmacs;
  else if (k == "algo_factor_cmacs") *value = S.algo_factor_cmacs;
  else if (k == "n_sweep_rows") *value = (double)S.n_sweep_rows;
  else if (k == "n_sweep_fronts") {
    double c = 0;
    for (const Front &F : S.fronts) c += F.sweep;
    *value = c;
  } else if (k == "k_total") *value = (double)S.k_total;
  else if (k == "xc_rows") *value = (double)h->plan.xc_rows;
  else if (k == "pivot_spread_min" || k == "pivot_spread_front") {
    // smallest pivot spread over the fronts of the last factorization
    if (h->state != 2 || !h->plan.pivq) return fail(APF_ESTATE, "no factorization has completed since the last assembly");
    std::vector<double> q(S.fronts.size());
    if (hipMemcpy(q.data(), h->plan.pivq, q.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(APF_EHIP, "copy of the pivot spreads failed");
    size_t arg = 0;
    for (size_t f = 1; f < q.size(); ++f)
      if (q[f] < q[arg]) arg = f;
    *value = k == "pivot_spread_min" ? q[arg] : (double)arg;
  }
  else if (k == "ws_bytes") *value = (double)h->plan.ws_elems * sizeof(cplx);
  else if (k == "factor_bytes") *value = (double)h->plan.fs_elems * sizeof(cplx);
  else if (k == "schur_store_bytes") *value = (double)S.k_total * (h->d.n_in + h->d.n_out) * sizeof(cplx);
  else if (k == "rhs_chunk") *value = h->planned ? (double)h->plan.rhs_chunk : -1.0;
  else if (k == "n_factorizations") *value = (double)h->n_factor;
  else if (k == "refine_chunk") *value = h->planned ? (double)h->plan.R.rc : -1.0;
  else if (k == "refine_residual") *value = h->plan.R.last_res;
  else if (k == "refine_residual_first") *value = h->plan.R.last_res1;
  else if (k == "retained_factor_bytes") *value = (double)h->plan.R.ss_elems * sizeof(cplx);
  else if (k == "lowrank_fronts") *value = h->planned ? (double)h->plan.n_wfronts : -1.0;
  else if (k == "lowrank_roots") *value = h->planned ? (double)h->plan.n_wroots : -1.0;
  else if (k == "gemm_cmacs_factor") *value = h->planned ? h->plan.gemm_cmacs_factor : -1.0;
  else if (k == "gemm_cmacs_schur") *value = h->planned ? h->plan.gemm_cmacs_schur : -1.0;
  else if (k == "gemm_cmacs_sweep") *value = h->planned ? h->plan.gemm_cmacs_sweep : -1.0;
  else if (k == "gemm_cmacs_k3") *value = h->planned ? h->plan.gemm_cmacs_k3 : -1.0;
  else if (k == "gemm_cmacs_vinit") *value = h->planned ? h->plan.vinit_cmacs : -1.0;
  else if (k == "adjoint_source_sparse_k") *value = h->planned ? (double)h->plan.last_sparse_k : -1.0;
  else if (k == "gemm_cmacs_lowrank_w") *value = h->planned ? h->plan.gemm_cmacs_w : -1.0;
  else if (k.rfind("ms_", 0) == 0 || k.rfind("launches_", 0) == 0) {
    bool ms = k[0] == 'm';
    std::string cls = k.substr(ms ? 3 : 9);
    int c = -1;
    for (int i = 0; i < P_NCLASS; ++i)
      if (cls == kProfNames[i]) c = i;
    if (c < 0) return fail(APF_EINVAL, "unknown profile class " + cls);
    *value = ms ? h->prof.ms[c] : (double)h->prof.count[c];
  } else return fail(APF_EINVAL, "unknown key " + k);
  return APF_OK;
}

extern "C" apf_status apf_front(apf_handle *h, int32_t f, int32_t info[8], int32_t *pivots, int32_t *boundary) {
  if (!h || !info) return fail(APF_EINVAL, "null argument");
  if (!h->analyzed) return fail(APF_ESTATE, "apf_analyze has not run");
  const Symbolic &S = h->sym;
  if (f < 0 || f >= (int32_t)S.fronts.size()) return fail(APF_EINVAL, "front index out of range");
  const Front &F = S.fronts[f];
  info[0] = F.parent; info[1] = F.height; info[2] = F.p(); info[3] = F.b();
  info[4] = F.hasB; info[5] = F.hasC; info[6] = F.sweep; info[7] = (int32_t)F.elim0;
  if (pivots) std::copy(F.piv.begin(), F.piv.end(), pivots);
  if (boundary) std::copy(F.bnd.begin(), F.bnd.end(), boundary);
  return APF_OK;
}

// ---------------------------------------------------------------------------
// Kernel test hook: one GEMM of the factorization's task format, cut into
// tiles and launched on the chosen kernel form, so that the kernel's
// semantics (operand layouts, triangular masks, row and column maps, Cin
// forms, edges, the LDS-direct stages) can be checked against a plain
// reference.  Allocates (the tile list) and synchronises `stream`.
// ---------------------------------------------------------------------------
extern "C" apf_status apf_test_gemm(int32_t form, int32_t flags, int32_t M, int32_t N, int32_t K,
                                    const double *A, int32_t lda, const double *B, int32_t ldb, int64_t b_offset,
                                    const double *Cin, int32_t ldcin, double *C, int32_t ldc,
                                    const int32_t *browmap, const int32_t *crowmap, const int32_t *ccolmap,
                                    int32_t cin_c0, int32_t cin_w, int32_t coff, int32_t nlim, int32_t xcd,
                                    const double *aux, const int32_t *auxmap, double *part, int32_t pstride,
                                    void *stream) {
  const int32_t allowed = G_TRANS_A | G_NEG | G_CIN | G_B_COFF | G_CIN_COFF | G_B_EXT | G_A_TRI_L | G_A_TRI_U |
                          G_B_TRI_L | G_B_TRI_U | G_CIN_OWN | G_C_ACC | G_K_LIM | G_ACC_CHUNK | G_C_COFF |
                          G_CIN_RANGE | G_CONTRACT | G_NO_STORE;
  if (form < 0 || form > 5) return fail(APF_EINVAL, "form must be 0 (four-product), 1 (three-product), "
                                                    "2 (four-product on the deep-K kernel), 3 (FP32), 4 "
                                                    "(four-product with the thin tiles on the thin kernels) or 5 "
                                                    "(FP32 with the thin tiles on the thin kernels)");
  if (flags & ~allowed) return fail(APF_EINVAL, "flag outside the tested set");
  if (M < 1 || N < 1 || K < 0 || !A || !B || !C || nlim < 1) return fail(APF_EINVAL, "bad shape or null operand");
  if ((flags & G_CIN) && !Cin) return fail(APF_EINVAL, "G_CIN without Cin");
  if ((flags & G_CONTRACT) && (!aux || !auxmap || !part || pstride < 1))
    return fail(APF_EINVAL, "G_CONTRACT without aux, auxmap, part or a positive pstride");
  if ((flags & G_CONTRACT) && coff % 32) return fail(APF_EINVAL, "G_CONTRACT with coff not a multiple of 32");
  return guarded([&]() -> apf_status {
    hipStream_t s = (hipStream_t)stream;
    const cplx *Bt = (flags & G_B_EXT) ? reinterpret_cast<const cplx *>((intptr_t)b_offset)
                                       : reinterpret_cast<const cplx *>(B);
    GemmTask t = gemm(reinterpret_cast<const cplx *>(A), lda, Bt, ldb, reinterpret_cast<cplx *>(C), ldc, M, N, K,
                      flags | (form == 1 ? G_K3 : 0), reinterpret_cast<const cplx *>(Cin), ldcin, browmap);
    t.crowmap = crowmap;
    t.ccolmap = ccolmap;
    t.cin_c0 = cin_c0;
    t.cin_w = cin_w;
    if (flags & G_CONTRACT) {
      t.aux = reinterpret_cast<const cplx *>(aux);
      t.auxmap = auxmap;
    }
    std::vector<GemmTask> v;
    if (xcd) add_tiles_xcd(v, t);
    else add_tiles(v, t);
    int ntri = 0;
    const int nthin = (form == 4 || form == 5) ? split_thin(v, &ntri) : 0;
    GemmTask *dv = nullptr;
    HIPCHK(hipMalloc(&dv, std::max<size_t>(v.size(), 1) * sizeof(GemmTask)));
    hipError_t e = hipMemcpyAsync(dv, v.data(), v.size() * sizeof(GemmTask), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = launch_gemm(dv, (int)v.size(), coff, nlim, (flags & G_B_EXT) ? reinterpret_cast<const cplx *>(B) : nullptr,
                      s, form == 3 || form == 5, (flags & G_CONTRACT) ? part : nullptr, (flags & G_CONTRACT) ? pstride : 0,
                      form == 1 || form == 2, nthin, ntri);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dv);
    HIPCHK(e);
    return APF_OK;
  });
}

// Kernel test hook: the pivot-block kernel on one p x p block.
extern "C" apf_status apf_test_pivot_block(int32_t p, const double *F_dev, double *tri_dev, int32_t *perm_dev,
                                           double *spread, int32_t sym, void *stream) {
  if (p < 1 || p > MAX_PIVOTS) return fail(APF_EINVAL, "p must be in [1, " + std::to_string(MAX_PIVOTS) + "]");
  if (sym != 0 && sym != 1) return fail(APF_EINVAL, "sym must be 0 or 1");
  if (!F_dev || !tri_dev || !perm_dev) return fail(APF_EINVAL, "null argument");
  return guarded([&]() -> apf_status {
    hipStream_t s = (hipStream_t)stream;
    FrontDev fd{};
    fd.p = p;
    fd.sweep_row0 = -1;
    fd.core = const_cast<cplx *>(reinterpret_cast<const cplx *>(F_dev));
    fd.tri = reinterpret_cast<cplx *>(tri_dev);
    fd.perm = perm_dev;
    fd.parent = -1;
    char *buf = nullptr;   // FrontDev, id, status, spread
    HIPCHK(hipMalloc(&buf, 256 * 4));
    FrontDev *dfd = reinterpret_cast<FrontDev *>(buf);
    int32_t *did = reinterpret_cast<int32_t *>(buf + 256);
    int *dst = reinterpret_cast<int *>(buf + 512);
    double *dq = reinterpret_cast<double *>(buf + 768);
    const int32_t zero = 0;
    hipError_t e = hipMemcpyAsync(dfd, &fd, sizeof fd, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(did, &zero, sizeof zero, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(dst, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_inverse(inverse_variant(p), dfd, did, 1, dst, dq, sym ? 1 : 0, s);
    int st = 0;
    double q = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&st, dst, sizeof st, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&q, dq, sizeof q, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(buf);
    HIPCHK(e);
    if (spread) *spread = q;
    if (st & ST_SINGULAR) return fail(APF_ESINGULAR, "zero or non-finite pivot in the block");
    return APF_OK;
  });
}
