// Host symbolic analysis: geometric nested dissection of the x-periodic
// nx-by-ny grid, elimination tree, frontal index sets and extend-add maps.
//
// The augmented matrix K = [A, B; C, 0] (Sec. 2) keeps the sparsity of A for
// its grid unknowns; the channel columns of B live on the source row and the
// channel rows of C on the projection row.  A front therefore carries the
// M_in channel columns when its subtree holds source-row nodes and the M_out
// channel rows when it holds projection-row nodes; the channel-by-channel
// block is never pivoted and is summed straight into S.
#include <algorithm>
#include <cstdlib>
#include <stdexcept>
#include <unordered_map>

#include "apf_internal.h"

namespace apf {

namespace {

// Default leaf size (nodes).  24000 x 160: 169.3 ms/solve at 48 against
// 179.4 at 40, 172.2 at 56 and 172.1 at 64.
constexpr int kLeafNodes = 48;
// A region is cut by a vertical separator (a full column of its height) only
// while it is at least kAspectPart times wider than tall; narrower regions
// are cut horizontally.  A vertical separator of a region that spans both the
// source and the projection row is a front that holds both channel blocks
// and adds its pivots to the Schur product's k dimension, so such regions
// keep being cut horizontally up to kAspectFull.  (24000 x 160 against a
// uniform aspect of 1, with the band-edge row cuts below: k_total 64,704 ->
// 34,176, factorization work -31%, gradient work -32%, workspace 55 -> 21 GB;
// measured 1.5 and 2 for kAspectPart, 2 to 4 for kAspectFull.)
constexpr double kAspectFull = 3.0;   // regions holding both channel rows
constexpr double kAspectPart = 2.0;   // the others

struct Builder {
  const Desc &d;
  Symbolic &s;
  int leaf;
  // Preferred rows of horizontal separators.  The first and the last design
  // row: cutting there separates the source row, the design band and the
  // projection row early and leaves the band's interior as its own subtree,
  // which shrinks the fronts the gradient sweeps visit (24000 x 160: sweep
  // work -15% against cuts midway between the band and the channel rows).
  // The source and the projection row themselves: a region cut along its
  // channel row leaves two subtrees without channel columns, so the dense
  // M-wide channel panels start at that separator instead of at every leaf
  // the row crosses (24000 x 160: work of the fronts other than the Schur
  // product -17%, 131,392 fronts instead of 157,248).
  std::vector<int> prefer;
  Builder(const Desc &d_, Symbolic &s_) : d(d_), s(s_), leaf(d_.leaf_size > 0 ? d_.leaf_size : kLeafNodes) {
    prefer.push_back(d.design_row0);
    prefer.push_back(d.design_row1 - 1);
    prefer.push_back(d.src_row);
    prefer.push_back(d.prj_row);
  }

  // Row of a horizontal separator of [y0, y1): the preferred row nearest the
  // middle when one lies in the middle half of the range, else the middle
  // row.
  int row_cut(int y0, int y1) const {
    const int hh = y1 - y0, mid = y0 + hh / 2;
    int best = -1;
    for (int r : prefer)
      if (r >= y0 + hh / 4 && r < y1 - hh / 4 && (best < 0 || std::abs(r - mid) < std::abs(best - mid))) best = r;
    return best >= 0 ? best : mid;
  }

  int node(int x, int y) const { return y * d.nx + x; }

  // Emit a front over `piv` with children c0, c1; separators longer than
  // MAX_PIVOTS become a chain of fronts (each the parent of the previous), so
  // that no pivot block exceeds what one workgroup factors in registers.
  int emit(std::vector<int> &&piv, int c0, int c1, int x0, int x1, int y0, int y1) {
    const int p = (int)piv.size();
    const int nchunk = (p + MAX_PIVOTS - 1) / MAX_PIVOTS;
    const int chunk = (p + nchunk - 1) / nchunk;
    int prev = -1;
    for (int j = 0; j < nchunk; ++j) {
      Front f;
      f.x0 = x0; f.x1 = x1; f.y0 = y0; f.y1 = y1;
      f.piv.assign(piv.begin() + j * chunk, piv.begin() + std::min(p, (j + 1) * chunk));
      int c[2] = {j == 0 ? c0 : prev, j == 0 ? c1 : -1};
      for (int k = 0; k < 2; ++k)
        if (c[k] >= 0) f.child[f.nchild++] = c[k];
      const int id = (int)s.fronts.size();
      s.fronts.push_back(std::move(f));
      for (int k = 0; k < s.fronts[id].nchild; ++k) s.fronts[s.fronts[id].child[k]].parent = id;
      prev = id;
    }
    return prev;
  }

  // Nested dissection of the rectangle [x0,x1) x [y0,y1): cut it with one
  // grid line of nodes (vertically while w >= aspect x h, else horizontally);
  // the two parts become children.  Children are emitted before their
  // parent, so `fronts` is a postorder.
  int region(int x0, int x1, int y0, int y1) {
    int w = x1 - x0, hh = y1 - y0;
    if (w <= 0 || hh <= 0) return -1;
    std::vector<int> piv;
    int c[2] = {-1, -1};
    if ((int64_t)w * hh <= leaf) {
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) piv.push_back(node(x, y));
    } else if (w >= ((y0 <= d.src_row && d.prj_row < y1) ? kAspectFull : kAspectPart) * hh) {
      int xs = x0 + w / 2;
      c[0] = region(x0, xs, y0, y1);
      c[1] = region(xs + 1, x1, y0, y1);
      for (int y = y0; y < y1; ++y) piv.push_back(node(xs, y));
    } else {
      int ys = row_cut(y0, y1);
      c[0] = region(x0, x1, y0, ys);
      c[1] = region(x0, x1, ys + 1, y1);
      for (int x = x0; x < x1; ++x) piv.push_back(node(x, ys));
    }
    return emit(std::move(piv), c[0], c[1], x0, x1, y0, y1);
  }
};

}  // namespace

void analyze(const Desc &d, Symbolic &s) {
  if (d.nx < 3 || d.ny < 1) throw std::runtime_error("grid must have nx >= 3 and ny >= 1");
  s = Symbolic();
  s.nx = d.nx;
  s.ny = d.ny;
  const int nx = d.nx, ny = d.ny;
  const int64_t N = (int64_t)nx * ny;
  Builder bld(d, s);

  // The periodic ring is opened by the root separator: grid column x = 0.
  int child = bld.region(1, nx, 0, ny);
  {
    std::vector<int> piv;
    for (int y = 0; y < ny; ++y) piv.push_back(bld.node(0, y));
    bld.emit(std::move(piv), child, -1, 0, nx, 0, ny);
  }
  const int nf = (int)s.fronts.size();

  // Elimination order, node -> (front, local) maps.
  s.node_front.assign(N, -1);
  s.node_local.assign(N, -1);
  s.node_elim.assign(N, -1);
  int64_t e = 0;
  for (int f = 0; f < nf; ++f) {
    Front &F = s.fronts[f];
    F.elim0 = e;
    for (int k = 0; k < F.p(); ++k) {
      int n = F.piv[k];
      if (s.node_front[n] != -1) throw std::runtime_error("node pivoted twice");
      s.node_front[n] = f;
      s.node_local[n] = k;
      s.node_elim[n] = e++;
    }
  }
  if (e != N) throw std::runtime_error("nested dissection does not cover the grid");

  // Boundary sets (symbolic factorization): the nodes a front's pivots couple
  // to that are eliminated later, plus its children's boundaries, minus its
  // own pivots.  With geometric dissection these are the grid neighbours of
  // the subtree's region (ancestor separators, the periodic wrap meeting the
  // root column) and, for a chained separator, its later parts.
  {
    std::vector<int> mark(N, -1);
    for (int f = 0; f < nf; ++f) {
      Front &F = s.fronts[f];
      std::vector<int> keep;
      auto add = [&](int v) {
        if (s.node_front[v] == f || mark[v] == f) return;
        mark[v] = f;
        keep.push_back(v);
      };
      for (int u : F.piv) {
        const int x = u % nx, y = u / nx;
        const int nb[4] = {y * nx + (x - 1 + nx) % nx, y * nx + (x + 1) % nx, y > 0 ? u - nx : -1,
                           y < ny - 1 ? u + nx : -1};
        for (int v : nb)
          if (v >= 0 && s.node_elim[v] > s.node_elim[u]) add(v);
      }
      for (int c = 0; c < F.nchild; ++c)
        for (int v : s.fronts[F.child[c]].bnd) add(v);
      std::sort(keep.begin(), keep.end(), [&](int a, int c) { return s.node_elim[a] < s.node_elim[c]; });
      for (int v : keep)
        if (s.node_elim[v] < F.elim0 + F.p()) throw std::runtime_error("boundary node eliminated before its front");
      F.bnd = std::move(keep);
    }
  }

  // Extend-add maps: child boundary node -> parent-local index.
  std::vector<int> stamp(N, -1);
  for (int f = 0; f < nf; ++f) {
    Front &P = s.fronts[f];
    for (int k = 0; k < P.p(); ++k) stamp[P.piv[k]] = k;
    for (int k = 0; k < P.b(); ++k) stamp[P.bnd[k]] = P.p() + k;
    for (int c = 0; c < P.nchild; ++c) {
      Front &Ch = s.fronts[P.child[c]];
      Ch.rmap.resize(Ch.b());
      for (int k = 0; k < Ch.b(); ++k) {
        int loc = stamp[Ch.bnd[k]];
        if (loc < 0) throw std::runtime_error("child boundary not in parent front");
        Ch.rmap[k] = loc;
      }
    }
    for (int k = 0; k < P.p(); ++k) stamp[P.piv[k]] = -1;
    for (int k = 0; k < P.b(); ++k) stamp[P.bnd[k]] = -1;
  }

  // Heights, channel blocks, sweep set, levels.
  int H = 0;
  for (int f = 0; f < nf; ++f) {
    Front &F = s.fronts[f];
    int h = 0;
    for (int c = 0; c < F.nchild; ++c) h = std::max(h, s.fronts[F.child[c]].height + 1);
    F.height = h;
    H = std::max(H, h);
    F.hasB = F.y0 <= d.src_row && d.src_row < F.y1;
    F.hasC = F.y0 <= d.prj_row && d.prj_row < F.y1;
    F.sweep = F.y0 < d.design_row1 && d.design_row0 < F.y1;
    F.sfront = F.hasB && F.hasC;
  }
  s.levels.assign(H + 1, {});
  for (int f = 0; f < nf; ++f) s.levels[s.fronts[f].height].push_back(f);

  s.node_sweep_row.assign(N, -1);
  int64_t r = 0;
  for (int f = 0; f < nf; ++f) {
    Front &F = s.fronts[f];
    if (!F.sweep) continue;
    for (int k = 0; k < F.p(); ++k) s.node_sweep_row[F.piv[k]] = r++;
  }
  s.n_sweep_rows = r;

  // Work counts (complex multiply-adds).
  const double Mi = d.n_in, Mo = d.n_out;
  s.k_total = 0;
  for (int f = 0; f < nf; ++f) {
    const Front &F = s.fronts[f];
    double p = F.p(), b = F.b(), mB = F.hasB ? Mi : 0, mC = F.hasC ? Mo : 0;
    s.max_front = std::max(s.max_front, F.p() + F.b());
    if (F.sfront) s.k_total += F.p();
    // rank-p elimination of the (p+b+mC) x (p+b+mB) front, channel block included
    double a = p + b + mC - 1, c = p + b + mB - 1;
    s.algo_factor_cmacs += p * a * c - (a + c) * p * (p - 1) / 2 + p * (p - 1) * (2 * p - 1) / 6;
    double w = p * p * p;                       // pivot-block inverse
    w += p * p * b + p * p * mB;                // X12, X1B
    w += b * p * b + b * p * mB + b * p * mC;   // Schur updates of the contribution block
    if (F.sweep) w += b * p * p + (F.hasC ? p * p * mC : 0);   // Y21, XC1T
    w += mC * p * mB;                           // channel block into S
    s.factor_cmacs += w;
    if (F.sweep) {
      s.grad_cmacs += 2 * p * b * Mi;           // two sweeps
      if (F.hasC) s.grad_cmacs += p * mC * Mi;  // weighted adjoint source
    }
  }
}

}  // namespace apf
