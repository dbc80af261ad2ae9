// Host-only driver of the nested-dissection analysis, built with the address
// and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.  It
// analyses a set of grids (channel rows, design band, leaf sizes, chained
// separators) and checks that every node is pivoted once and that every
// boundary node is eliminated after its front.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2306_09257_amd/csrc/apf_internal.h"

using namespace apf;

static int check(int nx, int ny, int leaf, int npml, int d0, int d1) {
  Desc d{};
  d.nx = nx; d.ny = ny; d.dx_over_lambda = 0.05;
  d.npml_top = npml; d.npml_bot = npml; d.pml_R0 = 1e-8; d.pml_power = 3;
  d.eps_top = 1.0; d.eps_bot = 2.25;
  d.src_row = npml + 1; d.prj_row = ny - npml - 2;
  d.design_row0 = d0; d.design_row1 = d1;
  d.n_in = 3; d.n_out = 3; d.in_orders = {-1, 0, 1}; d.out_orders = {-1, 0, 1};
  d.leaf_size = leaf;
  Symbolic s;
  analyze(d, s);
  std::vector<int> seen((size_t)nx * ny, 0);
  for (const Front &F : s.fronts) {
    if (F.p() > MAX_PIVOTS) return 1;
    for (int u : F.piv) seen[u]++;
    for (int v : F.bnd)
      if (s.node_elim[v] < F.elim0 + F.p()) return 2;
    if ((int)F.rmap.size() != F.b()) return 3;
  }
  for (int c : seen)
    if (c != 1) return 4;
  return 0;
}

int main() {
  struct G { int nx, ny, leaf, npml, d0, d1; } grids[] = {
      {3, 60, 0, 16, 20, 40},    {24, 60, 0, 16, 20, 40},   {37, 60, 16, 16, 20, 40},
      {240, 92, 0, 16, 36, 56},  {130, 60, 128, 16, 20, 40}, {12, 200, 0, 20, 80, 120},
      {48, 160, 96, 20, 60, 100}, {1200, 92, 0, 16, 36, 56}, {2000, 160, 0, 20, 60, 100},
  };
  for (const G &g : grids) {
    const int r = check(g.nx, g.ny, g.leaf, g.npml, g.d0, g.d1);
    std::printf("%dx%d leaf %d: %s\n", g.nx, g.ny, g.leaf, r ? "FAIL" : "ok");
    if (r) return 10 + r;
  }
  return 0;
}
