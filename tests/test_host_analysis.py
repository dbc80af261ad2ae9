"""Host-side checks of the C library (no GPU): it loads, exports every entry
point of include/apf.h, validates descriptors, and its nested-dissection
analysis is a valid multifrontal structure for the 5-point periodic grid."""
import os
import re

import numpy as np
import pytest

from paper_2306_09257_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apf.h")

binding = pytest.importorskip("paper_2306_09257_amd.binding")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libapf.so is not built (run paper_2306_09257_amd/build.py)")
    return binding.load_library()


def test_exports_every_declared_entry_point(lib):
    decl = re.findall(r"^\s*(?:const\s+char\s*\*\s*|apf_status\s+)(apf_\w+)\s*\(", open(HEADER).read(), re.M)
    assert set(decl) == set(binding.ENTRY_POINTS)
    for name in decl:
        assert hasattr(lib, name), name


def _problem(nx, ny, **kw):
    prob, eps, w = inputs.tiny_problem(nx=nx, ny=ny, **kw)
    return prob


@pytest.mark.parametrize("mut,msg", [
    (lambda p: setattr(p, "design_row0", 2), "PML"),
    (lambda p: setattr(p, "src_row", p.design_row0), "src_row"),
    (lambda p: setattr(p, "prj_row", p.design_row1 - 1), "prj_row"),
    (lambda p: setattr(p, "in_orders", np.array([40], dtype=np.int32)), "propagate"),
    (lambda p: setattr(p, "nx", 2), "nx"),
])
def test_descriptor_validation(lib, mut, msg):
    prob = _problem(24, 60)
    mut(prob)
    with pytest.raises(binding.APFError) as ei:
        binding.APF(prob)
    assert ei.value.status == binding.APF_EINVAL
    assert msg in str(ei.value)


def _structure(apf):
    nf = int(apf.query("n_fronts"))
    fronts = [apf.front(f) for f in range(nf)]
    return fronts


@pytest.mark.parametrize("nx,ny,leaf", [(24, 60, 0), (37, 60, 16), (9, 92, 0), (240, 92, 64), (50, 60, 4)])
def test_nested_dissection_is_a_valid_multifrontal_structure(lib, nx, ny, leaf):
    prob = _problem(nx, ny)
    apf = binding.APF(prob, leaf_size=leaf).analyze()
    fronts = _structure(apf)
    nf = len(fronts)
    N = nx * ny
    owner = -np.ones(N, dtype=np.int64)
    elim = -np.ones(N, dtype=np.int64)
    for f, (info, piv, bnd) in enumerate(fronts):
        assert (owner[piv] == -1).all(), "node pivoted twice"
        owner[piv] = f
        elim[piv] = info[7] + np.arange(piv.size)
    assert (owner >= 0).all(), "some node never pivoted"
    assert sorted(elim.tolist()) == list(range(N))
    # postorder and single root
    roots = [f for f, (info, _, _) in enumerate(fronts) if info[0] < 0]
    assert roots == [nf - 1]
    for f, (info, _, _) in enumerate(fronts):
        if info[0] >= 0:
            assert info[0] > f
            assert fronts[info[0]][0][1] > info[1], "parent height must exceed child height"
    # ancestors
    anc = []
    for f in range(nf):
        s, g = set(), fronts[f][0][0]
        while g >= 0:
            s.add(g)
            g = fronts[g][0][0]
        anc.append(s)
    varset = [set(piv.tolist()) | set(bnd.tolist()) for (_, piv, bnd) in fronts]
    for f, (info, piv, bnd) in enumerate(fronts):
        # boundary nodes are pivots of ancestors, sorted by elimination order
        assert all(owner[v] in anc[f] for v in bnd)
        assert (np.diff(elim[bnd]) > 0).all()
        # child contribution block fits in the parent front
        if info[0] >= 0:
            assert set(bnd.tolist()) <= varset[info[0]]
    # every grid edge (u, v): the later node is in the front of the earlier one
    for u in range(N):
        x, y = u % nx, u // nx
        nbs = [y * nx + (x - 1) % nx, y * nx + (x + 1) % nx]
        if y > 0:
            nbs.append(u - nx)
        if y < ny - 1:
            nbs.append(u + nx)
        for v in nbs:
            a, b = (u, v) if elim[u] < elim[v] else (v, u)
            assert b in varset[owner[a]], (u, v)
    # channel blocks and sweep set follow the subtree's rows
    rows_sub = [set() for _ in range(nf)]
    for f in range(nf):
        for v in fronts[f][1]:
            g = f
            while g >= 0:
                rows_sub[g].add(int(v) // nx)
                g = fronts[g][0][0]
    for f, (info, _, _) in enumerate(fronts):
        assert info[4] == (prob.src_row in rows_sub[f])
        assert info[5] == (prob.prj_row in rows_sub[f])
        assert info[6] == bool(rows_sub[f] & set(range(prob.design_row0, prob.design_row1)))


def test_work_counts_match_a_brute_force_symbolic_elimination(lib):
    """The algorithmic count (rank-p updates of each rectangular front) must
    equal a dense symbolic elimination of K in the same order on a tiny grid:
    sum over eliminated k of (#later rows in col k) * (#later cols in row k)."""
    prob = _problem(10, 60)
    apf = binding.APF(prob, leaf_size=16).analyze()
    fronts = _structure(apf)
    nx, ny = prob.nx, prob.ny
    N = nx * ny
    order = np.concatenate([piv for (_, piv, _) in fronts])
    pos = np.empty(N, dtype=np.int64)
    pos[order] = np.arange(N)
    Mi, Mo = prob.n_in, prob.n_out
    # pattern of K in elimination order: grid part plus channel rows/columns
    pat = np.zeros((N + Mo, N + Mi), dtype=bool)
    for u in range(N):
        x, y = u % nx, u // nx
        pat[pos[u], pos[u]] = True
        for v in (y * nx + (x - 1) % nx, y * nx + (x + 1) % nx):
            pat[pos[u], pos[v]] = True
        if y > 0:
            pat[pos[u], pos[u - nx]] = True
        if y < ny - 1:
            pat[pos[u], pos[u + nx]] = True
        if y == prob.src_row:
            pat[pos[u], N:] = True
        if y == prob.prj_row:
            pat[N:, pos[u]] = True
    count = 0.0
    for k in range(N):
        rows = np.nonzero(pat[k + 1:, k])[0] + k + 1
        cols = np.nonzero(pat[k, k + 1:])[0] + k + 1
        count += rows.size * cols.size
        pat[np.ix_(rows, cols)] = True
    # the multifrontal fronts are dense: their count bounds the exact fill count
    algo = apf.query("algo_factor_cmacs")
    assert algo >= count
    # and the channel-free part is tight for leaves and separators of a strip
    assert algo <= 1.6 * count


def test_profiling_modes_are_checked(lib):
    apf = binding.APF(_problem(24, 60)).analyze()
    for mode in (0, 1, 2, 0):
        assert lib.apf_set_profiling(apf._h, mode) == binding.APF_OK
    for bad in (-1, 3):
        assert lib.apf_set_profiling(apf._h, bad) == binding.APF_EINVAL


def test_host_side_argument_and_state_checks(lib):
    """Every entry point rejects null arguments, bad values and calls out of
    order on the host, before any device work (the buffers below are host
    placeholders that none of these calls reaches)."""
    import ctypes
    E, S = binding.APF_EINVAL, binding.APF_ESTATE
    buf = np.zeros(64)
    p = buf.ctypes.data_as(ctypes.c_void_p)
    v = ctypes.c_double()

    prob = _problem(24, 60)
    fresh = binding.APF(prob)                        # created, not analysed
    assert lib.apf_query(fresh._h, b"n_fronts", ctypes.byref(v)) == S
    assert lib.apf_assemble(fresh._h, p, None) == S
    info = (ctypes.c_int32 * 8)()
    assert lib.apf_front(fresh._h, 0, info, None, None) == S

    apf = binding.APF(prob).analyze()
    h = apf._h
    assert lib.apf_query(h, b"no_such_key", ctypes.byref(v)) == E
    assert lib.apf_query(h, b"rhs_chunk", ctypes.byref(v)) == binding.APF_OK and v.value == -1.0
    nf = int(apf.query("n_fronts"))
    for f in (-1, nf):
        assert lib.apf_front(h, f, info, None, None) == E
    for cap in (-64, 100, 63):
        assert lib.apf_set_rhs_chunk(h, cap) == E
    for cap in (0, 64, 4096):
        assert lib.apf_set_rhs_chunk(h, cap) == binding.APF_OK
    for on in (-1, 3):
        assert lib.apf_set_lowrank(h, on) == E
    for on in (0, 1, 2):
        assert lib.apf_set_lowrank(h, on) == binding.APF_OK
    assert lib.apf_set_lowrank(None, 1) == E
    # numeric calls before the first assembly
    assert lib.apf_factor_schur(h, binding.APF_FP64, p, None) == S
    assert lib.apf_factor_schur(h, 7, p, None) == E          # unknown precision first
    assert lib.apf_grad(h, p, p, None) == S
    assert lib.apf_weighted_power(h, p, p, p, p, None) == S
    assert lib.apf_splitter_fom(h, p, 0.5, p, p, None) == S
    assert lib.apf_group_fom(h, p, 2, 2, p, p, None) == S
    assert lib.apf_group_fom(h, p, 0, 2, p, p, None) == E
    # null arguments
    assert lib.apf_assemble(h, None, None) == E
    assert lib.apf_factor_schur(h, binding.APF_FP64, None, None) == E
    assert lib.apf_grad(h, None, p, None) == E
    assert lib.apf_weighted_power(h, p, None, p, p, None) == E
    assert lib.apf_set_profiling(None, 1) == E
    assert lib.apf_query(None, b"n_fronts", ctypes.byref(v)) == E
    assert lib.apf_destroy(None) == binding.APF_OK
    assert b"null" in lib.apf_last_error()


def test_factorization_counter_and_stale_factor_guard(lib):
    """The handle counts its factorizations ("n_factorizations"); the autograd
    backward refuses to run when the count moved since its forward (the
    factors then belong to another permittivity)."""
    apf = binding.APF(_problem(24, 60)).analyze()
    assert apf.query("n_factorizations") == 0.0

    class Fake:
        def __init__(self, n):
            self.n = n

        def query(self, key):
            assert key == "n_factorizations"
            return float(self.n)

    binding.check_factor_epoch(Fake(3), 3)
    with pytest.raises(binding.StaleFactorsError):
        binding.check_factor_epoch(Fake(4), 3)


def test_pivot_limit_is_shared_by_the_analysis_and_the_kernels(lib):
    """No front exceeds the pivot limit the kernels are sized for (a 200-row
    separator is chained into two fronts of 100)."""
    prob = _problem(12, 200, layout=(20, 60, 40, 60, 20))
    apf = binding.APF(prob).analyze()
    ps = [apf.front(f)[0][2] for f in range(int(apf.query("n_fronts")))]
    assert max(ps) <= 128
    assert 100 in ps


def test_refinement_switch_is_checked(lib):
    apf = binding.APF(_problem(24, 60)).analyze()
    h = apf._h
    E = binding.APF_EINVAL
    for it, tol in ((-1, 1e-10), (17, 1e-10), (2, 0.0), (2, 1.0), (2, float("nan"))):
        assert lib.apf_set_refinement(h, it, tol) == E
    assert lib.apf_set_refinement(None, 2, 1e-10) == E
    assert lib.apf_set_refinement(h, 2, 1e-10) == binding.APF_OK
    assert apf.query("retained_factor_bytes") > 0
    assert lib.apf_set_refinement(h, 0, 0.0) == binding.APF_OK
    assert apf.query("retained_factor_bytes") == 0
    assert apf.query("refine_chunk") == -1.0


def test_symmetric_switch_is_checked(lib):
    """apf_set_symmetric takes 0 or 1 before the first assembly, and refuses
    to combine with refinement or compressed channels, set either way round."""
    apf = binding.APF(_problem(24, 60)).analyze()
    h = apf._h
    E, OK = binding.APF_EINVAL, binding.APF_OK
    for bad in (-1, 2):
        assert lib.apf_set_symmetric(h, bad) == E
    assert lib.apf_set_symmetric(None, 1) == E
    assert lib.apf_set_symmetric(h, 1) == OK
    assert lib.apf_set_refinement(h, 2, 1e-10) == E
    assert lib.apf_set_compression(h, 8, 3.0) == E
    assert lib.apf_set_symmetric(h, 0) == OK
    assert lib.apf_set_refinement(h, 2, 1e-10) == OK
    assert lib.apf_set_symmetric(h, 1) == E
    assert lib.apf_set_refinement(h, 0, 0.0) == OK
    assert lib.apf_set_symmetric(h, 1) == OK


@pytest.mark.parametrize("nx,ny,leaf", [(24, 60, 0), (37, 60, 16), (48, 160, 96), (300, 92, 0)])
def test_boundary_maps_keep_the_elimination_order(lib, nx, ny, leaf):
    """Each front's boundary, listed in elimination order, lands in its
    parent's local order (pivots, then boundary) at strictly increasing
    positions: the lower triangle of a child's contribution block maps into
    the lower triangle of the parent's core, which the symmetric route
    relies on."""
    apf = binding.APF(_problem(nx, ny), leaf_size=leaf).analyze()
    nf = int(apf.query("n_fronts"))
    fr = [apf.front(f) for f in range(nf)]
    elim = {}
    for info, piv, bnd in fr:
        for k, u in enumerate(piv):
            elim[int(u)] = info[7] + k
    for info, piv, bnd in fr:
        e = [elim[int(u)] for u in bnd]
        assert e == sorted(e)
        parent = info[0]
        if parent < 0:
            assert len(bnd) == 0
            continue
        pinfo, ppiv, pbnd = fr[parent]
        local = {int(u): k for k, u in enumerate(list(ppiv) + list(pbnd))}
        pos = [local[int(u)] for u in bnd]
        assert all(b > a for a, b in zip(pos, pos[1:]))
