"""The remaining calls of the C ABI, through the binding, against the oracle:
occupied cells, systems built from the oracle's own matrices, the
per-context error record, the solver's row layout and column storage
options, and the largest coarsest depth solved directly.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_1505_03615_amd import meshgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cf():
    import torch
    from paper_1505_03615_amd import camfe
    assert torch.cuda.is_available()
    return camfe


@pytest.fixture(scope="module")
def ctx(cf):
    c = cf.camfe_ctx_create(0)
    yield c
    cf.camfe_ctx_destroy(c)


@pytest.fixture(scope="module")
def sheets(cf, ctx):
    V, F, f = meshgen.config_mesh("two_sheets", n=64, gap=1.0 / 64)
    say("[gpu] build sheets 64 depth 6")
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=6, max_coarse=512)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 6, max_coarse=512).check().assemble()
    yield V, F, f, h, s, o
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)


def test_export_cells_matches_oracle(cf, ctx, sheets):
    V, F, f, h, s, o = sheets
    for d in range(6, -1, -1):
        cells = cf.camfe_export_cells(h, d)
        assert cells.dtype == np.uint64
        assert np.array_equal(cells, o.cells(d)), d
        assert len(cells) == cf.camfe_hierarchy_info(h, d)[0]
    # every occupied cell's parent is occupied (the octree is a tree)
    for d in range(6, 0, -1):
        assert np.all(np.isin(cf.camfe_export_cells(h, d) >> np.uint64(3), cf.camfe_export_cells(h, d - 1)))


def _oracle_levels(o):
    levels = []
    for d in range(o.coarsest, o.depth + 1):
        M, L = o.matrices(d)
        levels.append({"depth": d, "keys": o.functions(d)[0], "M": M, "L": L,
                       "P": o.prolongation(d) if d > o.coarsest else None})
    return levels


@pytest.mark.parametrize("name", ["sheets", "sphere_deg2"])
def test_import_csr_reproduces_the_oracle_cycles(cf, ctx, sheets, name):
    """A system built from the oracle's M, L and P at every depth runs the
    oracle's stationary V-cycles (to 1e-9) and its CG solve (1e-6 residual)."""
    if name == "sheets":
        V, F, f, h, s, o = sheets
        t, degree = 1e-3, 1
    else:
        V, F, f = meshgen.config_mesh("icosphere_l3")
        o = Oracle(V, F, 4, degree=2, max_coarse=512).check().assemble()
        t, degree = 1e-3, 2
    si = cf.camfe_system_import_csr(ctx, degree, _oracle_levels(o), max_coarse=512)
    try:
        b = o.load_vector(f)
        for cyc in (1, 4):
            x, st = cf.camfe_solve(si, b, t=t, rtol=1e-30, max_iter=cyc, method=1)
            xo, io = o.solve(t, b, rtol=1e-30, max_iter=cyc, mode="vcycle")
            assert abs(x - xo).max() <= 1e-9 * abs(xo).max(), cyc
        x, st = cf.camfe_solve(si, b, t=t, rtol=1e-8, max_iter=2000)
        Mo, Lo = o.matrices(o.depth)
        r = np.linalg.norm(b - (Mo + t * Lo) @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert st["converged"] and np.all(r <= 1e-6), (st, r)
        # the finest matrices come back exactly as given
        import ctypes
        lib = cf.load()
        nnz = ctypes.c_int64()
        assert lib.camfe_export_matrix(si, o.depth, 0, None, None, None, 0, ctypes.byref(nnz)) == 0
        assert nnz.value == Mo.nnz
        ptr = np.zeros(Mo.shape[0] + 1, np.int64); col = np.zeros(Mo.nnz, np.int32); val = np.zeros(Mo.nnz)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.camfe_export_matrix(si, o.depth, 1, vp(ptr), vp(col), vp(val), Mo.nnz, ctypes.byref(nnz)) == 0
        assert np.array_equal(ptr, Lo.indptr) and np.array_equal(col, Lo.indices) and np.array_equal(val, Lo.data)
        # no mesh: the calls that need one say so
        with pytest.raises(cf.CamfeError, match="ESTATE"):
            cf.camfe_flow_step(si, np.zeros((len(b), 3)), 1e-3)
        out = np.zeros((len(b), 3), order="F")
        assert lib.camfe_linear_coeffs(si, vp(out)) == -7
        assert "no mesh" in cf.camfe_ctx_last_error(ctx)
    finally:
        cf.camfe_system_destroy(si)


def test_import_csr_rejects_bad_input(cf, ctx, sheets):
    V, F, f, h, s, o = sheets
    lv = _oracle_levels(o)
    bad = [dict(x) for x in lv]
    bad[1] = dict(bad[1], depth=bad[1]["depth"] + 1)          # depths not consecutive
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_system_import_csr(ctx, 1, bad)
    bad = [dict(x) for x in lv]
    # one key for every function: one colour, and its rows couple
    bad[-1] = dict(bad[-1], keys=np.zeros_like(bad[-1]["keys"]))
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_system_import_csr(ctx, 1, bad)
    assert "colour" in cf.camfe_ctx_last_error(ctx)
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_system_import_csr(ctx, 3, lv)


def test_ctx_last_error_is_per_context(cf, ctx, sheets):
    V, F, f, h, s, o = sheets
    other = cf.camfe_ctx_create(0)
    try:
        with pytest.raises(cf.CamfeError, match="ESTATE"):
            cf.camfe_export_functions(h, 0)                   # below the coarsest depth
        assert "coarsest" in cf.camfe_ctx_last_error(ctx)
        assert cf.camfe_ctx_last_error(other) == ""
        with pytest.raises(cf.CamfeError):
            cf.camfe_hierarchy_build(other, V, F, depth=13)
        assert "depth" in cf.camfe_ctx_last_error(other)
        assert "coarsest" in cf.camfe_ctx_last_error(ctx)
    finally:
        cf.camfe_ctx_destroy(other)


@pytest.mark.parametrize("name", ["sheets", "knot"])
def test_length_sorted_rows_track_the_oracle(cf, ctx, sheets, name):
    """Every colour length-sorted in 1024-row windows (the layout the library
    takes for colours of 2^19 rows and more): stationary cycles still match
    the oracle's to 1e-9 and the FP64 and mixed CG solves reach the oracle's
    residual bar; then the default layout again."""
    if name == "sheets":
        V, F, f, h, s, o = sheets
        t, own = 1e-3, False
    else:
        V, F = meshgen.torus_knot(nu=1024, nv=16, seed=3)
        f = V
        h = cf.camfe_hierarchy_build(ctx, V, F, depth=7, max_coarse=512)
        s = cf.camfe_assemble(h)
        o = Oracle(V, F, 7, max_coarse=512).check().assemble()
        t, own = 1e-4, True
    b = o.load_vector(f)
    Mo, Lo = o.matrices(o.depth)
    try:
        x_default, _ = cf.camfe_solve(s, b, t=t, rtol=1e-30, max_iter=3, method=1)
        cf.camfe_system_set_sell_sort(s, 1)
        for cyc in (1, 3):
            x, st = cf.camfe_solve(s, b, t=t, rtol=1e-30, max_iter=cyc, method=1)
            xo, io = o.solve(t, b, rtol=1e-30, max_iter=cyc, mode="vcycle")
            assert abs(x - xo).max() <= 1e-9 * abs(xo).max(), cyc
        assert abs(x - x_default).max() <= 1e-12 * abs(xo).max()
        for precision in (0, 1):
            x, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=1500, precision=precision)
            r = np.linalg.norm(b - (Mo + t * Lo) @ x, axis=0) / np.linalg.norm(b, axis=0)
            assert st["converged"] and np.all(r <= 1e-6), (precision, r)
    finally:
        cf.camfe_system_set_sell_sort(s, 0)
        if own:
            cf.camfe_system_destroy(s)
            cf.camfe_hierarchy_destroy(h)


@pytest.mark.parametrize("name", ["sheets", "knot_d9"])
def test_sixteen_bit_columns_give_the_same_bits(cf, ctx, sheets, name):
    """16-bit column codes (the default) hold the same columns in the same
    positions as 32-bit columns, so stationary cycles and CG in both
    precisions give the same bits with either storage, also with every
    colour length-sorted; most slices of the finest depth take the codes
    (on the depth-9 knot, 780k functions, some slices keep 32-bit columns
    where the Morton order jumps: both kinds in one launch)."""
    if name == "sheets":
        V, F, f, h, s, o = sheets
        t, own, depth = 1e-3, False, 6
        b = o.load_vector(f)
    else:
        V, F = meshgen.torus_knot(nu=8192, nv=32, seed=3)
        depth, t, own = 9, 1e-4, True
        h = cf.camfe_hierarchy_build(ctx, V, F, depth=depth, max_coarse=4096)
        s = cf.camfe_assemble(h)
        b = cf.camfe_load_vector(s, h, V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)
    runs = (dict(rtol=1e-30, max_iter=3, method=1), dict(rtol=1e-8, max_iter=2000, precision=0),
            dict(rtol=1e-8, max_iter=2000, precision=1))
    try:
        for sort in (0, 1):
            cf.camfe_system_set_sell_sort(s, sort)
            res = {}
            for bits in (16, 32):
                cf.camfe_system_set_sell_columns(s, bits)
                res[bits] = [cf.camfe_solve(s, b, t=t, **kw) for kw in runs]
                sl, c16, ent = cf.camfe_system_sell_stats(s, depth)
                say(f"[gpu] {name} sort {sort} bits {bits}: {c16} of {sl} slices with 16-bit codes, {ent} entries")
                if bits == 32:
                    assert c16 == 0
                else:
                    assert 0.5 * sl <= c16 <= sl
            for (x16, st16), (x32, st32) in zip(res[16], res[32]):
                assert np.array_equal(x16, x32) and st16["cycles"] == st32["cycles"]
    finally:
        cf.camfe_system_set_sell_columns(s, 16)
        cf.camfe_system_set_sell_sort(s, 0)
        if own:
            cf.camfe_system_destroy(s)
            cf.camfe_hierarchy_destroy(h)


def test_coarsest_of_3704_functions_tracks_the_oracle(cf, ctx):
    """Two concentric icospheres (level 4) at depth 5 with max_coarse 4096:
    the coarsest depth 4 has 3,704 functions, solved through the blocked
    dense inverse (up to 4096 functions, the size the bench's meshes use).
    Stationary cycles match the oracle's (dense Cholesky) to 1e-9."""
    V, F = meshgen.nested_spheres(4, 0.02)
    f = V[:, 2] + 0.1 * V[:, 0] ** 2
    h = cf.camfe_hierarchy_build(ctx, V, F, depth=5, max_coarse=4096)
    s = cf.camfe_assemble(h)
    o = Oracle(V, F, 5, max_coarse=4096).check().assemble()
    try:
        fin, d0 = cf.camfe_hierarchy_levels(h)
        assert d0 == o.coarsest == 4 and cf.camfe_hierarchy_info(h, d0)[2] == 3704
        b = o.load_vector(f)
        say("[gpu] 3704-function coarsest: 3 stationary cycles")
        x, st = cf.camfe_solve(s, b, t=1e-3, rtol=1e-30, max_iter=3, method=1)
        xo, io = o.solve(1e-3, b, rtol=1e-30, max_iter=3, mode="vcycle")
        assert abs(x - xo).max() <= 1e-9 * abs(xo).max()
    finally:
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
