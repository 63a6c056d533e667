"""Batched solves of many uneven systems (one launch per V-cycle phase for all
meshes) against the oracle: every mesh's solution must satisfy the oracle's
system to 1e-6 relative residual, per right-hand side, in FP64 and in mixed
precision; a zero right-hand side gives a zero solution; the batch agrees with
the same systems solved one at a time.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_1505_03615_amd import meshgen

pytestmark = pytest.mark.gpu
T = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _meshes():
    out = []
    V, F = meshgen.icosphere(2)
    out.append((V, F, 4, 1))
    V, F = meshgen.icosphere(3)
    out.append((V, F, 5, 3))
    V, F = meshgen.torus(2.0, 0.6, 48, 16)
    out.append((V, F, 5, 5))
    V, F = meshgen.noisy_sphere(3, seed=2)
    out.append((V, F, 6, 2))
    V, F, _, _ = meshgen.two_sheets(32, 1.0 / 32)
    out.append((V, F, 5, 1))
    V, F = meshgen.torus_knot(nu=1024, nv=16, seed=3)
    out.append((V, F, 7, 4))
    return out


@pytest.fixture(scope="module")
def cf():
    import torch
    from paper_1505_03615_amd import camfe
    assert torch.cuda.is_available()
    return camfe


@pytest.fixture(scope="module")
def setup(cf):
    ctx = cf.camfe_ctx_create(0)
    rng = np.random.default_rng(5)
    items = []
    for i, (V, F, depth, k) in enumerate(_meshes()):
        say(f"[gpu] batch: mesh {i} nt={len(F)} depth={depth} k={k}")
        h = cf.camfe_hierarchy_build(ctx, V, F, depth=depth, degree=1, max_coarse=256)
        s = cf.camfe_assemble(h)
        o = Oracle(V, F, depth, degree=1, max_coarse=256).check().assemble()
        fv = rng.normal(size=(len(V), k))
        if i == 2:
            fv[:, 1] = 0.0                      # one zero right-hand side
        b = o.load_vector(fv)
        items.append((h, s, o, b))
    say("[gpu] batch: create")
    bt = cf.camfe_batch_create(ctx, [it[1] for it in items], T)
    yield ctx, items, bt
    cf.camfe_batch_destroy(bt)
    for h, s, o, b in items:
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    cf.camfe_ctx_destroy(ctx)


def _check(items, xs, stats, tol=1e-6):
    for i, ((h, s, o, b), x, st) in enumerate(zip(items, xs, stats)):
        Mo, Lo = o.matrices(o.depth)
        A = Mo + T * Lo
        bn = np.linalg.norm(b, axis=0)
        r = np.linalg.norm(b - A @ x, axis=0) / np.where(bn > 0, bn, 1.0)
        assert np.all(r <= tol), (i, r, st)
        zero = bn == 0
        assert np.all(x[:, zero] == 0), i


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_solves_every_mesh(cf, setup, precision):
    ctx, items, bt = setup
    levels, rows = cf.camfe_batch_info(bt)
    assert rows >= sum(it[3].shape[0] for it in items) and levels >= 4
    say(f"[gpu] batch: solve precision={precision} levels={levels} rows={rows}")
    xs, stats = cf.camfe_batch_solve(bt, [it[3] for it in items], T, rtol=1e-8, max_iter=800, precision=precision)
    say("[gpu] batch: cycles " + " ".join(str(st["cycles"]) for st in stats) +
        f" ms {1e3 * stats[0]['seconds']:.2f}")
    assert all(st["converged"] for st in stats), stats
    _check(items, xs, stats)


def test_batch_sweeps_below_the_finest_depth(cf, setup):
    """nu_coarse reaches every member's coarse depths: V(3,3) at the finest
    depth with V(1,1) below meets the oracle's residual bar in both
    precisions, its iterates differ from V(3,3) everywhere, and the default
    solve afterwards gives the same bits as before (the captured cycles are
    kept apart per sweep schedule)."""
    ctx, items, bt = setup
    bs = [it[3] for it in items]
    x0, s0 = cf.camfe_batch_solve(bt, bs, T, rtol=1e-8, max_iter=800)
    for precision in (0, 1):
        say(f"[gpu] batch: nu 3 below 1, precision={precision}")
        xs, stats = cf.camfe_batch_solve(bt, bs, T, rtol=1e-8, max_iter=800, nu_pre=3, nu_post=3, nu_coarse=1,
                                         precision=precision)
        assert all(st["converged"] for st in stats), stats
        _check(items, xs, stats)
    x33, _ = cf.camfe_batch_solve(bt, bs, T, rtol=1e-30, max_iter=2, nu_pre=3, nu_post=3)
    x31, _ = cf.camfe_batch_solve(bt, bs, T, rtol=1e-30, max_iter=2, nu_pre=3, nu_post=3, nu_coarse=1)
    assert all(not np.array_equal(a, b) for a, b in zip(x33, x31))
    x1, s1 = cf.camfe_batch_solve(bt, bs, T, rtol=1e-8, max_iter=800)
    assert all(np.array_equal(a, b) for a, b in zip(x0, x1))
    assert [st["cycles"] for st in s0] == [st["cycles"] for st in s1]
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_batch_solve(bt, bs, T, nu_coarse=64)


def test_batch_matches_single_solves(cf, setup):
    ctx, items, bt = setup
    xs, stats = cf.camfe_batch_solve(bt, [it[3] for it in items], T, rtol=1e-10, max_iter=800)
    for i, (h, s, o, b) in enumerate(items):
        say(f"[gpu] batch: single solve {i}")
        x1, st1 = cf.camfe_solve(s, b, t=T, rtol=1e-10, max_iter=800)
        assert st1["converged"]
        Mo, Lo = o.matrices(o.depth)
        A = Mo + T * Lo
        # same system, both to 1e-10: the solutions agree to the solve accuracy in the A-norm
        e = xs[i] - x1
        num = np.sqrt(np.einsum("ij,ij->j", e, A @ e))
        den = np.sqrt(np.einsum("ij,ij->j", x1, A @ x1))
        assert np.all(num <= 1e-6 * np.where(den > 0, den, 1.0)), (i, num, den)


def test_converged_members_drop_out_without_changing_the_rest(cf, setup):
    """Members stop costing anything once all their columns converge (their
    slices, transfers, coarse solves and CG blocks are skipped).  Every
    member's arithmetic is its own, so its iterate, its iteration count and
    its residual are bit for bit those of a batch holding it alone: a gate
    that skipped a live member's rows, or let a frozen member change, fails
    here.  The iteration counts are the members' own, not the batch's."""
    ctx, items, bt = setup
    xs, stats = cf.camfe_batch_solve(bt, [it[3] for it in items], T, rtol=1e-10, max_iter=800)
    its = [st["iterations"] for st in stats]
    say(f"[gpu] batch: iterations per member {its}")
    assert min(its) < max(its)
    for i in (0, 2, 5):
        h, s, o, b = items[i]
        one = cf.camfe_batch_create(ctx, [s], T)
        try:
            x1, st1 = cf.camfe_batch_solve(one, [b], T, rtol=1e-10, max_iter=800)
        finally:
            cf.camfe_batch_destroy(one)
        assert st1[0]["iterations"] == stats[i]["iterations"], (i, st1[0], stats[i])
        assert st1[0]["rel_residual"] == stats[i]["rel_residual"], i
        assert np.array_equal(x1[0], xs[i]), (i, np.abs(x1[0] - xs[i]).max())


def test_batch_warm_start_and_errors(cf, setup):
    ctx, items, bt = setup
    xs, stats = cf.camfe_batch_solve(bt, [it[3] for it in items], T, rtol=1e-9, max_iter=800)
    xs2, stats2 = cf.camfe_batch_solve(bt, [it[3] for it in items], T, rtol=1e-9, max_iter=800, x0s=xs)
    assert all(st["iterations"] == 0 for st in stats2)
    _check(items, xs2, stats2)
    with pytest.raises(cf.CamfeError, match="EINVAL"):
        cf.camfe_batch_solve(bt, [it[3] for it in items], 2 * T)


def test_batch_with_a_system_listed_per_column_chunk(cf, setup):
    """A system may appear several times in one batch (here once per chunk of
    at most four right-hand sides), so one pass of the batch covers all its
    columns; each chunk must satisfy the oracle's system."""
    ctx, items, bt = setup
    h, s, o, b = items[2]                       # five right-hand sides, one of them zero
    chunks = [b[:, :4], b[:, 4:]]
    say("[gpu] batch: one system per column chunk")
    bt2 = cf.camfe_batch_create(ctx, [s, s, items[0][1]], T)
    try:
        xs, stats = cf.camfe_batch_solve(bt2, chunks + [items[0][3]], T, rtol=1e-8, max_iter=800)
        assert all(st["converged"] for st in stats), stats
        _check([(h, s, o, chunks[0]), (h, s, o, chunks[1]), items[0]], xs, stats)
    finally:
        cf.camfe_batch_destroy(bt2)


@pytest.fixture(scope="module")
def config4(cf):
    """Seventeen members of the config-4 batch generator: the first sixteen of
    at most 21k triangles at their own depths (6-7), and the 1,924-triangle
    torus (R/r = 5.49) at depth 9 (760k functions), each with its 1-16
    Gaussian right-hand sides; one batch member per (mesh, chunk of <= 4
    columns)."""
    ctx = cf.camfe_ctx_create(0)
    B = meshgen.config4_batch()
    picks = [(i, B[i]["depth"]) for i in range(len(B)) if len(B[i]["F"]) <= 21000 and B[i]["depth"] <= 7][:16]
    picks.append((55, 9))
    items = []
    for i, depth in picks:
        m = B[i]
        say(f"[gpu] config 4: member {i} ({m['kind']}) nt={len(m['F'])} depth={depth} k={m['fv'].shape[1]}")
        h = cf.camfe_hierarchy_build(ctx, m["V"], m["F"], depth=depth, max_coarse=4096)
        s = cf.camfe_assemble(h)
        o = Oracle(m["V"], m["F"], depth, max_coarse=4096).check().assemble()
        items.append((h, s, o, o.load_vector(m["fv"])))
    yield ctx, items
    for h, s, o, b in items:
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    cf.camfe_ctx_destroy(ctx)


def test_config4_batch_meets_the_oracle_per_mesh_and_column(cf, config4):
    ctx, items = config4
    assert len(items) >= 17 and max(it[2].depth for it in items) >= 9
    mem, chunks, owner = [], [], []
    for j, (h, s, o, b) in enumerate(items):
        for c0 in range(0, b.shape[1], 4):
            mem.append(s)
            chunks.append(np.asfortranarray(b[:, c0:c0 + 4]))
            owner.append(j)
    bt = cf.camfe_batch_create(ctx, mem, T)
    try:
        for tuned in (False, True):
            if tuned:
                tiles, ms = cf.camfe_batch_autotune(bt, precision=0, reps=3)
                levels, _ = cf.camfe_batch_info(bt)
                assert len(tiles) == levels and np.all((tiles >= 0) & (tiles < len(cf.TILES))) and np.all(ms > 0)
                say(f"[gpu] config 4: tiles {tiles.tolist()}")
            xs, stats = cf.camfe_batch_solve(bt, chunks, T, rtol=1e-8, max_iter=2000)
            say(f"[gpu] config 4 ({'autotuned' if tuned else 'default'} tiles): {len(mem)} members, "
                f"{1e3 * stats[0]['seconds']:.1f} ms, up to {max(st['iterations'] for st in stats)} iterations")
            assert all(st["converged"] for st in stats)
            _check([(items[j][0], items[j][1], items[j][2], c) for j, c in zip(owner, chunks)], xs, stats)
    finally:
        cf.camfe_batch_destroy(bt)


def test_system_autotune_keeps_the_solution(cf, config4):
    """The autotuner only picks among tiles of the same arithmetic: a solve
    after it gives the oracle's residual bar again, and the tiles survive a
    rebuilt solver (another t)."""
    ctx, items = config4
    h, s, o, b = items[-1]                       # the depth-9 torus
    tiles, ms = cf.camfe_system_autotune(s, T, precision=1, reps=3)
    assert len(tiles) == o.depth - o.coarsest + 1 and np.all(ms > 0)
    for t in (T, 2 * T):
        x, st = cf.camfe_solve(s, b[:, :2], t=t, rtol=1e-8, max_iter=2000, precision=1)
        Mo, Lo = o.matrices(o.depth)
        r = np.linalg.norm(b[:, :2] - (Mo + t * Lo) @ x, axis=0) / np.linalg.norm(b[:, :2], axis=0)
        assert st["converged"] and np.all(r <= 1e-6), (t, r)
