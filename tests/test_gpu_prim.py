"""The radix sort and prefix sums under the hierarchy build, through the C
ABI, against numpy's stable argsort and cumsum (independent of the library).
Sizes span one partial tile, several tiles with a ragged tail, and counts
large enough that the scans of tile partials run over several chunks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1505_03615_amd import camfe as cf
    ctx = cf.camfe_ctx_create(0)
    yield cf, ctx, torch
    cf.camfe_ctx_destroy(ctx)


def _keys(rng, n, kbits, spread):
    """n random keys of kbits bits, drawn from `spread` distinct values so
    that equal keys are common (stability is visible)."""
    pool = rng.integers(0, 2 ** 63, size=max(spread, 1), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=max(spread, 1), dtype=np.uint64)
    if kbits == 32:
        pool &= np.uint64(0xFFFFFFFF)
    return pool[rng.integers(0, len(pool), size=n)]


def _expected(keys, end_bit):
    mask = np.uint64((1 << end_bit) - 1) if end_bit < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    perm = np.argsort(keys & mask, kind="stable")
    return keys[perm], perm.astype(np.uint32)


@pytest.mark.parametrize("n,kbits,end_bit,spread,with_vals", [
    (0, 64, 64, 1, True), (1, 64, 64, 1, True), (2, 64, 64, 2, True), (2047, 64, 57, 300, True),
    (2048, 64, 64, 5000, True), (2049, 64, 13, 50, True), (100_003, 64, 64, 1000, True),
    (100_003, 64, 57, 100_000, False), (65_537, 64, 1, 5, True), (4097, 64, 0, 10, True),
    (3_000_001, 64, 60, 2_000_000, True), (20_000_003, 64, 57, 10_000_000, True),
    (0, 32, 32, 1, True), (5, 32, 32, 3, True), (77_777, 32, 5, 20, True), (300_001, 32, 21, 50_000, True),
    (300_001, 32, 32, 300_001, False), (2_500_000, 32, 32, 100_000, True),
])
def test_radix_sort_is_a_stable_sort(env, n, kbits, end_bit, spread, with_vals):
    cf, ctx, torch = env
    rng = np.random.default_rng(1000 + n + end_bit + kbits)
    keys = _keys(rng, n, kbits, spread)
    if kbits == 32:
        keys = keys.astype(np.uint32).astype(np.uint64)
    exp_keys, exp_perm = _expected(keys, end_bit)
    print(f"[prim] sort n={n} key bits={kbits} end_bit={end_bit} vals={with_vals}", flush=True)
    if kbits == 64:
        kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    else:
        kd = torch.from_numpy(keys.astype(np.uint32).view(np.int32).copy()).cuda()
    vd = torch.arange(n, dtype=torch.int32, device="cuda") if with_vals else None
    torch.cuda.synchronize()     # inputs written on torch's stream, sorted on the library's
    cf.camfe_radix_sort(ctx, kd, end_bit, vd)
    got = kd.cpu().numpy()
    got = got.view(np.uint64) if kbits == 64 else got.view(np.uint32).astype(np.uint64)
    assert np.array_equal(got, exp_keys)
    if with_vals:
        assert np.array_equal(vd.cpu().numpy().view(np.uint32), exp_perm)


def test_sort_keeps_bits_above_end_bit_in_input_order(env):
    """Keys equal below end_bit but different above it keep their input
    order: only bits [0, end_bit) decide."""
    cf, ctx, torch = env
    n = 9000
    lo = np.uint64(7)
    keys = (np.arange(n, dtype=np.uint64)[::-1] << np.uint64(20)) | lo
    kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vd = torch.arange(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    cf.camfe_radix_sort(ctx, kd, 20, vd)
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(vd.cpu().numpy(), np.arange(n))


@pytest.mark.parametrize("n", [0, 1, 2, 2047, 2048, 2049, 1_000_003, 5_000_000])
@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("in_place", [False, True])
def test_exclusive_sum(env, n, bits, in_place):
    cf, ctx, torch = env
    rng = np.random.default_rng(n + bits)
    dt = np.int32 if bits == 32 else np.int64
    x = rng.integers(-50, 1000, size=n).astype(dt)
    exp = np.zeros(n, dtype=dt)
    if n:
        exp[1:] = np.cumsum(x, dtype=dt)[:-1]
    print(f"[prim] scan n={n} bits={bits} in_place={in_place}", flush=True)
    xd = torch.from_numpy(x.copy()).cuda()
    out = xd if in_place else torch.empty_like(xd)
    torch.cuda.synchronize()
    cf.camfe_exclusive_sum(ctx, xd, out)
    assert np.array_equal(out.cpu().numpy(), exp)


def test_primitive_argument_errors(env):
    cf, ctx, torch = env
    k = torch.zeros(10, dtype=torch.int64, device="cuda")
    lib = cf.load()
    assert lib.camfe_radix_sort(ctx, cf._ptr(k), 8, None, 10, 65) == -1
    assert lib.camfe_radix_sort(ctx, cf._ptr(k), 2, None, 10, 8) == -1
    assert lib.camfe_radix_sort(ctx, cf._ptr(k), 8, None, -1, 8) == -1
    assert lib.camfe_radix_sort(ctx, None, 8, None, 10, 8) == -1
    assert lib.camfe_radix_sort(ctx, cf._ptr(k), 4, None, 10, 33) == -1
    assert lib.camfe_exclusive_sum(ctx, cf._ptr(k), cf._ptr(k), 10, 2) == -1
    assert lib.camfe_exclusive_sum(ctx, None, cf._ptr(k), 10, 8) == -1
