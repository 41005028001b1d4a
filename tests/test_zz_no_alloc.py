"""sd3_distance_noalloc (the allocation-free variant of sd3_distance, for
callers that cannot allocate) against sd3_distance, through the C-ABI.

Both entry points run the same kernels, so the bar is identical bits of
every distance and flag; the second of two calls in a row takes a smaller
input (the shared static scratch keeps the first call's contents).  Inputs
beyond the documented limits are refused with SD3_E_CAPACITY and leave the
outputs untouched.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1808_09571_amd import sd3, synth


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sd3.Context(0)


def _bits(x):
    return x.cpu().numpy().view(np.int64)


def _batches(rows, seed0):
    A, B = [], []
    for k in range(rows):
        a, b = synth.config_icospheres(seed0 + k)
        A.append(a)
        B.append(b)
    return (sd3.Batch.from_packed(synth.pack(A), "cuda:0"), sd3.Batch.from_packed(synth.pack(B), "cuda:0"))


def _soup_batches(rows, seed0):
    A = [synth.random_triangle_soup(300 + 17 * k, seed0 + k, scale=1.0, size=0.3) for k in range(rows)]
    B = [synth.random_triangle_soup(200 + 31 * k, seed0 + 100 + k, scale=1.0, size=0.3) for k in range(rows)]
    return (sd3.Batch.from_packed(synth.pack(A), "cuda:0"), sd3.Batch.from_packed(synth.pack(B), "cuda:0"))


def _check_pair(ctx, ba, bb, **kw):
    import torch
    d0, h0 = ctx.distance(ba, bb, **kw)
    d = torch.full((ba.count,), -1.0, dtype=torch.float64, device="cuda:0")
    h = torch.full((ba.count,), 7, dtype=torch.uint8, device="cuda:0")
    ctx.distance_noalloc(ba, bb, out=(d, h), **kw)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(d), _bits(d0)), (d.cpu().numpy(), d0.cpu().numpy())
    assert np.array_equal(h.cpu().numpy(), h0.cpu().numpy())
    return d, h


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_calls_match_sd3_distance(ctx, precision):
    # a larger call, then a smaller one: the second runs on the scratch the
    # first left behind
    ba, bb = _batches(12, 0)
    _check_pair(ctx, ba, bb, precision=precision)
    sa, sb = _batches(3, 40)
    _check_pair(ctx, sa, sb, precision=precision)


def test_orders_tiles_and_soups_match(ctx):
    ba, bb = _soup_batches(9, 5)
    for order in ("none", "bound"):
        for tile in (32, 64, 128):
            _check_pair(ctx, ba, bb, order=order, tile=tile)
    sa, sb = _soup_batches(2, 70)
    _check_pair(ctx, sa, sb, order="bound", tile=64)


def test_rescue_overflow_recomputes_inside_the_scratch(ctx):
    # a tiny rescue list forces the plain FP64 re-run, still without allocation
    ba, bb = _batches(4, 7)
    d, h = _check_pair(ctx, ba, bb, rescue_cap=1)
    _, _, st = ctx.distance_noalloc(ba, bb, rescue_cap=1, stats=True)
    assert st["fallback"] >= 1


def test_limits_are_refused_and_outputs_untouched(ctx):
    import torch
    # more rows than the staging allows
    rows = 4097
    tri = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64), np.array([[0, 1, 2]], np.int32))
    far = (tri[0] + 3.0, tri[1])
    ba = sd3.Batch.from_packed(synth.pack([tri] * rows), "cuda:0")
    bb = sd3.Batch.from_packed(synth.pack([far] * rows), "cuda:0")
    d = torch.full((rows,), -1.0, dtype=torch.float64, device="cuda:0")
    h = torch.full((rows,), 7, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(sd3.SD3Error) as e:
        ctx.distance_noalloc(ba, bb, out=(d, h))
    assert e.value.name == "SD3_E_CAPACITY" and "4096 rows" in str(e.value)
    assert bool((d == -1.0).all()) and bool((h == 7).all())
    # more triangles than the 128 MiB scratch holds (3e6 triangles: sort
    # buffers and FP32 tiles alone take about 200 MB)
    a = synth.random_triangle_soup(1_500_000, 1, scale=10.0, size=0.2)
    b = synth.random_triangle_soup(1_500_000, 2, scale=10.0, center=(30.0, 0.0, 0.0), size=0.2)
    ta = sd3.Batch.from_packed(synth.pack([a]), "cuda:0")
    tb = sd3.Batch.from_packed(synth.pack([b]), "cuda:0")
    d1 = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    h1 = torch.full((1,), 7, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(sd3.SD3Error) as e:
        ctx.distance_noalloc(ta, tb, out=(d1, h1))
    assert e.value.name == "SD3_E_CAPACITY" and "static scratch" in str(e.value)
    assert float(d1.cpu()[0]) == -1.0 and int(h1.cpu()[0]) == 7
    # timing would create events
    with pytest.raises(sd3.SD3Error) as e:
        o = ctx._opts("fp32", "bound", timing=True)
        ga, gb = ba.geoms(), bb.geoms()
        import ctypes
        st = ctx.lib.sd3_distance_noalloc(ctx.handle, ctypes.byref(ga), ctypes.byref(gb), d.data_ptr(),
                                          h.data_ptr(), ctypes.byref(o), None, ctx._stream(ba))
        if st != 0:
            ctx._raise(st)
    assert e.value.name == "SD3_E_INVALID_ARG"
    # the scratch still serves a valid call afterwards
    sa, sb = _batches(2, 90)
    _check_pair(ctx, sa, sb)


def test_host_inputs_match(ctx):
    A, B = [], []
    for k in range(5):
        a, b = synth.config_icospheres(200 + k)
        A.append(a)
        B.append(b)
    ha = sd3.Batch.from_packed(synth.pack(A))
    hb = sd3.Batch.from_packed(synth.pack(B))
    d0, h0 = ctx.distance(ha, hb)
    d1, h1 = ctx.distance_noalloc(ha, hb)
    assert np.array_equal(np.asarray(d0).view(np.int64), np.asarray(d1).view(np.int64))
    assert np.array_equal(np.asarray(h0), np.asarray(h1))
