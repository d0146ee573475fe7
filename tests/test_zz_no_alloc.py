"""GPU test of grca_cast_noalloc, the cast whose transient buffers live in a
static device array (for callers that cannot allocate): through the C ABI,
its outputs equal grca_cast's bitwise on two calls in a row, the second with
fewer rays; a cast too large for the array is refused before any launch; a
queue overflow, which it cannot recast, is reported by grca_synchronize."""
import numpy as np
import pytest

from paper_2605_10457_amd import grca, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _rays(s):
    return len(s["elevation"]) * s["rays_per_channel"]


def _outputs(torch, n):
    d = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
    t = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    return d, t


def _both(torch, ctx, ids, n, flags=0):
    """The same cast through grca_cast and grca_cast_noalloc (device outputs)."""
    st = torch.cuda.current_stream()
    d0, t0 = _outputs(torch, n)
    ctx.cast(ids, d0, t0, flags=flags, stream=st)
    ctx.synchronize(st)
    d1, t1 = _outputs(torch, n)
    ctx.cast_noalloc(ids, d1, t1, flags=flags, stream=st)
    ctx.synchronize(st)
    return (d0.cpu().numpy(), t0.cpu().numpy()), (d1.cpu().numpy(), t1.cpu().numpy())


def _equal(a, b, label):
    (da, ta), (db, tb) = a, b
    assert np.array_equal(ta, tb), f"{label}: ids differ at {np.nonzero(ta != tb)[0][:8]}"
    assert np.array_equal(da.view(np.uint32), db.view(np.uint32)), f"{label}: distances differ"


def test_noalloc_equals_cast_on_two_calls(torch):
    wl = synth.config1()
    big = wl.sensors[0]
    small = synth.sensor((3.0, -2.0, 1.5), 0.4, synth.elevations_uniform(-20, 10, 16), 200,
                         180.0, 0.05, 80.0)
    ctx = grca.Context(0)
    try:
        ctx.scene_update(0, wl.scene.vertices, wl.scene.indices)
        ctx.sensor_config(0, big, 0)
        ctx.sensor_config(1, small, 0)
        n1 = _rays(big) + _rays(small)
        _say(f"no-alloc call 1: config1 scene, sensors 0 and 1 ({n1} rays)")
        ref, got = _both(torch, ctx, [0, 1], n1)
        _equal(ref, got, "call 1")
        assert np.count_nonzero(np.isfinite(got[0])) > n1 // 4
        n2 = _rays(small)
        _say(f"no-alloc call 2: sensor 1 only ({n2} rays)")
        ref, got = _both(torch, ctx, [1], n2)
        _equal(ref, got, "call 2")
        _say("no-alloc call 3: single-sided, sensor 0")
        ref, got = _both(torch, ctx, [0], _rays(big), grca.GRCA_CULL_BACKFACE)
        _equal(ref, got, "call 3 (single-sided)")
    finally:
        ctx.close()


def test_noalloc_limits_and_overflow(torch):
    wl = synth.config1()
    ctx = grca.Context(0)
    st = torch.cuda.current_stream()
    try:
        ctx.scene_update(0, wl.scene.vertices, wl.scene.indices)
        ctx.sensor_config(0, wl.sensors[0], 0)
        # 160 x 65535 rays need 84 MB of keys alone: refused, nothing launched
        huge = synth.sensor((0.0, 0.0, 1.8), 0.0, synth.elevations_uniform(-15, 15, 160), 65535,
                            360.0, 0.05, 100.0)
        ctx.sensor_config(5, huge, 0)
        d, t = _outputs(torch, 16)
        _say("no-alloc: a cast too large for the scratch array is refused")
        with pytest.raises(grca.GrcaError) as e:
            ctx.cast_noalloc([5], d, t, stream=st)
        assert e.value.status == grca.GRCA_ERR_CAPACITY
        with pytest.raises(grca.GrcaError) as e:
            ctx.cast_noalloc(list(range(65)), d, t, stream=st)
        assert e.value.status == grca.GRCA_ERR_INVALID_ARG
        with pytest.raises(grca.GrcaError) as e:
            ctx.cast_noalloc([0], d, t, flags=grca.GRCA_CAST_ALL_PAIRS, stream=st)
        assert e.value.status == grca.GRCA_ERR_INVALID_ARG
        ctx.synchronize(st)
        n = _rays(wl.sensors[0])
        _say("no-alloc: one queue entry per shard overflows; grca_synchronize reports it")
        ctx.set_options(item_capacity=64, large_capacity=64)
        d, t = _outputs(torch, n)
        ctx.cast_noalloc([0], d, t, stream=st)
        with pytest.raises(grca.GrcaError) as e:
            ctx.synchronize(st)
        assert e.value.status == grca.GRCA_ERR_CAPACITY
        ctx.synchronize(st)  # reported once
        ctx.set_options(item_capacity=1 << 20, large_capacity=1 << 16)
        _say("no-alloc: after the overflow, a cast with the default capacities is whole again")
        ref, got = _both(torch, ctx, [0], n)
        _equal(ref, got, "after overflow")
    finally:
        ctx.close()
