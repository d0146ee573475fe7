"""GPU parity at the full sizes of the stated workloads: the 5M-triangle
deforming scene of 8 uneven sensors at two frames, the 22M-triangle scene of 8
128x4096 sensors at every range limit (1000, 100, 50 and 10 m), with the culled
cast of a full 360-degree sensor bitwise equal to testing every ray against
every triangle.  Oracle samples are seeded; every case prints its progress."""
import numpy as np
import pytest

from paper_2605_10457_amd import grca, synth
from tests import helpers

pytestmark = pytest.mark.gpu
say = helpers.say


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _rays(wl):
    return sum(len(s["elevation"]) * s["rays_per_channel"] for s in wl.sensors)


@pytest.mark.parametrize("frame", [0, 25])
def test_config3_full_scale(torch, frame):
    wl = synth.config3()
    sc = wl.scene
    say(f"config3 full scale frame {frame}: {sc.num_triangles} tris "
        f"({sc.n_dynamic_tris} deformable), 8 uneven sensors, 32 oracle rays per sensor")
    ctx = grca.Context(0)
    try:
        ctx.set_options(item_capacity=32 << 20, large_capacity=4 << 20)
        ids = grca.load_workload(ctx, wl, frame=frame)
        d, t = ctx.cast_host(ids, _rays(wl))
        print("stats", ctx.last_stats(), flush=True)
        v_or = helpers.oracle_pose(sc, frame)
        helpers.sample_parity(wl.sensors, v_or, sc.indices, d, t, 32, 300 + frame,
                              f"config3-f{frame}", hit_share=0.5)
    finally:
        ctx.close()


@pytest.fixture(scope="module")
def config4_loaded(torch):
    wl = synth.config4()
    say(f"config4 full scale: {wl.scene.num_triangles} tris, posed at frame 2")
    ctx = grca.Context(0)
    ctx.set_options(item_capacity=96 << 20, large_capacity=8 << 20)
    grca.load_workload(ctx, wl, frame=2, first_sensor_id=0)
    yield ctx, wl, helpers.oracle_pose(wl.scene, 2)
    ctx.close()


@pytest.mark.parametrize("dmax", [1000.0, 100.0, 50.0, 10.0])
def test_config4_range_limits_full_scale(config4_loaded, dmax):
    ctx, wl, v_or = config4_loaded
    sens = [dict(s, range_max=np.float32(dmax)) for s in wl.sensors]
    ids = list(range(100, 108))
    for i, s in zip(ids, sens):
        ctx.sensor_config(i, s, 0)
    say(f"config4 full scale, range_max {dmax:g} m: 8 x 128x4096 rays, 32 oracle rays per "
        f"sensor (half among hits)")
    d, t = ctx.cast_host(ids, _rays(wl))
    st = ctx.last_stats()
    print("stats", st, flush=True)
    assert st["recasts"] == 0
    assert np.all(np.isinf(d) | (d <= dmax * (1 + 1e-6)))
    helpers.sample_parity(sens, v_or, wl.scene.indices, d, t, 32, 400 + int(dmax),
                          f"config4-range{dmax:g}", hit_share=0.5)
    if dmax in (1000.0, 10.0):
        say(f"config4 range_max {dmax:g} m: sensor 0 (360 deg) culled vs all-pairs, bitwise")
        n0 = 128 * 4096
        d0, t0 = ctx.cast_host([ids[0]], n0, grca.GRCA_CAST_ALL_PAIRS)
        assert np.array_equal(t0, t[:n0])
        assert np.array_equal(d0.view(np.uint32), d[:n0].view(np.uint32))
        print(f"all-pairs equal, {int(np.count_nonzero(np.isfinite(d0)))} hits", flush=True)
