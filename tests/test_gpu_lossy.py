"""GPU tests of the paper's lossy accelerations (opt-in cast flags).  Each
mode only drops candidate pairs, so per ray its answer is the exact cast's,
or a farther hit, or a miss: its closest-hit key is never below the exact
key.  The match rate against the FP64 oracle at 1 mm (the paper's Hit%
criterion) is reported; the exact cast's rate is checked too."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_10457_amd import grca, synth
from tests import parity

pytestmark = pytest.mark.gpu

MODES = {
    "area": grca.GRCA_LOSSY_AREA,
    "cspan": grca.GRCA_LOSSY_CSPAN,
    "rspan": grca.GRCA_LOSSY_RSPAN,
    "all": grca.GRCA_LOSSY_AREA | grca.GRCA_LOSSY_CSPAN | grca.GRCA_LOSSY_RSPAN,
}


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def setup():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = synth.config1()
    sensors = [wl.sensors[0],
               synth.sensor((6.0, -4.0, 1.6), 0.8, synth.elevations_full_sphere(24), 256,
                            180.0, 0.05, 120.0),
               synth.sensor((-3.0, 9.0, 2.2), -2.0, synth.elevations_uniform(-30, 20, 40), 300,
                            360.0, 0.05, 200.0)]
    ctx = grca.Context(0)
    ctx.scene_update(0, wl.scene.vertices, wl.scene.indices)
    for i, s in enumerate(sensors):
        ctx.sensor_config(i, s, 0)
    sizes = [len(s["elevation"]) * s["rays_per_channel"] for s in sensors]
    orc = [O.cast(s, wl.scene.vertices, wl.scene.indices) for s in sensors]
    yield ctx, wl, sensors, sizes, orc
    ctx.close()


def _cast(ctx, sizes, flags):
    return ctx.cast_host(list(range(len(sizes))), int(sum(sizes)), flags)


def _hit_rate(orc, sizes, d):
    m, off = [], 0
    for o, n in zip(orc, sizes):
        m.append(parity.hit_match(o, d[off:off + n]))
        off += n
    return float(np.mean(np.concatenate(m)))


def test_exact_cast_matches_oracle_at_1mm(setup):
    ctx, wl, sensors, sizes, orc = setup
    _say("exact cast: hit-distance match rate at 1 mm against the oracle")
    d, t = _cast(ctx, sizes, 0)
    rate = _hit_rate(orc, sizes, d)
    print("exact hit rate", rate, flush=True)
    assert rate >= 0.999


@pytest.mark.parametrize("mode", list(MODES))
def test_lossy_mode_only_drops_candidates(setup, mode):
    ctx, wl, sensors, sizes, orc = setup
    _say(f"lossy mode {mode}: keys never below the exact cast's")
    d0, t0 = _cast(ctx, sizes, 0)
    st0 = ctx.last_stats()
    d1, t1 = _cast(ctx, sizes, MODES[mode])
    st1 = ctx.last_stats()
    k0, k1 = parity.sort_keys(d0, t0), parity.sort_keys(d1, t1)
    assert np.all(k1 >= k0), f"{mode}: a lossy cast found a closer hit"
    changed = int(np.count_nonzero(k1 != k0))
    rate = _hit_rate(orc, sizes, d1)
    print(f"{mode}: {changed} rays differ from the exact cast, hit rate {rate:.4f}, "
          f"items {st0['rect_items']} -> {st1['rect_items']}, "
          f"rtic {st0['rtic']} -> {st1['rtic']}", flush=True)
    # the mode ran: its candidate sets differ from the exact cast's
    assert (st1["rect_items"], st1["rtic"], st1["large_records"]) != \
        (st0["rect_items"], st0["rtic"], st0["large_records"])
    assert rate >= 0.9


def test_area_threshold_culls_more_when_raised(setup):
    ctx, wl, sensors, sizes, orc = setup
    _say("apparent-area cull: a larger epsilon_A drops more hits")
    misses = []
    try:
        for eps in (0.0, 1e-6, 1e-4):
            ctx.set_options(eps_area=eps)
            d, t = _cast(ctx, sizes, grca.GRCA_LOSSY_AREA)
            misses.append(int(np.count_nonzero(np.isinf(d))))
    finally:
        ctx.set_options(eps_area=1e-6)
    d0, _ = _cast(ctx, sizes, 0)
    print("misses at eps 0 / 1e-6 / 1e-4:", misses, "exact:", int(np.count_nonzero(np.isinf(d0))),
          flush=True)
    assert misses[0] == int(np.count_nonzero(np.isinf(d0)))
    assert misses[0] <= misses[1] <= misses[2]
    assert misses[2] > misses[0]
