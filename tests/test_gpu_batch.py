"""GPU tests of batched multi-set RK2 stepping: the persistent kernel, its
hipGraph replay and the one-launch-per-set path agree bit for bit with each
other and with each set stepped alone; every set matches the oracle; the
launch shape and the autotuner change nothing in the results."""
import os

import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import assert_fields_close, assert_positions_close

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")

SIZES = [1, 5, 63, 64, 1000, 4099, 1, 777, 2048, 33]


def make_sets(sizes, seed=0):
    sets, states = [], []
    for i, n in enumerate(sizes):
        arrays = si.random_state(si.BASE_FIELDS, int(n), seed=seed + i)
        ps = soax.ParticleSet(si.BASE_FIELDS, int(n))
        ps.upload_soa(arrays)
        sets.append(ps)
        states.append(arrays)
    return sets, states


def plan(k):
    _, dts, abc = si.batch_plan(k, seed=1)
    return dts, abc


def download(sets):
    torch.cuda.synchronize()
    return [s.download_soa() for s in sets]


def same(a, b):
    return all(np.array_equal(x, y) for sa, sb in zip(a, b) for x, y in zip(sa, sb))


@pytest.mark.parametrize("mode", [soax.PER_SET, soax.PERSISTENT, soax.GRAPH])
def test_batch_matches_oracle(ref, mode):
    sets, states = make_sets(SIZES)
    dts, abc = plan(len(SIZES))
    b = soax.Batch(sets)
    b.step(dts, abc, 25, mode=mode)
    got = download(sets)
    sch = ref.Schema(si.BASE_FIELDS)
    for s, (arrays, g) in enumerate(zip(states, got)):
        want = [a.copy() for a in arrays]
        ref.step_soa(sch, want, ref.RK2_ABC, dts[s], 25, abc=abc[s], wrap=True)
        assert np.array_equal(g[0], want[0])
        for d in range(3):
            assert_positions_close(g[1 + d], want[1 + d])
            assert_fields_close(g[4 + d], want[4 + d])


def test_one_large_step_set_switches_to_checked_kernel(ref):
    sets, states = make_sets(SIZES)
    dts, abc = plan(len(SIZES))
    dts = dts.copy()
    dts[3] = 0.2  # dt * (A+B+C) > 1/8 for this set only
    soax.Batch(sets).step(dts, abc, 6, mode=soax.GRAPH)
    got = download(sets)
    sch = ref.Schema(si.BASE_FIELDS)
    for s, (arrays, g) in enumerate(zip(states, got)):
        want = [a.copy() for a in arrays]
        ref.step_soa(sch, want, ref.RK2_ABC, dts[s], 6, abc=abc[s], wrap=True)
        for d in range(3):
            assert_positions_close(g[1 + d], want[1 + d])
            assert_fields_close(g[4 + d], want[4 + d])


def test_modes_and_single_sets_bit_identical():
    dts, abc = plan(len(SIZES))
    results = []
    for mode in (soax.PER_SET, soax.PERSISTENT, soax.GRAPH):
        sets, _ = make_sets(SIZES)
        soax.Batch(sets).step(dts, abc, 13, mode=mode)
        results.append(download(sets))
    assert same(results[0], results[1]) and same(results[0], results[2])
    sets, _ = make_sets(SIZES)
    for s, ps in enumerate(sets):
        ps.step("soa", "rk2_abc", dts[s], 13, abc=abc[s], wrap=True)
    assert same(results[0], download(sets))


def test_launch_shape_does_not_change_results():
    dts, abc = plan(len(SIZES))
    base = None
    for block, ppt, bpc in [(256, 1, 65536), (256, 2, 8), (64, 1, 1), (128, 4, 2), (512, 2, 16),
                            (512, 4, 1), (128, 2, 65536)]:
        sets, _ = make_sets(SIZES)
        b = soax.Batch(sets)
        b.config(block, ppt, bpc)
        assert b.get_config() == (block, ppt, bpc)
        b.step(dts, abc, 7, mode=soax.GRAPH)
        got = download(sets)
        if base is None:
            base = got
        assert same(base, got), (block, ppt, bpc)


def test_graph_replays_match_eager():
    dts, abc = plan(len(SIZES))
    gsets, _ = make_sets(SIZES, seed=3)
    esets, _ = make_sets(SIZES, seed=3)
    gb, eb = soax.Batch(gsets), soax.Batch(esets)
    for rep in range(4):
        d2 = dts * (1.0 + 0.1 * rep)  # new parameters each replay reach the captured kernels
        gb.step(d2, abc, 5, mode=soax.GRAPH)
        eb.step(d2, abc, 5, mode=soax.PERSISTENT)
        torch.cuda.synchronize()
        probe = torch.ones(1000, device="cuda").sum()  # eager work between replays
        assert probe.item() == 1000.0
        assert same(download(gsets), download(esets)), rep


def test_graphs_follow_the_largest_tier_of_the_step():
    # the batch kernel is instantiated for the largest shift tier among the
    # sets: a graph captured while every set is in the small tier must not be
    # replayed once a set needs the mid or the unbounded tier
    k = len(SIZES)
    _, abc = plan(k)
    small = np.full(k, 1e-3)
    mixed = small.copy()
    mixed[2] = 0.02  # dt (|A|+|B|+|C|) in (1/64, 1/8]: mid tier
    mixed[5] = 0.2   # beyond 1/8: unbounded tier
    gsets, _ = make_sets(SIZES, seed=9)
    gb = soax.Batch(gsets)
    for dts in (small, mixed, small, mixed):
        gb.step(dts, abc, 3, mode=soax.GRAPH)
    ssets, _ = make_sets(SIZES, seed=9)
    for dts in (small, mixed, small, mixed):
        for i, ps in enumerate(ssets):
            ps.step("soa", "rk2_abc", dts[i], 3, abc=abc[i], wrap=True)
    assert same(download(gsets), download(ssets))


def test_tuner_keeps_state_and_writes_cache(tmp_path):
    dts, abc = plan(len(SIZES))
    sets, _ = make_sets(SIZES, seed=5)
    b = soax.Batch(sets)
    before = download(sets)
    cache = str(tmp_path / "tune.json")
    cfg = b.tune(cache)
    after = download(sets)
    assert same(before, after)
    assert cfg[0] in (64, 128, 256, 512) and cfg[1] in (1, 2, 4) and cfg[2] in (2, 4, 8, 16, 32, 64, 65536)
    assert os.path.exists(cache)
    text = open(cache).read()
    assert "batch_rk2" in text and f'"block": {cfg[0]}' in text
    b2 = soax.Batch(make_sets(SIZES, seed=5)[0])
    assert b2.tune(cache) == cfg  # answered from the cache
    b.step(dts, abc, 3, mode=soax.GRAPH)
    b2.step(dts, abc, 3, mode=soax.GRAPH)
    assert same(download(b.sets), download(b2.sets))


def test_config_defaults_and_rejects_bad_shapes():
    sets, _ = make_sets(SIZES[:3])
    b = soax.Batch(sets)
    # default: one tile per workgroup, one particle per thread
    assert b.get_config() == (256, 1, 65536)
    for block, ppt, bpc in [(100, 0, 0), (1024, 0, 0), (0, 3, 0), (0, 0, 65537), (0, 0, -1)]:
        with pytest.raises(soax.SoaxError):
            b.config(block, ppt, bpc)
    assert b.get_config() == (256, 1, 65536)


@pytest.mark.parametrize("mode", [soax.PER_SET, soax.PERSISTENT, soax.GRAPH])
def test_empty_sets_in_a_batch(mode):
    # empty sets, one of them without any SoA arrays, change nothing for the others
    sizes = [5, 0, 1000, 0]
    dts, abc = plan(len(sizes))
    sets, _ = make_sets([5, 1000], seed=30)
    empty_soa = soax.ParticleSet(si.BASE_FIELDS, 0)
    empty_aos_only = soax.ParticleSet(si.BASE_FIELDS, 0, soa=False)
    batch_sets = [sets[0], empty_aos_only, sets[1], empty_soa]
    soax.Batch(batch_sets).step(dts, abc, 6, mode=mode)
    got = download(sets)
    alone, _ = make_sets([5, 1000], seed=30)
    for s, k in ((alone[0], 0), (alone[1], 2)):
        s.step("soa", "rk2_abc", dts[k], 6, abc=abc[k], wrap=True)
    assert same(got, download(alone))
    assert empty_soa.n == 0 and empty_aos_only.n == 0
