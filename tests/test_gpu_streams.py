"""The library enqueues on the caller's stream: steps issued on side streams
(one set per stream) and steps captured into a graph and replayed give the
oracle's results.  A replay is checked after every launch, with eager work
and synchronisations between replays."""
import numpy as np
import pytest
import torch

import synth_inputs as si

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")


def test_sets_on_side_streams(ref):
    fields = si.BASE_FIELDS
    sch = ref.Schema(fields)
    streams = [torch.cuda.Stream() for _ in range(2)]
    sets, inits = [], []
    for k, st in enumerate(streams):
        arrays = si.random_state(fields, 50_000 + k, 20 + k)
        ps = soax.ParticleSet(fields, len(arrays[0]))
        ps.upload_soa(arrays)
        torch.cuda.synchronize()
        sets.append(ps)
        inits.append(arrays)
    for ps, st in zip(sets, streams):
        with torch.cuda.stream(st):
            ps.step("soa", "euler", 1e-3, 30, wrap=True)
            ps.step("soa", "rk2_abc", 1e-3, 5, abc=[1, 1, 1], wrap=True)
    for st in streams:
        st.synchronize()
    for ps, arrays in zip(sets, inits):
        want = [a.copy() for a in arrays]
        ref.step_soa(sch, want, ref.EULER, 1e-3, 30, wrap=True)
        ref.step_soa(sch, want, ref.RK2_ABC, 1e-3, 5, abc=[1, 1, 1], wrap=True)
        got = ps.download_soa()
        assert np.array_equal(got[0], want[0])
        for d in range(3):
            diff = np.abs(got[1 + d] - want[1 + d])
            assert np.minimum(diff, si.BOX_L - diff).max() <= 1e-12 * si.BOX_L
        ps.close()


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_steps_captured_in_a_graph(ref, layout):
    fields = si.BASE_FIELDS
    sch = ref.Schema(fields)
    n = 20_011
    arrays = si.random_state(fields, n, 5)
    ps = soax.ParticleSet(fields, n)
    ps.upload_soa(arrays)
    ps.soa_to_aos()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        ps.step(layout, "euler", 1e-3, 1, wrap=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ps.step(layout, "euler", 1e-3, 3, wrap=True)
    torch.cuda.synchronize()
    done = 1
    want = [a.copy() for a in arrays]
    ref.step_soa(sch, want, ref.EULER, 1e-3, 1, wrap=True)
    for rep in range(3):
        g.replay()
        done += 3
        ref.step_soa(sch, want, ref.EULER, 1e-3, 3, wrap=True)
        torch.cuda.synchronize()
        if layout == "aos":
            ps.aos_to_soa()
        torch.cuda.synchronize()
        got = ps.download_soa()
        assert all(np.array_equal(g_, w) for g_, w in zip(got, want)), (rep, done)
        # eager work between replays
        ps.step(layout, "euler", 1e-3, 1, wrap=True)
        ref.step_soa(sch, want, ref.EULER, 1e-3, 1, wrap=True)
        torch.cuda.synchronize()
    ps.close()


@pytest.mark.parametrize("layout", ["soa", "aos", "aosoa"])
def test_step_graph_matches_eager_steps(ref, layout):
    """soax_step_graph: the captured steps replayed several times, with eager
    steps between, equal the oracle's; a resized set refuses the graph."""
    fields = si.WIDE_FIELDS
    sch = ref.Schema(fields)
    n = 10_007
    arrays = si.random_state(fields, n, 12)
    ps = soax.ParticleSet(fields, n, aosoa=True)
    ps.upload_soa(arrays)
    ps.soa_to_aos()
    ps.soa_to_aosoa()
    g = ps.step_graph(layout, "euler_acc", 1e-3, 4, wrap=True)
    want = [a.copy() for a in arrays]
    for rep in range(3):
        g.launch()
        ref.step_soa(sch, want, ref.EULER_ACC, 1e-3, 4, wrap=True)
        ps.step(layout, "euler_acc", 1e-3, 1, wrap=True)
        ref.step_soa(sch, want, ref.EULER_ACC, 1e-3, 1, wrap=True)
        torch.cuda.synchronize()
    if layout == "aos":
        ps.aos_to_soa()
    elif layout == "aosoa":
        ps.aosoa_to_soa()
    torch.cuda.synchronize()
    got = ps.download_soa()
    assert all(np.array_equal(a.view(np.uint8), b.view(np.uint8)) for a, b in zip(got, want))
    ps.resize(n - 7)
    with pytest.raises(soax.SoaxError) as e:
        g.launch()
    assert e.value.status == -7
    g.close()
    ps.close()


@pytest.mark.parametrize("layout", ["soa", "aos", "aosoa"])
def test_rk2_step_graph_equals_eager_steps(layout):
    """Two replays of a captured 3-step RK2 sequence equal 6 eager steps bit
    for bit (the same kernels, launched from a graph)."""
    fields = si.BASE_FIELDS
    n = 20_011
    arrays = si.random_state(fields, n, 31)
    runs = []
    for graph in (True, False):
        ps = soax.ParticleSet(fields, n, aosoa=True)
        ps.upload_soa(arrays)
        ps.soa_to_aos()
        ps.soa_to_aosoa()
        if graph:
            g = ps.step_graph(layout, "rk2_abc", 2e-3, 3, abc=[1.0, 0.7, 0.4], wrap=True)
            g.launch()
            g.launch()
            g.close()
        else:
            ps.step(layout, "rk2_abc", 2e-3, 6, abc=[1.0, 0.7, 0.4], wrap=True)
        if layout == "aos":
            ps.aos_to_soa()
        elif layout == "aosoa":
            ps.aosoa_to_soa()
        torch.cuda.synchronize()
        runs.append(ps.download_soa())
        ps.close()
    assert all(np.array_equal(a.view(np.uint8), b.view(np.uint8)) for a, b in zip(*runs))
