"""GPU parity of the streaming instantiations of the step and transpose
kernels: the ones the library selects once a step's arrays exceed the
caches (nontemporal loads and stores), which the benchmark times at 1e8 and
3e7 particles.

Sets of 4e6 particles are above the streaming threshold in every layout
(36 B of positions and velocities per particle for the base record, 48 B
with the acceleration, whole 48- and 80-byte records for AoS), yet small
enough for the oracle to step every particle: whole arrays are compared bit
for bit.  At the benchmark's own sizes sampled particles are compared: the
oracle's fill of each sampled range is written into the GPU's arrays before
the run, so both sides start from the same state and Euler results must be
identical to the last bit (eq. (1) of Section 2 is one multiply and one add
on both sides)."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import assert_fields_close, assert_positions_close, from_aos, to_aos

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")

STREAM_BYTES = 128 << 20  # footprint from which the library streams (nontemporal hints)


def sample_ranges(n, width=128, extra=4, seed=0):
    rng = np.random.default_rng(seed)
    starts = [0, max(0, n // 2 - width // 2), max(0, n - width)]
    starts += [int(s) for s in rng.integers(0, max(1, n - width), extra)]
    return [(s, min(width, n - s)) for s in sorted(set(starts))]


def plant(ps, r0, arrays):
    """Write host arrays into particles r0 .. r0 + len - 1 of the SoA copy."""
    for t, a in zip(ps.soa, arrays):
        t[r0:r0 + len(a)].copy_(torch.from_numpy(a))


@pytest.mark.parametrize("layout", ["soa", "aos", "aos_naive"])
def test_euler_streaming_whole_arrays_4e6(ref, layout):
    n = 4_000_003
    fields = si.BASE_FIELDS
    assert n * 36 >= STREAM_BYTES and n * 48 >= STREAM_BYTES
    arrays = si.random_state(fields, n, seed=41)
    ps = soax.ParticleSet(fields, n)
    if layout == "soa":
        ps.upload_soa(arrays)
    else:
        ps.upload_aos(to_aos(fields, arrays))
    ps.step(layout, "euler", 1e-3, 5, wrap=True)
    torch.cuda.synchronize()
    got = ps.download_soa() if layout == "soa" else from_aos(fields, ps.download_aos(), n)
    ps.close()
    want = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), want, ref.EULER, 1e-3, 5, wrap=True)
    for a, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), a


@pytest.mark.parametrize("layout", ["soa", "aos", "aos_naive"])
@pytest.mark.parametrize("integ", ["euler_acc", "symplectic_euler"])
def test_acceleration_steps_streaming_whole_arrays_4e6(ref, layout, integ):
    n = 4_000_037
    fields = si.WIDE_FIELDS
    assert n * 48 >= STREAM_BYTES
    arrays = si.random_state(fields, n, seed=43)
    ps = soax.ParticleSet(fields, n)
    if layout == "soa":
        ps.upload_soa(arrays)
    else:
        ps.upload_aos(to_aos(fields, arrays))
    ps.step(layout, integ, 1e-3, 4, wrap=True)
    torch.cuda.synchronize()
    got = ps.download_soa() if layout == "soa" else from_aos(fields, ps.download_aos(), n)
    raw = None if layout == "soa" else ps.download_aos()
    stride = ps.stride
    ps.close()
    want = [a.copy() for a in arrays]
    code = ref.EULER_ACC if integ == "euler_acc" else ref.SYMPLECTIC_EULER
    ref.step_soa(ref.Schema(fields), want, code, 1e-3, 4, wrap=True)
    for a, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), a
    if raw is not None:  # padding bytes of the records untouched (still 0)
        assert np.array_equal(raw[: n * stride], to_aos(fields, want))


@pytest.mark.parametrize("layout", ["soa", "aos", "aos_naive"])
@pytest.mark.parametrize("integ", ["rk2_abc", "heun_abc", "rk4_abc"])
def test_field_integrators_streaming_whole_arrays_4e6(ref, layout, integ):
    # the streaming kernels of the field integrators (two particles per
    # thread in SoA, so an odd n leaves a one-particle tail), every particle
    # against the oracle; SoA and AoS must also agree bit for bit
    n = 4_000_003
    fields = si.BASE_FIELDS
    assert n * 36 >= STREAM_BYTES
    arrays = si.random_state(fields, n, seed=47)
    abc = [1.0, 0.8, 0.6]
    ps = soax.ParticleSet(fields, n)
    if layout == "soa":
        ps.upload_soa(arrays)
    else:
        ps.upload_aos(to_aos(fields, arrays))
    ps.step(layout, integ, 2e-3, 3, abc=abc, wrap=True)
    torch.cuda.synchronize()
    got = ps.download_soa() if layout == "soa" else from_aos(fields, ps.download_aos(), n)
    ps.close()
    want = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), want, getattr(ref, integ.upper()), 2e-3, 3, abc=abc, wrap=True)
    assert np.array_equal(got[0], want[0])
    for d in range(3):
        assert_positions_close(got[1 + d], want[1 + d])
        assert_fields_close(got[4 + d], want[4 + d])
    if layout == "soa":
        _FIELD_SOA[integ] = got
    elif integ in _FIELD_SOA:
        soa = _FIELD_SOA[integ] if layout == "aos" else _FIELD_SOA.pop(integ)
        for a, (g, w) in enumerate(zip(got, soa)):
            assert np.array_equal(g, w), (layout, a)


_FIELD_SOA = {}


N_PAIRS = 3_840_000  # a multiple of 512: whole pairs of runs for runs of 128 and 256 particles


@pytest.mark.parametrize("block,per_thread", [(64, 2), (128, 2), (64, 1)])
@pytest.mark.parametrize("extra", [0, 5, 128, 200, 256 + 77])
def test_rk4_streaming_pairs_of_runs_match_aos(block, per_thread, extra):
    # the streaming RK4 step takes two runs of block * per_thread particles per
    # workgroup and steps an incomplete last pair one particle per thread:
    # every split of the last pair (none, a partial first run, one whole run,
    # a whole run and a partial one) must give the LDS-staged AoS kernel's
    # results bit for bit
    n = N_PAIRS + extra
    fields = si.BASE_FIELDS
    assert n * 36 >= STREAM_BYTES
    arrays = si.random_state(fields, n, seed=53)
    abc = [1.0, 0.8, 0.6]
    soa = soax.ParticleSet(fields, n, aos=False)
    soa.upload_soa(arrays)
    soa.step_config("soa", block, per_thread)
    soa.step("soa", "rk4_abc", 2e-3, 2, abc=abc, wrap=True)
    aos = soax.ParticleSet(fields, n, soa=False)
    aos.upload_aos(to_aos(fields, arrays))
    aos.step("aos", "rk4_abc", 2e-3, 2, abc=abc, wrap=True)
    torch.cuda.synchronize()
    got = soa.download_soa()
    want = from_aos(fields, aos.download_aos(), n)
    soa.close()
    aos.close()
    for a, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), a
    assert not np.array_equal(got[1], arrays[1])  # the step moved the particles



def test_euler_headline_1e8_every_layout(ref):
    """The benchmark's Euler rows: 20 steps in SoA, 20 in the LDS-staged AoS
    copy and 20 more per-thread (naive) AoS steps beside 20 more SoA steps, on
    the 1e8-particle set filled as the benchmark fills it."""
    n, abc = 100_000_000, [1.0, 1.0, 1.0]
    fields = si.BASE_FIELDS
    sch = ref.Schema(fields)
    ps = soax.ParticleSet(fields, n)
    ps.fill(seed=0, vel_mode=1, abc=abc)
    ranges = sample_ranges(n)
    init = {}
    for r0, cnt in ranges:
        init[r0] = ref.fill_range(sch, r0, cnt, seed=0, vel_mode=1, abc=abc)
        plant(ps, r0, init[r0])
    ps.soa_to_aos()
    rec = ps.aos[: n * ps.stride].view(n, ps.stride)

    def same_everywhere():
        for d in range(3):
            pos_aos = rec[:, 8 + 8 * d: 16 + 8 * d].contiguous().view(torch.float64).view(-1)
            assert torch.equal(pos_aos, ps.soa[1 + d]), d
            del pos_aos
        vel = rec[:, 32:44].contiguous().view(torch.float32).view(n, 3)
        for d in range(3):
            assert torch.equal(vel[:, d], ps.soa[4 + d]), d
        del vel

    ps.step("soa", "euler", 1e-3, 20, wrap=True)
    ps.step("aos", "euler", 1e-3, 20, wrap=True)
    torch.cuda.synchronize()
    same_everywhere()
    ps.step("soa", "euler", 1e-3, 20, wrap=True)
    ps.step("aos_naive", "euler", 1e-3, 20, wrap=True)
    torch.cuda.synchronize()
    same_everywhere()
    for r0, cnt in ranges:
        want = [a.copy() for a in init[r0]]
        ref.step_soa(sch, want, ref.EULER, 1e-3, 40, wrap=True)
        got = [t[r0:r0 + cnt].cpu().numpy() for t in ps.soa]
        for a, (g, w) in enumerate(zip(got, want)):
            assert np.array_equal(g, w), (r0, a)
        rbytes = ps.aos[r0 * ps.stride:(r0 + cnt) * ps.stride].cpu().numpy()
        assert np.array_equal(rbytes, ref.soa_to_aos(sch, want)), r0
    del rec
    ps.close()
    torch.cuda.empty_cache()


def test_wide_transposes_3e7_against_oracle(ref):
    """The benchmark's 3e7 wide-record transposes: sampled records of
    soa_to_aos equal the oracle's records byte for byte (padding 0), and
    aos_to_soa of the oracle's records restores the oracle's arrays."""
    n = 30_000_000
    fields = si.WIDE_FIELDS
    sch = ref.Schema(fields)
    ps = soax.ParticleSet(fields, n)
    assert n * ps.stride >= STREAM_BYTES
    ps.fill(seed=0)
    ranges = sample_ranges(n)
    init = {}
    for r0, cnt in ranges:
        init[r0] = ref.fill_range(sch, r0, cnt, seed=0)
        plant(ps, r0, init[r0])
    ps.aos.fill_(0xA5)  # every byte, padding included, must be rewritten
    ps.soa_to_aos()
    torch.cuda.synchronize()
    for r0, cnt in ranges:
        got = ps.aos[r0 * ps.stride:(r0 + cnt) * ps.stride].cpu().numpy()
        want = ref.soa_to_aos(sch, init[r0])
        assert np.array_equal(got, want), r0
    # records written by the oracle's transpose (another seed's values, which
    # depend only on the particle index, so overlapping ranges agree), read
    # back by the GPU's
    other = {r0: ref.fill_range(sch, r0, cnt, seed=5) for r0, cnt in ranges}
    for r0, cnt in ranges:
        rb = torch.from_numpy(ref.soa_to_aos(sch, other[r0]))
        ps.aos[r0 * ps.stride:(r0 + cnt) * ps.stride].copy_(rb)
    for t in ps.soa:
        t.fill_(0)
    ps.aos_to_soa()
    torch.cuda.synchronize()
    for r0, cnt in ranges:
        want = ref.aos_to_soa(sch, ref.soa_to_aos(sch, other[r0]), cnt)
        got = [t[r0:r0 + cnt].cpu().numpy() for t in ps.soa]
        for a, (g, w) in enumerate(zip(got, want)):
            assert np.array_equal(g, w), (r0, a)
    ps.close()
    torch.cuda.empty_cache()
