"""GPU tests of the fused multi-step SoA kernel (soax_step_fused): every
particle held in registers from the first step to the last.  Each step is the
one-step kernels' arithmetic, so the fused results must equal nsteps
separate steps bit for bit, in every integrator, with and without the wrap,
for cache-resident and streaming sets, double and float records and every
shift tier of the field integrators; one case is also compared with the
oracle directly."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import assert_fields_close, assert_positions_close

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")

INTEGRATORS = ["euler", "euler_acc", "symplectic_euler", "rk2_abc", "heun_abc", "rk4_abc"]
ABC = [1.0, 0.8, 0.6]


def stepped(fields, arrays, integ, dt, nsteps, fused, abc=ABC, wrap=True):
    n = len(arrays[0])
    ps = soax.ParticleSet(fields, n, aos=False)
    ps.upload_soa(arrays)
    if fused:
        ps.step_fused(integ, dt, nsteps, abc=abc, wrap=wrap)
    else:
        ps.step("soa", integ, dt, nsteps, abc=abc, wrap=wrap)
    torch.cuda.synchronize()
    out = ps.download_soa()
    ps.close()
    return out


def assert_same(a, b):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), k


@pytest.mark.parametrize("integ", INTEGRATORS)
@pytest.mark.parametrize("n,nsteps", [(1, 1), (257, 7), (100_003, 13)])
@pytest.mark.parametrize("wrap", [True, False])
def test_fused_equals_separate_steps(integ, n, nsteps, wrap):
    fields = si.WIDE_FIELDS
    arrays = si.random_state(fields, n, seed=61)
    dt = 2e-3
    got = stepped(fields, arrays, integ, dt, nsteps, True, wrap=wrap)
    want = stepped(fields, arrays, integ, dt, nsteps, False, wrap=wrap)
    assert_same(got, want)


@pytest.mark.parametrize("integ", ["euler", "rk2_abc", "rk4_abc"])
def test_fused_equals_separate_steps_streaming(integ):
    # 4e6 + 3 particles: the separate steps run the streaming kernels (two
    # particles per thread for the field integrators, two runs per workgroup
    # for RK4) and their tails
    n = 4_000_003
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, n, seed=67)
    got = stepped(fields, arrays, integ, 1e-3, 5, True)
    want = stepped(fields, arrays, integ, 1e-3, 5, False)
    assert_same(got, want)


@pytest.mark.parametrize("dt", [1e-3, 0.02, 0.2], ids=["small", "mid", "any"])
@pytest.mark.parametrize("integ", ["rk2_abc", "heun_abc", "rk4_abc"])
def test_fused_every_shift_tier(integ, dt):
    # dt (|A|+|B|+|C|) = 2.4 dt: within 1/64, within 1/8, beyond 1/8
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, 4099, seed=71)
    got = stepped(fields, arrays, integ, dt, 9, True)
    want = stepped(fields, arrays, integ, dt, 9, False)
    assert_same(got, want)


@pytest.mark.parametrize("integ", ["euler", "euler_acc", "symplectic_euler"])
def test_fused_float_records(integ):
    # fp32 positions and velocities (the paper's Particle<SIZE> record plus an
    # acceleration), no wrap: each step rounds the positions to float
    fields = [("pos", "f32", 3), ("vel", "f32", 3), ("acc", "f32", 3)]
    arrays = si.random_state(fields, 3001, seed=73)
    got = stepped(fields, arrays, integ, 1e-2, 17, True, abc=None, wrap=False)
    want = stepped(fields, arrays, integ, 1e-2, 17, False, abc=None, wrap=False)
    assert_same(got, want)


def test_fused_rk2_against_oracle(ref):
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, 4099, seed=79)
    got = stepped(fields, arrays, "rk2_abc", 1e-3, 25, True)
    want = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), want, ref.RK2_ABC, 1e-3, 25, abc=ABC, wrap=True)
    assert np.array_equal(got[0], want[0])
    for d in range(3):
        assert_positions_close(got[1 + d], want[1 + d])
        assert_fields_close(got[4 + d], want[4 + d])


def test_fused_zero_steps_and_errors():
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, 100, seed=83)
    ps = soax.ParticleSet(fields, 100, aos=False)
    ps.upload_soa(arrays)
    ps.step_fused("rk2_abc", 1e-3, 0, abc=ABC)
    torch.cuda.synchronize()
    assert_same(ps.download_soa(), arrays)
    with pytest.raises(soax.SoaxError):
        ps.step_fused("rk2_abc", 1e-3, -1, abc=ABC)
    with pytest.raises(soax.SoaxError):
        ps.step_fused("rk2_abc", float("nan"), 3, abc=ABC)
    ps.close()
    aos_only = soax.ParticleSet(fields, 100, soa=False)
    with pytest.raises(soax.SoaxError):
        aos_only.step_fused("euler", 1e-3, 3)
    aos_only.close()
    flt = soax.ParticleSet([("pos", "f32", 3), ("vel", "f32", 3)], 100, aos=False)
    with pytest.raises(soax.SoaxError):  # the ABC field needs f64 positions
        flt.step_fused("rk2_abc", 1e-3, 3, abc=ABC, wrap=False)
    flt.close()
