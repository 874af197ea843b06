"""GPU parity of the fill, the time steps in every layout and the transposes
against the CPU oracle, element by element, on the same seeded inputs.

Sizes span one partial tile, several full tiles plus a ragged tail, and the
1e5-particle Euler workload at its full size.  Integer, byte and Euler
results must be bit-exact; RK2 positions within 1e-12 of the box edge
(periodic distance) and fp32 velocities within 1e-6 relative (floor 1)."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import (L, assert_fields_close, assert_positions_close, from_aos, to_aos,
                      ulp_distance)

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")

SIZES = [1, 5, 257, 4099]
LAYOUTS = ["soa", "aos", "aos_naive"]


def _sync():
    torch.cuda.synchronize()


def run_gpu(fields, arrays, layout, integ, dt, nsteps, abc=None, wrap=True, packed=False,
            block=0, per_thread=0):
    n = len(arrays[0])
    ps = soax.ParticleSet(fields, n, packed=packed)
    if layout == "soa":
        ps.upload_soa(arrays)
    else:
        ps.upload_aos(to_aos(fields, arrays, packed))
    if block or per_thread:
        ps.step_config(layout, block, per_thread)
    ps.step(layout, integ, dt, nsteps, abc=abc, wrap=wrap)
    _sync()
    out = ps.download_soa() if layout == "soa" else from_aos(fields, ps.download_aos(), n, packed)
    ps.close()
    return out


def run_ref(ref, fields, arrays, integ, dt, nsteps, abc=None, wrap=True):
    out = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), out, integ, dt, nsteps, abc=abc, wrap=wrap)
    return out


# ------------------------------------------------------------------ fill

@pytest.mark.parametrize("fields", [si.BASE_FIELDS, si.WIDE_FIELDS], ids=["base", "wide"])
@pytest.mark.parametrize("n", [1, 300, 100_003])
def test_fill_matches_oracle(ref, fields, n):
    ps = soax.ParticleSet(fields, n)
    ps.fill(seed=7)
    got = ps.download_soa()
    want = ref.fill(ref.Schema(fields), n, seed=7)
    for (name, c, _), g, w in zip(ps.schema.arrays(), got, want):
        if name in ("vel", "acc"):  # Box-Muller: libm and device log/cos may differ by an ulp
            assert ulp_distance(g, w).max() <= 1, (name, c)
        else:
            assert np.array_equal(g, w), (name, c)


def test_fill_velocity_from_field(ref):
    n, abc = 20_001, [1.0, 1.0, 1.0]
    ps = soax.ParticleSet(si.BASE_FIELDS, n)
    ps.fill(seed=0, vel_mode=1, abc=abc)
    got = ps.download_soa()
    want = ref.fill(ref.Schema(si.BASE_FIELDS), n, seed=0, vel_mode=1, abc=abc)
    for a in range(4):
        assert np.array_equal(got[a], want[a])
    for a in range(4, 7):
        assert ulp_distance(got[a], want[a]).max() <= 1


# ----------------------------------------------------------------- Euler

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", SIZES + [100_000])
def test_euler_bit_exact(ref, layout, n):
    arrays = si.random_state(si.BASE_FIELDS, n, seed=n)
    got = run_gpu(si.BASE_FIELDS, arrays, layout, "euler", 1e-3, 100)
    want = run_ref(ref, si.BASE_FIELDS, arrays, ref.EULER, 1e-3, 100)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_euler_packed_and_edges(ref, layout):
    n = 3001
    arrays = si.random_state(si.BASE_FIELDS, n, seed=11)
    x = si.edge_positions(n, 11)
    for d in range(3):
        arrays[1 + d][:] = x[d]
        arrays[4 + d] *= np.float32(40.0)
    got = run_gpu(si.BASE_FIELDS, arrays, layout, "euler", 1e-3, 7, packed=True)
    want = run_ref(ref, si.BASE_FIELDS, arrays, ref.EULER, 1e-3, 7)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    for d in range(3):
        assert got[1 + d].min() >= 0.0 and got[1 + d].max() < L


@pytest.mark.parametrize("layout", LAYOUTS)
def test_euler_float_record_of_the_paper(ref, layout):
    fields = si.particle_size_fields(8)
    arrays = si.random_state(fields, 2053, seed=5)
    got = run_gpu(fields, arrays, layout, "euler", 1e-3, 10, wrap=False)
    want = run_ref(ref, fields, arrays, ref.EULER, 1e-3, 10, wrap=False)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("packed", [False, True])
def test_euler_acc_bit_exact(ref, layout, packed):
    fields = si.WIDE_FIELDS
    arrays = si.random_state(fields, 1111, seed=3)
    got = run_gpu(fields, arrays, layout, "euler_acc", 1e-3, 20, packed=packed)
    want = run_ref(ref, fields, arrays, ref.EULER_ACC, 1e-3, 20)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


# ------------------------------------------------------------------- RK2

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", SIZES + [20_000])
def test_rk2_matches_oracle(ref, layout, n):
    arrays = si.random_state(si.BASE_FIELDS, n, seed=100 + n)
    abc = [1.0, 1.0, 1.0]
    got = run_gpu(si.BASE_FIELDS, arrays, layout, "rk2_abc", 1e-3, 50, abc=abc)
    want = run_ref(ref, si.BASE_FIELDS, arrays, ref.RK2_ABC, 1e-3, 50, abc=abc)
    assert np.array_equal(got[0], want[0])
    for d in range(3):
        assert_positions_close(got[1 + d], want[1 + d])
        assert got[1 + d].min() >= 0.0 and got[1 + d].max() < L
        assert_fields_close(got[4 + d], want[4 + d])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rk2_edges_packed_and_f64_velocity(ref, layout):
    fields = [("id", "i32", 1), ("pos", "f64", 3), ("vel", "f64", 3)]
    n = 2049
    arrays = si.random_state(fields, n, seed=9)
    x = si.edge_positions(n, 9)
    for d in range(3):
        arrays[1 + d][:] = x[d]
    abc = [1.3, 0.7, 0.9]
    got = run_gpu(fields, arrays, layout, "rk2_abc", 1e-2, 9, abc=abc, packed=True)
    want = run_ref(ref, fields, arrays, ref.RK2_ABC, 1e-2, 9, abc=abc)
    for d in range(3):
        assert_positions_close(got[1 + d], want[1 + d])
        assert_fields_close(got[4 + d], want[4 + d], rel=1e-12)


def test_rk2_zero_field_is_identity():
    arrays = si.random_state(si.BASE_FIELDS, 999, seed=1)
    got = run_gpu(si.BASE_FIELDS, arrays, "soa", "rk2_abc", 1e-3, 5, abc=[0, 0, 0])
    for d in range(3):
        assert np.array_equal(got[1 + d], arrays[1 + d])
        assert not got[4 + d].any()


# -------------------------------------------------------- launch shapes

@pytest.mark.parametrize("integ", ["euler", "rk2_abc"])
def test_soa_results_do_not_depend_on_launch_shape(integ):
    n = 10_007
    arrays = si.random_state(si.BASE_FIELDS, n, seed=2)
    base = run_gpu(si.BASE_FIELDS, arrays, "soa", integ, 1e-3, 3, abc=[1, 1, 1])
    for block in (64, 128, 1024):
        for vec in (1, 2, 4):
            got = run_gpu(si.BASE_FIELDS, arrays, "soa", integ, 1e-3, 3, abc=[1, 1, 1],
                          block=block, per_thread=vec)
            assert all(np.array_equal(g, b) for g, b in zip(got, base)), (block, vec)


def test_float_record_results_do_not_depend_on_launch_shape():
    # 4-byte positions and velocities: four particles per thread is a single
    # 16-byte access per array (8-byte arrays are capped at two per thread)
    fields = si.particle_size_fields(3)
    n = 10_009
    arrays = si.random_state(fields, n, seed=5)
    base = run_gpu(fields, arrays, "soa", "euler", 1e-3, 3, wrap=False)
    for block in (64, 256):
        for vec in (1, 2, 4):
            got = run_gpu(fields, arrays, "soa", "euler", 1e-3, 3, wrap=False, block=block,
                          per_thread=vec)
            assert all(np.array_equal(g, b) for g, b in zip(got, base)), (block, vec)


@pytest.mark.parametrize("layout", ["aos", "aos_naive"])
def test_aos_results_do_not_depend_on_block(layout):
    n = 5003
    arrays = si.random_state(si.WIDE_FIELDS, n, seed=4)
    base = run_gpu(si.WIDE_FIELDS, arrays, layout, "euler_acc", 1e-3, 3)
    for block in (64, 512, 1024):
        got = run_gpu(si.WIDE_FIELDS, arrays, layout, "euler_acc", 1e-3, 3, block=block)
        assert all(np.array_equal(g, b) for g, b in zip(got, base)), block


def test_unaligned_soa_arrays_use_scalar_path(ref):
    # arrays that start 8 bytes past a 16-byte boundary
    import ctypes
    from paper_1710_03462_amd import _lib
    n = 1001
    arrays = si.random_state(si.BASE_FIELDS, n, seed=6)
    bufs = [torch.empty(n + 4, dtype=t, device="cuda")
            for t in (torch.int32, *(torch.float64,) * 3, *(torch.float32,) * 3)]
    views = []
    for b, a in zip(bufs, arrays):
        v = b[2:2 + n] if b.dtype == torch.float64 else b[1:1 + n]
        v.copy_(torch.from_numpy(a))
        views.append(v)
    sch, keep = _lib.make_schema(si.BASE_FIELDS)
    ptrs = (ctypes.c_void_p * 7)(*[v.data_ptr() for v in views])
    h = ctypes.c_void_p()
    _lib.check(_lib.lib().soax_bind(ctypes.byref(sch), n, ptrs, None, ctypes.byref(h)), "bind")
    p = _lib.Params(1.0, 1.0, 1.0, 1)
    _lib.check(_lib.lib().soax_step(h, 0, 2, 1e-3, 4, ctypes.byref(p), soax.current_stream()),
               "step")
    _sync()
    _lib.lib().soax_destroy(h)
    want = run_ref(ref, si.BASE_FIELDS, arrays, ref.RK2_ABC, 1e-3, 4, abc=[1, 1, 1])
    for d in range(3):
        assert_positions_close(views[1 + d].cpu().numpy(), want[1 + d])


# ------------------------------------------------------------ transposes

XSCHEMAS = {"base": si.BASE_FIELDS, "wide": si.WIDE_FIELDS,
            "particle5": si.particle_size_fields(5),
            "bytes": [("a", "u8", 1), ("b", "i64", 1), ("c", "i8", 3), ("d", "f32", 2)]}


@pytest.mark.parametrize("key", sorted(XSCHEMAS))
@pytest.mark.parametrize("packed", [False, True])
@pytest.mark.parametrize("n", [1, 15, 16, 255, 257, 4099])
def test_transposes_bit_exact(key, packed, n):
    fields = XSCHEMAS[key]
    arrays = si.random_state(fields, n, seed=n + 1)
    aos = to_aos(fields, arrays, packed)
    ps = soax.ParticleSet(fields, n, packed=packed)
    ps.upload_aos(aos)
    for t in ps.soa:
        t.fill_(0x5A)
    ps.aos_to_soa()
    _sync()
    assert all(np.array_equal(g, w) for g, w in zip(ps.download_soa(), arrays))
    ps.aos.fill_(0xA5)  # every byte, padding included, must be rewritten
    ps.soa_to_aos()
    _sync()
    assert np.array_equal(ps.download_aos(), aos)


def test_wide_pipeline_round_trip(ref):
    # AoS -> SoA, 20 Euler-with-acceleration steps, SoA -> AoS
    fields, n = si.WIDE_FIELDS, 30_011
    arrays = si.random_state(fields, n, seed=21)
    aos = to_aos(fields, arrays)
    ps = soax.ParticleSet(fields, n)
    ps.upload_aos(aos)
    ps.aos_to_soa()
    ps.step("soa", "euler_acc", 1e-3, 20)
    ps.soa_to_aos()
    _sync()
    sch = ref.Schema(fields)
    ref_soa = ref.aos_to_soa(sch, aos, n)
    ref.step_soa(sch, ref_soa, ref.EULER_ACC, 1e-3, 20, wrap=True)
    assert np.array_equal(ps.download_aos(), ref.soa_to_aos(sch, ref_soa))
    # and with no steps the round trip is the identity
    ps.upload_aos(aos)
    ps.aos_to_soa()
    ps.soa_to_aos()
    _sync()
    assert np.array_equal(ps.download_aos(), aos)


def test_get_record(ref):
    fields, n = si.WIDE_FIELDS, 100
    arrays = si.random_state(fields, n, seed=1)
    ps = soax.ParticleSet(fields, n)
    ps.upload_soa(arrays)
    ps.soa_to_aos()
    _sync()
    aos = to_aos(fields, arrays)
    stride = len(aos) // n
    for i in (0, 37, 99):
        want = aos[i * stride:(i + 1) * stride].tobytes()
        assert ps.get_record("soa", i) == want
        assert ps.get_record("aos", i) == want


def test_empty_set_is_a_no_op():
    ps = soax.ParticleSet(si.BASE_FIELDS, 0)
    ps.fill(seed=1)
    ps.step("soa", "rk2_abc", 1e-3, 3, abc=[1, 1, 1])
    ps.step("aos", "euler", 1e-3, 3)
    ps.soa_to_aos()
    ps.aos_to_soa()
    _sync()
    ps.close()


def test_copy_kernel():
    src = torch.arange(1 << 20, dtype=torch.int64, device="cuda")
    dst = torch.zeros_like(src)
    soax.copy(dst, src)
    _sync()
    assert torch.equal(dst, src)
    src8 = (torch.arange(1000, device="cuda") % 251 + 1).to(torch.uint8)  # ragged tail
    dst8 = torch.zeros(1008, dtype=torch.uint8, device="cuda")
    soax.copy(dst8, src8)
    _sync()
    assert torch.equal(dst8[:1000], src8) and not dst8[1000:].any()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("dt", [0.05, 0.1, 0.3])
def test_rk2_large_steps_use_checked_shifts(ref, layout, dt):
    # dt * (|A|+|B|+|C|) > 1/8: the kernels check every shift and some exceed
    # the angle-addition range, falling back to a full reduction
    n = 3001
    arrays = si.random_state(si.BASE_FIELDS, n, seed=77)
    abc = [1.0, 1.0, 1.0]
    got = run_gpu(si.BASE_FIELDS, arrays, layout, "rk2_abc", dt, 12, abc=abc)
    want = run_ref(ref, si.BASE_FIELDS, arrays, ref.RK2_ABC, dt, 12, abc=abc)
    for d in range(3):
        assert_positions_close(got[1 + d], want[1 + d])
        assert_fields_close(got[4 + d], want[4 + d])


# ------------------------------------------------------ integrator variants

@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("integ", ["heun_abc", "rk4_abc"])
@pytest.mark.parametrize("n", [5, 4099])
def test_field_integrators_match_oracle(ref, layout, integ, n):
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, n, 40 + n)
    abc = [1.0, 0.8, 0.6]
    got = run_gpu(fields, arrays, layout, integ, 2e-3, 7, abc=abc)
    want = run_ref(ref, fields, arrays, getattr(ref, integ.upper()), 2e-3, 7, abc=abc)
    assert np.array_equal(got[0], want[0])
    for d in range(3):
        assert_positions_close(got[1 + d], want[1 + d])
        assert_fields_close(got[4 + d], want[4 + d])


@pytest.mark.parametrize("integ", ["heun_abc", "rk4_abc"])
def test_field_integrators_large_steps_and_f64_velocity(ref, integ):
    # dt (|A|+|B|+|C|) above the unchecked shift bound: per-lane checked shifts
    fields = [("id", "i32", 1), ("pos", "f64", 3), ("vel", "f64", 3)]
    arrays = si.random_state(fields, 1000, 3)
    abc = [1.0, 1.0, 1.0]
    for layout in LAYOUTS:
        got = run_gpu(fields, arrays, layout, integ, 0.05, 3, abc=abc)
        want = run_ref(ref, fields, arrays, getattr(ref, integ.upper()), 0.05, 3, abc=abc)
        for d in range(3):
            assert_positions_close(got[1 + d], want[1 + d])
            assert np.abs(got[4 + d] - want[4 + d]).max() <= 1e-12


@pytest.mark.parametrize("integ", ["rk2_abc", "heun_abc", "rk4_abc"])
@pytest.mark.parametrize("scale", [0.02 * 3, 0.125 * (1 - 2.0 ** -19), 0.125 * (1 + 2.0 ** -19)])
def test_field_integrators_around_the_mid_tier_bound(ref, integ, scale):
    # dt (|A|+|B|+|C|) = scale: 0.06 and just inside 1/8 take the mid tier
    # (short or long angle-addition series per lane, no range check beyond
    # 1/8); just above 1/8 the unbounded tier.  Every layout runs the same
    # tier, so SoA and AoS also agree bit for bit.
    fields = si.BASE_FIELDS
    arrays = si.random_state(fields, 2053, 91)
    abc = [1.0, 1.0, 1.0]
    dt = scale / 3.0
    want = run_ref(ref, fields, arrays, getattr(ref, integ.upper()), dt, 4, abc=abc)
    got = {}
    for layout in LAYOUTS:
        got[layout] = run_gpu(fields, arrays, layout, integ, dt, 4, abc=abc)
        for d in range(3):
            assert_positions_close(got[layout][1 + d], want[1 + d])
            assert_fields_close(got[layout][4 + d], want[4 + d])
    for layout in LAYOUTS:
        for a, b in zip(got[layout], got["soa"]):
            assert np.array_equal(a, b), layout


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("packed", [False, True])
def test_symplectic_euler_bit_exact(ref, layout, packed):
    fields = si.WIDE_FIELDS
    arrays = si.random_state(fields, 4099, 77)
    got = run_gpu(fields, arrays, layout, "symplectic_euler", 1e-3, 9, packed=packed)
    want = run_ref(ref, fields, arrays, ref.SYMPLECTIC_EULER, 1e-3, 9)
    for a, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), a


def test_symplectic_euler_float_record(ref):
    fields = [("pos", "f32", 3), ("vel", "f32", 3), ("acc", "f32", 3)]
    arrays = si.random_state(fields, 257, 5)
    for layout in LAYOUTS:
        got = run_gpu(fields, arrays, layout, "symplectic_euler", 1e-2, 4, wrap=False)
        want = run_ref(ref, fields, arrays, ref.SYMPLECTIC_EULER, 1e-2, 4, wrap=False)
        assert all(np.array_equal(g, w) for g, w in zip(got, want))
