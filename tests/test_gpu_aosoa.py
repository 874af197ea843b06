"""GPU parity of the AoSoA (tiled) copy: conversions byte-exact against the
oracle's tiles, every integrator on the tiled copy against the oracle's SoA
steps (the same particles, so the same results), bit-identity with the SoA
kernels, records read back from tiles, and re-attachment after growth."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import assert_fields_close, assert_positions_close, to_aos

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")


def make(fields, n, seed, **kw):
    arrays = si.random_state(fields, n, seed)
    ps = soax.ParticleSet(fields, n, aosoa=True, **kw)
    ps.upload_soa(arrays)
    return ps, arrays


# arrays per element size (8, 4, 1 bytes): base 3/4/0, wide 4/8/1,
# bytes 1/2/4, particle5 0/11/0 -- every remainder of the 4-array blocks
XFIELDS = {"base": si.BASE_FIELDS, "wide": si.WIDE_FIELDS,
           "bytes": [("a", "u8", 1), ("b", "i64", 1), ("c", "i8", 3), ("d", "f32", 2)],
           "particle5": si.particle_size_fields(5)}


@pytest.mark.parametrize("key", sorted(XFIELDS))
@pytest.mark.parametrize("n", [1, 63, 64, 65, 4099])
def test_conversions_match_oracle_tiles(ref, key, n):
    fields = XFIELDS[key]
    ps, arrays = make(fields, n, n)
    ps.soa_to_aosoa()
    torch.cuda.synchronize()
    assert np.array_equal(ps.download_aosoa(), ref.soa_to_aosoa(ref.Schema(fields), arrays))
    for t in ps.soa:
        t.zero_()
    ps.aosoa_to_soa()
    torch.cuda.synchronize()
    for g, w in zip(ps.download_soa(), arrays):
        assert np.array_equal(g.view(np.uint8), w.view(np.uint8))
    ps.close()


EULERS = ["euler", "euler_acc", "symplectic_euler"]
FIELDS_INTEG = ["rk2_abc", "heun_abc", "rk4_abc"]


@pytest.mark.parametrize("integ", EULERS + FIELDS_INTEG)
@pytest.mark.parametrize("n", [5, 4099])
def test_steps_on_tiles_match_oracle(ref, integ, n):
    fields = si.WIDE_FIELDS
    ps, arrays = make(fields, n, 100 + n)
    ps.soa_to_aosoa()
    abc = [1.0, 0.8, 0.6]
    ps.step("aosoa", integ, 1e-3, 6, abc=abc, wrap=True)
    ps.aosoa_to_soa()
    torch.cuda.synchronize()
    got = ps.download_soa()
    want = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), want, getattr(ref, integ.upper()), 1e-3, 6, abc=abc, wrap=True)
    sch = ref.Schema(fields)
    pos = set(range(sch.array_index("pos"), sch.array_index("pos") + 3))
    vel = set(range(sch.array_index("vel"), sch.array_index("vel") + 3))
    for a, (g, w) in enumerate(zip(got, want)):
        if integ in FIELDS_INTEG and a in pos:
            assert_positions_close(g, w)
        elif integ in FIELDS_INTEG and a in vel:
            assert_fields_close(g, w)
        else:
            assert np.array_equal(g.view(np.uint8), w.view(np.uint8)), a
    ps.close()


@pytest.mark.parametrize("integ", EULERS + FIELDS_INTEG)
def test_steps_on_tiles_streaming_size(ref, integ):
    # above 128 MB of stepped arrays the tiled step streams through buffer
    # windows over each wave's tile; a ragged last tile, every particle
    # against the oracle, and the field steps bit-identical to the SoA kernels
    n = 4_000_037
    fields = si.WIDE_FIELDS
    ps, arrays = make(fields, n, 7)
    ps.soa_to_aosoa()
    abc = [1.0, 0.8, 0.6]
    ps.step("aosoa", integ, 1e-3, 3, abc=abc, wrap=True)
    ps.aosoa_to_soa()
    torch.cuda.synchronize()
    got = ps.download_soa()
    sch = ref.Schema(fields)
    want = [a.copy() for a in arrays]
    ref.step_soa(sch, want, getattr(ref, integ.upper()), 1e-3, 3, abc=abc, wrap=True)
    pos = set(range(sch.array_index("pos"), sch.array_index("pos") + 3))
    vel = set(range(sch.array_index("vel"), sch.array_index("vel") + 3))
    for a, (g, w) in enumerate(zip(got, want)):
        if integ in FIELDS_INTEG and a in pos:
            assert_positions_close(g, w)
        elif integ in FIELDS_INTEG and a in vel:
            assert_fields_close(g, w)
        else:
            assert np.array_equal(g.view(np.uint8), w.view(np.uint8)), a
    if integ in FIELDS_INTEG:
        ps.upload_soa(arrays)
        ps.step("soa", integ, 1e-3, 3, abc=abc, wrap=True)
        torch.cuda.synchronize()
        for a, (g, w) in enumerate(zip(got, ps.download_soa())):
            assert np.array_equal(g.view(np.uint8), w.view(np.uint8)), a
    ps.close()


def test_float_record_on_tiles(ref):
    fields = si.particle_size_fields(8)  # the paper's Particle<8>: float x, v, temp
    ps, arrays = make(fields, 1000, 9)
    ps.soa_to_aosoa()
    ps.step("aosoa", "euler", 1e-2, 5, wrap=False)
    ps.aosoa_to_soa()
    torch.cuda.synchronize()
    want = [a.copy() for a in arrays]
    ref.step_soa(ref.Schema(fields), want, ref.EULER, 1e-2, 5, wrap=False)
    assert all(np.array_equal(g, w) for g, w in zip(ps.download_soa(), want))
    ps.close()


def test_tiles_and_soa_kernels_agree_bit_for_bit():
    n = 100_003
    ps = soax.ParticleSet(si.BASE_FIELDS, n, aosoa=True)
    ps.fill(seed=4, vel_mode=1, abc=[1, 1, 1])
    ps.soa_to_aosoa()
    ps.step("aosoa", "rk2_abc", 1e-3, 5, abc=[1, 1, 1], wrap=True)
    ps.step("soa", "rk2_abc", 1e-3, 5, abc=[1, 1, 1], wrap=True)
    stepped = [t.clone() for t in ps.soa]
    ps.aosoa_to_soa()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(ps.soa, stepped))
    ps.close()


def test_records_from_tiles_and_growth(ref):
    fields = si.BASE_FIELDS
    ps, arrays = make(fields, 200, 1)
    ps.soa_to_aosoa()
    for i in (0, 63, 64, 199):
        assert ps.get_record("aosoa", i) == ps.get_record("soa", i) == \
            to_aos(fields, [a[i:i + 1] for a in arrays]).tobytes()
    # growth moves the arrays; the tiled copy is re-attached at the new size
    new = si.random_state(fields, 300, 2)
    ps.push_back(to_aos(fields, new))
    ps.soa_to_aosoa()
    torch.cuda.synchronize()
    cur = [np.concatenate([a, b]) for a, b in zip(arrays, new)]
    assert np.array_equal(ps.download_aosoa(), ref.soa_to_aosoa(ref.Schema(fields), cur))
    ps.close()


def test_conversions_with_unaligned_arrays(ref):
    # SoA arrays 8 bytes (4 for 4-byte elements) past a 16-byte boundary:
    # every tile, not only the last, goes through the per-lane kernel
    import ctypes
    from paper_1710_03462_amd import _lib
    fields = si.BASE_FIELDS
    n = 1000
    arrays = si.random_state(fields, n, seed=12)
    bufs = [torch.empty(n + 4, dtype=t, device="cuda")
            for t in (torch.int32, *(torch.float64,) * 3, *(torch.float32,) * 3)]
    views = []
    for b, a in zip(bufs, arrays):
        v = b[1:1 + n]
        v.copy_(torch.from_numpy(a))
        views.append(v)
    assert all(v.data_ptr() % 16 for v in views)
    L = _lib.lib()
    sch, keep = _lib.make_schema(fields)
    ptrs = (ctypes.c_void_p * 7)(*[v.data_ptr() for v in views])
    h = ctypes.c_void_p()
    _lib.check(L.soax_bind(ctypes.byref(sch), n, ptrs, None, ctypes.byref(h)), "bind")
    tile = ctypes.c_int64()
    _lib.check(L.soax_aosoa_layout(ctypes.byref(sch), None, ctypes.byref(tile)), "layout")
    nbytes = (n + 63) // 64 * tile.value
    buf = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    _lib.check(L.soax_bind_aosoa(h, ctypes.c_void_p(buf.data_ptr()), nbytes), "bind_aosoa")
    _lib.check(L.soax_soa_to_aosoa(h, soax.current_stream()), "soa_to_aosoa")
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), ref.soa_to_aosoa(ref.Schema(fields), arrays))
    for v in views:
        v.zero_()
    _lib.check(L.soax_aosoa_to_soa(h, soax.current_stream()), "aosoa_to_soa")
    torch.cuda.synchronize()
    L.soax_destroy(h)
    for g, w in zip(views, arrays):
        assert np.array_equal(g.cpu().numpy().view(np.uint8), w.view(np.uint8))
