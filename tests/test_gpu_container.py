"""GPU parity of the container operations (removal of Section 2; resize,
element access and push_back of Section 4.1) against the oracle.

Removal by overwriting with the last particle is a permutation of whole
records, so it is compared bit for bit with the oracle's sequential removal,
in both copies.  Resize keeps the prefix and zero-fills the tail; push_back
appends records to both copies; a batch that holds a resized set refuses to
step."""
import ctypes

import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import from_aos, to_aos

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")
from paper_1710_03462_amd import _lib  # noqa: E402

SCHEMAS = {"base": (si.BASE_FIELDS, False), "base_packed": (si.BASE_FIELDS, True),
           "wide": (si.WIDE_FIELDS, False), "wide_packed": (si.WIDE_FIELDS, True)}


def make_set(fields, packed, n, seed, capacity=None):
    arrays = si.random_state(fields, n, seed)
    ps = soax.ParticleSet(fields, n, packed=packed, capacity=capacity)
    if n:
        ps.upload_soa(arrays)
        ps.soa_to_aos()
    return ps, arrays


def flags_for(n, density, seed, clustered=False):
    rng = np.random.default_rng(seed)
    if clustered:  # runs of removals spanning whole tiles, plus scattered ones
        f = np.zeros(n, np.uint8)
        for s in rng.integers(0, max(n, 1), 12):
            f[s: s + int(rng.integers(1, 20000))] = 1
        f |= (rng.random(n) < density).astype(np.uint8)
        return f
    return (rng.random(n) < density).astype(np.uint8)


def check_against_oracle(ref, ps, fields, packed, arrays, flags):
    sch = ref.Schema(fields, packed)
    want, m = ref.remove_flagged(sch, arrays, flags)
    got_n = ps.remove_flagged(torch.from_numpy(flags).cuda())
    torch.cuda.synchronize()
    assert got_n == m == ps.n
    got = ps.download_soa()
    for a, (g, w) in enumerate(zip(got, want)):
        assert g.dtype == w.dtype and np.array_equal(g.view(np.uint8), w.view(np.uint8)), a
    assert np.array_equal(ps.download_aos(), to_aos(fields, want, packed))
    return want


@pytest.mark.parametrize("name", list(SCHEMAS))
@pytest.mark.parametrize("n", [1, 4096, 4097, 70_001])
@pytest.mark.parametrize("density", [0.0, 0.003, 0.5, 0.97, 1.0])
def test_remove_flagged_matches_oracle(ref, name, n, density):
    fields, packed = SCHEMAS[name]
    seed = n + int(density * 1000)
    ps, arrays = make_set(fields, packed, n, seed)
    check_against_oracle(ref, ps, fields, packed, arrays, flags_for(n, density, seed))
    ps.close()


@pytest.mark.parametrize("name", ["base", "wide_packed"])
def test_remove_flagged_many_tiles_and_repeated(ref, name):
    fields, packed = SCHEMAS[name]
    n = 3_000_017
    ps, arrays = make_set(fields, packed, n, 7)
    flags = flags_for(n, 0.1, 7, clustered=True)
    state = check_against_oracle(ref, ps, fields, packed, arrays, flags)
    # a second removal on the shrunk set
    flags2 = flags_for(ps.n, 0.02, 8, clustered=True)
    check_against_oracle(ref, ps, fields, packed, state, flags2)
    ps.close()


def test_remove_from_empty_set():
    ps = soax.ParticleSet(si.BASE_FIELDS, 0)
    assert ps.remove_flagged(torch.zeros(1, dtype=torch.uint8, device="cuda")) == 0
    ps.close()


def test_resize_keeps_prefix_and_zero_fills(ref):
    fields, packed = si.WIDE_FIELDS, False
    ps, arrays = make_set(fields, packed, 1000, 3)
    aos0 = ps.download_aos()
    ps.resize(5000)  # beyond the capacity: new buffers, particles copied over
    assert ps.n == 5000 and ps.capacity >= 5000
    got = ps.download_soa()
    for g, a in zip(got, arrays):
        assert np.array_equal(g[:1000], a) and not g[1000:].any()
    aos = ps.download_aos()
    assert np.array_equal(aos[: len(aos0)], aos0) and not aos[len(aos0):].any()
    ps.resize(10)
    assert [len(g) for g in ps.download_soa()] == [10] * len(arrays)
    ps.fill(seed=5)  # write the whole (shrunk) set, then regrow within capacity
    ps.resize(20)
    got = ps.download_soa()
    assert all(not g[10:].any() for g in got)
    want = ref.fill_range(ref.Schema(fields), 0, 10, seed=5)
    normals = set(range(ref.Schema(fields).array_index("vel"), ref.Schema(fields).array_index("acc") + 3))
    for a, (g, w) in enumerate(zip(got, want)):
        if a not in normals:
            assert np.array_equal(g[:10], w), a
    ps.close()


@pytest.mark.parametrize("name", list(SCHEMAS))
def test_push_back_appends_to_both_copies(name):
    fields, packed = SCHEMAS[name]
    ps, arrays = make_set(fields, packed, 37, 11)
    cur = [a.copy() for a in arrays]
    for k, count in enumerate([1, 0, 63, 500, 4099]):  # crosses several regrowths
        new = si.random_state(fields, count, 100 + k) if count else [a[:0] for a in arrays]
        recs = to_aos(fields, new, packed) if count else np.zeros(0, np.uint8)
        ps.push_back(recs)
        cur = [np.concatenate([c, x]) for c, x in zip(cur, new)]
        assert ps.n == len(cur[0])
        got = ps.download_soa()
        for g, w in zip(got, cur):
            assert np.array_equal(g.view(np.uint8), w.view(np.uint8))
        assert np.array_equal(ps.download_aos(), to_aos(fields, cur, packed))
    ps.close()


def test_push_back_keeps_record_bytes_verbatim():
    # padding bytes given by the caller are kept in the AoS copy
    fields = si.BASE_FIELDS
    ps, arrays = make_set(fields, False, 5, 2)
    rec = bytearray(np.random.default_rng(0).integers(0, 256, 48, dtype=np.uint8).tobytes())
    ps.push_back(bytes(rec))
    assert ps.get_record("aos", 5) == bytes(rec)
    want = from_aos(fields, np.frombuffer(bytes(rec), np.uint8), 1)
    for a, w in enumerate(want):
        assert np.array_equal(ps.soa[a][5:6].cpu().numpy().view(np.uint8), w.view(np.uint8))
    # read back from the SoA copy, the record has the same fields and zero padding
    assert ps.get_record("soa", 5) == to_aos(fields, want).tobytes()
    ps.close()


def test_set_record_writes_every_copy():
    fields = si.WIDE_FIELDS
    ps, arrays = make_set(fields, False, 300, 4)
    new = si.random_state(fields, 1, 99)
    rec = to_aos(fields, new).tobytes()
    ps.set_record(123, rec)
    assert ps.get_record("aos", 123) == rec
    assert ps.get_record("soa", 123) == rec
    assert ps.get_record("aos", 122) == to_aos(fields, [a[122:123] for a in arrays]).tobytes()
    ps.close()


def _owned(fields, n):
    sch, keep = _lib.make_schema(fields)
    h = ctypes.c_void_p()
    _lib.check(_lib.lib().soax_create(ctypes.byref(sch), n, ctypes.byref(h)), "soax_create")
    return h, (sch, keep)


def _owned_soa(h, fields, n):
    """The owned set's SoA arrays, copied out with the library's copy kernel."""
    L = _lib.lib()
    out = []
    a = 0
    for _, t, d in fields:
        for _ in range(d):
            p = ctypes.c_void_p()
            _lib.check(L.soax_buffer(h, a, ctypes.byref(p)), "soax_buffer")
            dst = torch.empty(max(n, 1), dtype=soax.particles.TORCH_DTYPE[t], device="cuda")
            if n:
                _lib.check(L.soax_copy(ctypes.c_void_p(dst.data_ptr()), p,
                                       n * dst.element_size(), None), "soax_copy")
            torch.cuda.synchronize()
            out.append(dst[:n].cpu().numpy())
            a += 1
    return out


def test_owned_set_grows_and_compacts(ref):
    """The library-owned path: soax_create, growth by push_back and resize
    (buffers reallocated and copied by the library), then removal."""
    fields = si.BASE_FIELDS
    L = _lib.lib()
    h, keep = _owned(fields, 0)
    n, cap = ctypes.c_int64(), ctypes.c_int64()
    state = [a[:0] for a in si.random_state(fields, 1, 0)]
    for k, count in enumerate([3, 200, 1000]):
        new = si.random_state(fields, count, 50 + k)
        recs = to_aos(fields, new)
        _lib.check(L.soax_push_back(h, recs.ctypes.data_as(ctypes.c_void_p), count, None),
                   "soax_push_back")
        state = [np.concatenate([s, x]) for s, x in zip(state, new)]
    _lib.check(L.soax_capacity(h, ctypes.byref(n), ctypes.byref(cap)), "soax_capacity")
    assert n.value == 1203 and cap.value >= 1203
    got = _owned_soa(h, fields, 1203)
    assert all(np.array_equal(g, w) for g, w in zip(got, state))
    _lib.check(L.soax_resize(h, 5000, None), "soax_resize")
    got = _owned_soa(h, fields, 5000)
    assert all(np.array_equal(g[:1203], w) and not g[1203:].any() for g, w in zip(got, state))
    state = [np.concatenate([w, np.zeros(5000 - 1203, w.dtype)]) for w in state]
    flags = flags_for(5000, 0.3, 5)
    want, m = ref.remove_flagged(ref.Schema(fields), state, flags)
    fl = torch.from_numpy(flags).cuda()
    new_n = ctypes.c_int64()
    _lib.check(L.soax_remove_flagged(h, ctypes.c_void_p(fl.data_ptr()), ctypes.byref(new_n), None),
               "soax_remove_flagged")
    assert new_n.value == m
    got = _owned_soa(h, fields, m)
    assert all(np.array_equal(g, w) for g, w in zip(got, want))
    # the AoS copy followed: record 17 from either copy is the same
    r_aos = (ctypes.c_uint8 * 48)()
    r_soa = (ctypes.c_uint8 * 48)()
    _lib.check(L.soax_get_record(h, 1, 17, r_aos), "get_record")
    _lib.check(L.soax_get_record(h, 0, 17, r_soa), "get_record")
    assert bytes(r_aos) == bytes(r_soa) == to_aos(fields, [w[17:18] for w in want]).tobytes()
    L.soax_destroy(h)


def test_batch_refuses_a_resized_set():
    sets = [soax.ParticleSet(si.BASE_FIELDS, 1000, aos=False) for _ in range(2)]
    for s, ps in enumerate(sets):
        ps.fill(seed=s, vel_mode=1, abc=[1.0, 1.0, 1.0])
    b = soax.Batch(sets)
    dts, abc = [1e-3, 1e-3], [[1.0, 1.0, 1.0]] * 2
    b.step(dts, abc, 1, mode=soax.PERSISTENT)
    sets[1].resize(500)
    with pytest.raises(_lib.SoaxError) as e:
        b.step(dts, abc, 1, mode=soax.PERSISTENT)
    assert e.value.status == -7
    b.close()


def test_element_access_like_get_element():
    fields = si.WIDE_FIELDS
    ps, arrays = make_set(fields, False, 50, 8)
    e = ps.element(7)
    assert int(e["id"]) == int(arrays[ps.schema.array_index("id")][7])
    assert float(e["pos"][1]) == float(arrays[ps.schema.array_index("pos", 1)][7])
    ps.set_element(7, id=42, pos=[3.14, 1.0, 2.0])
    e2 = ps.element(7, "aos")
    assert int(e2["id"]) == 42 and list(e2["pos"]) == [3.14, 1.0, 2.0]
    assert float(e2["mass"]) == float(arrays[ps.schema.array_index("mass")][7])
    assert ps.get_record("soa", 7) == ps.get_record("aos", 7)
    # push_back of a modified element, as in the paper's usage example
    e2["id"] = 50
    ps.push_back(e2.tobytes())
    assert ps.n == 51 and int(ps.element(50)["id"]) == 50
    ps.close()


@pytest.mark.parametrize("offset", [0, 1, 8])
def test_remove_flag_bytes_and_alignment(ref, offset):
    # any nonzero byte flags a particle; flags that do not start on a 16-byte
    # boundary, and a flags tensor longer than n, give the same result
    fields, packed = SCHEMAS["base"]
    n = 40_003
    ps, arrays = make_set(fields, packed, n, 21)
    rng = np.random.default_rng(21)
    vals = np.array([1, 2, 0x40, 0x7F, 0x80, 0xFF], np.uint8)
    flags = np.where(rng.random(n) < 0.05, rng.choice(vals, n), 0).astype(np.uint8)
    buf = torch.zeros(n + offset + 37, dtype=torch.uint8, device="cuda")
    buf[offset: offset + n] = torch.from_numpy(flags).cuda()
    buf[offset + n:] = 1  # past n: never read as flags
    want, m = ref.remove_flagged(ref.Schema(fields, packed), arrays, (flags != 0).astype(np.uint8))
    assert ps.remove_flagged(buf[offset:]) == m
    torch.cuda.synchronize()
    for g, w in zip(ps.download_soa(), want):
        assert np.array_equal(g.view(np.uint8), w.view(np.uint8))
    assert np.array_equal(ps.download_aos(), to_aos(fields, want, packed))
    ps.close()
