"""Pins of the oracle's bulk AoS<->SoA transposes: every field decoded by
numpy's own structured-dtype implementation of the C record, round trips
that are the identity byte for byte, and padding written as zero."""
import numpy as np
import pytest

import synth_inputs as si

NPT = {"i8": "i1", "u8": "u1", "i32": "<i4", "i64": "<i8", "f32": "<f4", "f64": "<f8"}
SCHEMAS = {"base": si.BASE_FIELDS, "wide": si.WIDE_FIELDS,
           "particle5": si.particle_size_fields(5),
           "bytes": [("a", "u8", 1), ("b", "i64", 1), ("c", "i8", 3), ("d", "f32", 2)]}


def np_dtype(fields, packed):
    return np.dtype([(n, NPT[t], (d,)) if d > 1 else (n, NPT[t]) for n, t, d in fields],
                    align=not packed)


@pytest.mark.parametrize("key", sorted(SCHEMAS))
@pytest.mark.parametrize("packed", [False, True])
@pytest.mark.parametrize("n", [0, 1, 255, 1000])
def test_soa_to_aos_matches_struct_view(ref, key, packed, n):
    fields = SCHEMAS[key]
    sch = ref.Schema(fields, packed=packed)
    arrs = si.random_state(fields, n, 7)
    aos = ref.soa_to_aos(sch, arrs)
    rec = aos.view(np_dtype(fields, packed)) if n else None
    a = 0
    for name, _, d in fields:
        for c in range(d):
            if n:
                got = rec[name] if d == 1 else rec[name][:, c]
                assert np.array_equal(got, arrs[a])
            a += 1
    # every byte not covered by a field is padding and must be zero
    offs, stride = sch.layout()
    covered = np.zeros(stride, bool)
    for (name, t, d), off in zip(fields, offs):
        covered[off: off + d * np.dtype(NPT[t]).itemsize] = True
    if n:
        assert not aos.reshape(n, stride)[:, ~covered].any()


@pytest.mark.parametrize("key", sorted(SCHEMAS))
@pytest.mark.parametrize("packed", [False, True])
def test_round_trips_are_identity(ref, key, packed):
    fields = SCHEMAS[key]
    n = 1001
    sch = ref.Schema(fields, packed=packed)
    arrs = si.random_state(fields, n, 8)
    aos = ref.soa_to_aos(sch, arrs)
    back = ref.aos_to_soa(sch, aos, n)
    assert all(np.array_equal(x, y) for x, y in zip(arrs, back))
    aos2 = ref.soa_to_aos(sch, back)
    assert np.array_equal(aos, aos2)


def test_aos_to_soa_ignores_padding(ref):
    sch = ref.Schema(si.BASE_FIELDS)
    n = 64
    arrs = si.random_state(si.BASE_FIELDS, n, 9)
    aos = ref.soa_to_aos(sch, arrs).reshape(n, 48)
    aos[:, 4:8] = 0xEE  # padding after id
    aos[:, 44:48] = 0x77  # tail padding
    back = ref.aos_to_soa(sch, aos.reshape(-1).copy(), n)
    assert all(np.array_equal(x, y) for x, y in zip(arrs, back))


def test_ids_and_count_preserved_through_steps_and_transposes(ref):
    n = 3333
    sch = ref.Schema(si.WIDE_FIELDS)
    arrs = si.random_state(si.WIDE_FIELDS, n, 10)
    aos = ref.soa_to_aos(sch, arrs)
    soa = ref.aos_to_soa(sch, aos, n)
    ref.step_soa(sch, soa, ref.EULER_ACC, 1e-3, 20, wrap=True)
    aos2 = ref.soa_to_aos(sch, soa)
    assert aos2.size == n * 80
    back = ref.aos_to_soa(sch, aos2, n)
    for name in ("tag", "id", "mass", "flags"):
        i = sch.array_index(name)
        assert np.array_equal(back[i], arrs[i])
