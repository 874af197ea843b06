"""Pins of the oracle's seeded fill: the generator against the published
SplitMix64 sequence, the field rules against their definitions, and the
distributions against their moments."""
import math
import os

import numpy as np

from synth_inputs import BASE_FIELDS, BOX_L, WIDE_FIELDS

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _golden_sequence():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
    return [int(ln, 16) for ln in open(path) if ln.strip() and not ln.startswith("#")]


def test_splitmix64_published_sequence(ref):
    seq = _golden_sequence()
    assert len(seq) == 5
    # the generator advances its state by the golden gamma and outputs mix64(state)
    for k, want in enumerate(seq):
        assert ref.mix64((GAMMA * (k + 1)) & M64) == want


def test_draw_is_a_splitmix_stream_keyed_by_a_splitmix_output(ref):
    seq = _golden_sequence()
    for s in range(4):  # stream s is keyed by the s-th output of SplitMix64(seed 0)
        key = seq[s]
        for i in (0, 1, 7, 12345):
            assert ref.draw(0, s, i) == ref.mix64((key + GAMMA * (i + 1)) & M64)


def test_fill_rules(ref):
    n = 4096
    sch = ref.Schema(WIDE_FIELDS)
    arrs = sch_fill = ref.fill(sch, n, seed=0)
    idx = {name: sch.array_index(name) for name, _, _ in WIDE_FIELDS}
    assert np.array_equal(arrs[idx["id"]], np.arange(n, dtype=np.int32))
    i = np.arange(n)
    for f, (name, _, dim) in enumerate(WIDE_FIELDS):
        for c in range(dim):
            a = sch_fill[idx[name] + c]
            stream = 8 * f + 2 * c
            r = [ref.draw(0, stream, int(k)) for k in (0, 1, 2, n - 1)]
            sel = [0, 1, 2, n - 1]
            if name == "tag":
                assert [int(x) & M64 for x in a[sel]] == r
            if name == "pos":
                want = [BOX_L * ((x >> 11) * 2.0 ** -53) for x in r]
                assert list(a[sel]) == want
                assert a.min() >= 0.0 and a.max() < BOX_L
            if name == "mass":
                want = [0.5 + 1.5 * ((x >> 11) * 2.0 ** -53) for x in r]
                assert list(a[sel]) == want
                assert a.min() >= 0.5 and a.max() < 2.0
            if name == "flags":
                assert [int(x) for x in a[sel]] == [x >> 56 for x in r]
    del i


def test_normal_moments(ref):
    n = 200_000
    sch = ref.Schema(BASE_FIELDS)
    arrs = ref.fill(sch, n, seed=3)
    for c in range(3):
        v = arrs[sch.array_index("vel", c)].astype(np.float64)
        se = 1.0 / math.sqrt(n)
        assert abs(v.mean()) < 5 * se
        assert abs(v.var() - 1.0) < 5 * math.sqrt(2.0) * se
        assert abs((v ** 4).mean() - 3.0) < 5 * math.sqrt(96.0) * se
        assert abs((v ** 3).mean()) < 5 * math.sqrt(15.0) * se
    for c in range(3):
        x = arrs[sch.array_index("pos", c)]
        assert abs(x.mean() / BOX_L - 0.5) < 5 * math.sqrt(1 / 12 / n)


def test_fill_is_seeded_and_deterministic(ref):
    sch = ref.Schema(BASE_FIELDS)
    a = ref.fill(sch, 1000, seed=5)
    b = ref.fill(sch, 1000, seed=5)
    c = ref.fill(sch, 1000, seed=6)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[1], c[1])


def test_fill_prefix_independent_of_n(ref):
    sch = ref.Schema(BASE_FIELDS)
    a = ref.fill(sch, 100, seed=0)
    b = ref.fill(sch, 1000, seed=0)
    assert all(np.array_equal(x, y[:100]) for x, y in zip(a, b))


def test_fill_velocity_from_field(ref):
    sch = ref.Schema(BASE_FIELDS)
    abc = [1.0, 0.8, 0.6]
    arrs = ref.fill(sch, 257, seed=0, vel_mode=1, abc=abc)
    for i in (0, 100, 256):
        x = [arrs[sch.array_index("pos", d)][i] for d in range(3)]
        u = ref.field(abc, x)
        for d in range(3):
            assert arrs[sch.array_index("vel", d)][i] == np.float32(u[d])


def test_fill_range_matches_full_fill(ref):
    sch = ref.Schema(WIDE_FIELDS)
    full = ref.fill(sch, 5000, seed=9, vel_mode=0)
    part = ref.fill_range(sch, 1234, 777, seed=9)
    assert all(np.array_equal(a[1234:1234 + 777], b) for a, b in zip(full, part))
    sch = ref.Schema(BASE_FIELDS)
    full = ref.fill(sch, 3000, seed=2, vel_mode=1, abc=[1, 1, 1])
    part = ref.fill_range(sch, 2990, 10, seed=2, vel_mode=1, abc=[1, 1, 1])
    assert all(np.array_equal(a[2990:], b) for a, b in zip(full, part))
