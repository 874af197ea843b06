"""Pins of the oracle's AoSoA (tiled) layout: the worked address of an
element, agreement with a numpy view of the tiles (a tile is a [arrays][64]
block for every element size), the zero lanes of a partial last tile, and
the round trip."""
import numpy as np
import pytest

import synth_inputs as si


def test_worked_layout_of_the_base_record(ref):
    sch = ref.Schema(si.BASE_FIELDS)  # id i32, pos f64 x3, vel f32 x3
    off, tile = ref.aosoa_layout(sch)
    # 64 * (4 + 3*8 + 3*4) = 2560 bytes per tile; arrays in schema order
    assert tile == 2560
    assert off == [0, 256, 768, 1280, 1792, 2048, 2304]
    # element 65 of pos.y (array 2): tile 1, lane 1 -> 2560 + 768 + 8
    n = 130
    arrays = si.random_state(si.BASE_FIELDS, n, 0)
    buf = ref.soa_to_aosoa(sch, arrays)
    assert buf.size == 3 * 2560
    assert buf[3336:3344].view(np.float64)[0] == arrays[2][65]


@pytest.mark.parametrize("fields", [si.BASE_FIELDS, si.WIDE_FIELDS], ids=["base", "wide"])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_tiles_are_array_blocks_and_round_trip(ref, fields, n):
    sch = ref.Schema(fields)
    arrays = si.random_state(fields, n, n)
    buf = ref.soa_to_aosoa(sch, arrays)
    off, tile = ref.aosoa_layout(sch)
    nt = -(-n // 64)
    tiles = buf.reshape(nt, tile)
    for a, arr in enumerate(arrays):
        es = arr.dtype.itemsize
        block = tiles[:, off[a]: off[a] + 64 * es].copy().view(arr.dtype).reshape(-1)
        assert np.array_equal(block[:n].view(np.uint8), arr.view(np.uint8))
        assert not block[n:].view(np.uint8).any()  # unused lanes are zero bytes
    back = ref.aosoa_to_soa(sch, buf, n)
    assert all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(back, arrays))
