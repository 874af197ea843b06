"""Pins of the oracle's removal by overwriting with the last particle
(Section 2): worked small cases, the survivors as a multiset, and the
invariant that only removed slots change."""
import numpy as np
import pytest

import synth_inputs as si


def run(ref, n, flagged):
    sch = ref.Schema([("id", "i64", 1), ("x", "f64", 2)])
    arrays = [np.arange(n, dtype=np.int64), np.arange(n) * 1.5, -np.arange(n) * 1.0]
    flags = np.zeros(n, np.uint8)
    flags[list(flagged)] = 1
    out, m = ref.remove_flagged(sch, arrays, flags)
    return out[0].tolist(), m


def test_worked_examples(ref):
    # removing 1 and 3 of 0..5: slot 1 takes 5, slot 3 takes 4
    assert run(ref, 6, [1, 3]) == ([0, 5, 2, 4], 4)
    # the last particle is itself removed: slot 1 takes 4 after 5 is dropped
    assert run(ref, 6, [1, 5]) == ([0, 4, 2, 3], 4)
    # everything removed; nothing removed; only the last removed
    assert run(ref, 4, [0, 1, 2, 3]) == ([], 0)
    assert run(ref, 4, []) == ([0, 1, 2, 3], 4)
    assert run(ref, 4, [3]) == ([0, 1, 2], 3)
    assert run(ref, 5, [0]) == ([4, 1, 2, 3], 4)
    assert run(ref, 1, [0]) == ([], 0)
    assert run(ref, 0, []) == ([], 0)


@pytest.mark.parametrize("seed", range(5))
def test_survivors_and_untouched_slots(ref, seed):
    rng = np.random.default_rng(seed)
    n = 2000
    fields = si.WIDE_FIELDS
    sch = ref.Schema(fields)
    arrays = si.random_state(fields, n, seed)
    flags = (rng.random(n) < rng.uniform(0.05, 0.9)).astype(np.uint8)
    out, m = ref.remove_flagged(sch, arrays, flags)
    keep = np.nonzero(flags == 0)[0]
    assert m == len(keep)
    ids = out[sch.array_index("id")]
    assert sorted(ids.tolist()) == keep.tolist()          # survivors, each once
    unflagged_low = keep[keep < m]
    assert np.array_equal(ids[unflagged_low], unflagged_low)  # they did not move
    # every record moved as a whole
    for a in range(len(arrays)):
        assert np.array_equal(out[a], arrays[a][ids])
    # the filled holes take the tail survivors, last first
    holes = np.nonzero(flags[:m])[0]
    movers = keep[keep >= m][::-1]
    assert np.array_equal(ids[holes], movers)
