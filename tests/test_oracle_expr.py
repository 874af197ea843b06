"""Pins of the oracle's fused-expression evaluation (the whole-array
expressions of Section 4.1): worked values for every op, operand order of
the non-commutative ops, the paper's example posArr(0) = velArr(1) -
velArr(2), rounding to a float destination, and agreement with the same
expression written in infix numpy."""
import numpy as np

import oracle as ref

A, C = ref.OP_ARRAY, ref.OP_CONST


def run(arrays, prog, dst=np.float64):
    return ref.eval_program(arrays, prog, dst)


def test_each_op_on_worked_values():
    a = np.array([6.0, -2.0, 9.0])
    b = np.array([3.0, 4.0, -9.0])
    two = [a, b]
    assert run(two, [(A, 0, 0), (A, 1, 0), (ref.OP_ADD, 0, 0)]).tolist() == [9.0, 2.0, 0.0]
    assert run(two, [(A, 0, 0), (A, 1, 0), (ref.OP_SUB, 0, 0)]).tolist() == [3.0, -6.0, 18.0]
    assert run(two, [(A, 1, 0), (A, 0, 0), (ref.OP_SUB, 0, 0)]).tolist() == [-3.0, 6.0, -18.0]
    assert run(two, [(A, 0, 0), (A, 1, 0), (ref.OP_MUL, 0, 0)]).tolist() == [18.0, -8.0, -81.0]
    assert run(two, [(A, 0, 0), (A, 1, 0), (ref.OP_DIV, 0, 0)]).tolist() == [2.0, -0.5, -1.0]
    assert run(two, [(A, 0, 0), (A, 1, 0), (ref.OP_MIN, 0, 0)]).tolist() == [3.0, -2.0, -9.0]
    assert run(two, [(A, 0, 0), (A, 1, 0), (ref.OP_MAX, 0, 0)]).tolist() == [6.0, 4.0, 9.0]
    assert run(two, [(A, 1, 0), (ref.OP_NEG, 0, 0)]).tolist() == [-3.0, -4.0, 9.0]
    assert run(two, [(A, 1, 0), (ref.OP_ABS, 0, 0)]).tolist() == [3.0, 4.0, 9.0]
    assert run([np.array([16.0, 2.25, 0.0])], [(A, 0, 0), (ref.OP_SQRT, 0, 0)]).tolist() == [4.0, 1.5, 0.0]
    assert run(two, [(A, 0, 0), (C, 0, 0.5), (ref.OP_MUL, 0, 0)]).tolist() == [3.0, -1.0, 4.5]


def test_paper_example_velocity_difference():
    # posArr(0) = velArr(1) - velArr(2) on float velocities: the difference of
    # two floats is exact in double
    rng = np.random.default_rng(0)
    v1 = rng.standard_normal(1000).astype(np.float32)
    v2 = rng.standard_normal(1000).astype(np.float32)
    got = run([v1, v2], [(A, 0, 0), (A, 1, 0), (ref.OP_SUB, 0, 0)])
    exact = v1.astype(np.float64) - v2.astype(np.float64)
    assert np.array_equal(got, exact)
    # a float destination rounds that exact difference once: the float subtraction
    assert np.array_equal(run([v1, v2], [(A, 0, 0), (A, 1, 0), (ref.OP_SUB, 0, 0)], np.float32),
                          v1 - v2)


def test_integer_sources_widen_exactly():
    ids = np.arange(-5, 5, dtype=np.int32)
    big = np.array([2 ** 53, -(2 ** 53)] * 5, dtype=np.int64)
    got = run([ids, big], [(A, 0, 0), (A, 1, 0), (ref.OP_ADD, 0, 0)])
    assert np.array_equal(got, ids.astype(np.float64) + big.astype(np.float64))


def test_composite_matches_infix():
    rng = np.random.default_rng(1)
    x, y, z = (rng.random(500) + 0.1 for _ in range(3))
    # sqrt(x*x + 2.5*y) - min(x, 1) / z
    prog = [(A, 0, 0), (A, 0, 0), (ref.OP_MUL, 0, 0), (C, 0, 2.5), (A, 1, 0), (ref.OP_MUL, 0, 0),
            (ref.OP_ADD, 0, 0), (ref.OP_SQRT, 0, 0), (A, 0, 0), (C, 0, 1.0), (ref.OP_MIN, 0, 0),
            (A, 2, 0), (ref.OP_DIV, 0, 0), (ref.OP_SUB, 0, 0)]
    want = np.sqrt(x * x + 2.5 * y) - np.minimum(x, 1.0) / z
    assert np.array_equal(run([x, y, z], prog), want)


def test_malformed_programs_raise():
    import pytest
    a = [np.ones(3)]
    with pytest.raises(ValueError):
        run(a, [(A, 0, 0), (A, 0, 0)])
    with pytest.raises(IndexError):
        run(a, [(ref.OP_NEG, 0, 0)])
