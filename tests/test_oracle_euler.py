"""Pins of the oracle's Euler steps (Section 2, eq. (1)) and periodic wrap:
closed forms for uniform velocity and constant acceleration, the zero-velocity
special case, the range invariant of the wrap, and SoA/AoS equality."""
import numpy as np
import pytest

import synth_inputs as si

L = si.BOX_L
EPS = 2.0 ** -52


def pdist(a, b):
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    return np.minimum(d, L - d)


def _state(ref, fields, n, seed):
    sch = ref.Schema(fields)
    return sch, si.random_state(fields, n, seed)


def test_uniform_velocity_closed_form(ref):
    n, nsteps, dt = 2000, 100, 1e-3
    sch, arrs = _state(ref, si.BASE_FIELDS, n, 1)
    v = np.array([0.7, -1.3, 2.1], dtype=np.float32)
    for d in range(3):
        arrs[sch.array_index("vel", d)][:] = v[d]
    x0 = [arrs[sch.array_index("pos", d)].copy() for d in range(3)]
    ref.step_soa(sch, arrs, ref.EULER, dt, nsteps, wrap=True)
    for d in range(3):
        exact = np.mod(x0[d] + nsteps * dt * np.float64(v[d]), L)
        got = arrs[sch.array_index("pos", d)]
        assert pdist(got, exact).max() <= nsteps * 2 * EPS * L
        assert got.min() >= 0.0 and got.max() < L
        assert np.array_equal(arrs[sch.array_index("vel", d)], np.full(n, v[d]))
    assert np.array_equal(arrs[0], np.arange(n, dtype=np.int32))


def test_zero_velocity_leaves_state_unchanged(ref):
    sch, arrs = _state(ref, si.BASE_FIELDS, 1000, 2)
    for d in range(3):
        arrs[sch.array_index("vel", d)][:] = 0.0
    before = [a.copy() for a in arrs]
    ref.step_soa(sch, arrs, ref.EULER, 1e-3, 50, wrap=True)
    assert all(np.array_equal(a, b) for a, b in zip(arrs, before))


def test_wrap_keeps_positions_in_box(ref):
    n = 5000
    sch, arrs = _state(ref, si.BASE_FIELDS, n, 3)
    x = si.edge_positions(n, 3)
    for d in range(3):
        arrs[sch.array_index("pos", d)][:] = x[d]
        arrs[sch.array_index("vel", d)][:] *= 50.0  # |dt v| up to ~0.25
    x0 = [arrs[sch.array_index("pos", d)].copy() for d in range(3)]
    vel = [arrs[sch.array_index("vel", d)].astype(np.float64) for d in range(3)]
    ref.step_soa(sch, arrs, ref.EULER, 1e-3, 7, wrap=True)
    for d in range(3):
        got = arrs[sch.array_index("pos", d)]
        assert got.min() >= 0.0 and got.max() < L
        assert pdist(got, np.mod(x0[d] + 7 * 1e-3 * vel[d], L)).max() <= 7 * 2 * EPS * L


def test_wrap_edge_cases(ref):
    # one coordinate per case; single step, dt = 1
    cases = [(-1e-300, 0.0), (L - 4e-16, 1e-15), (0.0, -1e-20), (L - 1e-9, 2e-9), (3.0, 0.0)]
    fields = [("pos", "f64", 3), ("vel", "f64", 3)]
    sch = ref.Schema(fields)
    n = len(cases)
    arrs = [np.zeros(n) for _ in range(6)]  # pos x, y, z then vel x, y, z
    for i, (x, v) in enumerate(cases):
        arrs[0][i], arrs[3][i] = x, v
    ref.step_soa(sch, arrs, ref.EULER, 1.0, 1, wrap=True)
    got = arrs[0]
    assert got.min() >= 0.0 and got.max() < L
    assert got[0] == 0.0  # -1e-300 + L rounds to L, which is snapped to 0
    assert got[2] == 0.0  # likewise for -1e-20
    assert got[1] < 1e-15
    assert pdist(got[3], 1e-9) < 1e-15


def test_no_wrap_leaves_box(ref):
    fields = [("pos", "f64", 3), ("vel", "f32", 3)]
    sch = ref.Schema(fields)
    arrs = [np.full(4, L - 1e-6), np.zeros(4), np.zeros(4)] + \
        [np.full(4, 1.0, np.float32) for _ in range(3)]
    ref.step_soa(sch, arrs, ref.EULER, 1e-3, 1, wrap=False)
    assert (arrs[0] > L).all()


@pytest.mark.parametrize("vt", ["f64", "f32"])
def test_euler_acc_closed_form_and_order(ref, vt):
    # constant acceleration a: v_k = v0 + k dt a and, with positions advanced
    # by the velocity from before the update, x_n = x0 + n dt v0 + dt^2 a n(n-1)/2
    n, nsteps, dt = 1000, 20, 1e-3
    fields = [("pos", "f64", 3), ("vel", vt, 3), ("acc", vt, 3)]
    sch = ref.Schema(fields)
    arrs = si.random_state(fields, n, 4)
    x0 = [arrs[d].copy() for d in range(3)]
    v0 = [arrs[3 + d].astype(np.float64) for d in range(3)]
    a = [arrs[6 + d].astype(np.float64) for d in range(3)]
    ref.step_soa(sch, arrs, ref.EULER_ACC, dt, nsteps, wrap=False)
    ulp = 2.0 ** -52 if vt == "f64" else 2.0 ** -23
    for d in range(3):
        vmax = np.abs(v0[d]) + nsteps * dt * np.abs(a[d]) + 1.0
        x_exact = x0[d] + nsteps * dt * v0[d] + dt * dt * a[d] * nsteps * (nsteps - 1) / 2
        v_exact = v0[d] + nsteps * dt * a[d]
        tol_x = nsteps * 2 * EPS * 8 + dt * nsteps * nsteps * ulp * vmax
        assert np.abs(arrs[d] - x_exact).max() <= tol_x.max()
        assert np.abs(arrs[3 + d] - v_exact).max() <= (nsteps * ulp * vmax).max()
        # the other order (velocity first) differs by dt^2 a n
        other = x_exact + dt * dt * a[d] * nsteps
        assert (np.abs(arrs[d] - other) > 0.5 * dt * dt * np.abs(a[d]) * nsteps).mean() > 0.99


@pytest.mark.parametrize("fields", [si.BASE_FIELDS, si.WIDE_FIELDS, si.particle_size_fields(4)],
                         ids=["base", "wide", "particle4"])
@pytest.mark.parametrize("packed", [False, True])
def test_soa_and_aos_steps_agree_bit_exact(ref, fields, packed):
    n = 777
    sch = ref.Schema(fields, packed=packed)
    arrs = si.random_state(fields, n, 5)
    aos = ref.soa_to_aos(sch, arrs)
    integ = ref.EULER_ACC if any(f[0] == "acc" for f in fields) else ref.EULER
    wrap = dict((f[0], f[1]) for f in fields)["pos"] == "f64"
    ref.step_soa(sch, arrs, integ, 1e-3, 10, wrap=wrap)
    ref.step_aos(sch, aos, n, integ, 1e-3, 10, wrap=wrap)
    back = ref.aos_to_soa(sch, aos, n)
    assert all(np.array_equal(a, b) for a, b in zip(arrs, back))


def test_float32_positions_follow_c_promotion(ref):
    # float x; double dt; float v:  x += dt*v is evaluated in double, then rounded
    fields = si.particle_size_fields(0)
    sch = ref.Schema(fields)
    arrs = si.random_state(fields, 3000, 6)
    x0 = [a.copy() for a in arrs[:3]]
    v = [a.copy() for a in arrs[3:6]]
    ref.step_soa(sch, arrs, ref.EULER, 1e-3, 1, wrap=False)
    for d in range(3):
        want = (x0[d].astype(np.float64) + 1e-3 * v[d].astype(np.float64)).astype(np.float32)
        assert np.array_equal(arrs[d], want)
