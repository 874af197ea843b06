"""Pins of the oracle's integrator variants in the ABC field -- Heun's rule
(explicit trapezoid) and classical fourth-order Runge-Kutta -- and of the
symplectic (velocity-first) Euler step with acceleration:

- zero amplitudes leave positions unchanged; one non-zero amplitude gives
  the closed-form straight-line motion for any consistent one-step method;
- the local error's h^3 coefficient: Heun H(u,u)/4, RK4 the exact flow's
  (H(u,u) + J J u)/6 (and not the midpoint rule's H(u,u)/8);
- global convergence of order 2 (Heun) and 4 (RK4);
- with constant acceleration the symplectic step gives
  x_n = x_0 + n dt v_0 + dt^2 a n(n+1)/2, the explicit one n(n-1)/2.
"""
import numpy as np
import pytest

import synth_inputs as si
from test_oracle_rk2 import _jacobian, _second_derivative_term, pdist

L = si.BOX_L
EPS = 2.0 ** -52
FIELDS = [("pos", "f64", 3), ("vel", "f64", 3)]


def run(ref, integ, x0, abc, dt, nsteps, wrap=True):
    sch = ref.Schema(FIELDS)
    n = x0.shape[1]
    arrs = [np.ascontiguousarray(x0[d]).copy() for d in range(3)] + [np.zeros(n) for _ in range(3)]
    ref.step_soa(sch, arrs, integ, dt, nsteps, abc=abc, wrap=wrap)
    return np.stack(arrs[:3]), np.stack(arrs[3:])


@pytest.mark.parametrize("integ", ["HEUN_ABC", "RK4_ABC"])
def test_zero_field_and_single_amplitude(ref, integ):
    it = getattr(ref, integ)
    x0 = si.edge_positions(300, 2)
    x, v = run(ref, it, x0, [0.0, 0.0, 0.0], 1e-3, 10)
    assert np.array_equal(x, x0) and not v.any()
    n, nsteps, dt, amp = 2000, 40, 1e-3, 0.9
    x0, _ = si.adjoint_inputs(n, 21)
    x, _ = run(ref, it, x0, [0.0, amp, 0.0], dt, nsteps)  # B: u = (0, B sin x, B cos x)
    T = nsteps * dt
    X, Y, Z = x0
    want = [X, Y + T * amp * np.sin(X), Z + T * amp * np.cos(X)]
    for d in range(3):
        assert pdist(x[d], np.mod(want[d], L)).max() <= nsteps * 6 * EPS * L


@pytest.mark.parametrize("integ,coef", [("HEUN_ABC", "heun"), ("RK4_ABC", "exact")])
def test_local_error_coefficient(ref, integ, coef):
    it = getattr(ref, integ)
    abc = [1.0, 0.8, 0.6]
    rng = np.random.default_rng(1)
    separation = 0.0
    for _ in range(5):
        x = rng.uniform(0.5, 5.5, 3)
        u = ref.field(abc, x)
        J = _jacobian(abc, x)
        H = _second_derivative_term(abc, x, u)
        c3 = {}
        for h in (2e-3, 1e-3):
            xn, _ = run(ref, it, x.reshape(3, 1), abc, h, 1, wrap=False)
            c3[h] = (xn[:, 0] - x - h * u - 0.5 * h * h * (J @ u)) / h ** 3
        est = 2 * c3[1e-3] - c3[2e-3]
        want = H / 4 if coef == "heun" else (H + J @ (J @ u)) / 6
        scale = np.abs(want).max() + 1e-3
        assert np.abs(est - want).max() < 3e-3 * scale + 1e-4
        separation = max(separation, np.abs(est - H / 8).max() / np.abs(H).max())
    assert separation > 0.05  # not the midpoint rule


@pytest.mark.parametrize("integ,order", [("HEUN_ABC", 2), ("RK4_ABC", 4)])
def test_convergence_order(ref, integ, order):
    it = getattr(ref, integ)
    abc = [1.0, 1.0, 1.0]
    x0, _ = si.adjoint_inputs(32, 3)
    T = 0.5
    xref, _ = run(ref, ref.RK4_ABC, x0, abc, T / 4096, 4096, wrap=False)
    errs = []
    for m in (8, 16, 32):
        x, _ = run(ref, it, x0, abc, T / m, m, wrap=False)
        errs.append(np.abs(x - xref).max())
    ratio = 2.0 ** order
    for e1, e2 in zip(errs, errs[1:]):
        assert 0.8 * ratio < e1 / e2 < 1.25 * ratio


def test_velocity_is_field_at_new_position(ref):
    abc = [1.0, 0.5, 0.25]
    x0, _ = si.adjoint_inputs(100, 4)
    for it in (ref.HEUN_ABC, ref.RK4_ABC):
        x, v = run(ref, it, x0, abc, 1e-3, 2)
        for i in range(0, 100, 17):
            assert np.array_equal(v[:, i], ref.field(abc, x[:, i]))


def test_symplectic_euler_constant_acceleration(ref):
    fields = [("pos", "f64", 3), ("vel", "f64", 3), ("acc", "f64", 3)]
    sch = ref.Schema(fields)
    n, nsteps, dt = 64, 12, 0.25  # dt and the values below are exact in binary
    x0 = np.full(n, 1.0)
    v0 = (np.arange(n) - 32) / 32.0
    a = np.full(n, 0.5)
    out = {}
    for it in (ref.SYMPLECTIC_EULER, ref.EULER_ACC):
        arrs = [x0.copy(), x0.copy(), x0.copy(), v0.copy(), v0.copy(), v0.copy(), a, a, a]
        ref.step_soa(sch, arrs, it, dt, nsteps, wrap=False)
        out[it] = arrs
    sym = x0 + nsteps * dt * v0 + dt * dt * 0.5 * nsteps * (nsteps + 1) / 2
    exp = x0 + nsteps * dt * v0 + dt * dt * 0.5 * nsteps * (nsteps - 1) / 2
    assert np.array_equal(out[ref.SYMPLECTIC_EULER][0], sym)
    assert np.array_equal(out[ref.EULER_ACC][0], exp)
    assert np.array_equal(out[ref.SYMPLECTIC_EULER][3], v0 + nsteps * dt * 0.5)


def test_symplectic_velocity_is_rounded_before_the_position_update(ref):
    fields = [("pos", "f64", 3), ("vel", "f32", 3), ("acc", "f32", 3)]
    sch = ref.Schema(fields)
    v = np.array([0.1], np.float32)
    acc = np.array([0.3], np.float32)
    arrs = [np.zeros(1), np.zeros(1), np.zeros(1), v.copy(), v.copy(), v.copy(), acc, acc, acc]
    ref.step_soa(sch, arrs, ref.SYMPLECTIC_EULER, 1e-3, 1, wrap=False)
    vn = np.float32(np.float64(v[0]) + 1e-3 * np.float64(acc[0]))
    assert arrs[3][0] == vn
    assert arrs[0][0] == 0.0 + 1e-3 * np.float64(vn)
