"""Pins of the oracle's RK2 (explicit midpoint) advection in the ABC field.

- the field at points where it has textbook values;
- zero amplitudes leave positions unchanged;
- one non-zero amplitude makes the field constant along each trajectory, so
  every consistent one-step method gives x0 + n dt u(x0) exactly (up to
  rounding): A only moves x and y at fixed z, B only y and z at fixed x,
  C only x and z at fixed y;
- second-order convergence in dt;
- the local error's h^3 coefficient, which separates the midpoint rule
  (H(u,u)/8) from Heun's rule (H(u,u)/4) and from the exact flow;
- the velocity written after a step is the field at the new position.
"""
import numpy as np
import pytest

import synth_inputs as si

L = si.BOX_L
EPS = 2.0 ** -52
FIELDS = [("pos", "f64", 3), ("vel", "f64", 3)]


def pdist(a, b):
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    return np.minimum(d, L - d)


def run(ref, x0, abc, dt, nsteps, wrap=True, fields=FIELDS):
    sch = ref.Schema(fields)
    n = x0.shape[1]
    arrs = [np.ascontiguousarray(x0[d]).copy() for d in range(3)]
    vt = dict((f[0], f[1]) for f in fields)["vel"]
    arrs += [np.zeros(n, dtype=np.float64 if vt == "f64" else np.float32) for _ in range(3)]
    ref.step_soa(sch, arrs, ref.RK2_ABC, dt, nsteps, abc=abc, wrap=wrap)
    return np.stack(arrs[:3]), np.stack([a.astype(np.float64) for a in arrs[3:]])


def test_field_textbook_values(ref):
    A, B, C = 1.3, 0.7, 0.4
    assert np.array_equal(ref.field([A, B, C], [0.0, 0.0, 0.0]), [C, A, B])
    u = ref.field([A, B, C], [np.pi / 2] * 3)
    assert np.allclose(u, [A, B, C], rtol=0, atol=1e-15)
    u = ref.field([A, B, C], [np.pi, np.pi, np.pi])
    assert np.allclose(u, [-C, -A, -B], rtol=0, atol=1e-15)


def test_zero_field_leaves_positions_unchanged(ref):
    x0 = si.edge_positions(500, 1)
    x, v = run(ref, x0, [0.0, 0.0, 0.0], 1e-3, 20)
    assert np.array_equal(x, x0)
    assert not v.any()


@pytest.mark.parametrize("which", [0, 1, 2])
def test_single_amplitude_closed_form(ref, which):
    n, nsteps, dt = 3000, 50, 1e-3
    x0, _ = si.adjoint_inputs(n, 10 + which)
    amp = 1.25
    abc = [0.0, 0.0, 0.0]
    abc[which] = amp
    x, v = run(ref, x0, abc, dt, nsteps)
    T = nsteps * dt
    X, Y, Z = x0
    if which == 0:    # A: u = (A sin z, A cos z, 0)
        want = [X + T * amp * np.sin(Z), Y + T * amp * np.cos(Z), Z]
    elif which == 1:  # B: u = (0, B sin x, B cos x)
        want = [X, Y + T * amp * np.sin(X), Z + T * amp * np.cos(X)]
    else:             # C: u = (C cos y, 0, C sin y)
        want = [X + T * amp * np.cos(Y), Y, Z + T * amp * np.sin(Y)]
    for d in range(3):
        assert pdist(x[d], np.mod(want[d], L)).max() <= nsteps * 4 * EPS * L
        assert x[d].min() >= 0 and x[d].max() < L


def _second_derivative_term(abc, x, u):
    """H(u,u)_r = sum_cd d^2 u_r / dx_c dx_d u_c u_d for the ABC field."""
    A, B, C = abc
    X, Y, Z = x
    return np.array([-A * np.sin(Z) * u[2] ** 2 - C * np.cos(Y) * u[1] ** 2,
                     -B * np.sin(X) * u[0] ** 2 - A * np.cos(Z) * u[2] ** 2,
                     -C * np.sin(Y) * u[1] ** 2 - B * np.cos(X) * u[0] ** 2])


def _jacobian(abc, x):
    A, B, C = abc
    X, Y, Z = x
    return np.array([[0.0, -C * np.sin(Y), A * np.cos(Z)],
                     [B * np.cos(X), 0.0, -A * np.sin(Z)],
                     [-B * np.sin(X), C * np.cos(Y), 0.0]])


def test_local_error_coefficient_is_midpoint(ref):
    # x+ = x + h u + h^2/2 J u + h^3 c3 + O(h^4); the midpoint rule has
    # c3 = H(u,u)/8, Heun's rule H(u,u)/4, the exact flow (H(u,u) + J J u)/6.
    abc = [1.0, 0.8, 0.6]
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.uniform(0.5, 5.5, 3)
        u = ref.field(abc, x)
        J = _jacobian(abc, x)
        H = _second_derivative_term(abc, x, u)
        c3 = {}
        for h in (2e-3, 1e-3):
            xn, _ = run(ref, x.reshape(3, 1), abc, h, 1, wrap=False)
            c3[h] = (xn[:, 0] - x - h * u - 0.5 * h * h * (J @ u)) / h ** 3
        est = 2 * c3[1e-3] - c3[2e-3]  # Richardson: removes the O(h) term
        scale = np.abs(H).max() + 1e-3
        assert np.abs(est - H / 8).max() < 2e-3 * scale + 1e-4
        assert np.abs(est - H / 4).max() > 0.05 * np.abs(H).max()


def test_second_order_convergence(ref):
    abc = [1.0, 1.0, 1.0]
    x0, _ = si.adjoint_inputs(64, 3)
    T = 0.5
    xref, _ = run(ref, x0, abc, T / 2048, 2048, wrap=False)
    errs = []
    for m in (16, 32, 64):
        x, _ = run(ref, x0, abc, T / m, m, wrap=False)
        errs.append(np.abs(x - xref).max())
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.5 < e1 / e2 < 4.5


def test_velocity_is_field_at_new_position(ref):
    abc = [1.0, 1.0, 1.0]
    x0, _ = si.adjoint_inputs(300, 4)
    x, v = run(ref, x0, abc, 1e-3, 3, fields=si.BASE_FIELDS[1:])
    for i in range(0, 300, 37):
        u = ref.field(abc, x[:, i])
        assert np.array_equal(v[:, i], u.astype(np.float32).astype(np.float64))


def test_positions_stay_in_box_near_edges(ref):
    x0 = si.edge_positions(2000, 5)
    x, _ = run(ref, x0, [1.0, 1.0, 1.0], 1e-2, 5)
    assert x.min() >= 0.0 and x.max() < L


@pytest.mark.parametrize("packed", [False, True])
def test_rk2_soa_and_aos_agree_bit_exact(ref, packed):
    n = 501
    sch = ref.Schema(si.BASE_FIELDS, packed=packed)
    arrs = si.random_state(si.BASE_FIELDS, n, 6)
    aos = ref.soa_to_aos(sch, arrs)
    ref.step_soa(sch, arrs, ref.RK2_ABC, 1e-3, 5, abc=[1, 1, 1], wrap=True)
    ref.step_aos(sch, aos, n, ref.RK2_ABC, 1e-3, 5, abc=[1, 1, 1], wrap=True)
    back = ref.aos_to_soa(sch, aos, n)
    assert all(np.array_equal(a, b) for a, b in zip(arrs, back))
