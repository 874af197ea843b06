"""Pins of the oracle's discrete adjoint of RK2 advection (positions only,
no wrap): central finite differences, an independent forward-mode (tangent)
computation, and the closed form for a single amplitude A."""
import numpy as np
import pytest

import synth_inputs as si


def loss_of(ref, x0, target, abc, dt, nsteps):
    xT = ref.rk2_forward(x0, abc, dt, nsteps)
    return ref.sqdist_loss(xT, target)[0]


@pytest.fixture(scope="module")
def case(ref):
    n, nsteps, dt = 400, 200, 5e-3
    abc = np.array([1.0, 0.8, 0.6])
    x0, target = si.adjoint_inputs(n, 11)
    xT = ref.rk2_forward(x0, abc, dt, nsteps)
    loss, lam = ref.sqdist_loss(xT, target)
    gx, gabc = ref.adjoint(x0, lam, abc, dt, nsteps)
    return dict(n=n, nsteps=nsteps, dt=dt, abc=abc, x0=x0, target=target, xT=xT, loss=loss,
                lam=lam, gx=gx, gabc=gabc)


def test_loss_and_seed_gradient(ref, case):
    d = case["xT"] - case["target"]
    assert np.isclose(case["loss"], (d * d).sum(), rtol=1e-13)
    assert np.array_equal(case["lam"], 2 * d)


def test_adjoint_equals_tangent(ref, case):
    gx, gabc = ref.tangent(case["x0"], case["lam"], case["abc"], case["dt"], case["nsteps"])
    assert np.abs(gx - case["gx"]).max() <= 1e-12 * np.abs(gx).max()
    assert np.abs(gabc - case["gabc"]).max() <= 1e-12 * np.abs(gabc).max()


def test_parameter_gradient_matches_finite_differences(ref, case):
    h = 1e-6
    for j in range(3):
        p, m = case["abc"].copy(), case["abc"].copy()
        p[j] += h
        m[j] -= h
        fd = (loss_of(ref, case["x0"], case["target"], p, case["dt"], case["nsteps"]) -
              loss_of(ref, case["x0"], case["target"], m, case["dt"], case["nsteps"])) / (2 * h)
        assert abs(fd - case["gabc"][j]) <= 1e-6 * abs(case["gabc"][j])


def test_position_gradient_matches_finite_differences(ref, case):
    h = 1e-6
    for i, d in [(0, 0), (17, 1), (123, 2), (399, 0), (250, 2)]:
        # per-particle loss: the other particles do not move
        x0 = case["x0"][:, i:i + 1].copy()
        t = case["target"][:, i:i + 1].copy()
        xp, xm = x0.copy(), x0.copy()
        xp[d, 0] += h
        xm[d, 0] -= h
        fd = (loss_of(ref, xp, t, case["abc"], case["dt"], case["nsteps"]) -
              loss_of(ref, xm, t, case["abc"], case["dt"], case["nsteps"])) / (2 * h)
        g = case["gx"][d, i]
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1.0)


def test_single_amplitude_closed_form_gradients(ref):
    # B = C = 0: z is constant, x_T = x0 + T A sin z0, y_T = y0 + T A cos z0
    n, nsteps, dt, A = 300, 40, 5e-3, 1.1
    T = nsteps * dt
    x0, target = si.adjoint_inputs(n, 12)
    abc = np.array([A, 0.0, 0.0])
    xT = ref.rk2_forward(x0, abc, dt, nsteps)
    _, lam = ref.sqdist_loss(xT, target)
    gx, gabc = ref.adjoint(x0, lam, abc, dt, nsteps)
    X, Y, Z = x0
    ex, ey, ez = (xT - target)
    dA = (2 * ex * T * np.sin(Z) + 2 * ey * T * np.cos(Z)).sum()
    assert abs(gabc[0] - dA) <= 1e-10 * abs(dA)
    assert np.allclose(gx[0], 2 * ex, rtol=0, atol=1e-12)
    assert np.allclose(gx[1], 2 * ey, rtol=0, atol=1e-12)
    dz = 2 * ex * T * A * np.cos(Z) - 2 * ey * T * A * np.sin(Z) + 2 * ez
    assert np.abs(gx[2] - dz).max() <= 1e-11 * np.abs(dz).max()


def test_zero_steps_gradient_is_seed(ref):
    x0, target = si.adjoint_inputs(10, 13)
    _, lam = ref.sqdist_loss(x0, target)
    gx, gabc = ref.adjoint(x0, lam, [1, 1, 1], 1e-2, 0)
    assert np.array_equal(gx, lam)
    assert not gabc.any()


def test_forward_states_chain(ref):
    x0, _ = si.adjoint_inputs(50, 14)
    xT, states = ref.rk2_forward(x0, [1, 0.8, 0.6], 5e-3, 30, store_states=True)
    assert np.array_equal(states[0], x0)
    assert np.array_equal(states[30], xT)
    mid = ref.rk2_forward(states[10], [1, 0.8, 0.6], 5e-3, 20)
    assert np.array_equal(mid, xT)
