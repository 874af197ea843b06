"""GPU parity of the checkpointed RK2 forward, the discrete adjoint and the
loss against the CPU oracle (which stores every state), plus properties the
checkpointing must keep: gradients bit-identical for every k, and a torch
autograd round trip."""
import numpy as np
import pytest
import torch

import synth_inputs as si
from gpu_util import L

pytestmark = pytest.mark.gpu

soax = pytest.importorskip("paper_1710_03462_amd")

ABC = [1.0, 0.8, 0.6]


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_fwd_bwd(x0, target, abc, dt, nsteps, k):
    abc_host = soax.autograd._host3(torch.tensor(abc, dtype=torch.float64))
    xT, tape = soax.forward_ckpt(gpu(x0), abc_host, dt, nsteps, k)
    loss, lam = soax.sqdist_loss(xT, gpu(target))
    gx, gabc = soax.adjoint(tape, lam, abc_host, dt, nsteps, k)
    torch.cuda.synchronize()
    return (xT.cpu().numpy(), tape.cpu().numpy(), float(loss.item()), gx.cpu().numpy(),
            gabc.cpu().numpy())


def ref_fwd_bwd(ref, x0, target, abc, dt, nsteps):
    xT, states = ref.rk2_forward(x0, abc, dt, nsteps, store_states=True)
    loss, lam = ref.sqdist_loss(xT, target)
    gx, gabc = ref.adjoint(x0, lam, abc, dt, nsteps)
    return xT, states, loss, gx, gabc


def check_grads(gx, gabc, rgx, rgabc):
    assert np.abs(gx - rgx).max() <= 1e-6 * np.abs(rgx).max()
    assert np.all(np.abs(gabc - rgabc) <= 1e-6 * np.abs(rgabc))


@pytest.mark.parametrize("n,nsteps,k", [(1, 200, 20), (2000, 200, 20), (777, 203, 20),
                                        (300, 50, 7), (257, 10, 64), (129, 40, 1),
                                        (600, 140, 60)])
def test_forward_adjoint_match_oracle(ref, n, nsteps, k):
    dt = 5e-3
    x0, target = si.adjoint_inputs(n, seed=n + nsteps)
    xT, tape, loss, gx, gabc = gpu_fwd_bwd(x0, target, ABC, dt, nsteps, k)
    rxT, states, rloss, rgx, rgabc = ref_fwd_bwd(ref, x0, target, ABC, dt, nsteps)
    assert np.abs(xT - rxT).max() <= 1e-12 * L
    for c in range(-(-nsteps // k)):
        assert np.abs(tape[c][:3] - states[c * k]).max() <= 1e-12 * L
        # rows 3..8: sin and cos of the checkpoint's coordinates, carried by
        # angle additions (at most 19 since the last full evaluation)
        for d in range(3):
            assert np.abs(tape[c][3 + 2 * d] - np.sin(tape[c][d])).max() <= 64 * 2.0 ** -52
            assert np.abs(tape[c][4 + 2 * d] - np.cos(tape[c][d])).max() <= 64 * 2.0 ** -52
    assert abs(loss - rloss) <= 1e-12 * abs(rloss)
    check_grads(gx, gabc, rgx, rgabc)


@pytest.mark.parametrize("dt", [0.05, 0.1])
def test_large_steps_match_oracle(ref, dt):
    # dt * (A+B+C) > 1/8: checked shifts with full-reduction fallback
    n, nsteps, k = 600, 30, 7
    x0, target = si.adjoint_inputs(n, seed=8)
    xT, tape, loss, gx, gabc = gpu_fwd_bwd(x0, target, ABC, dt, nsteps, k)
    rxT, states, rloss, rgx, rgabc = ref_fwd_bwd(ref, x0, target, ABC, dt, nsteps)
    assert np.abs(xT - rxT).max() <= 1e-12 * L
    assert abs(loss - rloss) <= 1e-12 * abs(rloss)
    check_grads(gx, gabc, rgx, rgabc)


def test_gradients_bit_identical_for_every_k():
    n, nsteps, dt = 1500, 200, 5e-3
    x0, target = si.adjoint_inputs(n, seed=5)
    base = gpu_fwd_bwd(x0, target, ABC, dt, nsteps, 20)
    # k = 20, 40, 60, 80, 200 and 1000 take the straight-line kernel for k and
    # nsteps that are multiples of 20 (60 and 80 with a shorter last segment),
    # the others the general one
    for k in (1, 7, 32, 33, 40, 60, 80, 200, 1000):
        got = gpu_fwd_bwd(x0, target, ABC, dt, nsteps, k)
        assert np.array_equal(got[0], base[0]), k
        assert np.array_equal(got[3], base[3]), k
        assert np.array_equal(got[4], base[4]), k


def test_zero_steps_and_empty():
    x0, target = si.adjoint_inputs(10, seed=1)
    xT, tape, loss, gx, gabc = gpu_fwd_bwd(x0, target, ABC, 5e-3, 0, 20)
    assert np.array_equal(xT, x0)
    assert np.array_equal(gx, 2 * (x0 - target))
    assert not gabc.any()
    e = np.zeros((3, 0))
    xT, tape, loss, gx, gabc = gpu_fwd_bwd(e, e, ABC, 5e-3, 10, 3)
    assert loss == 0.0 and not gabc.any()


def test_single_amplitude_closed_form_on_gpu():
    n, nsteps, dt, A = 1000, 40, 5e-3, 1.1
    T = nsteps * dt
    x0, target = si.adjoint_inputs(n, seed=2)
    xT, _, _, gx, gabc = gpu_fwd_bwd(x0, target, [A, 0.0, 0.0], dt, nsteps, 20)
    X, Y, Z = x0
    ex, ey, ez = xT - target
    dA = (2 * ex * T * np.sin(Z) + 2 * ey * T * np.cos(Z)).sum()
    assert abs(gabc[0] - dA) <= 1e-9 * abs(dA)
    dz = 2 * ex * T * A * np.cos(Z) - 2 * ey * T * A * np.sin(Z) + 2 * ez
    assert np.abs(gx[2] - dz).max() <= 1e-9 * np.abs(dz).max()


def test_autograd_function_matches_oracle(ref):
    n, nsteps, dt, k = 999, 120, 5e-3, 20
    x0, target = si.adjoint_inputs(n, seed=3)
    pos0 = gpu(x0).requires_grad_(True)
    abc = torch.tensor(ABC, dtype=torch.float64, device="cuda", requires_grad=True)
    xT = soax.rk2_advect(pos0, abc, dt, nsteps, k)
    loss = ((xT - gpu(target)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    _, _, rloss, rgx, rgabc = ref_fwd_bwd(ref, x0, target, ABC, dt, nsteps)
    assert abs(loss.item() - rloss) <= 1e-12 * rloss
    check_grads(pos0.grad.cpu().numpy(), abc.grad.cpu().numpy(), rgx, rgabc)


def test_parameter_gradient_matches_gpu_finite_differences():
    n, nsteps, dt, k, h = 4000, 200, 5e-3, 20, 1e-6
    x0, target = si.adjoint_inputs(n, seed=4)
    _, _, _, _, gabc = gpu_fwd_bwd(x0, target, ABC, dt, nsteps, k)
    for j in range(3):
        p, m = list(ABC), list(ABC)
        p[j] += h
        m[j] -= h
        fd = (gpu_fwd_bwd(x0, target, p, dt, nsteps, k)[2] -
              gpu_fwd_bwd(x0, target, m, dt, nsteps, k)[2]) / (2 * h)
        assert abs(fd - gabc[j]) <= 1e-6 * abs(gabc[j])


def _records(x, stride, pos_offset, fill=0):
    """uint8 record buffer (n records) with x [3, n] at pos_offset; other bytes `fill`."""
    n = x.shape[1]
    rec = torch.full((n, stride), fill, dtype=torch.uint8, device="cuda")
    rec[:, pos_offset:pos_offset + 24] = x.t().contiguous().view(torch.uint8).view(n, 24)
    return rec.view(-1)


def _positions(rec, n, stride, pos_offset):
    return rec.view(n, stride)[:, pos_offset:pos_offset + 24].contiguous().view(torch.float64).t()


@pytest.mark.parametrize("stride,pos_offset", [(48, 8), (80, 16), (24, 0)])
@pytest.mark.parametrize("n", [1, 1000])
def test_positions_in_records_match_soa_bit_for_bit(ref, stride, pos_offset, n):
    """Forward, loss and adjoint with the positions kept inside AoS records give
    the SoA results bit for bit, and leave every other record byte alone."""
    dt, nsteps, k = 5e-3, 60, 20
    x0, target = si.adjoint_inputs(n, seed=n)
    abc_host = soax.autograd._host3(torch.tensor(ABC, dtype=torch.float64))
    X0, TG = gpu(x0), gpu(target)
    xT, tape = soax.forward_ckpt(X0, abc_host, dt, nsteps, k)
    loss, lam = soax.sqdist_loss(xT, TG)
    gx, gabc = soax.adjoint(tape, lam, abc_host, dt, nsteps, k)
    from paper_1710_03462_amd import autograd as A
    rec = _records(X0, stride, pos_offset, fill=0xA5)
    before = rec.clone()
    tape_r = A.forward_ckpt_records(rec, rec, pos_offset, stride, n, abc_host, dt, nsteps, k)
    lam_rec = torch.zeros(n * stride, dtype=torch.uint8, device="cuda")
    loss_r = A.sqdist_loss_records(rec, TG, lam_rec, pos_offset, stride, n)
    gx_rec = torch.zeros(n * stride, dtype=torch.uint8, device="cuda")
    gabc_r = A.adjoint_records(tape_r, lam_rec, gx_rec, pos_offset, stride, n, abc_host, dt,
                               nsteps, k)
    torch.cuda.synchronize()
    assert torch.equal(_positions(rec, n, stride, pos_offset), xT)
    assert torch.equal(tape_r, tape)
    assert torch.equal(loss_r, loss)
    assert torch.equal(_positions(lam_rec, n, stride, pos_offset), lam)
    assert torch.equal(_positions(gx_rec, n, stride, pos_offset), gx)
    assert torch.equal(gabc_r, gabc)
    r, b = rec.view(n, stride), before.view(n, stride)
    assert torch.equal(r[:, :pos_offset], b[:, :pos_offset])
    assert torch.equal(r[:, pos_offset + 24:], b[:, pos_offset + 24:])
