"""Differentiable RK2 advection in the ABC field.

RK2Advect.apply(pos0, abc, dt, nsteps, k) advances positions pos0 ([3, n]
float64, on the GPU) by nsteps explicit-midpoint steps in the field with
amplitudes abc ([3] float64) and returns the final positions.  The forward
kernel keeps a checkpoint every k steps; backward runs the library's
discrete-adjoint kernel, which recomputes each k-step segment from its
checkpoint and sweeps it backwards, giving dL/dpos0 and dL/d(A, B, C).
"""
import ctypes

import torch

from ._lib import check, lib
from .particles import current_stream


# Rows of one checkpoint on the tape: the position and the sines and cosines
# of its three coordinates.
TAPE_ROWS = 9


def _rows(t):
    """Row pointers of a contiguous [3, n] float64 tensor."""
    assert t.dtype == torch.float64 and t.is_contiguous() and t.shape[0] == 3
    return (ctypes.c_void_p * 3)(*[t[d].data_ptr() for d in range(3)])


def _host3(abc):
    vals = [float(v) for v in abc.detach().to("cpu", torch.float64).reshape(3)]
    return (ctypes.c_double * 3)(*vals)


def forward_ckpt(pos0, abc_host, dt, nsteps, k):
    """(xT, tape) with the library's checkpointing forward kernel."""
    n = pos0.shape[1]
    xT = torch.empty_like(pos0)
    nck = max(1, -(-int(nsteps) // int(k)))
    tape = torch.empty((nck, TAPE_ROWS, max(n, 1)), dtype=torch.float64, device=pos0.device)
    check(lib().soax_rk2_forward_ckpt(_rows(pos0), _rows(xT), n, abc_host, float(dt), int(nsteps),
                                      int(k), ctypes.c_void_p(tape.data_ptr()), current_stream()),
          "soax_rk2_forward_ckpt")
    return xT, tape


def adjoint(tape, lamT, abc_host, dt, nsteps, k):
    """(dL/dx0, dL/d(A,B,C)) for the seed lamT = dL/dxT."""
    n = lamT.shape[1]
    gx = torch.empty_like(lamT)
    gabc = torch.empty(3, dtype=torch.float64, device=lamT.device)
    check(lib().soax_adjoint(ctypes.c_void_p(tape.data_ptr()), _rows(lamT), n, abc_host, float(dt),
                             int(nsteps), int(k), _rows(gx), ctypes.c_void_p(gabc.data_ptr()),
                             current_stream()), "soax_adjoint")
    return gx, gabc


def sqdist_loss(xT, target, want_grad=True):
    """(sum (xT - target)^2 as a 1-element tensor, 2 (xT - target) or None)."""
    n = xT.shape[1]
    loss = torch.empty(1, dtype=torch.float64, device=xT.device)
    lam = torch.empty_like(xT) if want_grad else None
    check(lib().soax_sqdist_loss(_rows(xT), _rows(target), n, _rows(lam) if want_grad else None,
                                 ctypes.c_void_p(loss.data_ptr()), current_stream()),
          "soax_sqdist_loss")
    return loss, lam


# ---------------------------------------------------- positions in AoS records

def _record_rows(buf, pos_offset, stride):
    """Pointers to pos[0..2] of record 0 in a uint8 record buffer, and the
    record stride in doubles."""
    assert buf.dtype == torch.uint8 and buf.is_contiguous()
    if pos_offset % 8 or stride % 8 or buf.data_ptr() % 8:
        raise ValueError("positions inside records must be 8-byte aligned")
    base = buf.data_ptr() + pos_offset
    return (ctypes.c_void_p * 3)(base, base + 8, base + 16), stride // 8


def forward_ckpt_records(x0_rec, xT_rec, pos_offset, stride, n, abc_host, dt, nsteps, k):
    """The checkpointing forward with x0 and xT inside AoS records (uint8
    buffers of n records; xT_rec may be x0_rec).  Returns the tape."""
    r0, sd = _record_rows(x0_rec, pos_offset, stride)
    rT, _ = _record_rows(xT_rec, pos_offset, stride)
    nck = max(1, -(-int(nsteps) // int(k)))
    tape = torch.empty((nck, TAPE_ROWS, max(n, 1)), dtype=torch.float64,
                       device=x0_rec.device)
    check(lib().soax_rk2_forward_ckpt_strided(r0, rT, n, sd, abc_host, float(dt), int(nsteps),
                                              int(k), ctypes.c_void_p(tape.data_ptr()),
                                              current_stream()), "soax_rk2_forward_ckpt_strided")
    return tape


def sqdist_loss_records(xT_rec, target, lam_rec, pos_offset, stride, n):
    """Loss with xT and the seed lam inside AoS records, target [3, n] SoA."""
    rT, sd = _record_rows(xT_rec, pos_offset, stride)
    rl, _ = _record_rows(lam_rec, pos_offset, stride)
    loss = torch.empty(1, dtype=torch.float64, device=xT_rec.device)
    check(lib().soax_sqdist_loss_strided(rT, sd, _rows(target), n, rl,
                                         ctypes.c_void_p(loss.data_ptr()), current_stream()),
          "soax_sqdist_loss_strided")
    return loss


def adjoint_records(tape, lam_rec, gx_rec, pos_offset, stride, n, abc_host, dt, nsteps, k):
    """dL/d(A,B,C); dL/dx0 written into gx_rec's position slots."""
    rl, sd = _record_rows(lam_rec, pos_offset, stride)
    rg, _ = _record_rows(gx_rec, pos_offset, stride)
    gabc = torch.empty(3, dtype=torch.float64, device=lam_rec.device)
    check(lib().soax_adjoint_strided(ctypes.c_void_p(tape.data_ptr()), rl, n, sd, abc_host,
                                     float(dt), int(nsteps), int(k), rg,
                                     ctypes.c_void_p(gabc.data_ptr()), current_stream()),
          "soax_adjoint_strided")
    return gabc


class RK2Advect(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos0, abc, dt, nsteps, k):
        pos0 = pos0.contiguous()
        abc_host = _host3(abc)
        xT, tape = forward_ckpt(pos0, abc_host, dt, nsteps, k)
        ctx.save_for_backward(tape)
        ctx.abc_host, ctx.dt, ctx.nsteps, ctx.k = abc_host, dt, nsteps, k
        ctx.abc_device = abc.device
        return xT

    @staticmethod
    def backward(ctx, grad_xT):
        (tape,) = ctx.saved_tensors
        lam = grad_xT.contiguous().to(torch.float64)
        gx, gabc = adjoint(tape, lam, ctx.abc_host, ctx.dt, ctx.nsteps, ctx.k)
        return gx, gabc.to(ctx.abc_device), None, None, None


def rk2_advect(pos0, abc, dt, nsteps, k=20):
    return RK2Advect.apply(pos0, abc, dt, nsteps, k)
