"""Energy as a differentiable torch function (thin marshalling over the C ABI).

``nep_energy(context, pos, cell, theta, ...)`` returns the per-cell energies
E_c of the NEP-ZBL potential (Eq. 1 of the paper).  Its backward is the
library's ``nep_backward`` kernel pass: dE/dpos = -F, dE/dcell at fixed
Cartesian positions = h^-T (sum_i x_i (x) F_i - W^T), and dE/dtheta for the
network weights and the descriptor coefficients,
theta = (c_rad, c_ang, w0, b0, w1, b1) flattened row-major (1057 values for
the default model; the block sizes come from the context's model).
No arithmetic of the method runs in Python: the forward and the backward are
single library calls; torch only holds the buffers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import EFV, DeviceSystem, Weights, _check, _stream_ptr, lib

def split_theta(theta: torch.Tensor, sizes):
    """Views of a flat parameter vector: c_rad, c_ang, w0, b0, w1, b1, with
    the block sizes of the context's model (Context.theta_sizes)."""
    if theta.numel() != sum(sizes):
        raise ValueError(f"parameter vector has {theta.numel()} values, the model takes {sum(sizes)}")
    o = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    return tuple(theta[o[k]:o[k + 1]] for k in range(5)) + (theta[o[5]],)


def set_weights_from_device(context, theta: torch.Tensor, q_scale: torch.Tensor, stream=None):
    """Copy a device parameter vector (float32) into the context (nep_set_weights, device mode)."""
    theta = theta.detach().to(torch.float32).contiguous()
    q_scale = q_scale.detach().to(device=theta.device, dtype=torch.float32).contiguous()
    c_rad, c_ang, w0, b0, w1, b1 = split_theta(theta, context.theta_sizes)
    w = Weights(c_rad.data_ptr(), c_ang.data_ptr(), q_scale.data_ptr(), w0.data_ptr(), b0.data_ptr(),
                w1.data_ptr(), float(b1.item()), 0)
    _check(lib().nep_set_weights(context._ptr, C.byref(w), 1, _stream_ptr(stream)), "nep_set_weights")
    return theta, q_scale   # keep alive until the copy completed (set_weights synchronises)


class NEPEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, cell, theta, context, cell_start, q_scale, pbc, mass):
        cell_np = cell.detach().double().cpu().numpy().reshape(-1, 9)
        theta32, q32 = set_weights_from_device(context, theta, q_scale)
        sysd = DeviceSystem.__new__(DeviceSystem)
        p = pos.detach().double()
        sysd.x, sysd.y, sysd.z = p[:, 0].contiguous(), p[:, 1].contiguous(), p[:, 2].contiguous()
        sysd.vx = sysd.vy = sysd.vz = sysd.x
        sysd.h = np.ascontiguousarray(cell_np)
        sysd.n_cells = cell_np.shape[0]
        sysd.cell_start = np.ascontiguousarray(cell_start, dtype=np.int64)
        sysd.pbc = tuple(int(v) for v in pbc)
        sysd.mass = float(mass)
        sysd.n_atoms = p.shape[0]
        out = EFV(sysd.n_atoms, sysd.n_cells, device=pos.device)
        # the lists are rebuilt only when due (an atom moved more than skin/2
        # since the last build, or another system)
        context.nep_update_neighbors(sysd)
        context.nep_compute_efv(sysd, out)
        # the context now holds this forward's weights and lists
        token = object()
        context.state_token = token
        ctx.token = token
        ctx.context, ctx.sysd, ctx.out = context, sysd, out
        ctx.theta32, ctx.q32 = theta32, q32
        ctx.theta_dtype = theta.dtype
        ctx.cell_dtype = cell.dtype
        ctx.cell_device = cell.device
        return out.energy.clone()

    @staticmethod
    def backward(ctx, gE):
        context = ctx.context
        if context.state_token is not ctx.token:
            # another forward ran on this context since: its weights and
            # lists are not this forward's, so restore them (the parameter
            # gradient pass reads both from the context)
            set_weights_from_device(context, ctx.theta32, ctx.q32)
            context.nep_build_neighbors(ctx.sysd)
            context.state_token = ctx.token
        gp, gpos, gh = context.nep_backward(ctx.sysd, ctx.out, gE.detach())
        return (gpos, gh.to(device=ctx.cell_device, dtype=ctx.cell_dtype), gp.to(ctx.theta_dtype),
                None, None, None, None, None)


def nep_energy(context, pos, cell, theta, q_scale, cell_start=None, pbc=(1, 1, 1), mass=183.84):
    """Per-cell energies E_c (FP64) as a differentiable function of positions
    (N,3), cells (C,3,3, rows = lattice vectors) and the parameter vector."""
    if cell_start is None:
        cell_start = np.array([0, pos.shape[0]], dtype=np.int64)
    if cell.dim() == 2:
        cell = cell.unsqueeze(0)
    return NEPEnergy.apply(pos, cell, theta, context, cell_start, q_scale, pbc, mass)
