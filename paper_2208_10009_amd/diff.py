"""Differentiable path quantities (sbr_path_gradients) for PyTorch.

For paths of fixed interaction sequences (the face sequences sbr_trace
returns), the delay, AOD, AOA and power of the image-method path that the
precise algorithm converges to are smooth in the transmitter and receiver
positions and in the materials' complex permittivities.  The forward values
and the hand-written adjoint both run in the library's HIP kernel; this
module only wires them into torch.autograd.  All tensors live on the
context's device and use its stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import sbr


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_inputs(tx, rx, eps, order, faces, device):
    """The C ABI reads raw FP64 / int32 device arrays of these shapes."""
    P = rx.shape[0]
    for name, t, dt, shape in (("tx", tx, torch.float64, (P, 3)), ("rx", rx, torch.float64, (P, 3)),
                               ("eps", eps, torch.float64, (eps.shape[0], 2)),
                               ("order", order, torch.int32, (P,)),
                               ("faces", faces, torch.int32, (P, sbr.MAX_ORDER))):
        if t.dtype != dt:
            raise TypeError("%s must be %s (got %s)" % (name, dt, t.dtype))
        if t.device != device:
            raise ValueError("%s must be on %s (got %s)" % (name, device, t.device))
        if tuple(t.shape) != shape:
            raise ValueError("%s must have shape %s (got %s)" % (name, shape, tuple(t.shape)))


def _setup():
    L = sbr.lib()
    if not getattr(L, "_grad_ready", False):
        vp = C.c_void_p
        L.sbr_path_gradients.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, C.c_double,
                                         C.c_double, vp, vp, vp, vp, vp]
        L.sbr_path_gradients.restype = C.c_int32
        L._grad_ready = True
    return L


class PathQuantities(torch.autograd.Function):
    """values[P, 8] = (delay s, AOD xyz, AOA xyz, power dBm) of each path, as a
    function of tx[P, 3], rx[P, 3] and eps[M, 2] (real, imaginary parts)."""

    @staticmethod
    def forward(ctx, tx, rx, eps, scene, order, faces, freq_hz, tx_power_dbm):
        L = _setup()
        dev = torch.device("cuda", scene.ctx.device)
        _check_inputs(tx, rx, eps, order, faces, dev)
        tx, rx, eps = tx.contiguous(), rx.contiguous(), eps.contiguous()
        order, faces = order.contiguous(), faces.contiguous()
        P = tx.shape[0]
        val = torch.empty((P, 8), dtype=torch.float64, device=tx.device)
        st = L.sbr_path_gradients(scene.h, P, _ptr(tx), _ptr(rx), _ptr(order), _ptr(faces),
                                  _ptr(eps), freq_hz, tx_power_dbm, None, _ptr(val), None, None,
                                  None)
        scene.ctx._check(st)
        ctx.save_for_backward(tx, rx, eps, order, faces)
        ctx.scene, ctx.freq_hz, ctx.tx_power_dbm = scene, freq_hz, tx_power_dbm
        return val

    @staticmethod
    def backward(ctx, gval):
        L = _setup()
        tx, rx, eps, order, faces = ctx.saved_tensors
        gval = gval.to(torch.float64).contiguous()
        gtx, grx = torch.empty_like(tx), torch.empty_like(rx)
        geps = torch.zeros_like(eps)
        st = L.sbr_path_gradients(ctx.scene.h, tx.shape[0], _ptr(tx), _ptr(rx), _ptr(order),
                                  _ptr(faces), _ptr(eps), ctx.freq_hz, ctx.tx_power_dbm,
                                  _ptr(gval), None, _ptr(gtx), _ptr(grx), _ptr(geps))
        ctx.scene.ctx._check(st)
        return gtx, grx, geps, None, None, None, None, None


def path_quantities(scene, tx, rx, eps, order, faces, freq_hz=28e9, tx_power_dbm=0.0):
    """Differentiable values[P, 8]; tx/rx [P, 3] (or tx [3], broadcast),
    eps [M, 2], order int32 [P], faces int32 [P, 8], all on the device."""
    if tx.dim() == 1:
        tx = tx.expand(rx.shape[0], 3)
    return PathQuantities.apply(tx, rx, eps, scene, order, faces, float(freq_hz),
                                float(tx_power_dbm))


def path_tensors(paths, rx_all, device="cuda"):
    """(rx[P, 3], order[P], faces[P, 8]) tensors for the paths sbr_trace
    returned (rx_all: the receivers of that call)."""
    rxp = torch.as_tensor(np.asarray(rx_all, np.float64)[paths["rx"]], device=device)
    order = torch.as_tensor(paths["order"].astype(np.int32), device=device)
    faces = torch.as_tensor(np.ascontiguousarray(paths["face"], np.int32), device=device)
    return rxp, order, faces


def fit_permittivity(scene, tx, rx, order, faces, target_dbm, eps0, steps=400, lr=0.05,
                     freq_hz=28e9, tx_power_dbm=0.0):
    """Adam fit (cosine-annealed step size) of the materials' permittivities
    eps[M, 2] so that the path powers (the power delay profile; delays do not
    depend on eps) match target_dbm[P].  Returns (eps, losses)."""
    eps = eps0.clone().detach().requires_grad_(True)
    opt = torch.optim.Adam([eps], lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=steps)
    losses = []
    for _ in range(steps):
        opt.zero_grad()
        val = path_quantities(scene, tx, rx, eps, order, faces, freq_hz, tx_power_dbm)
        loss = torch.mean((val[:, 7] - target_dbm) ** 2)
        loss.backward()
        opt.step()
        sched.step()
        losses.append(float(loss.detach()))
    return eps.detach(), losses
