"""Python front end of the equivalent-charge FMM library.

torch supplies device memory and streams; every step of the method runs in
libeqfmm.so.  `energy(pos, q, plan)` is a torch.autograd.Function whose
backward is the library's adjoint kernel (dE/dx and dE/dq).
"""
from __future__ import annotations

import torch

from . import native
from .native import (FP32, FP32_BF16FAR, FP64, FREE, FREE_CONTINUOUS, PERIODIC,  # noqa: F401
                     PERIODIC_CONTINUOUS)


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class Plan:
    """Operators of one (levels, order, boundary, precision, box) setting,
    uploaded to the current device."""

    def __init__(self, levels, order, boundary=FREE, precision=FP32, box=1.0,
                 origin=(0.0, 0.0, 0.0), split_d=0.0, node_shrink=0.0, max_fragments=0,
                 device="cuda"):
        p = native.Params()
        p.levels, p.order, p.boundary, p.precision = levels, order, boundary, precision
        p.origin = (native.ctypes.c_double * 3)(*origin)
        p.box, p.split_d, p.node_shrink, p.max_fragments = box, split_d, node_shrink, max_fragments
        self.params = p
        self.levels, self.order, self.boundary, self.precision = levels, order, boundary, precision
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.handle = native.eqfmm_plan_create(p)
        nbytes = native.eqfmm_plan_device_bytes(self.handle)
        self._dev = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        native.eqfmm_plan_upload(self.handle, self._dev.data_ptr(), nbytes, _stream())
        self._ws = {}
        self.dtype = torch.float64 if precision == FP64 else torch.float32

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                native.eqfmm_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def workspace_bytes(self, n):
        return native.eqfmm_workspace_bytes(self.handle, n)

    def workspace(self, n):
        ws = self._ws.get(n)
        if ws is None:
            self._ws.clear()
            ws = torch.empty(max(self.workspace_bytes(n), 256), dtype=torch.uint8, device=self.device)
            self._ws[n] = ws
        return ws

    # raw calls ------------------------------------------------------------
    def forward(self, pos, q, want_phi=True, want_field=True, ws=None, status=None):
        """E, phi, field of the charges.  With `status` (a device int32
        tensor of one element) the call does not wait for the GPU: the
        data-dependent status code lands in `status` (see `check_status`)."""
        pos = pos.detach().to(self.device, torch.float64).contiguous()
        q = q.detach().to(self.device, torch.float64).contiguous()
        n = q.numel()
        if pos.shape != (n, 3):
            raise ValueError("pos must be [n, 3]")
        ws = self.workspace(n) if ws is None else ws
        phi = torch.empty(n, dtype=self.dtype, device=self.device) if want_phi else None
        field = torch.empty((n, 3), dtype=self.dtype, device=self.device) if want_field else None
        E = torch.empty((), dtype=torch.float64, device=self.device)
        if status is None:
            native.eqfmm_forward(self.handle, n, pos.data_ptr(), q.data_ptr(), _ptr(phi), _ptr(field),
                                 E.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        else:
            if status.dtype != torch.int32 or status.numel() != 1 or status.device != self.device:
                raise ValueError("status must be one int32 on the plan's device")
            native.eqfmm_forward_async(self.handle, n, pos.data_ptr(), q.data_ptr(), _ptr(phi), _ptr(field),
                                       E.data_ptr(), status.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
        return E, phi, field

    @staticmethod
    def check_status(status):
        """Raise EqfmmError if the status word of an asynchronous forward
        holds an error (synchronises with it)."""
        code = int(status.item())
        if code != 0:
            raise native.EqfmmError(code, "eqfmm_forward_async")

    def backward(self, q, grad_E, ws=None, want_dx=True, want_dq=True):
        q = q.detach().to(self.device, torch.float64).contiguous()
        n = q.numel()
        ws = self.workspace(n) if ws is None else ws
        g = grad_E.detach().to(self.device, torch.float64).reshape(()).contiguous()
        dx = torch.empty((n, 3), dtype=self.dtype, device=self.device) if want_dx else None
        dq = torch.empty(n, dtype=self.dtype, device=self.device) if want_dq else None
        native.eqfmm_backward(self.handle, n, q.data_ptr(), g.data_ptr(), _ptr(dx), _ptr(dq),
                              ws.data_ptr(), ws.numel(), _stream())
        return dx, dq

    # profiling ------------------------------------------------------------
    def profile(self, stages=True):
        """Time stages with HIP events: True for every stage, False for none,
        or an iterable of stage names (native.STAGES).  Each timed launch
        costs an event pair, so time only the stages that are read."""
        if stages is True:
            mask = (1 << len(native.STAGES)) - 1
        elif not stages:
            mask = 0
        else:
            mask = 0
            for s in stages:
                mask |= 1 << native.STAGES.index(s)
        native.eqfmm_profile_enable(self.handle, mask)

    def profile_read(self):
        return {name: native.eqfmm_profile_read(self.handle, i) for i, name in enumerate(native.STAGES)}


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, plan):
        ws = torch.empty(max(plan.workspace_bytes(q.numel()), 256), dtype=torch.uint8, device=plan.device)
        E, phi, field = plan.forward(pos, q, ws=ws)
        ctx.plan, ctx.ws = plan, ws
        ctx.save_for_backward(pos, q)
        # In free space phi is linear in q with a symmetric matrix (the
        # method's pair terms are symmetric, Sec. 2.2), so its vector-Jacobian
        # product in q is phi of the upstream gradient taken as charges.  The
        # periodic modes' shape terms are not symmetric: phi stays constant
        # there, as does the field everywhere.
        if plan.boundary in (FREE, FREE_CONTINUOUS):
            ctx.mark_non_differentiable(field)
        else:
            ctx.mark_non_differentiable(phi, field)
        ctx.set_materialize_grads(False)
        ctx.pos_dtype, ctx.q_dtype = pos.dtype, q.dtype
        return E, phi, field

    @staticmethod
    def backward(ctx, gE, gphi, gfield):
        pos, q = ctx.saved_tensors
        dx = dq = None
        if gE is not None:
            dx, dq = ctx.plan.backward(q, gE, ws=ctx.ws, want_dx=ctx.needs_input_grad[0],
                                       want_dq=ctx.needs_input_grad[1])
        if gphi is not None:
            if ctx.needs_input_grad[0]:
                raise NotImplementedError("the gradient of phi with respect to the positions is not provided; "
                                          "only E is differentiable in the positions")
            if ctx.needs_input_grad[1]:
                # the plan's own workspace: ctx.ws keeps the forward's state
                _, vq, _ = ctx.plan.forward(pos, gphi, want_field=False)
                dq = vq if dq is None else dq + vq
        return (dx.to(ctx.pos_dtype) if dx is not None else None,
                dq.to(ctx.q_dtype) if dq is not None else None, None)


def energy(pos, q, plan):
    """(E, phi, field): E differentiable in pos and q; in the free modes phi
    differentiable in q (not in pos); field constant."""
    return _Energy.apply(pos, q, plan)
