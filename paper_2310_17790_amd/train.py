"""Field fitting with the hand-written HIP backward (torch.autograd.Function).

FieldFn.apply(X, z_rows, weights, width, d, precision) evaluates one field MLP at the
points X (n, 3) with per-point latents z_rows (n, r) and flat weights (layout of
nsf_sim_desc.weights) and returns (n, d). Its backward calls nsf_mlp_backward, which
returns dLoss/dweights (same flat layout), dLoss/dz_rows and, when X requires it,
dLoss/dX.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _abi as A


def _mlp(weights: torch.Tensor, r: int, width: int, d: int, precision: str) -> A.nsf_mlp:
    m = A.nsf_mlp()
    m.r, m.width, m.d = r, width, d
    m.precision = A.NSF_BF16 if precision == "bf16" else A.NSF_FP32
    m.weights = weights.data_ptr()
    return m


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


class FieldFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, z_rows, weights, width: int, d: int, precision: str = "fp32"):
        n, r = z_rows.shape
        assert X.shape == (n, 3) and X.dtype == torch.float32 and z_rows.dtype == torch.float32
        assert weights.numel() == A.lib().nsf_mlp_param_count(r, width, d)
        L = A.lib()
        Xs = X.t().contiguous()
        zr = z_rows.contiguous()
        w = weights.contiguous()
        m = _mlp(w, r, width, d, precision)
        out = torch.empty((d, n), dtype=torch.float32, device=X.device)
        saved = torch.empty(L.nsf_mlp_saved_floats(width, n), dtype=torch.float32, device=X.device)
        ws_bytes = L.nsf_mlp_workspace_bytes(C.byref(m), n)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
        A.check(L.nsf_mlp_forward(C.byref(m), Xs.data_ptr(), zr.data_ptr(), n, out.data_ptr(),
                                  saved.data_ptr(), ws.data_ptr(), ws_bytes, _stream()))
        ctx.save_for_backward(Xs, zr, w, saved)
        ctx.cfg = (width, d, precision)
        return out.t()

    @staticmethod
    def backward(ctx, gout):
        Xs, zr, w, saved = ctx.saved_tensors
        width, d, precision = ctx.cfg
        n, r = zr.shape
        L = A.lib()
        m = _mlp(w, r, width, d, precision)
        dout = gout.t().contiguous().float()
        dW = torch.zeros_like(w)
        dz = torch.empty_like(zr) if ctx.needs_input_grad[1] else None
        dX = torch.empty_like(Xs) if ctx.needs_input_grad[0] else None
        ws_bytes = L.nsf_mlp_workspace_bytes(C.byref(m), n)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=w.device)
        A.check(L.nsf_mlp_backward(C.byref(m), Xs.data_ptr(), zr.data_ptr(), n, saved.data_ptr(),
                                   dout.data_ptr(), dW.data_ptr(), None if dz is None else dz.data_ptr(),
                                   None if dX is None else dX.data_ptr(), ws.data_ptr(), ws_bytes,
                                   _stream()))
        return None if dX is None else dX.t(), dz, dW, None, None, None


class PairSquaredError(torch.autograd.Function):
    """PairSquaredError.apply(out_t, Y, rows, cols, P) = mean((out_t.t() - y)^2) with
    y[c][i] = Y[c][rows[i] P + cols[i]]: the minibatch's targets gathered, the loss and its
    gradient formed by nsf_squared_error in one pass (the loss summed in FP64 in a fixed
    order); out_t is the (n, d) view FieldFn returns."""

    @staticmethod
    def forward(ctx, out_t, Y, rows, cols, P: int):
        out = out_t.t()
        if not out.is_contiguous():
            out = out.contiguous()
        d, n = out.shape
        assert Y.dtype == torch.float32 and Y.is_contiguous() and Y.shape[0] == d
        assert rows.dtype == torch.int64 and cols.dtype == torch.int64 and rows.numel() == n == cols.numel()
        grad = torch.empty_like(out)
        loss = torch.empty((), dtype=torch.float32, device=out.device)
        ws = torch.empty(A.NSF_SQERR_WORKSPACE_BYTES, dtype=torch.uint8, device=out.device)
        A.check(A.lib().nsf_squared_error(out.data_ptr(), d, n, Y.data_ptr(), Y.shape[1], rows.data_ptr(),
                                          cols.data_ptr(), int(P), loss.data_ptr(), grad.data_ptr(),
                                          ws.data_ptr(), _stream()))
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (grad * g).t(), None, None, None, None


class RowsExpand(torch.autograd.Function):
    """RowsExpand.apply(table, offsets, n) -> (n, width): row i is table[s] for
    offsets[s] <= i < offsets[s + 1] (nsf_rows_expand); the backward sums each segment's
    gradient rows into the table's gradient (nsf_rows_segment_sum, fixed order)."""

    @staticmethod
    def forward(ctx, table, offsets, n: int):
        segments, width = table.shape
        assert table.dtype == torch.float32 and offsets.dtype == torch.int64 and offsets.numel() == segments + 1
        t = table.contiguous()
        out = torch.empty((n, width), dtype=torch.float32, device=table.device)
        A.check(A.lib().nsf_rows_expand(t.data_ptr(), offsets.data_ptr(), segments, width, out.data_ptr(), _stream()))
        ctx.save_for_backward(offsets)
        ctx.shape = (segments, width)
        return out

    @staticmethod
    def backward(ctx, gout):
        (offsets,) = ctx.saved_tensors
        segments, width = ctx.shape
        g = gout.contiguous().float()
        out = torch.empty((segments, width), dtype=torch.float32, device=g.device)
        A.check(A.lib().nsf_rows_segment_sum(g.data_ptr(), offsets.data_ptr(), segments, width, out.data_ptr(),
                                             _stream()))
        return out, None, None


class Adam:
    """Adam on FP32 device tensors through nsf_adam_step (PyTorch's update order, no weight
    decay); lr may change between steps."""

    def __init__(self, params, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8):
        self.params = list(params)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def zero_grad(self) -> None:
        for p in self.params:
            p.grad = None

    @torch.no_grad()
    def step(self) -> None:
        self.t += 1
        for p, m, v in zip(self.params, self.m, self.v):
            if p.grad is None:
                continue
            assert p.dtype == torch.float32 and p.is_contiguous() and p.grad.is_contiguous()
            A.check(A.lib().nsf_adam_step(p.data_ptr(), p.grad.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(),
                                          self.lr, self.betas[0], self.betas[1], self.eps, self.t, _stream()))
