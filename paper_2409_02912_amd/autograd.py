"""torch.autograd view of the NRX: LLRs as a differentiable function of the weights.

The forward runs nrx_forward keeping the activations in the workspace; the backward
runs the hand-written backward kernels (nrx_backward) on the gradient of the LLRs and
returns the gradient of the flat fp32 weight vector (Sec. II-B: the receiver is trained
end to end on the BCE of the coded bits).  The received grid is an input, not a
parameter, so it gets no gradient.

All calls of one Nrx share its workspace, which holds the activations of the last
forward only: each forward records the library's sequence token and its backward
checks it (nrx_check_token), so a backward whose activations were overwritten by a
later forward raises instead of returning a wrong gradient.
"""
import torch

from . import libnrx as L


class NrxFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w, y, model, slots, ws, n_llr):
        llr = torch.empty(n_llr, dtype=torch.float32, device=w.device)
        L.nrx_forward(model, w, slots, y, llr, ws, save_acts=True)
        ctx.model, ctx.slots, ctx.ws = model, slots, ws
        ctx.token = L.nrx_saved_token(model)
        ctx.save_for_backward(w)
        return llr

    @staticmethod
    def backward(ctx, dllr):
        (w,) = ctx.saved_tensors
        L.nrx_check_token(ctx.model, ctx.ws, ctx.token)
        dw = torch.empty_like(w)
        L.nrx_backward(ctx.model, w, ctx.slots, dllr.contiguous(), dw, ctx.ws)
        return dw, None, None, None, None, None


class Nrx:
    """Owns a model handle and a training workspace for one batch shape.

    nrx = Nrx(n_ant, d, n_blocks, n_rounds, m_max, precision, shapes)
    llr = nrx(w, y)            # differentiable in w
    """

    def __init__(self, n_ant, d, n_blocks, n_rounds, m_max, precision, shapes, device="cuda"):
        self.model = L.nrx_model_create(n_ant, d, n_blocks, n_rounds, m_max, precision)
        self.slots, self.sizes = L.make_slots(shapes, m_max)
        self.ws = torch.empty(L.nrx_workspace_bytes(self.model, self.slots, save_acts=True), dtype=torch.uint8,
                              device=device)

    def __call__(self, w, y):
        return NrxFunction.apply(w, y, self.model, self.slots, self.ws, self.sizes["llr"])

    def close(self):
        if self.model is not None:
            L.nrx_model_destroy(self.model)
            self.model = None
