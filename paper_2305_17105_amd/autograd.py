"""torch.autograd.Function over the library's forward and backward kernels.

    y = ntc_decode_fn(material, latents, mlp, queries, precision)

latents (latent_count,) and mlp (mlp_params,) are FP32 CUDA tensors; queries is a
uint8 CUDA tensor holding n 12-byte ntc_query records.  Gradients flow to latents
and mlp; the backward recomputes the forward per tile in the HIP kernels.  One
training pack of the weights serves both directions.
"""
from __future__ import annotations

import torch

from . import ntc

# dout_scale 0: the library scales dL/dy by the power of two that brings its largest
# magnitude near 1/4 (FP16 range), chosen on the device, so the backward does not
# synchronise with the host and can be captured in a graph.
AUTO_SCALE = 0.0


class NtcDecodeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, latents, mlp, queries, material, precision):
        n = queries.numel() // 12
        C = int(material.channels)
        tp = torch.empty(ntc.train_packed_bytes(material, precision), dtype=torch.uint8, device=latents.device)
        ntc.pack_mlp_train(material, mlp, precision, tp)
        out = torch.empty(n * C, dtype=torch.float32, device=latents.device)
        ntc.forward(material, latents, mlp, tp, precision, queries, n, out)
        ctx.save_for_backward(latents, mlp, queries, tp)
        ctx.material, ctx.precision = material, precision
        return out.view(n, C)

    @staticmethod
    def backward(ctx, dout):
        latents, mlp, queries, tp = ctx.saved_tensors
        m, prec = ctx.material, ctx.precision
        n = queries.numel() // 12
        dout = dout.contiguous().float()
        gl = torch.empty_like(latents)
        gm = torch.empty_like(mlp)
        ws = torch.empty(ntc.backward_workspace_bytes(m, n, prec), dtype=torch.uint8, device=latents.device)
        ntc.backward(m, latents, mlp, tp, prec, queries, n, dout, AUTO_SCALE, gl, gm, ws)
        return gl, gm, None, None, None


def ntc_decode_fn(material, latents, mlp, queries, precision=ntc.F32):
    return NtcDecodeFn.apply(latents, mlp, queries, material, precision)
