"""Shared helpers for the GPU parity tests (device buffers via PyTorch, oracle side in float64)."""
from __future__ import annotations

import numpy as np

from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth


def geometry(m):
    """Oracle geometry for a library material descriptor (independent implementation)."""
    act = "relu" if m.activation == 0 else "hardgelu"
    pe = "sincos" if m.posenc == 0 else "triangle"
    return O.make_geometry(m.width, m.height, m.channels, m.c0, m.c1, m.b0, m.b1, Hd=m.hidden, M=m.num_mips,
                           shift=m.grid_shift, act=act, pe=pe, lod_input=bool(m.lod_input))


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def queries_dev(q):
    import torch
    raw = np.ascontiguousarray(q).view(np.uint8)
    return torch.from_numpy(raw.copy()).cuda()


def quantized_latents_oracle(g, raw):
    """Oracle-side initial latents: raw values quantized and dequantized (float64)."""
    return O.dequantize_packed(g, O.quantize_latents(g, raw))


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def mlp_in_unit_range(seed, K, Hd, C):
    """Xavier weights with a damped output layer and b3 = 0.5, so outputs sit near [0, 1]."""
    p = synth.xavier_mlp(seed, K, Hd, C).astype(np.float64)
    w3 = K * Hd + Hd + Hd * Hd + Hd
    p[w3:w3 + Hd * C] *= 0.25
    p[w3 + Hd * C:] = 0.5
    return p.astype(np.float32)
