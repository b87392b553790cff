"""Seeded synthetic inputs: target texture sets, initial latents and weights, queries.

These generators feed both the HIP library and the CPU checker.  They hold none of
the compression method's arithmetic (no sampling, quantization or network math):
only random numbers, value-noise images standing in for the paper's material
texture sets, and a box-filtered mip chain of those images.

All randomness comes from numpy's PCG64 seeded by explicit integer tuples.
"""
from __future__ import annotations

import numpy as np

QUERY_DTYPE = np.dtype([("u", "<f4"), ("v", "<f4"), ("lod", "<i4")])


def _rng(*key):
    return np.random.Generator(np.random.PCG64(list(int(k) for k in key)))


def value_noise(seed: int, material: int, W: int, H: int, C: int, octaves: int = 4):
    """H x W x C float32 image in [0, 1]: per channel a normalised sum over octaves o of
    0.5^o * V_o, where V_o is smoothstep-interpolated periodic lattice noise with
    8 * 2^o cells per side and lattice values drawn uniformly in [0, 1)."""
    out = np.zeros((H, W, C), dtype=np.float32)
    norm = sum(0.5 ** o for o in range(octaves))
    ys = (np.arange(H, dtype=np.float64) + 0.5) / H
    xs = (np.arange(W, dtype=np.float64) + 0.5) / W
    for c in range(C):
        acc = np.zeros((H, W), dtype=np.float64)
        for o in range(octaves):
            cells = 8 * 2 ** o
            lat = _rng(seed, material, c, o).random((cells, cells))
            gx = xs * cells
            gy = ys * cells
            x0 = np.floor(gx).astype(np.int64)
            y0 = np.floor(gy).astype(np.int64)
            tx = gx - x0
            ty = gy - y0
            sx = tx * tx * (3.0 - 2.0 * tx)
            sy = ty * ty * (3.0 - 2.0 * ty)
            x0 %= cells
            y0 %= cells
            x1 = (x0 + 1) % cells
            y1 = (y0 + 1) % cells
            a = lat[y0[:, None], x0[None, :]]
            b = lat[y0[:, None], x1[None, :]]
            cc = lat[y1[:, None], x0[None, :]]
            d = lat[y1[:, None], x1[None, :]]
            top = a + (b - a) * sx[None, :]
            bot = cc + (d - cc) * sx[None, :]
            acc += 0.5 ** o * (top + (bot - top) * sy[:, None])
        out[:, :, c] = (acc / norm).astype(np.float32)
    return out


def value_noise_torch(seed: int, material: int, W: int, H: int, C: int, device, octaves: int = 4):
    """value_noise() evaluated with torch on `device` (same lattice values, same float64
    operation sequence), for sizes where the numpy version is slow."""
    import torch
    norm = sum(0.5 ** o for o in range(octaves))
    ys = (torch.arange(H, dtype=torch.float64, device=device) + 0.5) / H
    xs = (torch.arange(W, dtype=torch.float64, device=device) + 0.5) / W
    out = torch.empty((H, W, C), dtype=torch.float32, device=device)
    for c in range(C):
        acc = torch.zeros((H, W), dtype=torch.float64, device=device)
        for o in range(octaves):
            cells = 8 * 2 ** o
            lat = torch.from_numpy(_rng(seed, material, c, o).random((cells, cells))).to(device)
            gx, gy = xs * cells, ys * cells
            x0, y0 = torch.floor(gx), torch.floor(gy)
            tx, ty = gx - x0, gy - y0
            sx = tx * tx * (3.0 - 2.0 * tx)
            sy = ty * ty * (3.0 - 2.0 * ty)
            x0 = x0.long() % cells
            y0 = y0.long() % cells
            x1, y1 = (x0 + 1) % cells, (y0 + 1) % cells
            a = lat[y0[:, None], x0[None, :]]
            b = lat[y0[:, None], x1[None, :]]
            cc = lat[y1[:, None], x0[None, :]]
            d = lat[y1[:, None], x1[None, :]]
            top = a + (b - a) * sx[None, :]
            bot = cc + (d - cc) * sx[None, :]
            acc += 0.5 ** o * (top + (bot - top) * sy[:, None])
        out[:, :, c] = (acc / norm).to(torch.float32)
    return out


def target_chain_torch(seed: int, material: int, W: int, H: int, C: int, num_mips: int, device):
    """target_chain() on a torch device: flat float32 tensor, mip 0 first."""
    import torch
    img = value_noise_torch(seed, material, W, H, C, device)
    mips = [img]
    for _ in range(1, num_mips):
        m = mips[-1].double()
        h, w = m.shape[0], m.shape[1]
        h2, w2 = max(1, h // 2), max(1, w // 2)
        if h == 1:
            m = torch.cat([m, m], dim=0)
        if w == 1:
            m = torch.cat([m, m], dim=1)
        m = 0.25 * (m[0::2, 0::2] + m[1::2, 0::2] + m[0::2, 1::2] + m[1::2, 1::2])
        mips.append(m[:h2, :w2].to(torch.float32).contiguous())
    return torch.cat([m.reshape(-1) for m in mips])


def box_mips(img: np.ndarray, num_mips: int):
    """Mip chain by 2x2 box averaging (float32), down to num_mips levels."""
    mips = [np.ascontiguousarray(img, dtype=np.float32)]
    for _ in range(1, num_mips):
        m = mips[-1].astype(np.float64)
        h, w = m.shape[0], m.shape[1]
        h2, w2 = max(1, h // 2), max(1, w // 2)
        if h == 1:
            m = np.concatenate([m, m], axis=0)
        if w == 1:
            m = np.concatenate([m, m], axis=1)
        m = 0.25 * (m[0::2, 0::2] + m[1::2, 0::2] + m[0::2, 1::2] + m[1::2, 1::2])
        mips.append(m[:h2, :w2].astype(np.float32))
    return mips


def target_chain(seed: int, material: int, W: int, H: int, C: int, num_mips: int):
    """(list of mips, flat float32 concatenation mip 0 first, each [y][x][c])."""
    mips = box_mips(value_noise(seed, material, W, H, C), num_mips)
    return mips, np.concatenate([m.ravel() for m in mips]).astype(np.float32)


def uniform_latents(seed: int, count: int, lo: float = -1.0, hi: float = 1.0):
    return _rng(seed, 101).uniform(lo, hi, count).astype(np.float32)


def xavier_mlp(seed: int, K: int, Hd: int, C: int):
    """Flat float32 parameters in the order W1[K][Hd], b1, W2[Hd][Hd], b2, W3[Hd][C], b3:
    Xavier-uniform weights +-sqrt(6/(fan_in+fan_out)), zero biases."""
    r = _rng(seed, 202)
    parts = []
    for fi, fo in ((K, Hd), (Hd, Hd), (Hd, C)):
        a = np.sqrt(6.0 / (fi + fo))
        parts.append(r.uniform(-a, a, fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def random_queries(seed: int, n: int, num_mips: int, lod: int | None = None):
    """n queries with u, v ~ U[0, 1) and lod uniform over the mips (or fixed)."""
    r = _rng(seed, 303)
    q = np.zeros(n, dtype=QUERY_DTYPE)
    q["u"] = r.random(n, dtype=np.float32)
    q["v"] = r.random(n, dtype=np.float32)
    q["lod"] = lod if lod is not None else r.integers(0, num_mips, n)
    return q


def tile_queries(W: int, H: int, lod: int = 0, x0: int = 0, y0: int = 0, tw=None, th=None):
    """Queries at every texel centre of a rectangle of mip `lod` (row-major)."""
    Wl, Hl = max(1, W >> lod), max(1, H >> lod)
    tw = Wl if tw is None else tw
    th = Hl if th is None else th
    ys, xs = np.meshgrid(np.arange(y0, y0 + th), np.arange(x0, x0 + tw), indexing="ij")
    q = np.zeros(tw * th, dtype=QUERY_DTYPE)
    q["u"] = ((xs.ravel() + 0.5) / Wl).astype(np.float32)
    q["v"] = ((ys.ravel() + 0.5) / Hl).astype(np.float32)
    q["lod"] = lod
    return q


def random_param_indices(seed: int, count: int, total: int):
    return _rng(seed, 404).choice(total, size=count, replace=False)
