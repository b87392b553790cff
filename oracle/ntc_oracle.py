"""Plain float64 oracle of the neural texture compression hot path.

TEST INFRASTRUCTURE: imported only by tests/, the smoke check and the benchmark's
CPU-baseline leg.  Nothing here is called by the HIP library.

Notation follows the paper (arXiv 2305.17105, section 4):
  texture set W x H x C with mips l = 0..M-1, feature levels F^j = (G0^j, G1^j),
  latent channels C0, C1, bits B0, B1, N = 2^B quantization levels, Q = 1/N,
  MLP  K -> Hd -> Hd -> C  with K = 4*C0 + C1 + 12 (+ 1 with the LOD input).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Geometry", "make_geometry", "quant_range", "quantize_codes", "dequantize_codes",
    "pack_codes", "unpack_codes", "quantize_latents", "dequantize_packed",
    "splitmix64_mix", "noise_values", "pos_enc", "sample_inputs", "mlp_split",
    "mlp_param_count", "activation", "activation_grad", "mlp_forward", "decode",
    "loss_and_grads", "adam_update", "train_step", "loss_scale_update", "psnr",
    "storage_bytes_paper", "hard_gelu", "E4M3_MAX", "e4m3_value", "round_e4m3", "fp8_layer_scales",
    "mlp_forward_fp8", "decode_fp8", "crop_lod", "crop_queries", "FILTER_BILINEAR", "FILTER_TRILINEAR",
    "FILTER_STOCHASTIC", "FILTER_QUERY", "filter_randoms", "filter_taps", "decode_filtered",
]

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------------------
# Geometry: section 4.1 (feature pyramid) and Table 1.
# --------------------------------------------------------------------------------------
@dataclass
class Geometry:
    W: int
    H: int
    C: int
    M: int            # number of mips
    C0: int
    C1: int
    B0: int
    B1: int
    shift: int        # log2(W / width of G0 at level 0); 2 in Table 1, 1 for NTC 1.0/2.25
    Hd: int
    act: str = "relu"
    pe: str = "sincos"
    lod_input: bool = False
    J: int = 0
    mip_w: list = field(default_factory=list)
    mip_h: list = field(default_factory=list)
    g0: list = field(default_factory=list)      # (w, h) per level
    g1: list = field(default_factory=list)
    level_of_mip: list = field(default_factory=list)
    g0_off: list = field(default_factory=list)  # float offsets in the canonical latent buffer
    g1_off: list = field(default_factory=list)
    latent_count: int = 0
    K: int = 0
    mip_off: list = field(default_factory=list)  # float offsets of each mip in the target chain
    target_count: int = 0


def make_geometry(W, H, C, C0, C1, B0, B1, Hd=64, M=None, shift=2, act="relu", pe="sincos",
                  lod_input=False) -> Geometry:
    """Feature-pyramid geometry (section 4.1, Table 1).

    Level j holds G0^j at (W, H) >> (shift + 2j) and G1^j at half that.  Levels are
    added while G1 keeps at least one cell.  Mip l is predicted by level
    clamp(floor((l - shift) / 2), 0, J - 1): with shift = 2 this is Table 1's
    assignment (mips 0-3 -> F0, 4-5 -> F1, 6-7 -> F2, last level takes the rest).
    Only as many levels as the mip chain reaches are kept.
    """
    for v in (W, H):
        if v < 1 or v & (v - 1):
            raise ValueError("texture sides must be powers of two")
    full = int(math.log2(max(W, H))) + 1
    M = full if M is None else M
    if not 1 <= M <= full:
        raise ValueError("bad mip count")
    g = Geometry(W, H, C, M, C0, C1, B0, B1, shift, Hd, act, pe, bool(lod_input))
    jmax = 0
    while (W >> (shift + 2 * jmax + 1)) >= 1 and (H >> (shift + 2 * jmax + 1)) >= 1:
        jmax += 1
    if jmax == 0:
        raise ValueError("texture too small for the grid ratio")
    raw_last = max(0, (M - 1 - shift) // 2)
    g.J = min(jmax, raw_last + 1)
    g.mip_w = [max(1, W >> l) for l in range(M)]
    g.mip_h = [max(1, H >> l) for l in range(M)]
    g.level_of_mip = [min(max((l - shift) // 2, 0), g.J - 1) for l in range(M)]
    off = 0
    for j in range(g.J):
        w0, h0 = W >> (shift + 2 * j), H >> (shift + 2 * j)
        w1, h1 = w0 // 2, h0 // 2
        g.g0.append((w0, h0))
        g.g1.append((w1, h1))
        g.g0_off.append(off)
        off += w0 * h0 * C0
        g.g1_off.append(off)
        off += w1 * h1 * C1
    g.latent_count = off
    # section 4.4: 4 C0 + C1 + 12 inputs and, as the paper's network has it, a LOD value
    g.K = 4 * C0 + C1 + 12 + (1 if lod_input else 0)
    toff = 0
    for l in range(M):
        g.mip_off.append(toff)
        toff += g.mip_w[l] * g.mip_h[l] * C
    g.target_count = toff
    return g


def storage_bytes_paper(W, H, C0, C1, B0, B1, shift, levels=None):
    """Grid storage in bytes per Appendix 'Storage Cost' (Table 6): each grid costs
    w*h*C*B/8 bytes, independent of the texture channel count.  levels=None counts
    every level the pyramid has; levels=1 counts level 0 only."""
    total = 0
    j = 0
    while (W >> (shift + 2 * j + 1)) >= 1 and (H >> (shift + 2 * j + 1)) >= 1:
        if levels is not None and j >= levels:
            break
        w0, h0 = W >> (shift + 2 * j), H >> (shift + 2 * j)
        total += w0 * h0 * C0 * B0 / 8 + (w0 // 2) * (h0 // 2) * C1 * B1 / 8
        j += 1
    return total


# --------------------------------------------------------------------------------------
# Quantization: section 4.2.
# --------------------------------------------------------------------------------------
def quant_range(B):
    """Asymmetric range [-(N-1)Q/2, N Q/2] with N = 2^B, Q = 1/N (section 4.2)."""
    N = 2 ** B
    Q = 1.0 / N
    return -(N - 1) * Q / 2.0, N * Q / 2.0


def quantize_codes(x, B):
    """Fixed-rate scalar quantizer of section 4.2.

    Values sit on the grid k*Q, k = -(N/2-1) .. N/2 (zero is a bin centre, so it is
    exact).  Reading taken: round x*N to nearest, ties to even, then clamp to the
    N levels; stored code = k + N/2 - 1 in [0, N).  x*N is exact (N is a power of
    two).  Non-finite inputs map to the code of zero.
    """
    N = 2 ** B
    x = np.asarray(x, dtype=np.float64)
    finite = np.isfinite(x)
    k = np.rint(np.where(finite, x, 0.0) * N)
    k = np.clip(k, -(N // 2) + 1, N // 2)
    return (k + (N // 2 - 1)).astype(np.int64)


def dequantize_codes(codes, B):
    """Code k -> (k - (N/2 - 1)) / N (section 4.2)."""
    N = 2 ** B
    return (np.asarray(codes, dtype=np.float64) - (N // 2 - 1)) / N


def pack_codes(codes, B):
    """Dense LSB-first bitstream of B-bit codes in the given (cell-major, channel-minor)
    order, zero-padded to a multiple of 16 bytes.  The byte count before padding is
    the paper's w*h*C*B/8 (Appendix 'Storage Cost')."""
    codes = np.asarray(codes, dtype=np.int64).ravel()
    bits = ((codes[:, None] >> np.arange(B)[None, :]) & 1).astype(np.uint8).ravel()
    raw = np.packbits(bits, bitorder="little")
    padded = -(-len(raw) // 16) * 16
    out = np.zeros(padded, dtype=np.uint8)
    out[: len(raw)] = raw
    return out


def unpack_codes(buf, B, count):
    bits = np.unpackbits(np.asarray(buf, dtype=np.uint8), bitorder="little")[: count * B]
    bits = bits.reshape(count, B).astype(np.int64)
    return (bits << np.arange(B)[None, :]).sum(axis=1)


def _grids(geom: Geometry):
    """(offset, w, h, channels, bits) for every grid in canonical order."""
    out = []
    for j in range(geom.J):
        out.append((geom.g0_off[j],) + geom.g0[j] + (geom.C0, geom.B0))
        out.append((geom.g1_off[j],) + geom.g1[j] + (geom.C1, geom.B1))
    return out


def quantize_latents(geom: Geometry, latents):
    """Whole latent buffer -> concatenated packed grids (each padded to 16 bytes)."""
    parts = []
    for off, w, h, c, b in _grids(geom):
        parts.append(pack_codes(quantize_codes(latents[off: off + w * h * c], b), b))
    return np.concatenate(parts)


def dequantize_packed(geom: Geometry, packed):
    out = np.zeros(geom.latent_count, dtype=np.float64)
    pos = 0
    for off, w, h, c, b in _grids(geom):
        n = w * h * c
        raw = -(-(n * b) // 8)
        nbytes = -(-raw // 16) * 16
        out[off: off + n] = dequantize_codes(unpack_codes(packed[pos: pos + nbytes], b, n), b)
        pos += nbytes
    return out


def latent_bits(geom: Geometry):
    """Per-latent bit depth, canonical order."""
    bits = np.zeros(geom.latent_count, dtype=np.int64)
    for off, w, h, c, b in _grids(geom):
        bits[off: off + w * h * c] = b
    return bits


# --------------------------------------------------------------------------------------
# Simulated quantization noise (section 4.2): U(-Q/2, Q/2) added to every latent.
# Reading taken: one draw per latent per step from a stateless counter hash, the
# SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
# --------------------------------------------------------------------------------------
def splitmix64_mix(z):
    """SplitMix64 output mixing function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def noise_values(geom: Geometry, seed: int, step: int):
    """nu_i = (r24 - 2^23) * 2^-24 * Q_i in [-Q/2, Q/2) for every latent i, where
    r24 = top 24 bits of mix(mix(seed + gamma*(step+1)) + gamma*(i+1))."""
    key = splitmix64_mix(np.uint64((seed + GAMMA * (step + 1)) & MASK64))
    idx = np.arange(geom.latent_count, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        r = splitmix64_mix(key + np.uint64(GAMMA) * idx)
    r24 = (r >> np.uint64(40)).astype(np.int64)
    q = 1.0 / (2.0 ** latent_bits(geom))
    return (r24 - 2 ** 23).astype(np.float64) * 2.0 ** -24 * q


# --------------------------------------------------------------------------------------
# Training batches (section 5.1): eight random 256 x 256 texel crops from one level of
# detail per batch; LOD = floor(-log4 X), X ~ U(0, 1], clamped to the chain, except for
# 5% of the batches, whose LOD is uniform over the chain.  Readings taken: the random
# numbers are SplitMix64 outputs of counters (key = mix(mix(seed ^ CROP_TAG) + gamma *
# (step + 1)), r_i = mix(key + gamma * (i + 1))); X = 1 - (r_0 >> 11) * 2^-53; the batch
# is uniform when (r_1 >> 11) * 2^-53 < fraction, its LOD then r_2 mod M; crop c has
# origin r_(3+2c) mod (W_l - s + 1), r_(4+2c) mod (H_l - s + 1) for a crop side s <= the
# mip side; on mips smaller than the crop, the crop starts at 0 and wraps around the
# mip (the mip is tiled).  Samples are crop-major, row-major within a crop, at texel
# centres.
# --------------------------------------------------------------------------------------
CROP_TAG = 0x63726F70


def crop_lod(X, M):
    """Largest k with X <= 4^-k (that is floor(-log4 X) for X in (0, 1]), at most M - 1;
    by comparisons with exact powers of four, no logarithm."""
    k = 0
    while k + 1 < M and X <= 4.0 ** -(k + 1):
        k += 1
    return k


def crop_queries(geom: Geometry, seed: int, step: int, crops: int = 8, side: int = 256, fraction: float = 0.05):
    """Query records of one training batch (QUERY layout: u, v float32; lod int32)."""
    a = int(splitmix64_mix(np.uint64((seed ^ CROP_TAG) & MASK64)))
    key = int(splitmix64_mix(np.uint64((a + GAMMA * (step + 1)) & MASK64)))

    def r(i):
        return int(splitmix64_mix(np.uint64((key + GAMMA * (i + 1)) & MASK64)))

    X = 1.0 - (r(0) >> 11) * 2.0 ** -53
    if (r(1) >> 11) * 2.0 ** -53 < fraction:
        lod = r(2) % geom.M
    else:
        lod = crop_lod(X, geom.M)
    Wl, Hl = geom.mip_w[lod], geom.mip_h[lod]
    q = np.zeros(crops * side * side, dtype=[("u", "<f4"), ("v", "<f4"), ("lod", "<i4")])
    jj, ii = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    for c in range(crops):
        x0 = r(3 + 2 * c) % (Wl - side + 1) if Wl >= side else 0
        y0 = r(4 + 2 * c) % (Hl - side + 1) if Hl >= side else 0
        x = (x0 + ii.ravel()) % Wl
        y = (y0 + jj.ravel()) % Hl
        sl = slice(c * side * side, (c + 1) * side * side)
        q["u"][sl] = ((x + 0.5) / Wl).astype(np.float32)
        q["v"][sl] = ((y + 0.5) / Hl).astype(np.float32)
        q["lod"][sl] = lod
    return q


# --------------------------------------------------------------------------------------
# Sampling and concatenation: sections 4.3.1 (feature interpolation), 4.3.2 (positional
# encoding), Figure 4(c).
# --------------------------------------------------------------------------------------
def pos_enc(ix, iy, kind="sincos"):
    """Tiled positional encoding, section 4.3.2: log2(8) = 3 octaves, period 8x8
    texels, 6 values per axis.  Reading taken: a sine-like and a cosine-like wave at
    frequencies 1, 2, 4 per tile with texel-centre phase t = ((i mod 8) + 1/2) / 8; the
    last value per axis (the cosine-like wave at 4 cycles per tile) is identically zero
    at texel centres (the constant value of Figure 5).  kind "sincos": sin 2 pi f t and
    cos 2 pi f t; kind "triangle" (the paper's triangular waves): the piecewise-linear
    waves through the same zeros and extrema, 4 |frac(f t - 1/4) - 1/2| - 1 and
    4 |frac(f t) - 1/2| - 1."""
    cols = []
    for i in (ix, iy):
        t = ((np.asarray(i) % 8) + 0.5) / 8.0
        for f in (1, 2, 4):
            x = f * t
            if kind == "triangle":
                cols.append(4.0 * np.abs((x - 0.25) - np.floor(x - 0.25) - 0.5) - 1.0)
                cols.append(4.0 * np.abs(x - np.floor(x) - 0.5) - 1.0)
            else:
                cols.append(np.sin(2.0 * np.pi * x))
                cols.append(np.cos(2.0 * np.pi * x))
    return np.stack(cols, axis=-1)


def _snap(u, size):
    """Texel index of coordinate u in [0,1) on a mip of `size` texels (nearest texel,
    out-of-range and NaN clamp).  Computed in float32, as the query carries float32."""
    u = np.asarray(u, dtype=np.float32)
    s = np.float32(size)
    p = np.where(np.isnan(u), np.float32(0), u * s)
    i = np.floor(p)
    i = np.clip(i, 0, size - 1)
    return i.astype(np.int64)


def sample_inputs(geom: Geometry, lat, queries):
    """MLP input x (n x K) plus the gather record needed to scatter gradients.

    For query (u, v, lod): the texel (ix, iy) of mip l = clamp(lod, 0, M-1), its level j,
    then on G0^j the four cells around the texel centre (bilinear footprint, order
    (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1), edges clamped), concatenated
    unweighted (learned interpolation), and on G1^j the bilinear interpolation over
    the same footprint construction.  Texel centres are (i + 1/2)/size and grid cell
    centres sit at (k + 1/2)/grid, so bilinear reproduces grid values at cell centres.
    x = [G0 n0 | G0 n1 | G0 n2 | G0 n3 | G1 bilinear | PE (12)].
    """
    lat = np.asarray(lat, dtype=np.float64)
    u = queries["u"]
    v = queries["v"]
    lod = np.clip(queries["lod"].astype(np.int64), 0, geom.M - 1)
    n = len(u)
    x = np.zeros((n, geom.K), dtype=np.float64)
    rec = {
        "g0_idx": np.zeros((n, 4), dtype=np.int64),   # float offset of each G0 cell
        "g1_idx": np.zeros((n, 4), dtype=np.int64),
        "g1_w": np.zeros((n, 4), dtype=np.float64),
        "ix": np.zeros(n, dtype=np.int64), "iy": np.zeros(n, dtype=np.int64),
        "lod": lod,
    }
    C0, C1 = geom.C0, geom.C1
    for l in np.unique(lod):
        sel = np.nonzero(lod == l)[0]
        Wl, Hl = geom.mip_w[l], geom.mip_h[l]
        ix = _snap(u[sel], Wl)
        iy = _snap(v[sel], Hl)
        j = geom.level_of_mip[l]
        (w0, h0), (w1, h1) = geom.g0[j], geom.g1[j]
        cx = (ix + 0.5) / Wl
        cy = (iy + 0.5) / Hl
        # G0 footprint
        gx, gy = cx * w0 - 0.5, cy * h0 - 0.5
        x0, y0 = np.floor(gx).astype(np.int64), np.floor(gy).astype(np.int64)
        cells0 = []
        for dy in (0, 1):
            for dx in (0, 1):
                xx = np.clip(x0 + dx, 0, w0 - 1)
                yy = np.clip(y0 + dy, 0, h0 - 1)
                cells0.append(geom.g0_off[j] + (yy * w0 + xx) * C0)
        # G1 bilinear
        gx, gy = cx * w1 - 0.5, cy * h1 - 0.5
        x1, y1 = np.floor(gx).astype(np.int64), np.floor(gy).astype(np.int64)
        fx, fy = gx - x1, gy - y1
        cells1, wts = [], []
        for dy in (0, 1):
            for dx in (0, 1):
                xx = np.clip(x1 + dx, 0, w1 - 1)
                yy = np.clip(y1 + dy, 0, h1 - 1)
                cells1.append(geom.g1_off[j] + (yy * w1 + xx) * C1)
                wts.append((fx if dx else 1.0 - fx) * (fy if dy else 1.0 - fy))
        for k in range(4):
            x[sel, k * C0:(k + 1) * C0] = lat[cells0[k][:, None] + np.arange(C0)[None, :]]
            rec["g0_idx"][sel, k] = cells0[k]
            rec["g1_idx"][sel, k] = cells1[k]
            rec["g1_w"][sel, k] = wts[k]
        g1v = np.zeros((len(sel), C1))
        for k in range(4):
            g1v += wts[k][:, None] * lat[cells1[k][:, None] + np.arange(C1)[None, :]]
        x[sel, 4 * C0:4 * C0 + C1] = g1v
        x[sel, 4 * C0 + C1:4 * C0 + C1 + 12] = pos_enc(ix, iy, geom.pe)
        if geom.lod_input:  # the mip as a value in [0, 1] (reading: l / (M - 1))
            x[sel, -1] = l / (geom.M - 1) if geom.M > 1 else 0.0
        rec["ix"][sel] = ix
        rec["iy"][sel] = iy
    return x, rec


# --------------------------------------------------------------------------------------
# Network: section 4.4.  K -> Hd -> Hd -> C, activation on the two hidden layers only.
# Canonical flat parameter layout: W1[K][Hd], b1[Hd], W2[Hd][Hd], b2[Hd], W3[Hd][C], b3[C].
# --------------------------------------------------------------------------------------
def mlp_param_count(K, Hd, C):
    return K * Hd + Hd + Hd * Hd + Hd + Hd * C + C


def mlp_split(params, K, Hd, C):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    out = []
    for shape in ((K, Hd), (Hd,), (Hd, Hd), (Hd,), (Hd, C), (C,)):
        size = int(np.prod(shape))
        out.append(p[o:o + size].reshape(shape))
        o += size
    return out


def hard_gelu(z):
    """hardGELU of section 4.4: 0 below -3/2, identity above 3/2, x(x + 3/2)/3 between
    (the boundary points themselves take the middle branch)."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z < -1.5, 0.0, np.where(z > 1.5, z, z * (z + 1.5) / 3.0))


def activation(z, act):
    if act == "relu":
        return np.maximum(z, 0.0)
    if act == "hardgelu":
        return hard_gelu(z)
    raise ValueError(act)


def activation_grad(z, act):
    if act == "relu":
        return (z > 0).astype(np.float64)
    if act == "hardgelu":
        return np.where(z < -1.5, 0.0, np.where(z > 1.5, 1.0, (2.0 * z + 1.5) / 3.0))
    raise ValueError(act)


def mlp_forward(params, x, K, Hd, C, act="relu"):
    """y = W3^T a(W2^T a(W1^T x + b1) + b2) + b3, no output activation (section 4.4)."""
    W1, b1, W2, b2, W3, b3 = mlp_split(params, K, Hd, C)
    z1 = x @ W1 + b1
    h1 = activation(z1, act)
    z2 = h1 @ W2 + b2
    h2 = activation(z2, act)
    y = h2 @ W3 + b3
    return y, (z1, h1, z2, h2)


def relu_decisions_fp16(params, x, K, Hd, C):
    """ReLU decisions (z > 0) of both hidden layers taken the way an FP16 matrix-core
    evaluation takes them: inputs, weights and hidden activations rounded to FP16,
    products accumulated in FP32.  Used only to compare an FP16 evaluation with the
    float64 arithmetic under the same decisions (a decision near z = 0 legitimately
    differs between precisions)."""
    W1, b1, W2, b2, W3, b3 = mlp_split(params, K, Hd, C)
    h = lambda a: np.asarray(a, dtype=np.float16).astype(np.float32)
    z1 = h(x) @ h(W1) + b1.astype(np.float32)
    m1 = z1 > 0
    z2 = h(np.maximum(z1, 0)) @ h(W2) + b2.astype(np.float32)
    return m1, z2 > 0


def mlp_forward_masked(params, x, K, Hd, C, masks):
    """Forward with given ReLU decisions (float64 values): h = z * mask."""
    W1, b1, W2, b2, W3, b3 = mlp_split(params, K, Hd, C)
    z1 = x @ W1 + b1
    h1 = z1 * masks[0]
    z2 = h1 @ W2 + b2
    h2 = z2 * masks[1]
    return h2 @ W3 + b3, (z1, h1, z2, h2)


def decode(geom: Geometry, lat, params, queries):
    """Decode every channel of each queried texel (sections 4.3-4.4)."""
    x, _ = sample_inputs(geom, lat, queries)
    y, _ = mlp_forward(params, x, geom.K, geom.Hd, geom.C, geom.act)
    return y


# --------------------------------------------------------------------------------------
# Reduced-precision decode (section 7.3, Future Work, names lower-precision intermediates as the next
# speed-up).  Reading taken: FP8-e4m3 in the OCP definition (sign, 4 exponent bits with
# bias 7, 3 mantissa bits; exponent 0 is subnormal; largest finite magnitude 448, the
# all-ones pattern is NaN, no infinities), round to nearest even, saturating at 448.
# Weights of layer l are stored as W_l / s_l with s_l = max|W_l| / 448; inputs and
# hidden activations are rounded as they are; products accumulate in float64 here
# (FP32 on the GPU); s_l and the FP32 biases are applied after the sum.
# --------------------------------------------------------------------------------------
E4M3_MAX = 448.0


def e4m3_value(code):
    """Value of an e4m3 byte, from the bit fields (NaN for the all-ones patterns)."""
    code = int(code) & 0xFF
    sign = -1.0 if code & 0x80 else 1.0
    e, m = (code >> 3) & 15, code & 7
    if e == 15 and m == 7:
        return math.nan
    if e == 0:
        return sign * m * 2.0 ** -9
    return sign * (1 + m / 8) * 2.0 ** (e - 7)


def round_e4m3(x):
    """Nearest e4m3 value (ties to even), saturating to +-448; NaN stays NaN."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)            # below 2^-6 the spacing stays 2^-9 (subnormals)
    q = np.exp2(e - 3)                 # spacing of the values in [2^e, 2^(e+1))
    r = np.rint(a / q) * q             # np.rint rounds half to even
    r = np.minimum(r, E4M3_MAX)
    return np.where(np.isnan(x), np.nan, np.copysign(r, x))


def fp8_layer_scales(params, K, Hd, C):
    """Per-layer weight scales s_l = max|W_l| / 448 (1 for an all-zero layer)."""
    W1, _, W2, _, W3, _ = mlp_split(params, K, Hd, C)
    return [float(np.max(np.abs(W))) / E4M3_MAX if np.any(W) else 1.0 for W in (W1, W2, W3)]


def mlp_forward_fp8(params, x, K, Hd, C, act="relu"):
    """The network with e4m3 weights (per-layer scale), inputs and hidden activations."""
    W1, b1, W2, b2, W3, b3 = mlp_split(params, K, Hd, C)
    s1, s2, s3 = fp8_layer_scales(params, K, Hd, C)
    h1 = activation(s1 * (round_e4m3(x) @ round_e4m3(W1 / s1)) + b1, act)
    h2 = activation(s2 * (round_e4m3(h1) @ round_e4m3(W2 / s2)) + b2, act)
    return s3 * (round_e4m3(h2) @ round_e4m3(W3 / s3)) + b3


def decode_fp8(geom: Geometry, lat, params, queries):
    """decode() with the network evaluated in e4m3 as described above."""
    x, _ = sample_inputs(geom, lat, queries)
    return mlp_forward_fp8(params, x, geom.K, geom.Hd, geom.C, geom.act)


def _targets_at(geom: Geometry, targets, rec):
    t = np.zeros((len(rec["lod"]), geom.C))
    for l in np.unique(rec["lod"]):
        sel = np.nonzero(rec["lod"] == l)[0]
        base = geom.mip_off[l]
        idx = base + (rec["iy"][sel] * geom.mip_w[l] + rec["ix"][sel]) * geom.C
        t[sel] = np.asarray(targets, dtype=np.float64)[idx[:, None] + np.arange(geom.C)[None, :]]
    return t


def loss_and_grads(geom: Geometry, lat_fwd, params, queries, targets=None, dout=None, decisions=None):
    """L2 loss (section 4.5) and its exact gradient w.r.t. MLP parameters and latents.

    L = (1/(n C)) sum (y - t)^2.  With `dout` given instead of targets, the output
    gradient is dout itself and L is None (the differentiation path).  Latent
    gradients: every G0 cell receives its slot of dL/dx; every G1 tap receives its
    bilinear weight times the G1 slot of dL/dx; the positional encoding has no
    parameters.  Cells reached several times accumulate.
    """
    K, Hd, C = geom.K, geom.Hd, geom.C
    x, rec = sample_inputs(geom, lat_fwd, queries)
    masks = None
    if decisions == "fp16":
        if geom.act != "relu":
            raise ValueError("decision matching is defined for ReLU")
        masks = relu_decisions_fp16(params, x, K, Hd, C)
        y, (z1, h1, z2, h2) = mlp_forward_masked(params, x, K, Hd, C, masks)
    else:
        y, (z1, h1, z2, h2) = mlp_forward(params, x, K, Hd, C, geom.act)
    W1, b1, W2, b2, W3, b3 = mlp_split(params, K, Hd, C)
    agrad = (lambda z, k: masks[k].astype(np.float64)) if masks is not None else \
        (lambda z, k: activation_grad(z, geom.act))
    n = x.shape[0]
    if dout is None:
        t = _targets_at(geom, targets, rec)
        r = y - t
        L = float(np.sum(r * r) / (n * C))
        dy = 2.0 * r / (n * C)
    else:
        L = None
        dy = np.asarray(dout, dtype=np.float64)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dz2 = (dy @ W3.T) * agrad(z2, 1)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * agrad(z1, 0)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    dx = dz1 @ W1.T
    gparams = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    glat = np.zeros(geom.latent_count)
    C0, C1 = geom.C0, geom.C1
    for k in range(4):
        np.add.at(glat, rec["g0_idx"][:, k:k + 1] + np.arange(C0)[None, :], dx[:, k * C0:(k + 1) * C0])
        np.add.at(glat, rec["g1_idx"][:, k:k + 1] + np.arange(C1)[None, :],
                  rec["g1_w"][:, k:k + 1] * dx[:, 4 * C0:4 * C0 + C1])
    return L, gparams, glat, y


# --------------------------------------------------------------------------------------
# Optimisation: section 4.5 (Adam), section 4.2 (clamp after the update), section 5.1
# (separate learning rates for latents and network).
# --------------------------------------------------------------------------------------
def adam_update(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma and Ba) at 1-based step t; returns new
    (p, m, v).  Dense: every entry is updated every step."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def clamp_latents(geom: Geometry, lat):
    """Clamp every latent into its grid's quantization range (section 4.2)."""
    lat = np.array(lat, dtype=np.float64)
    for off, w, h, c, b in _grids(geom):
        lo, hi = quant_range(b)
        s = slice(off, off + w * h * c)
        lat[s] = np.clip(lat[s], lo, hi)
    return lat


def train_step(geom: Geometry, state: dict, queries, targets, hp: dict):
    """One training step of the autodecoder (sections 4.2, 4.5, 5.1).

    state: latents, mlp, lat_m, lat_v, mlp_m, mlp_v (float arrays).
    hp: lr_latent, lr_mlp, beta1, beta2, eps, seed, step (0-based), noise (bool),
        freeze_latents (bool).
    Forward latents are masters + U(-Q/2, Q/2) noise (noise on, not frozen).  After the
    Adam update latents are clamped to the quantization range.  With frozen latents
    only the network is updated.  If any gradient is not finite the step is skipped
    (returns overflow=True, state unchanged), which is how a loss-scaled low-precision
    trainer treats an overflow.
    """
    lat = np.asarray(state["latents"], dtype=np.float64)
    fwd = lat.copy()
    if hp.get("noise", False) and not hp.get("freeze_latents", False):
        fwd = lat + noise_values(geom, hp["seed"], hp["step"])
    L, gp, gl, _ = loss_and_grads(geom, fwd, state["mlp"], queries, targets)
    if not (np.all(np.isfinite(gp)) and np.all(np.isfinite(gl))):
        return dict(state), L, True
    t = hp["step"] + 1
    b1, b2, eps = hp.get("beta1", 0.9), hp.get("beta2", 0.999), hp.get("eps", 1e-8)
    new = dict(state)
    new["mlp"], new["mlp_m"], new["mlp_v"] = adam_update(
        state["mlp"], gp, state["mlp_m"], state["mlp_v"], t, hp["lr_mlp"], b1, b2, eps)
    if not hp.get("freeze_latents", False):
        p, new["lat_m"], new["lat_v"] = adam_update(
            lat, gl, state["lat_m"], state["lat_v"], t, hp["lr_latent"], b1, b2, eps)
        new["latents"] = clamp_latents(geom, p)
    return new, L, False


def loss_scale_update(scale, good_steps, overflow, growth_interval=2000):
    """Dynamic loss scaling policy: halve on overflow (and restart the count), double
    after `growth_interval` consecutive good steps."""
    if overflow:
        return scale * 0.5, 0
    good_steps += 1
    if good_steps >= growth_interval:
        return scale * 2.0, 0
    return scale, good_steps


# --------------------------------------------------------------------------------------
# Quality: Appendix 'Error and Quality Metrics', Eq. 1.
# --------------------------------------------------------------------------------------
def psnr(ref_mips, test_mips):
    """PSNR over a texture set and its mip chain (Eq. 1): squared error summed over
    every mip, divided by c * sum_j w_j h_j; values in [0, 1]."""
    se = 0.0
    count = 0
    for r, t in zip(ref_mips, test_mips):
        r = np.asarray(r, dtype=np.float64)
        t = np.asarray(t, dtype=np.float64)
        se += float(np.sum((r - t) ** 2))
        count += r.size
    return -10.0 * math.log10(se / count)


# --------------------------------------------------------------------------------------
# Filtered decode: section 5.3 (Filtering).  The network is fitted at discrete texels and
# mips only, so texture filtering combines decoded texels: bilinear (4 texels of the
# nearest mip), trilinear (bilinear in the two mips around a continuous LOD, blended),
# and stochastic filtering (one texel after a uniform jitter of up to half a texel of the
# position and a random choice between the two mips).  Positions are computed in float32
# (the arithmetic the decoder's texel addressing uses, so both pick the same texels);
# the combination is float64.  The random numbers of stochastic filtering are SplitMix64
# outputs of counters: key = mix(seed ^ FILTER_TAG), h1 = mix(key + gamma (2i + 1)),
# h2 = mix(key + gamma (2i + 2)) for output i; r1 = (h1 >> 40) 2^-24,
# r2 = ((h1 >> 16) & (2^24 - 1)) 2^-24, r3 = (h2 >> 40) 2^-24.
# --------------------------------------------------------------------------------------
FILTER_BILINEAR, FILTER_TRILINEAR, FILTER_STOCHASTIC = 1, 2, 3
FILTER_TAG = 0x66696C74
FILTER_QUERY = np.dtype([("u", "<f4"), ("v", "<f4"), ("lod", "<f4")])
_QREC = np.dtype([("u", "<f4"), ("v", "<f4"), ("lod", "<i4")])


def _filter_inputs(geom: Geometry, fq):
    f32 = np.float32
    u = np.where(np.isnan(fq["u"]), f32(0), fq["u"]).astype(f32)
    v = np.where(np.isnan(fq["v"]), f32(0), fq["v"]).astype(f32)
    lod = np.where(np.isnan(fq["lod"]), f32(0), fq["lod"]).astype(f32)
    lf = np.minimum(np.maximum(lod, f32(0)), f32(geom.M - 1))
    return u, v, lf


def _bilinear_taps(geom: Geometry, u, v, l):
    """The four texel centres around (u, v) in mip l (clamped) and their weights."""
    f32 = np.float32
    W = np.array([geom.mip_w[i] for i in range(geom.M)], dtype=np.int64)[l]
    H = np.array([geom.mip_h[i] for i in range(geom.M)], dtype=np.int64)[l]
    x = u * W.astype(f32) - f32(0.5)
    y = v * H.astype(f32) - f32(0.5)
    x0, y0 = np.floor(x), np.floor(y)
    fx, fy = (x - x0).astype(np.float64), (y - y0).astype(np.float64)
    taps, wts = [], []
    for dy in (0, 1):
        for dx in (0, 1):
            xi = np.clip(x0.astype(np.int64) + dx, 0, W - 1)
            yi = np.clip(y0.astype(np.int64) + dy, 0, H - 1)
            taps.append(((xi.astype(f32) + f32(0.5)) / W.astype(f32), (yi.astype(f32) + f32(0.5)) / H.astype(f32)))
            wts.append((fx if dx else 1.0 - fx) * (fy if dy else 1.0 - fy))
    return taps, wts


def filter_randoms(seed: int, n: int):
    """(r1, r2, r3) of outputs 0..n-1, each in [0, 1) with 24 bits, as float32."""
    key = int(splitmix64_mix(np.uint64((seed ^ FILTER_TAG) & MASK64)))
    i = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h1 = splitmix64_mix(np.uint64(key) + np.uint64(GAMMA) * (np.uint64(2) * i + np.uint64(1)))
        h2 = splitmix64_mix(np.uint64(key) + np.uint64(GAMMA) * (np.uint64(2) * i + np.uint64(2)))
    s = np.float32(2.0 ** -24)
    r1 = (h1 >> np.uint64(40)).astype(np.float32) * s
    r2 = ((h1 >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float32) * s
    r3 = (h2 >> np.uint64(40)).astype(np.float32) * s
    return r1, r2, r3


def filter_taps(geom: Geometry, fq, mode: int, seed: int = 0):
    """Point queries (QUERY records) [n, T] and float64 weights [n, T] that filtered output
    i combines: T = 4 (bilinear), 8 (trilinear) or 1 (stochastic)."""
    f32 = np.float32
    u, v, lf = _filter_inputs(geom, fq)
    n = len(u)
    l0 = np.floor(lf).astype(np.int64)
    if mode == FILTER_BILINEAR:
        levels = [np.minimum(np.floor(lf + f32(0.5)).astype(np.int64), geom.M - 1)]
        blend = [np.ones(n)]
    elif mode == FILTER_TRILINEAR:
        t = (lf - l0.astype(f32)).astype(np.float64)
        levels = [l0, np.minimum(l0 + 1, geom.M - 1)]
        blend = [1.0 - t, t]
    elif mode == FILTER_STOCHASTIC:
        r1, r2, r3 = filter_randoms(seed, n)
        l = np.minimum(l0 + (r3 < (lf - l0.astype(f32))).astype(np.int64), geom.M - 1)
        W = np.array(geom.mip_w, dtype=np.int64)[l].astype(f32)
        H = np.array(geom.mip_h, dtype=np.int64)[l].astype(f32)
        q = np.zeros((n, 1), dtype=_QREC)
        q["u"][:, 0] = u + (r1 - f32(0.5)) / W
        q["v"][:, 0] = v + (r2 - f32(0.5)) / H
        q["lod"][:, 0] = l
        return q, np.ones((n, 1))
    else:
        raise ValueError("unknown filter")
    cols, wcols = [], []
    for l, b in zip(levels, blend):
        taps, wts = _bilinear_taps(geom, u, v, l)
        for (tu, tv), w in zip(taps, wts):
            rec = np.zeros(n, dtype=_QREC)
            rec["u"], rec["v"], rec["lod"] = tu, tv, l
            cols.append(rec)
            wcols.append(w * b)
    return np.stack(cols, axis=1), np.stack(wcols, axis=1)


def decode_filtered(geom: Geometry, lat, params, fq, mode: int, seed: int = 0):
    """Filtered outputs [n, C]: the weighted sum of the decoded taps (section 5.3)."""
    q, w = filter_taps(geom, fq, mode, seed)
    n, T = q.shape
    y = decode(geom, lat, params, q.reshape(-1)).reshape(n, T, geom.C)
    return np.einsum("nt,ntc->nc", w, y)
