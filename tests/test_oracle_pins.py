"""Pins of the FP64 oracle against what the paper and mathematics fix (no GPU).

Each test names the passage it follows.  None of them re-derives an expected value
by calling the oracle function under test.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Table 1 / Table 6
def test_table1_levels_and_mips():
    """Table 1: 1024^2 set -> four levels, G0 256/64/16/4, G1 128/32/8/2, mips 0-3,4-5,6-7,8-10."""
    gold = json.load(open(os.path.join(GOLD, "table1_1024.json")))
    g = O.make_geometry(gold["width"], gold["height"], 9, 8, 8, 4, 4, shift=gold["shift"])
    assert g.J == len(gold["levels"])
    assert g.M == 11
    for j, lev in enumerate(gold["levels"]):
        assert list(g.g0[j]) == lev["g0"]
        assert list(g.g1[j]) == lev["g1"]
        assert [l for l in range(g.M) if g.level_of_mip[l] == j] == lev["mips"]


def test_table6_storage():
    gold = json.load(open(os.path.join(GOLD, "table6_storage.json")))
    MiB = 2.0 ** 20
    for name, p in gold["profiles"].items():
        for res, mb in gold["grids_mb"][name].items():
            res = int(res)
            if res < 8192:
                got = O.storage_bytes_paper(res, res, p["c0"], p["c1"], p["b0"], p["b1"], p["shift"], levels=1) / MiB
                assert got == pytest.approx(mb, abs=1e-12), (name, res)
            else:
                got = O.storage_bytes_paper(res, res, p["c0"], p["c1"], p["b0"], p["b1"], p["shift"]) / MiB
                assert abs(got - mb) < 3e-3, (name, res, got)


def test_packed_bytes_match_table6_level0():
    """The packer's byte count for level 0 of NTC 1.0 at 4k is 12 + 5 MiB (Table 6)."""
    g = O.make_geometry(4096, 4096, 9, 12, 10, 2, 4, shift=1)
    lat = np.zeros(g.latent_count)
    packed = O.quantize_latents(g, lat)
    level0 = (g.g0[0][0] * g.g0[0][1] * 12 * 2 + g.g1[0][0] * g.g1[0][1] * 10 * 4) // 8
    assert level0 == 17 * 2 ** 20
    # every grid padded to 16 bytes, so the total is at least the paper's all-level figure
    assert len(packed) >= O.storage_bytes_paper(4096, 4096, 12, 10, 2, 4, 1)
    assert len(packed) % 16 == 0


def test_input_width():
    """Section 4.4: input size 4*C0 + C1 + 12 (+1 for the LOD, off here)."""
    assert O.make_geometry(256, 256, 8, 8, 8, 4, 4).K == 52
    assert O.make_geometry(2048, 2048, 12, 12, 12, 4, 4).K == 72
    assert O.make_geometry(4096, 4096, 16, 16, 16, 2, 4).K == 92
    assert O.make_geometry(2048, 2048, 12, 12, 12, 4, 4, lod_input=True).K == 73


def test_lod_input_value():
    """Section 4.4's LOD input, read as the mip over the chain, l / (M - 1): a network
    whose only path is that input (W1 row K-1 to hidden 0, W2 = I, W3 hidden 0 to every
    output) outputs l / (M - 1) for each query's mip (M = 9: 0, 1/8, ..., 1)."""
    g = O.make_geometry(256, 256, 4, 4, 4, 4, 4, Hd=16, lod_input=True)
    assert g.M == 9 and g.K == 4 * 4 + 4 + 12 + 1
    K, Hd, C = g.K, g.Hd, g.C
    W1 = np.zeros((K, Hd)); W1[K - 1, 0] = 1.0
    W3 = np.zeros((Hd, C)); W3[0, :] = 1.0
    p = np.concatenate([W1.ravel(), np.zeros(Hd), np.eye(Hd).ravel(), np.zeros(Hd), W3.ravel(), np.zeros(C)])
    q = np.zeros(9, dtype=synth.QUERY_DTYPE)
    q["u"], q["v"], q["lod"] = 0.3, 0.7, np.arange(9)
    lat = np.random.default_rng(0).uniform(-0.5, 0.5, g.latent_count)
    y = O.decode(g, lat, p, q)
    assert np.array_equal(y, np.repeat((np.arange(9) / 8.0)[:, None], C, axis=1))


# ---------------------------------------------------------------- quantization (sec 4.2)
def test_quantizer_hand_table_2bit():
    # N = 4, Q = 1/4, levels k*Q for k = -1..2, codes k + 1; ties round to even k.
    xs = [0.0, 0.25, 0.5, -0.25, -0.375, 0.125, 0.375, -1.0, 7.0, 0.3, -0.1]
    want = [1, 2, 3, 0, 0, 1, 3, 0, 3, 2, 1]
    assert O.quantize_codes(np.array(xs), 2).tolist() == want


def test_quantizer_hand_table_4bit():
    # N = 16: codes k + 7, k in [-7, 8].  -15/32 is a tie at k = -7.5 -> even -8 -> clamp -7.
    xs = [0.0, 1 / 16, 0.5, -7 / 16, -15 / 32, 1 / 32, 3 / 32, 0.49, -0.6, np.nan, np.inf]
    want = [7, 8, 15, 0, 0, 7, 9, 15, 0, 7, 7]
    assert O.quantize_codes(np.array(xs), 4).tolist() == want


@pytest.mark.parametrize("B", [1, 2, 4, 8])
def test_quantizer_levels_and_roundtrip(B):
    N = 2 ** B
    codes = np.arange(N)
    vals = O.dequantize_codes(codes, B)
    assert vals.min() == -(N // 2 - 1) / N and vals.max() == 0.5
    assert O.quantize_codes(vals, B).tolist() == codes.tolist()
    assert 0.0 in vals.tolist()                       # zero is exactly representable
    lo, hi = O.quant_range(B)
    assert lo == -(N - 1) / (2 * N) and hi == 0.5
    dense = np.linspace(-2, 2, 10001)
    assert len(np.unique(O.quantize_codes(dense, B))) == N


def test_dequantized_values_exact_in_fp16_fp8():
    # values k/16 with |k| <= 8 and k/4 with |k| <= 2 need <= 4 significant bits
    for B in (2, 4):
        v = O.dequantize_codes(np.arange(2 ** B), B)
        assert np.array_equal(v.astype(np.float16).astype(np.float64), v)
        assert np.array_equal(O.round_e4m3(v), v)


def test_pack_lsb_first_hand_example():
    # B = 4, codes 1,2,3,4 -> nibbles LSB first -> bytes 0x21, 0x43, then zero padding
    out = O.pack_codes([1, 2, 3, 4], 4)
    assert out[:2].tolist() == [0x21, 0x43] and len(out) == 16 and not out[2:].any()
    out = O.pack_codes([3, 0, 1, 2, 1], 2)   # 11 00 01 10 | 01 -> 0b10010011, 0b01
    assert out[:2].tolist() == [0b10010011, 0b01]
    assert O.unpack_codes(out, 2, 5).tolist() == [3, 0, 1, 2, 1]


# ---------------------------------------------------------------- noise (sec 4.2)
def test_splitmix64_published_outputs():
    """SplitMix64 seeded with 0 (Steele et al. 2014; reference C by Vigna) emits
    0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f."""
    got = [int(O.splitmix64_mix(np.uint64((O.GAMMA * k) & O.MASK64))) for k in (1, 2, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_noise_distribution():
    from scipy import stats
    g = O.make_geometry(256, 256, 8, 8, 8, 4, 2, M=9)
    nu = O.noise_values(g, seed=7, step=3)
    bits = O.latent_bits(g)
    q = 1.0 / 2.0 ** bits
    assert np.all(nu >= -q / 2) and np.all(nu < q / 2)
    r = nu / q + 0.5                                          # should be U[0,1)
    assert stats.kstest(r, "uniform").pvalue > 1e-3
    assert abs(r.mean() - 0.5) < 0.01
    assert np.array_equal(nu, O.noise_values(g, 7, 3))
    assert not np.array_equal(nu, O.noise_values(g, 7, 4))
    assert not np.array_equal(nu, O.noise_values(g, 8, 3))


# ---------------------------------------------------------------- sampling (sec 4.3)
def _one(u, v, lod=0):
    q = np.zeros(1, dtype=synth.QUERY_DTYPE)
    q["u"], q["v"], q["lod"] = u, v, lod
    return q


def test_g0_neighbours_hand_table_8x8():
    """8x8 texture, G0 2x2, G1 1x1.  Footprint x-indices by hand:
    ix 0,1 -> (0,0); ix 2..5 -> (0,1); ix 6,7 -> (1,1) (edges clamp)."""
    g = O.make_geometry(8, 8, 1, 1, 1, 4, 4, M=1)
    assert g.g0 == [(2, 2)] and g.g1 == [(1, 1)]
    table = {0: (0, 0), 1: (0, 0), 2: (0, 1), 3: (0, 1), 4: (0, 1), 5: (0, 1), 6: (1, 1), 7: (1, 1)}
    lat = np.zeros(g.latent_count)
    lat[:4] = [10.0, 20.0, 30.0, 40.0]                # G0 cells (x,y) row-major
    lat[4] = 5.0                                      # the single G1 cell
    for iy in range(8):
        for ix in range(8):
            q = _one((ix + 0.5) / 8, (iy + 0.5) / 8)
            x, _ = O.sample_inputs(g, lat, q)
            xa, xb = table[ix]
            ya, yb = table[iy]
            want = [lat[ya * 2 + xa], lat[ya * 2 + xb], lat[yb * 2 + xa], lat[yb * 2 + xb]]
            assert x[0, :4].tolist() == want
            assert x[0, 4] == 5.0                     # bilinear of one cell is the cell


def test_bilinear_weights_and_centres():
    g = O.make_geometry(64, 64, 3, 2, 3, 4, 4)
    rng = np.random.default_rng(0)
    lat = rng.standard_normal(g.latent_count)
    q = synth.random_queries(1, 4000, g.M)
    _, rec = O.sample_inputs(g, lat, q)
    assert np.allclose(rec["g1_w"].sum(axis=1), 1.0, atol=0, rtol=0) or \
        np.max(np.abs(rec["g1_w"].sum(axis=1) - 1.0)) < 1e-15
    assert np.all(rec["g1_w"] >= 0)
    # At the mip whose resolution equals G1's, texel centres are G1 cell centres:
    # the interpolated value is the cell itself.  Level 0: G1 = 8x8 = mip 3.
    w1, h1 = g.g1[0]
    assert g.mip_w[3] == w1 and g.level_of_mip[3] == 0
    for iy in range(h1):
        for ix in range(w1):
            x, _ = O.sample_inputs(g, lat, _one((ix + 0.5) / w1, (iy + 0.5) / h1, 3))
            cell = g.g1_off[0] + (iy * w1 + ix) * 3
            assert np.array_equal(x[0, 8:11], lat[cell:cell + 3])


def test_bilinear_reproduces_affine_field():
    """Away from borders bilinear interpolation is exact on an affine field."""
    g = O.make_geometry(128, 128, 1, 1, 1, 4, 4, M=1)
    w1, h1 = g.g1[0]                                   # 16 x 16
    lat = np.zeros(g.latent_count)
    yy, xx = np.meshgrid(np.arange(h1), np.arange(w1), indexing="ij")
    lat[g.g1_off[0]:] = (0.3 * xx - 0.7 * yy + 0.1).ravel()
    for ix, iy in [(20, 30), (64, 64), (100, 17), (33, 90)]:
        x, _ = O.sample_inputs(g, lat, _one((ix + 0.5) / 128, (iy + 0.5) / 128))
        gx = (ix + 0.5) / 128 * w1 - 0.5
        gy = (iy + 0.5) / 128 * h1 - 0.5
        assert x[0, 4] == pytest.approx(0.3 * gx - 0.7 * gy + 0.1, abs=1e-12)


def test_pos_enc_values():
    """Section 4.3.2: period 8 texels, 3 octaves, last value per axis constant."""
    s8, c8 = math.sin(math.pi / 8), math.cos(math.pi / 8)
    r2 = math.sqrt(0.5)
    pe = O.pos_enc(np.array([0]), np.array([3]))[0]
    # x: t = 1/16 -> sin(pi/8), cos(pi/8), sin(pi/4), cos(pi/4), sin(pi/2), cos(pi/2)
    assert pe[:6] == pytest.approx([s8, c8, r2, r2, 1.0, 0.0], abs=1e-15)
    # y: t = 7/16 -> sin(7pi/8), cos(7pi/8), sin(7pi/4), cos(7pi/4), sin(7pi/2), cos(7pi/2)
    assert pe[6:] == pytest.approx([s8, -c8, -r2, r2, -1.0, 0.0], abs=1e-15)
    i = np.arange(64)
    a = O.pos_enc(i, i)
    assert np.allclose(a[:8], a[8:16]) and np.allclose(a, np.roll(a, 8, axis=0))
    assert np.all(np.abs(a[:, 5]) < 1e-14) and np.all(np.abs(a[:, 11]) < 1e-14)


def test_pos_enc_triangle_values():
    """Section 4.3.2's triangular waves: hand values at texel centres (x: i = 0,
    t = 1/16; y: i = 3, t = 7/16), period 8, the last value per axis constant 0, the
    signs of the sine/cosine encoding, and |S| + |K| = 1 for every pair (quadrature
    triangle waves)."""
    pe = O.pos_enc(np.array([0]), np.array([3]), "triangle")[0]
    assert list(pe[:6]) == [0.25, 0.75, 0.5, 0.5, 1.0, 0.0]
    assert list(pe[6:]) == [0.25, -0.75, -0.5, 0.5, -1.0, 0.0]
    i = np.arange(64)
    a = O.pos_enc(i, i, "triangle")
    b = O.pos_enc(i, i, "sincos")
    assert np.array_equal(a, np.roll(a, 8, axis=0))
    assert np.all(a[:, 5] == 0) and np.all(a[:, 11] == 0)
    nz = np.abs(b) > 1e-12
    assert np.array_equal(np.sign(a[nz]), np.sign(b[nz]))
    for k in range(0, 12, 2):
        assert np.allclose(np.abs(a[:, k]) + np.abs(a[:, k + 1]), 1.0, atol=0)


def test_lod_clamp_and_snap():
    g = O.make_geometry(16, 16, 1, 1, 1, 4, 4)
    q = np.zeros(4, dtype=synth.QUERY_DTYPE)
    q["u"] = [-0.5, 1.0, 2.0, np.nan]
    q["v"] = [0.0, 0.999, 0.5, 0.5]
    q["lod"] = [-3, 0, 99, 1]
    _, rec = O.sample_inputs(g, np.zeros(g.latent_count), q)
    assert rec["lod"].tolist() == [0, 0, g.M - 1, 1]
    assert rec["ix"].tolist() == [0, 15, 0, 0]


# ---------------------------------------------------------------- network (sec 4.4)
def test_mlp_selection_wiring():
    """W1 copies input k to hidden k (+1 shift keeps ReLU active), W2 = I, W3 reads
    hidden c into output c: y_c = x_c + 1 + b3_c.  A transposed or misrouted operand
    breaks this."""
    K, Hd, C = 52, 64, 8
    W1 = np.zeros((K, Hd)); W1[np.arange(K), np.arange(K)] = 1.0
    b1 = np.ones(Hd)
    W2 = np.eye(Hd); b2 = np.zeros(Hd)
    W3 = np.zeros((Hd, C)); W3[np.arange(C), np.arange(C)] = 1.0
    b3 = np.arange(C) * 0.01
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    x = np.random.default_rng(2).uniform(0, 1, (5, K))
    y, _ = O.mlp_forward(p, x, K, Hd, C)
    assert np.allclose(y, x[:, :C] + 1.0 + b3, atol=1e-14)


def test_constant_outputs():
    g = O.make_geometry(64, 64, 4, 2, 2, 4, 4, Hd=16)
    P = O.mlp_param_count(g.K, g.Hd, g.C)
    p = np.zeros(P)
    p[-g.C:] = [0.1, 0.2, 0.3, 0.4]                   # only b3
    q = synth.random_queries(3, 100, g.M)
    lat = np.random.default_rng(1).standard_normal(g.latent_count)
    assert np.allclose(O.decode(g, lat, p, q), [0.1, 0.2, 0.3, 0.4], atol=0)
    # constant latents + zero W1 rows on PE -> constant output
    p = np.random.default_rng(4).standard_normal(P)
    W1 = p[:g.K * g.Hd].reshape(g.K, g.Hd)
    W1[4 * g.C0 + g.C1:] = 0.0
    y = O.decode(g, np.full(g.latent_count, 0.25), p, q)
    assert np.allclose(y, y[0], atol=1e-12)


def test_hard_gelu():
    z = np.array([-2.0, -1.5, -1.0, 0.0, 1.0, 1.5, 2.0])
    want = [0.0, 0.0, -1.0 * 0.5 / 3, 0.0, 1.0 * 2.5 / 3, 1.5, 2.0]
    assert O.hard_gelu(z).tolist() == pytest.approx(want, abs=1e-15)
    e = 1e-9
    for b in (-1.5, 1.5):
        assert abs(O.hard_gelu(b - e) - O.hard_gelu(b + e)) < 1e-8


# ---------------------------------------------------------------- FP8-e4m3 decode (sec 8)
def test_e4m3_code_table():
    """The bit-field decoder against hand values, and the rounder against every code."""
    assert O.e4m3_value(0x00) == 0.0 and O.e4m3_value(0x01) == 2.0 ** -9
    assert O.e4m3_value(0x07) == 7 * 2.0 ** -9 and O.e4m3_value(0x08) == 2.0 ** -6
    assert O.e4m3_value(0x38) == 1.0 and O.e4m3_value(0x3C) == 1.5 and O.e4m3_value(0xB8) == -1.0
    assert O.e4m3_value(0x7E) == 448.0 and math.isnan(O.e4m3_value(0x7F)) and math.isnan(O.e4m3_value(0xFF))
    vals = np.array([O.e4m3_value(c) for c in range(256)])
    fin = vals[~np.isnan(vals)]
    assert len(fin) == 254                                     # 2 x 127 finite patterns (+0 and -0)
    assert np.array_equal(O.round_e4m3(fin), fin)              # every value is its own rounding


def test_e4m3_rounding_ties_and_saturation():
    pos = [O.e4m3_value(c) for c in range(0x7F)]               # increasing positive values, 0 .. 448
    for c in range(0x7E):
        a, b = pos[c], pos[c + 1]
        mid = 0.5 * (a + b)
        even = a if c % 2 == 0 else b                          # the pattern with mantissa lsb 0
        assert O.round_e4m3(mid) == even
        assert O.round_e4m3(mid - 1e-6 * (b - a)) == a
        assert O.round_e4m3(mid + 1e-6 * (b - a)) == b
        assert O.round_e4m3(-mid) == -even
    assert O.round_e4m3(0.3) == 0.3125                        # spacing 1/32 in [1/4, 1/2)
    assert O.round_e4m3(460.0) == 448.0 and O.round_e4m3(1e6) == 448.0 and O.round_e4m3(-1e6) == -448.0
    assert math.isnan(O.round_e4m3(np.nan))


def test_fp8_forward_exact_case():
    """Inputs, weights (after the per-layer scale) and hidden values all exact in e4m3:
    the FP8 network equals the float64 network.  A misapplied scale or a layer rounded
    in the wrong place breaks this."""
    K, Hd, C = 20, 16, 4
    rng = np.random.default_rng(8)
    def sparse_pm1(rows, cols):
        W = np.zeros((rows, cols))
        for j in range(cols):
            i = rng.choice(rows, 2, replace=False)
            W[i, j] = rng.choice([-1.0, 1.0], 2)
        return W
    W1, W2 = sparse_pm1(K, Hd), sparse_pm1(Hd, Hd)
    W3 = rng.choice([-1.0, -0.5, 0.25, 0.5, 1.0], (Hd, C))
    b1, b2, b3 = np.zeros(Hd), np.zeros(Hd), rng.uniform(-1, 1, C)
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    x = rng.choice([0.0, 0.5], (50, K))
    y8 = O.mlp_forward_fp8(p, x, K, Hd, C)
    y, _ = O.mlp_forward(p, x, K, Hd, C)
    assert np.max(np.abs(y8 - y)) < 1e-12
    assert O.fp8_layer_scales(p, K, Hd, C) == [1 / 448, 1 / 448, 1 / 448]
    # one inexact hidden value changes the result by exactly its rounding
    p2 = p.copy()
    p2[K * Hd] = 0.3                                           # b1[0]: h1[0] = z + 0.3 is not in e4m3
    p2[K * Hd + Hd] = 1.0                                      # W2[0][0]: h1[0] reaches the output
    y8b = O.mlp_forward_fp8(p2, x, K, Hd, C)
    _, (z1, h1, _, _) = O.mlp_forward(p2, x, K, Hd, C)
    assert not np.allclose(O.round_e4m3(h1[:, 0]), h1[:, 0])
    assert np.max(np.abs(y8b - O.mlp_forward(p2, x, K, Hd, C)[0])) > 0


# ---------------------------------------------------------------- training batches (sec 5.1)
def test_crop_lod_closed_form():
    """floor(-log4 X) at and around the powers of four, clamped to the chain."""
    M = 12
    assert O.crop_lod(1.0, M) == 0
    assert O.crop_lod(0.25, M) == 1 and O.crop_lod(0.25 + 1e-12, M) == 0
    assert O.crop_lod(1 / 16, M) == 2 and O.crop_lod(1 / 16 + 1e-12, M) == 1
    assert O.crop_lod(1e-300, M) == M - 1
    for X in np.random.default_rng(3).uniform(1e-6, 1, 1000):
        assert O.crop_lod(X, 40) == int(np.floor(-np.log(X) / np.log(4)))


def test_crop_lod_distribution():
    """Without the uniform batches, P(LOD = k) = 3/4 * 4^-k (the last mip takes the tail)."""
    g = O.make_geometry(256, 256, 4, 4, 4, 4, 4)          # 9 mips
    steps = 4000
    lods = np.array([O.crop_queries(g, 5, s, crops=1, side=1, fraction=0.0)["lod"][0] for s in range(steps)])
    k = np.arange(g.M)
    p = 0.75 * 4.0 ** -k
    p[-1] = 4.0 ** -(g.M - 1)
    counts = np.bincount(lods, minlength=g.M)
    big = p * steps >= 5
    chi2 = float(np.sum((counts[big] - steps * p[big]) ** 2 / (steps * p[big])))
    assert chi2 < 20.0, (counts, chi2)                   # 5 dof at the 0.1% level ~ 20.5
    # with fraction 1 every LOD is equally likely
    lods = np.array([O.crop_queries(g, 6, s, crops=1, side=1, fraction=1.0)["lod"][0] for s in range(2000)])
    c = np.bincount(lods, minlength=g.M)
    assert np.all(np.abs(c - 2000 / g.M) < 5 * np.sqrt(2000 / g.M))


def test_crop_geometry():
    g = O.make_geometry(512, 512, 4, 4, 4, 4, 4)
    for step in range(20):
        q = O.crop_queries(g, 9, step, crops=3, side=64)
        lod = int(q["lod"][0])
        assert np.all(q["lod"] == lod)
        W = g.mip_w[lod]
        x = q["u"].astype(np.float64) * W - 0.5
        y = q["v"].astype(np.float64) * W - 0.5
        assert np.all(x == np.round(x)) and np.all(y == np.round(y))   # texel centres
        for c in range(3):
            xc = x[c * 4096:(c + 1) * 4096].reshape(64, 64)
            yc = y[c * 4096:(c + 1) * 4096].reshape(64, 64)
            if W >= 64:    # a contiguous window inside the mip, row-major
                assert np.all(np.diff(xc, axis=1) == 1) and np.all(np.diff(yc, axis=0) == 1)
                assert xc.min() >= 0 and xc.max() <= W - 1
            else:          # the mip tiled from its origin
                assert np.array_equal(xc[0], np.arange(64) % W)


# ---------------------------------------------------------------- optimiser (sec 4.5, 5.1)
def test_adam_step1_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = O.adam_update(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), atol=1e-16)


def test_adam_constant_gradient_closed_form():
    g = np.array([0.5, -0.25])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 6):
        p, m, v = O.adam_update(p, g, m, v, t, 0.1)
    assert np.allclose(p, -5 * 0.1 * g / (np.abs(g) + 1e-8), atol=1e-12)


def test_train_step_clamps_after_update_and_freezes():
    g = O.make_geometry(16, 16, 2, 1, 1, 2, 2, Hd=16, M=1)
    P = O.mlp_param_count(g.K, g.Hd, g.C)
    st = dict(latents=np.full(g.latent_count, 0.5), mlp=np.full(P, 0.05),
              lat_m=np.zeros(g.latent_count), lat_v=np.zeros(g.latent_count),
              mlp_m=np.zeros(P), mlp_v=np.zeros(P))
    _, tgt = synth.target_chain(0, 0, 16, 16, 2, 1)
    tgt = np.zeros_like(tgt)                           # outputs > 0 -> latents pushed down
    tgt[:] = 5.0                                       # outputs < 5 -> latents pushed up, clamp at 0.5
    q = synth.random_queries(0, 64, 1, lod=0)
    hp = dict(lr_latent=0.1, lr_mlp=0.0, seed=0, step=0, noise=False)
    new, L, ovf = O.train_step(g, st, q, tgt, hp)
    assert not ovf and np.max(new["latents"]) <= 0.5 and np.min(new["latents"]) >= -3 / 8
    touched = np.nonzero(new["lat_m"])[0]
    assert len(touched) > 0
    hp2 = dict(hp, freeze_latents=True, lr_mlp=0.01)
    new2, _, _ = O.train_step(g, st, q, tgt, hp2)
    assert np.array_equal(new2["latents"], st["latents"]) and not np.array_equal(new2["mlp"], st["mlp"])
    bad = tgt.copy(); bad[0:2] = np.inf                # non-finite target -> skipped step
    q0 = synth.tile_queries(16, 16)
    new3, _, ovf3 = O.train_step(g, st, q0, bad, hp)
    assert ovf3 and np.array_equal(new3["latents"], st["latents"])


def test_loss_scale_policy():
    s, c = O.loss_scale_update(65536.0, 5, True)
    assert (s, c) == (32768.0, 0)
    s, c = 1024.0, 0
    for _ in range(1999):
        s, c = O.loss_scale_update(s, c, False)
    assert s == 1024.0 and c == 1999
    s, c = O.loss_scale_update(s, c, False)
    assert (s, c) == (2048.0, 0)


# ---------------------------------------------------------------- PSNR, Eq. 1
def test_psnr_eq1():
    r = [np.zeros((4, 4, 3)), np.zeros((2, 2, 3))]
    t = [np.full((4, 4, 3), 0.1), np.full((2, 2, 3), 0.1)]
    assert O.psnr(r, t) == pytest.approx(20.0, abs=1e-12)
    # errors only in the 2x2 mip: MSE = 4*3*0.25 / (3*(16+4)) = 0.05
    t = [np.zeros((4, 4, 3)), np.full((2, 2, 3), 0.5)]
    assert O.psnr(r, t) == pytest.approx(-10 * math.log10(0.05), abs=1e-12)


# ---------------------------------------------------------------- section 5.3 (filtering)
def _fq(u, v, lod):
    fq = np.zeros(len(u), dtype=O.FILTER_QUERY)
    fq["u"], fq["v"], fq["lod"] = u, v, lod
    return fq


def test_filter_bilinear_reproduces_position():
    """Bilinear weights reproduce an affine function of the texel position (interior):
    sum_k w_k x_k = u W - 1/2 and likewise in y, in the nearest mip; weights sum to 1."""
    g = O.make_geometry(256, 128, 4, 4, 4, 4, 4, Hd=16)
    r = np.random.default_rng(11)
    n = 2000
    lod = r.uniform(0, 3.4, n).astype(np.float32)
    u = r.uniform(0.1, 0.9, n).astype(np.float32)
    v = r.uniform(0.1, 0.9, n).astype(np.float32)
    q, w = O.filter_taps(g, _fq(u, v, lod), O.FILTER_BILINEAR)
    l = np.floor(lod.astype(np.float64) + 0.5).astype(np.int64)
    W = (256 >> l).astype(np.float64)
    H = (128 >> l).astype(np.float64)
    assert np.array_equal(q["lod"], np.repeat(l[:, None], 4, axis=1))
    xs = q["u"].astype(np.float64) * W[:, None] - 0.5
    ys = q["v"].astype(np.float64) * H[:, None] - 0.5
    assert np.allclose(w.sum(1), 1.0, atol=1e-15)
    assert np.allclose((w * xs).sum(1), u.astype(np.float64) * W - 0.5, atol=1e-9)
    assert np.allclose((w * ys).sum(1), v.astype(np.float64) * H - 0.5, atol=1e-9)


def test_filter_bilinear_at_texel_centre_is_point_decode():
    """At a texel centre the bilinear filter is that texel alone."""
    g = O.make_geometry(64, 64, 4, 4, 4, 4, 4, Hd=16)
    p = np.random.default_rng(2).standard_normal(O.mlp_param_count(g.K, g.Hd, g.C)) * 0.3
    lat = np.random.default_rng(3).uniform(-0.4, 0.4, g.latent_count)
    ix = np.arange(0, 64, 7)
    lod = np.zeros(len(ix), dtype=np.float32)
    u = ((ix + 0.5) / 64).astype(np.float32)
    got = O.decode_filtered(g, lat, p, _fq(u, u, lod), O.FILTER_BILINEAR)
    pq = np.zeros(len(ix), dtype=synth.QUERY_DTYPE)
    pq["u"], pq["v"] = u, u
    assert np.array_equal(got, O.decode(g, lat, p, pq))


def test_filter_trilinear_blend():
    """Trilinear at an integer LOD is bilinear in that mip; at LOD l + t it is
    (1 - t) bilinear(l) + t bilinear(l + 1)."""
    g = O.make_geometry(128, 128, 4, 4, 4, 4, 4, Hd=16)
    p = np.random.default_rng(5).standard_normal(O.mlp_param_count(g.K, g.Hd, g.C)) * 0.3
    lat = np.random.default_rng(6).uniform(-0.4, 0.4, g.latent_count)
    r = np.random.default_rng(7)
    u = r.uniform(0, 1, 300).astype(np.float32)
    v = r.uniform(0, 1, 300).astype(np.float32)
    li = r.integers(0, g.M - 1, 300).astype(np.float32)
    tri = O.decode_filtered(g, lat, p, _fq(u, v, li), O.FILTER_TRILINEAR)
    bil = O.decode_filtered(g, lat, p, _fq(u, v, li), O.FILTER_BILINEAR)
    assert np.allclose(tri, bil, atol=1e-14)
    t = np.float32(0.25)
    mid = O.decode_filtered(g, lat, p, _fq(u, v, li + t), O.FILTER_TRILINEAR)
    up = O.decode_filtered(g, lat, p, _fq(u, v, li + 1), O.FILTER_BILINEAR)
    assert np.allclose(mid, 0.75 * bil + 0.25 * up, atol=1e-12)


def test_stochastic_filter_is_bilinear_in_expectation():
    """Section 5.3: a uniform jitter of (-1/2, 1/2) texel followed by nearest sampling is
    bilinear filtering in expectation (each of the four texels is chosen with its
    bilinear weight); the mip is l0 + 1 with probability frac(lod); the jitter stays
    within half a texel."""
    g = O.make_geometry(64, 64, 4, 4, 4, 4, 4, Hd=16)
    n = 40000
    u0, v0, lod0 = np.float32(0.3), np.float32(0.61), np.float32(1.3)
    fq = _fq(np.full(n, u0), np.full(n, v0), np.full(n, lod0))
    q, w = O.filter_taps(g, fq, O.FILTER_STOCHASTIC, seed=9)
    assert np.all(w == 1.0)
    l = q["lod"][:, 0]
    p_up = np.mean(l == 2)
    assert set(np.unique(l)) <= {1, 2}
    assert abs(p_up - 0.3) < 5 * math.sqrt(0.3 * 0.7 / n)
    sel = l == 1
    Wl = 32
    x = q["u"][sel, 0].astype(np.float64) * Wl
    assert np.all(np.abs(x - float(u0) * Wl) <= 0.5)
    ix = np.floor(x).astype(np.int64)
    iy = np.floor(q["v"][sel, 0].astype(np.float64) * Wl).astype(np.int64)
    # expected: bilinear weights of the four texels around (u0 W - 1/2, v0 W - 1/2)
    gx, gy = float(u0) * Wl - 0.5, float(v0) * Wl - 0.5
    x0, y0 = math.floor(gx), math.floor(gy)
    fx, fy = gx - x0, gy - y0
    expect = {(x0, y0): (1 - fx) * (1 - fy), (x0 + 1, y0): fx * (1 - fy), (x0, y0 + 1): (1 - fx) * fy,
              (x0 + 1, y0 + 1): fx * fy}
    m = int(sel.sum())
    chi2 = 0.0
    for (a, b), pk in expect.items():
        cnt = np.sum((ix == a) & (iy == b))
        chi2 += (cnt - m * pk) ** 2 / (m * pk)
    assert np.sum(np.isin(ix, [x0, x0 + 1]) & np.isin(iy, [y0, y0 + 1])) == m
    assert chi2 < 16.3  # chi-square, 3 degrees of freedom, p = 0.001


def test_filter_randoms_are_splitmix_counters():
    """r1, r2, r3 of output 0 from the published SplitMix64 finalizer by hand."""
    def mix(z):
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9 & O.MASK64
        z = (z ^ (z >> 27)) * 0x94D049BB133111EB & O.MASK64
        return z ^ (z >> 31)
    key = mix((5 ^ 0x66696C74) & O.MASK64)
    h1 = mix((key + O.GAMMA) & O.MASK64)
    h2 = mix((key + 2 * O.GAMMA) & O.MASK64)
    r1, r2, r3 = O.filter_randoms(5, 1)
    assert float(r1[0]) == (h1 >> 40) * 2.0 ** -24
    assert float(r2[0]) == ((h1 >> 16) & 0xFFFFFF) * 2.0 ** -24
    assert float(r3[0]) == (h2 >> 40) * 2.0 ** -24
