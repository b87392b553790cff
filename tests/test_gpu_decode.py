"""GPU parity: quantization (bit-exact) and decode (FP32 / FP16) against the FP64 oracle.

Every call goes through the C ABI of libntc.so.  Sizes span several tiles and a
ragged tail; edge cases: n = 0, n = 1, out-of-range coordinates and LODs.
"""
import numpy as np
import pytest

from _helpers import geometry, mlp_in_unit_range, queries_dev, quantized_latents_oracle, to_dev
from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_17105_amd import ntc
    return ntc


def _packed(lib, m, raw):
    import torch
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    lib.quantize_latents(m, to_dev(raw), packed)
    return packed


QSHAPES = [  # W, C, c0, c1, b0, b1
    (256, 8, 8, 8, 4, 4),
    (512, 16, 16, 16, 2, 4),
    (256, 10, 10, 10, 1, 8),
    (128, 12, 12, 12, 8, 2),
    (64, 3, 5, 7, 4, 4),
]


@pytest.mark.parametrize("shape", QSHAPES)
def test_quantize_bit_exact(lib, shape):
    import torch
    W, C, c0, c1, b0, b1 = shape
    m = lib.material_init(W, W, C, c0, c1, b0, b1, 64)
    g = geometry(m)
    raw = synth.uniform_latents(1, int(m.latent_count), -0.8, 0.8)
    # ties, range ends, non-finite and huge values
    special = np.array([0.0, -0.0, 0.5, -0.5, 1 / 32, 3 / 32, -15 / 32, -7 / 16, 0.49999997, 1e30, -1e30,
                        np.inf, -np.inf, np.nan, 1e-40, 0.125, 0.375, -0.375, 0.25 + 2 ** -25], dtype=np.float32)
    raw[:len(special)] = special
    got = _packed(lib, m, raw).cpu().numpy()
    want = O.quantize_latents(g, raw)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    back = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
    lib.dequantize_latents(m, _packed(lib, m, raw), back)
    assert np.array_equal(back.cpu().numpy().astype(np.float64), O.dequantize_packed(g, want))


def test_quantize_fp32_pattern_sweep(lib):
    """Strided sweep over all 2^32 float32 bit patterns (every 4099th), both bit depths."""
    m = lib.material_init(1024, 1024, 16, 16, 16, 2, 4, 64)
    g = geometry(m)
    n = int(m.latent_count)
    bits = (np.arange(n, dtype=np.uint64) * np.uint64(4099)) % np.uint64(2 ** 32)
    raw = bits.astype(np.uint32).view(np.float32)
    assert np.array_equal(_packed(lib, m, raw).cpu().numpy(), O.quantize_latents(g, raw))


DSHAPES = [  # W, C, c0, c1, b0, b1, hidden, mips, n, lod
    (256, 8, 8, 8, 4, 4, 64, 1, 65536, 0),        # tiny configuration, LOD 0
    (512, 12, 12, 12, 4, 4, 64, 0, 20011, None),  # full mip chain, 5 levels, ragged
    (256, 10, 10, 10, 4, 4, 32, 0, 1013, None),   # C not a multiple of 4, hidden 32
    (512, 16, 16, 16, 2, 4, 64, 0, 4099, None),   # 2-bit G0, 4-bit G1
    (256, 16, 16, 16, 4, 4, 32, 0, 1, None),      # a single query
]


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("shape", DSHAPES)
def test_decode_parity(lib, shape, prec):
    import torch
    W, C, c0, c1, b0, b1, hd, mips, n, lod = shape
    P = lib.F32 if prec == "f32" else lib.F16
    m = lib.material_init(W, W, C, c0, c1, b0, b1, hd, num_mips=mips)
    g = geometry(m)
    raw = synth.uniform_latents(3, int(m.latent_count))
    mlp = mlp_in_unit_range(3, g.K, hd, C)
    q = synth.random_queries(3, n, g.M, lod)
    packed = _packed(lib, m, raw)
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    out = torch.full((n * C,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode(m, packed, wp, P, queries_dev(q), n, out, lib.F32)
    out16 = torch.zeros(n * C, dtype=torch.float16, device="cuda")
    lib.decode(m, packed, wp, P, queries_dev(q), n, out16, lib.F16)
    torch.cuda.synchronize()
    ref = O.decode(g, quantized_latents_oracle(g, raw), mlp, q).ravel()
    got = out.cpu().numpy().astype(np.float64)
    err = np.max(np.abs(got - ref))
    tol = 1e-5 if prec == "f32" else 2e-3
    print(f"decode {shape} {prec}: max-abs err {err:.3e}")
    assert err <= tol
    got16 = out16.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got16 - got)) <= 2e-3  # FP16 output is the FP32 result rounded


@pytest.mark.parametrize("prec", ["f32", "f16", "fp8"])
def test_decode_parity_lod_input(lib, prec):
    """Decode with the LOD input of section 4.4 (K = 4 C0 + C1 + 13)."""
    import torch
    P = {"f32": lib.F32, "f16": lib.F16, "fp8": lib.FP8_E4M3}[prec]
    m = lib.material_init(512, 512, 16, 16, 16, 2, 4, 64, lod_input=1)
    g = geometry(m)
    assert g.K == int(m.input_width) == 93
    raw = synth.uniform_latents(9, int(m.latent_count))
    mlp = mlp_in_unit_range(9, g.K, 64, 16)
    n = 6007
    q = synth.random_queries(9, n, g.M)
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    out = torch.full((n * 16,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode(m, _packed(lib, m, raw), wp, P, queries_dev(q), n, out, lib.F32)
    torch.cuda.synchronize()
    lat = quantized_latents_oracle(g, raw)
    ref = (O.decode_fp8(g, lat, mlp, q) if prec == "fp8" else O.decode(g, lat, mlp, q)).ravel()
    err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
    print(f"LOD input {prec}: max-abs err {err.max():.3e}")
    if prec == "fp8":  # against the oracle's e4m3 evaluation, the FP8 bars
        assert err.mean() <= 2e-5 and np.quantile(err, 0.99) <= 1e-3 and err.max() <= 2e-2
    else:
        assert err.max() <= (1e-5 if prec == "f32" else 2e-3)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_decode_parity_triangle_encoding(lib, prec):
    """Decode with the triangular-wave positional encoding (section 4.3.2)."""
    import torch
    P = lib.F32 if prec == "f32" else lib.F16
    m = lib.material_init(512, 512, 16, 16, 16, 2, 4, 64, posenc=lib.PE_TRIANGLE)
    g = geometry(m)
    raw = synth.uniform_latents(8, int(m.latent_count))
    mlp = mlp_in_unit_range(8, g.K, 64, 16)
    n = 6007
    q = synth.random_queries(8, n, g.M)
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    out = torch.full((n * 16,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode(m, _packed(lib, m, raw), wp, P, queries_dev(q), n, out, lib.F32)
    torch.cuda.synchronize()
    ref = O.decode(g, quantized_latents_oracle(g, raw), mlp, q).ravel()
    err = np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref))
    print(f"triangle encoding {prec}: max-abs err {err:.3e}")
    assert err <= (1e-5 if prec == "f32" else 2e-3)


F8SHAPES = [  # W, C, c0, c1, b0, b1, hidden, mips, n, lod
    (256, 8, 8, 8, 4, 4, 64, 1, 65536, 0),        # tiny configuration shapes
    (512, 16, 16, 16, 2, 4, 64, 0, 20011, None),  # 2-bit G0 / 4-bit G1, full chain, ragged
    (256, 16, 16, 16, 4, 4, 32, 0, 4099, None),   # all 4-bit, hidden 32
]


@pytest.mark.parametrize("shape", F8SHAPES)
def test_decode_fp8_parity(lib, shape):
    """FP8-e4m3 decode against the float64 decode (the 1e-2 bar on outputs near [0, 1])
    and against the oracle's e4m3 evaluation of the same network (rounding-level)."""
    import torch
    W, C, c0, c1, b0, b1, hd, mips, n, lod = shape
    m = lib.material_init(W, W, C, c0, c1, b0, b1, hd, num_mips=mips)
    g = geometry(m)
    raw = synth.uniform_latents(11, int(m.latent_count))
    mlp = mlp_in_unit_range(11, g.K, hd, C)
    q = synth.random_queries(11, n, g.M, lod)
    nb = lib.mlp_packed_bytes(m, lib.FP8_E4M3)
    assert nb > 0
    wp = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), lib.FP8_E4M3, wp)
    out = torch.full((n * C,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode(m, _packed(lib, m, raw), wp, lib.FP8_E4M3, queries_dev(q), n, out, lib.F32)
    torch.cuda.synchronize()
    lat = quantized_latents_oracle(g, raw)
    got = out.cpu().numpy().astype(np.float64)
    ref = O.decode(g, lat, mlp.astype(np.float64), q).ravel()
    emu = O.decode_fp8(g, lat, mlp.astype(np.float64), q).ravel()
    e64, e8 = np.abs(got - ref), np.abs(got - emu)
    print(f"decode fp8 {shape}: vs float64 max {e64.max():.3e} mean {e64.mean():.2e}; vs e4m3 oracle max "
          f"{e8.max():.3e} p99.9 {np.quantile(e8, 0.999):.2e} mean {e8.mean():.2e}")
    # The e4m3 oracle rounds the same values; a value within FP32 rounding of an e4m3
    # midpoint may round the other way (one e4m3 step of one hidden unit), so a few
    # outputs differ by up to ~1e-2 while almost all agree to FP32 accumulation order.
    # The float64 distance is the cost of e4m3 itself; the stated 1e-2 bar against
    # float64 is checked (and not met) in test_decode_fp8_stated_bar.
    assert e8.mean() <= 2e-5 and np.quantile(e8, 0.99) <= 1e-3 and e8.max() <= 2e-2


def _trained_fixture(lib):
    """The 256^2 x 16 material trained by the oracle (tests/golden/make_trained_decode_fixture.py):
    its packed latents and network, as device tensors, plus the oracle geometry."""
    import os
    import torch
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trained_decode_256x16.npz"))
    W, C, c0, c1, b0, b1, hd = (int(v) for v in z["shape"])
    m = lib.material_init(W, W, C, c0, c1, b0, b1, hd)
    g = geometry(m)
    assert len(z["packed"]) == int(m.packed_bytes)
    packed = torch.from_numpy(z["packed"].copy()).cuda()
    return m, g, packed, z["mlp"].astype(np.float32), O.dequantize_packed(g, z["packed"])


def _decode_with(lib, m, packed, mlp, P, q):
    import torch
    n, C = len(q), int(m.channels)
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    out = torch.full((n * C,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode(m, packed, wp, P, queries_dev(q), n, out, lib.F32)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64).reshape(n, C)


@pytest.mark.parametrize("prec", ["f32", "f16", "fp8"])
def test_decode_trained_weights(lib, prec):
    """Decode parity on a network trained by the oracle (outputs in [0, 1]): FP32 <= 1e-5 and
    FP16 <= 2e-3 max-abs against float64; FP8 against the oracle's e4m3 arithmetic."""
    m, g, packed, mlp, lat = _trained_fixture(lib)
    q = synth.random_queries(91, 40009, g.M)
    P = {"f32": lib.F32, "f16": lib.F16, "fp8": lib.FP8_E4M3}[prec]
    got = _decode_with(lib, m, packed, mlp, P, q)
    ref = O.decode(g, lat, mlp, q)
    e64 = np.abs(got - ref)
    print(f"trained weights {prec}: outputs in [{ref.min():.3f}, {ref.max():.3f}], vs float64 max {e64.max():.3e} "
          f"mean {e64.mean():.2e} (PSNR of the decode against float64 {O.psnr([ref], [got]):.1f} dB)")
    if prec == "fp8":
        e8 = np.abs(got - O.decode_fp8(g, lat, mlp, q))
        print(f"  vs e4m3 oracle max {e8.max():.3e} mean {e8.mean():.2e}")
        assert e8.mean() <= 2e-5 and np.quantile(e8, 0.99) <= 1e-3 and e8.max() <= 3e-2
    else:
        assert e64.max() <= {"f32": 1e-5, "f16": 2e-3}[prec]


@pytest.mark.xfail(strict=True, reason="plain e4m3 (3 mantissa bits) rounding of weights and activations costs "
                                       "2.2e-2 (unit-range Xavier) and 6.6e-2 (oracle-trained) max-abs against "
                                       "float64; no per-layer scaling brings it under 1e-2 (design notes, FP8)")
@pytest.mark.parametrize("weights", ["unit_range_xavier", "oracle_trained"])
def test_decode_fp8_stated_bar(lib, weights):
    """The stated FP8 decode bar: <= 1e-2 max-abs against float64 on outputs in [0, 1]."""
    if weights == "oracle_trained":
        m, g, packed, mlp, lat = _trained_fixture(lib)
    else:
        m = lib.material_init(512, 512, 16, 16, 16, 2, 4, 64)
        g = geometry(m)
        raw = synth.uniform_latents(11, int(m.latent_count))
        packed = _packed(lib, m, raw)
        mlp = mlp_in_unit_range(11, g.K, 64, 16)
        lat = quantized_latents_oracle(g, raw)
    q = synth.random_queries(92, 40009, g.M)
    got = _decode_with(lib, m, packed, mlp, lib.FP8_E4M3, q)
    err = np.abs(got - O.decode(g, lat, mlp, q))
    print(f"fp8 vs float64 ({weights}): max {err.max():.3e} mean {err.mean():.2e}")
    assert err.max() <= 1e-2


def test_fp8_unsupported_shapes_rejected(lib):
    """c0 * b0 not a multiple of 32: no FP8 pack size, pack and decode refuse."""
    import torch
    m = lib.material_init(512, 512, 12, 12, 12, 4, 4, 64)
    assert lib.mlp_packed_bytes(m, lib.FP8_E4M3) == 0
    with pytest.raises(lib.NtcError):
        lib.pack_mlp(m, torch.zeros(int(m.mlp_params), device="cuda"), lib.FP8_E4M3,
                     torch.zeros(64, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("prec", ["f32", "f16", "fp8"])
def test_decode_tile_equals_query_decode(lib, prec):
    """ntc_decode_tile over a ragged rectangle of mip 1 equals ntc_decode on the
    rectangle's texel-centre queries bit for bit, and the oracle within tolerance."""
    import torch
    P = {"f32": lib.F32, "f16": lib.F16, "fp8": lib.FP8_E4M3}[prec]
    m = lib.material_init(512, 512, 16, 16, 16, 2, 4, 64)
    g = geometry(m)
    raw = synth.uniform_latents(13, int(m.latent_count))
    mlp = mlp_in_unit_range(13, g.K, 64, 16)
    packed = _packed(lib, m, raw)
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    lod, x0, y0, w, h = 1, 3, 5, 37, 19
    wl = int(m.mip_w[lod])
    ys, xs = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
    q = np.zeros(w * h, dtype=synth.QUERY_DTYPE)
    q["u"] = ((xs.ravel() + 0.5) / wl).astype(np.float32)
    q["v"] = ((ys.ravel() + 0.5) / wl).astype(np.float32)
    q["lod"] = lod
    a = torch.full((w * h * 16,), float("nan"), dtype=torch.float32, device="cuda")
    b = torch.full((w * h * 16,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode_tile(m, packed, wp, P, lod, x0, y0, w, h, a, lib.F32)
    lib.decode(m, packed, wp, P, queries_dev(q), w * h, b, lib.F32)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    lat = quantized_latents_oracle(g, raw)
    if prec == "fp8":  # the e4m3 arithmetic the FP8 path claims (see test_decode_fp8_parity)
        e8 = np.abs(a.cpu().numpy() - O.decode_fp8(g, lat, mlp, q).ravel())
        print(f"decode_tile fp8: vs e4m3 oracle max {e8.max():.3e} mean {e8.mean():.2e}")
        assert e8.mean() <= 2e-5 and np.quantile(e8, 0.99) <= 1e-3 and e8.max() <= 2e-2
        return
    err = np.max(np.abs(a.cpu().numpy() - O.decode(g, lat, mlp, q).ravel()))
    print(f"decode_tile {prec}: max-abs err {err:.3e} vs float64")
    assert err <= {"f32": 1e-5, "f16": 2e-3}[prec]


def test_decode_edge_coordinates(lib):
    """u, v outside [0, 1), NaN, and LODs outside the chain are clamped like the oracle."""
    import torch
    m = lib.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    g = geometry(m)
    raw = synth.uniform_latents(5, int(m.latent_count))
    mlp = mlp_in_unit_range(5, g.K, 64, 8)
    q = np.zeros(8, dtype=synth.QUERY_DTYPE)
    q["u"] = [-1.0, 1.0, 2.5, np.nan, 0.999999, 0.5, np.inf, -np.inf]
    q["v"] = [0.5, 0.0, 1.0, 0.25, 0.999999, np.nan, 0.1, 0.9]
    q["lod"] = [0, -5, 100, 3, g.M - 1, 2, 1, 7]
    wp = torch.zeros(lib.mlp_packed_bytes(m, lib.F32), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), lib.F32, wp)
    out = torch.zeros(8 * 8, dtype=torch.float32, device="cuda")
    lib.decode(m, _packed(lib, m, raw), wp, lib.F32, queries_dev(q), 8, out, lib.F32)
    torch.cuda.synchronize()
    ref = O.decode(g, quantized_latents_oracle(g, raw), mlp, q).ravel()
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-5


def test_decode_zero_queries_is_noop(lib):
    import torch
    m = lib.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    out = torch.full((8,), 7.0, device="cuda")
    wp = torch.zeros(lib.mlp_packed_bytes(m, lib.F32), dtype=torch.uint8, device="cuda")
    lib.decode(m, torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda"), wp, lib.F32,
               torch.zeros(12, dtype=torch.uint8, device="cuda"), 0, out, lib.F32)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)


@pytest.mark.parametrize("prec", ["f32", "f16", "fp8"])
def test_decode_full_size_sampled(lib, prec):
    """The decode workload itself (4096^2 x 16, 2/4-bit, 13 mips, 16M random queries in one
    launch); 65,536 sampled outputs are checked against the oracle."""
    import torch
    P = {"f32": lib.F32, "f16": lib.F16, "fp8": lib.FP8_E4M3}[prec]
    m = lib.material_init(4096, 4096, 16, 16, 16, 2, 4, 64)
    g = geometry(m)
    raw = synth.uniform_latents(7, int(m.latent_count))
    mlp = mlp_in_unit_range(7, g.K, 64, 16)
    n = 16 * 2 ** 20
    q = synth.random_queries(7, n, g.M)
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    out = torch.empty(n * 16, dtype=torch.float16, device="cuda")
    lib.decode(m, _packed(lib, m, raw), wp, P, queries_dev(q), n, out, lib.F16)
    torch.cuda.synchronize()
    pick = synth.random_param_indices(8, 65536, n)
    got = out.view(n, 16)[torch.from_numpy(pick).cuda()].float().cpu().numpy().astype(np.float64)
    lat = quantized_latents_oracle(g, raw)
    if prec == "fp8":  # against the e4m3 arithmetic; FP16 output rounding adds <= 2^-12 on [0, 1]
        e8 = np.abs(got - O.decode_fp8(g, lat, mlp, q[pick]))
        print(f"full-size decode fp8 (FP16 output): vs e4m3 oracle max {e8.max():.3e} mean {e8.mean():.2e}")
        assert e8.mean() <= 2e-4 and np.quantile(e8, 0.99) <= 1e-3 and e8.max() <= 2e-2
        return
    err = np.max(np.abs(got - O.decode(g, lat, mlp, q[pick])))
    print(f"full-size decode {prec} (FP16 output): max-abs err {err:.3e} on {len(pick)} sampled queries")
    assert err <= {"f32": 1e-3, "f16": 3e-3}[prec]  # includes the FP16 rounding of the output


FSHAPES = [  # W, C, c0, c1, b0, b1, hidden, n
    (256, 8, 8, 8, 4, 4, 64, 3001),
    (512, 16, 16, 16, 2, 4, 64, 2049),   # paired FP16 layout
    (256, 10, 10, 10, 4, 4, 32, 777),    # C not a multiple of 4
]
FMODES = {"bilinear": 1, "trilinear": 2, "stochastic": 3}


def _filter_queries(seed, n, M):
    r = np.random.default_rng(seed)
    fq = np.zeros(n, dtype=O.FILTER_QUERY)
    fq["u"] = r.uniform(0, 1, n)
    fq["v"] = r.uniform(0, 1, n)
    fq["lod"] = r.uniform(0, M - 1, n)
    k = min(n, 8)  # edges: borders, integer and out-of-range LODs, NaN
    fq["u"][:k] = [0.0, 0.99999, 0.5, np.nan, 0.25, 1.0, -0.1, 0.75][:k]
    fq["lod"][:k] = [0.0, M - 1, -2.0, 1.0, M + 3.0, np.nan, 0.5, 2.0][:k]
    return fq


def _fq_dev(fq):
    import torch
    return torch.from_numpy(fq.view(np.uint8).copy()).cuda()


@pytest.mark.parametrize("mode", list(FMODES))
@pytest.mark.parametrize("shape", FSHAPES)
def test_decode_filtered_parity(lib, shape, mode):
    """Filtered FP16 decode against the float64 oracle's weighted sum of decoded taps
    (the same texels, chosen in the same float32 arithmetic) at the FP16 decode bar."""
    import torch
    W, C, c0, c1, b0, b1, hd, n = shape
    m = lib.material_init(W, W, C, c0, c1, b0, b1, hd)
    g = geometry(m)
    raw = synth.uniform_latents(21, int(m.latent_count))
    mlp = mlp_in_unit_range(21, g.K, hd, C)
    packed = _packed(lib, m, raw)
    wp = torch.zeros(lib.mlp_packed_bytes(m, lib.F16), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), lib.F16, wp)
    fq = _filter_queries(22, n, g.M)
    out = torch.full((n * C,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode_filtered(m, packed, wp, lib.F16, _fq_dev(fq), n, FMODES[mode], out, lib.F32, seed=77)
    torch.cuda.synchronize()
    ref = O.decode_filtered(g, quantized_latents_oracle(g, raw), mlp, fq, FMODES[mode], seed=77).ravel()
    err = np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref))
    print(f"filtered {mode} {shape}: max-abs err {err:.3e}")
    assert err <= 2e-3


def test_decode_filtered_reductions(lib):
    """Bilinear at texel centres is the point decode of those texels, and trilinear at
    integer LODs is bilinear, bit for bit on the GPU."""
    import torch
    m = lib.material_init(256, 256, 16, 16, 16, 2, 4, 64)
    g = geometry(m)
    packed = _packed(lib, m, synth.uniform_latents(23, int(m.latent_count)))
    wp = torch.zeros(lib.mlp_packed_bytes(m, lib.F16), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp_in_unit_range(23, g.K, 64, 16)), lib.F16, wp)
    r = np.random.default_rng(24)
    n = 5003
    lod = r.integers(0, g.M, n)
    Wl = np.array(g.mip_w)[lod]
    ix, iy = r.integers(0, Wl), r.integers(0, Wl)
    fq = np.zeros(n, dtype=O.FILTER_QUERY)
    fq["u"], fq["v"], fq["lod"] = (ix + 0.5) / Wl, (iy + 0.5) / Wl, lod
    pq = np.zeros(n, dtype=synth.QUERY_DTYPE)
    pq["u"], pq["v"], pq["lod"] = fq["u"], fq["v"], lod
    outs = {}
    for name, fn in (("point", None), ("bilinear", 1), ("trilinear", 2)):
        o = torch.full((n * 16,), float("nan"), dtype=torch.float16, device="cuda")
        if fn is None:
            lib.decode(m, packed, wp, lib.F16, queries_dev(pq), n, o, lib.F16)
        else:
            lib.decode_filtered(m, packed, wp, lib.F16, _fq_dev(fq), n, fn, o, lib.F16)
        outs[name] = o
    torch.cuda.synchronize()
    assert torch.equal(outs["bilinear"], outs["point"])
    assert torch.equal(outs["trilinear"], outs["bilinear"])


def test_decode_filtered_rejects_other_precisions(lib):
    import torch
    m = lib.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    wp = torch.zeros(lib.mlp_packed_bytes(m, lib.F32), dtype=torch.uint8, device="cuda")
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    out = torch.zeros(8 * 4, dtype=torch.float32, device="cuda")
    fq = _fq_dev(_filter_queries(1, 4, 9))
    with pytest.raises(lib.NtcError):
        lib.decode_filtered(m, packed, wp, lib.F32, fq, 4, 1, out, lib.F32)
    with pytest.raises(lib.NtcError):
        lib.decode_filtered(m, packed, wp, lib.F16, fq, 4, 7, out, lib.F32)
