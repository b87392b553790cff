"""GPU parity of Table 3's four compression profiles against the FP64 oracle, through
the C ABI, on a 9-channel texture set (the table's reference set is 4096^2 x 9):

  NTC 0.2   G0 at W/4, 8 x 2-bit,  G1 12 x 4-bit
  NTC 0.5   G0 at W/4, 12 x 4-bit, G1 20 x 4-bit
  NTC 1.0   G0 at W/2, 12 x 2-bit, G1 10 x 4-bit
  NTC 2.25  G0 at W/2, 16 x 4-bit, G1 12 x 4-bit

with the paper's network (section 4.4): two hidden layers of 64, hardGELU, the LOD input
and the triangular-wave positional encoding of section 4.3.2.  Decode (FP32, FP16) and
training gradients (FP32, FP16) on 256^2 materials with their full mip chains.
"""
import numpy as np
import pytest

from _helpers import geometry, mlp_in_unit_range, queries_dev, quantized_latents_oracle, to_dev
from _trainrun import Run, check_grads, fp16_grad_errors
from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth

pytestmark = pytest.mark.gpu

# name: (c0, b0, c1, b1, grid_shift)
PROFILES = {
    "NTC0.2": (8, 2, 12, 4, 2),
    "NTC0.5": (12, 4, 20, 4, 2),
    "NTC1.0": (12, 2, 10, 4, 1),
    "NTC2.25": (16, 4, 12, 4, 1),
}
C = 9


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_17105_amd import ntc
    return ntc


def _paper_net(lib):
    return dict(activation=lib.ACT_HARDGELU, lod_input=1, posenc=lib.PE_TRIANGLE)


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("name", list(PROFILES))
def test_profile_decode(lib, name, prec):
    import torch
    c0, b0, c1, b1, sh = PROFILES[name]
    P = lib.F32 if prec == "f32" else lib.F16
    m = lib.material_init(256, 256, C, c0, c1, b0, b1, 64, grid_shift=sh, **_paper_net(lib))
    assert lib.shape_supported(m, True) and lib.shape_supported(m, False)
    g = geometry(m)
    assert g.K == 4 * c0 + c1 + 12 + 1 == int(m.input_width)
    seed = 70 + c0 + c1
    raw = synth.uniform_latents(seed, int(m.latent_count))
    mlp = mlp_in_unit_range(seed, g.K, 64, C)
    n = 6007  # ragged: 375 tiles of 16 and a tail of 7
    q = synth.random_queries(seed, n, g.M)
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    lib.quantize_latents(m, to_dev(raw), packed)
    assert np.array_equal(packed.cpu().numpy(), O.quantize_latents(g, raw))
    wp = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp(m, to_dev(mlp), P, wp)
    out = torch.full((n * C,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode(m, packed, wp, P, queries_dev(q), n, out, lib.F32)
    torch.cuda.synchronize()
    ref = O.decode(g, quantized_latents_oracle(g, raw), mlp, q).ravel()
    err = float(np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)))
    print(f"{name} decode {prec}: max-abs err {err:.3e} (outputs in [{ref.min():.2f}, {ref.max():.2f}])")
    assert err <= (1e-5 if prec == "f32" else 2e-3)


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("name", list(PROFILES))
def test_profile_gradients(lib, name, prec):
    c0, b0, c1, b1, sh = PROFILES[name]
    P = lib.F32 if prec == "f32" else lib.F16
    run = Run(lib, 256, C, c0, c1, b0, b1, 64, 0, 8191, None, seed=90 + c0 + c1, prec=P, grid_shift=sh,
              **_paper_net(lib))
    assert run.g.act == "hardgelu"
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=True, seed=7)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    if prec == "f32":
        check_grads(run, hp)
    else:
        # hardGELU has no ReLU decisions to match: FP16 rounding alone separates the two
        errs, _, lerr = fp16_grad_errors(run, hp)
        print(f"{name} fp16 vs float64:", {k: f"{v:.2e}" for k, v in errs.items()}, f"loss {lerr:.2e}")
        assert lerr <= 2e-3
        for k, v in errs.items():
            assert v <= 1e-2, (k, v)
