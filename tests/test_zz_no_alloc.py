"""The allocation-free training step (static scratch array instead of a caller
workspace) against ntc_train_step, through the C ABI: two calls in a row on the same
states, the second with fewer samples (and another material size), FP32 and FP16.
The step is deterministic, so the states must be bit-identical."""
import numpy as np
import pytest

from _helpers import queries_dev, to_dev
from paper_2305_17105_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_17105_amd import ntc
    return ntc


KEYS = ("latents", "latents_fwd", "lat_grad", "mlp", "mlp_m", "mlp_v", "lat_m", "lat_v", "loss", "scale_state")


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_noalloc_step_equals_workspace_step(lib, prec):
    import torch
    P = lib.F32 if prec == "f32" else lib.F16
    calls = [(512, 12, 8192, 0), (256, 12, 3001, 1)]  # (side, channels, samples, step)
    for side, C, n, step in calls:
        m = lib.material_init(side, side, C, C, C, 4, 4, 64)
        raw = synth.uniform_latents(60 + side, int(m.latent_count))
        mlp = synth.xavier_mlp(60 + side, int(m.input_width), 64, C)
        _, tflat = synth.target_chain(60 + side, 0, side, side, C, int(m.num_mips))
        td = to_dev(tflat)
        q = queries_dev(synth.random_queries(61 + side, n, int(m.num_mips)))
        states = []
        for noalloc in (False, True):
            st = lib.TrainState(m, raw, to_dev(mlp), P)
            hp = lib.hparams(precision=P, step=step, lr_latent=0.01, lr_mlp=0.005, seed=12)
            lib.train_prepare(m, st, hp)
            if noalloc:
                lib.train_step_noalloc(m, st, q, n, td, hp)
            else:
                ws = torch.empty(lib.train_workspace_bytes(m, n, P), dtype=torch.uint8, device="cuda")
                lib.train_step(m, st, q, n, td, hp, ws)
            torch.cuda.synchronize()
            states.append(st)
        for k in KEYS:
            a, b = getattr(states[0], k), getattr(states[1], k)
            assert torch.equal(a, b), (side, n, k)
        assert float(states[1].loss.cpu()[0]) > 0.0
