"""GPU parity of the training step (FP32 path) against the FP64 oracle, via the C ABI.

Gradients are read back without any debug hook: a step with learning rate 0 leaves
the parameters unchanged and sets the first Adam moment to (1 - beta1) * gradient.
"""
import numpy as np
import pytest

from _helpers import geometry, queries_dev, rel_err, to_dev
from _trainrun import Run, check_grads as _check_grads, grad_groups as _grad_groups, ohp as _ohp
from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_17105_amd import ntc
    return ntc


CONFIGS = {  # W, C, c0, c1, b0, b1, hidden, mips, n, lod
    "tiny": (256, 8, 8, 8, 4, 4, 64, 1, 65536, 0),
    "chain": (512, 12, 12, 12, 4, 4, 64, 0, 30011, None),
    "ragged32": (256, 10, 10, 10, 4, 4, 32, 0, 4097, None),
    "c16": (256, 16, 16, 16, 2, 4, 64, 0, 2049, None),
}


@pytest.mark.parametrize("name", list(CONFIGS))
def test_gradients_fp32(lib, name):
    run = Run(lib, *CONFIGS[name])
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=False)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    _check_grads(run, hp)
    # lr = 0: parameters unchanged
    assert np.array_equal(run.get("latents"), run.ostate["latents"])
    assert np.array_equal(run.get("mlp"), run.ostate["mlp"])


def test_gradients_triangle_encoding(lib):
    """The triangular-wave positional encoding (section 4.3.2) through the training step."""
    run = Run(lib, *CONFIGS["chain"], seed=6, posenc=lib.PE_TRIANGLE)
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=False)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    _check_grads(run, hp)


@pytest.mark.parametrize("name", ["chain", "ragged32"])
def test_gradients_lod_input(lib, name):
    """Training gradients with the LOD input of section 4.4 (its W1 row included)."""
    run = Run(lib, *CONFIGS[name], seed=7, lod_input=1)
    assert run.g.K == int(run.m.input_width)
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=False)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    _check_grads(run, hp)


def test_gradients_with_noise(lib):
    run = Run(lib, *CONFIGS["chain"], seed=4)
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=True, seed=1234, step=7)
    lib.train_prepare(run.m, run.state, hp)
    # forward latents = masters + this step's counter-hash noise, as the oracle draws it
    want = run.ostate["latents"] + O.noise_values(run.g, 1234, 7)
    assert np.max(np.abs(run.get("latents_fwd") - want)) <= 1e-7
    run.step(hp)
    _check_grads(run, hp)
    # after the step: forward latents hold the noise of step 8
    want = run.ostate["latents"] + O.noise_values(run.g, 1234, 8)
    assert np.max(np.abs(run.get("latents_fwd") - want)) <= 1e-7


def _compare_step(run, new, gp, gl, lr):
    """Post-step parameters.  Adam's first step moves by ~lr*sign(g); entries whose
    gradient is within rounding of zero may legitimately take either sign."""
    for name, key, grad in (("latents", "latents", gl), ("mlp", "mlp", gp)):
        got = run.get(key)
        want = new[key]
        sure = np.abs(grad) > 1e-5 * np.sqrt(np.mean(grad ** 2)) + 1e-12
        err = np.max(np.abs(got - want)[sure]) if sure.any() else 0.0
        loose = np.max(np.abs(got - want)[~sure]) if (~sure).any() else 0.0
        print(f"{name}: max-abs err {err:.3e} on {sure.sum()} entries; {int((~sure).sum())} near-zero-gradient entries "
              f"(max {loose:.2e})")
        assert err <= 1e-5
        assert loose <= 2 * lr + 1e-6


@pytest.mark.parametrize("name", ["tiny", "chain"])
def test_one_adam_step_fp32(lib, name):
    """One full step at lr 1e-2 (tiny configuration: one Adam step at lr 1e-2)."""
    run = Run(lib, *CONFIGS[name], seed=2)
    hp = run.hp(lr_latent=1e-2, lr_mlp=1e-2, noise=name == "chain", seed=9)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    new, L, ovf = O.train_step(run.g, run.ostate, run.q, run.targets, _ohp(hp))
    lat_fwd = run.ostate["latents"] + (O.noise_values(run.g, 9, 0) if hp.noise else 0)
    _, gp, gl, _ = O.loss_and_grads(run.g, lat_fwd, run.ostate["mlp"], run.q, run.targets)
    assert not ovf
    assert abs(run.get("loss")[0] - L) <= 1e-5 * L
    _compare_step(run, new, gp, gl, 1e-2)
    lo, hi = O.quant_range(4)
    lat = run.get("latents")
    assert lat.min() >= min(lo, O.quant_range(run.g.B0)[0]) - 1e-7 and lat.max() <= 0.5


def test_three_steps_loss_trajectory(lib):
    run = Run(lib, *CONFIGS["chain"], seed=6)
    st = run.ostate
    hp0 = run.hp(lr_latent=1e-2, lr_mlp=5e-3, noise=True, seed=3, step=0)
    lib.train_prepare(run.m, run.state, hp0)
    for t in range(3):
        hp = run.hp(lr_latent=1e-2, lr_mlp=5e-3, noise=True, seed=3, step=t)
        run.step(hp)
        st, L, _ = O.train_step(run.g, st, run.q, run.targets, _ohp(hp))
        got = run.get("loss")[0]
        print(f"step {t}: loss {got:.7e} oracle {L:.7e}")
        assert abs(got - L) <= 1e-4 * L


def test_freeze_latents(lib):
    run = Run(lib, *CONFIGS["ragged32"], seed=8)
    hp = run.hp(lr_latent=1e-2, lr_mlp=1e-2, noise=True, freeze=True)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    new, L, _ = O.train_step(run.g, run.ostate, run.q, run.targets, _ohp(hp))
    assert np.array_equal(run.get("latents"), run.ostate["latents"])
    assert np.array_equal(run.get("latents_fwd"), run.ostate["latents"])
    assert not run.get("lat_m").any()
    assert abs(run.get("loss")[0] - L) <= 1e-5 * L
    _, gp, _, _ = O.loss_and_grads(run.g, run.ostate["latents"], run.ostate["mlp"], run.q, run.targets)
    _compare_step(run, dict(new, latents=run.ostate["latents"]), gp, np.zeros(run.g.latent_count), 1e-2)


def test_nonfinite_gradient_skips_step(lib):
    run = Run(lib, *CONFIGS["ragged32"], seed=9)
    hp = run.hp(lr_latent=1e-2, lr_mlp=1e-2, noise=False)
    lib.train_prepare(run.m, run.state, hp)
    bad = run.targets.copy()
    bad[:50] = np.inf
    q = synth.tile_queries(256, 256)[:2000]
    run.step(hp, q=q, n=len(q), targets=to_dev(bad))
    _, _, ovf = O.train_step(run.g, run.ostate, q, bad, _ohp(hp))
    assert ovf
    assert run.get("scale_state")[1] == 1
    assert np.array_equal(run.get("latents"), run.ostate["latents"])
    assert np.array_equal(run.get("mlp"), run.ostate["mlp"])
    # the next good step clears the flag
    run.step(run.hp(lr_latent=1e-2, lr_mlp=1e-2, noise=False, step=1))
    assert run.get("scale_state")[1] == 0


@pytest.mark.parametrize("name,lod_input", [("tiny", 0), ("chain", 0), ("c16", 0), ("ragged32", 0), ("chain", 1)])
def test_gradients_fp16(lib, name, lod_input):
    """FP16 matrix-core forward and backward, FP32 accumulation, loss scale 2^16 (and
    with the LOD input of section 4.4)."""
    run = Run(lib, *CONFIGS[name], seed=12, prec=lib.F16, lod_input=lod_input)
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=True, seed=2)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    g = run.g
    lat_fwd = run.ostate["latents"] + O.noise_values(g, 2, 0)
    L, gp, gl, _ = O.loss_and_grads(g, lat_fwd, run.ostate["mlp"], run.q, run.targets)
    gp_gpu = run.get("mlp_m") / (1 - hp.beta1)
    gl_gpu = run.get("lat_m") / (1 - hp.beta1)
    errs = {k: rel_err(_grad_groups(g, gp_gpu)[k], v) for k, v in _grad_groups(g, gp).items()}
    errs["latents"] = rel_err(gl_gpu, gl)
    errs["lat_grad"] = rel_err(run.get("lat_grad") / run.get("loss_scale")[0], gl)
    loss = run.get("loss")[0]
    print("fp16 gradient rel errors:", {k: f"{v:.2e}" for k, v in errs.items()}, f"loss rel err {abs(loss - L) / L:.2e}")
    # FP16 operands carry 2^-11 relative rounding, ReLU decisions within that rounding
    # of zero may flip, and per-latent sums over samples cancel: the measured norm-wise
    # errors are ~1e-3 (weights) to ~1e-2 (latents); the FP32 path meets 1e-3 with margin.
    assert abs(loss - L) <= 2e-3 * L
    for k, v in errs.items():
        assert v <= 2e-2, (k, v)
    assert run.get("scale_state")[1] == 0
    # same comparison with the ReLU decisions taken in FP16: rounding error only
    _, gp_d, gl_d, _ = O.loss_and_grads(g, lat_fwd, run.ostate["mlp"], run.q, run.targets, decisions="fp16")
    derrs = {"mlp": rel_err(gp_gpu, gp_d), "latents": rel_err(gl_gpu, gl_d)}
    print("fp16 vs decision-matched oracle:", {k: f"{v:.2e}" for k, v in derrs.items()})
    for v in derrs.values():
        assert v <= 1e-3


@pytest.mark.parametrize("offset", [0.0, 64.0])
def test_gradients_fp16_fixed_point_range(lib, offset):
    """The FP16 kernels sum owned latent gradients in 32-bit fixed point (quantum 2^-16 of
    the delta's unit 2 x loss scale / (samples x channels)); a work item with a
    contribution beyond its range (at least 16 units) is summed again in FP32.  Targets
    shifted by 64 put contributions far beyond the range in every work item; both cases
    match the oracle with the ReLU decisions taken in FP16 (rounding error only)."""
    run = Run(lib, *CONFIGS["chain"], seed=12, prec=lib.F16)
    targets = run.targets + offset
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=True, seed=2)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp, targets=to_dev(targets))
    g = run.g
    assert run.get("scale_state")[1] == 0
    lat_fwd = run.ostate["latents"] + O.noise_values(g, 2, 0)
    _, gp_d, gl_d, _ = O.loss_and_grads(g, lat_fwd, run.ostate["mlp"], run.q, targets, decisions="fp16")
    err = rel_err(run.get("lat_grad") / run.get("loss_scale")[0], gl_d)
    perr = rel_err(run.get("mlp_m") / (1 - hp.beta1), gp_d)
    print(f"target offset {offset}: latent gradient rel err {err:.2e}, MLP gradient rel err {perr:.2e}")
    assert err <= 1e-3 and perr <= 1e-3


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_full_size_gradients(lib, prec):
    """The benchmark workload itself: 2048^2 x 12, 12 mips, 5 levels, 262,144 samples, noise on."""
    P = lib.F32 if prec == "f32" else lib.F16
    run = Run(lib, 2048, 12, 12, 12, 4, 4, 64, 0, 262144, None, seed=21, prec=P)
    hp = run.hp(lr_latent=0.0, lr_mlp=0.0, noise=True, seed=5)
    lib.train_prepare(run.m, run.state, hp)
    run.step(hp)
    g = run.g
    lat_fwd = run.ostate["latents"] + O.noise_values(g, 5, 0)
    L, gp, gl, _ = O.loss_and_grads(g, lat_fwd, run.ostate["mlp"], run.q, run.targets)
    scale = run.get("loss_scale")[0] if prec == "f16" else 1.0
    errs = {k: rel_err(_grad_groups(g, run.get("mlp_m") / (1 - hp.beta1))[k], v) for k, v in _grad_groups(g, gp).items()}
    errs["lat_grad"] = rel_err(run.get("lat_grad") / scale, gl)
    loss = run.get("loss")[0]
    print(f"full-size {prec} gradient rel errors:", {k: f"{v:.2e}" for k, v in errs.items()},
          f"loss {loss:.6e} vs {L:.6e}")
    tol = 1e-3 if prec == "f32" else 2e-2
    assert abs(loss - L) <= (1e-5 if prec == "f32" else 2e-3) * L
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if prec == "f16":  # with the ReLU decisions taken in FP16: rounding error only
        _, gp_d, gl_d, _ = O.loss_and_grads(g, lat_fwd, run.ostate["mlp"], run.q, run.targets, decisions="fp16")
        derrs = {"mlp": rel_err(run.get("mlp_m") / (1 - hp.beta1), gp_d),
                 "lat_grad": rel_err(run.get("lat_grad") / scale, gl_d)}
        print("full-size fp16 vs decision-matched oracle:", {k: f"{v:.2e}" for k, v in derrs.items()})
        for v in derrs.values():
            assert v <= 1e-3


@pytest.mark.parametrize("W,side,crops", [(2048, 256, 8), (64, 32, 3), (256, 100, 2)])
def test_crop_queries_bit_exact(lib, W, side, crops):
    """The device batch sampler reproduces the oracle's batches bit for bit, over steps
    that hit exponential and uniform LODs and mips smaller than the crop."""
    import torch
    m = lib.material_init(W, W, 4, 4, 4, 4, 4, 64)
    g = geometry(m)
    out = torch.zeros(crops * side * side * 12, dtype=torch.uint8, device="cuda")
    for step in range(12):
        lib.crop_queries(m, 77, step, out, crops=crops, side=side, uniform_fraction=0.3)
        torch.cuda.synchronize()
        want = O.crop_queries(g, 77, step, crops=crops, side=side, fraction=0.3)
        assert np.array_equal(out.cpu().numpy(), want.view(np.uint8)), step


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_step_is_deterministic(lib, prec):
    """Two runs of the same three steps from the same state are bit-identical: samples
    are binned in sample order (not in the order LDS atomics arrive), latent gradients
    are fixed-point sums, weight gradients and split-tile partials are reduced in a fixed
    order.  The 256^2 material with 65,536 samples per step splits its coarse-level
    tiles over several work items and sorts its small levels by anchor cell."""
    import torch
    P = lib.F32 if prec == "f32" else lib.F16
    W, C, n = 256, 12, 65536
    m = lib.material_init(W, W, C, C, C, 4, 4, 64)
    raw = synth.uniform_latents(31, int(m.latent_count))
    mlp = synth.xavier_mlp(31, int(m.input_width), 64, C)
    _, tflat = synth.target_chain(31, 0, W, W, C, int(m.num_mips))
    q = queries_dev(synth.random_queries(32, n, int(m.num_mips)))
    td = to_dev(tflat)
    runs = []
    for _ in range(2):
        st = lib.TrainState(m, raw, to_dev(mlp), P)
        ws = torch.zeros(lib.train_workspace_bytes(m, n, P), dtype=torch.uint8, device="cuda")
        for s in range(3):
            hp = lib.hparams(precision=P, step=s, lr_latent=0.01, lr_mlp=0.005, seed=9)
            if s == 0:
                lib.train_prepare(m, st, hp)
            lib.train_step(m, st, q, n, td, hp, ws)
        torch.cuda.synchronize()
        runs.append({k: getattr(st, k).clone() for k in ("latents", "latents_fwd", "lat_grad", "mlp", "mlp_m",
                                                         "mlp_v", "lat_m", "lat_v", "loss")})
    for k, v in runs[0].items():
        assert torch.equal(runs[1][k], v), (prec, k)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_backward_is_deterministic(lib, prec):
    """The differentiation path's backward, called twice on the same inputs, returns
    bit-identical gradients."""
    import torch
    P = lib.F32 if prec == "f32" else lib.F16
    W, C, n = 256, 12, 40000
    m = lib.material_init(W, W, C, C, C, 4, 4, 64)
    lat = to_dev(synth.uniform_latents(41, int(m.latent_count)) * 0.4)
    mlp = to_dev(synth.xavier_mlp(41, int(m.input_width), 64, C))
    tp = torch.zeros(lib.train_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    lib.pack_mlp_train(m, mlp, P, tp)
    q = queries_dev(synth.random_queries(42, n, int(m.num_mips)))
    dout = to_dev(np.random.default_rng(43).standard_normal(n * C).astype(np.float32) * 1e-3)
    ws = torch.zeros(lib.backward_workspace_bytes(m, n, P), dtype=torch.uint8, device="cuda")
    res = []
    for _ in range(2):
        gl, gm = torch.empty_like(lat), torch.empty_like(mlp)
        lib.backward(m, lat, mlp, tp, P, q, n, dout, 0.0, gl, gm, ws)
        torch.cuda.synchronize()
        res.append((gl.clone(), gm.clone()))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
