"""Differentiation path (tiny-configuration shapes): torch.autograd.Function over the
library's forward/backward kernels, FP32 and FP16 matrix cores, against the FP64
oracle's analytic gradient and central finite differences (h = 1e-4) on 64 seeded
parameters."""
import numpy as np
import pytest

from _helpers import geometry, mlp_in_unit_range, queries_dev, rel_err, to_dev
from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_17105_amd import ntc
    m = ntc.material_init(256, 256, 8, 8, 8, 4, 4, 64, num_mips=1)
    g = geometry(m)
    rng = np.random.default_rng(31)
    lat = rng.uniform(-15 / 32, 0.5, g.latent_count).astype(np.float32)
    mlp = synth.xavier_mlp(31, g.K, 64, 8)
    n = 16384
    q = synth.random_queries(31, n, 1, 0)
    _, tflat = synth.target_chain(31, 0, 256, 256, 8, 1)
    return ntc, m, g, lat, mlp, q, tflat


def _targets_for(g, q, tflat):
    _, rec = O.sample_inputs(g, np.zeros(g.latent_count), q)
    return O._targets_at(g, tflat, rec)


def _run(setup, prec):
    import torch
    from paper_2305_17105_amd.autograd import ntc_decode_fn
    ntc, m, g, lat, mlp, q, tflat = setup
    P = ntc.F32 if prec == "f32" else ntc.F16
    tl = to_dev(lat).requires_grad_(True)
    tm = to_dev(mlp).requires_grad_(True)
    y = ntc_decode_fn(m, tl, tm, queries_dev(q), P)
    t = torch.from_numpy(_targets_for(g, q, tflat)).float().cuda()
    loss = ((y - t) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    return (y.detach().cpu().numpy().astype(np.float64), float(loss), tl.grad.cpu().numpy().astype(np.float64),
            tm.grad.cpu().numpy().astype(np.float64))


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_autograd_matches_oracle(setup, prec):
    ntc, m, g, lat, mlp, q, tflat = setup
    y, L, gl, gm = _run(setup, prec)
    yref = O.decode(g, lat.astype(np.float64), mlp, q)
    Lref, gp_ref, gl_ref, _ = O.loss_and_grads(g, lat.astype(np.float64), mlp, q, tflat)
    yerr = np.max(np.abs(y - yref))
    errs = {"latents": rel_err(gl, gl_ref)}
    W1, b1, W2, b2, W3, b3 = O.mlp_split(gm, g.K, g.Hd, g.C)
    R = O.mlp_split(gp_ref, g.K, g.Hd, g.C)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), (W1, b1, W2, b2, W3, b3), R):
        errs[name] = rel_err(a, b)
    print(f"{prec}: output max-abs err {yerr:.2e}, loss rel err {abs(L - Lref) / Lref:.2e}, gradient rel errors",
          {k: f"{v:.2e}" for k, v in errs.items()})
    if prec == "f32":
        assert yerr <= 1e-5
        for v in errs.values():
            assert v <= 1e-3
    else:
        assert yerr <= 2e-2  # raw Xavier outputs are O(1): 2e-3 applies to outputs in [0, 1] (below)
        for v in errs.values():
            assert v <= 2e-2
        # with the ReLU decisions taken in FP16 (as the kernel takes them) the
        # remaining difference is rounding only
        _, gp_d, gl_d, _ = O.loss_and_grads(g, lat.astype(np.float64), mlp, q, tflat, decisions="fp16")
        derrs = {"latents": rel_err(gl, gl_d), "mlp": rel_err(gm, gp_d)}
        print("f16 vs decision-matched oracle:", {k: f"{v:.2e}" for k, v in derrs.items()})
        for v in derrs.values():
            assert v <= 1e-3


def test_autograd_fp16_outputs_in_unit_range(setup):
    """The FP16 forward on a network whose outputs lie near [0, 1] (damped output layer,
    b3 = 1/2): within 2e-3 max-abs of the float64 oracle."""
    import torch
    from paper_2305_17105_amd.autograd import ntc_decode_fn
    ntc, m, g, lat, _, q, _ = setup
    mlp = mlp_in_unit_range(32, g.K, g.Hd, g.C)
    with torch.no_grad():
        y = ntc_decode_fn(m, to_dev(lat), to_dev(mlp), queries_dev(q), ntc.F16)
    yref = O.decode(g, lat.astype(np.float64), mlp, q)
    err = np.max(np.abs(y.cpu().numpy().astype(np.float64) - yref))
    print(f"f16 forward on [0,1] outputs: max-abs err {err:.2e} (outputs in [{yref.min():.2f}, {yref.max():.2f}])")
    assert err <= 2e-3


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_backward_device_scale_equals_explicit(setup, prec):
    """dout_scale = 0 picks 2^round(log2(1/4 / max|dout|)) on the device; the result is
    bit-identical to passing that power of two from the host."""
    import math
    import torch
    ntc, m, g, lat, mlp, q, _ = setup
    P = ntc.F32 if prec == "f32" else ntc.F16
    n = len(q)
    dout = torch.from_numpy(np.random.default_rng(5).normal(0, 3e-4, n * g.C).astype(np.float32)).cuda()
    tp = torch.zeros(ntc.train_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
    tl, tm = to_dev(lat), to_dev(mlp)
    ntc.pack_mlp_train(m, tm, P, tp)
    ws = torch.zeros(ntc.backward_workspace_bytes(m, n, P), dtype=torch.uint8, device="cuda")
    qd = queries_dev(q)
    amax = float(dout.abs().max())
    host_scale = 2.0 ** round(math.log2(0.25 / amax))
    res = []
    for sc in (0.0, host_scale):
        gl, gm = torch.empty_like(tl), torch.empty_like(tm)
        ntc.backward(m, tl, tm, tp, P, qd, n, dout, sc, gl, gm, ws)
        torch.cuda.synchronize()
        res.append((gl.cpu().numpy(), gm.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    # a zero dout gets scale 1 and zero gradients
    gl, gm = torch.empty_like(tl), torch.empty_like(tm)
    ntc.backward(m, tl, tm, tp, P, qd, n, torch.zeros_like(dout), 0.0, gl, gm, ws)
    torch.cuda.synchronize()
    assert not gl.cpu().numpy().any() and not gm.cpu().numpy().any()


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_autograd_central_differences(setup, prec):
    """Central differences of the float64 loss, h = 1e-4, on 64 seeded parameters, latents
    read by the batch and weights alternating (candidates whose +-h perturbation flips
    a ReLU decision are skipped and the next candidate taken)."""
    ntc, m, g, lat, mlp, q, tflat = setup
    _, _, gl, gm = _run(setup, prec)
    lat64 = lat.astype(np.float64)
    mlp64 = mlp.astype(np.float64)
    _, rec = O.sample_inputs(g, lat64, q)
    used = np.unique((rec["g0_idx"][:, :, None] + np.arange(g.C0)).ravel())
    rng = np.random.default_rng(77)
    cand_l = rng.choice(used, 96, replace=False)
    cand_w = rng.choice(len(mlp), 96, replace=False)
    picks = [p for pair in zip([("l", i) for i in cand_l], [("w", i) for i in cand_w]) for p in pair]
    h = 1e-4

    # FP16 evaluates the network with ReLU decisions taken in FP16; differences are taken
    # of that same function (float64 values, FP16-taken decisions)
    decisions = "fp16" if prec == "f16" else None

    def masks(p, l):
        x, _ = O.sample_inputs(g, l, q)
        if decisions:
            m1, m2 = O.relu_decisions_fp16(p, x, g.K, g.Hd, g.C)
            return np.concatenate([m1.ravel(), m2.ravel()])
        _, (z1, _, z2, _) = O.mlp_forward(p, x, g.K, g.Hd, g.C)
        return np.concatenate([(z1 > 0).ravel(), (z2 > 0).ravel()])

    base = masks(mlp64, lat64)
    scale_l = np.sqrt(np.mean(gl[used] ** 2))
    scale_w = np.sqrt(np.mean(gm ** 2))
    worst = 0.0
    checked = 0
    for kind, idx in picks:
        if checked == 64:
            break
        vals = []
        for sgn in (1, -1):
            p2, l2 = mlp64.copy(), lat64.copy()
            if kind == "w":
                p2[idx] += sgn * h
            else:
                l2[idx] += sgn * h
            if not np.array_equal(masks(p2, l2), base):
                vals = None
                break
            vals.append(O.loss_and_grads(g, l2, p2, q, tflat, decisions=decisions)[0])
        if vals is None:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        got = gl[idx] if kind == "l" else gm[idx]
        ref = max(abs(fd), scale_l if kind == "l" else scale_w)
        worst = max(worst, abs(got - fd) / ref)
        checked += 1
    print(f"{prec}: {checked} entries checked, worst |gpu - fd| / max(|fd|, rms) = {worst:.2e}")
    assert checked == 64
    assert worst <= 1e-2
