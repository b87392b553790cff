"""Gradient pins of the oracle: torch-CPU float64 autograd and central differences."""
import numpy as np
import pytest
import torch

from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth


def _setup(act="relu", n=512, seed=0):
    g = O.make_geometry(64, 64, 5, 3, 4, 4, 2, Hd=16, act=act)
    P = O.mlp_param_count(g.K, g.Hd, g.C)
    rng = np.random.default_rng(seed)
    params = rng.standard_normal(P) * 0.3
    lat = rng.uniform(-0.4, 0.5, g.latent_count)
    q = synth.random_queries(seed, n, g.M)
    _, tgt = synth.target_chain(seed, 0, 64, 64, 5, g.M)
    return g, params, lat, q, tgt


@pytest.mark.parametrize("act", ["relu", "hardgelu"])
def test_backward_matches_torch_autograd(act):
    """An independent float64 torch forward (same gather record) differentiated by
    autograd agrees with the oracle's analytic backward."""
    g, params, lat, q, tgt = _setup(act)
    L, gp, gl, _ = O.loss_and_grads(g, lat, params, q, tgt)
    _, rec = O.sample_inputs(g, lat, q)
    K, Hd, C, C0, C1 = g.K, g.Hd, g.C, g.C0, g.C1
    tl = torch.tensor(lat, dtype=torch.float64, requires_grad=True)
    tp = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    i0 = torch.tensor(rec["g0_idx"])
    i1 = torch.tensor(rec["g1_idx"])
    w1 = torch.tensor(rec["g1_w"])
    parts = [tl[i0[:, k:k + 1] + torch.arange(C0)] for k in range(4)]
    parts.append(sum(w1[:, k:k + 1] * tl[i1[:, k:k + 1] + torch.arange(C1)] for k in range(4)))
    parts.append(torch.tensor(O.pos_enc(rec["ix"], rec["iy"])))
    x = torch.cat(parts, dim=1)
    o = 0
    mats = []
    for shape in ((K, Hd), (Hd,), (Hd, Hd), (Hd,), (Hd, C), (C,)):
        size = int(np.prod(shape))
        mats.append(tp[o:o + size].reshape(shape))
        o += size
    W1, b1, W2, b2, W3, b3 = mats

    def a(z):
        if act == "relu":
            return torch.relu(z)
        return torch.where(z < -1.5, torch.zeros_like(z), torch.where(z > 1.5, z, z * (z + 1.5) / 3))

    y = a(a(x @ W1 + b1) @ W2 + b2) @ W3 + b3
    tt = []
    for s in range(len(q)):
        l = int(rec["lod"][s])
        base = g.mip_off[l] + (rec["iy"][s] * g.mip_w[l] + rec["ix"][s]) * C
        tt.append(tgt[base:base + C])
    t = torch.tensor(np.array(tt), dtype=torch.float64)
    loss = ((y - t) ** 2).mean()
    loss.backward()
    assert L == pytest.approx(loss.item(), rel=1e-13)
    assert np.allclose(gp, tp.grad.numpy(), rtol=1e-10, atol=1e-14)
    assert np.allclose(gl, tl.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_backward_central_differences():
    """Central differences, h = 1e-4, on 64 seeded parameters (latents and weights).
    Entries whose +-h perturbation flips any ReLU decision are skipped."""
    g, params, lat, q, tgt = _setup("relu", n=256, seed=5)
    L0, gp, gl, _ = O.loss_and_grads(g, lat, params, q, tgt)
    P = len(params)
    # latents that are actually read by this batch, plus weights
    _, rec = O.sample_inputs(g, lat, q)
    used = np.unique(np.concatenate([(rec["g0_idx"][:, :, None] + np.arange(g.C0)).ravel(),
                                     (rec["g1_idx"][:, :, None] + np.arange(g.C1)).ravel()]))
    rng = np.random.default_rng(11)
    pick_w = rng.choice(P, 32, replace=False)
    pick_l = rng.choice(used, 32, replace=False)
    h = 1e-4

    def masks(p, l):
        x, _ = O.sample_inputs(g, l, q)
        _, (z1, _, z2, _) = O.mlp_forward(p, x, g.K, g.Hd, g.C)
        return np.concatenate([(z1 > 0).ravel(), (z2 > 0).ravel()])

    base = masks(params, lat)
    checked = 0
    for kind, idx in [("w", i) for i in pick_w] + [("l", i) for i in pick_l]:
        vals = []
        ok = True
        for s in (+1, -1):
            p2, l2 = params.copy(), lat.copy()
            if kind == "w":
                p2[idx] += s * h
            else:
                l2[idx] += s * h
            if not np.array_equal(masks(p2, l2), base):
                ok = False
                break
            vals.append(O.loss_and_grads(g, l2, p2, q, tgt)[0])
        if not ok:
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        an = gp[idx] if kind == "w" else gl[idx]
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an), (kind, idx, fd, an)
        checked += 1
    assert checked >= 48


def test_latent_gradient_conservation():
    """Sum of all latent gradients equals the sum over samples of the G0 slots plus the
    G1 slots (bilinear weights sum to one)."""
    g, params, lat, q, tgt = _setup("relu", n=300, seed=2)
    _, gp, gl, y = O.loss_and_grads(g, lat, params, q, tgt)
    x, rec = O.sample_inputs(g, lat, q)
    _, (z1, _, z2, _) = O.mlp_forward(params, x, g.K, g.Hd, g.C)
    W1, b1, W2, b2, W3, b3 = O.mlp_split(params, g.K, g.Hd, g.C)
    t = O._targets_at(g, tgt, rec)
    dy = 2 * (y - t) / y.size
    dz2 = (dy @ W3.T) * (z2 > 0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    dx = dz1 @ W1.T
    assert gl.sum() == pytest.approx(dx[:, :4 * g.C0 + g.C1].sum(), rel=1e-10)


def test_decision_matched_mode_is_the_fp64_gradient_under_those_decisions():
    """On samples whose FP16-taken ReLU decisions agree with the float64 ones, the
    decision-matched mode returns exactly the float64 loss and gradients; on the full
    batch it returns the gradient of the masked function (torch autograd, fixed masks)."""
    g, params, lat, q, tgt = _setup("relu", n=3000, seed=4)
    x, _ = O.sample_inputs(g, lat, q)
    m16 = O.relu_decisions_fp16(params, x, g.K, g.Hd, g.C)
    _, (z1, _, z2, _) = O.mlp_forward(params, x, g.K, g.Hd, g.C)
    agree = np.all(m16[0] == (z1 > 0), axis=1) & np.all(m16[1] == (z2 > 0), axis=1)
    assert 0 < agree.sum() < len(q)          # some decisions do flip at FP16
    qa = q[agree]
    a = O.loss_and_grads(g, lat, params, qa, tgt)
    b = O.loss_and_grads(g, lat, params, qa, tgt, decisions="fp16")
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    # full batch: gradient of the masked function
    _, gp, gl, _ = O.loss_and_grads(g, lat, params, q, tgt, decisions="fp16")
    _, rec = O.sample_inputs(g, lat, q)
    K, Hd, C = g.K, g.Hd, g.C
    tp = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    tx = torch.tensor(x, dtype=torch.float64)
    W1 = tp[:K * Hd].reshape(K, Hd); o = K * Hd
    b1 = tp[o:o + Hd]; o += Hd
    W2 = tp[o:o + Hd * Hd].reshape(Hd, Hd); o += Hd * Hd
    b2 = tp[o:o + Hd]; o += Hd
    W3 = tp[o:o + Hd * C].reshape(Hd, C); o += Hd * C
    b3 = tp[o:o + C]
    h1 = (tx @ W1 + b1) * torch.tensor(m16[0], dtype=torch.float64)
    h2 = (h1 @ W2 + b2) * torch.tensor(m16[1], dtype=torch.float64)
    y = h2 @ W3 + b3
    t = torch.tensor(O._targets_at(g, tgt, rec))
    ((y - t) ** 2).mean().backward()
    assert np.allclose(gp, tp.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_fp16_decisions_hand_built_case():
    """ReLU decisions taken the FP16 way, pinned on a network built by hand so that each
    rounding point flips a decision on its own (K = 2 inputs, 3 hidden units, 1 output):
      inputs rounded:      unit 1/0 is x0 - x1; x0 = 1 + 2^-11 rounds (half to even) to 1,
                           so z = 2^-11 > 0 in float64 but 0 in FP16;
      weights rounded:     unit 1/1 is (1 + 2^-11) x0 - x1; at x = (1, 1) z = 2^-11 in
                           float64, 0 in FP16;
      activations rounded: unit 1/2 is the bias 1 + 2^-11 (biases stay FP32), so h = 1 + 2^-11
                           in float64 and 1 in FP16; unit 2/0 is h_2 - 1: 2^-11 > 0 vs 0;
      bias kept in FP32:   unit 2/1 is the bias 2^-26, which FP16 would flush to 0: stays on;
                           unit 2/2 is the bias -2^-26: off.
    The decisions are written out by hand, together with the float64 ones they differ from."""
    K, Hd, C = 2, 3, 1
    e = 2.0 ** -11
    W1 = np.array([[1.0, 1.0 + e, 0.0],
                   [-1.0, -1.0, 0.0]])
    b1 = np.array([0.0, 0.0, 1.0 + e])
    W2 = np.zeros((Hd, Hd))
    W2[2, 0] = 1.0
    b2 = np.array([-1.0, 2.0 ** -26, -2.0 ** -26])
    W3 = np.ones((Hd, C))
    b3 = np.zeros(C)
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    x = np.array([[1.0 + e, 1.0],
                  [1.0, 1.0]])
    m1, m2 = O.relu_decisions_fp16(params, x, K, Hd, C)
    assert m1.tolist() == [[False, False, True], [False, False, True]]
    assert m2.tolist() == [[False, True, False], [False, True, False]]
    # the float64 decisions of the same network (what an unrounded evaluation gives)
    _, (z1, _, z2, _) = O.mlp_forward(params, x, K, Hd, C)
    assert (z1 > 0).tolist() == [[True, True, True], [False, True, True]]
    assert (z2 > 0).tolist() == [[True, True, False], [True, True, False]]
