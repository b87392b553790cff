"""Many materials in one call (uneven sizes, channel counts, MLP widths), HIP-graph
replay of a training step, and the training-step tuner.  The per-material path these
calls run is pinned to the FP64 oracle by test_gpu_train / test_gpu_decode; here the
batched and replayed results are compared with that per-material path, and one
material's loss with the oracle."""
import numpy as np
import pytest

from _helpers import geometry, mlp_in_unit_range, queries_dev, quantized_latents_oracle, to_dev
from oracle import ntc_oracle as O
from paper_2305_17105_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [  # W, C (= c0 = c1), hidden, samples
    (256, 8, 32, 3000),
    (512, 12, 64, 9001),
    (256, 16, 64, 4097),
]


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_17105_amd import ntc
    return ntc


def _material(lib, W, C, hd, seed):
    import torch
    m = lib.material_init(W, W, C, C, C, 4, 4, hd)
    raw = synth.uniform_latents(seed, int(m.latent_count))
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    lib.quantize_latents(m, to_dev(raw), packed)
    lat = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
    lib.dequantize_latents(m, packed, lat)
    mlp = synth.xavier_mlp(seed, int(m.input_width), hd, C)
    _, tflat = synth.target_chain(seed, 0, W, W, C, int(m.num_mips))
    return m, raw, lat, mlp, to_dev(tflat), tflat


def _states(lib, mats, prec):
    out = []
    for m, raw, lat, mlp, td, _ in mats:
        out.append(lib.TrainState(m, lat, to_dev(mlp), prec))
    return out


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_batched_train_equals_per_material(lib, prec):
    import torch
    P = lib.F32 if prec == "f32" else lib.F16
    mats = [_material(lib, W, C, hd, 40 + i) for i, (W, C, hd, _) in enumerate(SHAPES)]
    ns = [n for (_, _, _, n) in SHAPES]
    offsets = np.concatenate([[0], np.cumsum(ns)])
    qs = [synth.random_queries(50 + i, n, int(mats[i][0].num_mips)) for i, n in enumerate(ns)]
    qall = queries_dev(np.concatenate(qs))
    ms = [x[0] for x in mats]
    # batched: two steps
    sb = _states(lib, mats, P)
    wsb = torch.zeros(lib.train_workspace_bytes_batched(ms, offsets, P), dtype=torch.uint8, device="cuda")
    for step in range(2):
        hp = lib.hparams(precision=P, step=step, lr_latent=0.01, lr_mlp=0.005, seed=3)
        if step == 0:
            for m, s in zip(ms, sb):
                lib.train_prepare(m, s, hp)
        lib.train_step_batched(ms, sb, qall, offsets, [x[4] for x in mats], hp, wsb)
    # one material at a time
    si = _states(lib, mats, P)
    for i, (m, s) in enumerate(zip(ms, si)):
        ws = torch.zeros(lib.train_workspace_bytes(m, ns[i], P), dtype=torch.uint8, device="cuda")
        qd = queries_dev(qs[i])
        for step in range(2):
            hp = lib.hparams(precision=P, step=step, lr_latent=0.01, lr_mlp=0.005, seed=3)
            if step == 0:
                lib.train_prepare(m, s, hp)
            lib.train_step(m, s, qd, ns[i], mats[i][4], hp, ws)
    torch.cuda.synchronize()
    _assert_states_equal(sb, si)
    # the first step's loss of one material against the oracle (masters at step 0)
    m0, raw0, _, mlp0, _, tflat0 = mats[1]
    g = geometry(m0)
    lat_fwd = quantized_latents_oracle(g, raw0) + O.noise_values(g, 3, 0)
    L, _, _, _ = O.loss_and_grads(g, lat_fwd, mlp0.astype(np.float64), qs[1], tflat0)
    si2 = _states(lib, [mats[1]], P)[0]
    ws = torch.zeros(lib.train_workspace_bytes(m0, ns[1], P), dtype=torch.uint8, device="cuda")
    hp = lib.hparams(precision=P, step=0, lr_latent=0.0, lr_mlp=0.0, seed=3)
    lib.train_prepare(m0, si2, hp)
    lib.train_step_batched([m0], [si2], queries_dev(qs[1]), [0, ns[1]], [mats[1][4]], hp, ws)
    torch.cuda.synchronize()
    got = float(si2.loss.cpu()[0])
    print(f"batched {prec}: loss {got:.7e} vs oracle {L:.7e}")
    assert abs(got - L) / L <= (1e-5 if prec == "f32" else 2e-3)


@pytest.mark.parametrize("prec", ["f16", "fp8", "f32"])
def test_batched_decode_equals_per_material(lib, prec):
    import torch
    P = {"f32": lib.F32, "f16": lib.F16, "fp8": lib.FP8_E4M3}[prec]
    shapes = [(256, 8, 8, 4, 4, 64, 1000), (512, 16, 16, 2, 4, 64, 3001), (256, 16, 16, 4, 4, 32, 77)]
    ms, pk, wp, qs, ns = [], [], [], [], []
    for i, (W, C, c0, b0, b1, hd, n) in enumerate(shapes):
        m = lib.material_init(W, W, C, c0, c0, b0, b1, hd)
        raw = synth.uniform_latents(60 + i, int(m.latent_count))
        p = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        lib.quantize_latents(m, to_dev(raw), p)
        mlp = mlp_in_unit_range(60 + i, int(m.input_width), hd, C)
        w = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
        lib.pack_mlp(m, to_dev(mlp), P, w)
        ms.append(m); pk.append(p); wp.append(w); ns.append(n)
        qs.append(synth.random_queries(70 + i, n, int(m.num_mips)))
    offsets = np.concatenate([[0], np.cumsum(ns)])
    total = sum(n * m.channels for n, m in zip(ns, ms))
    out = torch.full((total,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode_batched(ms, pk, wp, P, queries_dev(np.concatenate(qs)), offsets, out, lib.F32)
    o = 0
    for i, m in enumerate(ms):
        ref = torch.full((ns[i] * m.channels,), float("nan"), dtype=torch.float32, device="cuda")
        lib.decode(m, pk[i], wp[i], P, queries_dev(qs[i]), ns[i], ref, lib.F32)
        torch.cuda.synchronize()
        assert torch.equal(out[o:o + ns[i] * m.channels], ref), i
        o += ns[i] * m.channels


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_graph_replay_matches_eager(lib, prec):
    """One captured training step (device step index and learning rates) replayed four
    times, with eager work and synchronization between replays; every replay matches
    the eager step with the same index."""
    import torch
    P = lib.F32 if prec == "f32" else lib.F16
    W, C, hd, n = 512, 12, 64, 9001
    mat = _material(lib, W, C, hd, 81)
    m, _, lat, mlp, td, _ = mat
    q = queries_dev(synth.random_queries(82, n, int(m.num_mips)))
    lr = [(0.01 * (1 - 0.1 * s), 0.005 * (1 - 0.1 * s)) for s in range(4)]
    # eager reference
    se = lib.TrainState(m, lat, to_dev(mlp), P)
    wse = torch.zeros(lib.train_workspace_bytes(m, n, P), dtype=torch.uint8, device="cuda")
    ref = []
    for s in range(4):
        hp = lib.hparams(precision=P, step=s, lr_latent=lr[s][0], lr_mlp=lr[s][1], seed=5)
        if s == 0:
            lib.train_prepare(m, se, hp)
        lib.train_step(m, se, q, n, td, hp, wse)
        torch.cuda.synchronize()
        ref.append({k: getattr(se, k).clone() for k in ("latents", "latents_fwd", "mlp", "loss")})
    # captured step
    sg = lib.TrainState(m, lat, to_dev(mlp), P)
    wsg = torch.zeros_like(wse)
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    lr_dev = torch.tensor(lr[0], dtype=torch.float32, device="cuda")
    hp = lib.hparams(precision=P, step=0, seed=5, step_dev=step_dev, lr_dev=lr_dev)
    lib.train_prepare(m, sg, hp)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            lib.train_step(m, sg, q, n, td, hp, wsg)
    torch.cuda.synchronize()
    assert int(step_dev.item()) == 0  # capture does not run the step
    for s in range(4):
        lr_dev.copy_(torch.tensor(lr[s], dtype=torch.float32))
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1024, device="cuda").sum().item()  # eager work between replays
        assert int(step_dev.item()) == s + 1
        # the step is deterministic (samples are binned in sample order, latent gradients
        # are fixed-point sums), so every replay equals the eager step bit for bit
        for k, v in ref[s].items():
            assert torch.equal(getattr(sg, k), v), (s, k)


def test_autotune_picks_a_candidate_and_training_still_matches(lib):
    import torch
    W, C, hd, n = 512, 12, 64, 20011
    m, _, lat, mlp, td, _ = _material(lib, W, C, hd, 91)
    q = queries_dev(synth.random_queries(92, n, int(m.num_mips)))
    s0 = lib.TrainState(m, lat, to_dev(mlp), lib.F16)
    ws = torch.zeros(lib.train_workspace_bytes(m, n, lib.F16), dtype=torch.uint8, device="cuda")
    hp = lib.hparams(precision=lib.F16, step=0, seed=7)
    lib.train_prepare(m, s0, hp)
    lib.train_step(m, s0, q, n, td, hp, ws)  # default plan
    torch.cuda.synchronize()
    s1 = lib.TrainState(m, lat, to_dev(mlp), lib.F16)
    lib.train_prepare(m, s1, hp)
    chunk, tile, us = lib.train_autotune(m, s1, q, n, td, hp, ws)
    print(f"tuned: chunk {chunk}, tile {tile}, {us:.1f} us per gradient pass")
    assert chunk in (256, 512, 1024) and tile in (8, 16, 32) and us > 0
    lib.train_prepare(m, s1, hp)
    lib.train_step(m, s1, q, n, td, hp, ws)  # tuned plan
    torch.cuda.synchronize()
    # another work split sums the FP32 weight-gradient partials in another order; Adam's
    # normalised step turns that rounding into up to ~lr * 1e-2 on near-zero gradients
    for k in ("latents", "mlp", "loss"):
        a, b = getattr(s1, k).double(), getattr(s0, k).double()
        d = float((a - b).abs().max())
        if k == "mlp":
            assert d <= 1e-2 * hp.lr_mlp, (k, d)
        else:
            err = d / max(float(b.abs().max()), 1e-30)
            assert err <= 1e-4, (k, err)


def _decode_batch(lib, P, count, seed):
    """`count` small decode materials over several kernel shapes (one with hardGELU, one
    with an empty query group), their packs and queries."""
    import torch
    kinds = [(8, 8, 4, 4, 64), (16, 16, 4, 4, 32), (16, 16, 2, 4, 64), (8, 8, 4, 4, 32)]
    if P != lib.FP8_E4M3:
        kinds.append((12, 12, 4, 4, 64))
    r = np.random.default_rng(seed)
    ms, pk, wp, qs, ns = [], [], [], [], []
    for i in range(count):
        C, c0, b0, b1, hd = kinds[0] if (i % 4 or i < 4) else kinds[(i // 4) % len(kinds)]
        W = int(2 ** r.integers(6, 9))
        act = lib.ACT_HARDGELU if i == 1 else lib.ACT_RELU
        m = lib.material_init(W, W, C, c0, c0, b0, b1, hd, activation=act)
        p = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        lib.quantize_latents(m, to_dev(synth.uniform_latents(seed + i, int(m.latent_count))), p)
        w = torch.zeros(lib.mlp_packed_bytes(m, P), dtype=torch.uint8, device="cuda")
        lib.pack_mlp(m, to_dev(mlp_in_unit_range(seed + 100 + i, int(m.input_width), hd, C)), P, w)
        n = 0 if i == 3 else int(r.integers(1, 2500))
        ms.append(m); pk.append(p); wp.append(w); ns.append(n)
        qs.append(synth.random_queries(seed + 200 + i, n, int(m.num_mips)))
    offsets = np.concatenate([[0], np.cumsum(ns)])
    return ms, pk, wp, queries_dev(np.concatenate(qs)), offsets


@pytest.mark.parametrize("prec", ["f32", "f16", "fp8"])
@pytest.mark.parametrize("out_dtype", ["f32", "f16"])
def test_grouped_decode_equals_batched(lib, prec, out_dtype):
    """Grouped decode (one launch per kernel shape, more materials of one shape than a
    launch holds) writes exactly what per-material decode writes, for every material."""
    import torch
    P = {"f32": lib.F32, "f16": lib.F16, "fp8": lib.FP8_E4M3}[prec]
    OD, tdt = (lib.F32, torch.float32) if out_dtype == "f32" else (lib.F16, torch.float16)
    ms, pk, wp, q, offsets = _decode_batch(lib, P, 52, 900)
    total = sum(int(offsets[i + 1] - offsets[i]) * m.channels for i, m in enumerate(ms))
    ref = torch.full((total,), float("nan"), dtype=tdt, device="cuda")
    lib.decode_batched(ms, pk, wp, P, q, offsets, ref, OD)
    table = lib.DecodeTable(ms, pk, wp, P)
    for _ in range(2):  # the table is reused
        out = torch.full((total,), float("nan"), dtype=tdt, device="cuda")
        lib.decode_grouped(table, q, offsets, out, OD)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_grouped_decode_table_of_other_materials_decodes_nothing(lib):
    """A table built for one batch, used with the descriptors of another, leaves the
    output untouched."""
    import torch
    ms, pk, wp, q, offsets = _decode_batch(lib, lib.F16, 6, 950)
    ms2 = list(ms)
    ms2[0] = lib.material_init(512, 512, 8, 8, 8, 4, 4, 64)
    table = lib.DecodeTable(ms, pk, wp, lib.F16)
    total = sum(int(offsets[i + 1] - offsets[i]) * m.channels for i, m in enumerate(ms2))
    out = torch.full((total,), 7.0, dtype=torch.float16, device="cuda")
    t2 = lib.DecodeTable.__new__(lib.DecodeTable)
    t2.__dict__.update(table.__dict__)
    t2.mats = lib._materials(ms2)
    lib.decode_grouped(t2, q, offsets, out, lib.F16)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())


def _grouped_vs_batched(lib, P, mats, ns, seed, steps=2):
    """Runs `steps` steps of the batched and of the grouped step from the same start;
    returns both state lists."""
    import torch
    offsets = np.concatenate([[0], np.cumsum(ns)])
    qs = [synth.random_queries(seed + i, n, int(mats[i][0].num_mips)) for i, n in enumerate(ns)]
    qall = queries_dev(np.concatenate(qs))
    ms = [x[0] for x in mats]
    tg = [x[4] for x in mats]
    out = []
    for grouped in (False, True):
        st = _states(lib, mats, P)
        ws = torch.zeros(lib.train_workspace_bytes_batched(ms, offsets, P), dtype=torch.uint8, device="cuda")
        table = lib.TrainTable(ms, st, offsets, tg, P, ws) if grouped else None
        for step in range(steps):
            hp = lib.hparams(precision=P, step=step, lr_latent=0.01, lr_mlp=0.005, seed=seed)
            if step == 0:
                for m, s in zip(ms, st):
                    lib.train_prepare(m, s, hp)
            if grouped:
                lib.train_step_grouped(table, qall, hp)
            else:
                lib.train_step_batched(ms, st, qall, offsets, tg, hp, ws)
        torch.cuda.synchronize()
        out.append(st)
    return out


def _assert_states_equal(sb, sg):
    """Bit-identical states: the same kernels on the same data, and the step does not
    depend on the timing of the run (samples are binned in sample order, latent
    gradients are fixed-point sums, weight gradients are reduced in a fixed order)."""
    for i in range(len(sb)):
        for name in ("latents", "latents_fwd", "mlp", "lat_m", "lat_v", "mlp_m", "mlp_v", "loss"):
            a = getattr(sb[i], name)
            b = getattr(sg[i], name)
            assert torch_equal(a, b), (i, name, float((a.double() - b.double()).abs().max()))


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_grouped_train_equals_batched(lib, prec):
    """The grouped step (one launch per stage) gives the batched step's states."""
    P = lib.F32 if prec == "f32" else lib.F16
    mats = [_material(lib, W, C, hd, 140 + i) for i, (W, C, hd, _) in enumerate(SHAPES)]
    sb, sg = _grouped_vs_batched(lib, P, mats, [n for (_, _, _, n) in SHAPES], 150)
    _assert_states_equal(sb, sg)


def test_grouped_train_more_members_than_one_launch(lib):
    """70 small materials (two launches per stage) trained grouped and batched."""
    mats = [_material(lib, 64 if i % 3 else 128, 8, 32 if i % 2 else 64, 300 + i) for i in range(70)]
    ns = [200 + 37 * (i % 11) for i in range(70)]
    sb, sg = _grouped_vs_batched(lib, lib.F16, mats, ns, 310)
    _assert_states_equal(sb, sg)


def test_grouped_train_more_members_of_one_shape_than_one_fused_launch(lib):
    """65 materials of one kernel shape, interleaved with 5 of another: the fused pass of
    the first shape needs two launches (64 members each at most), the stage launches two
    as well; grouped equals batched."""
    mats = [_material(lib, 64, 8, 32 if i % 17 else 64, 600 + i) for i in range(70)]
    ns = [150 + 29 * (i % 7) for i in range(70)]
    sb, sg = _grouped_vs_batched(lib, lib.F16, mats, ns, 610)
    _assert_states_equal(sb, sg)


def test_grouped_train_table_of_other_group_does_nothing(lib):
    """A table built for other sample groups: the step leaves every state as it was."""
    import torch
    mats = [_material(lib, W, C, hd, 160 + i) for i, (W, C, hd, _) in enumerate(SHAPES)]
    ms = [x[0] for x in mats]
    ns = [n for (_, _, _, n) in SHAPES]
    offsets = np.concatenate([[0], np.cumsum(ns)])
    other = np.concatenate([[0], np.cumsum([n + 1 for n in ns])])
    st = _states(lib, mats, lib.F16)
    hp = lib.hparams(precision=lib.F16, step=0, lr_latent=0.01, lr_mlp=0.005, seed=4)
    for m, s in zip(ms, st):
        lib.train_prepare(m, s, hp)
    ws = torch.zeros(lib.train_workspace_bytes_batched(ms, other, lib.F16), dtype=torch.uint8, device="cuda")
    table = lib.TrainTable(ms, st, offsets, [x[4] for x in mats], lib.F16, ws)
    table.offsets = (lib.C.c_int64 * (len(ms) + 1))(*[int(o) for o in other])
    before = [s.latents.clone() for s in st]
    q = queries_dev(synth.random_queries(161, int(other[-1]), int(ms[0].num_mips)))
    lib.train_step_grouped(table, q, hp)
    torch.cuda.synchronize()
    for s, b in zip(st, before):
        assert torch.equal(s.latents, b)


def test_grouped_graph_replay_matches_eager(lib):
    """A captured grouped step (device step index and learning rates) replayed three
    times, with eager work between replays, matches eager grouped steps."""
    import torch
    P = lib.F16
    mats = [_material(lib, W, C, hd, 170 + i) for i, (W, C, hd, _) in enumerate(SHAPES)]
    ms = [x[0] for x in mats]
    ns = [n for (_, _, _, n) in SHAPES]
    offsets = np.concatenate([[0], np.cumsum(ns)])
    q = queries_dev(np.concatenate([synth.random_queries(180 + i, n, int(ms[i].num_mips)) for i, n in enumerate(ns)]))
    tg = [x[4] for x in mats]
    lr = [(0.01 * (1 - 0.1 * s), 0.005 * (1 - 0.1 * s)) for s in range(3)]
    runs = []
    for graph in (False, True):
        st = _states(lib, mats, P)
        ws = torch.zeros(lib.train_workspace_bytes_batched(ms, offsets, P), dtype=torch.uint8, device="cuda")
        table = lib.TrainTable(ms, st, offsets, tg, P, ws)
        step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
        lr_dev = torch.tensor(lr[0], dtype=torch.float32, device="cuda")
        hp = lib.hparams(precision=P, step=0, seed=6, step_dev=step_dev, lr_dev=lr_dev)
        for m, s in zip(ms, st):
            lib.train_prepare(m, s, hp)
        torch.cuda.synchronize()
        if graph:
            g = torch.cuda.CUDAGraph()
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                with torch.cuda.graph(g, stream=stream):
                    lib.train_step_grouped(table, q, hp)
            torch.cuda.synchronize()
            assert int(step_dev.item()) == 0
        snaps = []
        for s in range(3):
            lr_dev.copy_(torch.tensor(lr[s], dtype=torch.float32))
            if graph:
                g.replay()
            else:
                lib.train_step_grouped(table, q, hp)
            torch.cuda.synchronize()
            _ = torch.ones(1024, device="cuda").sum().item()
            assert int(step_dev.item()) == s + 1
            snaps.append([{k: getattr(x, k).clone() for k in ("latents", "mlp", "loss")} for x in st])
        runs.append(snaps)
    for s in range(3):
        for i in range(len(ms)):
            for k, v in runs[0][s][i].items():
                assert torch.equal(runs[1][s][i][k], v), (s, i, k)


@pytest.mark.parametrize("kind", [(16, 16, 2, 4, 64), (8, 8, 4, 4, 32), (10, 10, 4, 4, 64)])
@pytest.mark.parametrize("order", ["random", "runs"])
def test_mixed_decode_equals_per_material(lib, kind, order):
    """Mixed-material decode (Appendix A's divergence loop): queries naming one of six
    materials of a shape, in random order or in runs; every texel equals its
    material's own decode bit for bit, and the oracle's within the FP16 bar.  Material
    indices outside the set are clamped."""
    import torch
    C, c0, b0, b1, hd = kind
    r = np.random.default_rng(70)
    ms, pk, wp, raws, mlps = [], [], [], [], []
    for i in range(6):
        W = int(2 ** r.integers(6, 10))
        m = lib.material_init(W, W, C, c0, c0, b0, b1, hd)
        raw = synth.uniform_latents(700 + i, int(m.latent_count))
        p = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        lib.quantize_latents(m, to_dev(raw), p)
        mlp = mlp_in_unit_range(710 + i, int(m.input_width), hd, C)
        w = torch.zeros(lib.mlp_packed_bytes(m, lib.F16), dtype=torch.uint8, device="cuda")
        lib.pack_mlp(m, to_dev(mlp), lib.F16, w)
        ms.append(m); pk.append(p); wp.append(w); raws.append(raw); mlps.append(mlp)
    n = 20011
    mq = np.zeros(n, dtype=lib.MIXED_QUERY_DTYPE)
    mq["u"] = r.uniform(0, 1, n)
    mq["v"] = r.uniform(0, 1, n)
    mq["material"] = r.integers(0, 6, n) if order == "random" else np.repeat(r.integers(0, 6, n // 37 + 1), 37)[:n]
    mq["material"][:3] = [-3, 6, 99]  # clamped to 0, 5, 5
    mat = np.clip(mq["material"], 0, 5)
    for i, m in enumerate(ms):
        sel = mat == i
        mq["lod"][sel] = r.integers(0, int(m.num_mips), int(sel.sum()))
    table = lib.DecodeTable(ms, pk, wp, lib.F16)
    out = torch.full((n * C,), float("nan"), dtype=torch.float32, device="cuda")
    lib.decode_mixed(table, torch.from_numpy(mq.view(np.uint8).copy()).cuda(), n, out, lib.F32)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, C)
    for i, m in enumerate(ms):
        sel = np.nonzero(mat == i)[0]
        q = np.zeros(len(sel), dtype=synth.QUERY_DTYPE)
        q["u"], q["v"], q["lod"] = mq["u"][sel], mq["v"][sel], mq["lod"][sel]
        ref = torch.full((len(sel) * C,), float("nan"), dtype=torch.float32, device="cuda")
        lib.decode(m, pk[i], wp[i], lib.F16, queries_dev(q), len(sel), ref, lib.F32)
        torch.cuda.synchronize()
        assert np.array_equal(got[sel], ref.cpu().numpy().reshape(-1, C)), i
        g = geometry(m)
        o = O.decode(g, quantized_latents_oracle(g, raws[i]), mlps[i], q)
        assert np.max(np.abs(got[sel] - o)) <= 2e-3
