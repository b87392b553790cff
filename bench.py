#!/usr/bin/env python3
"""Benchmark of the neural texture compression hot path on one MI355X.

Step = one training step (forward, L2 loss, backward into MLP and latents, dense
Adam, clamp, next-step noise) of the full-size FP32-configuration material:
2048x2048x12 with its box-filtered mip chain (12 mips, 5 feature levels of 4-bit
latent grid pairs, G0 512x512x12 at level 0), MLP 72->64->64->12, 262,144 uniform
random (u, v, LOD) samples per step, quantization noise on, learning rates
0.01 / 0.005 with cosine annealing over the run.  `value` is train samples/s of
the FP16 matrix-core path; the FP32 path on the same GPU, the decode throughput
(4096x4096x16, 2/4-bit, MLP 92->64->64->16, 16M random queries per launch and a
coherent full mip-0 pass), the reconstruction PSNR (Eq. 1) after the timed run,
the roofline of the fused training kernel and the FP64 CPU oracle's throughput
are reported beside it.  All inputs are seeded synthetic data resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_F16_TFLOPS = 2500.0   # MI355X dense FP16 matrix peak
PEAK_F32_TFLOPS = 157.3    # MI355X FP32 matrix / vector peak
PEAK_HBM_GBS = 8000.0

TRAIN = dict(W=2048, C=12, c0=12, c1=12, b0=4, b1=4, hidden=64, n=262144, lr_lat=0.01, lr_mlp=0.005)
DECODE = dict(W=4096, C=16, c0=16, c1=16, b0=2, b1=4, hidden=64, train_steps=300)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAIN_SOURCES = ("train.hip", "ntc_device.h", "ntc_internal.h")
DECODE_SOURCES = ("decode.hip", "decode_impl.h", "ntc_device.h", "ntc_internal.h")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "train_fused_kernel_2048x12_counters.md")
DECODE_COUNTERS_FILE = os.path.join(ROOT, "profiles", "decode_kernel_4096x16_counters.md")


def kernel_source_hash(sources=TRAIN_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2305_17105_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_summary(path=COUNTERS_FILE, sources=TRAIN_SOURCES, plan=None):
    """Figures of a committed rocprofv3 counter summary (key: value lines), or None when
    the kernel sources changed since it was taken, or when it was taken with another
    training plan (samples per work item, tile side) than `plan`."""
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#") and line.startswith("- "):
                k, v = line.split(":", 1)
                kv[k.strip().lstrip("- ").strip("`")] = v.strip().strip("`")
        if kv.get("source_sha256") != kernel_source_hash(sources):
            return None
        if plan is not None and kv.get("plan") != plan_text(plan):
            return None
        return kv
    except OSError:
        return None


def plan_text(plan):
    return f"chunk {plan['chunk']}, tile {plan['tile']}"


def counter_traffic(path=COUNTERS_FILE, sources=TRAIN_SOURCES, plan=None):
    """HBM bytes per launch of the profiled kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, each scaled by what the counter reads for a plain
    copy of known size; None when the kernel sources (or the plan) changed since."""
    kv = counter_summary(path, sources, plan)
    try:
        f = float(kv["fetch_kib_per_launch"]) * float(kv["copy_fetch_scale"])
        w = float(kv["write_kib_per_launch"]) * float(kv["copy_write_scale"])
        return int(round((f + w) * 1024))
    except (TypeError, KeyError, ValueError):
        return None


def counter_limiter(path, sources, launch_ms, plan=None):
    """Measured busy fractions of the profiled kernel from its committed SQ counters:
    VALU issue (4 clocks per wave instruction) and matrix cores (16 clocks per 16x16x32
    MFMA) over the launch's SIMD-cycles (256 CUs x 4 SIMDs x 2.4 GHz), and HBM bytes over
    8 TB/s; None without a current summary."""
    kv = counter_summary(path, sources, plan)
    try:
        simd_cycles = 256 * 4 * 2.4e9 * launch_ms * 1e-3
        out = dict(valu_busy=round(float(kv["valu_insts_per_launch"]) * 4 / simd_cycles, 3),
                   mfma_busy=round(float(kv["mfma_insts_per_launch"]) * 16 / simd_cycles, 3))
        tr = counter_traffic(path, sources, plan)
        if tr is not None:
            out["hbm_frac"] = round(tr / (launch_ms * 1e-3) / (PEAK_HBM_GBS * 1e9), 3)
        return out
    except (TypeError, KeyError, ValueError):
        return None


def train_flops_per_sample(K, Hd, C, Klat):
    """Algorithmic FLOPs of one training sample: forward 2(K Hd + Hd^2 + Hd C), input
    gradient through layers 3, 2 and the latent slots of layer 1, and the three weight
    gradients."""
    fwd = 2 * (K * Hd + Hd * Hd + Hd * C)
    bwd_x = 2 * (Hd * C + Hd * Hd + Klat * Hd)
    bwd_w = 2 * (K * Hd + Hd * Hd + Hd * C)
    return fwd + bwd_x + bwd_w


def decode_flops_per_query(K, Hd, C):
    return 2 * (K * Hd + Hd * Hd + Hd * C)


class TrainBench:
    def __init__(self, ntc, synth, torch, seed=0):
        t = TRAIN
        self.ntc, self.torch = ntc, torch
        self.m = ntc.material_init(t["W"], t["W"], t["C"], t["c0"], t["c1"], t["b0"], t["b1"], t["hidden"])
        m = self.m
        log(f"[bench] train material: {t['W']}^2 x {t['C']}, {m.num_mips} mips, {m.num_levels} levels, "
            f"{m.latent_count} latents, K={m.input_width}")
        t0 = time.time()
        self.mips, tflat = synth.target_chain(seed, 0, t["W"], t["W"], t["C"], m.num_mips)
        self.targets = torch.from_numpy(tflat).cuda()
        log(f"[bench] targets generated in {time.time() - t0:.1f}s")
        raw = torch.from_numpy(synth.uniform_latents(seed, int(m.latent_count))).cuda()
        packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        ntc.quantize_latents(m, raw, packed)
        self.lat0 = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
        ntc.dequantize_latents(m, packed, self.lat0)
        self.mlp0 = torch.from_numpy(synth.xavier_mlp(seed, m.input_width, t["hidden"], t["C"])).cuda()
        self.pool = [torch.from_numpy(synth.random_queries(seed + 17 * i, t["n"], m.num_mips).view(np.uint8).copy())
                     .cuda() for i in range(8)]
        self.n = t["n"]

    def run(self, precision, steps, warmup, tune=True):
        ntc, torch = self.ntc, self.torch
        m, n = self.m, self.n
        st = ntc.TrainState(m, self.lat0, self.mlp0, precision)
        ws = torch.zeros(ntc.train_workspace_bytes(m, n, precision), dtype=torch.uint8, device="cuda")
        total = warmup + steps

        def hp(step):
            c = 0.5 * (1.0 + math.cos(math.pi * step / total))
            return ntc.hparams(lr_latent=TRAIN["lr_lat"] * c, lr_mlp=TRAIN["lr_mlp"] * c, step=step,
                               precision=precision, noise=True, seed=1)

        ntc.train_prepare(m, st, hp(0))
        # (samples per work item, tile side) picked by timing the library's candidates on
        # this batch; the tuner runs gradient passes only, the state is prepared afresh
        if tune:
            chunk, tile, tune_us = ntc.train_autotune(m, st, self.pool[0], n, self.targets, hp(0), ws)
            ntc.train_prepare(m, st, hp(0))
        else:
            (chunk, tile), tune_us = ntc.train_get_tuning(m, precision), 0.0
        for s in range(warmup):
            h = hp(s)
            ntc.train_step(m, st, self.pool[s % 8], n, self.targets, h, ws)
        hps = [hp(warmup + i) for i in range(steps)]
        torch.cuda.synchronize()
        # the library records HIP events around each launch of the fused kernel on the
        # launch stream (the roofline's per-launch duration)
        ntc.timing_begin(steps)
        t0 = time.perf_counter()
        for i in range(steps):
            ntc.train_step(m, st, self.pool[(warmup + i) % 8], n, self.targets, hps[i], ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ktot, kcnt = ntc.timing_read("train_fused")
        ntc.timing_end()
        fused_ms = ktot / kcnt
        loss = float(st.loss.cpu()[0])
        return dict(seconds=dt, ms_per_step=dt / steps * 1e3, samples_per_s=n * steps / dt, fused_ms=fused_ms,
                    tuning=dict(chunk=chunk, tile=tile, us_per_gradient_pass=round(tune_us, 1)),
                    loss=loss, state=st)

    def run_paper_schedule(self, precision, steps, seed=3):
        """The paper's optimiser schedule (section 5.1) on this material: batches of eight
        256^2 crops from one LOD (exponential LOD distribution, 5% uniform) generated on
        the device, cosine-annealed learning rates 0.01 / 0.005, noise on; at 95% of the
        steps the latents are quantized and frozen and the network alone trains on."""
        ntc, torch = self.ntc, self.torch
        m = self.m
        n = 8 * 256 * 256
        st = ntc.TrainState(m, self.lat0, self.mlp0, precision)
        ws = torch.zeros(ntc.train_workspace_bytes(m, n, precision), dtype=torch.uint8, device="cuda")
        qbuf = torch.zeros(n * 12, dtype=torch.uint8, device="cuda")
        freeze_at = int(0.95 * steps)
        packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")

        def hp(step, frozen):
            c = 0.5 * (1.0 + math.cos(math.pi * step / steps))
            return ntc.hparams(lr_latent=TRAIN["lr_lat"] * c, lr_mlp=TRAIN["lr_mlp"] * c, step=step,
                               precision=precision, noise=not frozen, freeze=frozen, seed=seed)

        ntc.train_prepare(m, st, hp(0, False))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            frozen = s >= freeze_at
            if s == freeze_at:  # quantize-and-freeze: masters become the dequantized codes
                ntc.quantize_latents(m, st.latents, packed)
                ntc.dequantize_latents(m, packed, st.latents)
                ntc.train_prepare(m, st, hp(s, True))
            ntc.crop_queries(m, seed, s, qbuf)
            ntc.train_step(m, st, qbuf, n, self.targets, hp(s, frozen), ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dict(steps=steps, frozen_from=freeze_at, samples_per_step=n, ms_per_step=dt / steps * 1e3,
                    samples_per_s=n * steps / dt, psnr_db=self.psnr(st), loss=float(st.loss.cpu()[0]))

    def psnr(self, st):
        """Eq. 1 over the full mip chain, decoding the quantized latents in FP32."""
        ntc, torch = self.ntc, self.torch
        from paper_2305_17105_amd import synth
        m = self.m
        packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        ntc.quantize_latents(m, st.latents, packed)
        wp = torch.zeros(ntc.mlp_packed_bytes(m, ntc.F32), dtype=torch.uint8, device="cuda")
        ntc.pack_mlp(m, st.mlp, ntc.F32, wp)
        se = 0.0
        count = 0
        for l in range(m.num_mips):
            q = synth.tile_queries(m.width, m.height, l)
            qd = torch.from_numpy(q.view(np.uint8).copy()).cuda()
            out = torch.empty(len(q) * m.channels, dtype=torch.float32, device="cuda")
            ntc.decode(m, packed, wp, ntc.F32, qd, len(q), out, ntc.F32)
            off = int(m.mip_offset[l])
            ref = self.targets[off:off + out.numel()]
            se += float(((out.double() - ref.double()) ** 2).sum())
            count += out.numel()
        return -10.0 * math.log10(se / count)


def _unit_mlp(synth, K, Hd, C, seed=0):
    p = synth.xavier_mlp(seed, K, Hd, C).astype(np.float64)
    w3 = K * Hd + Hd + Hd * Hd + Hd
    p[w3:w3 + Hd * C] *= 0.25
    p[w3 + Hd * C:] = 0.5
    return p.astype(np.float32)


def run_decode(ntc, synth, torch, nq, reps, seed=0):
    """Decode workload: the 4096^2 x 16 material (G0 2-bit, G1 4-bit) trained briefly in
    FP32 on its own value-noise targets, then decoded with FP16, FP8-e4m3 and FP32
    matrix cores: 16M random (u, v, LOD) queries per launch and the coherent full
    mip 0; PSNR (Eq. 1) of mip 0 for each precision."""
    d = DECODE
    m = ntc.material_init(d["W"], d["W"], d["C"], d["c0"], d["c1"], d["b0"], d["b1"], d["hidden"])
    t0 = time.time()
    targets = synth.target_chain_torch(seed, 1, d["W"], d["W"], d["C"], int(m.num_mips), "cuda")
    raw = torch.from_numpy(synth.uniform_latents(seed, int(m.latent_count))).cuda()
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    ntc.quantize_latents(m, raw, packed)
    lat0 = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
    ntc.dequantize_latents(m, packed, lat0)
    mlp0 = torch.from_numpy(synth.xavier_mlp(seed, m.input_width, d["hidden"], d["C"])).cuda()
    n = TRAIN["n"]
    st = ntc.TrainState(m, lat0, mlp0, ntc.F32)
    ws = torch.zeros(ntc.train_workspace_bytes(m, n, ntc.F32), dtype=torch.uint8, device="cuda")
    pool = [torch.from_numpy(synth.random_queries(seed + 31 * i, n, m.num_mips).view(np.uint8).copy()).cuda()
            for i in range(4)]
    steps = d["train_steps"]
    for s in range(steps):
        c = 0.5 * (1.0 + math.cos(math.pi * s / steps))
        h = ntc.hparams(lr_latent=TRAIN["lr_lat"] * c, lr_mlp=TRAIN["lr_mlp"] * c, step=s, precision=ntc.F32,
                        noise=True, seed=2)
        if s == 0:
            ntc.train_prepare(m, st, h)
        ntc.train_step(m, st, pool[s % 4], n, targets, h, ws)
    ntc.quantize_latents(m, st.latents, packed)
    mlp = st.mlp.clone()
    torch.cuda.synchronize()
    log(f"[bench] decode material: targets + {steps} FP32 training steps in {time.time() - t0:.1f}s")

    q_rand = torch.from_numpy(synth.random_queries(seed + 5, nq, m.num_mips).view(np.uint8).copy()).cuda()
    n_tile = d["W"] * d["W"]
    out = torch.empty(max(nq, n_tile) * d["C"], dtype=torch.float16, device="cuda")
    out32 = torch.empty(n_tile * d["C"], dtype=torch.float32, device="cuda")
    ref0 = targets[:n_tile * d["C"]].double()
    fl_q = decode_flops_per_query(m.input_width, d["hidden"], d["C"])
    res = {"steps_trained_fp32": steps}
    for name, prec in (("f16", ntc.F16), ("fp8", ntc.FP8_E4M3), ("f32", ntc.F32)):
        wp = torch.zeros(ntc.mlp_packed_bytes(m, prec), dtype=torch.uint8, device="cuda")
        ntc.pack_mlp(m, mlp, prec, wp)
        for kind, nn in (("random", nq), ("coherent", n_tile)):
            if kind == "random":
                call = lambda: ntc.decode(m, packed, wp, prec, q_rand, nq, out, ntc.F16)
            else:  # the whole of mip 0 through the rectangle entry point, no query buffer
                call = lambda: ntc.decode_tile(m, packed, wp, prec, 0, 0, 0, d["W"], d["W"], out, ntc.F16)
            for _ in range(2):
                call()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ntc.timing_begin(reps)
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            ktot, kcnt = ntc.timing_read("decode")
            ntc.timing_end()
            ms = e0.elapsed_time(e1) / reps
            kms = ktot / kcnt
            res[f"{kind}_{name}"] = dict(queries=nn, ms=round(ms, 4), kernel_ms=round(kms, 4),
                                         texels_per_s=nn / (ms * 1e-3), tflops=fl_q * nn / (kms * 1e-3) / 1e12)
            log(f"[bench] decode {kind} {name}: {ms:.3f} ms for {nn} queries -> {nn / (ms * 1e-3):.3e} texels/s "
                f"(kernel {kms:.3f} ms)")
        ntc.decode_tile(m, packed, wp, prec, 0, 0, 0, d["W"], d["W"], out32, ntc.F32)
        mse = float(((out32.double() - ref0) ** 2).mean())
        res[f"psnr_mip0_{name}"] = round(-10.0 * math.log10(mse), 3)
    log(f"[bench] decode PSNR of mip 0: f32 {res['psnr_mip0_f32']} dB, f16 {res['psnr_mip0_f16']} dB, "
        f"fp8 {res['psnr_mip0_fp8']} dB")
    # a seeded sample of mip-0 texels decoded by every path, kept for the comparison with
    # the FP64 oracle (made in the CPU-baseline leg)
    ns = ORACLE_SAMPLE
    rs = np.random.default_rng(seed + 9)
    idx = np.sort(rs.choice(n_tile, ns, replace=False))
    qs = np.zeros(ns, dtype=[("u", "<f4"), ("v", "<f4"), ("lod", "<i4")])
    qs["u"] = ((idx % d["W"]) + 0.5) / d["W"]
    qs["v"] = ((idx // d["W"]) + 0.5) / d["W"]
    qs_dev = torch.from_numpy(qs.view(np.uint8).copy()).cuda()
    outs = {}
    for name, prec in (("f32", ntc.F32), ("f16", ntc.F16), ("fp8", ntc.FP8_E4M3)):
        wp = torch.zeros(ntc.mlp_packed_bytes(m, prec), dtype=torch.uint8, device="cuda")
        ntc.pack_mlp(m, mlp, prec, wp)
        o = torch.empty(ns * d["C"], dtype=torch.float32, device="cuda")
        ntc.decode(m, packed, wp, prec, qs_dev, ns, o, ntc.F32)
        outs[name] = o.cpu().numpy().astype(np.float64)
    res["_oracle_sample"] = dict(queries=qs, packed=packed.cpu().numpy(), mlp=mlp.cpu().numpy().astype(np.float64),
                                 targets=targets[:n_tile * d["C"]].view(n_tile, d["C"])[torch.from_numpy(idx).cuda()]
                                 .cpu().numpy().astype(np.float64), outputs=outs)
    # filtered decode (FP16): the same random positions with a continuous LOD
    r = np.random.default_rng(seed + 6)
    fq = np.zeros(nq, dtype=[("u", "<f4"), ("v", "<f4"), ("lod", "<f4")])
    fq["u"] = r.random(nq, dtype=np.float32)
    fq["v"] = r.random(nq, dtype=np.float32)
    fq["lod"] = r.random(nq, dtype=np.float32) * np.float32(m.num_mips - 1)
    fq_dev = torch.from_numpy(fq.view(np.uint8).copy()).cuda()
    del fq
    wp = torch.zeros(ntc.mlp_packed_bytes(m, ntc.F16), dtype=torch.uint8, device="cuda")
    ntc.pack_mlp(m, mlp, ntc.F16, wp)
    for name, mode, taps in (("bilinear", ntc.FILTER_BILINEAR, 4), ("trilinear", ntc.FILTER_TRILINEAR, 8),
                             ("stochastic", ntc.FILTER_STOCHASTIC, 1)):
        call = lambda: ntc.decode_filtered(m, packed, wp, ntc.F16, fq_dev, nq, mode, out, ntc.F16, seed=3)
        for _ in range(2):
            call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"filtered_{name}_f16"] = dict(outputs=nq, texels_decoded=nq * taps, ms=round(ms, 4),
                                          outputs_per_s=nq / (ms * 1e-3),
                                          cost_vs_point_decode=round(ms / res["random_f16"]["ms"], 3))
        log(f"[bench] decode filtered {name} f16: {ms:.3f} ms for {nq} outputs ({taps} texels each) -> "
            f"{nq / (ms * 1e-3):.3e} outputs/s, {ms / res['random_f16']['ms']:.2f}x a point decode")
    return res


ORACLE_SAMPLE = 16384  # mip-0 texels decoded by the FP64 oracle beside each GPU decode path


def _timed_ms(torch, call, reps):
    for _ in range(2):
        call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_small_configs(ntc, synth, torch, reps=20):
    """The two small configurations on their own shapes: a 256^2 x 8 material (G0 64^2 x 8,
    G1 32^2 x 8, 4-bit; MLP 52-64-64-8), 65,536 uniform queries at LOD 0.  Plain FP32
    method: one training step (forward, loss, backward, Adam at lr 1e-2).  Differentiation
    path: FP16 forward + backward through the torch.autograd.Function (L2 loss)."""
    from paper_2305_17105_amd.autograd import ntc_decode_fn
    W, C, n = 256, 8, 65536
    m = ntc.material_init(W, W, C, C, C, 4, 4, 64, num_mips=1)
    raw = torch.from_numpy(synth.uniform_latents(0, int(m.latent_count))).cuda()
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    ntc.quantize_latents(m, raw, packed)
    lat = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
    ntc.dequantize_latents(m, packed, lat)
    mlp = torch.from_numpy(synth.xavier_mlp(0, m.input_width, 64, C)).cuda()
    _, tflat = synth.target_chain(0, 0, W, W, C, 1)
    targets = torch.from_numpy(tflat).cuda()
    q = torch.from_numpy(synth.random_queries(0, n, 1, 0).view(np.uint8).copy()).cuda()
    st = ntc.TrainState(m, lat, mlp, ntc.F32)
    ws = torch.zeros(ntc.train_workspace_bytes(m, n, ntc.F32), dtype=torch.uint8, device="cuda")
    hp = ntc.hparams(lr_latent=1e-2, lr_mlp=1e-2, step=0, precision=ntc.F32, noise=False)
    ntc.train_prepare(m, st, hp)
    ms1 = _timed_ms(torch, lambda: ntc.train_step(m, st, q, n, targets, hp, ws), reps)
    tq = targets.view(W * W, C)  # n = W * W: one target row per query

    lat_p = lat.clone().requires_grad_(True)
    mlp_p = mlp.clone().requires_grad_(True)

    def fwd_bwd():
        y = ntc_decode_fn(m, lat_p, mlp_p, q, ntc.F16)
        loss = ((y - tq) ** 2).mean()
        loss.backward()
    ms3 = _timed_ms(torch, fwd_bwd, reps)
    out = {"config1_fp32_train_step": dict(material="256x256x8, G0 64^2x8 / G1 32^2x8 4-bit, MLP 52-64-64-8",
                                           samples=n, ms=round(ms1, 4), samples_per_s=n / (ms1 * 1e-3)),
           "config3_fp16_autograd_fwd_bwd": dict(material="as config 1", samples=n, ms=round(ms3, 4),
                                                 samples_per_s=n / (ms3 * 1e-3))}
    log(f"[bench] config 1 FP32 step: {ms1:.3f} ms ({n / (ms1 * 1e-3):.3e} samples/s); config 3 FP16 autograd "
        f"forward+backward: {ms3:.3f} ms ({n / (ms3 * 1e-3):.3e} samples/s)")
    return out


def run_profile(ntc, synth, torch, steps, warmup, nq, reps, seed=21):
    """Table 3's NTC 1.0 profile on the table's 4096^2 x 9 reference size with the paper's
    network (hardGELU, LOD input, triangle-wave encoding): G0 2048^2 x 12 at 2 bits, G1
    1024^2 x 10 at 4 bits.  FP16 training steps of 262,144 random samples, then FP16
    decode of 16M random queries and of the full coherent mip 0."""
    W, C = 4096, 9
    m = ntc.material_init(W, W, C, 12, 10, 2, 4, 64, grid_shift=1, activation=ntc.ACT_HARDGELU, lod_input=1,
                          posenc=ntc.PE_TRIANGLE)
    targets = synth.target_chain_torch(seed, 2, W, W, C, int(m.num_mips), "cuda")
    raw = torch.from_numpy(synth.uniform_latents(seed, int(m.latent_count))).cuda()
    packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
    ntc.quantize_latents(m, raw, packed)
    lat = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
    ntc.dequantize_latents(m, packed, lat)
    del raw
    mlp = torch.from_numpy(synth.xavier_mlp(seed, m.input_width, 64, C)).cuda()
    n = TRAIN["n"]
    st = ntc.TrainState(m, lat, mlp, ntc.F16)
    ws = torch.zeros(ntc.train_workspace_bytes(m, n, ntc.F16), dtype=torch.uint8, device="cuda")
    pool = [torch.from_numpy(synth.random_queries(seed + 13 * i, n, m.num_mips).view(np.uint8).copy()).cuda()
            for i in range(4)]
    hps = [ntc.hparams(lr_latent=TRAIN["lr_lat"], lr_mlp=TRAIN["lr_mlp"], step=s, precision=ntc.F16, noise=True,
                       seed=4) for s in range(warmup + steps)]
    ntc.train_prepare(m, st, hps[0])
    for s in range(warmup):
        ntc.train_step(m, st, pool[s % 4], n, targets, hps[s], ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ntc.train_step(m, st, pool[(warmup + i) % 4], n, targets, hps[warmup + i], ws)
    torch.cuda.synchronize()
    tms = (time.perf_counter() - t0) / steps * 1e3
    ntc.quantize_latents(m, st.latents, packed)
    wp = torch.zeros(ntc.mlp_packed_bytes(m, ntc.F16), dtype=torch.uint8, device="cuda")
    ntc.pack_mlp(m, st.mlp, ntc.F16, wp)
    q = torch.from_numpy(synth.random_queries(seed + 5, nq, m.num_mips).view(np.uint8).copy()).cuda()
    out = torch.empty(max(nq, W * W) * C, dtype=torch.float16, device="cuda")
    ms_r = _timed_ms(torch, lambda: ntc.decode(m, packed, wp, ntc.F16, q, nq, out, ntc.F16), reps)
    ms_c = _timed_ms(torch, lambda: ntc.decode_tile(m, packed, wp, ntc.F16, 0, 0, 0, W, W, out, ntc.F16), reps)
    fq = decode_flops_per_query(m.input_width, 64, C)
    res = dict(profile="NTC 1.0 (Table 3): 4096x4096x9, G0 2048^2 x 12 at 2 bits, G1 1024^2 x 10 at 4 bits, "
                       "MLP 71-64-64-9 (hardGELU, LOD input, triangle waves)",
               packed_mib=round(int(m.packed_bytes) / 2 ** 20, 3),
               train_f16=dict(samples=n, ms_per_step=round(tms, 4), samples_per_s=n / (tms * 1e-3),
                              steps=steps, loss=float(st.loss.cpu()[0])),
               decode_random_f16=dict(queries=nq, ms=round(ms_r, 4), texels_per_s=nq / (ms_r * 1e-3),
                                      tflops=fq * nq / (ms_r * 1e-3) / 1e12),
               decode_coherent_f16=dict(queries=W * W, ms=round(ms_c, 4), texels_per_s=W * W / (ms_c * 1e-3),
                                        tflops=fq * W * W / (ms_c * 1e-3) / 1e12))
    log(f"[bench] NTC 1.0 profile 4096^2 x 9: train f16 {tms:.3f} ms/step ({n / (tms * 1e-3):.3e} samples/s); "
        f"decode random f16 {ms_r:.3f} ms ({nq / (ms_r * 1e-3):.3e} texels/s), coherent mip 0 {ms_c:.3f} ms")
    return res


BATCH = dict(materials=64, samples=4 * 2 ** 20, steps=20, warmup=3, decode_queries=4 * 2 ** 20)


def batched_materials(seed=7, count=64):
    """Seeded uneven material set: side 2^9..2^12 (log-uniform), C in {8, 10, 12, 16}
    with C0 = C1 = C at 4 bits, hidden width 32 or 64."""
    r = np.random.Generator(np.random.PCG64([seed, 505]))
    sides = 2 ** r.integers(9, 13, count)
    chans = r.choice([8, 10, 12, 16], count)
    widths = r.choice([32, 64], count)
    return [(int(w), int(c), int(h)) for w, c, h in zip(sides, chans, widths)]


def run_batched(ntc, synth, torch, steps, warmup, seed=7):
    """Many-material workload: every material trained (FP16 matrix cores) in one grouped
    step (one launch per stage, the fused kernel per material) captured in a HIP graph
    and replayed, samples per material proportional to its area; then decoded grouped
    (one launch per kernel shape; queries proportional to area) and through the coherent
    rectangle entry point (all of mip 0).  Tile shapes per (hidden width, channels) come
    from the step tuner."""
    b = BATCH
    spec = batched_materials(seed, b["materials"])
    t0 = time.time()
    mats, states, targets, nsamp = [], [], [], []
    area = np.array([w * w for w, _, _ in spec], dtype=np.float64)
    shares = np.maximum(1, np.floor(b["samples"] * area / area.sum())).astype(np.int64)
    for i, (w, c, hd) in enumerate(spec):
        m = ntc.material_init(w, w, c, c, c, 4, 4, hd)
        raw = torch.from_numpy(synth.uniform_latents(seed * 1000 + i, int(m.latent_count))).cuda()
        packed = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        ntc.quantize_latents(m, raw, packed)
        lat = torch.zeros(int(m.latent_count), dtype=torch.float32, device="cuda")
        ntc.dequantize_latents(m, packed, lat)
        mlp = torch.from_numpy(synth.xavier_mlp(seed * 1000 + i, m.input_width, hd, c)).cuda()
        mats.append(m)
        states.append(ntc.TrainState(m, lat, mlp, ntc.F16))
        targets.append(synth.target_chain_torch(seed, 100 + i, w, w, c, int(m.num_mips), "cuda"))
        nsamp.append(int(shares[i]))
    offsets = np.concatenate([[0], np.cumsum(nsamp)])
    ntot = int(offsets[-1])
    qpool = []
    for k in range(2):
        qs = [synth.random_queries(seed * 7919 + 31 * i + k, n, int(m.num_mips)) for i, (m, n) in
              enumerate(zip(mats, nsamp))]
        qpool.append(torch.from_numpy(np.concatenate(qs).view(np.uint8).copy()).cuda())
    ws = torch.zeros(ntc.train_workspace_bytes_batched(mats, offsets, ntc.F16), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    log(f"[bench] batched: {len(mats)} materials, {int(area.sum())} mip-0 texels, "
        f"{sum(int(m.latent_count) for m in mats)} latents, {ntot} samples/step, set-up {time.time() - t0:.1f}s")

    # tuner: one representative (the largest) material per (hidden width, channels)
    tuned = {}
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    lr_dev = torch.tensor([TRAIN["lr_lat"], TRAIN["lr_mlp"]], dtype=torch.float32, device="cuda")
    hp = ntc.hparams(precision=ntc.F16, step=0, seed=11, noise=True, step_dev=step_dev, lr_dev=lr_dev)
    hp_host = ntc.hparams(precision=ntc.F16, step=0, seed=11, noise=True)
    for m, st in zip(mats, states):
        ntc.train_prepare(m, st, hp_host)
    for key in sorted({(m.hidden, m.channels) for m in mats}):
        i = max((j for j, m in enumerate(mats) if (m.hidden, m.channels) == key), key=lambda j: mats[j].width)
        n = nsamp[i]
        wsi = torch.zeros(ntc.train_workspace_bytes(mats[i], n, ntc.F16), dtype=torch.uint8, device="cuda")
        qi = qpool[0][offsets[i] * 12:offsets[i + 1] * 12]
        chunk, tile, us = ntc.train_autotune(mats[i], states[i], qi, n, targets[i], hp_host, wsi)
        tuned[f"hidden{key[0]}_c{key[1]}"] = dict(chunk=chunk, tile=tile, us_per_gradient_pass=round(us, 1),
                                                  tuned_on=f"{mats[i].width}^2, {n} samples")
        del wsi
    for m, st in zip(mats, states):
        ntc.train_prepare(m, st, hp_host)
    log(f"[bench] batched: tuned tiles {tuned}")

    # eager steps with per-material launches, eager grouped steps (one launch per
    # stage), then one captured grouped step replayed
    for s in range(warmup):
        ntc.train_step_batched(mats, states, qpool[s % 2], offsets, targets, hp, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(steps):
        ntc.train_step_batched(mats, states, qpool[s % 2], offsets, targets, hp, ws)
    torch.cuda.synchronize()
    per_material_ms = (time.perf_counter() - t1) / steps * 1e3
    table = ntc.TrainTable(mats, states, offsets, targets, ntc.F16, ws)
    for s in range(warmup):
        ntc.train_step_grouped(table, qpool[s % 2], hp)
    torch.cuda.synchronize()
    # the library's HIP events around the fused launches (one per kernel shape) give the
    # fused part of the eager steps
    ntc.timing_begin(64 * steps)
    t1 = time.perf_counter()
    for s in range(steps):
        ntc.train_step_grouped(table, qpool[s % 2], hp)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t1) / steps * 1e3
    fused_tot, fused_cnt = ntc.timing_read("train_fused")
    ntc.timing_end()
    fused_step_ms = fused_tot / steps
    step_flop = sum(float(offsets[i + 1] - offsets[i]) * train_flops_per_sample(
        m.input_width, m.hidden, m.channels, 4 * m.c0 + m.c1) for i, m in enumerate(mats))
    graphs = []
    stream = torch.cuda.Stream()
    for k in range(2):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(g, stream=stream):
                ntc.train_step_grouped(table, qpool[k], hp)
        graphs.append(g)
    torch.cuda.synchronize()
    graphs[0].replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(steps):
        graphs[s % 2].replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t1) / steps * 1e3
    loss = float(np.mean([float(st.loss.cpu()[0]) for st in states]))
    log(f"[bench] batched train: per-material launches {per_material_ms:.3f} ms/step, grouped eager "
        f"{eager_ms:.3f} ms/step (fused launches {fused_step_ms:.3f} ms in {fused_cnt // steps} launches), grouped "
        f"graph replay {graph_ms:.3f} ms/step -> {ntot / (graph_ms * 1e-3):.3e} samples/s, mean loss {loss:.5f}, "
        f"step index {int(step_dev.item())}")
    del graphs, table, ws

    # decode: random queries proportional to area in one batched call; coherent mip 0
    packed, wpacks = [], []
    for m, st in zip(mats, states):
        p = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        ntc.quantize_latents(m, st.latents, p)
        w = torch.zeros(ntc.mlp_packed_bytes(m, ntc.F16), dtype=torch.uint8, device="cuda")
        ntc.pack_mlp(m, st.mlp, ntc.F16, w)
        packed.append(p)
        wpacks.append(w)
    dq = np.maximum(1, np.floor(b["decode_queries"] * area / area.sum())).astype(np.int64)
    doff = np.concatenate([[0], np.cumsum(dq)])
    qd = torch.from_numpy(np.concatenate([synth.random_queries(seed * 31 + i, int(n), int(m.num_mips)) for i, (m, n)
                                          in enumerate(zip(mats, dq))]).view(np.uint8).copy()).cuda()
    out = torch.empty(int(sum(int(n) * m.channels for n, m in zip(dq, mats))), dtype=torch.float16, device="cuda")
    for _ in range(2):
        ntc.decode_batched(mats, packed, wpacks, ntc.F16, qd, doff, out, ntc.F16)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        ntc.decode_batched(mats, packed, wpacks, ntc.F16, qd, doff, out, ntc.F16)
    torch.cuda.synchronize()
    dec_ms = (time.perf_counter() - t1) / 5 * 1e3
    nd = int(doff[-1])
    # the same batch grouped: one launch per kernel shape
    table = ntc.DecodeTable(mats, packed, wpacks, ntc.F16)
    out_g = torch.empty_like(out)
    for _ in range(2):
        ntc.decode_grouped(table, qd, doff, out_g, ntc.F16)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        ntc.decode_grouped(table, qd, doff, out_g, ntc.F16)
    torch.cuda.synchronize()
    grp_ms = (time.perf_counter() - t1) / 5 * 1e3
    grp_same = bool(torch.equal(out_g, out))
    per_shape = {}
    for m, n in zip(mats, dq):
        if n > 0:
            k = (m.c0, m.c1, m.channels, m.hidden, m.b0, m.b1, m.activation, m.posenc)
            per_shape[k] = per_shape.get(k, 0) + 1
    classes = sum((c + 31) // 32 for c in per_shape.values())  # launches: at most 32 materials each
    big = max(int(m.width) ** 2 * m.channels for m in mats)
    tile_out = torch.empty(big, dtype=torch.float16, device="cuda")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for m, p, w in zip(mats, packed, wpacks):
        ntc.decode_tile(m, p, w, ntc.F16, 0, 0, 0, m.width, m.height, tile_out, ntc.F16)
    torch.cuda.synchronize()
    coh_ms = (time.perf_counter() - t1) * 1e3
    log(f"[bench] grouped decode: {nd} random queries in {classes} launches {grp_ms:.3f} ms -> "
        f"{nd / (grp_ms * 1e-3):.3e} texels/s (equal to per-material launches: {grp_same})")
    log(f"[bench] batched decode: {nd} random queries {dec_ms:.3f} ms -> {nd / (dec_ms * 1e-3):.3e} texels/s; "
        f"coherent mip 0 of all materials ({int(area.sum())} texels) {coh_ms:.3f} ms -> "
        f"{area.sum() / (coh_ms * 1e-3):.3e} texels/s")
    return dict(materials=len(mats), mip0_texels=int(area.sum()), samples_per_step=ntot,
                train_ms_per_step_graph=round(graph_ms, 4), train_ms_per_step_eager=round(eager_ms, 4),
                train_ms_per_step_per_material_launches=round(per_material_ms, 4),
                train_samples_per_s=ntot / (graph_ms * 1e-3), mean_loss=loss, tuned_tiles=tuned,
                train_fused_ms_per_step_eager=round(fused_step_ms, 4), fused_launches_per_step=fused_cnt // steps,
                train_flop_per_step=step_flop,
                fused_mfma_frac=round(step_flop / (fused_step_ms * 1e-3) / (PEAK_F16_TFLOPS * 1e12), 4),
                step_mfma_frac=round(step_flop / (graph_ms * 1e-3) / (PEAK_F16_TFLOPS * 1e12), 4),
                decode_random=dict(queries=nd, ms=round(dec_ms, 4), texels_per_s=nd / (dec_ms * 1e-3),
                                   launches=sum(1 for n in dq if n > 0)),
                decode_random_grouped=dict(queries=nd, ms=round(grp_ms, 4), texels_per_s=nd / (grp_ms * 1e-3),
                                           launches=classes, equal_to_per_material=grp_same),
                decode_coherent_mip0=dict(texels=int(area.sum()), ms=round(coh_ms, 4),
                                          texels_per_s=float(area.sum() / (coh_ms * 1e-3))))


def run_mixed(ntc, synth, torch, nq=4 * 2 ** 20, reps=5, seed=11):
    """Mixed-material decode (Appendix A): 8 materials of the decode shape (16 channels,
    2/4-bit, hidden 64; sides 512..4096), 4M queries naming their material in random
    order, in runs of 64 (screen regions), and for comparison sorted by material and
    decoded grouped."""
    d = DECODE
    r = np.random.default_rng(seed)
    mats, packed, wpacks = [], [], []
    for i in range(8):
        w = int(2 ** (9 + i % 4))
        m = ntc.material_init(w, w, d["C"], d["c0"], d["c1"], d["b0"], d["b1"], d["hidden"])
        raw = torch.from_numpy(synth.uniform_latents(seed + i, int(m.latent_count))).cuda()
        p = torch.zeros(int(m.packed_bytes), dtype=torch.uint8, device="cuda")
        ntc.quantize_latents(m, raw, p)
        mlp = torch.from_numpy(synth.xavier_mlp(seed + i, m.input_width, d["hidden"], d["C"])).cuda()
        wp = torch.zeros(ntc.mlp_packed_bytes(m, ntc.F16), dtype=torch.uint8, device="cuda")
        ntc.pack_mlp(m, mlp, ntc.F16, wp)
        mats.append(m); packed.append(p); wpacks.append(wp)
    table = ntc.DecodeTable(mats, packed, wpacks, ntc.F16)
    out = torch.empty(nq * d["C"], dtype=torch.float16, device="cuda")

    def timed(call):
        for _ in range(2):
            call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {}
    for order in ("random", "runs64"):
        mat = r.integers(0, 8, nq) if order == "random" else np.repeat(r.integers(0, 8, nq // 64 + 1), 64)[:nq]
        mq = np.zeros(nq, dtype=ntc.MIXED_QUERY_DTYPE)
        mq["u"] = r.random(nq, dtype=np.float32)
        mq["v"] = r.random(nq, dtype=np.float32)
        mq["material"] = mat
        mq["lod"] = np.floor(r.random(nq) * np.array([m.num_mips for m in mats])[mat]).astype(np.int32)
        mq_dev = torch.from_numpy(mq.view(np.uint8).copy()).cuda()
        ms = timed(lambda: ntc.decode_mixed(table, mq_dev, nq, out, ntc.F16))
        res[order] = dict(queries=nq, ms=round(ms, 4), texels_per_s=nq / (ms * 1e-3))
        log(f"[bench] mixed-material decode ({order}, 8 materials): {ms:.3f} ms for {nq} queries -> "
            f"{nq / (ms * 1e-3):.3e} texels/s")
        if order == "random":  # the same queries sorted by material, decoded grouped
            idx = np.argsort(mat, kind="stable")
            qs = np.zeros(nq, dtype=synth.QUERY_DTYPE)
            qs["u"], qs["v"], qs["lod"] = mq["u"][idx], mq["v"][idx], mq["lod"][idx]
            offs = np.concatenate([[0], np.cumsum(np.bincount(mat, minlength=8))])
            qs_dev = torch.from_numpy(qs.view(np.uint8).copy()).cuda()
            ms = timed(lambda: ntc.decode_grouped(table, qs_dev, offs, out, ntc.F16))
            res["sorted_grouped"] = dict(queries=nq, ms=round(ms, 4), texels_per_s=nq / (ms * 1e-3))
            log(f"[bench] same queries sorted by material, grouped decode: {ms:.3f} ms -> "
                f"{nq / (ms * 1e-3):.3e} texels/s")
    return res


def cpu_baseline():
    """FP64 oracle on the host: one training step of the same material, gradient part
    on 32,768 of the 262,144 samples, dense per-latent part (noise, Adam, clamp) on all
    latents; per-step time extrapolated linearly in the sample count."""
    from oracle import ntc_oracle as O
    from paper_2305_17105_amd import synth
    t = TRAIN
    g = O.make_geometry(t["W"], t["W"], t["C"], t["c0"], t["c1"], t["b0"], t["b1"], Hd=t["hidden"])
    _, tflat = synth.target_chain(0, 0, t["W"], t["W"], t["C"], g.M)
    lat = O.dequantize_packed(g, O.quantize_latents(g, synth.uniform_latents(0, g.latent_count)))
    mlp = synth.xavier_mlp(0, g.K, t["hidden"], t["C"]).astype(np.float64)
    ns = 32768
    q = synth.random_queries(1, ns, g.M)
    t0 = time.perf_counter()
    fwd = lat + O.noise_values(g, 1, 0)
    t1 = time.perf_counter()
    _, gp, gl, _ = O.loss_and_grads(g, fwd, mlp, q, tflat)
    t2 = time.perf_counter()
    O.adam_update(mlp, gp, np.zeros_like(mlp), np.zeros_like(mlp), 1, 0.005)
    p, _, _ = O.adam_update(lat, gl, np.zeros_like(lat), np.zeros_like(lat), 1, 0.01)
    O.clamp_latents(g, p)
    t3 = time.perf_counter()
    dense = (t1 - t0) + (t3 - t2)
    per_step = (t2 - t1) * (t["n"] / ns) + dense
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = 1
    return dict(value=t["n"] / per_step, unit="samples/s", cores=int(cores), kind="oracle",
                sample=f"one FP64 oracle training step on the full-size material: gradients of {ns} of the "
                       f"{t['n']} samples ({t2 - t1:.2f}s) extrapolated x{t['n'] // ns}, plus the dense noise/Adam/"
                       f"clamp pass over all {g.latent_count} latents ({dense:.2f}s)", extrapolated=True,
                cpu=_cpu_model())


def oracle_psnr(sample):
    """PSNR (Eq. 1, peak 1) of a seeded sample of mip-0 texels of the decode material
    against its targets: the FP64 oracle's decode of the same packed latents and weights,
    and every GPU decode path's, with the delta and max-abs difference to the oracle."""
    from oracle import ntc_oracle as O
    d = DECODE
    g = O.make_geometry(d["W"], d["W"], d["C"], d["c0"], d["c1"], d["b0"], d["b1"], Hd=d["hidden"])
    lat = O.dequantize_packed(g, sample["packed"])
    t0 = time.perf_counter()
    ref = O.decode(g, lat, sample["mlp"], sample["queries"])
    dt = time.perf_counter() - t0
    t = sample["targets"]

    def psnr(y):
        return -10.0 * math.log10(float(np.mean((y.reshape(t.shape) - t) ** 2)))
    p_or = psnr(ref)
    out = dict(texels=len(sample["queries"]), oracle_psnr_db=round(p_or, 4), oracle_seconds=round(dt, 2))
    for name, y in sample["outputs"].items():
        p = psnr(y)
        out[name] = dict(psnr_db=round(p, 4), delta_db=round(p - p_or, 4),
                         max_abs_vs_oracle=float(np.max(np.abs(y.reshape(ref.shape) - ref))))
    log(f"[bench] PSNR vs FP64 oracle on {len(t)} mip-0 texels: oracle {p_or:.3f} dB; " +
        ", ".join(f"{k} {v['delta_db']:+.4f} dB (max-abs {v['max_abs_vs_oracle']:.2e})"
                  for k, v in out.items() if isinstance(v, dict)))
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--decode-queries", type=int, default=16 * 2 ** 20)
    ap.add_argument("--decode-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-decode", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="train the benchmark material with its untuned plan (profiling runs)")
    ap.add_argument("--no-paper-schedule", action="store_true")
    ap.add_argument("--paper-steps", type=int, default=1000)
    ap.add_argument("--no-small", action="store_true", help="skip the two small configurations")
    ap.add_argument("--no-profile", action="store_true", help="skip Table 3's NTC 1.0 profile at 4096^2 x 9")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the method trains and decodes one material per GPU and this "
              "build has no multi-GPU path (materials or query batches would be sharded across GPUs with no "
              "exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_17105_amd import ntc, synth
    torch.cuda.set_device(0)

    tb = TrainBench(ntc, synth, torch)
    log("[bench] FP32 training run")
    r32 = tb.run(ntc.F32, args.steps, args.warmup, tune=not args.no_tune)
    log(f"[bench] f32: {r32['ms_per_step']:.3f} ms/step, fused {r32['fused_ms']:.3f} ms, loss {r32['loss']:.5f}, "
        f"tuning {r32['tuning']}")
    psnr32 = tb.psnr(r32.pop("state"))
    log("[bench] FP16 training run")
    r16 = tb.run(ntc.F16, args.steps, args.warmup, tune=not args.no_tune)
    log(f"[bench] f16: {r16['ms_per_step']:.3f} ms/step, fused {r16['fused_ms']:.3f} ms, loss {r16['loss']:.5f}, "
        f"tuning {r16['tuning']}")
    psnr16 = tb.psnr(r16.pop("state"))
    log(f"[bench] PSNR after {args.warmup + args.steps} steps: f16 {psnr16:.2f} dB, f32 {psnr32:.2f} dB")

    paper = None
    if not args.no_paper_schedule:
        paper = tb.run_paper_schedule(ntc.F16, args.paper_steps)
        log(f"[bench] paper schedule f16 ({paper['steps']} steps of 8 x 256^2 crops, frozen from "
            f"{paper['frozen_from']}): {paper['ms_per_step']:.3f} ms/step -> {paper['samples_per_s']:.3e} samples/s, "
            f"PSNR {paper['psnr_db']:.2f} dB")

    m = tb.m
    fps = train_flops_per_sample(m.input_width, m.hidden, m.channels, 4 * m.c0 + m.c1)
    ach = fps * tb.n / (r16["fused_ms"] * 1e-3) / 1e12
    # Algorithmic HBM bytes of a launch: the queries (12 B), FP32 targets, one read of the
    # FP32 forward latents and one write of the FP32 latent gradient.  The bound is the roof
    # whose floor is the longer (matrix work at the FP16 peak, or these bytes at 8 TB/s: the
    # two are within 10% here); `limiter` gives the measured busy fractions of the VALU,
    # the matrix cores and HBM from the committed counters of the same source.
    abytes = tb.n * (12 + 4 * m.channels) + 2 * 4 * int(m.latent_count)
    t_mfma = fps * tb.n / (PEAK_F16_TFLOPS * 1e12)
    t_hbm = abytes / (PEAK_HBM_GBS * 1e9)
    hbm_ach = abytes / (r16["fused_ms"] * 1e-3) / 1e9
    if t_hbm > t_mfma:
        roof = dict(bound="hbm", kernel="train_fused_kernel (FP16)", achieved=round(hbm_ach, 1), peak=PEAK_HBM_GBS,
                    unit="GB/s", frac=round(hbm_ach / PEAK_HBM_GBS, 4))
    else:
        roof = dict(bound="mfma", kernel="train_fused_kernel (FP16)", achieved=round(ach, 2), peak=PEAK_F16_TFLOPS,
                    unit="TFLOP/s", frac=round(ach / PEAK_F16_TFLOPS, 4))
    roof.update(traffic=counter_traffic(COUNTERS_FILE, TRAIN_SOURCES, r16["tuning"]),
                algorithmic_bytes=abytes, flops_per_sample=fps, samples_per_launch=tb.n,
                avg_launch_ms=round(r16["fused_ms"], 4), mfma_tflops=round(ach, 2),
                mfma_frac=round(ach / PEAK_F16_TFLOPS, 4), hbm_frac_algorithmic=round(hbm_ach / PEAK_HBM_GBS, 4),
                floor_us=dict(mfma=round(t_mfma * 1e6, 2), hbm=round(t_hbm * 1e6, 2)),
                limiter=counter_limiter(COUNTERS_FILE, TRAIN_SOURCES, r16["fused_ms"], r16["tuning"]))
    ach32 = fps * tb.n / (r32["fused_ms"] * 1e-3) / 1e12

    decode = None
    decode_roof = None
    oracle_sample = None
    if not args.no_decode:
        decode = run_decode(ntc, synth, torch, args.decode_queries, args.decode_reps)
        oracle_sample = decode.pop("_oracle_sample")
        decode["mixed_material"] = run_mixed(ntc, synth, torch)
        d = DECODE
        fq = decode_flops_per_query(d["c0"] * 4 + d["c1"] + 12, d["hidden"], d["C"])
        kms = decode["random_f16"]["kernel_ms"]
        achd = fq * args.decode_queries / (kms * 1e-3) / 1e12
        decode_roof = dict(bound="mfma", kernel="decode_kernel (FP16, 4096^2 x 16, G0 2-bit / G1 4-bit, random)",
                           achieved=round(achd, 2), peak=PEAK_F16_TFLOPS, unit="TFLOP/s",
                           frac=round(achd / PEAK_F16_TFLOPS, 4),
                           traffic=counter_traffic(DECODE_COUNTERS_FILE, DECODE_SOURCES), flops_per_query=fq,
                           queries_per_launch=args.decode_queries, avg_launch_ms=kms,
                           limiter=counter_limiter(DECODE_COUNTERS_FILE, DECODE_SOURCES, kms))
        log(f"[bench] decode roofline (FP16 random): {achd:.1f} TFLOP/s = {achd / PEAK_F16_TFLOPS:.3f} of peak")

    small = None
    if not args.no_small:
        small = run_small_configs(ntc, synth, torch)

    profile = None
    if not args.no_profile:
        profile = run_profile(ntc, synth, torch, max(5, min(args.steps, 20)), 3, args.decode_queries,
                              max(3, min(args.decode_reps, 10)))

    batched = None
    if not args.no_batched:
        batched = run_batched(ntc, synth, torch, BATCH["steps"], BATCH["warmup"])

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host")
        cpu = cpu_baseline()
        if oracle_sample is not None:
            cpu["decode_psnr_vs_oracle"] = oracle_psnr(oracle_sample)

    out = {
        "metric": "decoded texels/s + train samples/s (fwd+bwd), FP16 MFMA vs FP32 at stated PSNR",
        "value": round(r16["samples_per_s"], 1),
        "unit": "train samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r16["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": "train step, 2048x2048x12 + 12-mip chain, 5 levels of 4-bit 512^2/256^2 (level 0) "
                               "latent grids, MLP 72-64-64-12, 262144 random (u,v,LOD) samples, noise on",
                   "global_batch": tb.n, "parallelism": "single GPU"},
        "psnr_db": {"f16": round(psnr16, 3), "f32": round(psnr32, 3), "steps_trained": args.warmup + args.steps},
        "fp32": {"value": round(r32["samples_per_s"], 1), "unit": "train samples/s",
                 "ms_per_step": round(r32["ms_per_step"], 4), "fused_ms": round(r32["fused_ms"], 4),
                 "fused_tflops": round(ach32, 2), "fused_frac_of_fp32_peak": round(ach32 / PEAK_F32_TFLOPS, 4),
                 "tuning": r32["tuning"]},
        "fused_ms_f16": round(r16["fused_ms"], 4),
        "tuning_f16": r16["tuning"],
        "paper_schedule_f16": paper,
        "decode": decode,
        "decode_roofline": decode_roof,
        "small_configs": small,
        "table3_profile": profile,
        "batched": batched,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
