"""Writes trained_decode_256x16.npz: a 256^2 x 16-channel material (G0 2-bit, G1 4-bit,
MLP 92-64-64-16) trained by the float64 oracle alone, for decode parity on realistic
weights (the precision bars apply to trained networks whose outputs lie in [0, 1]).

    python tests/golden/make_trained_decode_fixture.py

Training: 1,000 oracle steps (section 4.5: L2 loss, Adam; section 4.2: quantization
noise) of 8,192 uniform random (u, v, LOD) samples each on seeded 4-octave value-noise
targets with the full box-filtered mip chain, learning rates 0.01 (latents) / 0.005
(network) with cosine annealing.  Stored: the network (float32, canonical layout) and
the latents quantized by the oracle's packer (bytes of the canonical packed layout).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ntc_oracle as O  # noqa: E402
from paper_2305_17105_amd import synth  # noqa: E402

SHAPE = dict(W=256, C=16, C0=16, C1=16, B0=2, B1=4, Hd=64)
OUT = os.path.join(HERE, "trained_decode_256x16.npz")


def geometry():
    s = SHAPE
    return O.make_geometry(s["W"], s["W"], s["C"], s["C0"], s["C1"], s["B0"], s["B1"], Hd=s["Hd"])


def main(steps=1000, n=8192):
    g = geometry()
    _, tflat = synth.target_chain(0, 1, g.W, g.H, g.C, g.M)
    lat = O.dequantize_packed(g, O.quantize_latents(g, synth.uniform_latents(0, g.latent_count)))
    mlp = synth.xavier_mlp(0, g.K, g.Hd, g.C).astype(np.float64)
    P = len(mlp)
    st = dict(latents=lat, mlp=mlp, lat_m=np.zeros(g.latent_count), lat_v=np.zeros(g.latent_count),
              mlp_m=np.zeros(P), mlp_v=np.zeros(P))
    for s in range(steps):
        c = 0.5 * (1.0 + np.cos(np.pi * s / steps))
        q = synth.random_queries(1000 + s, n, g.M)
        st, L, _ = O.train_step(g, st, q, tflat,
                                dict(lr_latent=0.01 * c, lr_mlp=0.005 * c, seed=2, step=s, noise=True))
        if s % 100 == 0:
            print(f"step {s}: loss {L:.5f}", flush=True)
    packed = O.quantize_latents(g, st["latents"])
    np.savez_compressed(OUT, mlp=st["mlp"].astype(np.float32), packed=packed,
                        shape=np.array([SHAPE[k] for k in ("W", "C", "C0", "C1", "B0", "B1", "Hd")]))
    print(f"wrote {OUT}: loss {L:.5f}")


if __name__ == "__main__":
    main()
