"""Input generators: the torch value-noise path reproduces the numpy one bit for bit."""
import numpy as np

from paper_2305_17105_amd import synth


def test_target_chain_torch_matches_numpy():
    _, flat = synth.target_chain(3, 1, 128, 64, 5, 8)
    t = synth.target_chain_torch(3, 1, 128, 64, 5, 8, "cpu").numpy()
    assert t.dtype == np.float32 and np.array_equal(flat, t)


def test_value_noise_range_and_period():
    img = synth.value_noise(0, 0, 64, 64, 3)
    assert img.min() >= 0.0 and img.max() <= 1.0
    assert img.std() > 0.01
