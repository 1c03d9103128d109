"""The seeded input generators: the torch form of the label-keyed values equals the numpy form."""
import numpy as np
import torch

from synth.vectors import label_keyed_values, label_keyed_values_torch


def test_label_keyed_torch_equals_numpy():
    rng = np.random.default_rng(3)
    lab = rng.integers(0, 2 ** 63 - 1, 4000, dtype=np.int64).view(np.uint64)
    lab[:4] = [0, (1 << 40) - 1, (1 << 63) + 5, (1 << 64) - 1]      # 64-bit labels too
    k = rng.integers(0, 12, 4000).astype(np.uint64)
    v = rng.integers(0, 256, 4000).astype(np.uint64)
    for seed in (0, 0x5EED0005, (1 << 63) + 17):
        a = label_keyed_values(seed, lab, k, v)
        b = label_keyed_values_torch(seed, torch.from_numpy(lab.view(np.int64)), torch.from_numpy(k.view(np.int64)),
                                     torch.from_numpy(v.view(np.int64))).numpy()
        assert np.array_equal(a, b)
        assert a.min() >= -1.0 and a.max() < 1.0
