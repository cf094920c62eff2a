"""Seeded random weights for the parameter-inference CNN.

Architecture (shapes only; no arithmetic here): four 3x3 convolutions
1->32->32->64->64 on a 1x16x64 dynamic spectrum, a dense layer
65536->128 and a dense head 128->14 (4 means + 10 packed Cholesky entries).
Weights are He-normal (std sqrt(2/fan_in)), biases U(-0.05, 0.05), all
float32, drawn from a Philox generator keyed by the seed.
"""

from __future__ import annotations

import numpy as np

CONV_CH = (1, 32, 32, 64, 64)
GRID_H, GRID_W = 16, 64
HIDDEN = 128
N_OUT = 14

LAYER_ORDER = ("conv1.w", "conv1.b", "conv2.w", "conv2.b", "conv3.w", "conv3.b",
               "conv4.w", "conv4.b", "fc1.w", "fc1.b", "fc2.w", "fc2.b")


def layer_shapes():
    shapes = {}
    for l in range(4):
        cin, cout = CONV_CH[l], CONV_CH[l + 1]
        shapes[f"conv{l+1}.w"] = (cout, cin, 3, 3)
        shapes[f"conv{l+1}.b"] = (cout,)
    flat = CONV_CH[-1] * GRID_H * GRID_W
    shapes["fc1.w"] = (HIDDEN, flat)
    shapes["fc1.b"] = (HIDDEN,)
    shapes["fc2.w"] = (N_OUT, HIDDEN)
    shapes["fc2.b"] = (N_OUT,)
    return shapes


def cnn_weights(seed: int = 2103_15418, leaky_alpha: float = 0.0) -> dict:
    """dict name -> float32 array (PyTorch layouts: conv [out][in][kh][kw],
    dense [out][in]); key "alpha" holds the activation's negative slope."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 4_000_004])))
    out = {}
    for name, shp in layer_shapes().items():
        if name.endswith(".w"):
            fan_in = int(np.prod(shp[1:]))
            out[name] = (g.standard_normal(shp) * np.sqrt(2.0 / fan_in)).astype(np.float32)
        else:
            out[name] = g.uniform(-0.05, 0.05, shp).astype(np.float32)
    out["alpha"] = float(leaky_alpha)
    return out
