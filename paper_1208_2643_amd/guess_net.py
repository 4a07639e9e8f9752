"""Parameter blobs of the learned initial guess (layout, seeded initial
weights, files).

The blob is the float32 vector documented with mpfc_cnn_load in
include/mpfc.h: 8 header values [2, 3, 32, 4, in_scale, out_scale, dt, 0],
then W1 (3,3,3,32), b1 (32), W2 (3,3,32,32), b2, W3 (3,3,32,32), b3,
W4 (3,3,32,1), b4 (1), weights ordered [ky][kx][ci][co].  The arithmetic of
the network runs in the library's kernels only.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

LAYERS = ((3, 32), (32, 32), (32, 32), (32, 1))
HEADER = 8
N_PARAMS = sum(9 * ci * co + co for ci, co in LAYERS)
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "guess_cnn_scheme2.f32")


def initial_blob(seed: int, dt: float, in_scale: float = 2.0, out_scale: float = 1.0) -> np.ndarray:
    """He-normal hidden weights (std sqrt(2 / fan_in)) from a seeded generator,
    zero biases and a zero output layer: the untrained network's guess is the
    extrapolated one."""
    rng = np.random.default_rng(seed)
    parts = [np.array([2, 3, 32, 4, in_scale, out_scale, dt, 0], dtype=np.float32)]
    for k, (ci, co) in enumerate(LAYERS):
        if k == len(LAYERS) - 1:
            w = np.zeros(9 * ci * co)
        else:
            w = rng.standard_normal(9 * ci * co) * math.sqrt(2.0 / (9 * ci))
        parts += [w.astype(np.float32), np.zeros(co, dtype=np.float32)]
    blob = np.concatenate(parts)
    assert blob.size == HEADER + N_PARAMS
    return blob


def with_out_scale(blob: np.ndarray, out_scale: float) -> np.ndarray:
    b = np.array(blob, dtype=np.float32)
    b[5] = out_scale
    return b


def save(blob: np.ndarray, path: str = DEFAULT_WEIGHTS, meta: dict | None = None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.asarray(blob, dtype="<f4").tofile(path)
    if meta is not None:
        with open(path + ".json", "w") as f:
            json.dump(meta, f, indent=1, sort_keys=True)


def load(path: str = DEFAULT_WEIGHTS) -> np.ndarray:
    blob = np.fromfile(path, dtype="<f4")
    if blob.size != HEADER + N_PARAMS:
        raise ValueError(f"{path}: {blob.size} values, expected {HEADER + N_PARAMS}")
    return blob


def meta(path: str = DEFAULT_WEIGHTS) -> dict:
    with open(path + ".json") as f:
        return json.load(f)
