"""CPU reference of the learned initial guess (FP64, numpy).

TEST INFRASTRUCTURE ONLY: the GPU network's forward pass, gradients and
optimiser step are checked against these functions; the product package
never imports this module.

The initial guess of each implicit step is free (the step has exactly one
solution, Sec. 3, unique solvability theorems), so any predictor may supply
it.  The predictor here is a small convolutional network:

  inputs   x0 = in_scale * phi^n,  x1 = (phi^n - phi^{n-1}) / sigma1,
           x2 = (s psi^n - (phi^n - phi^{n-1})) / sigma1,
           sigma1 = rms(phi^n - phi^{n-1}) over the grid (x1 = x2 = 0 if
           sigma1 = 0), s the time step.  psi^n is an input because the step's
           solution depends on it and, for the second-order scheme, it is not
           a function of phi^n and phi^{n-1}: it carries the history of the run
           (eq. discrete_2_b);
  layers   four 3x3 convolutions with periodic (circular) padding,
           3 -> 32 -> 32 -> 32 -> 1 channels, tanh-form GELU after the first
           three (Hendrycks and Gimpel, 2016);
  output   delta; the guess is 2 phi^n - phi^{n-1} + c, c = out_scale * sigma1
           * delta minus its grid mean (so the guess keeps the mass of phi^n,
           which every step conserves, Sec. 3).

Training minimises the mean over all pixels of (delta - t)^2 with the target
t = (phi^{n+1} - 2 phi^n + phi^{n-1}) / (out_scale * sigma1), by Adam
(Kingma and Ba, 2015).

Parameter blob (float32): 8 header values [version 2, cin 3, channels 32,
layers 4, in_scale, out_scale, s, 0], then per layer its weights
W[ky][kx][ci][co] (ky, kx = 0..2 for offsets -1..1 in y and x) and biases b[co].

Grids are (n, m) arrays with x fastest, as everywhere in the oracle.
"""
from __future__ import annotations

import math

import numpy as np

HEADER = 8
CIN = 3
CH = 32
LAYERS = ((CIN, CH), (CH, CH), (CH, CH), (CH, 1))


def layout():
    """(name, shape) of every parameter array in blob order."""
    out = []
    for k, (ci, co) in enumerate(LAYERS):
        out.append((f"W{k + 1}", (3, 3, ci, co)))
        out.append((f"b{k + 1}", (co,)))
    return out


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in layout())


def unpack(blob):
    """Blob -> (params dict of float64 arrays, in_scale, out_scale); the time
    step is blob[6] (see dt_of)."""
    blob = np.asarray(blob, dtype=np.float32)
    if blob.size != HEADER + n_params():
        raise ValueError("blob size does not match the network layout")
    hdr = blob[:HEADER].astype(np.float64)
    if int(hdr[0]) != 2 or int(hdr[1]) != CIN or int(hdr[2]) != CH or int(hdr[3]) != len(LAYERS):
        raise ValueError("blob header does not match the network layout")
    params, off = {}, HEADER
    for name, shape in layout():
        cnt = int(np.prod(shape))
        params[name] = blob[off:off + cnt].astype(np.float64).reshape(shape)
        off += cnt
    return params, float(hdr[4]), float(hdr[5])


def dt_of(blob) -> float:
    return float(np.asarray(blob, dtype=np.float32)[6])


def pack(params, in_scale, out_scale, dt):
    hdr = np.array([2, CIN, CH, len(LAYERS), in_scale, out_scale, dt, 0], dtype=np.float32)
    parts = [hdr] + [np.asarray(params[name], dtype=np.float32).reshape(-1)
                     for name, _ in layout()]
    return np.concatenate(parts)


def init_blob(seed: int, in_scale: float = 2.0, out_scale: float = 1.0, dt: float = 0.05,
              zero_last: bool = True):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the last layer
    zero (the untrained network then reproduces the extrapolated guess)."""
    rng = np.random.default_rng(seed)
    params = {}
    for k, (ci, co) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (9 * ci))
        W = rng.standard_normal((3, 3, ci, co)) * std
        if zero_last and k == len(LAYERS) - 1:
            W[:] = 0.0
        params[f"W{k + 1}"] = W
        params[f"b{k + 1}"] = np.zeros(co)
    return pack(params, in_scale, out_scale, dt)


# ---- building blocks ---------------------------------------------------------------
_GC = math.sqrt(2.0 / math.pi)


def gelu(x):
    """tanh form of GELU: x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + np.tanh(_GC * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = _GC * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _GC * (1.0 + 3.0 * 0.044715 * x * x)


def shifted(x, ky, kx):
    """s[y, x] = x[(y + ky - 1) mod n, (x + kx - 1) mod m] (periodic neighbour)."""
    return np.roll(x, shift=(1 - ky, 1 - kx), axis=(0, 1))


def conv(x, W, b):
    """Periodic 3x3 convolution (cross-correlation): x (n, m, ci) -> (n, m, co)."""
    out = np.broadcast_to(b, x.shape[:2] + (W.shape[3],)).copy()
    for ky in range(3):
        for kx in range(3):
            out += shifted(x, ky, kx) @ W[ky, kx]
    return out


def conv_backward(x, W, gout):
    """Gradients of sum(gout * conv(x, W, b)) with respect to x, W and b."""
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    ci, co = W.shape[2], W.shape[3]
    g2 = gout.reshape(-1, co)
    for ky in range(3):
        for kx in range(3):
            dW[ky, kx] = shifted(x, ky, kx).reshape(-1, ci).T @ g2
            # x[p + off] received W[off] gout[p]: shift back by -off
            dx += np.roll(gout @ W[ky, kx].T, shift=(ky - 1, kx - 1), axis=(0, 1))
    db = g2.sum(axis=0)
    return dx, dW, db


# ---- the network -------------------------------------------------------------------
def inputs(phi_nm1, phi_n, psi_n, dt, in_scale):
    """Input channels and sigma1 = rms(phi^n - phi^{n-1})."""
    d1 = phi_n - phi_nm1
    sigma1 = math.sqrt(float(np.mean(d1 * d1)))
    if sigma1 > 0:
        x1 = d1 / sigma1
        x2 = (dt * psi_n - d1) / sigma1
    else:
        x1 = np.zeros_like(d1)
        x2 = np.zeros_like(d1)
    return np.stack([in_scale * phi_n, x1, x2], axis=-1), sigma1


def forward(params, x):
    """delta and the intermediate pre-activations (for the backward pass)."""
    cache = {"a0": x}
    a = x
    for k in range(1, len(LAYERS)):
        z = conv(a, params[f"W{k}"], params[f"b{k}"])
        cache[f"z{k}"] = z
        a = gelu(z)
        cache[f"a{k}"] = a
    L = len(LAYERS)
    delta = conv(a, params[f"W{L}"], params[f"b{L}"])[..., 0]
    return delta, cache


def guess(blob, phi_nm1, phi_n, psi_n):
    """The learned initial guess phi^(0) (mean-corrected)."""
    params, in_scale, out_scale = unpack(blob)
    x, sigma1 = inputs(phi_nm1, phi_n, psi_n, dt_of(blob), in_scale)
    delta, _ = forward(params, x)
    c = out_scale * sigma1 * delta
    c = c - np.mean(c)
    return 2.0 * phi_n - phi_nm1 + c


def delta(blob, phi_nm1, phi_n, psi_n):
    params, in_scale, _ = unpack(blob)
    x, _ = inputs(phi_nm1, phi_n, psi_n, dt_of(blob), in_scale)
    return forward(params, x)[0]


def target(phi_nm1, phi_n, phi_np1, out_scale):
    d1 = phi_n - phi_nm1
    sigma1 = math.sqrt(float(np.mean(d1 * d1)))
    so = out_scale * sigma1
    d2 = phi_np1 - 2.0 * phi_n + phi_nm1
    return d2 / so if so > 0 else np.zeros_like(d2)


def loss_and_grad(blob, samples):
    """Mean squared error over every pixel of every sample (phi^{n-1},
    phi^n, psi^n, phi^{n+1}) and its gradient with respect to every
    parameter, in blob order (without the header)."""
    params, in_scale, out_scale = unpack(blob)
    dt = dt_of(blob)
    npix = sum(s[1].size for s in samples)
    grads = {name: np.zeros(shape) for name, shape in layout()}
    loss = 0.0
    L = len(LAYERS)
    for phi_nm1, phi_n, psi_n, phi_np1 in samples:
        x, _ = inputs(phi_nm1, phi_n, psi_n, dt, in_scale)
        d, cache = forward(params, x)
        t = target(phi_nm1, phi_n, phi_np1, out_scale)
        err = d - t
        loss += float(np.sum(err * err))
        g = (2.0 / npix) * err[..., None]
        ga, dW, db = conv_backward(cache[f"a{L - 1}"], params[f"W{L}"], g)
        grads[f"W{L}"] += dW
        grads[f"b{L}"] += db
        for k in range(L - 1, 0, -1):
            gz = ga * gelu_grad(cache[f"z{k}"])
            ga, dW, db = conv_backward(cache[f"a{k - 1}"], params[f"W{k}"], gz)
            grads[f"W{k}"] += dW
            grads[f"b{k}"] += db
    flat = np.concatenate([grads[name].reshape(-1) for name, _ in layout()])
    return loss / npix, flat


def adam(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1, 2, ...): returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def with_params(blob, flat):
    """Blob with the parameters replaced by `flat` (header kept)."""
    out = np.asarray(blob, dtype=np.float32).copy()
    out[HEADER:] = np.asarray(flat, dtype=np.float32)
    return out
