"""FP64 reference of the learned initial-guess network (oracle).

The network predicts psi_{n+1} element by element (every (instance, channel, component, radial)
entry is one row) from the last four states and the field:

  rho   = sqrt(|psi_n|^2 + |psi_{n-1}|^2 + tau^2)                  (per-row scale)
  u_k   = psi_{n-k} / rho,  k = 0..3                               (complex)
  x     = [Re u_0, Im u_0, ..., Re u_3, Im u_3, f(t_n + dt/2), f(t_n - dt/2), s, 0 ...]  (32 features)
  h1    = silu(W1 x + b1),  h2 = silu(W2 h1 + b2),  y = W3 h2 + b3   (256, 256, 2)
  out   = sum_k c[s][k] u_k + sigma (y_0 + i y_1),   guess = rho * out

c[s][k] is the least-squares four-step predictor of psi_{n+1} / rho per spinor component
(``fit_skip``); sigma is the RMS residual of that fit. Loss: mean over rows of
|out - psi_{n+1}/rho|^2 / sigma^2. Adam (Kingma & Ba 2015) on the network parameters, a dict of
float64 arrays: W1 [H][F], b1 [H], W2 [H][H], b2 [H], W3 [2][H], b3 [2].
"""
from __future__ import annotations

import numpy as np

N_FEAT = 32
N_USED = 11


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def features(hist, f_half, f_mhalf, s_flag, tau):
    """hist: complex [4][M] = psi_n, psi_{n-1}, psi_{n-2}, psi_{n-3}; returns (x [M][32], u [4][M], rho [M])."""
    rho = np.sqrt(np.abs(hist[0]) ** 2 + np.abs(hist[1]) ** 2 + tau * tau)
    u = hist / rho[None, :]
    M = hist.shape[1]
    x = np.zeros((M, N_FEAT))
    for k in range(4):
        x[:, 2 * k] = u[k].real
        x[:, 2 * k + 1] = u[k].imag
    x[:, 8] = f_half
    x[:, 9] = f_mhalf
    x[:, 10] = s_flag
    return x, u, rho


def fit_skip(u, t, s_flag):
    """Least-squares c[s] (complex [2][4]) with t ~ sum_k c[s][k] u_k per component; returns (c, sigma)."""
    s = s_flag.astype(int)
    c = np.zeros((2, 4), dtype=complex)
    res2 = 0.0
    for sv in (0, 1):
        m = s == sv
        X = u[:, m].T
        c[sv], *_ = np.linalg.lstsq(X, t[m], rcond=None)
        res2 += float(np.sum(np.abs(X @ c[sv] - t[m]) ** 2))
    return c, max(np.sqrt(res2 / len(t)), 1e-300)


def forward(p, x, u, s_flag, c, sigma):
    """Prediction out = sum_k c[s][k] u_k + sigma (y_0 + i y_1) for every row."""
    z1 = x @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["W3"].T + p["b3"]
    s = s_flag.astype(int)
    lin = np.sum(c[s].T * u, axis=0)  # [M]
    out = lin + sigma * (y[:, 0] + 1j * y[:, 1])
    cache = dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, u=u, s=s, sigma=sigma)
    return out, cache


def loss_and_grads(p, out, target, cache):
    """L = mean |out - target|^2 / sigma^2; returns (L, grads dict) by the chain rule."""
    M = out.shape[0]
    sig = cache["sigma"]
    e = (out - target) / sig
    L = float(np.mean(np.abs(e) ** 2))
    dout = 2.0 * e / M  # dL/dy_0 + i dL/dy_1 (y enters out as sigma * y)
    g = {}
    dy = np.stack([dout.real, dout.imag], axis=1)
    g["W3"] = dy.T @ cache["h2"]
    g["b3"] = dy.sum(0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * dsilu(cache["z2"])
    g["W2"] = dz2.T @ cache["h1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * dsilu(cache["z1"])
    g["W1"] = dz1.T @ cache["x"]
    g["b1"] = dz1.sum(0)
    return L, g


def adam_update(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), in place on p, m, v."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


PARAM_ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]


def param_shapes(hidden=256, n_feat=N_FEAT):
    return {"W1": (hidden, n_feat), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,), "W3": (2, hidden),
            "b3": (2,)}


def unflatten(flat, hidden=256):
    out, o = {}, 0
    for k in PARAM_ORDER:
        shp = param_shapes(hidden)[k]
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounding = ((bits >> 16) & 1) + 0x7FFF
    bits = ((bits + rounding) >> 16) << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)
