"""FP64 oracle of the column-physics surrogate (test infrastructure only).

The paper has no learned component; the surrogate replaces the column
physics (section "Architecture-Dependant Parallelization Granularity" treats
that physics as one column-local operator), so its inputs are exactly what the
plain physics reads and its outputs are the physics tendencies.  Readings:

* Features (294 per column): five profiles of 58 values (k = 0 first) built
  from the post-dycore theta' = theta - 300 K, q and the cell-centred winds
  (u, v) of the column, then theta_s - 300 K, q_s, F0, C_h:
    1. theta'_0, then the differences theta'_k - theta'_{k-1};
    2. q_0, then q_k - q_{k-1};
    3. the wind speed |(u, v)_0|, then the shear S_k = |(u, v)_k - (u, v)_{k-1}|;
    4. 0, then S_k (theta'_k - theta'_{k-1});
    5. 0, then S_k (q_k - q_{k-1}).
  The implicit diffusion acts on the vertical differences with a coefficient
  set by the shear (the mixing length closure), and the radiation on q, so
  these are the quantities the column operator depends on; differences keep
  their full relative precision when rounded to BF16, where nearly equal
  neighbouring levels would not.  Each feature is z-scored with the FP64
  training-set mean and standard deviation (a deviation below 1e-12 is
  replaced by 1).
* Targets (116): the 58 theta tendencies then the 58 q tendencies of the plain
  physics, centred per output and scaled by the pooled standard deviation of
  their variable (sigma_theta or sigma_q), so that the training loss weighs
  every level as the judge's pooled RMSE does.
* Network: h1 = ReLU(W1 x + b1) (294 -> 512), h2 = ReLU(W2 h1 + b2)
  (512 -> 512), y = W3 h2 + b3 (512 -> 116).  GEMM operands are rounded to
  BF16 (round to nearest, ties to even): x, h1, h2, the weights and the
  upstream gradients; accumulation, bias, ReLU, loss and bias gradients stay
  in higher precision.  ReLU'(0) = 0; the ReLU mask is (BF16 activation > 0).
* Loss: mean of (y - t)^2 over the batch and the 116 outputs.
* Adam: beta = (0.9, 0.999), eps = 1e-8, bias-corrected, no weight decay.
* Init: He-uniform +-sqrt(6 / fan_in) drawn with SplitMix64, zero biases.
* Judge: column c is sampled at step t when SplitMix64(seed ^ (t << 32) ^ c)
  mod 100 == 0; per variable the RMSE pooled over the sampled columns and all
  levels is compared with 0.05 times the training-set standard deviation of
  that tendency; strictly greater means the whole step falls back.  Also
  reported: the fraction of sampled columns whose own RMSE over the levels
  of a variable exceeds the same bound.

Arrays are float64 unless stated.  Weight matrices are (fan_out, fan_in).
"""
from __future__ import annotations

from typing import Dict, NamedTuple

import numpy as np

NZ = 58
N_IN = 5 * NZ + 4          # 294
N_HID = 512
N_OUT = 2 * NZ             # 116

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x) -> np.ndarray:
    """SplitMix64 output for state increments x (Steele, Lea & Flood 2014).

    z = x + 0x9E3779B97F4A7C15; z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB; return z ^ (z >> 31), all mod 2^64.
    """
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def bf16(x) -> np.ndarray:
    """Round to BF16 (8 significant bits, nearest, ties to even) via FP32."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


# --------------------------------------------------------------------------
# features, targets, normalisation
# --------------------------------------------------------------------------
THETA_REF = 300.0


def features(rho, theta, q, u, v, theta_s, q_s, f0, ch, dtype=np.float64) -> np.ndarray:
    """(ncol, 5 nz + 4) inputs, column c = i + nx j.

    ``dtype`` is the arithmetic precision of the differences, speeds and
    products (theta - 300 K is formed in float64 first); rho is not an input."""
    del rho
    nz, ny, nx = theta.shape
    ub = ((np.roll(u, 1, axis=2).astype(dtype) + u.astype(dtype)) * dtype(0.5)).reshape(nz, -1).T
    vb = ((np.roll(v, 1, axis=1).astype(dtype) + v.astype(dtype)) * dtype(0.5)).reshape(nz, -1).T
    th = (theta - THETA_REF).astype(dtype).reshape(nz, -1).T
    qq = q.astype(dtype).reshape(nz, -1).T
    dth = th[:, 1:] - th[:, :-1]
    dq = qq[:, 1:] - qq[:, :-1]
    du = ub[:, 1:] - ub[:, :-1]
    dv = vb[:, 1:] - vb[:, :-1]
    shear = np.sqrt(du * du + dv * dv)
    speed0 = np.sqrt(ub[:, :1] * ub[:, :1] + vb[:, :1] * vb[:, :1])
    zero = np.zeros_like(speed0)
    prof = [np.concatenate([th[:, :1], dth], 1), np.concatenate([qq[:, :1], dq], 1),
            np.concatenate([speed0, shear], 1), np.concatenate([zero, shear * dth], 1),
            np.concatenate([zero, shear * dq], 1)]
    surf = [np.asarray(a, dtype=np.float64).reshape(ny * nx, 1).astype(dtype)
            for a in (theta_s - THETA_REF, q_s, f0, ch)]
    return np.concatenate(prof + surf, axis=1).astype(np.float64)


def targets(t_theta, t_q) -> np.ndarray:
    """(ncol, 2 nz) tendencies, theta first."""
    nz, ny, nx = t_theta.shape
    return np.concatenate([t_theta.reshape(nz, ny * nx).T, t_q.reshape(nz, ny * nx).T], axis=1)


class Norm(NamedTuple):
    x_mean: np.ndarray
    x_std: np.ndarray
    y_mean: np.ndarray
    y_std: np.ndarray
    sigma_theta: float      # pooled std of the theta tendencies
    sigma_q: float          # pooled std of the q tendencies


def norm_stats(x: np.ndarray, y: np.ndarray) -> Norm:
    """Feature mean / std per column; target mean per output and the pooled std
    of its variable (outputs 0..nz-1 theta, nz..2nz-1 q)."""
    xs = x.std(axis=0)
    nz = y.shape[1] // 2
    s_t, s_q = float(y[:, :nz].std()), float(y[:, nz:].std())
    ys = np.concatenate([np.full(nz, s_t if s_t >= 1e-12 else 1.0), np.full(nz, s_q if s_q >= 1e-12 else 1.0)])
    return Norm(x.mean(axis=0), np.where(xs < 1e-12, 1.0, xs), y.mean(axis=0), ys, s_t, s_q)


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------
def he_uniform(seed: int, tensor_id: int, fan_out: int, fan_in: int) -> np.ndarray:
    """He-uniform weights: element e = row * fan_in + col draws
    u = (SplitMix64((seed << 32) | (tensor_id << 28) | e) >> 40) * 2^-24 and
    w = fp32(fp32(2u - 1) * fp32(sqrt(6 / fan_in)))."""
    e = np.arange(fan_out * fan_in, dtype=np.uint64)
    key = (np.uint64(seed) << np.uint64(32)) | (np.uint64(tensor_id) << np.uint64(28)) | e
    u = (splitmix64(key) >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
    bound = np.float32(np.sqrt(6.0 / fan_in))
    w = (np.float32(2.0) * u - np.float32(1.0)) * bound
    return w.astype(np.float64).reshape(fan_out, fan_in)


def init_params(seed: int, n_in=N_IN, n_hid=N_HID, n_out=N_OUT) -> Dict[str, np.ndarray]:
    return {"W1": he_uniform(seed, 0, n_hid, n_in), "b1": np.zeros(n_hid),
            "W2": he_uniform(seed, 2, n_hid, n_hid), "b2": np.zeros(n_hid),
            "W3": he_uniform(seed, 4, n_out, n_hid), "b3": np.zeros(n_out)}


def _r(a, on):
    return bf16(a) if on else a


def forward(p: Dict[str, np.ndarray], x: np.ndarray, bf: bool = True):
    """Returns (y, cache).  ``bf`` rounds the GEMM operands to BF16."""
    xb = _r(x, bf)
    w1, w2, w3 = (_r(p[k], bf) for k in ("W1", "W2", "W3"))
    h1 = _r(np.maximum(xb @ w1.T + p["b1"], 0.0), bf)
    h2 = _r(np.maximum(h1 @ w2.T + p["b2"], 0.0), bf)
    y = h2 @ w3.T + p["b3"]
    return y, {"x": xb, "h1": h1, "h2": h2, "w1": w1, "w2": w2, "w3": w3}


def loss(y: np.ndarray, t: np.ndarray) -> float:
    return float(np.mean((y - t) ** 2))


def backward(cache, y: np.ndarray, t: np.ndarray, bf: bool = True) -> Dict[str, np.ndarray]:
    """Gradients of the mean squared error."""
    g3 = 2.0 * (y - t) / y.size
    g3b = _r(g3, bf)
    grads = {"W3": g3b.T @ cache["h2"], "b3": g3.sum(axis=0)}
    g2 = (g3b @ cache["w3"]) * (cache["h2"] > 0)
    g2b = _r(g2, bf)
    grads["W2"] = g2b.T @ cache["h1"]
    grads["b2"] = g2.sum(axis=0)
    g1 = (g2b @ cache["w2"]) * (cache["h1"] > 0)
    g1b = _r(g1, bf)
    grads["W1"] = g1b.T @ cache["x"]
    grads["b1"] = g1.sum(axis=0)
    return grads


class AdamState(NamedTuple):
    m: Dict[str, np.ndarray]
    v: Dict[str, np.ndarray]
    t: int


def adam_init(p) -> AdamState:
    return AdamState({k: np.zeros_like(a) for k, a in p.items()},
                     {k: np.zeros_like(a) for k, a in p.items()}, 0)


def adam_step(p, g, st: AdamState, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    t = st.t + 1
    newp, m, v = {}, {}, {}
    for k in p:
        m[k] = b1 * st.m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * st.v[k] + (1.0 - b2) * g[k] ** 2
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        newp[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return newp, AdamState(m, v, t)


# --------------------------------------------------------------------------
# judge
# --------------------------------------------------------------------------
def sample_mask(seed: int, t: int, ncol: int) -> np.ndarray:
    c = np.arange(ncol, dtype=np.uint64)
    key = np.uint64(seed) ^ (np.uint64(t) << np.uint64(32)) ^ c
    return (splitmix64(key) % np.uint64(100)) == np.uint64(0)


def judge(t_hat: np.ndarray, t_ref: np.ndarray, mask: np.ndarray, sigma_theta: float,
          sigma_q: float, rel: float = 0.05):
    """Pooled RMSE per variable over the sampled columns; True means fall back."""
    nz = t_hat.shape[1] // 2
    d = (t_hat - t_ref)[mask]
    r_theta = float(np.sqrt(np.mean(d[:, :nz] ** 2)))
    r_q = float(np.sqrt(np.mean(d[:, nz:] ** 2)))
    return r_theta, r_q, (r_theta > rel * sigma_theta) or (r_q > rel * sigma_q)


def judge_columns(t_hat: np.ndarray, t_ref: np.ndarray, mask: np.ndarray, sigma_theta: float,
                  sigma_q: float, rel: float = 0.05):
    """Fractions of the sampled columns whose own RMSE over the levels of one
    variable exceeds rel * sigma of that variable (theta, q)."""
    nz = t_hat.shape[1] // 2
    d = (t_hat - t_ref)[mask]
    if d.shape[0] == 0:
        return 0.0, 0.0
    r_theta = np.sqrt(np.mean(d[:, :nz] ** 2, axis=1))
    r_q = np.sqrt(np.mean(d[:, nz:] ** 2, axis=1))
    return float(np.mean(r_theta > rel * sigma_theta)), float(np.mean(r_q > rel * sigma_q))

