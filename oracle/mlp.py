"""FP64 oracle of the per-mode coarse-correction MLP (test infrastructure).

Learned correction of G (an addition to the paper's method): for slice n and
spectral mode k the coarse step becomes
    G~(v) = E_G v + r_n + delta_n,  delta_{n,k} = dT * s * NN(x).
The inputs come from z = D lambda_k dT and the eight forcing samples
g_s = ghat_k(T_n + s dT / 7), s = 0..7.  The samples are expanded in the
discrete orthonormal polynomials q_0..q_7 of the points t_s = (s - 3.5)/3.5
(Gram-Schmidt of 1, t, .., t^7, positive leading coefficients):
c_j = q_j . g.  Both propagators integrate forcing that is a cubic in time
exactly (the exponential Runge-Kutta weights reproduce polynomials up to
degree p - 1 = 3), so the correction depends on the part of degree >= 4; its
size s = ||(c_4..c_7)|| scales the output, and the inputs are
    x = [ln(z)/8, e^{-z}, phi_1(-z), 2 phi_2(-z),
         c_0/|g|, .., c_3/|g|,  c_4/s, .., c_7/s]
(|g| the Euclidean norm of the samples; zero parts give zero features).
The training target of a row is (R_n - r_n)_k / (dT s) with R_n = F^J(0) and
r_n = G(0) on slice n: the state-independent fine and coarse forcing
responses (eq. 4.5 and the Lipschitz identity in the proof of Theorem 4.3 make
both responses independent of the state).

Network: 12 inputs -> 64 -> 64 -> 64 (GELU, x Phi(x)) -> 1 (linear).
Parameters (flat float vector, this order): W1[12][64], b1[64], W2[64][64],
b2[64], W3[64][64], b3[64], w4[64], b4[1]  (W[in][out], y = x W + b).

Pinned in the tests by central differences of the loss (the backward pass
below is written out by hand, not derived automatically).
"""
from __future__ import annotations

import math

import numpy as np

N_IN = 12
WIDTH = 64
SAMPLES = 8

SHAPES = [("W1", (N_IN, WIDTH)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("w4", (WIDTH,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    """x * Phi(x), Phi the standard normal distribution (erfc form: no
    cancellation for negative x)."""
    from scipy.special import erfc
    return 0.5 * x * erfc(-x / _SQRT2)


def gelu_grad(x):
    from scipy.special import erfc
    return 0.5 * erfc(-x / _SQRT2) + x * _INV_SQRT_2PI * np.exp(-0.5 * x * x)


def z_features(z: np.ndarray) -> np.ndarray:
    """[ln z / 8, e^{-z}, phi_1(-z), 2 phi_2(-z)] for z > 0 (FP64; the small-z
    branches use series to avoid cancellation)."""
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(-z)
    small = z < 1e-3
    zs = np.where(small, 1.0, z)
    phi1 = np.where(small, 1 - z / 2 + z * z / 6 - z ** 3 / 24, -np.expm1(-zs) / zs)
    phi2 = np.where(small, 0.5 - z / 6 + z * z / 24 - z ** 3 / 120, (zs - 1 + np.exp(-zs)) / (zs * zs))
    return np.stack([np.log(z) / 8.0, e, phi1, 2.0 * phi2], axis=-1)


def sample_basis() -> np.ndarray:
    """Q[s][j] = q_j(t_s): orthonormal columns from Gram-Schmidt of the
    monomials in t_s = (s - 3.5)/3.5 (numpy QR, signs fixed so that every
    diagonal entry of R is positive)."""
    t = (np.arange(SAMPLES) - 3.5) / 3.5
    V = np.vander(t, SAMPLES, increasing=True)
    Q, R = np.linalg.qr(V)
    return Q * np.sign(np.diag(R))[None, :]


def features(z: np.ndarray, samples: np.ndarray):
    """Rows of network inputs from z[rows] and samples[rows, 8]; returns
    (x[rows, 12], s[rows]) with s the norm of the degree 4..7 coefficients."""
    samples = np.asarray(samples, dtype=np.float64)
    c = samples @ sample_basis()
    gn = np.linalg.norm(samples, axis=-1)
    hi = np.linalg.norm(c[:, 4:], axis=-1)
    gsafe = np.where(gn > 0, gn, 1.0)
    hsafe = np.where(hi > 0, hi, 1.0)
    x = np.concatenate([z_features(z), c[:, :4] / gsafe[:, None], c[:, 4:] / hsafe[:, None]],
                       axis=-1)
    return x, hi


def forward(theta: np.ndarray, x: np.ndarray, keep: bool = False):
    p = unpack(theta)
    z1 = x @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    z3 = h2 @ p["W3"] + p["b3"]
    h3 = gelu(z3)
    y = h3 @ p["w4"] + p["b4"][0]
    if keep:
        return y, (x, z1, h1, z2, h2, z3, h3)
    return y


def loss(theta, x, target):
    y = forward(theta, x)
    return float(np.mean((y - target) ** 2))


def loss_and_grad(theta, x, target):
    """Mean squared error and its gradient, by hand-written backpropagation."""
    p = unpack(theta)
    y, (x, z1, h1, z2, h2, z3, h3) = forward(theta, x, keep=True)
    B = x.shape[0]
    r = y - target
    L = float(np.mean(r * r))
    dy = 2.0 * r / B                              # dL/dy
    g = {}
    g["w4"] = h3.T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, p["w4"]) * gelu_grad(z3)
    g["W3"] = h2.T @ dz3
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ p["W3"].T) * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(z1)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def init_params(seed: int) -> np.ndarray:
    """Scaled-normal initialisation (used by CPU-side checks only)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("b"):
            parts.append(np.zeros(shape))
        else:
            fan_in = shape[0]
            parts.append(rng.normal(size=shape) / math.sqrt(fan_in))
    return np.concatenate([q.ravel() for q in parts])


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def correction(theta, z, samples, dT):
    """delta = dT * s * NN(x) per row (zero where the samples have no part of
    degree >= 4)."""
    x, s = features(z, samples)
    y = forward(theta, x)
    return np.where(s > 0, s * dT * y, 0.0)
