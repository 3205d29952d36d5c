"""Learned correction stage: conv net, training step, residual pairs, FGMRES stage.

Test infrastructure (float64 numpy): only the test suite, the smoke check and
the benchmark's CPU-baseline leg may use it.

The paper describes no learned component; everything here follows the
readings stated below, written from their definitions.

Network (reading): three 3x3 convolutions on the periodic grid,
    y1 = W1 * x, a1 = relu(y1); y2 = W2 * a1, a2 = relu(y2); y3 = W3 * a2,
channels 3 -> 32 -> 32 -> 3, no biases (so the map is positively homogeneous),
periodic padding. The three input/output channels are the u, v and p blocks of
a grid vector, each an N x N array [i][j], so u_ij, v_ij and p_ij share a pixel.
A convolution here is the cross-correlation
    out[co, i, j] = sum_{ci, a, c} W[co, ci, a, c] x[ci, i + a - 1, j + c - 1]
with indices mod N. The flat parameter vector holds W1 (32,3,3,3), W2
(32,32,3,3) and W3 (3,32,3,3) in that order, each C-ordered: 10 944 numbers.

Reduced precision (reading): with `bf16=True` the weights, the network input and
the two hidden activations are rounded to bfloat16 (first to float32, then to
bfloat16, round-to-nearest-even each time) before they enter a convolution;
sums are exact here (float64). The float32 accumulation of the device kernels
differs from this only by the order and precision of the sums.

Training (reading): pairs (r_hat, e_hat) = (r, e) / ||r||; error loss
    L = (1/B) sum_b ||N(r_hat_b) - e_hat_b||^2 / ||e_hat_b||^2,
or residual loss L = (1/B) sum_b ||K N(r_hat_b) - r_hat_b||^2 / ||r_hat_b||^2
(the same error measured through K, since K e_hat = r_hat), or its
scale-invariant form, the residual left by the best multiple of N(r_hat_b)
(minimal-residual loss); gradients by the
chain rule through the stored activations (the bf16 weight rounding is passed
straight through to the float32 master weights), Adam.

Pairs (reading): x* with random entries, b = K x*, x_0 = 0,
x_k = x_{k-1} + V(b - K x_{k-1}); the pair after iteration k is
(r_k, e_k) = (b - K x_k, x* - x_k), so K e_k = r_k.

FGMRES stage (reading): after z0 = V(v), r' = v - K z0, c = ||r'|| N(r'/||r'||)
with its pressure mean removed, gamma = <r', K c> / ||K c||^2 (the minimiser
of ||r' - gamma K c||), and z = z0 + gamma c is accepted only if
||r' - gamma K c||^2 <= (1 - margin) ||r'||^2, i.e. (at that gamma)
<r', K c>^2 / ||K c||^2 >= margin ||r'||^2; otherwise z = z0.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Tuple

import numpy as np

CH = 32
SHAPES = ((CH, 3, 3, 3), (CH, CH, 3, 3), (3, CH, 3, 3))
N_WEIGHTS = sum(int(np.prod(s)) for s in SHAPES)  # 10 944


def split_weights(w: np.ndarray) -> List[np.ndarray]:
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(w[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def round_fp32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """float64 -> float32 -> bfloat16 (8 significant bits), round to nearest,
    ties to even, returned as float64. bfloat16 is the upper half of the
    float32 bit pattern; rounding adds 0x7FFF plus the lowest kept bit."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    keep = (bits >> 16) & 1
    bits = ((bits + 0x7FFF + keep) >> 16) << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def conv(x: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Periodic 3x3 cross-correlation. x: (B, Cin, N, N), W: (Cout, Cin, 3, 3)."""
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for a in range(3):
        for c in range(3):
            # shifted[..., i, j] = x[..., i + a - 1, j + c - 1]
            shifted = np.roll(x, shift=(1 - a, 1 - c), axis=(2, 3))
            out += np.einsum("oc,bcij->boij", W[:, :, a, c], shifted)
    return out


def conv_transpose(dy: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of `conv` in x: dx[b, ci, p] = sum_{co,a,c} W[co,ci,a,c] dy[b, co, p - (a-1, c-1)]."""
    out = np.zeros((dy.shape[0], W.shape[1]) + dy.shape[2:])
    for a in range(3):
        for c in range(3):
            contrib = np.einsum("oc,boij->bcij", W[:, :, a, c], dy)
            out += np.roll(contrib, shift=(a - 1, c - 1), axis=(2, 3))
    return out


def conv_weight_grad(dy: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dW[co, ci, a, c] = sum_{b,i,j} dy[b, co, i, j] x[b, ci, i + a - 1, j + c - 1]."""
    dW = np.zeros((dy.shape[1], x.shape[1], 3, 3))
    for a in range(3):
        for c in range(3):
            shifted = np.roll(x, shift=(1 - a, 1 - c), axis=(2, 3))
            dW[:, :, a, c] = np.einsum("boij,bcij->oc", dy, shifted)
    return dW


@dataclasses.dataclass
class Cache:
    x: np.ndarray
    Ws: List[np.ndarray]
    a1: np.ndarray
    a2: np.ndarray
    y3: np.ndarray


def forward(x: np.ndarray, w: np.ndarray, bf16: bool = False) -> Tuple[np.ndarray, Cache]:
    """x: (B, 3, N, N). Returns y3 (B, 3, N, N) and the activations for backward."""
    r = round_bf16 if bf16 else (lambda t: t)
    Ws = [r(W) for W in split_weights(w)]
    xin = r(x)
    a1 = r(np.maximum(conv(xin, Ws[0]), 0.0))
    a2 = r(np.maximum(conv(a1, Ws[1]), 0.0))
    y3 = conv(a2, Ws[2])
    if bf16:
        y3 = round_fp32(y3)
    return y3, Cache(xin, Ws, a1, a2, y3)


def loss_and_grad(x: np.ndarray, e: np.ndarray, w: np.ndarray, bf16: bool = False):
    """Loss (1/B) sum_b ||y3_b - e_b||^2 / ||e_b||^2 and its gradient (flat, 10 944)."""
    y3, cc = forward(x, w, bf16)
    B = x.shape[0]
    d = y3 - e
    ne2 = np.einsum("bcij,bcij->b", e, e)
    loss = float(np.mean(np.einsum("bcij,bcij->b", d, d) / ne2))
    g3 = (2.0 / B) * d / ne2[:, None, None, None]
    return loss, backward(cc, g3)


def residual_loss_and_grad(x: np.ndarray, K, w: np.ndarray, bf16: bool = False):
    """Residual-norm loss (reading): with c_b = N(r_b) as a grid vector,
        L = (1/B) sum_b ||K c_b - r_b||^2 / ||r_b||^2,
    i.e. the error c_b - e_b measured in the norm ||K .|| (K e_b = r_b), which is
    what the stage's minimal-residual step sees. Gradient through K^T."""
    y3, cc = forward(x, w, bf16)
    B = x.shape[0]
    loss = 0.0
    g3 = np.zeros_like(y3)
    for b in range(B):
        r = x[b].ravel()
        res = K @ y3[b].ravel() - r
        nr2 = float(r @ r)
        loss += float(res @ res) / nr2
        g3[b] = ((2.0 / B) * (K.T @ res) / nr2).reshape(y3.shape[1:])
    return loss / B, backward(cc, g3)


def minres_loss_and_grad(x: np.ndarray, K, w: np.ndarray, bf16: bool = False):
    """Minimal-residual loss (reading): with c_b = N(r_b), a = <K c_b, r_b>,
    b = ||K c_b||^2, n = ||r_b||^2,
        L = (1/B) sum_b (1 - a^2 / (b n)) = (1/B) sum_b min_g ||r_b - g K c_b||^2 / n,
    the residual the stage's minimal-residual step leaves, scale-invariant in c.
    dL/dc_b = -(2/B) (a / (n b)) K^T (r_b - (a/b) K c_b)."""
    y3, cc = forward(x, w, bf16)
    B = x.shape[0]
    loss = 0.0
    g3 = np.zeros_like(y3)
    for k in range(B):
        r = x[k].ravel()
        kc = K @ y3[k].ravel()
        a, b, n = float(kc @ r), float(kc @ kc), float(r @ r)
        loss += 1.0 - a * a / (b * n)
        g3[k] = (-(2.0 / B) * (a / (n * b)) * (K.T @ (r - (a / b) * kc))).reshape(y3.shape[1:])
    return loss / B, backward(cc, g3)


def backward(cc: Cache, g3: np.ndarray) -> np.ndarray:
    """Flat gradient (10 944) of a loss whose derivative in y3 is g3."""
    dW3 = conv_weight_grad(g3, cc.a2)
    g2 = conv_transpose(g3, cc.Ws[2]) * (cc.a2 > 0)
    dW2 = conv_weight_grad(g2, cc.a1)
    g1 = conv_transpose(g2, cc.Ws[1]) * (cc.a1 > 0)
    dW1 = conv_weight_grad(g1, cc.x)
    return np.concatenate([dW1.ravel(), dW2.ravel(), dW3.ravel()])


@dataclasses.dataclass
class Adam:
    """Adam with bias correction (Kingma & Ba): m, v moments, step counter t."""
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def init(self, n: int):
        return np.zeros(n), np.zeros(n), 0

    def step(self, w: np.ndarray, g: np.ndarray, state):
        m, v, t = state
        t += 1
        m = self.beta1 * m + (1 - self.beta1) * g
        v = self.beta2 * v + (1 - self.beta2) * g * g
        mhat = m / (1 - self.beta1 ** t)
        vhat = v / (1 - self.beta2 ** t)
        return w - self.lr * mhat / (np.sqrt(vhat) + self.eps), (m, v, t)


def to_image(vec: np.ndarray, N: int) -> np.ndarray:
    """Grid vector [u | v | p] -> (3, N, N)."""
    return np.asarray(vec).reshape(3, N, N)


def residual_pairs(K, vcycle: Callable[[np.ndarray], np.ndarray], xstar: np.ndarray, iters: int):
    """(r_hat_k, e_hat_k) for k = 1..iters of x_k = x_{k-1} + V(b - K x_{k-1}), b = K x*."""
    b = K @ xstar
    x = np.zeros_like(xstar)
    out = []
    for _ in range(iters):
        x = x + vcycle(b - K @ x)
        r = b - K @ x
        e = xstar - x
        nr = float(np.linalg.norm(r))
        out.append((r / nr, e / nr))
    return out


def remove_pressure_mean(vec: np.ndarray, N: int) -> np.ndarray:
    out = np.array(vec, dtype=np.float64)
    out[2 * N * N:] -= out[2 * N * N:].mean()
    return out


class LearnedStage:
    """Variable preconditioner z = V(v) + gamma c with the accept rule above.
    `corrector(r_hat) -> c_hat` maps a unit-norm residual to a correction;
    `net_corrector` builds it from network weights."""

    def __init__(self, K, vcycle, corrector, N: int, margin: float = 1e-3):
        self.K, self.V, self.corr, self.N, self.margin = K, vcycle, corrector, N, margin
        self.accepted = 0
        self.rejected = 0

    def __call__(self, v: np.ndarray) -> np.ndarray:
        z0 = self.V(v)
        r = v - self.K @ z0
        nr2 = float(r @ r)
        if nr2 == 0.0:
            self.rejected += 1
            return z0
        nr = np.sqrt(nr2)
        c = remove_pressure_mean(nr * self.corr(r / nr), self.N)
        Kc = self.K @ c
        den = float(Kc @ Kc)
        num = float(r @ Kc)
        if not (den > 0.0 and np.isfinite(den) and np.isfinite(num)):
            self.rejected += 1
            return z0
        gamma = num / den
        if num * num / den >= self.margin * nr2:
            self.accepted += 1
            return z0 + gamma * c
        self.rejected += 1
        return z0


def net_corrector(w: np.ndarray, N: int, bf16: bool = True):
    def corr(rhat: np.ndarray) -> np.ndarray:
        y3, _ = forward(to_image(rhat, N)[None], w, bf16)
        return y3[0].ravel()
    return corr
