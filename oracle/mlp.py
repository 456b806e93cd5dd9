"""Plain FP64 reference of the interpolation-weight MLP (96 -> 64 -> 64 -> 8,
ReLU). TEST INFRASTRUCTURE ONLY: used by the test-suite to check the GPU
forward, gradient and optimiser kernels; never by the product path.

The network is not part of the paper: it predicts the F rows of the
interpolation operator P (eq. ls_interpolation, eq. Pstructure) from
per-point features. Parameter order (row-major, out x in):
W1[64][96], b1[64], W2[64][64], b2[64], W3[8][64], b3[8].

Loss over N points with targets T and mask M (N x 8):
    L = 1/(2N) sum_p sum_t M_pt (y_pt - T_pt)^2
"""
import numpy as np

N_IN, N_HID, N_OUT = 96, 64, 8
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def round_bf16(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP64."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, bf16=False):
    """Outputs y (N x 8) and the pre-activations (a1, a2). With bf16=True the
    weights, the inputs and both hidden activations are rounded to BF16
    (biases and accumulation stay exact), the arithmetic of the MFMA path."""
    w = unpack(p)
    X = np.asarray(X, np.float64)
    if bf16:
        W1, W2, W3 = (round_bf16(w[k]) for k in ("W1", "W2", "W3"))
        X = round_bf16(X)
    else:
        W1, W2, W3 = w["W1"], w["W2"], w["W3"]
    a1 = X @ W1.T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    if bf16:
        h1 = round_bf16(h1)
    a2 = h1 @ W2.T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    if bf16:
        h2 = round_bf16(h2)
    y = h2 @ W3.T + w["b3"]
    return y, (a1, a2)


def loss_grad(p, X, T, M):
    """Loss and its gradient with respect to the packed parameters, by
    backpropagation through the three layers."""
    w = unpack(p)
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    M = np.asarray(M, np.float64)
    n = X.shape[0]
    y, (a1, a2) = forward(p, X)
    h1, h2 = np.maximum(a1, 0.0), np.maximum(a2, 0.0)
    d = M * (y - T)
    loss = 0.5 * float((d * (y - T)).sum()) / n
    dy = d / n
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    d2 = (dy @ w["W3"]) * (a2 > 0)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ w["W2"]) * (a1 > 0)
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[1])
        else:
            d[name] = np.zeros(shape)
    return pack(d).astype(np.float32)
