"""Reference MLP for the learned initial weights -- TEST INFRASTRUCTURE ONLY.

Plain numpy in float64: 4 -> 64 -> 64 -> 64 -> 1 with the tanh form of GELU
(Hendrycks and Gimpel), MSE loss and its gradient by the chain rule.  With
rounding on, every matrix-product input (inputs, weights, biases,
activations and back-propagated pre-activation gradients) is rounded to
bfloat16 (round to nearest even, through float32) at the same points as the
HIP kernels; with rounding off the function is the exact float64 network.
Pins: the float64 gradient against central finite differences, the rounding
against hand-worked bfloat16 cases, GELU against the exact x*Phi(x) within the
tanh form's error, and Adam (Kingma and Ba) against the closed forms of its
first step, of a constant gradient and of a single impulse.  term_scales (the
yardstick of the element-wise comparison, not a result) is pinned by the
triangle inequality and by equality when every term is non-negative.

Parameter vector layout (8705 floats): W1[64][4], b1[64], W2[64][64], b2[64],
W3[64][64], b3[64], W4[64], b4[1].
"""
import numpy as np

N_PARAMS = 8705
_C = np.sqrt(2.0 / np.pi)


def bf16(a):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, np.float64)
    return dict(W1=p[0:256].reshape(64, 4), b1=p[256:320], W2=p[320:4416].reshape(64, 64), b2=p[4416:4480],
                W3=p[4480:8576].reshape(64, 64), b3=p[8576:8640], W4=p[8640:8704], b4=p[8704:8705])


def pack(d):
    return np.concatenate([d["W1"].ravel(), d["b1"], d["W2"].ravel(), d["b2"], d["W3"].ravel(), d["b3"],
                           d["W4"], d["b4"]])


def gelu(z):
    t = np.tanh(_C * (z + 0.044715 * z ** 3))
    return 0.5 * z * (1.0 + t), 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _C * (1.0 + 3 * 0.044715 * z * z)


def forward(p, x, round_bf16=True):
    R = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    w = {k: R(v) for k, v in unpack(p).items()}
    cache = {"x0": R(x)}
    z1 = cache["x0"] @ w["W1"].T + w["b1"]
    a1 = R(gelu(z1)[0])
    z2 = a1 @ w["W2"].T + w["b2"]
    a2 = R(gelu(z2)[0])
    z3 = a2 @ w["W3"].T + w["b3"]
    a3 = R(gelu(z3)[0])
    y = a3 @ w["W4"] + w["b4"][0]
    cache.update(z1=z1, z2=z2, z3=z3, a1=a1, a2=a2, a3=a3, w=w)
    return y, cache


def loss_and_grad(p, x, t, round_bf16=True):
    """MSE loss and its gradient with respect to the parameter vector."""
    R = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    y, c = forward(p, x, round_bf16)
    w = c["w"]
    n = y.shape[0]
    loss = np.mean((y - t) ** 2)
    dy = 2.0 * (y - t) / n
    g = {}
    g["W4"] = c["a3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    G3 = R(dy[:, None] * w["W4"][None, :] * gelu(c["z3"])[1])
    g["W3"] = G3.T @ c["a2"]
    g["b3"] = G3.sum(axis=0)
    G2 = R((G3 @ w["W3"]) * gelu(c["z2"])[1])
    g["W2"] = G2.T @ c["a1"]
    g["b2"] = G2.sum(axis=0)
    G1 = R((G2 @ w["W2"]) * gelu(c["z1"])[1])
    g["W1"] = G1.T @ c["x0"]
    g["b1"] = G1.sum(axis=0)
    return loss, pack(g)


def term_scales(p, x, t, round_bf16=True):
    """For every output y[s] and every gradient element: the sum of the
    absolute values of the terms that element sums (|b4| + sum_i |W4_i a3_si|
    for y; sum_s |G_so a_si| for a weight gradient, sum_s |G_so| for a bias
    gradient, with the pre-activation gradients G at the same rounding as
    loss_and_grad).  A sum of K terms evaluated in another order or precision
    differs from the exact sum by at most a multiple of this scale, so it is
    the yardstick of an element-wise comparison.  Returns (y_scale, g_scale)."""
    R = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    y, c = forward(p, x, round_bf16)
    w = c["w"]
    n = y.shape[0]
    dy = 2.0 * (y - t) / n
    ys = np.abs(w["b4"][0]) + np.abs(c["a3"]) @ np.abs(w["W4"])
    G3 = R(dy[:, None] * w["W4"][None, :] * gelu(c["z3"])[1])
    G2 = R((G3 @ w["W3"]) * gelu(c["z2"])[1])
    G1 = R((G2 @ w["W2"]) * gelu(c["z1"])[1])
    s = dict(W4=np.abs(c["a3"]).T @ np.abs(dy), b4=np.array([np.abs(dy).sum()]),
             W3=np.abs(G3).T @ np.abs(c["a2"]), b3=np.abs(G3).sum(axis=0),
             W2=np.abs(G2).T @ np.abs(c["a1"]), b2=np.abs(G2).sum(axis=0),
             W1=np.abs(G1).T @ np.abs(c["x0"]), b1=np.abs(G1).sum(axis=0))
    return ys, pack(s)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
