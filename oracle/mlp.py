"""Plain FP64 reference of the learned form's network (TEST INFRASTRUCTURE:
only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline may use
it; it shares nothing with the HIP path).

Network 6 -> 64 -> 64 -> 2: h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2),
y = h2 W3 + b3.  Losses: squared error L = sum_r sum_o C[r,o] (y - T)^2, or
the log-link Poisson deviance L = sum C[r,o] (e^y - T y), whose minimiser
over y is ln E[T] (unbiased for targets with many zeros).
Parameter vector order: W1[6][64], b1[64], W2[64][64], b2[64], W3[64][2],
b3[2].  The gradient is written out by the chain rule; it is pinned against
central finite differences in tests/test_oracle_mlp.py.  The same code with
every matrix-product operand rounded to bfloat16 (nearest even) is the
reference of matrix-core kernels that take BF16 operands and accumulate in
FP32.  This network is not from the paper, which names bias tuning as
future work (Conclusions)."""
import numpy as np

N_IN, N_H, N_OUT = 6, 64, 2
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init(seed=0):
    """Uniform (Glorot) initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            d[name] = rng.uniform(-lim, lim, shp)
        else:
            d[name] = np.zeros(shp)
    return pack(d)


SQUARED, POISSON = 0, 1


def _same(a):
    return a


def forward(p, X, rnd=_same):
    """Outputs and activations; rnd is applied to every operand of a
    matrix product (identity: exact FP64)."""
    W = unpack(p)
    x = np.asarray(X, dtype=np.float64)[:, :N_IN]
    h1 = np.tanh(rnd(x) @ rnd(W["W1"]) + W["b1"])
    h2 = np.tanh(rnd(h1) @ rnd(W["W2"]) + W["b2"])
    y = rnd(h2) @ rnd(W["W3"]) + W["b3"]
    return y, (x, h1, h2)


def _loss_terms(y, T, C, kind):
    if kind == POISSON:
        return C * (np.exp(y) - T * y), C * (np.exp(y) - T)
    return C * (y - T) ** 2, 2.0 * C * (y - T)


def loss(p, X, T, C, kind=SQUARED):
    y, _ = forward(p, X)
    return float(np.sum(_loss_terms(y, T, C, kind)[0]))


def grad(p, X, T, C, kind=SQUARED, rnd=_same):
    """Gradient and loss; with rnd = bf16 every product operand (inputs,
    weights, activations, back-propagated errors) is rounded as the
    matrix cores see it."""
    W = unpack(p)
    y, (x, h1, h2) = forward(p, X, rnd)
    lt, dy = _loss_terms(y, T, C, kind)                 # dL/dy
    g = {"W3": rnd(h2).T @ rnd(dy), "b3": dy.sum(0)}
    dz2 = (rnd(dy) @ rnd(W["W3"]).T) * (1.0 - h2 ** 2)  # through tanh
    g["W2"], g["b2"] = rnd(h1).T @ rnd(dz2), dz2.sum(0)
    dz1 = (rnd(dz2) @ rnd(W["W2"]).T) * (1.0 - h1 ** 2)
    g["W1"], g["b1"] = rnd(x).T @ rnd(dz1), dz1.sum(0)
    return pack(g), float(np.sum(lt))


def grad_bf16(p, X, T, C, kind=SQUARED):
    """The gradient with BF16 product operands (see grad)."""
    return grad(p, X, T, C, kind, rnd=bf16)


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v


def bf16(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
