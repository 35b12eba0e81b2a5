"""Oracle of the plan-selection cost model: a 7 -> 64 -> 64 -> 1 ReLU network, its mean
squared error loss and the loss gradient, in float64 with plain numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper leaves the BSGS split and the depth of the transform decomposition open
(Sec. 2.6: the best point depends on the parameters and the ciphertext level); the
library picks them by measured or predicted latency, with this network as the
predictor.  Its shape and loss are the library's interface.  The gradient is the
textbook backpropagation of the definitions below; tests pin it to central finite
differences of `loss`.

Parameter vector layout (same as the library's): W1 [7][64], b1 [64], W2 [64][64]
(row = input unit), b2 [64], w3 [64], b3.
"""
import numpy as np

F, H = 7, 64
SIZES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    """f(x) = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 for each row x of X"""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ q["W1"] + q["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ q["W2"] + q["b2"]
    h2 = np.maximum(a2, 0.0)
    return h2 @ q["w3"] + q["b3"][0], (a1, h1, a2, h2)


def loss(p, X, y):
    out, _ = forward(p, X)
    return float(np.mean((out - np.asarray(y, dtype=np.float64)) ** 2))


def grad(p, X, y):
    """d loss / d p by the chain rule, layer by layer"""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    out, (a1, h1, a2, h2) = forward(p, X)
    n = X.shape[0]
    dout = 2.0 * (out - np.asarray(y, dtype=np.float64)) / n
    g = {"w3": h2.T @ dout, "b3": np.array([dout.sum()])}
    dh2 = np.outer(dout, q["w3"]) * (a2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ q["W2"].T) * (a1 > 0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return pack(g)
