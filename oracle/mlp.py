"""FP64 forward and backward of the surrogate network (oracle; test only).

The surrogate stands in for Section 5.1's rescaled inverse P_nu(U; y) of the
non-central chi-squared distribution at fixed nu.  Network (the library
implements the same definition independently):

  inputs     w  = an approximate normal of U (a fixed, non-learned feature)
             g  = 2 (log lambda - lo) / (hi - lo) - 1   (lambda range [e^lo, e^hi])
  layer 1    a1 = W1 [w, g] + b1        W1: 64 x 2, FP32
             h1 = relu(a1),  relu(t) = max(t, 0)
             (bf16=True, the inference kernels' form: every FP32 value
             x of w, g, W1 and b1 is split into BF16 parts x = x_hi + x_lo
             + r, x_hi = bf16(x), x_lo = bf16(x - x_hi), and
             a1 = Ww_hi w_hi + Ww_lo w_hi + Ww_hi w_lo + Wg_hi g_hi
                  + Wg_lo g_hi + Wg_hi g_lo + b_hi + b_lo,
             the products of BF16 matrix-core operands; it differs from
             the exact a1 by about 2^-16 relative)
  layer 2    a2 = W2 bf16(h1) + b2      W2: 64 x 64 stored in BF16, FP32 sums
             h2 = relu(a2)
  layer 3    o  = W3 . h2 + b3          W3: 64, FP32
  output     P~ = w + o

`bf16=True` rounds h1 and W2 to BF16 (round to nearest even) before the
layer-2 products, as the inference and training kernels do; all sums are FP64
here.  Parity unpinned for trained weights (they are learned); the forward and
backward definitions are pinned by finite differences and by hand-computed
tiny cases in the tests.
"""
import numpy as np

from .dtypes import round_bf16

H = 64
PARAM_SHAPES = {"W1": (H, 2), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H,), "b3": ()}
PARAM_ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]


def relu(t):
    return np.maximum(t, 0.0)


def drelu(t):
    """The derivative of relu, taken as 0 at t = 0."""
    return (np.asarray(t) > 0.0).astype(np.float64)


def g_feature(loglam, lo, hi):
    return 2.0 * (np.asarray(loglam, float) - lo) / (hi - lo) - 1.0


def split_bf16(x):
    """(hi, lo): hi = bf16(x), lo = bf16(x - hi) of FP32 values x."""
    x = np.asarray(x, float).astype(np.float32).astype(np.float64)
    hi = round_bf16(x)
    return hi, round_bf16(x - hi)  # x - hi is exact in FP32


def layer1_split(params, w, g):
    """a1 of the split-BF16 layer 1 (module docstring), summed in FP64."""
    W1 = np.asarray(params["W1"], float)
    wh, wl = split_bf16(w)
    gh, gl = split_bf16(g)
    Wwh, Wwl = split_bf16(W1[:, 0])
    Wgh, Wgl = split_bf16(W1[:, 1])
    bh, bl = split_bf16(params["b1"])
    return (np.outer(wh, Wwh) + np.outer(wh, Wwl) + np.outer(wl, Wwh)
            + np.outer(gh, Wgh) + np.outer(gh, Wgl) + np.outer(gl, Wgh) + bh + bl)


def forward(params, w, g, bf16=True, return_cache=False):
    w = np.asarray(w, float)
    g = np.asarray(g, float)
    x = np.stack([w, g], axis=-1)                    # (n, 2)
    if bf16:
        a1 = layer1_split(params, w, g)
    else:
        a1 = x @ np.asarray(params["W1"], float).T + params["b1"]
    h1 = relu(a1)
    W2 = np.asarray(params["W2"], float)
    h1q = round_bf16(h1) if bf16 else h1
    W2q = round_bf16(W2) if bf16 else W2
    a2 = h1q @ W2q.T + params["b2"]
    h2 = relu(a2)
    o = h2 @ np.asarray(params["W3"], float) + float(params["b3"])
    P = w + o
    if return_cache:
        return P, dict(x=x, a1=a1, h1q=h1q, W2q=W2q, a2=a2, h2=h2)
    return P


def loss_and_grads(params, w, g, target, bf16=True):
    """Mean squared error L = mean((P~ - target)^2) and dL/dparams (FP64).

    With bf16=True the gradient is taken through the rounded values as if the
    rounding were the identity (the straight-through convention the training
    kernels use): dL/dW2 uses bf16(h1), dL/dh1 uses bf16(W2).
    """
    P, c = forward(params, w, g, bf16=bf16, return_cache=True)
    n = P.shape[0]
    r = P - np.asarray(target, float)
    L = float(np.mean(r * r))
    dP = 2.0 * r / n                                  # dL/dP~ = dL/do
    gW3 = c["h2"].T @ dP
    gb3 = np.sum(dP)
    dh2 = np.outer(dP, params["W3"])
    da2 = dh2 * drelu(c["a2"])
    gW2 = da2.T @ c["h1q"]
    gb2 = np.sum(da2, axis=0)
    dh1 = da2 @ c["W2q"]
    da1 = dh1 * drelu(c["a1"])
    gW1 = da1.T @ c["x"]
    gb1 = np.sum(da1, axis=0)
    return L, {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def init_params(seed):
    """A seeded initialisation (uniform +-1/sqrt(fan_in)); for tests."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, fan in (("W1", 2), ("b1", 2), ("W2", H), ("b2", H), ("W3", H), ("b3", H)):
        p[name] = rng.uniform(-1.0, 1.0, PARAM_SHAPES[name]) / np.sqrt(fan)
    return p
