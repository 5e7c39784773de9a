"""Seeded synthetic inputs shared by the oracle side and the GPU side of the
tests.  Only random draws and hand-picked edge values live here; none of the
method's arithmetic does."""
import numpy as np


def edge_uniforms(dtype=np.float64):
    """Hand-picked inputs: 1/2, 0, 1, NaN, dyadic boundaries 2^-k and their
    neighbours on both sides of 1/2, subnormals, values close to 1."""
    ft = np.dtype(dtype).type
    vals = [0.5, 0.0, 1.0, np.nan, 0.25, 0.75]
    for k in range(1, 70):
        b = ft(2.0) ** ft(-k)
        if b == 0:
            break
        for x in (b, np.nextafter(b, ft(0)), np.nextafter(b, ft(1))):
            vals += [x, ft(1) - x]
    vals += [np.finfo(dtype).tiny, np.finfo(dtype).tiny / 2, np.nextafter(ft(0), ft(1)),
             np.nextafter(ft(1), ft(0)), np.nextafter(ft(0.5), ft(0)), np.nextafter(ft(0.5), ft(1))]
    return np.array(vals, dtype=dtype)


def random_uniforms(n, seed, dtype=np.float64):
    """A mix of plain uniforms (3/4) and log-uniform tails mirrored at random
    (1/4), so that every dyadic row is populated."""
    rng = np.random.default_rng(seed)
    n_tail = n // 4
    body = rng.random(n - n_tail)
    tmin = np.log10(np.finfo(dtype).tiny)
    tail = 10.0 ** rng.uniform(tmin + 1, -0.3, n_tail)
    flip = rng.random(n_tail) < 0.5
    tail = np.where(flip, 1.0 - tail, tail)
    u = np.concatenate([body, tail]).astype(dtype)
    rng.shuffle(u)
    return u


def random_u24(n, seed):
    """Uniforms on the u24 grid (odd multiples of 2^-24) as float32."""
    rng = np.random.default_rng(seed)
    m = rng.integers(0, 1 << 23, n)
    return ((m + 0.5) * 2.0 ** -23).astype(np.float32)
