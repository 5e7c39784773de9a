"""Counter-based uniforms: Philox-4x32-10 and the uniform grids (oracle).

Test infrastructure only.  Written from the published definition of Philox
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): a 4 x 32-bit counter and a 2 x 32-bit key; each of ten rounds takes
the 32 x 32 -> 64-bit products of the multipliers 0xD2511F53 and 0xCD9E8D57
with counter words 0 and 2, mixes the high halves with the other two words and
the key, and the key is bumped by the Weyl constants 0x9E3779B9, 0xBB67AE85
between rounds.

The paper assumes cheap uniforms (Section 1) and couples the exact and the
approximate normal of one time step through one shared uniform (Section 4.1).
The uniform grids used here:

u53 (FP64)  k = the top 53 bits of the 64-bit word (hi << 32 | lo);
            u = ((double)k + 0.5) * 2^-53, each IEEE operation rounded to
            nearest even; the single value that rounds to 1.0 (k = 2^53 - 1)
            is replaced by 1 - 2^-53.
u24 (FP32)  m = the top 23 bits of one 32-bit word; u = (m + 0.5) * 2^-23,
            i.e. the odd multiples of 2^-24; exact in FP32, symmetric about
            1/2, never 0 or 1.  In a coupled pair its word is the `hi` word of
            the u53 draw, so both uniforms share their leading 23 bits.

Stream layouts (shared definition with the library's documented layout):
uniform fill, FP32 : element i -> word g = offset + i; counter
                     (lo32(g/4), hi32(g/4), lo32(stream), hi32(stream)),
                     key (lo32(seed), hi32(seed)); word g mod 4.
uniform fill, FP64 : element i -> draw g = offset + i; counter
                     (lo32(g/2), hi32(g/2), lo32(stream), hi32(stream));
                     words (2 (g mod 2), 2 (g mod 2) + 1) as (hi, lo).
path streams       : path P, block b: counter (b, lo32(P), hi32(P), tag) with
                     tag = level | (stream_kind << 8); key = seed.  One-word
                     draws take step n from block n/4, word n mod 4; two-word
                     draws take block n/2, words 2 (n mod 2), 2 (n mod 2) + 1.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox-4x32-10 on arrays.  ctr: (..., 4) uint32, key: (..., 2) uint32
    (broadcastable).  Returns (..., 4) uint32."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = key[..., 0].copy(), key[..., 1].copy()
    for r in range(10):
        p0 = M0 * c0  # < 2^64: product of two 32-bit values
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
    out = np.stack(np.broadcast_arrays(c0, c1, c2, c3), axis=-1)
    return out.astype(np.uint32)


def _split64(x):
    x = np.asarray(x, dtype=np.uint64)
    return (x & MASK32).astype(np.uint32), (x >> np.uint64(32)).astype(np.uint32)


def u53_from_words(hi, lo):
    """u53 grid (see the module header)."""
    w = (np.asarray(hi, dtype=np.uint64) << np.uint64(32)) | np.asarray(lo, dtype=np.uint64)
    k = (w >> np.uint64(11)).astype(np.float64)  # exact, k < 2^53
    u = (k + 0.5) * 2.0 ** -53
    return np.where(u == 1.0, 1.0 - 2.0 ** -53, u)


def u24_from_word(w):
    """u24 grid as float32 values (see the module header)."""
    m = (np.asarray(w, dtype=np.uint32) >> np.uint32(9)).astype(np.float64)
    return ((m + 0.5) * 2.0 ** -23).astype(np.float32)


def fill_words(seed, stream, offset, n):
    """The 32-bit words of the FP32 uniform fill (layout in the header)."""
    g = np.uint64(offset) + np.arange(n, dtype=np.uint64)
    blk = g >> np.uint64(2)
    blo, bhi = _split64(blk)
    slo, shi = _split64(np.uint64(stream))
    klo, khi = _split64(np.uint64(seed))
    ctr = np.stack([blo, bhi, np.full(n, slo), np.full(n, shi)], axis=-1)
    x = philox4x32_10(ctr, np.array([klo, khi], dtype=np.uint32))
    return x[np.arange(n), (g & np.uint64(3)).astype(np.int64)]


def uniform_fill_f32(seed, stream, offset, n):
    return u24_from_word(fill_words(seed, stream, offset, n))


def uniform_fill_f64(seed, stream, offset, n):
    g = np.uint64(offset) + np.arange(n, dtype=np.uint64)
    blk = g >> np.uint64(1)
    blo, bhi = _split64(blk)
    slo, shi = _split64(np.uint64(stream))
    klo, khi = _split64(np.uint64(seed))
    ctr = np.stack([blo, bhi, np.full(n, slo), np.full(n, shi)], axis=-1)
    x = philox4x32_10(ctr, np.array([klo, khi], dtype=np.uint32))
    j = (g & np.uint64(1)).astype(np.int64)
    rows = np.arange(n)
    return u53_from_words(x[rows, 2 * j], x[rows, 2 * j + 1])


def path_words(seed, paths, tag, n_blocks):
    """Philox output for blocks 0..n_blocks-1 of each path: (n_paths, n_blocks, 4)."""
    paths = np.asarray(paths, dtype=np.uint64)
    plo, phi_ = _split64(paths)
    klo, khi = _split64(np.uint64(seed))
    b = np.arange(n_blocks, dtype=np.uint32)
    P, B = len(paths), n_blocks
    ctr = np.empty((P, B, 4), dtype=np.uint32)
    ctr[..., 0] = b[None, :]
    ctr[..., 1] = plo[:, None]
    ctr[..., 2] = phi_[:, None]
    ctr[..., 3] = np.uint32(tag)
    return philox4x32_10(ctr, np.array([klo, khi], dtype=np.uint32))


def path_u24(seed, paths, tag, n_steps):
    """One-word draws: (n_paths, n_steps) float32 u24 uniforms."""
    nb = (n_steps + 3) // 4
    x = path_words(seed, paths, tag, nb).reshape(len(paths), nb * 4)[:, :n_steps]
    return u24_from_word(x)


def path_u53_u24(seed, paths, tag, n_steps):
    """Two-word draws: (u53, u24) pairs sharing the hi word, each (n_paths, n_steps)."""
    nb = (n_steps + 1) // 2
    x = path_words(seed, paths, tag, nb).reshape(len(paths), nb * 2, 2)[:, :n_steps]
    hi, lo = x[..., 0], x[..., 1]
    return u53_from_words(hi, lo), u24_from_word(hi)


def stream_tag(level, stream_kind):
    return (int(level) & 0xFF) | (int(stream_kind) << 8)
