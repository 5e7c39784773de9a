"""IEEE round-to-nearest-even into FP32, FP16 and BF16 (oracle; test only).

Used to give the oracle the same stored coefficients and output precisions as
the precision sweep (coefficients and outputs in FP32, FP16 or BF16).  Values
are returned widened back to float64 so the oracle keeps computing in FP64.
"""
import numpy as np


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_f16(x):
    # numpy converts float64 -> float16 with a single correctly rounded step
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def bf16_bits_from_f64(x):
    """BF16 bit patterns of float64 values, one RNE rounding step.

    BF16 keeps 8 significand bits (7 stored).  The float64 value is split at
    the BF16 ulp with exact integer arithmetic on its bits, so there is no
    intermediate FP32 rounding.  Normal-range inputs only (|x| in
    [2^-126, 2^127]) or exact zeros; the coefficient and output ranges of this
    method lie well inside that range.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    out = np.zeros(x.shape, dtype=np.uint16)
    bits = x.view(np.uint64)
    sign = (bits >> np.uint64(63)).astype(np.uint16)
    mag = np.abs(x)
    nz = mag != 0
    if np.any(nz & ((mag < 2.0 ** -126) | (mag > 2.0 ** 127) | ~np.isfinite(mag))):
        raise ValueError("bf16_bits_from_f64: value outside the normal BF16 range")
    mbits = mag.view(np.uint64)
    exp = ((mbits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    frac = (mbits & np.uint64((1 << 52) - 1)) | np.uint64(1 << 52)  # 53-bit significand
    # keep 8 significant bits: drop 45 bits with round-half-even
    drop = np.uint64(45)
    keep = frac >> drop
    rem = frac & np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    up = (rem > half) | ((rem == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    keep = keep + up.astype(np.uint64)
    carry = keep == np.uint64(1 << 8)
    keep = np.where(carry, keep >> np.uint64(1), keep)
    exp = exp + carry.astype(np.int64)
    ebits = (exp + 127).astype(np.uint16)
    mant = (keep & np.uint64(0x7F)).astype(np.uint16)
    val = (sign << np.uint16(15)) | (ebits << np.uint16(7)) | mant
    out[nz] = val[nz]
    out[~nz] = (sign[~nz] << np.uint16(15))
    return out


def bf16_bits_to_f64(b):
    b = np.atleast_1d(np.asarray(b, dtype=np.uint16)).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def round_bf16(x):
    x = np.asarray(x, dtype=np.float64)
    return bf16_bits_to_f64(bf16_bits_from_f64(x)).reshape(x.shape)


ROUND = {"f64": lambda x: np.asarray(x, dtype=np.float64),
         "f32": round_f32, "f16": round_f16, "bf16": round_bf16}


def ulp(x, dtype):
    """Spacing of the output dtype at |x| (for 1-ulp tolerances)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    if dtype == "f32":
        return np.spacing(x.astype(np.float32)).astype(np.float64)
    if dtype == "f16":
        return np.spacing(x.astype(np.float16)).astype(np.float64)
    if dtype == "bf16":
        r = round_bf16(np.maximum(x, 2.0 ** -126))
        e = np.floor(np.log2(r))
        return 2.0 ** (e - 7)
    if dtype == "f64":
        return np.spacing(x)
    raise ValueError(dtype)
