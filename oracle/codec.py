"""Reduced-precision storage of matrix values (oracle, test-only).

The paper names the switch to single precision as its most promising next step
(Sec. 5.4: it doubles the arithmetic intensity of the bandwidth-bound SpMV).  The
mixed-precision form stores A in FP32, or in FP16 / BF16 with one power-of-two scale
per scalar row, runs the V-cycle in FP32 and keeps the outer defect in FP64.

Encoding (exact reading, reproduced bit for bit by the library at setup):
  s_i  = 2^e_i, e_i the smallest integer with max_j |a_ij| <= 2^e_i  (s_i = 1 for a zero row)
  q_ij = round-to-nearest-even(a_ij / s_i) in FP16 or BF16, straight from FP64
  decode: a_ij ~ s_i * q_ij evaluated in FP32.
"""
from __future__ import annotations

import numpy as np


def row_exponents(A_csr) -> np.ndarray:
    """e_i per scalar row of a scipy CSR matrix."""
    n = A_csr.shape[0]
    mx = np.zeros(n)
    nz = np.diff(A_csr.indptr) > 0
    mx[nz] = np.maximum.reduceat(np.abs(A_csr.data), A_csr.indptr[:-1][nz])
    m, e = np.frexp(mx)                 # mx = m 2^e, m in [0.5, 1)
    e = np.where(m == 0.5, e - 1, e)
    e = np.where(mx == 0.0, 0, e)
    return e.astype(np.int32)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to BF16 (8 significant bits, RNE) and return the uint16 bits."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                  # x = m 2^e, |m| in [0.5, 1)
    q = np.rint(m * 256.0)              # 8 significant bits, ties to even
    r = np.ldexp(q, e - 8)
    if np.any((r != 0) & (np.abs(r) < 2.0 ** -126)):
        raise ValueError("value below the BF16 normal range")
    f32 = r.astype(np.float32)          # exact: r has 8 significant bits
    return (f32.view(np.uint32) >> 16).astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def encode(A_csr, fmt: str):
    """Returns (exponents per row, uint16 codes aligned with A_csr.data)."""
    e = row_exponents(A_csr)
    rows = np.repeat(np.arange(A_csr.shape[0]), np.diff(A_csr.indptr))
    scaled = np.ldexp(A_csr.data, -e[rows])            # exact division by a power of two
    if fmt == "fp16":
        codes = scaled.astype(np.float16).view(np.uint16)
    elif fmt == "bf16":
        codes = to_bf16_bits(scaled)
    else:
        raise ValueError(fmt)
    return e, codes


def decode_f32(A_csr, e, codes, fmt: str) -> np.ndarray:
    """FP32 values s_i * q_ij aligned with A_csr.data."""
    rows = np.repeat(np.arange(A_csr.shape[0]), np.diff(A_csr.indptr))
    q = codes.view(np.float16).astype(np.float32) if fmt == "fp16" else bf16_bits_to_f32(codes)
    return (np.ldexp(np.float32(1.0), e[rows]).astype(np.float32) * q).astype(np.float32)
