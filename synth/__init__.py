"""Seeded synthetic inputs for triangular multiply / solve workloads.

This module is shared by the tests, the benchmark and the CPU reference
checks.  It only draws random numbers and lays them out; it holds none of the
triangular arithmetic.  Every matrix is column-major (numpy ``order='F'``):
element (i, j) of an m-by-n matrix sits at flat index ``i + j*ld``.

Random streams come from numpy's Philox4x32-10 counter-based generator, keyed
by ``(seed, workload, instance, tag)`` so that any matrix of any workload can be
regenerated alone.

Generators
----------
* ``tri``   : triangular factor.  Referenced off-diagonal entries U(-1,1),
              diagonal chosen by ``diag_kind``; the unreferenced triangle is
              filled with ``fill`` (NaN in tests so a stray read shows up, 0 in
              timing runs).
* ``dense`` : dense right-hand side / multiplicand, entries U(-1,1).
* ``exact_tri`` / ``exact_dense`` : small-integer inputs for which every
              intermediate of a triangular multiply or solve is exactly
              representable, so all correct implementations agree bit for bit.
"""
from __future__ import annotations

import numpy as np

SEED = 250413821

# workload ids used to key the random streams
W_SMALL = 1        # m=n=512 FP64 parity case
W_SWEEP = 2        # square sweep 1024..16384
W_MIXED = 3        # mixed precision, m=n=8192
W_BATCH = 4        # batched uneven instances
W_SERVE = 5        # serving stream
W_TEST = 9         # ad-hoc test cases

T_A, T_B, T_X, T_META = 1, 2, 3, 4


def rng(workload: int, *keys: int, seed: int = SEED) -> np.random.Generator:
    """Philox4x32-10 stream keyed by (seed, workload, *keys), e.g. keys = (instance, tag)."""
    ss = np.random.SeedSequence([seed, workload, *[int(k) for k in keys]])
    return np.random.Generator(np.random.Philox(ss))


def _u11(g: np.random.Generator, shape) -> np.ndarray:
    return 2.0 * g.random(shape) - 1.0


def tri(m: int, uplo: str, g: np.random.Generator, diag_kind: str = "base",
        fill: float = np.nan, c: float | None = None) -> np.ndarray:
    """m-by-m triangular factor, column-major, float64.

    diag_kind:
      "base"   diagonal m + U(0,1)                  (the sweep generator)
      "stress" diagonal sqrt(m) * (1 + U(0,1))       (off-diagonal part not damped)
      "cond"   diagonal c + U(0,1)                   (c sets the 1-norm condition)
      "unit"   off-diagonals U(-1,1)/m, diagonal = ``fill`` (never read with diag=U)
    """
    uplo = uplo.upper()
    # draw in column-major order directly (the transpose of a C-order draw is
    # Fortran-ordered), then shape it in place, one column at a time
    a = g.random((m, m)).T
    a *= 2.0
    a -= 1.0
    d = g.random(m)
    if diag_kind == "base":
        dv = m + d
    elif diag_kind == "stress":
        dv = np.sqrt(m) * (1.0 + d)
    elif diag_kind == "cond":
        if c is None:
            raise ValueError("diag_kind='cond' needs c")
        dv = c + d
    elif diag_kind == "unit":
        a /= m
        dv = np.full(m, fill)
    else:
        raise ValueError(diag_kind)
    for j in range(m):
        if uplo == "L":
            a[:j, j] = fill
        else:
            a[j + 1:, j] = fill
        a[j, j] = dv[j]
    return a


def dense(m: int, n: int, g: np.random.Generator) -> np.ndarray:
    """m-by-n matrix with entries U(-1,1), column-major float64."""
    return np.asfortranarray(_u11(g, (m, n)))


def exact_tri(m: int, uplo: str, g: np.random.Generator, offdiag=(-1, 0, 1),
              diag=(1.0,), fill: float = np.nan) -> np.ndarray:
    """Small-integer triangular factor: off-diagonals drawn from ``offdiag``,
    diagonal drawn from ``diag`` (e.g. powers of two with signs)."""
    uplo = uplo.upper()
    off = g.choice(np.asarray(offdiag, dtype=np.float64), size=(m, m))
    dv = g.choice(np.asarray(diag, dtype=np.float64), size=m)
    mask = np.tril(np.ones((m, m), dtype=bool), -1) if uplo == "L" else np.triu(np.ones((m, m), dtype=bool), 1)
    out = np.where(mask, off, fill)
    out[np.arange(m), np.arange(m)] = dv
    return np.asfortranarray(out)


def exact_dense(m: int, n: int, g: np.random.Generator, bound: int = 8) -> np.ndarray:
    """m-by-n integer-valued matrix with entries in [-bound, bound]."""
    return np.asfortranarray(g.integers(-bound, bound + 1, size=(m, n)).astype(np.float64))


def round_to(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round float64 values to a narrower type with round-to-nearest-even and
    return them (still exactly) as float64.  dtype in {"f64","f32","f16","bf16"}.
    """
    x = np.asarray(x, dtype=np.float64)
    if dtype == "f64":
        return x.copy(order="F")
    if dtype == "f32":
        return np.asfortranarray(x.astype(np.float32).astype(np.float64))
    if dtype == "f16":
        return np.asfortranarray(x.astype(np.float16).astype(np.float64))
    if dtype == "bf16":
        return np.asfortranarray(bf16_bits_to_f32(f32_to_bf16_bits(x.astype(np.float32))).astype(np.float64))
    raise ValueError(dtype)


def f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round-to-nearest-even; NaN kept quiet."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint32)
    nan = np.isnan(x32.reshape(-1)).reshape(u.shape)
    r = np.where(nan, (u >> 16).astype(np.uint32) | 0x40, r)
    return r.astype(np.uint16).reshape(np.shape(x32))


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def loguniform_int(g: np.random.Generator, lo: int, hi: int, size) -> np.ndarray:
    """Integers log-uniform on [lo, hi] (rounded)."""
    v = np.exp(g.uniform(np.log(lo), np.log(hi), size=size))
    return np.clip(np.rint(v).astype(np.int64), lo, hi)


def batch_shapes(count: int, g: np.random.Generator, m_lo: int = 16, m_hi: int = 1024, n_lo: int = 1,
                 n_hi: int = 128):
    """Shapes of a batch of independent problems: m log-uniform on [m_lo, m_hi],
    number of right-hand sides uniform on [n_lo, n_hi], uplo 'L'/'U' 50/50."""
    ms = loguniform_int(g, m_lo, m_hi, count)
    ns = g.integers(n_lo, n_hi + 1, size=count)
    uplos = np.where(g.random(count) < 0.5, "L", "U")
    return [(int(m), int(n), str(u)) for m, n, u in zip(ms, ns, uplos)]


# ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter-based -------
_PHILOX_M0, _PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
_PHILOX_W0, _PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
_M32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on arrays of 32-bit words (held as uint64)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _M32 for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _M32
    k1 = np.asarray(k1, dtype=np.uint64) & _M32
    for _ in range(10):
        p0 = np.uint64(_PHILOX_M0) * c0
        p1 = np.uint64(_PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_M32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_M32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(_PHILOX_W0)) & np.uint64(_M32)
        k1 = (k1 + np.uint64(_PHILOX_W1)) & np.uint64(_M32)
    return c0, c1, c2, c3


def philox_matrix(kind: int, seed: int, stream: int, ident: int, m: int, n: int, param: float = 0.0) -> np.ndarray:
    """The host twin of the library's on-device synthetic fill: element (i, j)
    from counter (i, j, id_lo, id_hi), key (seed_lo ^ stream, seed_hi);
    u = 53 bits of words (1, 0) * 2^-53.  kind 0: 2u-1; kind 1 / 2: lower / upper
    triangular with off-diagonal 2u-1, diagonal param + u, zero elsewhere."""
    i = np.repeat(np.arange(m, dtype=np.uint64)[:, None], n, axis=1)
    j = np.repeat(np.arange(n, dtype=np.uint64)[None, :], m, axis=0)
    k0 = (seed & _M32) ^ (stream & _M32)
    k1 = (seed >> 32) & _M32
    x0, x1, _, _ = philox4x32_10(i, j, ident & _M32, (ident >> 32) & _M32, k0, k1)
    bits = ((x1 << np.uint64(32)) | x0) >> np.uint64(11)
    u = bits.astype(np.float64) * 2.0 ** -53
    if kind == 0:
        out = 2.0 * u - 1.0
    else:
        ii, jj = np.indices((m, n))
        tri = (ii >= jj) if kind == 1 else (ii <= jj)
        out = np.where(tri, np.where(ii == jj, param + u, 2.0 * u - 1.0), 0.0)
    return np.asfortranarray(out)
