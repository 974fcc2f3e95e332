"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the method (no modular add/sub/mul over
limbs, no transform).  It only draws numbers and picks parameters:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014), used as a counter-based generator: output ``i`` of
  a stream with key ``s`` is ``mix(s + (i + 1) * GAMMA)``, vectorised in numpy.
* NTT-friendly primes ``q = c * 2**32 + 1`` of exactly ``lam - 4`` bits for a
  bit-width class ``lam`` (the paper's evaluation uses moduli four bits short
  of the class width so that the Barrett constant fits the class width,
  Section 5.2), found by a seeded search with Miller-Rabin.
* Primitive power-of-two roots of unity ``omega_n = z**((q-1)/n)`` where ``z``
  is the least quadratic non-residue (Euler's criterion), so ``omega_n`` has
  order exactly ``n`` for every power of two ``n`` dividing ``q - 1``.
* Uniform residues in ``[0, q)`` by rejection sampling, returned element-major
  (shape ``(n, L)``, little-endian 32-bit limbs: limb 0 least significant).

Python's built-in ``pow`` is used for the number-theoretic parameter choice
(primality, roots); that is input selection, not the computation under test.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

BASE_SEED = 250107535
GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1

# purpose ids: keep stable, they define every stream
P_PRIME, P_VEC_A, P_VEC_B, P_VEC_C, P_SCALAR, P_JOBS, P_MLP = 1, 2, 3, 4, 5, 6, 7


def mix64(z: int) -> int:
    """SplitMix64 finaliser on a Python int (mod 2**64)."""
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def stream_key(*ids: int) -> int:
    """Key of the stream named by a tuple of small integers, rooted at BASE_SEED."""
    s = BASE_SEED
    for i in ids:
        s = mix64(s + ((int(i) + 1) * GAMMA))
    return s


def _sm64_chunk(key: np.uint64, idx: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = key + (idx + np.uint64(1)) * np.uint64(GAMMA)
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


_POOL = None


def _pool():
    global _POOL
    if _POOL is None:
        from concurrent.futures import ThreadPoolExecutor
        _POOL = ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)))
    return _POOL


def splitmix64_at(key: int, idx: np.ndarray) -> np.ndarray:
    """Outputs number idx (0-based, any uint64 array) of the stream with this key."""
    idx = np.ascontiguousarray(idx, dtype=np.uint64).reshape(-1)
    k = np.uint64(key)
    chunk = 1 << 20
    if idx.size <= chunk:
        return _sm64_chunk(k, idx)
    out = np.empty_like(idx)
    parts = [(i, min(i + chunk, idx.size)) for i in range(0, idx.size, chunk)]

    def run(p):
        out[p[0]:p[1]] = _sm64_chunk(k, idx[p[0]:p[1]])
    list(_pool().map(run, parts))
    return out


def splitmix64(key: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream with this key (uint64)."""
    return splitmix64_at(key, np.arange(start, start + count, dtype=np.uint64))


def splitmix64_scalar(key: int, i: int) -> int:
    """Output i of the stream (Python int), for cross-checking the vector form."""
    return mix64(key + (i + 1) * GAMMA)


# ----------------------------------------------------------------------------- primes

SMALL_PRIMES = [p for p in range(2, 200) if all(p % d for d in range(2, int(p ** 0.5) + 1))]
MR_BASES = SMALL_PRIMES[:32]


def is_probable_prime(n: int) -> bool:
    """Trial division by primes < 100, then Miller-Rabin to the first 32 prime bases."""
    if n < 2:
        return False
    for p in SMALL_PRIMES:
        if p >= 100:
            break
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


@dataclass(frozen=True)
class Field:
    """A prime field Z_q for one bit-width class ``lam``."""
    lam: int       # bit-width class (64, 96, ..., 1024)
    q: int         # the prime, bitlen(q) == lam - 4 (lam for a full-width one), 2**32 | q - 1
    z: int         # least quadratic non-residue

    @property
    def limbs(self) -> int:
        return (self.lam + 31) // 32

    @property
    def bits(self) -> int:
        return self.q.bit_length()

    @property
    def two_adicity(self) -> int:
        v, t = 0, self.q - 1
        while t % 2 == 0:
            t //= 2
            v += 1
        return v

    def root(self, n: int) -> int:
        """Primitive n-th root of unity for a power of two n dividing q - 1."""
        if n < 1 or n & (n - 1) or (self.q - 1) % n:
            raise ValueError(f"n={n} is not a power of two dividing q-1")
        return pow(self.z, (self.q - 1) // n, self.q)

    def limbs_of(self, v: int, L: int | None = None) -> np.ndarray:
        L = self.limbs if L is None else L
        return int_to_limbs(v, L)


def find_prime(lam: int, *ids: int, bits: int | None = None) -> Field:
    """Seeded NTT-friendly prime of exactly M = lam-4 bits (or `bits`, e.g. lam
    for a full-width modulus): q = c*2**32 + 1.

    c is drawn with exactly M-32 bits (top bit set), then incremented (wrapping
    inside its range) until q passes Miller-Rabin; the first hit is taken.
    """
    M = lam - 4 if bits is None else bits
    cb = M - 32
    if cb < 2:
        raise ValueError("class too small for c*2**32+1 primes")
    key = stream_key(P_PRIME, lam, *ids) if bits is None else stream_key(P_PRIME, lam, *ids, 1 << 20, M)
    words = (cb + 63) // 64
    r = 0
    for i in range(words):
        r = (r << 64) | splitmix64_scalar(key, i)
    lo, span = 1 << (cb - 1), 1 << (cb - 1)
    c = lo + (r % span)
    for _ in range(1 << 20):
        q = (c << 32) + 1
        if is_probable_prime(q):
            z = 2
            while pow(z, (q - 1) // 2, q) != q - 1:
                z += 1
            return Field(lam=lam, q=q, z=z)
        c += 1
        if c >= lo + span:
            c = lo
    raise RuntimeError("no prime found")


# ----------------------------------------------------------------------------- limbs

def int_to_limbs(v: int, L: int) -> np.ndarray:
    if v < 0 or v >> (32 * L):
        raise ValueError("value does not fit")
    return np.array([(v >> (32 * j)) & 0xFFFFFFFF for j in range(L)], dtype=np.uint32)


def limbs_to_int(a) -> int:
    a = np.asarray(a, dtype=np.uint64)
    v = 0
    for j in range(a.shape[-1] - 1, -1, -1):
        v = (v << 32) | int(a[..., j])
    return v


def rows_to_ints(x: np.ndarray) -> list[int]:
    """(n, L) uint32 element-major limbs -> list of Python ints."""
    x = np.asarray(x, dtype=np.uint32)
    out = [0] * x.shape[0]
    L = x.shape[1]
    acc = np.zeros(x.shape[0], dtype=object)
    for j in range(L - 1, -1, -1):
        acc = acc * (1 << 32) + x[:, j].astype(object)
    out = [int(v) for v in acc]
    return out


def ints_to_rows(vals, L: int) -> np.ndarray:
    vals = list(vals)
    out = np.zeros((len(vals), L), dtype=np.uint32)
    for i, v in enumerate(vals):
        for j in range(L):
            out[i, j] = (v >> (32 * j)) & 0xFFFFFFFF
    return out


def residues(field: Field, n: int, L: int, *ids: int) -> np.ndarray:
    """n uniform residues in [0, q) as (n, L) uint32, element-major.

    Element i, attempt t takes 32-bit words from the stream (ids..., t): word j
    is the low (j even) or high (j odd) half of output i*ceil(Lq/2) + j//2,
    where Lq is the number of limbs of q.  The top limb of q is masked to the
    bit length of q, limbs above it are zero, and attempts >= q are redrawn
    with t + 1.
    """
    if n == 0:
        return np.zeros((0, L), dtype=np.uint32)
    q = field.q
    Lq = (q.bit_length() + 31) // 32
    if Lq > L:
        raise ValueError("q does not fit L limbs")
    ql = int_to_limbs(q, L)
    top_bits = q.bit_length() - 32 * (Lq - 1)
    top_mask = np.uint32((1 << top_bits) - 1) if top_bits < 32 else np.uint32(0xFFFFFFFF)
    half = (Lq + 1) // 2

    def draw(t, rows):
        key = stream_key(*ids, t)
        if rows is None:
            raw = splitmix64(key, 0, n * half)
            m = n
        else:
            idx = rows.astype(np.uint64)[:, None] * np.uint64(half) + np.arange(half, dtype=np.uint64)[None, :]
            raw = splitmix64_at(key, idx)
            m = rows.size
        words = raw.view(np.uint32).reshape(m, 2 * half)   # little-endian: low half first
        cand = np.zeros((m, L), dtype=np.uint32)
        cand[:, :Lq] = words[:, :Lq]
        cand[:, Lq - 1] &= top_mask
        lt = np.zeros(m, dtype=bool)
        eq = np.ones(m, dtype=bool)
        for j in range(Lq - 1, -1, -1):
            col = cand[:, j]
            lt |= eq & (col < ql[j])
            eq &= col == ql[j]
        return cand, lt

    out, ok = draw(0, None)
    todo = np.flatnonzero(~ok)
    t = 1
    while todo.size:
        cand, ok = draw(t, todo)
        out[todo[ok]] = cand[ok]
        todo = todo[~ok]
        t += 1
        if t > 200:
            raise RuntimeError("rejection sampling did not converge")
    return out


def scalar_residue(field: Field, *ids: int) -> int:
    return limbs_to_int(residues(field, 1, field.limbs, *ids)[0])


def to_planar(x: np.ndarray) -> np.ndarray:
    """(n, L) element-major -> (L, n) limb-planar (limb j of element i at j*n + i)."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint32).T)


def from_planar(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint32).T)


def edge_vectors(field: Field, n: int, L: int) -> dict[str, np.ndarray]:
    """Structured inputs: zeros, all q-1, alternating 0/q-1, delta_0, delta_1,
    all ones, full-carry low limbs, and a pair whose sum is exactly q."""
    q = field.q
    qm1 = ints_to_rows([q - 1], L)[0]
    one = ints_to_rows([1], L)[0]
    z = np.zeros((n, L), dtype=np.uint32)
    d = {"zeros": z.copy()}
    d["all_qm1"] = np.tile(qm1, (n, 1))
    alt = z.copy()
    alt[1::2] = qm1
    d["alt_0_qm1"] = alt
    d0 = z.copy(); d0[0] = one; d["delta0"] = d0
    d1 = z.copy()
    if n > 1:
        d1[1] = one
    d["delta1"] = d1
    d["ones"] = np.tile(one, (n, 1))
    # low limbs all-ones (carry runs the whole chain), top part below q
    lowones = (1 << (32 * (L - 1))) - 1 if L > 1 else 0
    v = lowones if lowones < q else q - 2
    d["carry_run"] = np.tile(ints_to_rows([v], L)[0], (n, 1))
    return d


def sum_to_q_pair(field: Field, n: int, L: int, *ids: int) -> tuple[np.ndarray, np.ndarray]:
    """a uniform, b = q - a (with a != 0), so that a + b == q exactly."""
    a = residues(field, n, L, *ids)
    ai = rows_to_ints(a)
    ai = [v if v else 1 for v in ai]
    return ints_to_rows(ai, L), ints_to_rows([field.q - v for v in ai], L)


def log2_exact(n: int) -> int:
    k = int(math.log2(n)) if n > 0 else -1
    if n <= 0 or (1 << k) != n:
        raise ValueError(f"{n} is not a power of two")
    return k


# ----------------------------------------------------------------------------- batched workload

BATCH_WIDTHS = (64, 128, 256, 384)
BATCH_LOGN = tuple(range(10, 17))


@dataclass(frozen=True)
class BatchJob:
    index: int
    lam: int
    logn: int
    field: Field

    @property
    def n(self) -> int:
        return 1 << self.logn

    @property
    def limbs(self) -> int:
        return self.field.limbs

    @property
    def omega(self) -> int:
        return self.field.root(self.n)


def batch_shape(index: int, config: int = 3) -> tuple[int, int]:
    """(bit-width class, log2 n) of job `index`: the class uniform over
    {64, 128, 256, 384} and log2 n uniform over the integers 10..16."""
    r = splitmix64_scalar(stream_key(P_JOBS, config), index)
    lam = BATCH_WIDTHS[(r & 0xFFFF) % len(BATCH_WIDTHS)]
    logn = BATCH_LOGN[((r >> 16) & 0xFFFF) % len(BATCH_LOGN)]
    return lam, logn


def _make_job(args):
    index, config = args
    lam, logn = batch_shape(index, config)
    return BatchJob(index=index, lam=lam, logn=logn, field=find_prime(lam, config, index))


def batch_jobs(count: int, config: int = 3, workers: int | None = None) -> list[BatchJob]:
    """`count` jobs of the batched workload, each with its own seeded prime."""
    work = [(i, config) for i in range(count)]
    if count < 64:
        return [_make_job(w) for w in work]
    from concurrent.futures import ProcessPoolExecutor
    nw = workers or max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=nw) as ex:
        return list(ex.map(_make_job, work, chunksize=32))


def batch_inputs(jobs: list[BatchJob], config: int = 3) -> list[np.ndarray]:
    """Uniform residues for each job, element-major (n, L)."""
    return [residues(j.field, j.n, j.limbs, config, 1000 + j.index) for j in jobs]


# ----------------------------------------------------------------------------- cost-model inputs

MLP_IN, MLP_H = 7, 64
MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def mlp_init(seed: int) -> np.ndarray:
    """He-normal initial weights (N(0, 2/fan_in)), zero biases, flat float64 in the
    layout W1[64][7], b1, W2[64][64], b2, W3[64], b3.  Normal draws come from
    SplitMix64 by the Box-Muller transform: u = (top 53 bits + 1) / 2^53,
    z = sqrt(-2 ln u1) cos(2 pi u2)."""
    sizes = [(MLP_H * MLP_IN, MLP_IN), (MLP_H, 0), (MLP_H * MLP_H, MLP_H), (MLP_H, 0), (MLP_H, MLP_H), (1, 0)]
    out = []
    key = stream_key(P_MLP, seed)
    pos = 0
    for count, fan_in in sizes:
        if fan_in == 0:
            out.append(np.zeros(count))
            continue
        r = splitmix64(key, pos, 2 * count)
        pos += 2 * count
        u = ((r >> np.uint64(11)).astype(np.float64) + 1.0) / 2.0 ** 53
        z = np.sqrt(-2.0 * np.log(u[0::2])) * np.cos(2.0 * np.pi * u[1::2])
        out.append(z * np.sqrt(2.0 / fan_in))
    return np.concatenate(out)


def uniform01(n: int, *ids: int) -> np.ndarray:
    """n doubles uniform in (0, 1] from the stream ids (53-bit resolution)."""
    r = splitmix64(stream_key(*ids), 0, n)
    return ((r >> np.uint64(11)).astype(np.float64) + 1.0) / 2.0 ** 53
