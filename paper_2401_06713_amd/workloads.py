"""Seeded synthetic Pauli-string workloads.

This module only draws inputs; it holds none of the colouring method's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

The paper's inputs are molecular Hamiltonians (Jordan-Wigner encoded Pauli
strings, Sec. VII, Table II), which are not available here.  They stand in
as i.i.d. per-position draws from a categorical (pI, pX, pY, pZ): with
pI = 0.7-0.8 this reproduces the paper's ~50% anticommuting density
(density ~ 0.499-0.500 for the configurations below).  Draws use numpy's
PCG64 stream; all-identity strings and duplicates are rejected (the paper
excludes the identity string, Sec. III) and acceptance order is the vertex id.

Layout: x and z are (n, W) uint64 arrays, W = ceil(q/64); qubit k is bit
k % 64 of word k // 64; (x,z) = (0,0) I, (1,0) X, (1,1) Y, (0,1) Z.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def words(q: int) -> int:
    return (q + 63) // 64


def _pack_bits(bits: np.ndarray, q: int) -> np.ndarray:
    """bits (B, q) of {0,1} -> (B, W) uint64 words."""
    B = bits.shape[0]
    W = words(q)
    padded = np.zeros((B, W * 64), dtype=np.uint64)
    padded[:, :q] = bits
    shifts = np.arange(64, dtype=np.uint64)
    return np.bitwise_or.reduce(padded.reshape(B, W, 64) << shifts, axis=2)


def pauli_strings(n: int, q: int, probs=(0.25, 0.25, 0.25, 0.25), seed: int = 0,
                  max_rounds: int = 10000):
    """n distinct non-identity strings on q qubits; returns (x, z)."""
    p = np.asarray(probs, dtype=np.float64)
    if p.shape != (4,) or np.any(p < 0) or abs(p.sum() - 1.0) > 1e-9:
        raise ValueError("probs must be 4 non-negative numbers summing to 1")
    cum = np.cumsum(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    W = words(q)
    xs, zs = [], []
    seen = set()
    got = 0
    rounds = 0
    while got < n:
        rounds += 1
        if rounds > max_rounds:
            raise ValueError(f"could not draw {n} distinct strings on {q} qubits")
        batch = max(1024, int((n - got) * 1.1) + 16)
        u = rng.random((batch, q))
        code = np.searchsorted(cum[:3], u, side="right")  # 0=I 1=X 2=Y 3=Z
        xb = ((code == 1) | (code == 2)).astype(np.uint64)
        zb = ((code == 2) | (code == 3)).astype(np.uint64)
        xw = _pack_bits(xb, q)
        zw = _pack_bits(zb, q)
        nonid = np.any(xw != 0, axis=1) | np.any(zw != 0, axis=1)
        key = np.concatenate([xw, zw], axis=1)
        for i in np.nonzero(nonid)[0]:
            kb = key[i].tobytes()
            if kb in seen:
                continue
            seen.add(kb)
            xs.append(xw[i])
            zs.append(zw[i])
            got += 1
            if got == n:
                break
    if n == 0:
        return np.zeros((0, W), dtype=np.uint64), np.zeros((0, W), dtype=np.uint64)
    return np.stack(xs).astype(np.uint64), np.stack(zs).astype(np.uint64)


def pauli_strings_fast(n: int, q: int, probs, seed: int = 0):
    """Same distribution as pauli_strings for large n: vectorised dedup.

    First occurrences are kept in draw order (np.unique on the packed rows).
    """
    p = np.asarray(probs, dtype=np.float64)
    cum = np.cumsum(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    W = words(q)
    keep_x, keep_z = np.zeros((0, W), np.uint64), np.zeros((0, W), np.uint64)
    rounds = 0
    while keep_x.shape[0] < n:
        rounds += 1
        if rounds > 64:
            raise ValueError(f"could not draw {n} distinct strings on {q} qubits")
        need = n - keep_x.shape[0]
        batch = int(need * 1.02) + 64
        xw = np.zeros((batch, W), np.uint64)
        zw = np.zeros((batch, W), np.uint64)
        chunk = 1 << 16
        for s in range(0, batch, chunk):
            e = min(batch, s + chunk)
            u = rng.random((e - s, q))
            code = np.searchsorted(cum[:3], u, side="right")
            xw[s:e] = _pack_bits(((code == 1) | (code == 2)).astype(np.uint64), q)
            zw[s:e] = _pack_bits(((code == 2) | (code == 3)).astype(np.uint64), q)
        allx = np.concatenate([keep_x, xw])
        allz = np.concatenate([keep_z, zw])
        nonid = np.any(allx != 0, axis=1) | np.any(allz != 0, axis=1)
        key = np.ascontiguousarray(np.concatenate([allx, allz], axis=1))
        kv = key.view(np.dtype((np.void, key.dtype.itemsize * key.shape[1]))).ravel()
        _, first = np.unique(kv, return_index=True)
        first = np.sort(first)
        first = first[nonid[first]]
        keep_x, keep_z = allx[first], allz[first]
    return np.ascontiguousarray(keep_x[:n]), np.ascontiguousarray(keep_z[:n])


def majorana_strings(q: int):
    """The 2q Jordan-Wigner Majorana strings Z..Z {X,Y} I..I (pairwise
    anticommuting: their anticommutation graph is complete)."""
    W = words(q)
    x = np.zeros((2 * q, W), np.uint64)
    z = np.zeros((2 * q, W), np.uint64)
    for j in range(q):
        for t, (xb, zb) in enumerate(((1, 0), (1, 1))):  # X then Y at position j
            r = 2 * j + t
            for k in range(j):  # Z string before j
                z[r, k // 64] |= np.uint64(1) << np.uint64(k % 64)
            x[r, j // 64] |= np.uint64(xb) << np.uint64(j % 64)
            z[r, j // 64] |= np.uint64(zb) << np.uint64(j % 64)
    return x, z


def iz_strings(n: int, q: int, seed: int = 0):
    """n distinct strings over {I, Z} only (pairwise commuting and QWC)."""
    return pauli_strings(n, q, probs=(0.5, 0.0, 0.0, 0.5), seed=seed)


@dataclass(frozen=True)
class Config:
    name: str
    n: int
    q: int
    probs: tuple
    seed: int
    frac: float
    alpha: float
    relation: int  # 0 anticommute, 1 QWC


# The single-instance workloads (iteration-1 sizes in the design notes).
C1 = Config("C1 n=2000 q=16 uniform", 2000, 16, (0.25, 0.25, 0.25, 0.25), 0, 0.125, 2.0, 0)
C2 = Config("C2 n=200000 q=48 pI=0.7", 200_000, 48, (0.7, 0.1, 0.1, 0.1), 0, 0.125, 2.0, 0)
C4 = Config("C4 n=2000000 q=128 pI=0.8", 2_000_000, 128, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3), 0, 0.125, 2.0, 0)
LHELD_PROBS = (0.75, 0.25 / 3, 0.25 / 3, 0.25 / 3)
# The first held-out instance of the learned-parameter evaluation (generator
# and colouring seed 7,000,000), at the fixed parameters.
LHELD0 = Config("L-held[0] n=500000 q=96 pI=0.75", 500_000, 96, LHELD_PROBS, 7_000_000, 0.125, 2.0, 0)


def make(cfg: Config):
    if cfg.n <= 20000:
        return pauli_strings(cfg.n, cfg.q, cfg.probs, cfg.seed)
    return pauli_strings_fast(cfg.n, cfg.q, cfg.probs, cfg.seed)


def batch_instances(count: int = 512, seed: int = 0xB47C):
    """The batched workload: n log-uniform in [500, 50000], q uniform in
    {20..64}, pI uniform in [0.5, 0.85] with X/Y/Z equal, relation
    anticommute or QWC with probability 1/2; instance i uses seed i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(500), math.log(50000)))))
        q = int(rng.integers(20, 65))
        pI = float(rng.uniform(0.5, 0.85))
        rel = int(rng.random() < 0.5)
        r = (1.0 - pI) / 3.0
        out.append(Config(f"batch[{i}]", n, q, (pI, r, r, r), i, 0.125, 2.0, rel))
    return out
