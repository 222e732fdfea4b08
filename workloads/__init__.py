"""Seeded synthetic workloads.

Only random input generation lives here (no compression arithmetic), so both
the HIP path's tests and the CPU oracle can draw the same bytes from it.  Every
generator is keyed by (config seed, block index) through numpy's PCG64 with a
SeedSequence, so a block's bytes do not depend on how many other blocks are
drawn.

Sources (the paper has no datasets; these stand in for the workloads the
method is aimed at):

* ``uniform``  -- i.i.d. bytes 0..255 (incompressible).
* ``text``     -- order-3 Markov chain over 27 symbols ('a'..'z', ' '); every
                  context owns a seeded permutation of the alphabet and the
                  next symbol is the permutation entry at a Zipf(1.1) rank.
* ``sparse``   -- each byte is 0 with probability 0.95, else uniform 1..255.
* ``markov64`` -- order-2 Markov chain over the 64 bytes 0x20..0x5F, same
                  construction.
* ``periodic`` -- a block of p uniform bytes (p log-uniform in 1..4096) tiled
                  to the block length, then 0.01% of the positions XORed with a
                  uniform nonzero byte.
* ``same``     -- one uniform byte repeated.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

MIB = 1 << 20
LEVEL9_BLOCK = 900_000
SOURCES = ("uniform", "text", "sparse")


def rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def zipf_ranks(g: np.random.Generator, size: int, k: int, s: float = 1.1) -> np.ndarray:
    """0-based ranks r with P(r) proportional to (r+1)^-s, r < k."""
    w = np.arange(1, k + 1, dtype=np.float64) ** -s
    cdf = np.cumsum(w) / w.sum()
    cdf[-1] = 1.0
    return np.minimum(np.searchsorted(cdf, g.random(size), side="right"), k - 1)


_walk = None


def build() -> str:
    """Compiles markov_walk.c (the Markov sources' sampling loop) with gcc."""
    import os, subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    src, lib = os.path.join(here, "markov_walk.c"), os.path.join(here, "libmarkov_walk.so")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", src, "-o", lib + ".tmp"])
    os.replace(lib + ".tmp", lib)
    return lib


def _walk_lib():
    """The recurrence in C (markov_walk.c; compiled by build(), or here on
    first use if it is missing or stale); None when no compiler is available
    (the numpy walk below gives identical bytes)."""
    global _walk
    if _walk is None:
        import ctypes, os, subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        src, lib = os.path.join(here, "markov_walk.c"), os.path.join(here, "libmarkov_walk.so")
        try:
            if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
                subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", src, "-o", lib + ".tmp"])
                os.replace(lib + ".tmp", lib)
            L = ctypes.CDLL(lib)
            L.markov_walk.restype = None
            L.markov_walk.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
            _walk = L
        except Exception:
            _walk = False
    return _walk or None


def _markov(lengths: Sequence[int], gens: Sequence[np.random.Generator], alphabet: np.ndarray,
            order: int, table_gen: np.random.Generator) -> List[np.ndarray]:
    """Independent order-`order` chains, one per block."""
    k = alphabet.size
    perms = np.ascontiguousarray(
        table_gen.permuted(np.tile(np.arange(k, dtype=np.int64), (k ** order, 1)), axis=1))
    lib = _walk_lib()

    def one(g, n):
        n = int(n)
        sym = np.zeros(n, dtype=np.uint8)
        start = g.integers(0, k, size=min(order, n))
        sym[:start.size] = start
        ranks = np.ascontiguousarray(zipf_ranks(g, max(n - order, 0), k).astype(np.uint8))
        if lib is not None:
            lib.markov_walk(n, order, k, perms.ctypes.data, ranks.ctypes.data, sym.ctypes.data)
        else:
            kk = k ** order
            ctx = 0
            for t in range(min(order, n)):
                ctx = (ctx * k + int(sym[t])) % kk
            pf = perms.ravel().tolist()
            rl = ranks.tolist()
            sl = sym.tolist()
            for t in range(order, n):
                x = pf[ctx * k + rl[t - order]]
                sl[t] = x
                ctx = (ctx * k + x) % kk
            sym = np.asarray(sl, dtype=np.uint8)
        return alphabet[sym].astype(np.uint8)

    return _pmap(one, gens, lengths)


TEXT_ALPHABET = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz ", dtype=np.uint8)
M64_ALPHABET = np.arange(0x20, 0x60, dtype=np.uint8)


def _pmap(fn, gens, lengths) -> List[np.ndarray]:
    """fn(gen, n) for every block, over a few threads (numpy's generators and
    the C walk release the GIL; each block has its own generator, so the
    bytes do not depend on the scheduling)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    items = list(zip(gens, lengths))
    workers = min(16, os.cpu_count() or 1)
    if len(items) < 8 or workers == 1:
        return [fn(g, n) for g, n in items]
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda a: fn(*a), items))


def source_blocks(kind: str, lengths: Sequence[int], seed: int, first_index: int = 0,
                  indices: Sequence[int] | None = None) -> List[np.ndarray]:
    """Blocks of one source; block i is seeded by (seed, index_i)."""
    idx = list(indices) if indices is not None else [first_index + i for i in range(len(lengths))]
    gens = [rng(seed, i) for i in idx]
    if kind == "uniform":
        return _pmap(lambda g, n: g.integers(0, 256, size=n, dtype=np.uint8), gens, lengths)
    if kind == "sparse":
        def sparse(g, n):
            nz = g.random(n) < 0.05
            v = g.integers(1, 256, size=n, dtype=np.uint8)
            return np.where(nz, v, 0).astype(np.uint8)
        return _pmap(sparse, gens, lengths)
    if kind == "text":
        return _markov(lengths, gens, TEXT_ALPHABET, 3, rng(seed, 1 << 40, 3))
    if kind == "markov64":
        return _markov(lengths, gens, M64_ALPHABET, 2, rng(seed, 1 << 40, 2))
    if kind == "periodic":
        out = []
        for g, n in zip(gens, lengths):
            p = int(min(max(np.floor(np.exp(g.random() * np.log(4097.0))), 1), 4096))
            pat = g.integers(0, 256, size=p, dtype=np.uint8)
            blk = np.resize(pat, n).astype(np.uint8)
            nflip = max(1, round(n * 1e-4)) if n >= 2 else 0
            pos = g.choice(n, size=min(nflip, n), replace=False)
            blk[pos] ^= g.integers(1, 256, size=pos.size, dtype=np.uint8)
            out.append(blk)
        return out
    if kind == "same":
        return [np.full(n, g.integers(0, 256), dtype=np.uint8) for g, n in zip(gens, lengths)]
    raise ValueError(kind)


def balanced_sources(nb: int, seed: int, kinds: Sequence[str] = SOURCES) -> List[str]:
    """Each kind gets nb/len(kinds) blocks (the remainder to the first kinds),
    in a seeded shuffle."""
    base = [kinds[i % len(kinds)] for i in range(nb)]
    perm = rng(seed, 1 << 41).permutation(nb)
    return [base[i] for i in perm]


@dataclass
class Batch:
    """A concatenated batch: data uint8[N] and block offsets uint64[nb+1]."""
    name: str
    data: np.ndarray
    offsets: np.ndarray
    kinds: List[str]

    @property
    def n_blocks(self) -> int:
        return self.offsets.size - 1

    def block(self, k: int) -> np.ndarray:
        return self.data[int(self.offsets[k]):int(self.offsets[k + 1])]


def _assemble(name: str, lengths: Sequence[int], kinds: Sequence[str], seed: int) -> Batch:
    lengths = [int(n) for n in lengths]
    blocks: List[np.ndarray] = [None] * len(lengths)
    for kind in sorted(set(kinds)):
        ids = [i for i, k in enumerate(kinds) if k == kind]
        for i, b in zip(ids, source_blocks(kind, [lengths[i] for i in ids], seed, indices=ids)):
            blocks[i] = b
    offs = np.zeros(len(lengths) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lengths)
    data = np.concatenate(blocks) if blocks else np.zeros(0, np.uint8)
    return Batch(name, data.astype(np.uint8), offs, list(kinds))


def cut(total: int, block: int) -> List[int]:
    return [min(block, total - o) for o in range(0, total, block)]


def config1(n: int = 100_000, seed: int = 1) -> Batch:
    """One level-1 block from the order-2, 64-symbol Markov source."""
    return _assemble("single 100000 B block, order-2 Markov over 64 symbols",
                     [n], ["markov64"], seed)


def config2(total: int = 64 * MIB, block: int = LEVEL9_BLOCK, seed: int = 2) -> Batch:
    """64 MiB in 900,000-byte blocks, sources 1/3 each uniform/text/sparse."""
    lens = cut(total, block)
    return _assemble(f"{total} B in {block} B blocks, uniform/text/sparse thirds",
                     lens, balanced_sources(len(lens), seed), seed)


def config3(nb: int = 256, block: int = LEVEL9_BLOCK, seed: int = 3, n_same: int | None = None) -> Batch:
    """Sort worst case: period-p blocks with 0.01% flips, 1/8 all-same-byte."""
    n_same = nb // 8 if n_same is None else n_same
    kinds = ["periodic"] * (nb - n_same) + ["same"] * n_same
    perm = rng(seed, 1 << 41).permutation(nb)
    kinds = [kinds[i] for i in perm]
    return _assemble(f"{nb} x {block} B periodic / all-same blocks", [block] * nb, kinds, seed)


def config4(nb: int = 8192, lo: int = 1000, hi: int = LEVEL9_BLOCK, seed: int = 4) -> Batch:
    """Uneven batch: sizes log-uniform in [lo, hi], sources as config 2."""
    g = rng(seed, 1 << 42)
    lens = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=nb))).astype(np.int64)
    return _assemble(f"{nb} blocks log-uniform {lo}..{hi} B", lens.tolist(),
                     balanced_sources(nb, seed), seed)


@dataclass
class Request:
    arrival_s: float
    data: np.ndarray
    kind: str


def requests(n: int, qps: float, lo: int = 4000, hi: int = 64_000_000, seed: int = 5) -> List[Request]:
    """Poisson arrivals (exponential gaps) of log-uniform sized requests, one
    source per request."""
    g = rng(seed, 1 << 43)
    gaps = g.exponential(1.0 / qps, size=n)
    sizes = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=n))).astype(np.int64)
    kinds = balanced_sources(n, seed)
    t = np.cumsum(gaps)
    out = []
    for i in range(n):
        (blk,) = source_blocks(kinds[i], [int(sizes[i])], seed + 1000, indices=[i])
        out.append(Request(float(t[i]), blk, kinds[i]))
    return out
