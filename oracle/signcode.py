"""Sign-code coarse pre-selection, CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import or call this module.

What it computes (Sec. 5.3, last paragraph; appendix "Optimizing System on
GPU", Quantization):

* Encoding (OP+ORP-like).  The embedding's coordinates are permuted at
  random, the permuted sequence is cut into equal bins, and each bin gives
  one sample: the sum of its coordinates, each multiplied by a random sign.
  The code keeps one bit per sample, set when the sample is positive.
* Score.  The number of code bits two vectors have in common: per 64-bit
  word, the complement of the XOR of the two words, counted with popcount,
  summed over numBits / 64 words.
* Pre-selection.  Among the documents that pass the term predicate, the
  quantK best by this score survive (quantK = 200 k in the paper), and only
  they are scored exactly; the result is their top k by exact score.

Readings (the paper is silent or leaves the case undefined; the design doc lists
them as well):

* numBits larger than the dimension (512 bits for d = 128): one permutation
  cannot make more bins than coordinates.  The code is then built from
  several independent permutations concatenated, cut into bins of two
  positions each; with numBits <= d / 2 it is the paper's single
  permutation with bins of d / numBits coordinates.  The permutations and
  signs are random inputs drawn by ``datagen.sign_projection`` and passed to
  both sides, as a table: bit j sums positions bin_off[j] .. bin_off[j+1]
  of (bin_dim, bin_sign).
* A bin's sum is evaluated in FP32, adding the signed coordinates in table
  order starting from +0.0; the bit is set iff that FP32 sum is > 0 (the
  library's encoder makes the same FP32 decisions).
* Ties in the quantised score are broken by external id ascending (as for
  exact scores); the exact stage is the plain definition (FP64 dot product of
  the FP32 vectors, top k by (score desc, id asc)).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .core import OracleIndex, OracleResult


def sign_bits(rows: np.ndarray, bin_off: np.ndarray, bin_dim: np.ndarray,
              bin_sign: np.ndarray) -> np.ndarray:
    """Code bits [n, numBits] (bool) of FP32 rows: bit j is set iff the FP32
    sum over bin j of sign * coordinate, added in table order, is > 0."""
    x = np.asarray(rows, dtype=np.float32)
    if x.ndim == 1:
        x = x[None, :]
    n_bits = len(bin_off) - 1
    out = np.zeros((x.shape[0], n_bits), dtype=bool)
    for j in range(n_bits):
        acc = np.zeros(x.shape[0], dtype=np.float32)
        for e in range(int(bin_off[j]), int(bin_off[j + 1])):
            # sign is +-1, so sign * x is exact; each addition rounds to FP32
            acc = (acc + np.float32(bin_sign[e]) * x[:, int(bin_dim[e])]).astype(np.float32)
        out[:, j] = acc > 0
    return out


def pack_words(bits: np.ndarray) -> np.ndarray:
    """Bits [n, numBits] -> uint64 words [n, numBits / 64]; bit b of word w
    is code bit 64 w + b."""
    bits = np.asarray(bits, dtype=bool)
    n, nb = bits.shape
    assert nb % 64 == 0, "numBits must be a multiple of 64"
    by = np.packbits(bits, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8").reshape(n, nb // 64)


def quant_score(x_words: np.ndarray, y_words: np.ndarray) -> np.ndarray:
    """Bits in common: sum over words of popcount(~(x XOR y)).  x_words is
    [n, W] (or [W]), y_words [W]; returns int64 [n]."""
    x = np.atleast_2d(np.asarray(x_words, dtype=np.uint64))
    y = np.asarray(y_words, dtype=np.uint64)
    same = np.bitwise_not(np.bitwise_xor(x, y[None, :]))
    return np.bitwise_count(same).astype(np.int64).sum(axis=1)


class SignCodes:
    """The sign codes of every row of an OracleIndex, for one table."""

    def __init__(self, o: OracleIndex, bin_off, bin_dim, bin_sign):
        self.bin_off = np.asarray(bin_off, dtype=np.int64)
        self.bin_dim = np.asarray(bin_dim, dtype=np.int64)
        self.bin_sign = np.asarray(bin_sign, dtype=np.float32)
        self.n_bits = len(self.bin_off) - 1
        self.o = o
        self.words = pack_words(sign_bits(o.emb, self.bin_off, self.bin_dim, self.bin_sign))

    def refresh(self) -> None:
        """Re-encode after updates of the oracle's rows."""
        self.words = pack_words(sign_bits(self.o.emb, self.bin_off, self.bin_dim,
                                          self.bin_sign))

    def query_words(self, q: np.ndarray) -> np.ndarray:
        return pack_words(sign_bits(q, self.bin_off, self.bin_dim, self.bin_sign))[0]

    def survivors(self, q: np.ndarray, cnf, quant_k: int) -> np.ndarray:
        """Rows kept by the pre-selection: the quant_k best matches by
        (quantised score desc, id asc)."""
        o = self.o
        rows = o.match_rows(cnf)
        qs = quant_score(self.words[rows], self.query_words(q))
        order = np.lexsort((o.ids[rows], -qs))
        return rows[order[:min(int(quant_k), len(rows))]]

    def search_one(self, q: np.ndarray, cnf, k: int, quant_k: int) -> OracleResult:
        """Pre-selection then exact scoring of the survivors: top k by
        (exact score desc, id asc)."""
        o = self.o
        n_match = len(o.match_rows(cnf))
        rows = self.survivors(q, cnf, quant_k)
        s = o.scores(q, rows)
        order = np.lexsort((o.ids[rows], -s))[:min(int(k), len(rows))]
        return OracleResult(o.ids[rows[order]].copy(), s[order].copy(), len(order), n_match)


def brute_search(emb: Sequence[Sequence[float]], ids: Sequence[int],
                 term_sets: Sequence[set], live: Sequence[bool], q, cnf, k: int,
                 quant_k: int, bin_off, bin_dim, bin_sign):
    """Pure-Python reference for tiny inputs (pins the vectorised functions):
    bit by bit encoding with Python floats rounded to FP32 after each
    addition, agreement counted bit by bit, selection by sorting tuples."""
    import math
    import struct

    def f32(v: float) -> float:
        return struct.unpack("<f", struct.pack("<f", v))[0]

    def code(vec):
        bits = []
        for j in range(len(bin_off) - 1):
            acc = 0.0
            for e in range(int(bin_off[j]), int(bin_off[j + 1])):
                acc = f32(acc + float(bin_sign[e]) * float(vec[int(bin_dim[e])]))
            bits.append(acc > 0)
        return bits

    cq = code(q)
    cand = []
    for r in range(len(ids)):
        if not live[r]:
            continue
        if any(not term_sets[r].intersection(c) for c in cnf):
            continue
        agree = sum(1 for a, b in zip(code(emb[r]), cq) if a == b)
        cand.append((-agree, int(ids[r]), r))
    n_match = len(cand)
    cand.sort()
    kept = cand[:quant_k]
    scored = sorted((-math.fsum(float(a) * float(b) for a, b in zip(q, emb[r])), i)
                    for _a, i, r in kept)
    top = scored[:k]
    return [i for _s, i in top], [-s for s, _i in top], n_match
