"""Seeded regular LDPC parity-check matrices (inputs to the decoder).

The paper evaluates MacKay's regular codes (PEGReg504x1008, 4000.2000.4.244,
4376.282.4.9598; Sec. IV-A).  Those files are not available here, so the
workloads use seeded stand-ins of the same kind: regular (d_v, d_c) codes
built by a random socket permutation, then repaired until the Tanner graph
has no repeated edge and no 4-cycle (no two bits share two checks).

H is returned in CSR form: row i lists N(i), the bits checked by check i
(Sec. III-A notation), with column indices ascending.  Construction draws
from numpy's PCG64 generator seeded with ``seed``; on failure to repair
within a step budget it restarts with ``seed + 1``.  Nothing here is part of
the decoder's arithmetic.
"""
from __future__ import annotations

import dataclasses
import functools
import hashlib
from typing import Dict, List, Optional, Set, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class LdpcCode:
    """A binary m x n parity-check matrix in CSR form (rows = checks)."""

    name: str
    n: int
    m: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    seed: int

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def k_info(self) -> int:
        """Information bits K = n - m (design rate R = 1 - m/n, Sec. IV-A)."""
        return self.n - self.m

    @property
    def rate(self) -> float:
        return 1.0 - self.m / self.n

    def rows(self) -> List[np.ndarray]:
        return [self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]] for i in range(self.m)]

    def dense(self) -> np.ndarray:
        """Dense uint8 H (m x n); for small codes and tests."""
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        for i in range(self.m):
            h[i, self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]] = 1
        return h

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64([self.n, self.m]).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col_idx, dtype=np.int32).tobytes())
        return h.hexdigest()[:16]


def from_rows(name: str, n: int, rows: List[List[int]], seed: int = -1) -> LdpcCode:
    """Build an LdpcCode from explicit check rows (each a list of bit indices)."""
    m = len(rows)
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    cols: List[int] = []
    for i, r in enumerate(rows):
        r = sorted(int(c) for c in r)
        cols.extend(r)
        row_ptr[i + 1] = len(cols)
    return LdpcCode(name, n, m, row_ptr, np.asarray(cols, dtype=np.int32), seed)


def _conflicts_of(b: int, bit_checks: List[List[int]], check_bits: List[List[int]],
                  girth6: bool = True) -> int:
    """Repeated edges of bit b plus 4-cycles through b (other bits sharing >= 2 checks)."""
    cs = bit_checks[b]
    score = len(cs) - len(set(cs))
    if not girth6:
        return score
    seen: Dict[int, int] = {}
    for c in set(cs):
        for b2 in check_bits[c]:
            if b2 != b:
                seen[b2] = seen.get(b2, 0) + 1
    for v in seen.values():
        score += v * (v - 1) // 2
    return score


def _try_build(n: int, dv: int, dc: int, seed: int, max_steps: int,
               girth6: bool = True) -> Optional[List[List[int]]]:
    """Random socket matching, one bit at a time in a random order.

    Each of a bit's d_v sockets is joined to a free check socket drawn
    uniformly among the checks that would not close a 4-cycle (a check that
    holds a bit already sharing a check with this bit).  When no such check
    is left, any free socket is taken and the conflict is repaired afterwards
    by swapping check endpoints between edges."""
    m = n * dv // dc
    rng = np.random.Generator(np.random.PCG64(seed))
    free = np.full(m, dc, dtype=np.int64)
    bit_checks: List[List[int]] = [[] for _ in range(n)]
    check_bits: List[List[int]] = [[] for _ in range(m)]
    for b in rng.permutation(n):
        b = int(b)
        blocked = np.zeros(m, dtype=bool)
        for _ in range(dv):
            avail = (free > 0) & ~blocked
            if not avail.any():
                avail = free > 0
                avail[bit_checks[b]] = False
                if not avail.any():
                    avail = free > 0
            cand = np.nonzero(avail)[0]
            weights = free[cand].astype(np.float64)
            c = int(cand[rng.choice(len(cand), p=weights / weights.sum())])
            bit_checks[b].append(c)
            check_bits[c].append(b)
            free[c] -= 1
            if girth6:
                for b2 in check_bits[c]:
                    blocked[bit_checks[b2]] = True
            else:
                blocked[c] = True
    # repair leftovers: swap the check of an offending edge with a random edge
    score = lambda bb: _conflicts_of(bb, bit_checks, check_bits, girth6)  # noqa: E731
    bad = {b for b in range(n) if score(b)}
    steps = 0
    while bad:
        b = min(bad)
        sb = score(b)
        if sb == 0:
            bad.discard(b)
            continue
        steps += 1
        if steps > max_steps:
            return None
        slot, b2, slot2 = int(rng.integers(dv)), int(rng.integers(n)), int(rng.integers(dv))
        c, c2 = bit_checks[b][slot], bit_checks[b2][slot2]
        if b2 == b or c == c2:
            continue
        before = sb + score(b2)
        check_bits[c].remove(b); check_bits[c2].remove(b2)
        check_bits[c].append(b2); check_bits[c2].append(b)
        bit_checks[b][slot], bit_checks[b2][slot2] = c2, c
        after_b = score(b)
        after_b2 = score(b2)
        if after_b + after_b2 < before or (after_b + after_b2 == before and rng.random() < 0.05):
            if after_b2:
                bad.add(b2)
            for cc in (c, c2):  # bits that lost a partner may now be clean
                for b3 in check_bits[cc]:
                    if b3 not in bad and score(b3):
                        bad.add(b3)
            continue
        check_bits[c].remove(b2); check_bits[c2].remove(b)
        check_bits[c].append(b); check_bits[c2].append(b2)
        bit_checks[b][slot], bit_checks[b2][slot2] = c, c2
    rows: List[List[int]] = [sorted(r) for r in check_bits]
    # final global check, independent of the incremental bookkeeping
    if any(len(r) != dc or len(set(r)) != dc for r in rows):
        return None
    if girth6 and not _girth_at_least_6(n, rows):
        return None
    return rows


def _girth_at_least_6(n: int, rows: List[List[int]]) -> bool:
    """True iff no row repeats a bit and no two rows share two bits."""
    seen: Set[Tuple[int, int]] = set()
    for r in rows:
        if len(set(r)) != len(r):
            return False
        for a in range(len(r)):
            for b in range(a + 1, len(r)):
                key = (r[a], r[b])
                if key in seen:
                    return False
                seen.add(key)
    return True


@functools.lru_cache(maxsize=None)
def regular_code(n: int, dv: int, dc: int, seed: int, name: str = "",
                 girth6: bool = True) -> LdpcCode:
    """Regular (dv, dc) LDPC code of length n from ``seed``: no repeated edge,
    and (girth6) no 4-cycle."""
    if (n * dv) % dc:
        raise ValueError("n * dv must be a multiple of dc")
    s = seed
    for _ in range(64):
        rows = _try_build(n, dv, dc, s, max_steps=400 * n, girth6=girth6)
        if rows is not None:
            return from_rows(name or f"reg{dv}{dc}_{n}", n, rows, seed=s)
        s += 1
    raise RuntimeError("code construction did not converge")


# The four seeded codes of the workloads: (name, n, dv, dc, seed).
CODE_TABLE = {
    "C96": (96, 3, 6, 96),
    "C1008": (1008, 3, 6, 1008),
    "C2048": (2048, 6, 32, 2048),
    "C4000": (4000, 3, 6, 4000),
}


def named_code(name: str) -> LdpcCode:
    n, dv, dc, seed = CODE_TABLE[name]
    return regular_code(n, dv, dc, seed, name)
