"""GF(2) linear algebra for tests: codewords of H by elimination, dense H c."""
import numpy as np


def nullspace_basis(h: np.ndarray) -> np.ndarray:
    """Rows spanning {c : H c = 0 over GF(2)} (uint8 [k, n])."""
    a = (h.copy() % 2).astype(np.uint8)
    m, n = a.shape
    pivots = []
    r = 0
    for c in range(n):
        if r == m:
            break
        rows = np.nonzero(a[r:, c])[0]
        if len(rows) == 0:
            continue
        p = r + rows[0]
        a[[r, p]] = a[[p, r]]
        for i in range(m):
            if i != r and a[i, c]:
                a[i] ^= a[r]
        pivots.append(c)
        r += 1
    free = [c for c in range(n) if c not in pivots]
    basis = []
    for f in free:
        v = np.zeros(n, dtype=np.uint8)
        v[f] = 1
        for i, pc in enumerate(pivots):
            v[pc] = a[i, f]
        basis.append(v)
    return np.array(basis, dtype=np.uint8).reshape(len(basis), n)


def random_codewords(h: np.ndarray, count: int, seed: int) -> np.ndarray:
    basis = nullspace_basis(h)
    rng = np.random.Generator(np.random.PCG64(seed))
    coef = rng.integers(0, 2, size=(count, basis.shape[0]), dtype=np.uint8)
    return ((coef.astype(np.int64) @ basis.astype(np.int64)) % 2).astype(np.uint8)


def syndrome(h: np.ndarray, c: np.ndarray) -> np.ndarray:
    """H c over GF(2) for each row of c (uint8 [F, m])."""
    return ((c.astype(np.int64) @ h.T.astype(np.int64)) % 2).astype(np.uint8)
