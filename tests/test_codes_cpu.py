"""The seeded codes: regular degrees, no repeated edge, no 4-cycle, and the
same matrix from the same seed."""
import numpy as np
import pytest

from synth import codes


@pytest.mark.parametrize("name", ["C96", "C1008", "C2048", "C4000"])
def test_named_code_structure(name):
    n, dv, dc, seed = codes.CODE_TABLE[name]
    c = codes.named_code(name)
    assert (c.n, c.m) == (n, n * dv // dc) and c.nnz == n * dv
    rows = c.rows()
    assert all(len(r) == dc for r in rows)                  # row weight d_c
    assert all(len(set(r.tolist())) == dc for r in rows)    # no repeated edge
    col = np.bincount(c.col_idx, minlength=n)
    assert (col == dv).all()                                # column weight d_v
    # no 4-cycle: no two bits share two checks
    seen = set()
    for r in rows:
        rl = sorted(r.tolist())
        for a in range(len(rl)):
            for b in range(a + 1, len(rl)):
                pair = (rl[a], rl[b])
                assert pair not in seen, f"4-cycle through bits {pair}"
                seen.add(pair)


def test_construction_is_deterministic():
    a = codes.regular_code(240, 3, 6, seed=5)
    codes.regular_code.cache_clear()
    b = codes.regular_code(240, 3, 6, seed=5)
    assert a.digest() == b.digest()
    c = codes.regular_code(240, 3, 6, seed=6)
    assert c.digest() != a.digest()


def test_rate_convention():
    """Design rate R = 1 - m/n (the paper's rate 0.9356 for 4376.282)."""
    assert abs((1 - 282 / 4376) - 0.9356) < 1e-4
    assert codes.named_code("C2048").rate == 1 - 384 / 2048
