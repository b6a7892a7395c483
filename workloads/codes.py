"""Seeded parity-check matrices for the decoder's synthetic workloads.

A code is the sparse m x n matrix H of Section II: H[i, j] = 1 joins check
node i to variable node j of the Tanner graph.  Everything here builds inputs
(matrices and their structure reports); nothing decodes.

Constructions
-------------
* ``gallager_regular``  random (dv, dc)-regular code, Gallager's three-block
  construction, then seeded degree-preserving edge swaps until no 4-cycle is
  left.
* ``qc_base`` / ``qc_code``  quasi-cyclic code: an mb x nb base matrix of
  circulant shifts in [0, Z) with exactly round(frac * mb * nb) empty blocks,
  lifted by Z.  Block (i, j) with shift s joins row i*Z + r to column
  j*Z + (r + s) mod Z.
* ``staircase_irregular``  rate-1/2 irregular code with a dual-diagonal parity
  part (variable degrees 8 / 3 / 2 on 1/5, 3/10, 1/2 of the columns), check
  degree 7 (one row of degree 6), no 4-cycles.
* ``qc_row_degrees`` / ``random_rows``  codes with chosen row degrees (QC
  with given block-row degrees; CSR with degrees drawn from a range and
  optionally one dense column), for covering every kernel body size.
* small fixtures: single parity check, repetition chain, Hamming(7,4),
  random cycle-free Tanner graphs.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Code:
    m: int
    n: int
    row_ptr: np.ndarray  # int32, m + 1
    col_idx: np.ndarray  # int32, nnz; columns strictly increasing within a row
    name: str = ""
    qc: Optional[dict] = None  # {"mb","nb","Z","shifts"(int32 mb x nb, -1 = empty)}

    @property
    def edges(self) -> int:
        return int(self.row_ptr[-1])

    @staticmethod
    def from_dense(H: np.ndarray, name: str = "", qc=None) -> "Code":
        H = np.asarray(H, dtype=np.uint8)
        m, n = H.shape
        rows, cols = np.nonzero(H)
        row_ptr = np.zeros(m + 1, dtype=np.int32)
        np.add.at(row_ptr, rows + 1, 1)
        row_ptr = np.cumsum(row_ptr).astype(np.int32)
        return Code(m, n, row_ptr, cols.astype(np.int32), name, qc)

    @staticmethod
    def from_row_lists(m: int, n: int, row_lists, name: str = "") -> "Code":
        row_ptr = np.zeros(m + 1, dtype=np.int32)
        cols = []
        for i, lst in enumerate(row_lists):
            s = sorted(lst)
            assert len(set(s)) == len(s), "duplicate edge"
            cols.extend(s)
            row_ptr[i + 1] = row_ptr[i] + len(s)
        return Code(m, n, row_ptr, np.asarray(cols, dtype=np.int32), name)

    def to_dense(self) -> np.ndarray:
        H = np.zeros((self.m, self.n), dtype=np.uint8)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        H[rows, self.col_idx] = 1
        return H

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def col_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.n)


# --------------------------------------------------------------------------
# 4-cycle bookkeeping and repair (degree preserving edge swaps)
# --------------------------------------------------------------------------

def count_4cycles(code: Code) -> int:
    """Number of column pairs sharing >= 2 rows, counted per shared row pair."""
    cols_rows = [[] for _ in range(code.n)]
    for i in range(code.m):
        for c in code.col_idx[code.row_ptr[i]:code.row_ptr[i + 1]]:
            cols_rows[c].append(i)
    seen = {}
    total = 0
    m = code.m
    for rows in cols_rows:
        rows = sorted(rows)
        for a in range(len(rows)):
            for b in range(a + 1, len(rows)):
                key = rows[a] * m + rows[b]
                k = seen.get(key, 0)
                total += k
                seen[key] = k + 1
    return total


class _PairRepair:
    """Seeded edge-swap repair: removes duplicate edges, 4-cycles and forbidden
    row pairs from the movable columns while keeping every row and column degree."""

    def __init__(self, m, col_rows, movable, forbidden_adjacent, rng, fixed_pairs=()):
        self.m = m
        self.col_rows = col_rows          # list of lists (rows of each column)
        self.movable = movable            # list of movable column ids
        self.adj = forbidden_adjacent     # forbid pairs (i, i+1)
        self.rng = rng
        self.cnt = {}
        for rows in col_rows:
            for key in self._pairs(rows):
                self.cnt[key] = self.cnt.get(key, 0) + 1
        for key in fixed_pairs:
            self.cnt[key] = self.cnt.get(key, 0) + 1

    def _key(self, a, b):
        return a * self.m + b if a < b else b * self.m + a

    def _pairs(self, rows):
        out = []
        for a in range(len(rows)):
            for b in range(a + 1, len(rows)):
                if rows[a] != rows[b]:
                    out.append(self._key(rows[a], rows[b]))
        return out

    def _bad_pair(self, a, b):
        return a == b or (self.adj and abs(a - b) == 1)

    def edge_bad(self, c, i):
        rows = self.col_rows[c]
        r = rows[i]
        for j, x in enumerate(rows):
            if j == i:
                continue
            if self._bad_pair(r, x) or self.cnt.get(self._key(r, x), 0) > 1:
                return True
        return False

    def try_swap(self, c1, i1, c2, i2):
        R1, R2 = self.col_rows[c1], self.col_rows[c2]
        r1, r2 = R1[i1], R2[i2]
        if r1 == r2:
            return False
        o1 = R1[:i1] + R1[i1 + 1:]
        o2 = R2[:i2] + R2[i2 + 1:]
        if r2 in o1 or r1 in o2:
            return False
        for x in o1:
            if self._bad_pair(r2, x):
                return False
        for y in o2:
            if self._bad_pair(r1, y):
                return False
        for x in o1:
            if x != r1:
                self.cnt[self._key(r1, x)] -= 1
        for y in o2:
            if y != r2:
                self.cnt[self._key(r2, y)] -= 1
        added = []
        ok = True
        for x in o1:
            k = self._key(r2, x)
            if self.cnt.get(k, 0) != 0:
                ok = False
                break
            self.cnt[k] = 1
            added.append(k)
        if ok:
            for y in o2:
                k = self._key(r1, y)
                if self.cnt.get(k, 0) != 0:
                    ok = False
                    break
                self.cnt[k] = 1
                added.append(k)
        if not ok:
            for k in added:
                self.cnt[k] -= 1
            for x in o1:
                if x != r1:
                    self.cnt[self._key(r1, x)] += 1
            for y in o2:
                if y != r2:
                    self.cnt[self._key(r2, y)] += 1
            return False
        R1[i1] = r2
        R2[i2] = r1
        return True

    def bad_edges(self):
        out = []
        for c in self.movable:
            for i in range(len(self.col_rows[c])):
                if self.edge_bad(c, i):
                    out.append((c, i))
        return out

    def run(self, max_rounds=50):
        mov = np.asarray(self.movable)
        for _ in range(max_rounds):
            bad = self.bad_edges()
            if not bad:
                return
            order = self.rng.permutation(len(bad))
            for t in order:
                c1, i1 = bad[t]
                if not self.edge_bad(c1, i1):
                    continue
                for _attempt in range(2000):
                    c2 = int(mov[self.rng.integers(len(mov))])
                    if c2 == c1:
                        continue
                    i2 = int(self.rng.integers(len(self.col_rows[c2])))
                    if self.try_swap(c1, i1, c2, i2):
                        break
        if self.bad_edges():
            raise RuntimeError("4-cycle repair did not converge")


def _code_from_col_rows(m, n, col_rows, name):
    row_lists = [[] for _ in range(m)]
    for c, rows in enumerate(col_rows):
        for r in rows:
            row_lists[r].append(c)
    return Code.from_row_lists(m, n, row_lists, name)


def gallager_regular(n: int, dv: int, dc: int, seed: int) -> Code:
    """Random (dv, dc)-regular code without 4-cycles (Gallager's construction + swaps)."""
    assert n % dc == 0
    mblk = n // dc
    m = mblk * dv
    rng = np.random.Generator(np.random.PCG64(seed))
    col_rows = [[] for _ in range(n)]
    for b in range(dv):
        perm = np.arange(n) if b == 0 else rng.permutation(n)
        for pos, c in enumerate(perm):
            col_rows[int(c)].append(b * mblk + pos // dc)
    rep = _PairRepair(m, col_rows, list(range(n)), False, rng)
    rep.run()
    return _code_from_col_rows(m, n, col_rows, f"gallager({dv},{dc}) n={n} seed={seed}")


def qc_base(mb: int, nb: int, Z: int, empty_frac: float, seed: int) -> np.ndarray:
    """Base matrix of shifts (int32, -1 = empty block): exactly round(frac*mb*nb)
    empty positions chosen uniformly, shifts uniform in [0, Z); redrawn until
    no base row or column is empty."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_empty = int(round(empty_frac * mb * nb))
    while True:
        shifts = rng.integers(0, Z, size=(mb, nb)).astype(np.int32)
        empty = rng.choice(mb * nb, size=n_empty, replace=False)
        shifts.reshape(-1)[empty] = -1
        filled = shifts >= 0
        if filled.any(axis=0).all() and filled.any(axis=1).all():
            return shifts


def qc_expand(shifts: np.ndarray, Z: int, name: str = "") -> Code:
    shifts = np.asarray(shifts, dtype=np.int32)
    mb, nb = shifts.shape
    m, n = mb * Z, nb * Z
    row_lists = []
    for i in range(mb):
        for r in range(Z):
            row_lists.append([j * Z + (r + int(shifts[i, j])) % Z
                              for j in range(nb) if shifts[i, j] >= 0])
    code = Code.from_row_lists(m, n, row_lists, name)
    code.qc = {"mb": mb, "nb": nb, "Z": Z, "shifts": shifts.copy()}
    return code


def qc_code(mb: int, nb: int, Z: int, seed: int, empty_frac: float = 0.3) -> Code:
    s = qc_base(mb, nb, Z, empty_frac, seed)
    return qc_expand(s, Z, f"qc {mb}x{nb} Z={Z} seed={seed}")


def qc_row_degrees(degrees, nb: int, Z: int, seed: int) -> Code:
    """QC code whose block-row i has exactly degrees[i] non-empty blocks (at
    distinct base columns drawn uniformly), shifts uniform in [0, Z): a code
    with chosen row degrees, e.g. a dense block-row.  Redrawn until no base
    column is empty."""
    rng = np.random.Generator(np.random.PCG64(seed))
    assert all(1 <= d <= nb for d in degrees)
    for _ in range(1000):
        s = -np.ones((len(degrees), nb), dtype=np.int32)
        for i, d in enumerate(degrees):
            cols = rng.choice(nb, size=d, replace=False)
            s[i, cols] = rng.integers(0, Z, size=d)
        if (s >= 0).any(axis=0).all():
            return qc_expand(s, Z, f"qc rows {list(degrees)} nb={nb} Z={Z} seed={seed}")
    raise ValueError("block-row degrees leave a base column empty in every draw")


def random_rows(m: int, n: int, dmin: int, dmax: int, seed: int, dense_col: bool = False) -> Code:
    """Irregular code (CSR only): row i joins d_i ~ U{dmin..dmax} distinct
    columns; with dense_col, column 0 is in every row (a column of degree m).
    The other columns are dealt from a sequence of shuffled decks (each a
    seeded permutation of them), so every column is used once before any is
    used twice; a column already in the row is skipped for the next one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    first = 1 if dense_col else 0
    degrees = rng.integers(dmin, dmax + 1, size=m)
    assert dmax <= n and int(degrees.sum()) - first * m >= n - first, "too few edges to cover every column"
    deck: list = []
    rows = []
    for d in degrees:
        row = [0] if dense_col else []
        while len(row) < d:
            if not deck:
                deck = (first + rng.permutation(n - first)).tolist()
            c = deck.pop()
            if c in row:
                deck.insert(0, c)
                continue
            row.append(c)
        rows.append(sorted(row))
    return Code.from_row_lists(m, n, rows, f"random rows {dmin}-{dmax} m={m} n={n} seed={seed}")


def staircase_irregular(n: int, seed: int) -> Code:
    """Rate-1/2 irregular code: info columns of degree 8 (n/5 of all columns) and
    3 (3n/10), parity part a dual diagonal (column i joins rows i and i+1, the
    last column only row m-1).  Every row gets exactly 5 info edges, so check
    degrees are 7 except row 0 (6).  Seeded socket matching, then swaps remove
    duplicate edges, 4-cycles among info columns and info columns touching two
    adjacent rows (which would close a 4-cycle with a staircase column)."""
    assert n % 10 == 0
    m = n // 2
    n8, n3 = n // 5, 3 * n // 10
    k = n8 + n3
    assert k == m
    rng = np.random.Generator(np.random.PCG64(seed))
    degs = np.concatenate([np.full(n8, 8), np.full(n3, 3)])
    assert int(degs.sum()) == 5 * m
    sockets = np.repeat(np.arange(m), 5)
    sockets = sockets[rng.permutation(sockets.size)]
    col_rows = []
    pos = 0
    for d in degs:
        col_rows.append([int(x) for x in sockets[pos:pos + d]])
        pos += int(d)
    rep = _PairRepair(m, col_rows, list(range(k)), True, rng)
    rep.run()
    for i in range(m):  # staircase parity columns
        col_rows.append([i, i + 1] if i + 1 < m else [i])
    return _code_from_col_rows(m, n, col_rows, f"staircase irregular n={n} seed={seed}")


def staircase_encode(code: Code, u: np.ndarray) -> np.ndarray:
    """Encode info bits u (F, m) for ``staircase_irregular`` codes: row i gives
    p_i = s_i xor p_{i-1} where s_i is the parity of the row's info bits."""
    m, n = code.m, code.n
    u = np.atleast_2d(np.asarray(u, dtype=np.uint8))
    F = u.shape[0]
    rows = np.repeat(np.arange(m), np.diff(code.row_ptr))
    is_info = code.col_idx < m
    info_cols, info_rows = code.col_idx[is_info], rows[is_info]
    starts = np.searchsorted(info_rows, np.arange(m))  # every row has >= 1 info edge
    s = np.bitwise_xor.reduceat(u[:, info_cols], starts, axis=1)
    p = np.bitwise_xor.accumulate(s, axis=1)
    return np.concatenate([u, p], axis=1)


# --------------------------------------------------------------------------
# small fixtures
# --------------------------------------------------------------------------

def single_parity_check(n: int) -> Code:
    return Code.from_row_lists(1, n, [list(range(n))], f"spc n={n}")


def repetition_chain(n: int) -> Code:
    """n variables, n-1 degree-2 checks x_i + x_{i+1} = 0 (a path graph)."""
    return Code.from_row_lists(n - 1, n, [[i, i + 1] for i in range(n - 1)], f"repetition n={n}")


def hamming74() -> Code:
    """H columns are the seven non-zero 3-bit vectors (column j = binary of j+1)."""
    H = np.array([[((j + 1) >> b) & 1 for j in range(7)] for b in range(3)], dtype=np.uint8)
    return Code.from_dense(H, "hamming(7,4)")


def random_tree_code(nv: int, seed: int) -> Code:
    """Random connected cycle-free Tanner graph on nv variables; every check has
    degree >= 2.  Grown by hanging a new check (with 1-3 new variables) off a
    random existing variable, or adding a new variable to a random check."""
    rng = np.random.Generator(np.random.PCG64(seed))
    checks = []
    nvars = 1
    while nvars < nv:
        if checks and rng.random() < 0.3:
            checks[int(rng.integers(len(checks)))].append(nvars)
            nvars += 1
        else:
            v = int(rng.integers(nvars))
            kk = int(min(rng.integers(1, 4), nv - nvars))
            checks.append([v] + list(range(nvars, nvars + kk)))
            nvars += kk
    perm = rng.permutation(nv)  # relabel so leaves are not all at the end
    rows = [[int(perm[c]) for c in ch] for ch in checks]
    return Code.from_row_lists(len(rows), nv, rows, f"tree nv={nv} seed={seed}")


def tanner_vn_diameter(code: Code) -> int:
    """Largest variable-to-variable distance, counted in Tanner-graph edges."""
    H = code.to_dense()
    adj_v = [np.flatnonzero(H[:, j]) for j in range(code.n)]
    adj_c = [np.flatnonzero(H[i]) for i in range(code.m)]
    best = 0
    for s in range(code.n):
        dist = {("v", s): 0}
        frontier = [("v", s)]
        while frontier:
            nxt = []
            for kind, x in frontier:
                d = dist[(kind, x)]
                nbrs = adj_v[x] if kind == "v" else adj_c[x]
                nk = "c" if kind == "v" else "v"
                for y in nbrs:
                    key = (nk, int(y))
                    if key not in dist:
                        dist[key] = d + 1
                        nxt.append(key)
            frontier = nxt
        best = max(best, max(d for (k, _), d in dist.items() if k == "v"))
    return best
