"""Block-level model of the dense leaf's task schedule (16x16 blocks).

The leaf kernel factors an NB x NB block (NB = 64 or 128) and inverts its
Cholesky factor in LDS with 16-column panels and two workgroup barriers per
panel.  This model lists the tasks of every phase exactly as the kernel deals
them out to its waves, with the blocks each task reads and writes, and checks

* that no two tasks of one phase conflict (one writes a block the other reads
  or writes): the waves run them concurrently;
* that running the phases' tasks in any order gives L^-1 of the Cholesky
  factor (up to rounding).

Tasks that one wave runs in sequence (wave 0's panel row and block update,
an inversion column) are one task here.
"""
import itertools
import random

import numpy as np
import pytest


def schedule(P):
    """Phases of the leaf with P panels: a list of lists of tasks; a task is a
    tuple of (op, args) steps.  ops: factor(p), panel(p, i), trail(p, i, j),
    inv_y(p, c), inv_col(p, i, c)."""
    phases = [[(("factor", 0),)]]
    for p in range(P):
        npan = P - 1 - p
        a = []
        if npan > 0:  # wave 0: panel row p + 1, then block (p+1, p+1)
            a.append((("panel", p, p + 1), ("trail", p, p + 1, p + 1)))
        a += [(("panel", p, p + 1 + t),) for t in range(1, npan)]
        if p > 0:  # column p - 1 of the inversion, over L_{i,p-1}
            a.append((("inv_y", p - 1, p - 1),))
            a += [(("inv_col", p - 1, i, p - 1),) for i in range(p, P)]
        phases.append(a)
        look = p + 1 < P
        m = P - 1 - p
        b = [(("factor", p + 1),)] if look else []
        ncol = p if look else p + 1
        for c in range(ncol):
            if c < p:
                b.append((("inv_y", p, c),) + tuple(("inv_col", p, i, c) for i in range(p + 1, P)))
            else:
                b.append((("inv_y", p, p),))
        first = 1 if look else 0
        for t in range(m * (m + 1) // 2 - first):
            jj, rem = 0, t + first
            while rem >= m - jj:
                rem -= m - jj
                jj += 1
            b.append((("trail", p, p + 1 + jj + rem, p + 1 + jj),))
        phases.append(b)
    return phases


def access(step):
    """(reads, writes) of one step: ('b', i, j) blocks, ('D', p) inverses."""
    op, *a = step
    if op == "factor":
        p, = a
        return {("b", p, p)}, {("b", p, p), ("D", p)}
    if op == "panel":
        p, i = a
        return {("b", i, p), ("D", p)}, {("b", i, p)}
    if op == "trail":
        p, i, j = a
        return {("b", i, p), ("b", j, p), ("b", i, j)}, {("b", i, j)}
    if op == "inv_y":
        p, c = a
        return {("D", p), ("b", p, c)}, {("b", p, c)}
    p, i, c = a  # inv_col
    if c == p:
        return {("b", i, p), ("D", p)}, {("b", i, p)}
    return {("b", i, p), ("b", p, c), ("b", i, c)}, {("b", i, c)}


def run(A, phases, rng):
    P = A.shape[0] // 16
    blk = {(i, j): A[16 * i:16 * i + 16, 16 * j:16 * j + 16].copy()
           for i in range(P) for j in range(P) if i >= j}
    D = {}
    for ph in phases:
        order = list(ph)
        rng.shuffle(order)
        for task in order:
            for op, *a in task:
                if op == "factor":
                    p, = a
                    L = np.linalg.cholesky(blk[(p, p)])
                    blk[(p, p)] = L
                    D[p] = np.linalg.inv(L)
                elif op == "panel":
                    p, i = a
                    blk[(i, p)] = blk[(i, p)] @ D[p].T
                elif op == "trail":
                    p, i, j = a
                    blk[(i, j)] = blk[(i, j)] - blk[(i, p)] @ blk[(j, p)].T
                elif op == "inv_y":
                    p, c = a
                    blk[(p, c)] = D[p].copy() if c == p else D[p] @ blk[(p, c)]
                else:
                    p, i, c = a
                    blk[(i, c)] = (-(blk[(i, p)] @ D[p]) if c == p
                                   else blk[(i, c)] - blk[(i, p)] @ blk[(p, c)])
    X = np.zeros_like(A)
    for (i, j), b in blk.items():
        X[16 * i:16 * i + 16, 16 * j:16 * j + 16] = b
    return np.tril(X)


@pytest.mark.parametrize("NB", [64, 128])
def test_phases_have_no_conflicts(NB):
    for ph in schedule(NB // 16):
        acc = []
        for task in ph:
            r, w = set(), set()
            for step in task:
                rs, ws = access(step)
                r |= rs
                w |= ws
            acc.append((r, w))
        for (r1, w1), (r2, w2) in itertools.combinations(acc, 2):
            assert not (w1 & (r2 | w2)) and not (w2 & (r1 | w1))


@pytest.mark.parametrize("NB", [64, 128])
def test_schedule_gives_inverse_factor(NB):
    rng = np.random.default_rng(NB)
    B = rng.standard_normal((NB, NB))
    A = B @ B.T / NB + np.eye(NB)
    ref = np.linalg.inv(np.linalg.cholesky(A))
    for seed in range(4):
        X = run(A, schedule(NB // 16), random.Random(seed))
        assert np.abs(X - ref).max() < 1e-12


def test_every_block_of_the_inverse_is_written():
    """Each lower block (p, c) ends as Y(p, c): written by inv_y(p, c)."""
    P = 8
    done = {step[1:] for ph in schedule(P) for task in ph for step in task if step[0] == "inv_y"}
    assert done == {(p, c) for p in range(P) for c in range(p + 1)}


def diag_lanes(S):
    """Lane-level model of the 16 x 16 diagonal step on one wave of 64 lanes,
    lane 16 q + r holding a[k] = A[r][4k + q] (both triangles, read from the
    lower one) and t[k] = T[4k + q][r] of the forward elimination L T = I.
    Column j: the pivot from lane 16 (j % 4) + j; A[r][j] and T[j][r] from
    lane 16 (j % 4) + r (the crossbar); row j at a lane's own columns from
    lane j of its own row of 16 lanes (the DPP broadcast).  Row j of T is
    stored at step j and scaled by the pivot's inverse square root after the
    last column; the registers of final rows and columns keep being updated
    with values that are never read again."""
    lane = np.arange(64)
    r, q = lane & 15, lane >> 4
    a = np.zeros((64, 4))
    t = np.zeros((64, 4))
    for k in range(4):
        c = 4 * k + q
        a[:, k] = S[np.maximum(r, c), np.minimum(r, c)]
        t[:, k] = (c == r)
    T = np.full((16, 16), np.nan)  # rows of T as stored, before their scaling
    pv = np.ones(64)
    for j in range(16):
        kj, qj = j // 4, j % 4
        piv = a[16 * qj + j, kj]
        pv = np.where(r == j, piv, pv)
        src = 16 * qj + r
        col, tj = a[src, kj].copy(), t[src, kj].copy()
        w2, tz = col / piv, tj / piv
        T[j, r] = tj  # every column group stores the same row
        for k in range(kj, 4):
            bc = a[16 * q + j, k].copy()
            a[:, k] -= w2 * bc
            t[:, k] -= tz * bc
    Y = T.copy()
    for k in range(4):  # lane 16 q + r scales row r at its columns 4k + q
        Y[r, 4 * k + q] = T[r, 4 * k + q] / np.sqrt(pv)
    return Y


def test_diagonal_lane_scheme_gives_the_inverse_factor():
    """The lane scheme reads only the lower triangle (the upper one of the
    block in LDS is stale) and stores every entry of L^-1, zeros above the
    diagonal included."""
    rng = np.random.default_rng(7)
    B = rng.standard_normal((16, 16))
    A = B @ B.T + 4 * np.eye(16)
    S = np.tril(A) + np.triu(rng.standard_normal((16, 16)) * 1e3, 1)
    Y = diag_lanes(S)
    ref = np.linalg.inv(np.linalg.cholesky(A))
    assert not np.isnan(Y).any()
    assert np.abs(Y - ref).max() < 1e-13
    assert np.all(np.triu(Y, 1) == 0)


@pytest.mark.parametrize("NB,NT", [(128, 512), (64, 256)])
def test_second_phase_deals_every_trailing_block_once(NB, NT):
    """The kernel's dealing of the second phase: inversion column u to wave
    u (one chain of NPAN - p block products each), the trailing blocks first
    to the waves without a column, up to a column's length each, the rest
    round-robin.  Every block is dealt exactly once, and no wave gets more
    than a column's chain plus its share of the remainder."""
    P, NW = NB // 16, NT // 64
    for p in range(P):
        m = P - 1 - p
        look = p + 1 < P
        nw, first = (NW - 1, 1) if look else (NW, 0)
        ncol = p if look else p + 1
        assert ncol <= nw
        ntrail = m * (m + 1) // 2 - first
        nfree = nw - ncol
        cap = min(ntrail, nfree * (P - p))
        dealt, loads = [], []
        for u in range(nw):
            js = list(range(u - ncol, cap, nfree)) if u >= ncol else []
            js += list(range(cap + u, ntrail, nw))
            dealt += js
            chain = (1 + (m if u < p else 0)) if u < ncol else 0
            loads.append(chain + len(js))
        assert sorted(dealt) == list(range(ntrail))
        rest = max(0, ntrail - cap)
        assert max(loads) <= max(P - p, -(-cap // max(nfree, 1))) + -(-rest // nw)
