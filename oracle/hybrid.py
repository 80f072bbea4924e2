"""Oracle of the paper's hybrid matrix layout (Section 3.1): ELL part B with
the value array V, the column array I and the transpose-slot array J, plus a
CRS part C for the entries that do not fit.

TEST INFRASTRUCTURE ONLY: used by the tests and never by the product path.
Plain Python written from the definitions of Section 3.1, in the paper's
row-major notation (row i, slot k); it shares no code with the library.

Readings taken where the section leaves a choice:
* a row holds the diagonal and the row's neighbours in ascending column
  order; its first K entries go to B, the rest (rows longer than K) to C;
* an unused slot of B (a row shorter than K) holds I = i, J = its own slot
  and the value 0, so the row and column sweeps read a harmless zero;
* J[i][k] = k' when the transposed entry (j, i) sits in B at slot k' of row
  j; when it sits in C at position c, J[i][k] = -1 - c (the section only asks
  for a negative value);
* C is stored row-wise: c_start[N + 1], c_col[nC], and c_tr[nC] locating
  each entry's transpose: K * j + k' in B, or -1 - c' in C;
* the packed index Q = K * I + J (decoded by integer division and
  remainder); the second formula of the section cannot be decoded (I ranges
  up to N - 1 > K), and Q is defined only where J >= 0 (-1 elsewhere).
"""
from __future__ import annotations

import numpy as np


def hybrid_structure(n_cells: int, owner, neighbour, K: int):
    """I, J, Q as [N][K] int32 arrays and the CRS part (c_start, c_col, c_tr)
    of the structurally symmetric matrix whose off-diagonal entries are the
    internal faces (owner[f], neighbour[f])."""
    N = int(n_cells)
    rows = [[i] for i in range(N)]
    for a, b in zip(np.asarray(owner[:len(neighbour)]).tolist(), np.asarray(neighbour).tolist()):
        rows[a].append(b)
        rows[b].append(a)
    for r in rows:
        r.sort()
    # where each (row, column) entry lives: ("B", slot) or ("C", index)
    c_start = [0]
    c_col = []
    where = {}
    for i in range(N):
        for k, j in enumerate(rows[i]):
            if k < K:
                where[(i, j)] = ("B", k)
            else:
                where[(i, j)] = ("C", len(c_col))
                c_col.append(j)
        c_start.append(len(c_col))
    I = np.empty((N, K), np.int32)
    J = np.empty((N, K), np.int32)
    for i in range(N):
        for k in range(K):
            if k >= len(rows[i]):
                I[i, k], J[i, k] = i, k
                continue
            j = rows[i][k]
            I[i, k] = j
            kind, pos = where[(j, i)]
            J[i, k] = pos if kind == "B" else -1 - pos
    c_tr = np.empty(len(c_col), np.int32)
    for i in range(N):
        for c in range(c_start[i], c_start[i + 1]):
            kind, pos = where[(c_col[c], i)]
            c_tr[c] = K * c_col[c] + pos if kind == "B" else -1 - pos
    Q = np.where(J >= 0, K * I.astype(np.int64) + J, -1).astype(np.int32)
    return dict(I=I, J=J, Q=Q, c_start=np.array(c_start, np.int32), c_col=np.array(c_col, np.int32), c_tr=c_tr)


def decode_q(Q, K: int):
    """I and J back from Q = K * I + J (entries with J >= 0)."""
    Q = np.asarray(Q)
    return Q // K, Q % K
