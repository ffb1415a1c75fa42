"""Filter outputs at sampled rows, from the reference's sparse rows.

The degree-n filter (Fig. fig:ChebFD) at row r depends only on the rows
within n hops of r, so its value there follows from the reference matrix
rows and the input rows of that neighbourhood: the recurrence
T_{k+1} = 2 (alpha H + beta) T_k - T_{k-1} evaluated on nested row sets
(T_k on the rows within n - k hops).  Test infrastructure: the sums are
plain numpy over the reference's CSR rows.
"""
import numpy as np


def neighbourhoods(H, rows, n):
    """sets[k] = the rows within k hops of `rows` (sorted), k = 0..n."""
    sets = [np.unique(np.asarray(rows, np.int64))]
    for _ in range(n):
        s = sets[-1]
        cols = np.concatenate([H.col[H.rowptr[r]:H.rowptr[r + 1]] for r in s])
        sets.append(np.union1d(s, cols.astype(np.int64)))
    return sets


def sampled_filter(H, a, b, gam, rows, xrows):
    """p(alpha H + beta) X at `rows` (returned in sorted order, with the
    rows), for gamma_0..gamma_n; xrows(idx) gives the input rows idx."""
    n = len(gam) - 1
    sets = neighbourhoods(H, rows, n)
    base = sets[n]
    pos = {int(r): i for i, r in enumerate(base)}
    alpha, beta = 2.0 / (b - a), (a + b) / (a - b)
    X = np.asarray(xrows(base), np.complex128)

    def apply(T, on):
        # (alpha H + beta) T on the rows `on`; T holds rows of `base`
        out = np.zeros_like(T)
        for r in on:
            lo, hi = H.rowptr[r], H.rowptr[r + 1]
            idx = [pos[int(c)] for c in H.col[lo:hi]]
            out[pos[int(r)]] = alpha * (H.val[lo:hi] @ T[idx]) + beta * T[pos[int(r)]]
        return out

    t_prev, t_cur = X, apply(X, sets[n - 1])
    sel = [pos[int(r)] for r in sets[0]]
    acc = gam[0] * X[sel] + gam[1] * t_cur[sel]
    for k in range(2, n + 1):
        t_next = 2.0 * apply(t_cur, sets[n - k]) - t_prev
        acc = acc + gam[k] * t_next[sel]
        t_prev, t_cur = t_cur, t_next
    return sets[0], acc
