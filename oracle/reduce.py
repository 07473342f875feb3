"""Exact contact reduction (test infrastructure only).

Section III-C of the paper reduces candidates into patches: FindDeepest picks
the deepest candidate and BinReduce gathers the remaining candidates with a
similar normal.  With a fixed table of normal-direction bins standing in for
the data-dependent patches, the result for each (environment, bin) is the
candidate of greatest depth; equal depths go to the lowest vertex index
(the vertex's position in its environment's mesh).  -0.0 counts as +0.0; NaN
never reaches here because it is never a candidate.

The comparison is on the given float32 depths, so the result is exact and
unique; it does not depend on the order of the candidates.
"""
from __future__ import annotations

import numpy as np


def canonical_depth(depth32):
    d = np.asarray(depth32, dtype=np.float32).copy()
    d[d == 0.0] = np.float32(0.0)  # -0.0 -> +0.0
    return d


def reduce_contacts(env, vidx, depth32, bins, cand, n_env, K):
    """Winner per (env, bin).

    Returns (win_vidx int64 [n_env, K] with -1 for an empty bin,
             win_depth float32 [n_env, K] with 0 for an empty bin,
             win_row  int64 [n_env, K], the candidate's row, or -1).
    """
    env = np.asarray(env, dtype=np.int64)
    vidx = np.asarray(vidx, dtype=np.int64)
    bins = np.asarray(bins, dtype=np.int64)
    cand = np.asarray(cand, dtype=bool)
    d = canonical_depth(depth32)
    rows = np.nonzero(cand)[0]
    win_vidx = np.full((n_env, K), -1, dtype=np.int64)
    win_depth = np.zeros((n_env, K), dtype=np.float32)
    win_row = np.full((n_env, K), -1, dtype=np.int64)
    if len(rows) == 0:
        return win_vidx, win_depth, win_row
    e, b, dd, v = env[rows], bins[rows], d[rows].astype(np.float64), vidx[rows]
    order = np.lexsort((v, -dd, b, e))  # last key is primary
    e, b = e[order], b[order]
    first = np.ones(len(order), dtype=bool)
    first[1:] = (e[1:] != e[:-1]) | (b[1:] != b[:-1])
    sel = rows[order[first]]
    win_vidx[env[sel], bins[sel]] = vidx[sel]
    win_depth[env[sel], bins[sel]] = d[sel]
    win_row[env[sel], bins[sel]] = sel
    return win_vidx, win_depth, win_row


def reduce_contacts_bruteforce(env, vidx, depth32, bins, cand, n_env, K):
    """Same definition by exhaustive comparison (tiny inputs only)."""
    d = canonical_depth(depth32)
    win_vidx = np.full((n_env, K), -1, dtype=np.int64)
    win_depth = np.zeros((n_env, K), dtype=np.float32)
    for i in range(len(env)):
        if not cand[i]:
            continue
        e, b = int(env[i]), int(bins[i])
        cur = win_vidx[e, b]
        if cur < 0:
            better = True
        else:
            better = (float(d[i]) > float(win_depth[e, b])) or (
                float(d[i]) == float(win_depth[e, b]) and int(vidx[i]) < cur)
        if better:
            win_vidx[e, b] = int(vidx[i])
            win_depth[e, b] = d[i]
    return win_vidx, win_depth
