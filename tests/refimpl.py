"""Independent test-side helpers (numpy / pure Python), used to pin the oracle.

  * ``brute_np``: the plain definition of the result with explicit float32
    elementwise operations (no reductions that could reassociate).
  * ``ordered_walk``: the ordered traversal with an explicit stack, recording
    the nodes it processes and the tour of node entries, to check the
    oracle's recursion and the trip counts of a two-integer state machine
    (Sec. 3.1: every move is to a child or to the parent, so the next node
    follows from the current and the previous one).
  * ``eytzinger``: textbook breadth-first layout of a sorted array, filled by
    an in-order walk of the implicit complete binary tree.
"""
import numpy as np


def d2_np(points, q):
    P = np.asarray(points, np.float32)
    q = np.asarray(q, np.float32)
    dx = (q[None, :] - P).astype(np.float32)
    s = (dx[:, 0] * dx[:, 0]).astype(np.float32)
    for j in range(1, P.shape[1]):
        s = (s + (dx[:, j] * dx[:, j]).astype(np.float32)).astype(np.float32)
    return s


def brute_np(points, q, k, R2):
    P = np.asarray(points, np.float32)
    idx = np.full(k, -1, np.int32)
    d = np.full(k, np.inf, np.float32)
    if P.shape[0] == 0:
        return idx, d
    s = d2_np(P, q)
    ok = np.nonzero(s <= np.float32(R2))[0]
    if len(ok) == 0:
        return idx, d
    o = np.lexsort((ok, s[ok]))[:k]
    sel = ok[o]
    idx[: len(sel)] = sel
    d[: len(sel)] = s[sel]
    return idx, d


def ordered_walk(points, order, q, k, R2, dims=None):
    """The ordered traversal of Sec. 3.1 (node first, then the close child,
    then the far child if its split plane is within the current search
    radius) written with an explicit stack of frames, independently of the
    oracle's recursion.  The close child is entered even when it does not
    exist (an immediate return), the far child only when in range; a missing
    node is entered and left at once.  Returns (processed positions in order,
    the tour of entered positions -- every node as it is entered and again
    each time a child returns to it --, idx list, d2 list).  The tour is the
    sequence of `curr` values a two-integer state machine passes through: one
    loop trip per entry.  dims: stored split dimension by position (else the
    level's, floor(log2(pos + 1)) mod D)."""
    P = np.asarray(points, np.float32)
    N, D = P.shape
    q = np.asarray(q, np.float32)
    lst = [(np.float32(R2), 2**31 - 1)] * k
    seq, tour = [], []
    # frame: [position, stage]; stage 0 = entering, 1 = close child done,
    # 2 = far child done (or skipped)
    stack = [[0, 0]]
    while stack:
        fr = stack[-1]
        pos = fr[0]
        tour.append(pos)
        if pos >= N:  # missing node: entered and left at once
            stack.pop()
            continue
        p = P[order[pos]]
        dim = int(dims[pos]) if dims is not None else int(np.floor(np.log2(pos + 1))) % D
        sd = np.float32(q[dim] - p[dim])
        close = 2 * pos + (2 if sd > 0 else 1)
        far = 2 * pos + (1 if sd > 0 else 2)
        if fr[1] == 0:
            seq.append(pos)
            dd = d2_np(p[None, :], q)[0]
            key = (dd, int(order[pos]))
            if key < lst[-1]:
                lst = sorted(lst[:-1] + [key])
            fr[1] = 1
            stack.append([close, 0])
        elif fr[1] == 1:
            fr[1] = 2
            if np.float32(sd * sd) <= lst[-1][0]:
                stack.append([far, 0])
            else:
                stack.pop()
        else:
            stack.pop()
    idx = np.array([i if i != 2**31 - 1 else -1 for _, i in lst], np.int32)
    d = np.array([dd if i != 2**31 - 1 else np.inf for dd, i in lst], np.float32)
    return seq, tour, idx, d


def eytzinger(sorted_ids):
    n = len(sorted_ids)
    out = [None] * n
    it = iter(sorted_ids)

    def walk(i):
        if i >= n:
            return
        walk(2 * i + 1)
        out[i] = next(it)
        walk(2 * i + 2)

    walk(0)
    return np.array(out, np.int32)


def subtree_positions(pos, n):
    """All level-order positions < n in the subtree rooted at pos."""
    out = []
    stack = [pos]
    while stack:
        p = stack.pop()
        if p < n:
            out.append(p)
            stack.append(2 * p + 1)
            stack.append(2 * p + 2)
    return out
