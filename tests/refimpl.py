"""Independent test-side helpers (numpy / pure Python), used to pin the oracle.

  * ``brute_np``: the plain definition of the result with explicit float32
    elementwise operations (no reductions that could reassociate).
  * ``stackfree_sequence``: the two-integer state machine of the paper's
    Sec. 3.2 run on the CPU, recording the nodes it processes, to check the
    paper's claim (Sec. 3.1) that it processes the same nodes in the same
    order as the ordered recursion.
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


def stackfree_sequence(points, order, q, k, R2):
    """Run the Sec. 3.2 state machine; processNode keeps a k-list of
    (d2, idx) and the search radius is the list's worst d2.  Returns
    (processed positions in order, loop iterations, idx list, d2 list)."""
    P = np.asarray(points, np.float32)
    N, D = P.shape
    q = np.asarray(q, np.float32)
    lst = [(np.float32(R2), 2**31 - 1)] * k
    seq = []
    curr, prev = 0, -1
    iters = 0
    while True:
        iters += 1
        parent = (curr + 1) // 2 - 1
        if curr >= N:
            prev, curr = curr, parent
            continue
        from_parent = prev < curr
        p = P[order[curr]]
        if from_parent:
            seq.append(curr)
            dd = d2_np(p[None, :], q)[0]
            key = (dd, int(order[curr]))
            if key < lst[-1]:
                lst = sorted(lst[:-1] + [key])
        level = int(np.floor(np.log2(curr + 1)))
        dim = level % D
        sd = np.float32(q[dim] - p[dim])
        close_side = 1 if sd > 0 else 0
        close_c = 2 * curr + 1 + close_side
        far_c = 2 * curr + 2 - close_side
        far_in = np.float32(sd * sd) <= lst[-1][0]
        if from_parent:
            nxt = close_c
        elif prev == close_c:
            nxt = far_c if far_in else parent
        else:
            nxt = parent
        if nxt == -1:
            break
        prev, curr = curr, nxt
    idx = np.array([i if i != 2**31 - 1 else -1 for _, i in lst], np.int32)
    d = np.array([dd if i != 2**31 - 1 else np.inf for dd, i in lst], np.float32)
    return seq, iters, idx, d


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
