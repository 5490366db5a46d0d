"""Oracle: reverse Cuthill-McKee ordering of a symmetric sparsity graph.

Test infrastructure only (see oracle/__init__.py).

Not part of the paper (its local problems are solved by a sparse direct solver, Sec. 6.1); the
library orders each local matrix before its banded factorisation and this module fixes that
ordering so the two can be compared integer for integer:

* key(u) = (degree(u), u), degree = number of neighbours other than u itself;
* per connected component, start from the unvisited vertex of least key and move to a
  pseudo-peripheral vertex (George-Liu): build the level structure from the current root, take
  the least-key vertex x of its last level, and replace the root by x while x's level structure
  is strictly deeper;
* Cuthill-McKee breadth-first order from that root, each vertex's unvisited neighbours appended
  in increasing key;
* the concatenated order is reversed; perm[new] = old.
"""
import numpy as np


def _levels(adj_ptr, adj_idx, root, allowed):
    depth = 0
    seen = {root}
    frontier = [root]
    last = [root]
    while frontier:
        depth += 1
        last = frontier
        nxt = []
        for u in frontier:
            for v in adj_idx[adj_ptr[u]:adj_ptr[u + 1]]:
                v = int(v)
                if v not in seen and allowed[v]:
                    seen.add(v)
                    nxt.append(v)
        frontier = nxt
    return depth, last


def rcm(adj_ptr, adj_idx):
    """adj_ptr/adj_idx: CSR of the symmetric neighbour lists (self loops are ignored)."""
    n = len(adj_ptr) - 1
    nbr = []
    for u in range(n):
        row = adj_idx[adj_ptr[u]:adj_ptr[u + 1]]
        nbr.append(np.unique(row[row != u]).astype(np.int64))
    deg = np.array([len(x) for x in nbr], dtype=np.int64)
    ptr = np.zeros(n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(deg)
    idx = np.concatenate(nbr) if n else np.zeros(0, dtype=np.int64)
    key = lambda u: (int(deg[u]), int(u))
    visited = np.zeros(n, dtype=bool)
    order = []
    by_key = sorted(range(n), key=key)
    cursor = 0
    while len(order) < n:
        while visited[by_key[cursor]]:
            cursor += 1
        s = by_key[cursor]
        allowed = ~visited
        root = s
        depth, last = _levels(ptr, idx, root, allowed)
        while True:
            x = min(last, key=key)
            dx, lx = _levels(ptr, idx, x, allowed)
            if dx > depth:
                root, depth, last = x, dx, lx
            else:
                break
        visited[root] = True
        q = [root]
        head = 0
        while head < len(q):
            u = q[head]
            head += 1
            cand = [int(v) for v in idx[ptr[u]:ptr[u + 1]] if not visited[v]]
            cand.sort(key=key)
            for v in cand:
                visited[v] = True
            q.extend(cand)
        order.extend(q)
    return np.array(order[::-1], dtype=np.int64)


def envelope(adj_ptr, adj_idx, perm):
    """first[i] = least new column index in new row i of P A P^T (diagonal included)."""
    n = len(perm)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    first = np.arange(n, dtype=np.int64)
    for new_i, old in enumerate(perm):
        row = adj_idx[adj_ptr[old]:adj_ptr[old + 1]]
        if len(row):
            first[new_i] = min(first[new_i], int(inv[row].min()))
    return first


def pattern_graph(P):
    """CSR neighbour lists of a structural pattern matrix (self loops kept, ignored by rcm)."""
    P = P.tocsr()
    P.sort_indices()
    return P.indptr.astype(np.int64), P.indices.astype(np.int64)
