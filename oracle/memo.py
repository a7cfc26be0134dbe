"""O4: the memoized multi-tensor contraction, run directly, and its counts.

Follows Appendix C ("Details of Multi-tensor algorithm"):

* Each leaf variable X_j takes values from V_j; a tuple t^i lists the value
  index of every variable, variables enumerated in the order they occur in
  the tree (depth-first, left first).  For circuits the leaf values differ
  only by the bits fixed on their legs: the string's bits on output legs and
  the slice assignment's bits on sliced legs.  Value indices are those bit
  keys ranked in ascending order.
* eval_all(T, V, t) sorts t lexicographically, makes empty caches K_L and K_R
  and evaluates every tuple with eval'.
* eval'(T, ..., i, i_next): a leaf returns its value.  If T's key t^i_T is new
  (i is the first tuple or the key differs from tuple i-1), T = T_L * T_R:
  the right subtree's results for all its distinct keys are computed once by
  a nested eval_all and kept in K_R(T); the left subtree recurses with the
  index just past the run of tuples sharing T's key; the pair is contracted;
  the result goes to K_L(T) only if tuple i_next still has the same key; K_R(T)
  is dropped after the last run (i_next beyond the list).  An unchanged key
  returns K_L(T).
* Evaluation counts: T is contracted |t_T| times, the number of distinct
  restrictions of the tuples to T's variables; the bound
  k_T <= min(k_L * k_R, k) holds.

Tensors here are real numpy arrays (FP64 complex), so running the procedure
yields amplitudes that must equal the plain definition (O1/O2), and a
counter records every pairwise contraction.  An assertion checks the claim
that lexicographic order makes the single K_L entry per subtree sufficient:
a reused entry always carries the key being asked for.
"""

from __future__ import annotations

import numpy as np

from .tn import _fix


class Tree:
    """Contraction tree in the library's format: leaves 0..L-1, internal node
    L+i has children children[i] = (a, b) with a, b < L+i; the root is the last
    node."""

    def __init__(self, n_leaves: int, children):
        self.n_leaves = int(n_leaves)
        self.children = [tuple(int(x) for x in c) for c in children]
        self.root = self.n_leaves + len(self.children) - 1 if self.children else 0

    def kids(self, t):
        return self.children[t - self.n_leaves]

    def is_leaf(self, t):
        return t < self.n_leaves

    def leaves_dfs(self, t):
        if self.is_leaf(t):
            return [t]
        a, b = self.kids(t)
        return self.leaves_dfs(a) + self.leaves_dfs(b)

    def internal_nodes(self):
        return list(range(self.n_leaves, self.n_leaves + len(self.children)))


def leaf_key_bits(net, sliced):
    """For each leaf: the qubits whose output leg it carries and the slice
    bit positions j of the sliced legs it carries."""
    slot = {int(l): j for j, l in enumerate(sliced)}
    out = []
    for lf in net.leaves:
        qs = [net.leg_qubit[l] for l in lf.legs if net.leg_qubit[l] >= 0]
        js = [slot[l] for l in lf.legs if l in slot]
        out.append((qs, js))
    return out


def leaf_key(bits, s: int, sigma: int):
    qs, js = bits
    return tuple((int(s) >> q) & 1 for q in qs) + tuple((int(sigma) >> j) & 1 for j in js)


def distinct_key_counts(net, tree: Tree, bitstrings, sliced=(), sigmas=(0,)):
    """|t_T| for every internal node T: the number of distinct restrictions of
    the (string, slice) tuples to T's leaves (brute-force set counting)."""
    bits = leaf_key_bits(net, sliced)
    uniq = sorted(set(int(s) for s in bitstrings))
    counts = {}
    for t in tree.internal_nodes():
        lv = tree.leaves_dfs(t)
        keys = set()
        for s in uniq:
            for sg in sigmas:
                keys.add(tuple(leaf_key(bits[j], s, sg) for j in lv))
        counts[t] = len(keys)
    return counts


class _Run:
    def __init__(self, net, tree, sliced):
        self.net = net
        self.tree = tree
        self.sliced = [int(x) for x in sliced]
        self.bits = leaf_key_bits(net, sliced)
        self.contractions = {t: 0 for t in tree.internal_nodes()}
        self.leaf_pos = {}

    # ---- values ----------------------------------------------------------
    def leaf_value(self, j: int, key):
        lf = self.net.leaves[j]
        qs, js = self.bits[j]
        fixed = {}
        qi = 0
        for l in lf.legs:
            if self.net.leg_qubit[l] >= 0:
                fixed[l] = key[qi]
                qi += 1
        for l in lf.legs:
            if l in self.sliced:
                fixed[l] = key[qi]
                qi += 1
        return _fix(lf.tensor, lf.legs, fixed)

    def contract(self, t, u, v):
        self.contractions[t] += 1
        (tu, lu), (tv, lv) = u, v
        shared = [l for l in lu if l in lv]
        r = np.tensordot(tu, tv, axes=([lu.index(l) for l in shared],
                                       [lv.index(l) for l in shared]))
        legs = [l for l in lu if l not in shared] + [l for l in lv if l not in shared]
        return (r, legs)

    # ---- Algorithm 3 -----------------------------------------------------
    def eval_all(self, T, tuples):
        """tuples: set of tuples over T's leaves (DFS order) of leaf keys."""
        t = sorted(set(tuples))
        K_L, K_R = {}, {}
        R = {}
        for i in range(len(t)):
            R[t[i]] = self.eval_p(T, t, i, i + 1, K_L, K_R)
        return R

    # ---- Algorithm 4 -----------------------------------------------------
    def span(self, T):
        """Positions of T's leaves inside the enclosing tuple (set by caller)."""
        return self.pos[T]

    def eval_p(self, T, t, i, i_next, K_L, K_R):
        lo, hi = self.pos[T]
        if self.tree.is_leaf(T):
            return self.leaf_value(T, t[i][lo])
        key = t[i][lo:hi]
        if i == 0 or t[i - 1][lo:hi] != key:
            TL, TR = self.tree.kids(T)
            if T not in K_R:
                rlo, rhi = self.pos[TR]
                sub = {tp[rlo:rhi] for tp in t}
                saved = self.pos
                self.pos = self._positions(TR)
                K_R[T] = (self.eval_all(TR, sub), (rlo, rhi))
                self.pos = saved
            # i_next for the left child: one past the last tuple sharing T's key.
            j = i
            while j + 1 < len(t) and t[j + 1][lo:hi] == key:
                j += 1
            u_l = self.eval_p(TL, t, i, j + 1, K_L, K_R)
            table, (rlo, rhi) = K_R[T]
            u_r = table[t[i][rlo:rhi]]
            u = self.contract(T, u_l, u_r)
            if i_next < len(t) and t[i_next][lo:hi] == key:
                K_L[T] = (key, u)
            if i_next >= len(t):
                del K_R[T]
            return u
        stored_key, u = K_L[T]
        assert stored_key == key, "lexicographic order violated: stale K_L entry"
        return u

    def _positions(self, top):
        """Map each subtree of `top` to its [lo, hi) span in top's DFS leaf list."""
        pos = {}

        def rec(T, lo):
            if self.tree.is_leaf(T):
                pos[T] = (lo, lo + 1)
                return lo + 1
            a, b = self.tree.kids(T)
            mid = rec(a, lo)
            hi = rec(b, mid)
            pos[T] = (lo, hi)
            return hi

        rec(top, 0)
        return pos


def memo_amplitudes(net, tree: Tree, bitstrings, sliced=(), sigmas=None):
    """Run eval_all over the (string, slice) tuples and sum each string's
    partials over the slice assignments.  Returns (amps for the input order,
    per-node contraction counts)."""
    import math

    run = _Run(net, tree, sliced)
    if sigmas is None:
        sigmas = range(1 << len(sliced))
    sigmas = list(sigmas)
    run.pos = run._positions(tree.root)
    lv = tree.leaves_dfs(tree.root)
    uniq = sorted(set(int(s) for s in bitstrings))
    tup_of = {}
    for s in uniq:
        for sg in sigmas:
            tup_of[(s, sg)] = tuple(leaf_key(run.bits[j], s, sg) for j in lv)
    if tree.children:
        R = run.eval_all(tree.root, set(tup_of.values()))
        val = {k: complex(R[v][0]) for k, v in tup_of.items()}
    else:
        val = {k: complex(run.leaf_value(0, v[0])[0]) for k, v in tup_of.items()}
    out = []
    for s in bitstrings:
        parts = [val[(int(s), sg)] for sg in sigmas]
        out.append(complex(math.fsum(p.real for p in parts),
                           math.fsum(p.imag for p in parts)))
    return np.array(out, dtype=np.complex128), run.contractions
