"""Contraction-tree optimizer by local search (Appendix A, "Contraction trees
optimization"; multi-tensor costs of Appendix C).

State: a binary contraction tree plus a set S of sliced legs.  Moves:
* the four local rotations of Appendix A, which at a node v = (u * y) with
  u = (p * q) exchange y with p or with q (the other two are the same moves
  with the roles of v's children swapped);
* every `slice_every` steps, a slicing move (Appendix A, paragraph
  "Slicing"): either the paper's (with probability 1/2 the leg giving the
  best memory reduction joins S, else a random leg leaves it) or, with the
  size of S fixed, one random leg leaves S and the leg giving the best
  reduction of the largest tensor joins it.

Each node's term is its estimated time for all slices,
    ev_T * (max(C_T / CMAC_RATE, RW_T / ELEM_RATE) + LAUNCH_S),
with C_T = k_T 2^(q+r) and RW_T = |L table| + |R table| + |T table| (k_T the
number of distinct string keys, Appendix C) and ev_T = 2^(sliced legs below
T): the efficiency-profile objective the paper suggests in place of
log2(C + alpha RW).  A rotation changes only the terms of u and v, so its
gain is computed locally (Appendix C, local cost update).  The objective is
    log(total time) + beta * max(log2(largest tensor) - size_log2_max, 0),
the memory penalty of the paper's f(T) with the largest intermediate as M,
plus, when a byte budget is given, beta * max(log2(tables / budget), 0) with
tables = sum_T k_T |T| * 8 bytes, the memory of the executor that keeps every
node's table of keys resident (also a local update: a rotation changes only
u's table).  The paper's own objective, beta max(log2(M / M_max), 0) +
log2(C + alpha RW), is available too, with M either those tables or the
Appendix C estimate M(T, k) (locally updated like the costs).  Acceptance is
Metropolis with a geometric temperature schedule.
"""

from __future__ import annotations

import math
import random

from .planner import CMAC_RATE, ELEM_RATE, LAUNCH_S, Structure, VariantCounter


def _popcount(x: int) -> int:
    return bin(x).count("1")


class TreeState:
    def __init__(self, st: Structure, count: VariantCounter, children, sliced=()):
        self.st = st
        self.count = count
        L = st.n_leaves
        self.L = L
        n = 2 * L - 1
        # Legs as bit masks over internal leg ids.
        self.legs = [0] * n
        self.om = [0] * n
        self.left = [-1] * n
        self.right = [-1] * n
        self.parent = [-1] * n
        for j in range(L):
            m = 0
            for l in st.legs[j]:
                m |= 1 << l
            self.legs[j] = m
            self.om[j] = st.outmask[j]
        for i, (a, b) in enumerate(children):
            v = L + i
            self.left[v], self.right[v] = a, b
            self.parent[a] = self.parent[b] = v
        self.root = n - 1
        self.S = 0
        for l in sliced:
            self.S |= 1 << l
        self.k = [1] * n
        self.sdep = [0] * n
        self.term = [0.0] * n
        self.cterm = [0.0] * n   # ev_T C_T (complex MACs over all slices)
        self.rwterm = [0.0] * n  # ev_T RW_T (elements over all slices)
        self.memv = [0.0] * n
        self.mkv = [0] * n       # m_K(T) of the Appendix C memory estimate (bytes, exact)
        self.pnv = [0] * n       # m(T)^P_NORM (exact integers: no drift under updates)
        self.size_hist = {}
        self.recompute_all()

    P_NORM = 8  # the p of the Appendix C estimate's p-norm

    # -- per-node quantities ----------------------------------------------------
    def _refresh(self, v: int) -> None:
        a, b = self.left[v], self.right[v]
        self.legs[v] = self.legs[a] ^ self.legs[b]
        self.om[v] = self.om[a] | self.om[b]
        self.k[v] = self.count(self.om[v])
        self.sdep[v] = self.sdep[a] | self.sdep[b] | ((self.legs[a] | self.legs[b]) & self.S)

    def _term(self, v: int) -> float:
        """Estimated seconds of node v over all slices; also sets its C and RW
        terms."""
        a, b = self.left[v], self.right[v]
        nS = ~self.S
        la, lb = self.legs[a] & nS, self.legs[b] & nS
        c = self.k[v] * 2.0 ** _popcount(la | lb)
        rw = (self.k[a] * 2.0 ** _popcount(la) + self.k[b] * 2.0 ** _popcount(lb)
              + self.k[v] * 2.0 ** _popcount(la ^ lb))
        ev = 2.0 ** _popcount(self.sdep[v])
        self._c_new, self._rw_new = ev * c, ev * rw
        return ev * (max(c / CMAC_RATE, rw / ELEM_RATE) + LAUNCH_S)

    def _m(self, v: int) -> int:
        """m(T): bytes of one evaluation of v (after slicing)."""
        return 8 << self._size_log2(v)

    def _mk(self, v: int) -> int:
        """m_K(T) of the Appendix C memory estimate: the caches' share of a
        node evaluated k_T times (0 for leaves and for k_T = 1)."""
        if v < self.L or self.k[v] == 1:
            return 0
        a, b = self.left[v], self.right[v]
        ka, kb, kv = self.k[a], self.k[b], self.k[v]
        ma, mb = self._m(a), self._m(b)
        if min(ka, kb) < kv:
            return min(ka * ma + mb, ma + kb * mb)
        return min(ka * ma, kb * mb)

    def _pn(self, v: int) -> int:
        return self._m(v) ** self.P_NORM

    def appc_memory(self) -> float:
        """M(T, k) of Appendix C: sum of m_K over all nodes plus twice the
        p-norm of the node sizes (a smooth stand-in for twice the largest)."""
        return float(self.mk_sum) + 2.0 * math.exp(math.log(self.pn_sum) / self.P_NORM)

    def _size_log2(self, v: int) -> int:
        return _popcount(self.legs[v] & ~self.S)

    def _mem(self, v: int) -> float:
        """Bytes of v's resident table (a leaf's holds every slice key)."""
        m = 8.0 * self.k[v] * 2.0 ** self._size_log2(v)
        if v < self.L:
            m *= 2.0 ** _popcount(self.legs[v] & self.S)
        return m

    def _hist_add(self, e: int, d: int) -> None:
        c = self.size_hist.get(e, 0) + d
        if c:
            self.size_hist[e] = c
        else:
            self.size_hist.pop(e, None)

    def recompute_all(self) -> None:
        for j in range(self.L):
            self.k[j] = self.count(self.om[j])
            self.sdep[j] = self.legs[j] & self.S
        self.size_hist = {}
        self.mem = 0.0
        self.mk_sum = 0
        self.pn_sum = 0
        for j in range(self.L):
            self._hist_add(self._size_log2(j), 1)
            self.memv[j] = self._mem(j)
            self.mem += self.memv[j]
            self.mkv[j] = 0
            self.pnv[j] = self._pn(j)
            self.pn_sum += self.pnv[j]
        self.total = 0.0
        self.C = 0.0
        self.RW = 0.0
        for v in range(self.L, 2 * self.L - 1):
            self._refresh(v)
            self.term[v] = self._term(v)
            self.cterm[v], self.rwterm[v] = self._c_new, self._rw_new
            self.total += self.term[v]
            self.C += self.cterm[v]
            self.RW += self.rwterm[v]
            self._hist_add(self._size_log2(v), 1)
            self.memv[v] = self._mem(v)
            self.mem += self.memv[v]
            self.mkv[v] = self._mk(v)
            self.mk_sum += self.mkv[v]
            self.pnv[v] = self._pn(v)
            self.pn_sum += self.pnv[v]

    def max_size_log2(self) -> int:
        return max(self.size_hist)

    def children(self):
        """The tree in the library's format: internal nodes renumbered in
        post-order so every child id is smaller than its parent's."""
        L = self.L
        new_id = {}
        out = []
        stack = [(self.root, False)]
        while stack:
            v, done = stack.pop()
            if v < L:
                continue
            if done:
                a, b = self.left[v], self.right[v]
                out.append((a if a < L else new_id[a], b if b < L else new_id[b]))
                new_id[v] = L + len(out) - 1
            else:
                stack.append((v, True))
                stack.append((self.right[v], False))
                stack.append((self.left[v], False))
        return out

    # -- rotations ------------------------------------------------------------------
    def rotate(self, v: int, side: int, pick: int):
        """At v = (u * y), u the child on `side` (0 left, 1 right), exchange y
        with u's child number `pick`.  Returns an undo record or None."""
        u = self.left[v] if side == 0 else self.right[v]
        if u < self.L:
            return None
        y = self.right[v] if side == 0 else self.left[v]
        g = self.left[u] if pick == 0 else self.right[u]
        undo = (v, u, self.left[v], self.right[v], self.left[u], self.right[u],
                self.legs[u], self.om[u], self.k[u], self.sdep[u], self.term[u], self.term[v],
                self.memv[u], self.cterm[u], self.cterm[v], self.rwterm[u], self.rwterm[v],
                self.mkv[u], self.mkv[v], self.pnv[u])
        # u keeps its other child and takes y; v takes u and g (u stays v's child).
        if pick == 0:
            self.left[u] = y
        else:
            self.right[u] = y
        if side == 0:
            self.right[v] = g
        else:
            self.left[v] = g
        self.parent[y] = u
        self.parent[g] = v
        self._hist_add(self._size_log2(u), -1)
        self._refresh(u)
        self._hist_add(self._size_log2(u), 1)
        m_u = self._mem(u)
        self.mem += m_u - self.memv[u]
        self.memv[u] = m_u
        t_u = self._term(u)
        c_u, rw_u = self._c_new, self._rw_new
        t_v = self._term(v)
        c_v, rw_v = self._c_new, self._rw_new
        self.total += t_u + t_v - self.term[u] - self.term[v]
        self.term[u], self.term[v] = t_u, t_v
        self.C += c_u + c_v - self.cterm[u] - self.cterm[v]
        self.RW += rw_u + rw_v - self.rwterm[u] - self.rwterm[v]
        self.cterm[u], self.cterm[v], self.rwterm[u], self.rwterm[v] = c_u, c_v, rw_u, rw_v
        mk_u, mk_v, pn_u = self._mk(u), self._mk(v), self._pn(u)
        self.mk_sum += mk_u + mk_v - self.mkv[u] - self.mkv[v]
        self.pn_sum += pn_u - self.pnv[u]
        self.mkv[u], self.mkv[v], self.pnv[u] = mk_u, mk_v, pn_u
        return undo

    def undo(self, rec) -> None:
        (v, u, lv, rv, lu, ru, legs_u, om_u, k_u, sdep_u, term_u, term_v, mem_u,
         c_u, c_v, rw_u, rw_v, mk_u, mk_v, pn_u) = rec
        self._hist_add(self._size_log2(u), -1)
        self.mem += mem_u - self.memv[u]
        self.memv[u] = mem_u
        self.total += term_u + term_v - self.term[u] - self.term[v]
        self.C += c_u + c_v - self.cterm[u] - self.cterm[v]
        self.RW += rw_u + rw_v - self.rwterm[u] - self.rwterm[v]
        self.cterm[u], self.cterm[v], self.rwterm[u], self.rwterm[v] = c_u, c_v, rw_u, rw_v
        self.mk_sum += mk_u + mk_v - self.mkv[u] - self.mkv[v]
        self.pn_sum += pn_u - self.pnv[u]
        self.mkv[u], self.mkv[v], self.pnv[u] = mk_u, mk_v, pn_u
        self.left[v], self.right[v], self.left[u], self.right[u] = lv, rv, lu, ru
        for c in (lv, rv):
            self.parent[c] = v
        for c in (lu, ru):
            self.parent[c] = u
        self.legs[u], self.om[u], self.k[u], self.sdep[u] = legs_u, om_u, k_u, sdep_u
        self.term[u], self.term[v] = term_u, term_v
        self._hist_add(self._size_log2(u), 1)

    # -- slicing --------------------------------------------------------------------
    def sliced(self):
        out = []
        S = self.S
        while S:
            low = S & -S
            out.append(low.bit_length() - 1)
            S ^= low
        return out

    def set_slices(self, S: int) -> None:
        self.S = S
        self.recompute_all()


def anneal(st: Structure, count: VariantCounter, children, sliced=(), steps: int = 100000,
           t0: float = 0.05, t1: float = 0.0005, beta: float = 8.0, size_log2_max=None,
           slice_every: int = 20000, seed: int = 0, mem_max=None, objective: str = "time",
           alpha: float = 19.7, memory: str = "tables", slicing: str = "swap"):
    """Simulated annealing from (children, sliced).  Returns (children, sliced,
    info).

    objective "time" (the efficiency-profile form): log(estimated seconds)
    plus beta * max(log2(largest tensor) - size_log2_max, 0) (size_log2_max
    None: the starting tree's largest tensor) plus, with a byte budget
    mem_max, beta * max(log2(M / mem_max), 0).
    objective "paper" (Appendix A): f = beta * max(log2(M / mem_max), 0) +
    log2(C + alpha RW) with C complex MACs and RW elements over all slices;
    alpha is the arithmetic intensity in complex MACs per element (19.7 for
    complex64 on FP32 MFMA, about 105 for the split forms).
    memory: M is "tables" (the executor's resident tables, sum k_T |T| 8 B)
    or "appc" (the Appendix C estimate M(T, k)).
    slicing "swap": every slice_every steps one random sliced leg is traded
    for the leg that most reduces the largest tensor (|S| fixed).  slicing
    "paper" (Appendix A, "Slicing"): every slice_every steps, with
    probability 1/2, the leg giving the largest reduction of M joins S, else
    a random leg leaves S."""
    rng = random.Random(seed)
    ts = TreeState(st, count, children, sliced)
    if size_log2_max is None:
        size_log2_max = ts.max_size_log2()
    n_slice = len(list(sliced))
    open_legs = getattr(st, "open_legs", frozenset())

    def mem_of():
        return ts.mem if memory == "tables" else ts.appc_memory()

    def objective_value():
        if objective == "paper":
            f = math.log2(ts.C + alpha * ts.RW)
            if mem_max:
                f += beta * max(math.log2(mem_of() / mem_max), 0.0)
            return f
        f = math.log(ts.total) + beta * max(ts.max_size_log2() - size_log2_max, 0)
        if mem_max:
            f += beta * max(math.log2(mem_of() / mem_max), 0.0)
        return f

    def candidates(base):
        """Legs of the tensors within one bit of the largest (not open)."""
        cand = set()
        mx = ts.max_size_log2()
        for w in range(ts.L, 2 * ts.L - 1):
            if _popcount(ts.legs[w] & ~base) >= mx - 1:
                x = ts.legs[w] & ~base
                while x:
                    low = x & -x
                    cand.add(low.bit_length() - 1)
                    x ^= low
        return cand - open_legs

    objective_fn = objective_value

    cur = objective_fn()
    best = (cur, ts.children(), ts.sliced(), ts.total, ts.max_size_log2(), ts.mem)
    internal = list(range(ts.L, 2 * ts.L - 1))
    accepted = 0
    for step in range(steps):
        temp = t0 * (t1 / t0) ** (step / max(steps - 1, 1))
        v = internal[rng.randrange(len(internal))]
        rec = ts.rotate(v, rng.randrange(2), rng.randrange(2))
        if rec is None:
            continue
        new = objective_fn()
        if new <= cur or rng.random() < math.exp(-(new - cur) / temp):
            cur = new
            accepted += 1
            if cur < best[0]:
                best = (cur, ts.children(), ts.sliced(), ts.total, ts.max_size_log2(), ts.mem)
        else:
            ts.undo(rec)
        if slicing == "paper" and slice_every and (step + 1) % slice_every == 0:
            S = ts.S
            if S and rng.random() < 0.5:
                cur_S = ts.sliced()
                ts.set_slices(S & ~(1 << cur_S[rng.randrange(len(cur_S))]))
            else:
                cand = candidates(S)
                choice = None
                for l in sorted(cand):
                    ts.set_slices(S | (1 << l))
                    key = (mem_of(), objective_fn(), l)
                    if choice is None or key < choice[0]:
                        choice = (key, l)
                ts.set_slices(S if choice is None else S | (1 << choice[1]))
            cur = objective_fn()
            if cur < best[0]:
                best = (cur, ts.children(), ts.sliced(), ts.total, ts.max_size_log2(), ts.mem)
            continue
        if n_slice and slice_every and (step + 1) % slice_every == 0:
            # Slicing move: drop a random sliced leg, add the leg that most
            # reduces the largest tensor (ties: lower time).
            cur_S = ts.sliced()
            drop = cur_S[rng.randrange(len(cur_S))]
            base = ts.S & ~(1 << drop)
            ts.set_slices(base)
            cand = candidates(base)
            if not cand:
                ts.set_slices(ts.S | (1 << drop))
                continue
            choice = None
            for l in sorted(cand):
                ts.set_slices(base | (1 << l))
                key = (ts.max_size_log2(), ts.total, l)
                if choice is None or key < choice[0]:
                    choice = (key, l)
            ts.set_slices(base | (1 << choice[1]))
            cur = objective_fn()
            if cur < best[0]:
                best = (cur, ts.children(), ts.sliced(), ts.total, ts.max_size_log2(), ts.mem)
    info = dict(objective=best[0], seconds=best[3], max_log2=best[4], table_bytes=best[5],
                accepted=accepted, steps=steps, n_sliced=len(best[2]))
    return best[1], best[2], info
