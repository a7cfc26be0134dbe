"""Contraction-tree and slicing planner (host side).

Produces the `contraction_tree` and `sliced_legs` inputs of xeb_plan_create.

* Tree: randomized greedy over connected pairs.  The score of contracting a
  and b compares the size of the result with the sizes of the operands, each
  weighted by its number of distinct string keys (the evaluation count k_T of
  Appendix C), so the batch's shared sub-contractions are preferred; several
  randomized trials keep the cheapest tree under the multi-tensor cost
  C(T, k) = sum_T k_T 2^(q_T + r_T) (Appendix C, "Complexity estimation").
* Slicing: the paper's rule of adding the leg that gives the best memory
  reduction (Appendix A, "Slicing"), applied greedily until the requested
  number of legs is sliced (ties: lower total cost).
* Slice-bit order: slices run in increasing id order and a node is contracted
  again only when one of its slice bits changes, so the legs that expensive
  nodes depend on get the high bits (greedy from bit 0 upwards).

The local-search optimizer of Appendix A lives in `optimizer` and refines the
greedy result when `anneal_steps` > 0.
"""

from __future__ import annotations

import math
import random

import numpy as np

from . import xeb as _xeb


class Structure:
    """Leaf legs (internal legs only) and output masks of a circuit's network.

    The output legs of `open_qubits` (multi-batch output) stay tensor legs up
    to the root and are in `open_legs`; they are never sliced."""

    def __init__(self, circ, fuse_1q=True, fold_kets=True, open_qubits: int = 0):
        leaves, n_legs, leg_qubit = _xeb.network_describe(circ, fuse_1q, fold_kets)
        self.n_legs = n_legs
        self.leg_qubit = leg_qubit
        self.open_legs = frozenset(l for l, q in enumerate(leg_qubit)
                                   if q >= 0 and (open_qubits >> q) & 1)
        self.legs = []
        self.outmask = []
        for legs in leaves:
            om = 0
            internal = []
            for l in legs:
                q = leg_qubit[l]
                if q >= 0 and l not in self.open_legs:
                    om |= 1 << q
                else:
                    internal.append(l)
            self.legs.append(frozenset(internal))
            self.outmask.append(om)
        self.n_leaves = len(leaves)


class VariantCounter:
    """Number of distinct keys s & mask over the distinct strings (cached).

    Exact for batches of at most `exact_limit` distinct strings.  Larger
    batches use the expected number of distinct values of k draws over the
    2^v values of the mask's varying bits (bits that differ somewhere in the
    batch), which is what the tree search needs; the plan compiler counts
    exactly."""

    def __init__(self, bitstrings, exact_limit: int = 20000):
        self.s = np.unique(np.asarray(bitstrings, dtype=np.uint64))
        self.cache = {0: 1}
        self.exact = self.s.size <= exact_limit
        if self.s.size:
            self.varying = int(np.bitwise_or.reduce(self.s ^ self.s[0]))
        else:
            self.varying = 0

    def __call__(self, mask: int) -> int:
        r = self.cache.get(mask)
        if r is None:
            if not self.s.size:
                r = 1
            elif self.exact:
                r = int(np.unique(self.s & np.uint64(mask)).size)
            else:
                v = bin(mask & self.varying).count("1")
                n_vals = 2.0 ** v
                k = float(self.s.size)
                r = int(round(n_vals * -math.expm1(k * math.log1p(-1.0 / n_vals)))) if v else 1
            r = max(r, 1)
            self.cache[mask] = r
        return r


def greedy_tree(st: Structure, count: VariantCounter, rng: random.Random, temp: float):
    act = {i: (st.legs[i], st.outmask[i]) for i in range(st.n_leaves)}
    owners = {}
    for i, (legs, _) in act.items():
        for l in legs:
            owners.setdefault(l, set()).add(i)
    children = []
    nid = st.n_leaves
    while len(act) > 1:
        cands = set()
        for l, who in owners.items():
            if len(who) == 2:
                a, b = sorted(who)
                cands.add((a, b))
        if not cands:
            ks = sorted(act)
            cands = {(ks[0], ks[1])}
        best = None
        for a, b in sorted(cands):
            la, oa = act[a]
            lb, ob = act[b]
            res = la ^ lb
            out = math.log2(count(oa | ob)) + len(res)
            inp = math.log2(count(oa) * 2.0 ** len(la) + count(ob) * 2.0 ** len(lb))
            score = out - inp
            if temp > 0:
                score -= temp * -math.log(-math.log(rng.random() or 1e-300))
            if best is None or score < best[0]:
                best = (score, a, b)
        _, a, b = best
        la, oa = act.pop(a)
        lb, ob = act.pop(b)
        res = la ^ lb
        for l in la | lb:
            owners[l].discard(a)
            owners[l].discard(b)
            if l in res:
                owners[l].add(nid)
            else:
                del owners[l]
        act[nid] = (res, oa | ob)
        children.append((a, b))
        nid += 1
    return children


def node_sets(st: Structure, children, sliced=frozenset()):
    """Per node: legs (after slicing), outmask, set of sliced legs below."""
    legs = [l - sliced for l in st.legs]
    full = list(st.legs)
    om = list(st.outmask)
    sdep = [l & sliced for l in st.legs]
    for a, b in children:
        full.append(full[a] ^ full[b])
        legs.append(full[-1] - sliced)
        om.append(om[a] | om[b])
        sdep.append(sdep[a] | sdep[b])
    return full, legs, om, sdep


# Rates of one MI355X for the time estimate: complex MACs/s on FP32 MFMA
# (157.3 TFLOP/s / 8) and complex64 elements/s of HBM (8 TB/s / 8 B), plus a
# fixed cost per launch.
CMAC_RATE = 157.3e12 / 8
ELEM_RATE = 8e12 / 8
LAUNCH_S = 4e-6


def tree_cost(st: Structure, children, count: VariantCounter, sliced=(), order=None):
    """Multi-tensor cost over all slices under the executor's schedule, the
    largest tensor (log2 elements) after slicing, per-slice cost, and an
    estimated time: per evaluation max(C / CMAC_RATE, RW / ELEM_RATE) + launch,
    with C = k_T 2^(q+r) and RW = |L table| + |R table| + |T table| (Appendix A
    measures C and RW; the estimate stands in for the efficiency profile the
    paper suggests in place of log2(C + alpha RW))."""
    sliced = frozenset(sliced)
    bit = {l: j for j, l in enumerate(order)} if order is not None else None
    full, legs, om, sdep = node_sets(st, children, sliced)
    L = st.n_leaves
    s = len(sliced)
    total = 0.0
    per_slice = 0.0
    seconds = 0.0
    maxsz = max((len(x) for x in legs), default=0)
    for i, (a, b) in enumerate(children):
        t = L + i
        allg = (full[a] | full[b]) - sliced
        kt = count(om[t])
        c = kt * 2.0 ** len(allg)
        rw = (count(om[a]) * 2.0 ** len(legs[a]) + count(om[b]) * 2.0 ** len(legs[b])
              + kt * 2.0 ** len(legs[t]))
        per_slice += c
        if not sdep[t]:
            ev = 1.0
        elif bit is None:
            ev = 2.0 ** len(sdep[t])        # ideal reuse across slices
        else:
            ev = 2.0 ** (s - min(bit[l] for l in sdep[t]))
        total += ev * c
        seconds += ev * (max(c / CMAC_RATE, rw / ELEM_RATE) + LAUNCH_S)
    return total, maxsz, per_slice, seconds


def greedy_slices(st: Structure, children, count: VariantCounter, n_slice: int):
    """Add legs one at a time, each the one that most reduces the largest
    tensor (Appendix A, "Slicing"); ties go to the lower estimated time."""
    sliced = set()
    for _ in range(n_slice):
        full, legs, om, sdep = node_sets(st, children, frozenset(sliced))
        maxsz = max(len(x) for x in legs)
        cand = set()
        for x in legs:
            if len(x) >= maxsz - 1:
                cand |= x
        if not cand:
            for x in legs:
                cand |= x
        cand -= st.open_legs
        best = None
        for l in sorted(cand):
            _, mx, _, sec = tree_cost(st, children, count, sliced | {l})
            key = (mx, sec, l)
            if best is None or key < best[0]:
                best = (key, l)
        if best is None:
            break
        sliced.add(best[1])
    return sorted(sliced)


def order_slices(st: Structure, children, count: VariantCounter, sliced):
    """Slice-id bit order: bit b goes to the leg whose dependent, not yet
    assigned nodes cost least when recomputed every 2^b slices."""
    sliced = list(sliced)
    full, legs, om, sdep = node_sets(st, children, frozenset(sliced))
    L = st.n_leaves
    costs = []
    for i, (a, b) in enumerate(children):
        t = L + i
        allg = (full[a] | full[b]) - frozenset(sliced)
        costs.append((sdep[t], count(om[t]) * 2.0 ** len(allg)))
    order = []
    covered = [False] * len(costs)
    remaining = set(sliced)
    while remaining:
        best = None
        for l in sorted(remaining):
            add = sum(c for j, (dep, c) in enumerate(costs) if not covered[j] and l in dep)
            if best is None or add < best[0]:
                best = (add, l)
        l = best[1]
        order.append(l)
        remaining.discard(l)
        for j, (dep, _) in enumerate(costs):
            if l in dep:
                covered[j] = True
    return order


_ANNEAL_CTX = None


def _anneal_job(job):
    from .optimizer import anneal

    st, count = _ANNEAL_CTX
    return anneal(st, count, **job)


def _run_anneals(st, count, jobs, workers):
    """Runs optimizer.anneal for each job, in order; in forked workers when
    workers > 1 (each restart is independent and seeded)."""
    global _ANNEAL_CTX
    _ANNEAL_CTX = (st, count)
    try:
        if workers > 1 and len(jobs) > 1:
            import multiprocessing as mp

            with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
                return pool.map(_anneal_job, jobs)
        return [_anneal_job(j) for j in jobs]
    finally:
        _ANNEAL_CTX = None


def plan(circ, bitstrings, n_sliced: int = 0, trials: int = 16, seed: int = 0,
         temp: float = 0.3, fuse_1q: bool = True, fold_kets: bool = True,
         objective: str = "time", anneal_steps: int = 0, anneal_restarts: int = 4,
         size_log2_max=None, table_bytes_max=None, workers: int = 1, open_qubits: int = 0,
         anneal_objective: str = "time", alpha: float = 19.7, memory: str = "tables",
         slicing: str = "swap", slice_every: int = 20000, beta: float = 8.0):
    """Returns (children [(a, b), ...], sliced_legs [leg of bit 0, ...], info).

    Every greedy trial tree is sliced and its slice bits ordered; the kept
    trial has the lowest estimated time (objective "time") or the fewest
    complex MACs (objective "cmacs").  With anneal_steps > 0 the local-search
    optimizer (optimizer.anneal) then runs `anneal_restarts` times from the
    kept tree with different seeds, holding the largest tensor at the greedy
    tree's size (or `size_log2_max`), and the best result by estimated time
    under the executor's slice order is returned.  `workers` > 1 runs the
    restarts in that many forked processes (same results as one process; fork
    before the process touches the GPU).  anneal_objective, alpha, memory,
    slicing, slice_every and beta select the optimizer's objective and
    slicing moves (optimizer.anneal); with slicing "paper" the number of
    sliced legs floats and n_sliced only seeds the start."""
    st = Structure(circ, fuse_1q, fold_kets, open_qubits)
    count = VariantCounter(np.asarray(bitstrings, dtype=np.uint64) & ~np.uint64(open_qubits))
    if st.n_leaves == 1:
        return [], [], dict(cost=0.0, max_log2=0, seconds=0.0)
    rng = random.Random(seed)
    best = None
    for t in range(max(trials, 1)):
        ch = greedy_tree(st, count, rng, 0.0 if t == 0 else temp)
        unsliced = tree_cost(st, ch, count)[0]
        sliced = greedy_slices(st, ch, count, n_sliced) if n_sliced else []
        order = order_slices(st, ch, count, sliced) if sliced else []
        total, mx, per_slice, sec = tree_cost(st, ch, count, order, order)
        key = sec if objective == "time" else total
        if best is None or key < best[0]:
            best = (key, ch, order, dict(cost=total, cost_per_slice=per_slice, max_log2=mx,
                                         unsliced_cost=unsliced, seconds=sec, trial=t))
    if anneal_steps > 0:
        ch0, sl0, info0 = best[1], best[2], best[3]
        cap = info0["max_log2"] if size_log2_max is None else size_log2_max
        jobs = [dict(children=ch0, sliced=sl0, steps=anneal_steps, size_log2_max=cap,
                     seed=seed * 1000 + r + 1, mem_max=table_bytes_max, objective=anneal_objective,
                     alpha=alpha, memory=memory, slicing=slicing, slice_every=slice_every,
                     beta=beta)
                for r in range(max(anneal_restarts, 1))]
        for r, (ch, sl, ainfo) in enumerate(_run_anneals(st, count, jobs, workers)):
            order = order_slices(st, ch, count, sl) if sl else []
            total, mx, per_slice, sec = tree_cost(st, ch, count, order, order)
            if table_bytes_max is None:
                better = mx <= cap and sec < best[3]["seconds"]
            else:
                # Prefer fitting the table budget; among trees that do not fit,
                # prefer less table memory (string blocks absorb the rest).
                tb, best_tb = ainfo["table_bytes"], best[3].get("table_bytes", float("inf"))
                fits, best_fits = tb <= table_bytes_max, best_tb <= table_bytes_max
                better = mx <= cap and ((fits and (not best_fits or sec < best[3]["seconds"]))
                                        or (not fits and not best_fits and tb < best_tb))
            if better:
                best = (sec, ch, order, dict(cost=total, cost_per_slice=per_slice, max_log2=mx,
                                             unsliced_cost=tree_cost(st, ch, count)[0],
                                             seconds=sec, trial=info0["trial"], anneal_restart=r,
                                             table_bytes=ainfo["table_bytes"]))
    return best[1], best[2], best[3]


def choose_slicing(circ, bitstrings, memory_budget: int, max_sliced: int = 40, stack: bool = True,
                   precision: str = "c64", trials: int = 8, seed: int = 0, anneal_steps: int = 0,
                   anneal_restarts: int = 4, workers: int = 1, fuse_1q: bool = True,
                   fold_kets: bool = True):
    """The emulation-mode planner (Appendix C: run the memory bookkeeping
    without the tensors): the smallest number of sliced legs s whose plan fits
    `memory_budget` bytes of device workspace, decided by the plan compiler's
    exact host dry run (xeb_plan_create without a device), then the largest
    number of stacked slice bits J <= s that still fits.

    For s = 0, 1, 2, ... the tree and slices come from `plan` (the table
    budget steering the optimizer when anneal_steps > 0); a plan fits when
    the dry run's workspace, after cutting the strings into blocks if it
    must, is within the budget.  Stacking stops short of the J that would
    need more string blocks than the unstacked plan.  Returns a dict with
    the tree (`children`),
    `sliced` legs, `stack_slices`, the dry run's `workspace_bytes` and
    `n_blocks`, the planner's `info`, and `tried`: one record per s tried,
    each with the workspace it needed (None when no block count fits)."""
    tried = []
    for s in range(0, max_sliced + 1):
        ch, sl, info = plan(circ, bitstrings, n_sliced=s, trials=trials, seed=seed,
                            fuse_1q=fuse_1q, fold_kets=fold_kets, anneal_steps=anneal_steps,
                            anneal_restarts=anneal_restarts, workers=workers,
                            table_bytes_max=memory_budget if anneal_steps > 0 else None)
        if len(sl) < s:  # no leg left to slice
            break
        need = None
        try:
            p = _xeb.Plan(circ, bitstrings, ch, sl, fuse_1q=fuse_1q, fold_kets=fold_kets,
                          precision=precision, memory_budget=memory_budget, bind=False)
            st = p.stats()
            need = int(st["workspace_bytes"])
            p.close()
        except _xeb.XebError as e:
            if e.code != _xeb.XEB_ENOMEM:
                raise
        tried.append({"s": s, "workspace_bytes": need})
        if need is None:
            continue
        best = {"children": ch, "sliced": sl, "stack_slices": 0, "workspace_bytes": need,
                "n_blocks": int(st["n_blocks"]), "info": info, "tried": tried}
        if stack:
            J, st = choose_stacking(circ, bitstrings, ch, sl, memory_budget, precision=precision,
                                    max_blocks=best["n_blocks"], fuse_1q=fuse_1q,
                                    fold_kets=fold_kets)
            if J > 0:
                best.update(stack_slices=J, workspace_bytes=int(st["workspace_bytes"]),
                            n_blocks=int(st["n_blocks"]))
        return best
    raise ValueError(f"no slicing up to {max_sliced} legs fits {memory_budget} bytes")


def choose_stacking(circ, bitstrings, children, sliced, memory_budget: int, precision: str = "c64",
                    max_stack: int | None = None, max_blocks: int | None = None,
                    fuse_1q: bool = True, fold_kets: bool = True):
    """The largest number J of stacked slice bits (at most len(sliced), at
    most max_stack, n_qubits + J <= 64) whose plan compiles within
    `memory_budget` with at most `max_blocks` string blocks (default: the
    unstacked plan's count), by the plan compiler's host dry run.  Returns
    (J, the plan's stats); (0, None) when no J > 0 qualifies."""
    if max_blocks is None:
        p = _xeb.Plan(circ, bitstrings, children, sliced, fuse_1q=fuse_1q, fold_kets=fold_kets,
                      precision=precision, memory_budget=memory_budget, bind=False)
        max_blocks = int(p.stats()["n_blocks"])
        p.close()
    top = len(sliced) if max_stack is None else min(len(sliced), max_stack)
    for J in range(top, 0, -1):
        if circ.n_qubits + J > 64:
            continue
        try:
            p = _xeb.Plan(circ, bitstrings, children, sliced, fuse_1q=fuse_1q, fold_kets=fold_kets,
                          precision=precision, memory_budget=memory_budget, stack_slices=J,
                          bind=False)
        except _xeb.XebError as e:
            if e.code != _xeb.XEB_ENOMEM:
                raise
            continue
        st = p.stats()
        p.close()
        if int(st["n_blocks"]) <= max_blocks:
            return J, st
    return 0, None
