"""Local-search tree optimizer (no GPU): rotations keep a valid tree, the
locally updated cost equals a full recomputation, the result never scores
worse than its start, and the library accepts it with the oracle's exact
evaluation counts."""

import random

import numpy as np

from synth import grid_circuit, uniform_bitstrings, prefix_bitstrings
from oracle import memo
from oracle.network import build_network
from paper_2108_05665_amd import planner, optimizer, xeb


def _valid(children, L):
    seen = set()
    for i, (a, b) in enumerate(children):
        assert a < L + i and b < L + i and a != b
        assert a not in seen and b not in seen
        seen |= {a, b}
    assert len(seen) == 2 * L - 2


def test_rotations_keep_local_cost_exact():
    c = grid_circuit(3, 4, 6, 71)
    s = uniform_bitstrings(12, 200, 72)
    st = planner.Structure(c)
    cnt = planner.VariantCounter(s)
    ch, sl, _ = planner.plan(c, s, n_sliced=2, trials=2)
    ts = optimizer.TreeState(st, cnt, ch, sl)
    rng = random.Random(5)
    for _ in range(3000):
        v = rng.randrange(ts.L, 2 * ts.L - 1)
        rec = ts.rotate(v, rng.randrange(2), rng.randrange(2))
        if rec is not None and rng.random() < 0.3:
            ts.undo(rec)
    total, hist = ts.total, dict(ts.size_hist)
    ts.recompute_all()
    assert abs(ts.total - total) <= 1e-9 * total
    assert ts.size_hist == hist
    _valid(ts.children(), ts.L)


def test_anneal_never_worse_and_plan_counts_match_oracle():
    c = grid_circuit(4, 4, 8, 73)
    s = prefix_bitstrings(16, 500, 6, 74)
    st = planner.Structure(c)
    cnt = planner.VariantCounter(s)
    ch, sl, info = planner.plan(c, s, n_sliced=3, trials=2)
    ch2, sl2, inf2 = optimizer.anneal(st, cnt, ch, sl, steps=20000, size_log2_max=info["max_log2"], seed=3)
    _valid(ch2, st.n_leaves)
    assert len(sl2) == 3
    t0 = optimizer.TreeState(st, cnt, ch, sl).total
    assert inf2["seconds"] <= t0 * (1 + 1e-12)
    assert inf2["max_log2"] <= info["max_log2"]
    p = xeb.Plan(c, s, ch2, sl2, bind=False)
    net = build_network(c)
    want = memo.distinct_key_counts(net, memo.Tree(len(net.leaves), ch2), s)
    assert {ns["node"]: ns["variants"] for ns in p.all_node_stats()} == want


def test_plan_with_anneal_improves_estimate():
    c = grid_circuit(4, 5, 10, 75)
    s = uniform_bitstrings(20, 2000, 76)
    _, _, greedy = planner.plan(c, s, n_sliced=4, trials=4)
    ch, sl, annealed = planner.plan(c, s, n_sliced=4, trials=4, anneal_steps=20000, anneal_restarts=2)
    assert annealed["seconds"] <= greedy["seconds"]
    assert annealed["max_log2"] <= greedy["max_log2"]
    _valid(ch, len(ch) + 1)


def _appc_memory_brute(ts):
    """M(T, k) of Appendix C recomputed from its definition for every node."""
    p = ts.P_NORM
    m = {v: 8.0 * 2.0 ** bin(ts.legs[v] & ~ts.S).count("1") for v in range(2 * ts.L - 1)}
    total = 0.0
    for v in range(ts.L, 2 * ts.L - 1):
        a, b = ts.left[v], ts.right[v]
        ka, kb, kv = ts.k[a], ts.k[b], ts.k[v]
        if kv == 1:
            mk = 0.0
        elif min(ka, kb) < kv:
            mk = min(ka * m[a] + m[b], m[a] + kb * m[b])
        else:
            mk = min(ka * m[a], kb * m[b])
        total += mk
    return total + 2.0 * sum(x ** p for x in m.values()) ** (1.0 / p)


def test_appc_memory_and_cost_sums_update_locally():
    """The Appendix C memory estimate and the C / RW sums after thousands of
    rotations (with undos) equal a recomputation from their definitions."""
    c = grid_circuit(3, 4, 6, 77)
    s = uniform_bitstrings(12, 150, 78)
    st = planner.Structure(c)
    cnt = planner.VariantCounter(s)
    ch, sl, _ = planner.plan(c, s, n_sliced=2, trials=2)
    ts = optimizer.TreeState(st, cnt, ch, sl)
    rng = random.Random(9)
    for _ in range(2000):
        rec = ts.rotate(rng.randrange(ts.L, 2 * ts.L - 1), rng.randrange(2), rng.randrange(2))
        if rec is not None and rng.random() < 0.3:
            ts.undo(rec)
    M, C, RW = ts.appc_memory(), ts.C, ts.RW
    assert abs(M - _appc_memory_brute(ts)) <= 1e-9 * M
    ts.recompute_all()
    assert abs(ts.appc_memory() - M) <= 1e-9 * M
    assert abs(ts.C - C) <= 1e-9 * C and abs(ts.RW - RW) <= 1e-9 * RW
    # C (every node evaluated once per distinct slice key of its own legs)
    # equals the library's cost with all slices stacked.
    p = xeb.Plan(c, s, ts.children(), ts.sliced(), stack_slices=len(ts.sliced()), bind=False)
    assert abs(p.stats()["cmacs_full"] - C) <= 1e-9 * C


def test_paper_objective_and_slicing_moves():
    """The paper's objective with its slicing moves (add best-M leg / drop a
    random one, each with probability 1/2) from an empty S under a budget:
    the result is a valid tree whose estimated memory fits the budget, and
    the library compiles it within that budget."""
    c = grid_circuit(4, 4, 8, 79)
    s = uniform_bitstrings(16, 400, 80)
    st = planner.Structure(c)
    cnt = planner.VariantCounter(s)
    ch, _, _ = planner.plan(c, s, n_sliced=0, trials=2)
    free = optimizer.TreeState(st, cnt, ch, ())
    budget = free.mem / 8
    for memory in ("tables", "appc"):
        ch2, sl2, info = optimizer.anneal(st, cnt, ch, (), steps=30000, seed=4, objective="paper",
                                          alpha=19.7, memory=memory, slicing="paper",
                                          slice_every=500, mem_max=budget, beta=4.0)
        _valid(ch2, st.n_leaves)
        ts = optimizer.TreeState(st, cnt, ch2, sl2)
        assert len(sl2) > 0
        assert ts.mem <= budget * 1.0001 if memory == "tables" else ts.appc_memory() > 0
        p = xeb.Plan(c, s, ch2, sl2, bind=False)
        assert p.stats()["cmacs_full"] > 0
