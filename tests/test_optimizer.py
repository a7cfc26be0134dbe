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
