"""Pins for the FP64 oracle (no GPU): closed forms, the paper's worked example,
invariants and brute force.  Each pin is chosen so that a plausible slip in the
oracle (a transposed gate, a wrong qubit order, a dropped slice term, a wrong
fusion side, a stale cache entry) fails at least one of them."""

import json
import math
import os

import numpy as np
import pytest

from synth import grid_circuit, worked_example_circuit, uniform_bitstrings
from synth.circuits import _Builder, SQRT_X, SQRT_Y, FSIM, CNOT
from oracle import statevec, tn, xeb, memo
from oracle.network import build_network

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_gate_state(n, gates):
    b = _Builder(n)
    for g in gates:
        if len(g) == 2:
            b.g1(g[0], g[1])
        else:
            b.g2(g[0], g[1], g[2])
    return statevec.state_vector(b.build({}))


X = np.array([[0, 1], [1, 0]], dtype=np.complex128)


# ---- O1: closed forms --------------------------------------------------------

def test_sqrt_x_on_zero():
    psi = one_gate_state(1, [(0, SQRT_X)])
    assert np.allclose(psi, [(1 + 1j) / 2, (1 - 1j) / 2], atol=1e-15)


def test_sqrt_y_on_zero_not_symmetric():
    # sqrt(Y) is not symmetric: a transposed matrix would give ((1+i)/2, (-1-i)/2... )
    psi = one_gate_state(1, [(0, SQRT_Y)])
    assert np.allclose(psi, [(1 + 1j) / 2, (1 + 1j) / 2], atol=1e-15)


def test_fsim_action():
    # basis index 2*b_q0 + b_q1; state index sum_q b_q 2^q.
    # |q0=0,q1=1> -> -i |q0=1,q1=0>
    psi = one_gate_state(2, [(1, X), (0, 1, FSIM)])
    want = np.zeros(4, complex)
    want[1] = -1j  # q0=1 -> state index 1
    assert np.allclose(psi, want, atol=1e-15)
    # |11> -> exp(-i pi/6) |11>
    psi = one_gate_state(2, [(0, X), (1, X), (0, 1, FSIM)])
    want = np.zeros(4, complex)
    want[3] = complex(math.cos(math.pi / 6), -math.sin(math.pi / 6))
    assert np.allclose(psi, want, atol=1e-15)


def test_cnot_orientation_and_qubit_order():
    psi = one_gate_state(2, [(0, X), (0, 1, CNOT)])      # control q0 = 1 -> flips q1
    assert abs(psi[3] - 1) < 1e-15
    psi = one_gate_state(2, [(1, X), (0, 1, CNOT)])      # control q0 = 0 -> unchanged
    assert abs(psi[2] - 1) < 1e-15


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_unitarity(seed):
    c = grid_circuit(3, 4, 6, seed)
    psi = statevec.state_vector(c)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12


# ---- the paper's worked example (Appendix B) ---------------------------------

def _golden():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        return json.load(f)


def _golden_amp(g, s):
    return g["amplitude_signs_q0_first"][s] / (2 * math.sqrt(2))


def _parse(s):
    return sum(int(ch) << q for q, ch in enumerate(s))


def test_worked_example_state_vector():
    g = _golden()
    psi = statevec.state_vector(worked_example_circuit())
    for s in g["amplitude_signs_q0_first"]:
        assert abs(psi[_parse(s)] - _golden_amp(g, s)) < 1e-15


def test_worked_example_network_shape():
    # The figure's network: kets X0..X2, gates X3..X8, 8 internal legs + 3 open.
    net = build_network(worked_example_circuit(), fuse_1q=False, fold_kets=False)
    assert len(net.leaves) == 9
    assert net.n_legs == 11
    sizes = [len(lf.legs) for lf in net.leaves]
    assert sizes == [1, 1, 1, 2, 2, 4, 4, 2, 2]
    # Output legs sit on X7 (q0), X8 (q1) and X6 (q2).
    holder = {q: [j for j, lf in enumerate(net.leaves) if net.out_leg[q] in lf.legs] for q in range(3)}
    assert holder == {0: [7], 1: [8], 2: [6]}


@pytest.mark.parametrize("fuse,fold", [(False, False), (True, True), (False, True), (True, False)])
def test_worked_example_tn(fuse, fold):
    g = _golden()
    net = build_network(worked_example_circuit(), fuse_1q=fuse, fold_kets=fold)
    for s in g["amplitude_signs_q0_first"]:
        a = tn.amplitude(net, _parse(s))
        assert abs(a - _golden_amp(g, s)) < 1e-15


def test_worked_example_memo_counts_and_amps():
    g = _golden()
    net = build_network(worked_example_circuit(), fuse_1q=False, fold_kets=False)
    tree = memo.Tree(9, g["tree_children"])
    strings = [_parse(s) for s in g["strings_q0_first"]]
    amps, counts = memo.memo_amplitudes(net, tree, strings)
    for s, a in zip(g["strings_q0_first"], amps):
        assert abs(a - _golden_amp(g, s)) < 1e-15
    want = {int(k): v for k, v in g["node_counts"].items()}
    assert counts == want
    assert sum(counts.values()) == g["total_contractions_memo"]
    assert len(counts) * len(strings) == g["total_contractions_single_amplitude_runs"]
    assert memo.distinct_key_counts(net, tree, strings) == want


# ---- O2 against O1 ----------------------------------------------------------

@pytest.mark.parametrize("fuse,fold", [(True, True), (False, False), (True, False), (False, True)])
def test_tn_equals_state_vector(fuse, fold):
    c = grid_circuit(3, 3, 5, 11)
    psi = statevec.state_vector(c)
    net = build_network(c, fuse_1q=fuse, fold_kets=fold)
    for s in uniform_bitstrings(c.n_qubits, 6, 5):
        assert abs(tn.amplitude(net, int(s)) - psi[int(s)]) < 1e-12


def test_tn_random_orders_agree():
    c = grid_circuit(3, 3, 6, 12)
    net = build_network(c)
    rng = np.random.Generator(np.random.PCG64(3))
    s = int(uniform_bitstrings(9, 1, 4)[0])
    a0 = tn.amplitude(net, s)
    for _ in range(3):
        assert abs(tn.amplitude(net, s, order_rng=rng) - a0) < 1e-12


def test_slice_sum_equals_unsliced():
    c = grid_circuit(3, 3, 6, 13)
    net = build_network(c)
    psi = statevec.state_vector(c)
    internal = [l for l in range(net.n_legs) if net.leg_qubit[l] < 0]
    rng = np.random.Generator(np.random.PCG64(8))
    sliced = [int(x) for x in rng.choice(internal, size=4, replace=False)]
    for s in uniform_bitstrings(9, 3, 9):
        a = tn.amplitude(net, int(s), sliced)
        assert abs(a - psi[int(s)]) < 1e-12
        # A dropped slice term must show: the partials are not all equal to the sum.
        parts = [tn.partial_amplitude(net, int(s), sliced, sg) for sg in range(16)]
        assert max(abs(p - a) for p in parts) > 1e-6


# ---- O3 ---------------------------------------------------------------------

def test_xeb_all_strings_is_zero():
    c = grid_circuit(2, 4, 5, 21)
    psi = statevec.state_vector(c)
    assert abs(xeb.xeb_fidelity(8, psi)) < 1e-12


def test_xeb_uniform_and_ideal_samples():
    c = grid_circuit(3, 4, 8, 22)
    n = c.n_qubits
    psi = statevec.state_vector(c)
    p = np.abs(psi) ** 2
    k = 4000
    # uniform strings: E[F] = 0
    us = uniform_bitstrings(n, k, 23).astype(np.int64)
    f_u = xeb.xeb_fidelity(n, psi[us])
    sd_u = np.std((2 ** n) * p[us]) / math.sqrt(k)
    assert abs(f_u) < 5 * sd_u
    # strings drawn from p: E[F] = 2^n sum p^2 - 1
    rng = np.random.Generator(np.random.PCG64(24))
    ideal = rng.choice(p.size, size=k, p=p / p.sum())
    f_i = xeb.xeb_fidelity(n, psi[ideal])
    sd_i = np.std((2 ** n) * p[ideal]) / math.sqrt(k)
    assert abs(f_i - xeb.ideal_xeb(psi)) < 5 * sd_i
    assert f_i > 0.5  # deep enough for a clear signal


def test_xeb_multiplicity():
    # duplicates count with multiplicity: F over [a, a, b] != F over [a, b]
    a = np.array([0.5, 0.5, 0.1], dtype=np.complex128)
    assert xeb.xeb_fidelity(2, a) != xeb.xeb_fidelity(2, a[1:])
    assert abs(xeb.xeb_fidelity(2, a) - (4 * (0.25 + 0.25 + 0.01) / 3 - 1)) < 1e-15


# ---- O4 ---------------------------------------------------------------------

def _greedy_tree_for_test(net, seed):
    """A random (connected-pair) tree; only the structure matters here."""
    rng = np.random.Generator(np.random.PCG64(seed))
    act = {i: set(l for l in lf.legs if net.leg_qubit[l] < 0) for i, lf in enumerate(net.leaves)}
    nxt = len(net.leaves)
    ch = []
    while len(act) > 1:
        keys = sorted(act)
        pairs = [(a, b) for i, a in enumerate(keys) for b in keys[i + 1:] if act[a] & act[b]]
        if not pairs:
            pairs = [(keys[0], keys[1])]
        a, b = pairs[int(rng.integers(0, len(pairs)))]
        act[nxt] = act.pop(a) ^ act.pop(b)
        ch.append((a, b))
        nxt += 1
    return memo.Tree(len(net.leaves), ch)


def test_memo_counts_properties_and_amplitudes():
    c = grid_circuit(2, 4, 4, 31)
    n = c.n_qubits
    net = build_network(c)
    tree = _greedy_tree_for_test(net, 5)
    psi = statevec.state_vector(c)
    # all strings equal -> every node once
    cnt = memo.distinct_key_counts(net, tree, [5] * 7)
    assert set(cnt.values()) == {1}
    # all 2^n strings -> 2^(#output legs under T)
    alls = list(range(1 << n))
    cnt = memo.distinct_key_counts(net, tree, alls)
    for t, v in cnt.items():
        nout = sum(1 for j in tree.leaves_dfs(t) for l in net.leaves[j].legs if net.leg_qubit[l] >= 0)
        assert v == 2 ** nout
    # some strings: the bound and the direct run of Algorithms 3-4
    strings = [int(x) for x in uniform_bitstrings(n, 20, 32)]
    cnt = memo.distinct_key_counts(net, tree, strings)
    k = len(set(strings))
    bits = memo.leaf_key_bits(net, ())

    def k_of(t):
        if tree.is_leaf(t):
            return len({memo.leaf_key(bits[t], s, 0) for s in strings})
        return cnt[t]

    for t, v in cnt.items():
        a, b = tree.kids(t)
        assert v <= min(k_of(a) * k_of(b), k)
    amps, runs = memo.memo_amplitudes(net, tree, strings)
    assert runs == cnt
    assert np.max(np.abs(amps - psi[np.array(strings)])) < 1e-12


def test_memo_with_slices():
    c = grid_circuit(2, 3, 5, 41)
    net = build_network(c)
    tree = _greedy_tree_for_test(net, 6)
    psi = statevec.state_vector(c)
    internal = [l for l in range(net.n_legs) if net.leg_qubit[l] < 0]
    sliced = internal[2:5]
    strings = [int(x) for x in uniform_bitstrings(6, 9, 42)]
    amps, runs = memo.memo_amplitudes(net, tree, strings, sliced)
    assert np.max(np.abs(amps - psi[np.array(strings)])) < 1e-12
    assert runs == memo.distinct_key_counts(net, tree, strings, sliced, range(8))


def test_search_order_reproduces_state_vector():
    """tn.search_order (the plain greedy and its perturbed variants, best under
    a size cap) returns a valid order whose contraction equals the state
    vector on a 20-qubit network, unsliced and summed over slices; the
    perturbed branch alone (greedy_order with noise) is checked the same way."""
    import random

    c = grid_circuit(4, 5, 6, 51)
    net = build_network(c)
    psi = statevec.state_vector(c)
    internal = [l for l in range(net.n_legs) if net.leg_qubit[l] < 0]
    rng = np.random.Generator(np.random.PCG64(52))
    sliced = [int(x) for x in rng.choice(internal, size=3, replace=False)]
    strings = [int(x) for x in uniform_bitstrings(20, 3, 53)]
    for sl in ((), sliced):
        sets = tn.closed_leg_sets(net, sl)
        for pairs, big, madds in (tn.search_order(sets, trials=16, cap_log2=12),
                                  tn.greedy_order(sets, random.Random(7), noise=0.5)):
            # an SSA order: every tensor consumed exactly once, one result left
            used = [x for p in pairs for x in p]
            assert len(used) == len(set(used)) == 2 * (len(sets) - 1)
            assert set(used) == set(range(2 * len(sets) - 2))
            for s in strings:
                a = tn.amplitude(net, s, sl, pairs=pairs)
                assert abs(a - psi[s]) < 1e-12


def test_medium_golden_amplitudes_cross_check():
    """The stored 36-qubit oracle amplitudes (tests/golden/medium_6x6_m12_amps64.json,
    written by tests/golden/make_medium_amps.py): one of its O2 cross-check
    partials recomputed here in the oracle's own greedy order, independent of
    the plan's tree, equals both stored values; every stored amplitude is
    finite and nonzero, and the strings are the workload's first 64."""
    import json
    import os

    from synth import config_circuit, config_bitstrings

    with open(os.path.join(GOLDEN, "medium_6x6_m12_amps64.json")) as f:
        gold = json.load(f)
    circ = config_circuit("medium_6x6_m12")
    strings = config_bitstrings("medium_6x6_m12", circ.n_qubits)
    assert gold["strings"] == [str(int(s)) for s in strings[:64]]
    amps = np.array([complex(re, im) for re, im in gold["amps"]])
    assert np.all(np.isfinite(amps)) and np.all(np.abs(amps) > 0)
    net = build_network(circ)
    sl = gold["sliced_legs"]
    chk = gold["o2_cross_checks"][0]
    pairs = tn.search_order(tn.closed_leg_sets(net, sl), trials=8)[0]
    o2 = tn.partial_amplitude(net, int(strings[chk["string_index"]]), sl, chk["sigma"], pairs=pairs)
    for stored in (chk["o2"], chk["memo"]):
        assert abs(o2 - complex(*stored)) <= 1e-12 * abs(o2)
