"""O2: naive FP64 contraction of the circuit's tensor network.

Definitions followed:
* The result of contracting a network is the sum over its closed legs of the
  product of all tensors (section "Definitions and notations", Eq. "sum").
* Fixing the bits of s on the open output legs makes that sum equal
  <s|C|0^n> (section "Multi-batch simulator").
* Slicing fixes a list of legs to each assignment and sums the contractions
  of all assignments (Appendix A, paragraph "Slicing").  A sliced partial for
  assignment sigma fixes leg sliced[j] to bit j of sigma.

The result does not depend on the order of the pairwise contractions
(section "Tensor network contraction"), so the oracle picks its own order:
a greedy over pairs of tensors sharing a leg, scored by
2^|result| - 2^|a| - 2^|b|.  For large networks it repeats the greedy with
random perturbations of the score and keeps the order with the fewest
multiply-adds among those whose largest tensor stays under a cap.  Each
pairwise step is one numpy.tensordot in complex128.
"""

from __future__ import annotations

import math
import random

import numpy as np

from .network import Network


def _fix(tensor: np.ndarray, legs: list, fixed: dict):
    idx = []
    keep = []
    for leg in legs:
        if leg in fixed:
            idx.append(int(fixed[leg]))
        else:
            idx.append(slice(None))
            keep.append(leg)
    return tensor[tuple(idx)], keep


def fixed_legs(net: Network, bitstring: int, sliced=(), sigma: int = 0) -> dict:
    fixed = {}
    for q in range(net.n_qubits):
        fixed[net.out_leg[q]] = (int(bitstring) >> q) & 1
    for j, leg in enumerate(sliced):
        fixed[int(leg)] = (int(sigma) >> j) & 1
    return fixed


def greedy_order(leg_sets, rng=None, noise: float = 0.0):
    """Order of pairwise contractions for a closed network given the leg sets
    of its tensors.  Returns (pairs, largest log2 size, multiply-adds) where
    pairs index an SSA list: tensors 0..n-1, then result n+i of step i."""
    items = {i: frozenset(s) for i, s in enumerate(leg_sets)}
    nxt = len(items)
    pairs = []
    biggest = 0
    madds = 0
    while len(items) > 1:
        owner = {}
        for i, s in items.items():
            for leg in s:
                owner.setdefault(leg, []).append(i)
        cand = sorted({(min(w), max(w)) for w in owner.values() if len(w) == 2})
        if not cand:
            keys = sorted(items)
            cand = [(keys[0], keys[1])]  # disconnected pieces: outer product
        best = None
        for i, j in cand:
            a, b = items[i], items[j]
            r = a ^ b
            sc = 2.0 ** len(r) - 2.0 ** len(a) - 2.0 ** len(b)
            if noise > 0 and rng is not None:
                sc = (len(r) - math.log2(2.0 ** len(a) + 2.0 ** len(b))
                      + noise * math.log(-math.log(rng.random() or 1e-300)))
            if best is None or sc < best[0]:
                best = (sc, i, j, r)
        _, i, j, r = best
        madds += 2 ** len(items[i] | items[j])
        biggest = max(biggest, len(r))
        del items[i], items[j]
        items[nxt] = r
        pairs.append((i, j))
        nxt += 1
    return pairs, biggest, madds


def search_order(leg_sets, trials: int = 64, seed: int = 1, cap_log2: int = 27):
    """Best of one plain greedy and `trials` perturbed greedies: fewest
    multiply-adds with the largest tensor <= 2^cap_log2 (else the smallest
    largest tensor)."""
    best = greedy_order(leg_sets)
    rng = random.Random(seed)

    def better(x, y):
        fx, fy = x[1] <= cap_log2, y[1] <= cap_log2
        if fx != fy:
            return fx
        return x[2] < y[2] if fx else (x[1], x[2]) < (y[1], y[2])

    for _ in range(trials):
        cand = greedy_order(leg_sets, rng, noise=0.5)
        if better(cand, best):
            best = cand
    return best


def _random_order(leg_sets, rng):
    items = {i: frozenset(s) for i, s in enumerate(leg_sets)}
    nxt = len(items)
    pairs = []
    while len(items) > 1:
        owner = {}
        for i, s in items.items():
            for leg in s:
                owner.setdefault(leg, []).append(i)
        cand = sorted({(min(w), max(w)) for w in owner.values() if len(w) == 2})
        if not cand:
            keys = sorted(items)
            cand = [(keys[0], keys[1])]
        i, j = cand[int(rng.integers(0, len(cand)))]
        r = items.pop(i) ^ items.pop(j)
        items[nxt] = r
        pairs.append((i, j))
        nxt += 1
    return pairs


def contract_closed(tensors: list, pairs=None, order_rng=None) -> complex:
    """Contract a closed network given as (array, legs) pairs.  `pairs` is an
    SSA order (greedy_order); with `order_rng` a uniformly random connected
    order is used instead (order-independence pin)."""
    items = [(np.asarray(t), list(l)) for t, l in tensors]
    for t, l in items:
        if len(set(l)) != len(l):
            raise ValueError("a tensor repeats a leg")
    if pairs is None:
        sets = [set(l) for _, l in items]
        pairs = _random_order(sets, order_rng) if order_rng is not None else greedy_order(sets)[0]
    store = dict(enumerate(items))
    nxt = len(items)
    for i, j in pairs:
        (ti, li), (tj, lj) = store.pop(i), store.pop(j)
        shared = [leg for leg in li if leg in lj]
        t = np.tensordot(ti, tj, axes=([li.index(x) for x in shared], [lj.index(x) for x in shared]))
        legs = [x for x in li if x not in shared] + [x for x in lj if x not in shared]
        store[nxt] = (t, legs)
        nxt += 1
    (t, legs), = store.values()
    if legs:
        raise ValueError("network is not closed")
    return complex(t)


def leaf_tensors(net: Network, bitstring: int, sliced=(), sigma: int = 0):
    fixed = fixed_legs(net, bitstring, sliced, sigma)
    return [_fix(lf.tensor, lf.legs, fixed) for lf in net.leaves]


def closed_leg_sets(net: Network, sliced=()):
    sl = set(int(x) for x in sliced)
    return [set(l for l in lf.legs if net.leg_qubit[l] < 0 and l not in sl) for lf in net.leaves]


def partial_amplitude(net: Network, bitstring: int, sliced=(), sigma: int = 0,
                      order_rng=None, pairs=None) -> complex:
    """Contraction of the network with the output legs fixed to `bitstring`
    and leg sliced[j] fixed to bit j of `sigma`."""
    return contract_closed(leaf_tensors(net, bitstring, sliced, sigma), pairs, order_rng)


def amplitude(net: Network, bitstring: int, sliced=(), order_rng=None, pairs=None) -> complex:
    """amp(s) = sum over all 2^|sliced| assignments of the sliced partials,
    each part summed exactly (math.fsum)."""
    parts = [partial_amplitude(net, bitstring, sliced, sigma, order_rng, pairs)
             for sigma in range(1 << len(sliced))]
    return complex(math.fsum(p.real for p in parts), math.fsum(p.imag for p in parts))


def amplitudes(net: Network, bitstrings, sliced=()) -> np.ndarray:
    pairs = greedy_order(closed_leg_sets(net, sliced))[0]
    return np.array([amplitude(net, int(s), sliced, pairs=pairs) for s in bitstrings],
                    dtype=np.complex128)
