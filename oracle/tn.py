"""O2: naive FP64 contraction of the circuit's tensor network.

Definitions followed:
* The result of contracting a network is the sum over its closed legs of the
  product of all tensors (section "Definitions and notations", Eq. "sum").
* Fixing the bits of s on the open output legs makes that sum equal
  <s|C|0^n> (section "Multi-batch simulator").
* Slicing fixes a list of legs to each assignment and sums the contractions
  of all assignments (Appendix A, paragraph "Slicing").  A sliced partial for
  assignment sigma fixes leg sliced[j] to bit j of sigma.

The contraction order is the oracle's own: repeatedly contract the pair of
tensors sharing a leg whose result is smallest (ties: the pair with the
smallest tensor indices), then multiply the scalars of disconnected pieces.
The result does not depend on that order (section "Tensor network
contraction"), so any order checks any other.  Each pairwise step is one
numpy.tensordot in complex128.
"""

from __future__ import annotations

import math

import numpy as np

from .network import Network


def _fix(tensor: np.ndarray, legs: list, fixed: dict):
    idx = []
    keep = []
    for ax, leg in enumerate(legs):
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


def contract_closed(tensors: list, order_rng=None) -> complex:
    """Contract a list of (array, legs) whose legs each appear exactly twice
    (closed network).  With `order_rng` the next pair is drawn at random among
    the connected pairs instead of the greedy choice (order-independence pin).
    """
    items = [(np.asarray(t), list(l)) for t, l in tensors]
    scalar = complex(1.0)
    while True:
        # Absorb scalars immediately.
        rest = []
        for t, l in items:
            if not l:
                scalar *= complex(t)
            else:
                rest.append((t, l))
        items = rest
        if not items:
            return scalar
        owner = {}
        for i, (_, l) in enumerate(items):
            for leg in l:
                owner.setdefault(leg, []).append(i)
        pairs = set()
        for leg, who in owner.items():
            if len(who) == 2 and who[0] != who[1]:
                pairs.add((min(who), max(who)))
            elif len(who) != 2:
                raise ValueError(f"leg {leg} is not closed")
        if not pairs:
            # A tensor with a leg appearing twice on itself would be a trace;
            # the circuit networks never produce one.
            raise ValueError("no contractible pair")
        if order_rng is not None:
            cand = sorted(pairs)
            i, j = cand[int(order_rng.integers(0, len(cand)))]
        else:
            best = None
            for i, j in sorted(pairs):
                li, lj = set(items[i][1]), set(items[j][1])
                size = len(li ^ lj)
                if best is None or size < best[0]:
                    best = (size, i, j)
            _, i, j = best
        (ti, li), (tj, lj) = items[i], items[j]
        shared = [leg for leg in li if leg in lj]
        ai = [li.index(leg) for leg in shared]
        aj = [lj.index(leg) for leg in shared]
        t = np.tensordot(ti, tj, axes=(ai, aj))
        legs = [leg for leg in li if leg not in shared] + [leg for leg in lj if leg not in shared]
        items = [it for k, it in enumerate(items) if k not in (i, j)] + [(t, legs)]


def partial_amplitude(net: Network, bitstring: int, sliced=(), sigma: int = 0,
                      order_rng=None) -> complex:
    """Contraction of the network with the output legs fixed to `bitstring`
    and leg sliced[j] fixed to bit j of `sigma`."""
    fixed = fixed_legs(net, bitstring, sliced, sigma)
    tensors = [_fix(lf.tensor, lf.legs, fixed) for lf in net.leaves]
    return contract_closed(tensors, order_rng)


def amplitude(net: Network, bitstring: int, sliced=(), order_rng=None) -> complex:
    """amp(s) = sum over all 2^|sliced| assignments of the sliced partials,
    each part summed exactly (math.fsum)."""
    parts = [partial_amplitude(net, bitstring, sliced, sigma, order_rng)
             for sigma in range(1 << len(sliced))]
    return complex(math.fsum(p.real for p in parts), math.fsum(p.imag for p in parts))


def amplitudes(net: Network, bitstrings, sliced=()) -> np.ndarray:
    return np.array([amplitude(net, int(s), sliced) for s in bitstrings],
                    dtype=np.complex128)
