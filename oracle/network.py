"""Tensor network of a quantum circuit (oracle side).

Follows the paper's section "Multi-batch simulator": a circuit becomes a
tensor network with one open leg per qubit (its output), gate fusion is a
standard simplification assumed already applied, and fixing the bits of a
string on the open legs gives the network whose contraction is <s|C|0^n>.

The network convention (shared by definition, implemented independently by
the library):

1. Fusion (when `fuse_1q`): walk the gates in time order with a pending
   single-qubit product P_q per qubit.  A one-qubit gate U on q sets
   P_q := U P_q.  A two-qubit gate W on (a, b) is emitted as W (P_a (x) P_b)
   (absent P = identity) and clears P_a, P_b.  After the walk, every qubit q
   (ascending id) with a pending P_q either left-multiplies it into the last
   emitted two-qubit gate touching q, on q's side, or, if no two-qubit gate
   touches q, is emitted as a one-qubit gate.  Without fusion the emitted
   list is the gate list itself.
2. Leaves: ket leaves first, then one leaf per emitted gate in order.  With
   `fold_kets` the kets are projected into the first gate on each qubit and a
   ket leaf exists only for a qubit that no emitted gate touches; without it
   every qubit has a ket leaf (ascending qubit id).
3. Legs are wire segments numbered in creation order: ket segments first
   (ascending qubit id), then for each emitted gate one new output segment
   per qubit it acts on (first qubit's, then second qubit's).
4. A gate leaf's legs are its input segments (first qubit's, then second's;
   an input still in the initial state under `fold_kets` is dropped, i.e.
   projected onto |0>), followed by its output segments.  Its entries are
   T[inputs..., outputs...] = U[2 o0 + o1, 2 i0 + i1] (U[o, i] for one qubit).
5. The last segment of each qubit is its open output leg.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Leaf:
    legs: list          # leg ids, in tensor axis order
    tensor: np.ndarray  # complex128, one axis of size 2 per leg
    kind: str           # "ket" or "gate"


@dataclass
class Network:
    n_qubits: int
    leaves: list        # list[Leaf]
    n_legs: int
    out_leg: list       # out_leg[q] = leg id of qubit q's output
    leg_qubit: list     # leg_qubit[l] = q if l is q's output leg, else -1

    def leaf_legs(self):
        return [list(lf.legs) for lf in self.leaves]


def _emitted_gates(circ, fuse_1q: bool):
    n = circ.n_qubits
    out = []  # list of [qubits tuple, matrix]
    if not fuse_1q:
        for g in range(circ.n_gates):
            a, b = (int(x) for x in circ.gate_qubits[g])
            out.append([(a,) if b < 0 else (a, b), circ.matrix(g).copy()])
        return out
    pend = [None] * n
    last2 = [-1] * n
    eye = np.eye(2, dtype=np.complex128)
    for g in range(circ.n_gates):
        a, b = (int(x) for x in circ.gate_qubits[g])
        u = circ.matrix(g)
        if b < 0:
            pend[a] = u if pend[a] is None else u @ pend[a]
        else:
            pa = eye if pend[a] is None else pend[a]
            pb = eye if pend[b] is None else pend[b]
            out.append([(a, b), u @ np.kron(pa, pb)])
            pend[a] = pend[b] = None
            last2[a] = last2[b] = len(out) - 1
    for q in range(n):
        if pend[q] is None:
            continue
        if last2[q] >= 0:
            qs, w = out[last2[q]]
            side = np.kron(pend[q], eye) if q == qs[0] else np.kron(eye, pend[q])
            out[last2[q]][1] = side @ w
        else:
            out.append([(q,), pend[q]])
    return out


def build_network(circ, fuse_1q: bool = True, fold_kets: bool = True) -> Network:
    n = circ.n_qubits
    gates = _emitted_gates(circ, fuse_1q)
    touched = set()
    for qs, _ in gates:
        touched.update(qs)
    leaves = []
    wire = [None] * n   # current segment of each qubit (None = initial state, folded)
    n_legs = 0
    for q in range(n):
        if (not fold_kets) or (q not in touched):
            leaves.append(Leaf([n_legs], np.array([1.0, 0.0], dtype=np.complex128), "ket"))
            wire[q] = n_legs
            n_legs += 1
    for qs, u in gates:
        k = len(qs)
        t = u.reshape((2,) * (2 * k))   # axes: outs..., ins...
        t = np.transpose(t, list(range(k, 2 * k)) + list(range(k)))  # ins..., outs...
        in_legs = []
        idx = []
        for j, q in enumerate(qs):
            if wire[q] is None:
                idx.append(0)       # folded ket: project the input onto |0>
            else:
                idx.append(slice(None))
                in_legs.append(wire[q])
        t = t[tuple(idx) + (slice(None),) * k]
        out_legs = []
        for q in qs:
            wire[q] = n_legs
            out_legs.append(n_legs)
            n_legs += 1
        leaves.append(Leaf(in_legs + out_legs, np.ascontiguousarray(t), "gate"))
    leg_qubit = [-1] * n_legs
    for q in range(n):
        leg_qubit[wire[q]] = q
    return Network(n, leaves, n_legs, list(wire), leg_qubit)
