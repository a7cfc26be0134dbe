"""O1: dense FP64 state-vector simulation (the plain definition of an amplitude).

amp(s) = <s|C|0^n> (section "Introduction", the probability p_C(s) = |amp|^2
that linear XEB averages).  The state starts as e_0 and each gate in time
order multiplies the amplitudes of the qubits it acts on; the basis index is
sum_q s_q 2^q (qubit 0 is the least significant bit) and a two-qubit matrix
is indexed by 2*b_{q0} + b_{q1}.  Memory is 16 * 2^n bytes: n <= 28 here.
"""

from __future__ import annotations

import numpy as np


def _axis(n: int, q: int) -> int:
    # state reshaped to (2,)*n in C order: axis 0 is the most significant bit,
    # so qubit q (bit q) is axis n-1-q.
    return n - 1 - q


def state_vector(circ) -> np.ndarray:
    n = circ.n_qubits
    if n > 28:
        raise ValueError("state vector limited to n <= 28")
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    psi = psi.reshape((2,) * n)
    for g in range(circ.n_gates):
        a, b = (int(x) for x in circ.gate_qubits[g])
        if b < 0:
            u = circ.matrix(g)
            ax = _axis(n, a)
            psi = np.moveaxis(np.tensordot(u, psi, axes=([1], [ax])), 0, ax)
        else:
            u = circ.matrix(g).reshape(2, 2, 2, 2)  # (o_a, o_b, i_a, i_b)
            xa, xb = _axis(n, a), _axis(n, b)
            psi = np.tensordot(u, psi, axes=([2, 3], [xa, xb]))
            psi = np.moveaxis(psi, [0, 1], [xa, xb])
    return psi.reshape(-1)


def amplitudes(circ, bitstrings) -> np.ndarray:
    psi = state_vector(circ)
    idx = np.asarray(bitstrings, dtype=np.uint64).astype(np.int64)
    return psi[idx]
