"""O3: linear cross-entropy benchmark fidelity (Eq. 1 of the Introduction).

F_XEB = (2^n / k) * sum_{i=1..k} p_C(s_i) - 1, p_C(s) = |<s|C|0^n>|^2, the
sum running over the k sampled strings with multiplicity.  Sums are exactly
rounded (math.fsum), so the result is the FP64 rounding of the exact value
for the given amplitudes.
"""

from __future__ import annotations

import math

import numpy as np


def xeb_fidelity(n_qubits: int, amps) -> float:
    a = np.asarray(amps, dtype=np.complex128)
    k = a.shape[0]
    if k == 0:
        raise ValueError("XEB needs at least one sample")
    p = [float(x.real) ** 2 + float(x.imag) ** 2 for x in a]
    # Scale after the exact sum: 2^n / k is applied once.
    s = math.fsum(p)
    return math.ldexp(s, n_qubits) / k - 1.0


def ideal_xeb(psi) -> float:
    """Expectation of F_XEB when the strings are drawn from p_C itself:
    E[F] = 2^n * sum_s p(s)^2 - 1 (the sum over every basis state)."""
    p = np.abs(np.asarray(psi)) ** 2
    n = int(round(math.log2(p.size)))
    return math.ldexp(math.fsum((p * p).tolist()), n) - 1.0
