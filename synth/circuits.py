"""Random grid circuits and the three-qubit worked example, as explicit FP64 gate lists.

Circuit model (the paper defers the gate set to Google's ABCD supremacy
circuits; the readings below are the ones this repository fixes):

* Qubits sit on an R x C grid, id q = r*C + c, with optional removed sites
  (ids are then renumbered densely in row-major order).
* Cycle c (0-based) applies a single-qubit layer and then a coupler layer:
  - each qubit draws a gate from {sqrt(X), sqrt(Y), sqrt(W)}, W = (X+Y)/sqrt(2);
    in cycle 0 the draw is uniform over the three, afterwards uniform over the
    two that differ from the qubit's previous gate;
  - fSim(theta=pi/2, phi=pi/6) acts on every coupler of pattern
    PATTERN[c mod len(PATTERN)], PATTERN = "ABCDCDAB".
* One closing single-qubit layer follows the last cycle (same draw rule).
* Couplers: A = horizontal (r,c)-(r,c+1) with c even, B = horizontal with c
  odd, C = vertical (r,c)-(r+1,c) with r even, D = vertical with r odd.
  Couplers touching a removed site are dropped.
* Square roots are the principal ones: for P in {X, Y, W} (P^2 = I),
  sqrt(P) = ((1+i)/2) I + ((1-i)/2) P.
* fSim(theta, phi) = [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],
  [0,0,0,exp(-i phi)]] in the basis index 2*b_q0 + b_q1; cos(pi/2) is stored
  as an exact 0.
* Random draws come from numpy's PCG64(seed), one integer per (cycle, qubit)
  in that order.

The returned `Circuit` is the contract between every consumer: gate matrices
are stored explicitly so that every side reads identical numbers.
"""

from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

PATTERN = "ABCDCDAB"

_S = 1.0 / math.sqrt(2.0)
_I2 = np.eye(2, dtype=np.complex128)
_PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_PW = np.array([[0, (1 - 1j) * _S], [(1 + 1j) * _S, 0]], dtype=np.complex128)


def _sqrt_pauli(p: np.ndarray) -> np.ndarray:
    return 0.5 * (1 + 1j) * _I2 + 0.5 * (1 - 1j) * p


SQRT_X = _sqrt_pauli(_PX)
SQRT_Y = _sqrt_pauli(_PY)
SQRT_W = _sqrt_pauli(_PW)
ONE_QUBIT_SET = (SQRT_X, SQRT_Y, SQRT_W)
ONE_QUBIT_NAMES = ("sqrtX", "sqrtY", "sqrtW")


def fsim(theta: float, phi: float) -> np.ndarray:
    c = 0.0 if theta == math.pi / 2 else math.cos(theta)
    s = 1.0 if theta == math.pi / 2 else math.sin(theta)
    return np.array(
        [
            [1, 0, 0, 0],
            [0, c, -1j * s, 0],
            [0, -1j * s, c, 0],
            [0, 0, 0, complex(math.cos(phi), -math.sin(phi))],
        ],
        dtype=np.complex128,
    )


FSIM = fsim(math.pi / 2, math.pi / 6)

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) * _S
T = np.array([[1, 0], [0, complex(_S, _S)]], dtype=np.complex128)
CNOT = np.array(
    [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128
)


@dataclass
class Circuit:
    """A gate list in time order.

    gate_qubits: int32 [G, 2]; column 1 is -1 for a single-qubit gate.  For a
        two-qubit gate the matrix basis index is 2*b_{q0} + b_{q1}.
    gate_mats: complex128 [G, 16]; a 4x4 row-major matrix for two-qubit gates,
        the first 4 entries a 2x2 row-major matrix for single-qubit gates
        (the rest zero).
    """

    n_qubits: int
    gate_qubits: np.ndarray
    gate_mats: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return int(self.gate_qubits.shape[0])

    def gate_mats_f64(self) -> np.ndarray:
        """[G, 32] float64 view: (re, im) pairs, the layout the C ABI takes."""
        return np.ascontiguousarray(self.gate_mats).view(np.float64).reshape(
            self.n_gates, 32
        )

    def matrix(self, g: int) -> np.ndarray:
        if self.gate_qubits[g, 1] < 0:
            return self.gate_mats[g, :4].reshape(2, 2)
        return self.gate_mats[g].reshape(4, 4)


class _Builder:
    def __init__(self, n: int):
        self.n = n
        self.q: list[tuple[int, int]] = []
        self.m: list[np.ndarray] = []

    def g1(self, q: int, u: np.ndarray) -> None:
        row = np.zeros(16, dtype=np.complex128)
        row[:4] = u.reshape(4)
        self.q.append((q, -1))
        self.m.append(row)

    def g2(self, a: int, b: int, u: np.ndarray) -> None:
        self.q.append((a, b))
        self.m.append(u.reshape(16).astype(np.complex128))

    def build(self, meta: dict) -> Circuit:
        gq = np.array(self.q, dtype=np.int32).reshape(-1, 2)
        gm = np.array(self.m, dtype=np.complex128).reshape(-1, 16)
        return Circuit(self.n, gq, gm, meta)


def grid_sites(rows: int, cols: int, removed=()) -> dict:
    """Map (r, c) -> dense qubit id in row-major order, skipping removed sites."""
    rem = {tuple(x) for x in removed}
    ids = {}
    for r in range(rows):
        for c in range(cols):
            if (r, c) not in rem:
                ids[(r, c)] = len(ids)
    return ids


def couplers(rows: int, cols: int, letter: str, removed=()) -> list:
    ids = grid_sites(rows, cols, removed)
    out = []
    if letter in "AB":
        par = 0 if letter == "A" else 1
        for r in range(rows):
            for c in range(par, cols - 1, 2):
                if (r, c) in ids and (r, c + 1) in ids:
                    out.append((ids[(r, c)], ids[(r, c + 1)]))
    elif letter in "CD":
        par = 0 if letter == "C" else 1
        for r in range(par, rows - 1, 2):
            for c in range(cols):
                if (r, c) in ids and (r + 1, c) in ids:
                    out.append((ids[(r, c)], ids[(r + 1, c)]))
    else:
        raise ValueError(f"unknown coupler pattern {letter!r}")
    return out


def grid_circuit(
    rows: int,
    cols: int,
    cycles: int,
    seed: int,
    removed=(),
    pattern: str = PATTERN,
    closing_layer: bool = True,
) -> Circuit:
    ids = grid_sites(rows, cols, removed)
    n = len(ids)
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder(n)
    prev = [-1] * n
    names = []

    def one_qubit_layer() -> None:
        row = []
        for q in range(n):
            if prev[q] < 0:
                g = int(rng.integers(0, 3))
            else:
                choices = [x for x in range(3) if x != prev[q]]
                g = choices[int(rng.integers(0, 2))]
            prev[q] = g
            row.append(g)
            b.g1(q, ONE_QUBIT_SET[g])
        names.append(row)

    for c in range(cycles):
        one_qubit_layer()
        for a, bq in couplers(rows, cols, pattern[c % len(pattern)], removed):
            b.g2(a, bq, FSIM)
    if closing_layer:
        one_qubit_layer()
    meta = dict(
        kind="grid",
        rows=rows,
        cols=cols,
        removed=[list(x) for x in removed],
        cycles=cycles,
        seed=seed,
        pattern=pattern,
        closing_layer=closing_layer,
        fsim=[math.pi / 2, math.pi / 6],
        one_qubit_draws=names,
    )
    return b.build(meta)


def worked_example_circuit() -> Circuit:
    """The three-qubit circuit of the paper's worked example (Appendix B, figure
    "Example of multi-amplitude contraction"): H(q0), T(q2), CNOT(q0->q1),
    CNOT(q1->q2), H(q0), H(q1), in that time order."""
    b = _Builder(3)
    b.g1(0, H)
    b.g1(2, T)
    b.g2(0, 1, CNOT)
    b.g2(1, 2, CNOT)
    b.g1(0, H)
    b.g1(1, H)
    return b.build(dict(kind="worked_example"))


# Named workloads: (rows, cols, cycles, seed, removed).
CONFIGS = {
    "small_4x5_m8": dict(rows=4, cols=5, cycles=8, seed=1001),
    "medium_6x6_m12": dict(rows=6, cols=6, cycles=12, seed=1002),
    "share_53q_m14": dict(rows=6, cols=9, cycles=14, seed=1005, removed=((0, 4),)),
}


def config_circuit(name: str) -> Circuit:
    return grid_circuit(**CONFIGS[name])


# The batch workload: circuits of uneven size.  Circuit i (seed 1004 + i) takes
# its grid from BATCH_GRIDS and its cycle count from {10..14}, both drawn with
# PCG64(1004 + i); its string count is floor(10^u), u uniform in [3, 5), drawn
# with PCG64(2004 + i).
BATCH_GRIDS = ((5, 6), (4, 8), (5, 7), (4, 9), (6, 6), (4, 10), (5, 8))


def batch_spec(i: int) -> dict:
    rng = np.random.Generator(np.random.PCG64(1004 + i))
    rows, cols = BATCH_GRIDS[int(rng.integers(0, len(BATCH_GRIDS)))]
    cycles = int(rng.integers(10, 15))
    krng = np.random.Generator(np.random.PCG64(2004 + i))
    k = int(math.floor(10 ** krng.uniform(3.0, 5.0)))
    return dict(rows=rows, cols=cols, cycles=cycles, seed=1004 + i, k=k, string_seed=2004 + i)


def batch_circuit(i: int) -> Circuit:
    sp = batch_spec(i)
    return grid_circuit(sp["rows"], sp["cols"], sp["cycles"], sp["seed"])
