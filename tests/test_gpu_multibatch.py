"""GPU parity of the multi-batch output (section "Multi-batch simulator": the
output legs of w chosen qubits stay open, so each string yields 2^w
amplitudes).  The plain definition is the oracle: entry (i, o) is the
amplitude of string i with its open qubits set to o, read from the FP64 state
vector, and the XEB counts each string's own entry (Eq. (1)).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import grid_circuit, uniform_bitstrings, prefix_bitstrings
from oracle import statevec, tn
from oracle import xeb as oxeb
from oracle.network import build_network
from paper_2108_05665_amd import xeb, planner

pytestmark = pytest.mark.gpu
TOL = {"c64": 1e-5, "split_fp16": 1e-3, "split_bf16": 1e-3}
SMALL_MFMA = dict(mfma_min_cmacs=65536.0)


def _deposit(o: int, mask: int) -> int:
    r, j = 0, 0
    for q in range(64):
        if (mask >> q) & 1:
            if (o >> j) & 1:
                r |= 1 << q
            j += 1
    return r


def _reference(psi, strings, open_q):
    w = bin(open_q).count("1")
    base = strings.astype(np.int64) & ~open_q
    cols = np.array([_deposit(o, open_q) for o in range(1 << w)], dtype=np.int64)
    return psi[base[:, None] | cols[None, :]]


def _own(strings, open_q):
    out = []
    for s in strings.tolist():
        o, j = 0, 0
        for q in range(64):
            if (open_q >> q) & 1:
                o |= ((s >> q) & 1) << j
                j += 1
        out.append(o)
    return np.array(out)


@pytest.mark.parametrize("precision", ["c64", "split_fp16", "split_bf16"])
@pytest.mark.parametrize("open_q,J", [(0b1, 0), (0b100000000010, 2), (0b1110000, 3)])
def test_open_qubits_vs_state_vector(open_q, J, precision):
    circ = grid_circuit(3, 4, 8, 800 + J)
    strings = prefix_bitstrings(12, 300, 4, 801)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=4, trials=4, open_qubits=open_q)
    psi = statevec.state_vector(circ)
    ref = _reference(psi, strings, open_q)
    p = xeb.Plan(circ, strings, ch, sl, precision=precision, stack_slices=J, open_qubits=open_q,
                 **SMALL_MFMA)
    amps = p.new_amps()
    p.contract(amps)
    torch.cuda.synchronize()
    got = amps.cpu().numpy()
    assert got.shape == ref.shape
    assert float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) <= TOL[precision]
    own = got[np.arange(len(strings)), _own(strings, open_q)]
    f = p.fidelity(amps)
    assert abs(f - oxeb.xeb_fidelity(12, psi[strings.astype(np.int64)])) <= 1e-4
    assert abs(f - oxeb.xeb_fidelity(12, own)) <= 1e-12


def test_open_qubits_ranges_graph_and_partials():
    """Slice ranges add up, one slice equals the oracle's partials of the 2^w
    completions, and the graph form equals the eager form bit for bit."""
    open_q = 0b10000000100
    circ = grid_circuit(3, 4, 8, 820)
    strings = uniform_bitstrings(12, 150, 821)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=3, trials=4, open_qubits=open_q)
    p = xeb.Plan(circ, strings, ch, sl, stack_slices=1, open_qubits=open_q)
    full = p.new_amps()
    p.contract(full)
    parts = p.new_amps()
    for b, e in ((0, 3), (3, 8)):
        p.contract(parts, b, e)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(parts - full) / torch.linalg.norm(full)) <= 1e-12
    net = build_network(circ)
    one = p.new_amps()
    p.contract(one, 5, 6)
    torch.cuda.synchronize()
    got = one.cpu().numpy()[:12]
    want = np.array([[tn.partial_amplitude(net, (s & ~open_q) | _deposit(o, open_q), sl, 5)
                      for o in range(4)] for s in strings[:12].tolist()])
    assert float(np.linalg.norm(got - want) / np.linalg.norm(want)) <= 1e-5
    b = xeb.Batch([p], [full])
    for _ in range(2):
        b.launch()
        torch.cuda.synchronize()
        eager = p.new_amps()
        p.contract(eager)
        torch.cuda.synchronize()
        assert torch.equal(b.amps[0], eager)
    b.close()
