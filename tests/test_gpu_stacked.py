"""GPU parity of stacked slices (xeb_options_t.stack_slices = J): the J lowest
slice-id bits become key bits of every node (Appendix A, "Slicing": sliced
legs are summed over; section "Multi-batch simulator": fixed legs make the
leaves that carry them variables), so one step evaluates 2^J consecutive
slices.  The amplitudes do not depend on J: every case is checked against
the FP64 oracle (state vector, single-slice partials, or the stored 36-qubit
amplitudes) at the bounds of the unstacked tests.
"""

import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import grid_circuit, uniform_bitstrings, prefix_bitstrings, config_circuit, config_bitstrings
from oracle import statevec, tn
from oracle import xeb as oxeb
from oracle.network import build_network
from paper_2108_05665_amd import xeb, planner

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = {"c64": 1e-5, "split_fp16": 1e-3, "split_bf16": 1e-3}
XEB_TOL = 1e-4
SMALL_MFMA = dict(mfma_min_cmacs=65536.0)


def _rel(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _contract(p, ranges=None):
    amps = p.new_amps()
    if ranges is None:
        p.contract(amps)
    else:
        for b, e in ranges:
            p.contract(amps, b, e)
    torch.cuda.synchronize()
    return amps


@pytest.mark.parametrize("precision", ["c64", "split_fp16", "split_bf16"])
@pytest.mark.parametrize("J", [1, 3, 5])
def test_stacked_vs_state_vector(J, precision):
    circ = grid_circuit(3, 4, 8, 700 + J)
    strings = prefix_bitstrings(12, 300, 5, 701)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=5, trials=4)
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    p = xeb.Plan(circ, strings, ch, sl, precision=precision, stack_slices=J, **SMALL_MFMA)
    assert p.stats()["n_stacked"] == J
    got = _contract(p).cpu().numpy()
    assert _rel(got, ref) <= TOL[precision]
    f = p.fidelity(_contract(p))
    assert abs(f - oxeb.xeb_fidelity(12, ref)) <= XEB_TOL


def test_stacked_ranges_inside_steps():
    """Slice ranges that start and end inside a step of 2^J slices add up to
    the full amplitude; one slice equals the oracle's partial; reruns are
    bit-identical."""
    circ = grid_circuit(3, 4, 8, 720)
    strings = uniform_bitstrings(12, 200, 721)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=4, trials=4)
    p = xeb.Plan(circ, strings, ch, sl, stack_slices=2)
    full = _contract(p)
    parts = _contract(p, [(0, 3), (3, 9), (9, 16)])
    parts2 = _contract(p, [(0, 3), (3, 9), (9, 16)])
    assert torch.equal(parts, parts2)
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    assert _rel(parts.cpu().numpy(), ref) <= TOL["c64"]
    assert _rel(parts.cpu().numpy(), full.cpu().numpy()) <= 1e-12
    net = build_network(circ)
    for sigma in (5, 14):
        one = _contract(p, [(sigma, sigma + 1)]).cpu().numpy()
        want = np.array([tn.partial_amplitude(net, int(s), sl, sigma) for s in strings[:40]])
        assert _rel(one[:40], want) <= TOL["c64"]
    empty = _contract(p, [(6, 6)])
    assert not torch.any(empty != 0)


@pytest.mark.parametrize("precision", ["c64", "split_fp16", "split_bf16"])
def test_stacked_blocks_graph_autotune(precision):
    """String blocks (a memory budget), duplicates, the graph form and the
    autotuner with stacked slices."""
    # Many strings on a shallow 20-qubit circuit: the tables hold more keys
    # than a block has keyed strings, so blocks shrink them (4 blocks at w/2).
    circ = grid_circuit(4, 5, 7, 741)
    strings = uniform_bitstrings(20, 6000, 742)
    strings = np.concatenate([strings, strings[:37]])
    ch, sl, _ = planner.plan(circ, strings, n_sliced=4, trials=4)
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    one = xeb.Plan(circ, strings, ch, sl, precision=precision, stack_slices=3, **SMALL_MFMA)
    a1 = _contract(one).cpu().numpy()
    assert _rel(a1, ref) <= TOL[precision]
    budget = int(one.workspace_bytes() * 0.5)
    blk = xeb.Plan(circ, strings, ch, sl, precision=precision, stack_slices=3, memory_budget=budget,
                   **SMALL_MFMA)
    assert blk.stats()["n_blocks"] > 1 and blk.workspace_bytes() <= budget
    a2 = _contract(blk).cpu().numpy()
    assert _rel(a2, ref) <= TOL[precision]
    assert _rel(a2, a1) <= 1e-5
    assert np.all(a2[6000:] == a2[:37])
    one.autotune(reps=1)
    eager = _contract(one)
    assert _rel(eager.cpu().numpy(), ref) <= TOL[precision]
    b = xeb.Batch([one])
    for _ in range(3):
        b.launch()
        torch.cuda.synchronize()
        assert torch.equal(b.amps[0], eager)


@pytest.mark.parametrize("precision", ["c64", "split_fp16", "split_bf16"])
def test_stacked_medium_full_amplitudes_vs_oracle(precision):
    """The 36-qubit workload (benchmark tree and slices) with 2^6 slices per
    step: the first 64 amplitudes, each summed over all 1024 slices, against
    the stored oracle values, element by element and by XEB."""
    with open(os.path.join(ROOT, "tests", "golden", "medium_6x6_m12_amps64.json")) as f:
        gold = json.load(f)
    with open(os.path.join(ROOT, "tests", "data", "medium_6x6_m12_plan.json")) as f:
        fx = json.load(f)
    circ = config_circuit("medium_6x6_m12")
    strings = config_bitstrings("medium_6x6_m12", circ.n_qubits)
    ref = np.array([complex(re, im) for re, im in gold["amps"]])
    p = xeb.Plan(circ, strings, fx["children"], fx["sliced"], precision=precision, stack_slices=6)
    p.autotune(reps=1)
    amps = _contract(p)
    got = amps.cpu().numpy()
    d = got[:64] - ref
    rel = float(np.linalg.norm(d) / np.linalg.norm(ref))
    peak = float(np.max(np.abs(d)) / np.sqrt(np.mean(np.abs(ref) ** 2)))
    f_ref = oxeb.xeb_fidelity(circ.n_qubits, ref)
    f_got = oxeb.xeb_fidelity(circ.n_qubits, got[:64])
    print(f"{precision} J=6: normwise {rel:.2e}, max/rms {peak:.2e}, |dF64| {abs(f_got - f_ref):.2e}")
    assert rel <= TOL[precision]
    assert peak <= 5 * TOL[precision]
    assert abs(f_got - f_ref) <= XEB_TOL
    F = p.fidelity(amps)
    assert abs(F - oxeb.xeb_fidelity(circ.n_qubits, got)) <= 1e-12
    p.close()
