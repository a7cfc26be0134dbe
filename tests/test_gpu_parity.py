"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (complex64 contraction, FP32 accumulation inside every pairwise
contraction, FP64 across slices):
  amplitudes: normwise relative error ||a - a_ref|| / ||a_ref|| <= 1e-5;
  XEB: |F - F_ref| <= 1e-4 (F_ref from the oracle's amplitudes);
  the XEB kernel itself on identical amplitudes: |F - F_oracle| <= 1e-12.
"""

import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import (grid_circuit, worked_example_circuit, uniform_bitstrings, prefix_bitstrings,
                   config_circuit, config_bitstrings)
from oracle import statevec, tn
from oracle import xeb as oxeb
from oracle.network import build_network
from paper_2108_05665_amd import xeb, planner

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
AMP_TOL = 1e-5
XEB_TOL = 1e-4


def _run(circ, strings, ch, sl, rng=None, **kw):
    p = xeb.Plan(circ, strings, ch, sl, **kw)
    amps = p.new_amps()
    if rng is None:
        p.contract(amps)
    else:
        for b, e in rng:
            p.contract(amps, b, e)
    torch.cuda.synchronize()
    return p, amps


def _rel(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def test_worked_example_through_abi():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "worked_example.json")))
    allstr = list(g["amplitude_signs_q0_first"])
    strings = [sum(int(ch) << q for q, ch in enumerate(s)) for s in allstr]
    p, amps = _run(worked_example_circuit(), strings, g["tree_children"], [],
                   fuse_1q=False, fold_kets=False)
    got = amps.cpu().numpy()
    for s, a in zip(allstr, got):
        want = g["amplitude_signs_q0_first"][s] / (2 * math.sqrt(2))
        assert abs(a - want) < 1e-6, (s, a, want)


@pytest.mark.parametrize("force_generic", [False, True])
def test_small_config_vs_state_vector(force_generic):
    """4x5 grid, 8 cycles, 1000 uniform strings, no slicing (the small
    workload), every amplitude checked."""
    circ = config_circuit("small_4x5_m8")
    strings = config_bitstrings("small_4x5_m8", circ.n_qubits)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=0, trials=8)
    p, amps = _run(circ, strings, ch, sl, force_generic=force_generic)
    kinds = {ns["kernel"] for ns in p.all_node_stats()}
    if force_generic:
        assert kinds == {"generic"}
    else:
        assert "mfma" in kinds
    psi = statevec.state_vector(circ)
    ref = psi[strings.astype(np.int64)]
    got = amps.cpu().numpy()
    assert _rel(got, ref) <= AMP_TOL
    f = p.fidelity(amps)
    assert abs(f - oxeb.xeb_fidelity(circ.n_qubits, ref)) <= XEB_TOL
    assert abs(f - oxeb.xeb_fidelity(circ.n_qubits, got)) <= 1e-12


@pytest.mark.parametrize("n_sliced", [1, 3, 5])
def test_sliced_vs_state_vector(n_sliced):
    circ = grid_circuit(3, 4, 8, 300 + n_sliced)
    strings = prefix_bitstrings(12, 333, 5, 301)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=n_sliced, trials=4)
    p, amps = _run(circ, strings, ch, sl)
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    assert _rel(amps.cpu().numpy(), ref) <= AMP_TOL


def test_slice_ranges_accumulate_and_are_deterministic():
    circ = grid_circuit(3, 4, 8, 310)
    strings = uniform_bitstrings(12, 257, 311)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=4, trials=4)
    _, full = _run(circ, strings, ch, sl)
    _, full2 = _run(circ, strings, ch, sl)
    assert torch.equal(full, full2)  # fixed order: bit-identical reruns
    _, split = _run(circ, strings, ch, sl, rng=[(0, 5), (5, 11), (11, 16)])
    _, split2 = _run(circ, strings, ch, sl, rng=[(0, 5), (5, 11), (11, 16)])
    assert torch.equal(split, split2)
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    assert _rel(split.cpu().numpy(), ref) <= AMP_TOL
    assert _rel(split.cpu().numpy(), full.cpu().numpy()) <= 1e-12


def test_single_slice_partials_match_oracle():
    circ = grid_circuit(3, 3, 7, 320)
    strings = uniform_bitstrings(9, 40, 321)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=3, trials=4)
    net = build_network(circ)
    p = xeb.Plan(circ, strings, ch, sl)
    for sigma in (0, 5, 7):
        amps = p.new_amps()
        p.contract(amps, sigma, sigma + 1)
        got = amps.cpu().numpy()
        ref = np.array([tn.partial_amplitude(net, int(s), sl, sigma) for s in strings])
        assert _rel(got, ref) <= AMP_TOL


def test_duplicates_tiny_batches_and_empty_range():
    circ = grid_circuit(3, 3, 6, 330)
    psi = statevec.state_vector(circ)
    for strings in ([5], [5, 5], [0, 511, 0, 7, 511]):
        s = np.array(strings, dtype=np.uint64)
        ch, sl, _ = planner.plan(circ, s, n_sliced=2, trials=2)
        p, amps = _run(circ, s, ch, sl)
        got = amps.cpu().numpy()
        assert _rel(got, psi[s.astype(np.int64)]) <= AMP_TOL
        z = p.new_amps()
        p.contract(z, 2, 2)
        torch.cuda.synchronize()
        assert not torch.any(z != 0)


def test_non_default_stream():
    circ = grid_circuit(3, 4, 6, 340)
    strings = uniform_bitstrings(12, 100, 341)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=2, trials=2)
    p = xeb.Plan(circ, strings, ch, sl)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        amps = p.new_amps()
        p.contract(amps, stream=st)
        f = p.fidelity(amps, stream=st)
    st.synchronize()
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    assert _rel(amps.cpu().numpy(), ref) <= AMP_TOL
    assert abs(f - oxeb.xeb_fidelity(12, ref)) <= XEB_TOL


def test_medium_config_sampled_partials():
    """The 36-qubit, 12-cycle workload at full size (10^4 strings, 2^10 slices)
    in the benchmark's launch configuration: one slice contracted for every
    string; sampled strings checked against the oracle's partials."""
    name = "medium_6x6_m12"
    circ = config_circuit(name)
    strings = config_bitstrings(name, circ.n_qubits)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=10, trials=16, seed=0)
    assert len(sl) == 10
    net = build_network(circ)
    pairs = tn.search_order(tn.closed_leg_sets(net, sl), trials=64)[0]
    p = xeb.Plan(circ, strings, ch, sl)
    sigma = 777
    amps = p.new_amps()
    p.contract(amps, sigma, sigma + 1)
    got = amps.cpu().numpy()
    idx = [0, 4321, 9999]
    ref = np.array([tn.partial_amplitude(net, int(strings[i]), sl, sigma, pairs=pairs) for i in idx])
    assert _rel(got[idx], ref) <= AMP_TOL
    # duplicates in the batch receive identical values
    s = strings
    first = {}
    for i, x in enumerate(s.tolist()):
        if x in first:
            assert got[i] == got[first[x]]
        else:
            first[x] = i
