"""GPU parity at full size against stored FP64 oracle values.

* The 36-qubit workload (6x6 grid, 12 cycles, 10^4 strings with qubits 0-19
  fixed, 2^10 slices) in the benchmark's configuration: the plan fixture the
  benchmark contracts (tree and sliced legs), its kernel choices made the
  way the benchmark makes them (the autotuner, or node configurations saved
  from a benchmark run), eager and hipGraph launch forms.  The first 64
  amplitudes, each summed over all 1024 slices, are compared element by
  element with the oracle's (tests/golden/medium_6x6_m12_amps64.json, written
  by tests/golden/make_medium_amps.py from the oracle alone), and so is the
  XEB of those 64 strings (Eq. (1)).
* The small workload (4x5 grid, 8 cycles) with 1000 strings drawn from the
  ideal distribution |psi|^2 (F close to 2^n sum p^2 - 1) and with all 2^20
  strings once each (F = 0 exactly, because the probabilities sum to one).

Bounds (amplitudes normwise, R17 of the readings): complex64 1e-5, split
forms 1e-3; no single amplitude may be off by more than 5x that bound times
the rms amplitude; XEB within 1e-4.
"""

import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import config_circuit, config_bitstrings
from oracle import statevec
from oracle import xeb as oxeb
from paper_2108_05665_amd import xeb, planner

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "medium_6x6_m12_amps64.json")
PLAN = os.path.join(ROOT, "tests", "data", "medium_6x6_m12_plan.json")
CONFIGS = os.path.join(ROOT, "tests", "data", "medium_6x6_m12_configs.json")
TOL = {"c64": 1e-5, "split_fp16": 1e-3, "split_bf16": 1e-3}
XEB_TOL = 1e-4


def _errors(got, ref):
    d = got - ref
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    return float(np.linalg.norm(d) / np.linalg.norm(ref)), float(np.max(np.abs(d)) / rms)


@pytest.mark.parametrize("precision", ["c64", "split_fp16", "split_bf16"])
def test_medium_full_amplitudes_vs_oracle(precision):
    with open(GOLDEN) as f:
        gold = json.load(f)
    with open(PLAN) as f:
        plan_fx = json.load(f)
    circ = config_circuit("medium_6x6_m12")
    strings = config_bitstrings("medium_6x6_m12", circ.n_qubits)
    assert [str(int(s)) for s in strings[:64]] == gold["strings"]
    assert plan_fx["sliced"] == gold["sliced_legs"]
    ref = np.array([complex(re, im) for re, im in gold["amps"]])
    p = xeb.Plan(circ, strings, plan_fx["children"], plan_fx["sliced"], precision=precision)
    saved = {}
    if os.path.exists(CONFIGS):
        with open(CONFIGS) as f:
            saved = json.load(f).get(precision, {})
    if saved:
        for node, c in saved.items():
            p.set_node_config(int(node), **c)
    else:
        p.autotune(reps=2)
    amps = p.new_amps()
    p.contract(amps)
    F = p.fidelity(amps)
    torch.cuda.synchronize()
    got = amps.cpu().numpy()
    rel, peak = _errors(got[:64], ref)
    f_ref = oxeb.xeb_fidelity(circ.n_qubits, ref)
    f_got = oxeb.xeb_fidelity(circ.n_qubits, got[:64])
    print(f"{precision}: normwise {rel:.2e}, max/rms {peak:.2e}, |dF64| {abs(f_got - f_ref):.2e}")
    assert rel <= TOL[precision]
    assert peak <= 5 * TOL[precision]
    assert abs(f_got - f_ref) <= XEB_TOL
    # The XEB kernel over all strings agrees with the exact sum of the same amplitudes.
    assert abs(F - oxeb.xeb_fidelity(circ.n_qubits, got)) <= 1e-12
    # The graph form (the benchmark's `value`) equals the eager form bit for bit.
    b = xeb.Batch([p])
    b.launch()
    fb = b.fidelities()[0]
    torch.cuda.synchronize()
    assert torch.equal(b.amps[0], amps)
    assert fb == F
    b.close()
    # Duplicates in the batch receive identical values.
    first = {}
    for i, x in enumerate(strings.tolist()):
        if x in first:
            assert got[i] == got[first[x]]
        else:
            first[x] = i
    p.close()


def test_small_config_ideal_samples():
    """1000 strings drawn from |psi|^2 (seed 3001): amplitudes match the state
    vector, and F matches the ideal expectation 2^n sum p^2 - 1 within five
    standard errors (readings R18)."""
    circ = config_circuit("small_4x5_m8")
    n = circ.n_qubits
    psi = statevec.state_vector(circ)
    p = np.abs(psi) ** 2
    rng = np.random.Generator(np.random.PCG64(3001))
    strings = rng.choice(p.size, size=1000, p=p / p.sum()).astype(np.uint64)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=0, trials=8)
    plan = xeb.Plan(circ, strings, ch, sl)
    amps = plan.new_amps()
    plan.contract(amps)
    F = plan.fidelity(amps)
    ref = psi[strings.astype(np.int64)]
    got = amps.cpu().numpy()
    rel, peak = _errors(got, ref)
    assert rel <= TOL["c64"] and peak <= 5 * TOL["c64"]
    f_ideal = oxeb.ideal_xeb(psi)
    sd = np.std((2 ** n) * p[strings.astype(np.int64)]) / math.sqrt(len(strings))
    assert abs(F - f_ideal) <= 5 * sd, (F, f_ideal, sd)
    assert abs(F - oxeb.xeb_fidelity(n, ref)) <= XEB_TOL
    assert F > 0.5


def test_small_config_all_strings_xeb_zero():
    """Every one of the 2^20 strings once: the amplitudes are the whole state
    vector and F = 2^n / 2^n sum p - 1 = 0."""
    circ = config_circuit("small_4x5_m8")
    n = circ.n_qubits
    strings = np.arange(1 << n, dtype=np.uint64)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=0, trials=4)
    plan = xeb.Plan(circ, strings, ch, sl)
    amps = plan.new_amps()
    plan.contract(amps)
    F = plan.fidelity(amps)
    psi = statevec.state_vector(circ)
    rel, peak = _errors(amps.cpu().numpy(), psi)
    assert rel <= TOL["c64"] and peak <= 5 * TOL["c64"]
    assert abs(F) <= 1e-5, F
