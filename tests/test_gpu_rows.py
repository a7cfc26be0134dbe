"""GPU parity of the per-element kernel's row-streaming form (a short
contracted leg between a wide and a narrow side): against the FP64 state
vector, against the one-thread-per-element form on the same nodes, and with
the FP16 scale it publishes consumed by MFMA nodes downstream.

Tolerances: complex64 path normwise 1e-5 against the state vector (as the
other parity tests).  The two per-element forms sum each output's K terms in
the same ascending order in FP32 but fuse different products into FMAs, so
they differ by rounding, which grows with the depth of the tree (2.3e-6
normwise measured on the 36-qubit workload's first step); they are held to
the same 1e-5 normwise.  Split FP16 normwise 1e-3.
"""

import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import grid_circuit, prefix_bitstrings, config_circuit, config_bitstrings
from oracle import statevec
from paper_2108_05665_amd import xeb, planner

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
AMP_TOL = 1e-5
FORM_TOL = 1e-5
SPLIT_TOL = 1e-3


def _rel(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _amps(p, b=0, e=None):
    a = p.new_amps()
    p.contract(a, b, e)
    torch.cuda.synchronize()
    return a.cpu().numpy()


def _case24():
    circ = grid_circuit(4, 6, 12, seed=77)
    strings = prefix_bitstrings(24, 4000, 16, 5)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=3, trials=6)
    return circ, strings, ch, sl


def _rows_nodes(p):
    return [ns for ns in p.all_node_stats() if ns["kernel"] == "generic" and ns["tile"] == -2]


def test_rows_form_vs_state_vector_and_per_element_form():
    circ, strings, ch, sl = _case24()
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    p = xeb.Plan(circ, strings, ch, sl, force_generic=True)
    rows = _rows_nodes(p)
    print("row-streaming nodes", [(ns["node"], ns["m_bits"], ns["k_bits"], ns["n_bits"]) for ns in rows],
          flush=True)
    # Both thread shapes (one and four stream rows per thread) are exercised.
    assert any(max(ns["m_bits"], ns["n_bits"]) >= 10 for ns in rows)
    assert any(max(ns["m_bits"], ns["n_bits"]) < 10 for ns in rows)
    a_rows = _amps(p)
    assert _rel(a_rows, ref) <= AMP_TOL
    assert np.array_equal(a_rows, _amps(p))  # reruns are deterministic
    for ns in rows:
        p.set_node_config(ns["node"], "generic", tile=-1)
        assert p.node_config(ns["node"])["tile"] == -1
    a_elem = _amps(p)
    assert _rel(a_elem, ref) <= AMP_TOL
    assert _rel(a_rows, a_elem) <= FORM_TOL


@pytest.mark.parametrize("precision", ["split_fp16", "split_bf16"])
def test_rows_form_feeds_split_mfma_nodes(precision):
    """Row-streaming nodes whose tables MFMA nodes consume (for FP16, through
    the largest magnitude the row-streaming kernel publishes for the scale)."""
    circ, strings, ch, sl = _case24()
    ref = statevec.state_vector(circ)[strings.astype(np.int64)]
    p = xeb.Plan(circ, strings, ch, sl, precision=precision, mfma_min_cmacs=65536.0)
    assert _rows_nodes(p)
    assert any(ns["kernel"] == "mfma" for ns in p.all_node_stats())
    assert _rel(_amps(p), ref) <= SPLIT_TOL


def test_rows_form_medium_workload_one_slice_step():
    """The 36-qubit workload's first step of 2^6 stacked slices at the
    default kernel choice: the row-streaming form on the per-element nodes it
    fits (both stream sides occur) agrees with the one-thread-per-element
    form."""
    circ = config_circuit("medium_6x6_m12")
    strings = config_bitstrings("medium_6x6_m12", circ.n_qubits)
    fx = json.load(open(os.path.join(ROOT, "tests", "data", "medium_6x6_m12_plan.json")))
    p = xeb.Plan(circ, strings, fx["children"], fx["sliced"], precision="c64", stack_slices=6)
    rows = _rows_nodes(p)
    assert {ns["swapped"] for ns in rows} == {0, 1}
    print("medium row-streaming nodes", len(rows), flush=True)
    a_rows = _amps(p, 0, 64)
    for ns in rows:
        p.set_node_config(ns["node"], "generic", tile=-1)
    a_elem = _amps(p, 0, 64)
    assert np.isfinite(a_rows).all()
    assert _rel(a_rows, a_elem) <= FORM_TOL
