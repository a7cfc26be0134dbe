"""Stop and resume of a slice range (Appendix A, "Slicing": slices are
independent, so recovery after a failure means contracting the slices that
are missing).  The failure is injected from the host (the plan option
abort_after_slices); every kernel of the aborted call runs to completion."""

import re

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import grid_circuit, uniform_bitstrings
from oracle import statevec
from paper_2108_05665_amd import xeb, planner

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,J", [("c64", 0), ("split_fp16", 2)])
def test_injected_abort_then_resume(precision, J):
    circ = grid_circuit(3, 4, 8, 830)
    strings = uniform_bitstrings(12, 200, 831)
    ch, sl, _ = planner.plan(circ, strings, n_sliced=4, trials=4)
    psi = statevec.state_vector(circ)
    stop = 5
    aborting = xeb.Plan(circ, strings, ch, sl, precision=precision, stack_slices=J,
                        abort_after_slices=stop)
    clean = xeb.Plan(circ, strings, ch, sl, precision=precision, stack_slices=J)
    amps = aborting.new_amps()
    with pytest.raises(xeb.XebError) as err:
        aborting.contract(amps, 0, 16)
    assert err.value.code == xeb.XEB_EABORT
    assert int(re.search(r"resume at slice (\d+)", str(err.value)).group(1)) == stop
    assert aborting.stats()["slices_done"] == stop
    # The limit is reached: a further call contracts nothing and leaves amps alone.
    before = amps.clone()
    with pytest.raises(xeb.XebError) as err2:
        aborting.contract(amps, stop, 16)
    assert err2.value.code == xeb.XEB_EABORT
    torch.cuda.synchronize()
    assert torch.equal(amps, before)
    # Resume on a plan without the injected fault.
    clean.contract(amps, stop, 16)
    ref = clean.new_amps()
    clean.contract(ref, 0, stop)
    clean.contract(ref, stop, 16)
    torch.cuda.synchronize()
    assert torch.equal(amps, ref)
    assert clean.stats()["slices_done"] == 2 * 16 - stop
    want = psi[strings.astype(np.int64)]
    got = amps.cpu().numpy()
    tol = 1e-5 if precision == "c64" else 1e-3
    assert float(np.linalg.norm(got - want) / np.linalg.norm(want)) <= tol
    aborting.close()
    clean.close()
