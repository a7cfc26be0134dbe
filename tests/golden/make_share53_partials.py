"""Writes tests/golden/share_53q_m14_partials.json: FP64 oracle partial
amplitudes of the 53-qubit share (6x9 grid minus site (0, 4), 14 cycles, the
3 * 10^5 seeded uniform strings) for its first 8 strings at two slice
assignments sigma inside the first 256-slice block.

A partial amplitude is the contraction with the output legs fixed to the
string and the sliced legs fixed to sigma (Appendix A, paragraph "Slicing";
bit j of sigma is the value of sliced leg j).  Only the oracle computes here
(plus the seeded input descriptions in `synth`): O2, pairwise contraction in
the oracle's own order (its randomized greedy search), in complex128.  The
sliced legs are an input of the problem, read from the plan fixture
tests/data/share_53q_m14_plan.json.  Cross-check: every value is also
computed along a second oracle order (another search seed), and the two must
agree to 1e-12 relative.

Run:  python tests/golden/make_share53_partials.py   (a few minutes)
"""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PLAN = os.path.join(ROOT, "tests", "data", "share_53q_m14_plan.json")
OUT = os.path.join(HERE, "share_53q_m14_partials.json")
N_STRINGS = 8
SIGMAS = (0, 137)


def main() -> int:
    sys.path.insert(0, ROOT)
    from synth import config_circuit, config_bitstrings
    from oracle.network import build_network
    from oracle import tn

    circ = config_circuit("share_53q_m14")
    strings = config_bitstrings("share_53q_m14", circ.n_qubits)[:N_STRINGS]
    with open(PLAN) as f:
        sliced = [int(x) for x in json.load(f)["sliced"]]
    net = build_network(circ)
    sets = tn.closed_leg_sets(net, sliced)
    orders = [tn.search_order(sets, trials=32, seed=seed)[0] for seed in (1, 2)]
    vals = []
    for sigma in SIGMAS:
        for s in strings.tolist():
            t0 = time.time()
            a, b = (tn.partial_amplitude(net, int(s), sliced, sigma, pairs=pr) for pr in orders)
            rel = abs(a - b) / max(abs(a), 1e-300)
            assert rel <= 1e-12, (s, sigma, a, b)
            vals.append({"string": str(s), "sigma": sigma, "partial": [a.real, a.imag],
                         "second_order_rel_diff": rel})
            print(f"sigma {sigma} string {s}: {a} ({time.time() - t0:.1f} s, orders agree {rel:.1e})",
                  flush=True)
    with open(OUT, "w") as f:
        json.dump({"workload": "share_53q_m14", "sliced_legs": sliced, "n_strings": N_STRINGS,
                   "sigmas": list(SIGMAS), "partials": vals,
                   "oracle": "O2 (oracle/tn.py partial_amplitude), two randomized greedy orders"},
                  f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
