"""Writes tests/golden/medium_6x6_m12_amps64.json: FP64 oracle amplitudes of
the 36-qubit workload (6x6 grid, 12 cycles, the 10^4-string batch with qubits
0-19 fixed) for its first 64 strings, each the full sum over all 2^10 slices.

Only the oracle computes here (plus the seeded input descriptions in `synth`):

* amp(s) = sum over all assignments sigma of the sliced legs of the partial
  contraction with the output legs fixed to s and the sliced legs to sigma
  (Appendix A, paragraph "Slicing"; the amplitude itself is the contraction
  of section "Multi-batch simulator").  The sum is exact (math.fsum of the
  per-group sums, each group an fsum of its partials).
* The partials come from the oracle's run of Algorithms 3-4 (Appendix C) on
  FP64 tensors, over groups of 16 consecutive slices with the slice bits as
  variables.  Its contraction order follows the tree in the plan fixture
  (tests/data/medium_6x6_m12_plan.json, an input of the problem like the
  circuit): the order does not change the result (section "Tensor network
  contraction"), it only makes the FP64 run take minutes instead of hours.
* Cross-check independent of that tree: for a few (string, sigma) pairs the
  partial is recomputed by O2 (plain pairwise contraction in the oracle's own
  greedy order) and must agree with the memo partial to 1e-12 relative; the
  pairs and both values are stored.

Run:  python tests/golden/make_medium_amps.py [--procs 6]
(about 15-30 minutes on 6-8 host cores).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PLAN = os.path.join(ROOT, "tests", "data", "medium_6x6_m12_plan.json")
OUT = os.path.join(HERE, "medium_6x6_m12_amps64.json")
N_STRINGS = 64
GROUP = 16


def _setup():
    sys.path.insert(0, ROOT)
    from synth import config_circuit, config_bitstrings
    from oracle.network import build_network
    from oracle import memo

    circ = config_circuit("medium_6x6_m12")
    strings = config_bitstrings("medium_6x6_m12", circ.n_qubits)[:N_STRINGS]
    net = build_network(circ)
    with open(PLAN) as f:
        plan = json.load(f)
    tree = memo.Tree(len(net.leaves), plan["children"])
    return circ, strings, net, tree, [int(x) for x in plan["sliced"]]


def _group(g: int):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import memo

    _, strings, net, tree, sliced = _setup()
    t0 = time.perf_counter()
    amps, _ = memo.memo_amplitudes(net, tree, strings, sliced,
                                   sigmas=range(g * GROUP, (g + 1) * GROUP))
    return g, [(float(a.real), float(a.imag)) for a in amps], time.perf_counter() - t0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    os.environ["OMP_NUM_THREADS"] = "1"
    import multiprocessing as mp

    import numpy as np

    circ, strings, net, tree, sliced = _setup()
    n_groups = (1 << len(sliced)) // GROUP
    sums = [None] * n_groups
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(args.procs) as pool:
        for g, vals, sec in pool.imap_unordered(_group, range(n_groups)):
            sums[g] = vals
            done = sum(x is not None for x in sums)
            print(f"group {g} ({sec:.1f} s), {done}/{n_groups} done, "
                  f"{time.perf_counter() - t0:.0f} s", flush=True)
    amps = []
    for i in range(N_STRINGS):
        amps.append((math.fsum(sums[g][i][0] for g in range(n_groups)),
                     math.fsum(sums[g][i][1] for g in range(n_groups))))

    # Tree-independent cross-check: O2 partials in the oracle's own order.
    from oracle import memo, tn

    pairs = tn.search_order(tn.closed_leg_sets(net, sliced), trials=64)[0]
    rng = np.random.Generator(np.random.PCG64(4242))
    checks = []
    for _ in range(4):
        i = int(rng.integers(0, N_STRINGS))
        sg = int(rng.integers(0, 1 << len(sliced)))
        o2 = tn.partial_amplitude(net, int(strings[i]), sliced, sg, pairs=pairs)
        m4 = memo.memo_amplitudes(net, tree, [strings[i]], sliced, sigmas=[sg])[0][0]
        err = abs(o2 - m4) / max(abs(o2), 1e-300)
        print(f"cross-check string {i} sigma {sg}: |O2 - memo| / |O2| = {err:.2e}", flush=True)
        assert err < 1e-12, err
        checks.append({"string_index": i, "sigma": sg, "o2": [o2.real, o2.imag],
                       "memo": [float(m4.real), float(m4.imag)]})

    with open(PLAN, "rb") as f:
        plan_sha = hashlib.sha256(f.read()).hexdigest()
    doc = {
        "source": "FP64 oracle (tests/golden/make_medium_amps.py): Appendix A 'Slicing' sum of "
                  "Appendix C (Algorithms 3-4) partials; amplitudes <s|C|0^n> of section "
                  "'Multi-batch simulator'",
        "workload": "medium_6x6_m12: 6x6 grid, 12 cycles + closing layer, circuit seed 1002; "
                    "strings: first 64 of the 10^4 batch (qubits 0-19 fixed, seed 2002)",
        "n_qubits": circ.n_qubits,
        "sliced_legs": sliced,
        "plan_fixture_sha256": plan_sha,
        "strings": [str(int(s)) for s in strings],
        "amps": [[re, im] for re, im in amps],
        "o2_cross_checks": checks,
        "seconds": time.perf_counter() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
