"""Benchmark of the multi-tensor contraction on one MI355X.

Workload (36 qubits): a 6x6 grid circuit with 12 cycles of sqrt(X)/sqrt(Y)/
sqrt(W) layers and fSim(pi/2, pi/6) couplers in the ABCDCDAB order plus a
closing layer, 10^4 seeded bitstrings whose qubits 0..19 share one fixed
value (the rest uniform), sliced over 10 legs (2^10 slices), complex64.

A step is one pass of the whole hot path over the batch: every slice's
contraction with the memo tables (all 2^10 slices), the FP64 cross-slice sum
and the XEB reduction.  Planning (tree, slicing, plan compilation) happens
once before the timed region and is reported separately.

Prints one JSON line.  Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "medium_6x6_m12"
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
METRIC = "amplitudes/sec + contraction TFLOP/s (%MFMA peak), FP16-split vs c64 at stated err"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(circ, strings, sliced, budget_s: float):
    """The FP64 oracle timed on the host on a bounded sample: full partial
    amplitudes (one string, one slice each) until about `budget_s` seconds of
    contraction time; amplitudes/s = partials/s / 2^s."""
    from oracle import tn
    from oracle.network import build_network

    try:
        from threadpoolctl import threadpool_info

        cores = max((int(x.get("num_threads", 1)) for x in threadpool_info()), default=1)
    except Exception:
        cores = os.cpu_count() or 1
    net = build_network(circ)
    pairs = tn.search_order(tn.closed_leg_sets(net, sliced), trials=64)[0]
    done = 0
    t0 = time.perf_counter()
    while True:
        s = int(strings[done % len(strings)])
        tn.partial_amplitude(net, s, sliced, done % (1 << len(sliced)), pairs=pairs)
        done += 1
        el = time.perf_counter() - t0
        log(f"oracle partial {done} done, {el:.1f} s")
        if el >= budget_s or done >= 64:
            break
    per_partial = el / done
    value = 1.0 / (per_partial * (1 << len(sliced)))
    return {
        "value": value,
        "unit": "amplitudes/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{done} single-string single-slice FP64 partials of the same network "
                  f"({per_partial:.2f} s each); an amplitude needs all {1 << len(sliced)} slices",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trials", type=int, default=16, help="planner trials")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slices", type=int, default=None,
                    help="contract only the first N slices per step (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(slices would shard across GPUs with one all-reduce of the amplitudes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from synth import config_circuit, config_bitstrings
    from paper_2108_05665_amd import planner, xeb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    circ = config_circuit(WORKLOAD)
    strings = config_bitstrings(WORKLOAD, circ.n_qubits)
    t0 = time.perf_counter()
    children, sliced, info = planner.plan(circ, strings, n_sliced=10, trials=args.trials, seed=0)
    t_tree = time.perf_counter() - t0
    log(f"planned tree in {t_tree:.1f} s: cost {info['cost']:.3e} cmacs, max 2^{info['max_log2']}")
    t0 = time.perf_counter()
    plan = xeb.Plan(circ, strings, children, sliced, device=0)
    t_plan = time.perf_counter() - t0
    st = plan.stats()
    n_slices = 1 << len(sliced)
    run_slices = n_slices if args.slices is None else min(args.slices, n_slices)
    log(f"plan compiled in {t_plan:.1f} s, workspace {st['workspace_bytes'] / 2**30:.2f} GiB")
    amps = plan.new_amps()

    def step():
        amps.zero_()
        plan.contract(amps, 0, run_slices)
        return plan.fidelity(amps)  # waits for the stream

    for w in range(args.warmup):
        F = step()
        log(f"warmup {w + 1}/{args.warmup} done, F = {F:.6f}")
    torch.cuda.synchronize()
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        F = step()
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {name: plan.read_profile(name) for name in ("mfma", "generic", "accumulate")}
    plan.set_profiling(False)

    sec_per_step = elapsed / args.steps
    frac_slices = run_slices / n_slices
    amps_per_s = len(strings) * frac_slices / sec_per_step
    cm = st["cmacs_full"] * frac_slices if run_slices == n_slices else None
    if cm is None:
        cm = sum(p["cmacs"] for p in prof.values()) / args.steps
    useful_tflops = 8.0 * cm / sec_per_step / 1e12
    mf = prof["mfma"]
    mfma_tflops = 8.0 * mf["cmacs"] / mf["seconds"] / 1e12 if mf["seconds"] > 0 else 0.0
    mfma_gbs = mf["bytes"] / mf["seconds"] / 1e9 if mf["seconds"] > 0 else 0.0
    ai = 8.0 * mf["cmacs"] / mf["bytes"] if mf["bytes"] > 0 else 0.0
    ridge = FP32_MFMA_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai >= ridge:
        roof = {"bound": "mfma", "achieved": mfma_tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": mfma_tflops / FP32_MFMA_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": mfma_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": mfma_gbs / HBM_PEAK_GBS}
    roof.update({"kernel": "k_contract_mfma", "traffic": None,
                 "launches_per_step": mf["launches"] / args.steps,
                 "flops_per_launch": 8.0 * mf["cmacs"] / max(mf["launches"], 1),
                 "bytes_per_launch": mf["bytes"] / max(mf["launches"], 1),
                 "avg_launch_us": 1e6 * mf["seconds"] / max(mf["launches"], 1),
                 "arith_intensity_flop_per_byte": ai})
    kernel_share = {name: p["seconds"] / args.steps / sec_per_step for name, p in prof.items()}

    out = {
        "metric": METRIC,
        "value": amps_per_s,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD}: 36 qubits on a 6x6 grid, 12 cycles (ABCDCDAB + closing "
                        "layer), 10^4 strings with qubits 0-19 fixed, 2^10 slices, complex64",
            "strings": int(len(strings)),
            "distinct_strings": int(st["k_distinct"]),
            "slices": n_slices,
            "slices_per_step": run_slices,
            "precision": "c64",
        },
        "contraction_tflops_useful": useful_tflops,
        "mfma_frac_useful": useful_tflops / FP32_MFMA_PEAK_TFLOPS,
        "kernel_time_share": kernel_share,
        "plan": {"tree_s": t_tree, "compile_s": t_plan, "cmacs_full": st["cmacs_full"],
                 "cmacs_unsliced_tree": info["unsliced_cost"], "max_log2": info["max_log2"],
                 "workspace_gib": st["workspace_bytes"] / 2**30, "sum_variants": st["sum_variants"],
                 "evals_full": st["evals_full"]},
        "xeb": F,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(circ, strings, sliced, args.cpu_budget)
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
