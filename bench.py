"""Benchmark of the multi-tensor contraction on one MI355X.

Workload (36 qubits): a 6x6 grid circuit with 12 cycles of sqrt(X)/sqrt(Y)/
sqrt(W) layers and fSim(pi/2, pi/6) couplers in the ABCDCDAB order plus a
closing layer, 10^4 seeded bitstrings whose qubits 0..19 share one fixed
value (the rest uniform), sliced over 10 legs (2^10 slices).

A step is one pass of the whole hot path over the batch: every slice's
contraction with the memo tables (all 2^10 slices, 2^6 consecutive slices per
contraction step by default: the low slice bits are stacked into the table
keys), the FP64 cross-slice sum and the XEB reduction.  Planning (tree, slicing, plan compilation) happens
once before the timed region and is reported separately.

Three precisions run: split-FP16 MFMA products (the headline `value`),
split-BF16 products, and plain complex64 on FP32 MFMA, with the speedups and
the split-vs-c64 amplitude and XEB differences over all strings, and the
first 64 full amplitudes (all slices summed) and their XEB checked against
stored FP64 oracle values for each.  Each precision is timed in two launch
forms: eager (one host launch per node evaluation) and the hipGraph batch
form (the same launches captured once, one graph launch per step; `value`).
The timed steps carry no profiling events; a separate eager pass with HIP
events on the launch stream gives the per-kernel durations behind `roofline`.

Prints one JSON line.  Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "medium_6x6_m12"
PEAK_TFLOPS = {"c64": 157.3, "split_fp16": 2516.6, "split_bf16": 2516.6}  # dense MFMA
ISSUED_PER_CMAC = {"c64": 8.0, "split_fp16": 24.0, "split_bf16": 24.0}   # real FLOPs issued
HBM_PEAK_GBS = 8000.0
DTYPE = {"c64": "c64 (f32 MFMA)", "split_fp16": "f16 hi/lo split, f32 acc",
         "split_bf16": "bf16 hi/lo split, f32 acc"}
METRIC = "amplitudes/sec + contraction TFLOP/s (%MFMA peak), FP16-split vs c64 at stated err"
ERR_BOUND = {"c64": 1e-5, "split_fp16": 1e-3, "split_bf16": 1e-3}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(net, pairs, strings, sliced, budget_s: float):
    """The FP64 oracle timed on the host on a bounded sample: full partial
    amplitudes (one string, one slice each) until about `budget_s` seconds of
    contraction time; amplitudes/s = partials/s / 2^s."""
    from oracle import tn

    try:
        from threadpoolctl import threadpool_info

        cores = max((int(x.get("num_threads", 1)) for x in threadpool_info()), default=1)
    except Exception:
        cores = os.cpu_count() or 1
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
    return {
        "value": 1.0 / (per_partial * (1 << len(sliced))),
        "unit": "amplitudes/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{done} single-string single-slice FP64 partials of the same network "
                  f"({per_partial:.2f} s each); an amplitude needs all {1 << len(sliced)} slices",
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", f"contract_split_{WORKLOAD}_traffic.json")


def measured_traffic(prec: str):
    """HBM bytes per split-form MFMA launch from the committed PMC summary, or
    None when it covers another precision or the kernel / launch sources have
    changed since the counters were taken."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            doc = json.load(f)
    except OSError:
        return None
    if doc.get("precision") != prec or doc.get("workload") != WORKLOAD:
        return None
    for rel, digest in doc["sources_sha256"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return float(doc["bytes_per_launch"])


def roofline(prof: dict, prec: str) -> dict:
    mf = prof["mfma"]
    if mf["seconds"] <= 0:
        return {"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None}
    # Algorithmic work: 8 real FLOP per complex MAC.  The split forms issue
    # ISSUED_PER_CMAC / 8 = 3 times as many on their 16-bit MFMAs (hi.hi +
    # hi.lo + lo.hi), so their roof in algorithmic FLOP/s is a third of the
    # instruction peak, and so is the ridge in algorithmic FLOP per byte.
    flops = 8.0 * mf["cmacs"]
    issued = ISSUED_PER_CMAC[prec] * mf["cmacs"]
    tflops = flops / mf["seconds"] / 1e12
    issued_tflops = issued / mf["seconds"] / 1e12
    gbs = mf["bytes"] / mf["seconds"] / 1e9
    ai = flops / mf["bytes"]
    mfma_roof = PEAK_TFLOPS[prec] * 8.0 / ISSUED_PER_CMAC[prec]  # algorithmic TFLOP/s
    ridge = mfma_roof * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai >= ridge:
        r = {"bound": "mfma", "achieved": tflops, "peak": mfma_roof, "unit": "TFLOP/s",
             "frac": tflops / mfma_roof}
    else:
        r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": gbs / HBM_PEAK_GBS}
    traffic = measured_traffic(prec)
    bytes_per_launch = mf["bytes"] / max(mf["launches"], 1)
    # One launch of the split forms is a k_contract_split* dispatch, or the two
    # k_presplit conversions and the k_contract_planes GEMM (one event pair).
    kernel = ("k_contract_mfma" if prec == "c64"
              else "split MFMA launch (k_contract_split*, or k_presplit x2 + k_contract_planes)")
    r.update({"traffic": traffic, "kernel": kernel,
              "hbm_frac": gbs / HBM_PEAK_GBS,
              "mfma_issue_frac": issued_tflops / PEAK_TFLOPS[prec],
              "algorithmic_bytes_per_launch": bytes_per_launch,
              "algorithmic_flop_per_launch": flops / max(mf["launches"], 1),
              "issued_flop_per_launch": issued / max(mf["launches"], 1),
              "issued_tflops": issued_tflops, "instruction_peak_tflops": PEAK_TFLOPS[prec],
              "traffic_over_algorithmic": None if traffic is None else traffic / bytes_per_launch,
              "launches": mf["launches"], "avg_launch_us": 1e6 * mf["seconds"] / max(mf["launches"], 1),
              "algorithmic_flop_per_byte": ai, "ridge_flop_per_byte": ridge,
              "algorithmic_tflops": tflops, "gbs": gbs})
    return r


GOLDEN = os.path.join(ROOT, "tests", "golden", f"{WORKLOAD}_amps64.json")
PLAN_FIXTURE = os.path.join(ROOT, "tests", "data", f"{WORKLOAD}_plan.json")


def oracle_errors(amps, n_qubits: int):
    """Errors of the first 64 amplitudes (each summed over all slices) against
    the stored FP64 oracle values: normwise, largest |difference| over the rms
    amplitude, and the XEB of those 64 strings (Eq. (1))."""
    import math

    import numpy as np

    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        gold = json.load(f)
    ref = np.array([complex(re, im) for re, im in gold["amps"]])
    got = np.asarray(amps[: len(ref)])
    d = got - ref
    rms = math.sqrt(float(np.mean(np.abs(ref) ** 2)))

    def F(a):
        return math.ldexp(math.fsum(float(x) for x in np.abs(a) ** 2), n_qubits) / len(a) - 1.0

    return {"strings": len(ref), "amp_rel_err": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "amp_max_over_rms": float(np.max(np.abs(d)) / rms),
            "xeb_abs_err": abs(F(got) - F(ref)), "xeb_oracle": F(ref)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--trials", type=int, default=16, help="planner greedy trials")
    ap.add_argument("--anneal-steps", type=int, default=500000, help="tree optimizer steps")
    ap.add_argument("--anneal-restarts", type=int, default=6)
    ap.add_argument("--precisions", default=None,
                    help="comma list; the first one gives `value` (default: split_fp16, "
                         "split_bf16, c64; batch32: split_fp16, c64)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--plan-only", metavar="PATH",
                    help="plan the tree and slices, write them to PATH as JSON and exit "
                         "(no GPU use)")
    ap.add_argument("--tree", metavar="PATH",
                    help="take the tree and slices from a --plan-only file (default for the "
                         "36-qubit workload: the committed plan fixture "
                         "tests/data/medium_6x6_m12_plan.json)")
    ap.add_argument("--replan", action="store_true",
                    help="plan the tree and slices afresh instead of reading the fixture")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the compile-time kernel choices (no per-node autotuning)")
    ap.add_argument("--autotune-reps", type=int, default=3)
    ap.add_argument("--save-configs", metavar="PATH",
                    help="write every node's kernel configuration (after tuning) as JSON")
    ap.add_argument("--configs", metavar="PATH",
                    help="apply node configurations from a --save-configs file instead of "
                         "autotuning (the same kernels in every run, e.g. for counters)")
    ap.add_argument("--stack-slices", type=int, default=6,
                    help="evaluate 2^J consecutive slices per contraction step "
                         "(xeb_options_t.stack_slices; 0 = one slice at a time)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager form only (value then comes from it)")
    ap.add_argument("--workload", default=WORKLOAD, choices=[WORKLOAD, "batch32", "share53"],
                    help="the 36-qubit workload (default), the 32-circuit batch, or one GPU's "
                         "share of the 53-qubit contraction (a block of slices)")
    ap.add_argument("--share53-tree", default="single", choices=["single", "sliced"],
                    help="share53: the single-amplitude tree without slicing, or the sliced fixture")
    ap.add_argument("--share53-strings", type=int, default=1024,
                    help="share53 single: strings contracted (the first ones)")
    ap.add_argument("--slice-block", type=int, default=256,
                    help="share53: slices contracted (a contiguous block from slice 0)")
    ap.add_argument("--batch-budget-gib", type=float, default=None,
                    help="batch32: HBM workspace budget per circuit (default: a 32nd of 270 GiB)")
    ap.add_argument("--batch-skip", default="",
                    help="batch32 --plan-only: circuits (comma-separated) left unplanned")
    ap.add_argument("--no-batch", action="store_true",
                    help="leave the batch workload out of the default run's record")
    ap.add_argument("--batch-max-seconds", type=float, default=2.0,
                    help="batch32: circuits whose best plan is estimated above this many "
                         "seconds per full contraction are planned but left out of the run")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain scale kernel (read + write of this many MiB) "
                         "whose HBM counters calibrate the contraction's")
    args = ap.parse_args()
    if args.precisions is None:
        args.precisions = {"batch32": "split_fp16,c64", "share53": "split_fp16"}.get(
            args.workload, "split_fp16,split_bf16,c64")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(slices would shard across GPUs with one all-reduce of the amplitudes)",
              file=sys.stderr)
        return 2

    if args.workload == "batch32":
        return batch_main(args)
    if args.workload == "share53":
        return share53_main(args)

    import numpy as np
    import torch

    from synth import config_circuit, config_bitstrings
    from paper_2108_05665_amd import planner, xeb

    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    circ = config_circuit(WORKLOAD)
    strings = config_bitstrings(WORKLOAD, circ.n_qubits)
    # Planning forks its optimizer workers, so it runs before the GPU is touched.
    t0 = time.perf_counter()
    if not args.tree and not args.replan and not args.plan_only and os.path.exists(PLAN_FIXTURE):
        args.tree = PLAN_FIXTURE
    if args.tree:
        with open(args.tree) as f:
            saved = json.load(f)
        assert saved["workload"] == WORKLOAD, saved["workload"]
        children, sliced, info = saved["children"], saved["sliced"], saved["info"]
    else:
        children, sliced, info = planner.plan(circ, strings, n_sliced=10, trials=args.trials,
                                              seed=0, anneal_steps=args.anneal_steps,
                                              anneal_restarts=args.anneal_restarts,
                                              workers=min(args.anneal_restarts, 8))
    t_tree = time.perf_counter() - t0
    if args.plan_only:
        with open(args.plan_only, "w") as f:
            json.dump({"workload": WORKLOAD, "children": [[int(a), int(b)] for a, b in children],
                       "sliced": [int(x) for x in sliced], "info": info}, f)
        log(f"tree and slices written to {args.plan_only}")
        return 0
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration_mib > 0:
        # out = 1.0 * src: reads and writes exactly n bytes each, three times.
        n = args.copy_calibration_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"calibration: 3 scale kernels of {n} bytes read + {n} bytes written")
        del src, dst
    log(f"planned tree in {t_tree:.1f} s: cost {info['cost']:.3e} cmacs, max 2^{info['max_log2']}")
    n_slices = 1 << len(sliced)

    oracle_net = oracle_pairs = None
    if not args.no_cpu_baseline:
        from oracle import tn
        from oracle.network import build_network

        oracle_net = build_network(circ)
        oracle_pairs = tn.search_order(tn.closed_leg_sets(oracle_net, sliced), trials=64)[0]

    results = {}
    saved_configs = {}
    for prec in precs:
        t0 = time.perf_counter()
        plan = xeb.Plan(circ, strings, children, sliced, device=0, precision=prec,
                        stack_slices=args.stack_slices)
        t_plan = time.perf_counter() - t0
        st = plan.stats()
        tune = None
        if args.configs:
            with open(args.configs) as f:
                for node, c in json.load(f)[prec].items():
                    plan.set_node_config(int(node), **c)
            log(f"{prec}: node configurations from {args.configs}")
        elif not args.no_autotune:
            tune = plan.autotune(reps=args.autotune_reps)
            log(f"{prec}: autotuned {tune['nodes_tuned']} nodes ({tune['nodes_changed']} changed, "
                f"{tune['candidates']} candidates) in {tune['tuning_seconds']:.1f} s; model "
                f"{tune['default_seconds']:.3f} s -> {tune['tuned_seconds']:.3f} s per call")
        if args.save_configs:
            saved_configs[prec] = {ns["node"]: plan.node_config(ns["node"])
                                   for ns in plan.all_node_stats()}
        amps = plan.new_amps()

        def eager_step():
            amps.zero_()
            plan.contract(amps)
            return plan.fidelity(amps)  # waits for the stream

        def timed(step, label):
            for w in range(args.warmup):
                step()
                log(f"{prec} {label}: warmup {w + 1}/{args.warmup} done")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                step()
                log(f"{prec} {label}: step {k + 1}/{args.steps} done")
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / args.steps

        # Eager form: one launch per node evaluation from the host.
        sec_eager = timed(eager_step, "eager")
        F_eager = plan.fidelity(amps)
        eager_amps = amps.cpu().numpy()
        # Graph form: the same launches captured once as a hipGraph (zeroing,
        # contraction, slice sum and XEB in one graph launch).
        batch = None
        if not args.no_graph:
            t0 = time.perf_counter()
            try:
                batch = xeb.Batch([plan], [amps])
            except xeb.XebError as e:
                if e.code != xeb.XEB_ELIMIT:
                    raise
                log(f"{prec}: graph over the node limit ({e}); eager form only")
            t_capture = time.perf_counter() - t0
        if batch is None:
            t_capture, sec_graph, F, final = None, None, F_eager, eager_amps
        else:

            def graph_step():
                batch.launch()

            sec_graph = timed(graph_step, "graph")
            F = batch.fidelities()[0]
            final = amps.cpu().numpy()
            batch.close()
        # One more eager pass with HIP events around every launch (outside the
        # timed region) for the per-kernel durations.
        torch.cuda.synchronize()
        plan.set_profiling(True)
        eager_step()
        torch.cuda.synchronize()
        prof = {name: plan.read_profile(name) for name in ("mfma", "generic", "accumulate", "splitk")}
        nodes = []
        for ns in plan.all_node_stats():
            np_ = plan.read_node_profile(ns["node"])
            if np_["launches"] == 0 or np_["seconds"] <= 0:
                continue
            nodes.append({"node": ns["node"], "kernel": ns["kernel"], "tile": ns["tile"],
                          "swapped": ns["swapped"], "pair_mode": ns["pair_mode"],
                          "ksplit": ns["ksplit"], "keys": ns["variants"],
                          "m_k_n_bits": [ns["m_bits"], ns["k_bits"], ns["n_bits"]],
                          "launches": np_["launches"], "seconds": np_["seconds"],
                          "algorithmic_tflops": 8.0 * np_["cmacs"] / np_["seconds"] / 1e12,
                          "gbs": np_["bytes"] / np_["seconds"] / 1e9})
        nodes.sort(key=lambda x: -x["seconds"])
        plan.set_profiling(False)
        # Full amplitudes of the timed graph form against the stored FP64
        # oracle values (first 64 strings, all slices summed).
        oerr = None if args.no_oracle_check else oracle_errors(final, circ.n_qubits)
        sec = sec_eager if sec_graph is None else sec_graph
        results[prec] = dict(
            sec=sec, sec_eager=sec_eager, F=F, amps=final, prof=prof, st=st, t_plan=t_plan,
            t_capture=t_capture, oracle=oerr, tune=tune, top_nodes=nodes[:12],
            graph_vs_eager_max_abs=float(np.max(np.abs(final - eager_amps))) if len(final) else 0.0,
            F_eager=F_eager, amps_per_s=len(strings) / sec,
            useful_tflops=8.0 * st["cmacs_full"] / sec / 1e12,
            share={n: p["seconds"] / max(sum(q["seconds"] for q in prof.values()), 1e-30)
                   for n, p in prof.items()},
        )
        log(f"{prec}: {1e3 * sec:.0f} ms/step ({len(strings) / sec:.0f} amplitudes/s), "
            f"eager {1e3 * sec_eager:.0f} ms/step, oracle errors {oerr}")
        plan.close()
        del amps

    if args.save_configs:
        with open(args.save_configs, "w") as f:
            json.dump(saved_configs, f)
    head = precs[0]
    r = results[head]
    ref_prec = "c64" if "c64" in results else None
    compare = {}
    for prec, x in results.items():
        if ref_prec and prec != ref_prec:
            a, b = x["amps"], results[ref_prec]["amps"]
            compare[prec] = {
                "speedup_vs_c64": results[ref_prec]["sec"] / x["sec"],
                "amp_rel_diff_vs_c64_all_strings": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "xeb_abs_diff_vs_c64": abs(x["F"] - results[ref_prec]["F"]),
            }
    forms = {
        prec: {
            "amplitudes_per_s": x["amps_per_s"], "ms_per_step": 1e3 * x["sec"],
            "eager_ms_per_step": 1e3 * x["sec_eager"],
            "eager_amplitudes_per_s": len(strings) / x["sec_eager"],
            "graph_capture_s": x["t_capture"],
            "autotune": x["tune"],
            "graph_vs_eager_max_abs_diff": x["graph_vs_eager_max_abs"],
            "contraction_tflops_useful": x["useful_tflops"],
            "useful_frac_of_mfma_peak": x["useful_tflops"] / PEAK_TFLOPS[prec],
            "issued_frac_of_mfma_peak": x["useful_tflops"] * ISSUED_PER_CMAC[prec] / 8.0 / PEAK_TFLOPS[prec],
            "xeb": x["F"], "oracle_check": x["oracle"],
            "err_bound": ERR_BOUND[prec], "kernel_time_share": x["share"],
            "roofline": roofline(x["prof"], prec), "plan_compile_s": x["t_plan"],
            "generic_kernel": {
                "gbs": x["prof"]["generic"]["bytes"] / max(x["prof"]["generic"]["seconds"], 1e-30) / 1e9,
                "hbm_frac": x["prof"]["generic"]["bytes"] / max(x["prof"]["generic"]["seconds"], 1e-30)
                            / (HBM_PEAK_GBS * 1e9),
                "launches": x["prof"]["generic"]["launches"], "seconds": x["prof"]["generic"]["seconds"]},
            "top_nodes": x["top_nodes"],
            **compare.get(prec, {}),
        }
        for prec, x in results.items()
    }
    st = r["st"]
    out = {
        "metric": METRIC,
        "value": r["amps_per_s"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["sec"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD}: 36 qubits on a 6x6 grid, 12 cycles (ABCDCDAB + closing "
                        "layer), 10^4 strings with qubits 0-19 fixed, 2^10 slices",
            "strings": int(len(strings)),
            "distinct_strings": int(st["k_distinct"]),
            "slices": n_slices,
            "slices_per_step": 1 << args.stack_slices,
            "precision": head,
            "launch_form": "eager" if r["t_capture"] is None else "hipgraph",
        },
        "contraction_tflops_useful": r["useful_tflops"],
        "roofline": roofline(r["prof"], head),
        "forms": forms,
        "plan": {"tree_s": t_tree, "cmacs_full": st["cmacs_full"],
                 "cmacs_unsliced_tree": info["unsliced_cost"], "max_log2": info["max_log2"],
                 "estimated_s": info.get("seconds"), "workspace_gib": st["workspace_bytes"] / 2**30,
                 "sum_variants": st["sum_variants"], "evals_full": st["evals_full"]},
        "xeb": r["F"],
        "cpu_baseline": None,
    }
    if not args.no_batch and os.path.exists(BATCH_PLANS):
        # The batch workload in the same record: its split-FP16 hipGraph form,
        # one timed step.
        with open(BATCH_PLANS) as f:
            saved_batch = json.load(f)
        b = run_batch(args, saved_batch, ["split_fp16"], 1)
        out["batch32"] = {k: b[k] for k in ("metric", "value", "unit", "ms_per_step", "config", "forms")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(oracle_net, oracle_pairs, strings, sliced, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


BATCH_PLANS = os.path.join(ROOT, "tests", "data", "batch32_plans.json")
BATCH_SLICINGS = (6, 10, 16)
BATCH_SINGLE_SLICINGS = (0, 4, 8)
BATCH_SINGLE_LOG2 = (24, 26)  # largest tensors tried for a one-string tree (2^24, 2^26 complex):
                              # smaller ones cost more per string but let more strings share a block
BATCH_CMAC_RATE = 2.2e13      # complex MACs/s of a whole split-FP16 pass (36-qubit workload)
BATCH_LAUNCH_S = 8e-5         # per launch: small string blocks leave the kernels latency-bound
                              # (the batch ran 2-2.4 times its MAC-rate estimate, ~70-100 us
                              # per launch beyond it)
BATCH_PLAN_PROCS = 6          # circuits planned at once, one process each
BATCH_MULTI_MAX_STRINGS = 30000  # all-strings trees only for batches up to this size
BATCH_HBM_GIB = 270.0  # of the 288 GB of HBM, what the batch's workspaces may take
BATCH_MAX_STACK = 6


def batch_workload(i: int):
    from synth import batch_spec, batch_circuit, uniform_bitstrings

    sp = batch_spec(i)
    circ = batch_circuit(i)
    return sp, circ, uniform_bitstrings(circ.n_qubits, sp["k"], sp["string_seed"])


def run_batch(args, saved, precs, steps: int) -> dict:
    """Runs the batch plans `saved` (as written by --plan-only) whose
    estimate is within --batch-max-seconds, in the precisions `precs`, and
    returns the result record."""
    import torch
    from paper_2108_05665_amd import xeb

    def included(rec):
        # Every circuit with a plan within the budget, estimated at most
        # --batch-max-seconds per contraction (the run's cap).
        est = rec.get("estimated_s", rec.get("info", {}).get("seconds", float("inf")))
        return "children" in rec and est <= args.batch_max_seconds

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    total_k = 0
    specs = []
    results = {}
    for prec in precs:
        plans, amps = [], []
        for rec in saved["plans"]:
            if not included(rec):
                continue
            sp, circ, strings = batch_workload(rec["i"])
            plan = xeb.Plan(circ, strings, rec["children"], rec["sliced"], precision=prec,
                            memory_budget=rec.get("budget_bytes", saved["budget"]),
                            stack_slices=rec.get("stack_slices", 0))
            if not args.no_autotune:
                plan.autotune(reps=2)
            plans.append(plan)
            amps.append(plan.new_amps())
            if prec == precs[0]:
                total_k += len(strings)
                specs.append({"circuit": rec["i"], "qubits": circ.n_qubits, "cycles": sp["cycles"],
                              "strings": sp["k"], "tree": rec.get("tree"),
                              "slices": 1 << len(rec["sliced"]), "stacked": rec.get("stack_slices", 0),
                              "string_blocks": rec.get("n_blocks"), "estimated_s": rec.get("estimated_s")})
        log(f"{prec}: {len(plans)} plans bound, "
            f"{sum(p.stats()['workspace_bytes'] for p in plans) / 2**30:.1f} GiB of workspace")

        def eager_step():
            for plan, a in zip(plans, amps):
                a.zero_()
                plan.contract(a)
            return [plan.fidelity(a) for plan, a in zip(plans, amps)]

        t0 = time.perf_counter()
        F_eager = eager_step()
        torch.cuda.synchronize()
        sec_eager = time.perf_counter() - t0
        eager_amps = [a.cpu() for a in amps]
        log(f"{prec}: eager loop {sec_eager:.2f} s")
        batch = xeb.BatchSet(plans, amps)
        log(f"{prec}: {len(batch.batches)} graphs of at most {xeb.BATCH_MAX_NODES} nodes, "
            f"{len(batch.eager)} plans eager")
        batch.launch()
        batch.fidelities()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            batch.launch()
            log(f"{prec}: graph step {k + 1}/{steps} launched")
        F = batch.fidelities()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        same = all(torch.equal(a.cpu(), b) for a, b in zip(amps, eager_amps))
        log(f"{prec}: graph {sec:.2f} s per batch ({total_k / sec:.0f} amplitudes/s), "
            f"graph == eager: {same}")
        results[prec] = dict(sec=sec, sec_eager=sec_eager, F=F, same=same,
                             F_diff=max(abs(a - b) for a, b in zip(F, F_eager)),
                             graphs=len(batch.batches), eager=len(batch.eager))
        batch.close()
        for plan in plans:
            plan.close()
        del amps, eager_amps
        torch.cuda.empty_cache()
    head = results[precs[0]]
    out = {
        "metric": "amplitudes/sec (32-circuit batch, all slices, hipGraph launches)",
        "value": total_k / head["sec"],
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": 1e3 * head["sec"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[precs[0]],
        "data": "synthetic",
        "config": {"workload": "batch32: 32 circuits, 30-40 qubits on rectangular grids, 10-14 "
                               "cycles, 10^3-10^5 uniform strings each, each planned within a 32nd "
                               "of 270 GiB (a tree for one string with the strings in blocks, or "
                               "one for all strings); the circuits estimated above "
                               f"{args.batch_max_seconds} s per contraction left out",
                   "strings": total_k, "budget_gib_per_circuit": saved["budget"] / 2**30,
                   "circuits": specs,
                   "left_out": [{"circuit": r["i"],
                                 "estimated_s": r.get("estimated_s"),
                                 "reason": "estimated above the cap" if "children" in r
                                 else "no plan within the budget"}
                                for r in saved["plans"] if not included(r)]},
        "forms": {prec: {"amplitudes_per_s": total_k / r["sec"], "sec_per_batch": r["sec"],
                         "eager_loop_s": r["sec_eager"],
                         "graph_speedup_vs_eager_loop": r["sec_eager"] / r["sec"],
                         "graph_equals_eager": r["same"], "max_xeb_diff_graph_vs_eager": r["F_diff"],
                         "graphs": r["graphs"], "plans_run_eagerly": r["eager"],
                         "xeb": r["F"]}
                  for prec, r in results.items()},
    }
    return out


def _batch_estimate(st) -> float:
    # Seconds on one GPU: complex MACs at the split form's measured
    # whole-pass rate plus a fixed cost per kernel launch.
    return st["cmacs_full"] / BATCH_CMAC_RATE + st["evals_full"] * BATCH_LAUNCH_S


def _batch_plan_part(i: int, budget: int, max_seconds: float, parts: str, skip: bool = False) -> dict:
    if skip:
        return {"i": i, "included": False, "reason": "not planned (--batch-skip)",
                "log": f"circuit {i}: not planned (--batch-skip)"}
    path = os.path.join(parts, f"{i}.json")
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("budget") == budget:
            return rec["plan"]
    rec = _batch_plan_one(i, budget, max_seconds)
    with open(path + ".tmp", "w") as f:
        json.dump({"budget": budget, "plan": rec}, f)
    os.replace(path + ".tmp", path)
    return rec


def _batch_plan_one(i: int, budget: int, max_seconds: float) -> dict:
    """Plan circuit i of the batch within `budget` bytes (a process of the
    planning pool): the cheaper by estimated time of (a) the tree annealed
    for one string (uniform strings share little) with the fewest sliced legs
    that compile, the strings cut into blocks by the plan compiler, and (b)
    a greedy tree for all strings at once (shared subtrees evaluated once per
    key) at a few slice counts."""
    from paper_2108_05665_amd import planner, xeb

    sp, circ, strings = batch_workload(i)
    t0 = time.perf_counter()
    cands = []
    for log2 in BATCH_SINGLE_LOG2:
        for ns in BATCH_SINGLE_SLICINGS:
            ch, sl, info = planner.plan(circ, strings[:1], n_sliced=ns, trials=8, seed=1,
                                        anneal_steps=1_000_000, anneal_restarts=2, workers=1,
                                        anneal_objective="paper", size_log2_max=log2)
            try:
                st = xeb.Plan(circ, strings, ch, sl, memory_budget=budget, bind=False).stats()
            except xeb.XebError:
                continue
            cands.append(("single", ch, sl, info, st))
            break
    log(f"circuit {i}: single-string tree done at {time.perf_counter() - t0:.0f} s")
    for ns in BATCH_SLICINGS:
        if len(strings) > BATCH_MULTI_MAX_STRINGS:
            break
        ch, sl, info = planner.plan(circ, strings, n_sliced=ns, trials=4, seed=0, table_bytes_max=budget)
        try:
            st = xeb.Plan(circ, strings, ch, sl, memory_budget=budget, bind=False).stats()
        except xeb.XebError:
            continue
        cands.append(("multi", ch, sl, info, st))
        log(f"circuit {i}: all-strings tree at s = {ns} done at {time.perf_counter() - t0:.0f} s")
    if not cands:
        return {"i": i, "included": False, "reason": "no plan within the budget",
                "log": f"circuit {i}: no plan fits {budget} bytes"}
    kind, ch, sl, info, st = min(cands, key=lambda c: _batch_estimate(c[4]))
    best = {"i": i, "tree": kind, "children": [[int(a), int(b)] for a, b in ch],
            "sliced": [int(x) for x in sl], "info": info,
            "workspace_bytes": int(st["workspace_bytes"]), "n_blocks": int(st["n_blocks"]),
            "cmacs_full": float(st["cmacs_full"]), "evals_full": float(st["evals_full"]),
            "estimated_s": _batch_estimate(st),
            "candidates": [{"tree": c[0], "sliced": len(c[2]), "estimated_s": _batch_estimate(c[4]),
                            "cmacs_full": float(c[4]["cmacs_full"]), "n_blocks": int(c[4]["n_blocks"])}
                           for c in cands]}
    # Stack the low slice bits as far as the budget allows without more
    # string blocks (at most 2^6 slices per launch).  A plan that already
    # cuts its strings into blocks would need more of them (stacked tables
    # are 2^J times larger), so only one-block plans try.
    J, stj = 0, None
    if best["sliced"] and best["n_blocks"] == 1:
        J, stj = planner.choose_stacking(circ, strings, best["children"], best["sliced"], budget,
                                         max_stack=BATCH_MAX_STACK, max_blocks=1)
    best["stack_slices"] = J
    if J:
        best.update(workspace_bytes=int(stj["workspace_bytes"]), evals_full=float(stj["evals_full"]),
                    estimated_s=_batch_estimate(stj))
    best["included"] = best["estimated_s"] <= max_seconds
    if not best["included"]:
        best["reason"] = "estimated above --batch-max-seconds"
    best["log"] = (f"circuit {i}: {circ.n_qubits} qubits, {sp['cycles']} cycles, k={sp['k']}, {kind} tree, "
                   f"s={len(best['sliced'])}, J={J}, {best['n_blocks']} blocks, "
                   f"estimated {best['estimated_s']:.3f} s")
    return best


def batch_main(args) -> int:
    """The batch workload: 32 circuits of 30-40 qubits (rectangular grids,
    10-14 cycles) with 10^3-10^5 uniform strings each.  Every circuit is
    planned against a per-circuit HBM budget of a 32nd of 270 GiB (all
    circuits resident for one launch): the cheaper by estimated time of a
    tree annealed for one string (fewest sliced legs that compile, strings
    cut into blocks) and a greedy tree for all strings at once (a few slice
    counts); then HBM left unused goes to the costliest plans while it cuts
    their string blocks.  A step is the contraction of all slices of
    all circuits and their XEB: `value` is total amplitudes / s of one
    launch of the whole batch as hipGraphs of at most 49152 nodes each (a
    plan too large for one graph runs eagerly inside the step); a sequential
    eager loop over the circuits is timed beside it.  Circuits estimated above --batch-max-seconds
    (the deep 36-40 qubit ones need minutes to hours each on one GPU) are
    listed with their estimates and left out of the launch."""
    import numpy as np

    # One launch holds all 32 circuits, so all their workspaces are resident at
    # once: each circuit's budget is a 32nd of the HBM left for workspaces.
    budget = int((args.batch_budget_gib if args.batch_budget_gib else BATCH_HBM_GIB / 32) * 2**30)
    if args.plan_only:
        import multiprocessing as mp

        from paper_2108_05665_amd import xeb

        # Each circuit's plan is also kept in PATH.parts/ as it completes, so an
        # interrupted run resumes where it stopped.
        parts = args.plan_only + ".parts"
        os.makedirs(parts, exist_ok=True)
        skip = {int(x) for x in args.batch_skip.split(",") if x.strip()}
        with mp.get_context("fork").Pool(BATCH_PLAN_PROCS) as pool:
            plans = pool.starmap(_batch_plan_part,
                                 [(i, budget, args.batch_max_seconds, parts, i in skip) for i in range(32)])
        for rec in plans:
            log(rec["log"])
        # All circuits are resident in one launch: the HBM the plans leave
        # unused goes to the costliest ones, as long as it cuts their string
        # blocks (fewer blocks: fewer launches, less repeated work).
        spare = int(BATCH_HBM_GIB * 2**30) - sum(r["workspace_bytes"] for r in plans if "children" in r)
        for rec in sorted((r for r in plans if "children" in r), key=lambda r: -r["estimated_s"]):
            if spare <= 0 or rec["n_blocks"] == 1:
                continue
            sp, circ, strings = batch_workload(rec["i"])
            b2 = rec["workspace_bytes"] + spare
            st2 = xeb.Plan(circ, strings, rec["children"], rec["sliced"], memory_budget=b2, bind=False,
                           stack_slices=rec["stack_slices"]).stats()
            if st2["n_blocks"] < rec["n_blocks"]:
                spare -= int(st2["workspace_bytes"]) - rec["workspace_bytes"]
                log(f"circuit {rec['i']}: {rec['n_blocks']} -> {st2['n_blocks']} string blocks with "
                    f"{b2 / 2**30:.1f} GiB")
                rec.update(budget_bytes=int(b2), workspace_bytes=int(st2["workspace_bytes"]),
                           n_blocks=int(st2["n_blocks"]), cmacs_full=float(st2["cmacs_full"]),
                           evals_full=float(st2["evals_full"]), estimated_s=_batch_estimate(st2))
        with open(args.plan_only, "w") as f:
            json.dump({"workload": "batch32", "budget": budget,
                       "made_by": "python bench.py --workload batch32 --plan-only PATH "
                                  f"--batch-max-seconds {args.batch_max_seconds:g}"
                                  + (f" --batch-skip {args.batch_skip}" if args.batch_skip else ""),
                       "max_seconds": args.batch_max_seconds, "plans": plans}, f)
        return 0
    if not args.tree:
        print("batch32 needs --tree PATH from a --plan-only run (planning takes minutes)",
              file=sys.stderr)
        return 2
    with open(args.tree) as f:
        saved = json.load(f)
    assert saved["workload"] == "batch32"
    out = run_batch(args, saved, [p.strip() for p in args.precisions.split(",") if p.strip()], args.steps)
    print(json.dumps(out), flush=True)
    return 0


SHARE53 = "share_53q_m14"
SHARE53_PLAN = os.path.join(ROOT, "tests", "data", f"{SHARE53}_plan.json")
SHARE53_SINGLE_PLAN = os.path.join(ROOT, "tests", "data", f"{SHARE53}_single_plan.json")
SHARE53_GOLDEN = os.path.join(ROOT, "tests", "golden", f"{SHARE53}_partials.json")
SHARE53_BUDGET = 270 * 2**30


def share53_main(args) -> int:
    """One GPU's share of the 53-qubit contraction (6x9 grid minus site
    (0, 4), 14 cycles, 3 * 10^5 uniform strings), in one of two plans:

    * "single" (default): the tree annealed for one amplitude (the paper's
      objective, largest tensor 2^28), no sliced legs: with 270 GiB of HBM the
      plan compiler cuts the strings into blocks of 32.  The first
      --share53-strings strings are contracted completely and timed; the full
      share is extrapolated as 3 * 10^5 strings at that rate (each string's
      work is the same: the uniform strings share only the smallest
      subtrees).  The amplitudes of those strings give their XEB and the
      Porter-Thomas mean of 2^n |amp|^2 (both near 0 and 1 for uniform
      strings), and the first 8 are checked against the same tree with 4
      sliced legs summed over its 16 slices.
    * "sliced": the fixture's tree and 2^25 slices compiled within 270 GiB;
      a contiguous block of slices [0, --slice-block) contracted with the memo
      tables; the time per slice and the full contraction extrapolated as
      t_block * 2^s / block, with single-slice partials of the first strings
      checked against the stored FP64 oracle values (a partial block yields
      no amplitude)."""
    import numpy as np

    from synth import config_circuit, config_bitstrings
    from paper_2108_05665_amd import planner, xeb

    circ = config_circuit(SHARE53)
    strings = config_bitstrings(SHARE53, circ.n_qubits)
    single = args.share53_tree == "single"
    if args.plan_only:
        t0 = time.perf_counter()
        if single:
            ch, sl, info = planner.plan(circ, strings[:1], n_sliced=0, trials=16, seed=1,
                                        anneal_steps=10_000_000, anneal_restarts=8, workers=8,
                                        anneal_objective="paper", size_log2_max=28)
        else:
            ch, sl, info = planner.plan(circ, strings, n_sliced=20, trials=8, seed=0,
                                        anneal_steps=200000, anneal_restarts=4, workers=4,
                                        anneal_objective="paper", table_bytes_max=250 * 2**30,
                                        memory="tables", slicing="paper", slice_every=5000,
                                        size_log2_max=34)
        with open(args.plan_only, "w") as f:
            json.dump({"workload": SHARE53, "children": [[int(a), int(b)] for a, b in ch],
                       "sliced": [int(x) for x in sl], "info": info,
                       "made_by": f"python bench.py --workload share53 --share53-tree "
                                  f"{args.share53_tree} --plan-only PATH"}, f)
        log(f"planned in {time.perf_counter() - t0:.0f} s: cost {info['cost']:.3e}, s = {len(sl)}")
        return 0
    import torch

    precs = [p.strip() for p in (args.precisions or "split_fp16").split(",") if p.strip()]
    if single:
        return share53_single(args, circ, strings, precs)
    with open(SHARE53_PLAN) as f:
        fx = json.load(f)
    n_slices = 1 << len(fx["sliced"])
    block = min(args.slice_block, n_slices)
    gold = None
    if os.path.exists(SHARE53_GOLDEN):
        with open(SHARE53_GOLDEN) as f:
            gold = json.load(f)
    results = {}
    for prec in precs:
        t0 = time.perf_counter()
        plan = xeb.Plan(circ, strings, fx["children"], fx["sliced"], precision=prec,
                        memory_budget=SHARE53_BUDGET)
        st = plan.stats()
        t_plan = time.perf_counter() - t0
        log(f"{prec}: plan compiled and bound in {t_plan:.1f} s, workspace "
            f"{st['workspace_bytes'] / 2**30:.1f} GiB, {st['n_blocks']} string blocks")
        parity = None
        if gold is not None:
            errs = []
            for sigma in gold["sigmas"]:
                a = plan.new_amps()
                plan.contract(a, sigma, sigma + 1)
                torch.cuda.synchronize()
                got = a[: gold["n_strings"]].cpu().numpy()
                ref = np.array([complex(*x["partial"]) for x in gold["partials"] if x["sigma"] == sigma])
                errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
                log(f"{prec}: slice {sigma} partials vs oracle {errs[-1]:.2e}")
            parity = {"sigmas": gold["sigmas"], "strings": gold["n_strings"], "rel_err": errs}
        amps = plan.new_amps()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(0, block, 16):
            plan.contract(amps, b, min(b + 16, block))
            torch.cuda.synchronize()
            log(f"{prec}: slices [0, {min(b + 16, block)}) done, {time.perf_counter() - t0:.1f} s")
        sec = time.perf_counter() - t0
        results[prec] = {"block_s": sec, "per_slice_s": sec / block,
                         "extrapolated_full_s": sec * n_slices / block,
                         "extrapolated_amplitudes_per_s": len(strings) / (sec * n_slices / block),
                         "plan_s": t_plan, "workspace_gib": st["workspace_bytes"] / 2**30,
                         "oracle_partials": parity,
                         "cmacs_per_slice_block_avg": st["cmacs_full"] / n_slices}
        plan.close()
        del amps
        torch.cuda.empty_cache()
    head = results[precs[0]]
    out = {
        "metric": "amplitudes/sec (53-qubit share: slice block, extrapolated to all slices)",
        "value": head["extrapolated_amplitudes_per_s"], "unit": "amplitudes/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": 1e3 * head["block_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[precs[0]], "data": "synthetic",
        "config": {"workload": f"{SHARE53}: 53 qubits (6x9 grid minus (0, 4)), 14 cycles, 3*10^5 "
                               f"uniform strings, 2^{len(fx['sliced'])} slices, block of {block}",
                   "slices": n_slices, "block": block},
        "forms": results, "plan": fx["info"],
    }
    print(json.dumps(out), flush=True)
    return 0


def share53_single(args, circ, strings, precs) -> int:
    import numpy as np
    import torch

    from paper_2108_05665_amd import planner, xeb

    with open(SHARE53_SINGLE_PLAN) as f:
        fx = json.load(f)
    k = min(args.share53_strings, len(strings))
    sub = strings[:k]
    results = {}
    for prec in precs:
        t0 = time.perf_counter()
        plan = xeb.Plan(circ, sub, fx["children"], [], precision=prec, memory_budget=SHARE53_BUDGET)
        st = plan.stats()
        t_plan = time.perf_counter() - t0
        log(f"{prec}: plan for {k} strings compiled and bound in {t_plan:.1f} s, workspace "
            f"{st['workspace_bytes'] / 2**30:.1f} GiB, {st['n_blocks']} string blocks, "
            f"{st['cmacs_full']:.3e} complex MACs")
        tune = None
        if not args.no_autotune:
            r = plan.autotune(reps=1)
            tune = {k: r[k] for k in ("nodes_tuned", "nodes_changed", "candidates", "tuning_seconds")}
            log(f"{prec}: autotuned {r['nodes_tuned']} nodes in {r['tuning_seconds']:.1f} s, "
                f"{r['nodes_changed']} changed")
        amps = plan.new_amps()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.contract(amps)
        F = plan.fidelity(amps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        a = amps.cpu().numpy()
        # Where the time goes: one more pass with the library's per-node
        # events.
        plan.set_profiling(True)
        prof_amps = plan.new_amps()
        plan.contract(prof_amps)
        torch.cuda.synchronize()
        nodes = []
        for ns in plan.all_node_stats():
            np_ = plan.read_node_profile(ns["node"])
            if np_["launches"] == 0 or np_["seconds"] <= 0:
                continue
            nodes.append({"node": ns["node"], "kernel": ns["kernel"], "tile": ns["tile"],
                          "keys": ns["variants"], "m_k_n_bits": [ns["m_bits"], ns["k_bits"], ns["n_bits"]],
                          "launches": np_["launches"], "seconds": np_["seconds"],
                          "algorithmic_tflops": 8.0 * np_["cmacs"] / np_["seconds"] / 1e12,
                          "gbs": np_["bytes"] / np_["seconds"] / 1e9})
        nodes.sort(key=lambda x: -x["seconds"])
        plan.set_profiling(False)
        del prof_amps
        pt = float(np.mean(np.ldexp(np.abs(a) ** 2, circ.n_qubits)))
        log(f"{prec}: {k} strings in {sec:.1f} s ({k / sec:.1f} amplitudes/s), XEB {F:.4f}, "
            f"mean 2^n|amp|^2 {pt:.4f}")
        plan.close()
        del amps
        torch.cuda.empty_cache()
        # The same tree with 4 sliced legs: 16 slices summed for the first 8 strings.
        st_ = planner.Structure(circ)
        cnt = planner.VariantCounter(sub[:8])
        ch = [tuple(x) for x in fx["children"]]
        sl = planner.order_slices(st_, ch, cnt, planner.greedy_slices(st_, ch, cnt, 4))
        p2 = xeb.Plan(circ, sub[:8], fx["children"], sl, precision=prec, memory_budget=SHARE53_BUDGET)
        b = p2.new_amps()
        p2.contract(b)
        torch.cuda.synchronize()
        sliced = b.cpu().numpy()
        p2.close()
        del b
        torch.cuda.empty_cache()
        diff = float(np.linalg.norm(a[:8] - sliced) / np.linalg.norm(sliced))
        log(f"{prec}: first 8 strings vs the 16-slice contraction: {diff:.2e}")
        results[prec] = {"strings": k, "seconds": sec, "amplitudes_per_s": k / sec,
                         "extrapolated_full_s": len(strings) * sec / k,
                         "cmacs": st["cmacs_full"],
                         "algorithmic_tflops": 8 * st["cmacs_full"] / sec / 1e12,
                         "n_blocks": st["n_blocks"], "workspace_gib": st["workspace_bytes"] / 2**30,
                         "plan_s": t_plan, "autotune": tune, "top_nodes": nodes[:10],
                         "xeb": F, "porter_thomas_mean": pt,
                         "sliced_check": {"strings": 8, "sliced_legs": len(sl), "rel_diff": diff}}
    head = results[precs[0]]
    out = {
        "metric": "amplitudes/sec (53-qubit share, full contraction of a string sample, "
                  "extrapolated to all strings)",
        "value": head["amplitudes_per_s"], "unit": "amplitudes/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": 1e3 * head["seconds"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[precs[0]], "data": "synthetic",
        "config": {"workload": f"{SHARE53}: 53 qubits (6x9 grid minus (0, 4)), 14 cycles, 3*10^5 "
                               f"uniform strings; single-amplitude tree, no slicing, strings in "
                               f"blocks under 270 GiB; the first {k} strings contracted",
                   "strings_total": len(strings), "strings_run": k},
        "forms": results, "plan": fx["info"],
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
