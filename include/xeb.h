/*
 * xeb.h — C ABI of the MI355X (gfx950) multi-tensor contraction library.
 *
 * The library computes the amplitudes <s_i|C|0^n> of a quantum circuit C for a
 * whole batch of bitstrings s_1..s_k by one sliced contraction of the circuit's
 * tensor network, reusing every sub-contraction that several strings (and
 * several slices) share, and reduces them to the linear XEB fidelity.
 *
 * Paper: Kalachev, Panteleev, Yung, "Multi-Tensor Contraction for XEB
 * Verification of Quantum Circuits" (arXiv 2108.05665).
 *   - amplitudes as contractions of per-string networks: section
 *     "Multi-batch simulator";
 *   - reuse of shared sub-expressions, lexicographic tuple order, one cached
 *     entry per subtree: section "Multi-tensor contraction algorithm" and
 *     Appendix C (procedures eval_all / eval');
 *   - pairwise contraction cost 2^(q+r): Appendix A; slicing: Appendix A,
 *     paragraph "Slicing";
 *   - linear XEB: Eq. (1) of the Introduction.
 *
 * Conventions for every call:
 *   - Every call returns an int: XEB_OK (0) or a negative error code.  No call
 *     throws across the ABI.  xeb_last_error() returns a thread-local message
 *     describing the last failure on the calling thread.
 *   - Handles are opaque.  The caller owns every buffer it passes; the plan
 *     owns its host-side schedule; device memory for the plan's tables comes
 *     from the caller (xeb_plan_bind_workspace).
 *   - Pointers named "host" point to host memory, "dev" to device memory on
 *     the plan's device.  A hipStream_t is passed as void* (NULL = the null
 *     stream).
 *   - Calls on one plan must be ordered: the plan keeps which slice's tables
 *     are resident, so two xeb_contract calls on one plan must not run
 *     concurrently and must use streams ordered with each other.
 */
#ifndef XEB_H
#define XEB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define XEB_OK 0
#define XEB_EINVAL (-1)  /* bad argument: circuit, tree, slice list, range, sizes */
#define XEB_ENOMEM (-2)  /* host allocation failed, or workspace too small / over budget */
#define XEB_EHIP (-3)    /* HIP runtime error; the message carries HIP's text */
#define XEB_ESTATE (-4)  /* call out of order (e.g. contract before bind) */
#define XEB_ELIMIT (-5)  /* a documented size limit exceeded (e.g. batch graph nodes) */
#define XEB_EABORT (-6)  /* injected abort (xeb_options_t.abort_after_slices); the work
                            done before it is kept and can be resumed */

/* Opaque plan handle. */
typedef struct xeb_plan* xeb_plan_t;

/* ---- precision of the contraction kernels ------------------------------ */
/*
 * Tables are complex64 in HBM in every mode; the precision selects how the
 * MFMA contractions multiply (the generic kernel always works in FP32):
 *   C64: FP32 MFMA (v_mfma_f32_32x32x2f32 / 16x16x4f32), FP32 accumulation.
 *   SPLIT_FP16: each operand float x, scaled by a power of two 2^e chosen from
 *     the tensor's largest magnitude, is split into hi = fp16(x 2^e) and
 *     lo = fp16(x 2^e - hi); hi.hi + hi.lo + lo.hi accumulate in FP32 on FP16
 *     MFMA (lo.lo dropped); the result is scaled back by 2^-(eA+eB).
 *   SPLIT_BF16: the same with bf16 halves and no scale.
 */
#define XEB_PREC_C64 0
#define XEB_PREC_SPLIT_FP16 1
#define XEB_PREC_SPLIT_BF16 2

/*
 * A circuit: gates in time order.
 *   gate_qubits (host) int32 [n_gates][2]: the qubits of gate g; column 1 is -1
 *     for a one-qubit gate.  The two qubits of a two-qubit gate differ.
 *   gate_mats (host) double [n_gates][32]: (re, im) pairs.  A two-qubit gate is
 *     a 4x4 row-major matrix U[out][in] with basis index 2*b_q0 + b_q1; a
 *     one-qubit gate uses the first 4 complex entries as a 2x2 row-major
 *     matrix U[out][in] (the rest is ignored).
 *   1 <= n_qubits <= 64.
 */
typedef struct {
  int32_t n_qubits;
  int32_t n_gates;
  const int32_t* gate_qubits;
  const double* gate_mats;
} xeb_circuit_t;

/*
 * A binary contraction tree (section "Tensor network contraction": leaves are
 * the tensors, internal nodes the pairwise contractions).
 *   Node ids: 0..n_leaves-1 are the network's leaves (xeb_network_describe
 *   order); internal node n_leaves+i has children children[2i], children[2i+1],
 *   both ids smaller than n_leaves+i.  Every node except the last (the root)
 *   is the child of exactly one internal node.  n_leaves >= 1; children may be
 *   NULL when n_leaves == 1.
 *   The left child is the first of the pair; variables are ordered as they
 *   occur in the tree, left first (Appendix C).
 */
typedef struct {
  int32_t n_leaves;
  const int32_t* children; /* host, int32 [n_leaves-1][2] */
} xeb_tree_t;

typedef struct {
  int32_t fuse_1q;        /* 1: fuse one-qubit gates into two-qubit gates (default 1) */
  int32_t fold_kets;      /* 1: project |0> into the first gate on each qubit (default 1) */
  int32_t precision;      /* XEB_PREC_* (default XEB_PREC_C64) */
  int32_t device;         /* HIP device ordinal of the plan (default 0) */
  uint64_t memory_budget; /* max workspace bytes, 0 = unlimited (default 0) */
  int32_t trace;          /* >0: print one JSON line per node at plan creation */
  int32_t force_generic;  /* 1: use the generic per-element kernel for every node */
  int32_t max_ksplit;     /* MFMA split-K chunks per node: 0 = automatic (up to 64),
                             1 = never split, else a power of two bounding the split */
  double mfma_min_cmacs;  /* a node evaluation with fewer complex MACs than this (or
                             fewer than 8 rows) uses the generic kernel; 0 = default 2^23 */
  int32_t stack_slices;   /* J, 0 <= J <= s and n_qubits + J <= 64 (default 0): the J
                             lowest slice-id bits are evaluated together.  Their sliced
                             legs become variables exactly like output legs (Appendix A,
                             "Slicing": a sliced leg is summed over its values; section
                             "Multi-batch simulator": fixed legs make leaves variables),
                             so every node keeps one table entry per distinct (string
                             key, low slice key) and one xeb_contract step covers 2^J
                             consecutive slices.  Tables of nodes that depend on those
                             bits grow by 2^(their count); launches fall by up to 2^J,
                             and a node whose low slice bits are sparse is no longer
                             recomputed for slices that do not change its key. */
  uint64_t open_qubits;   /* multi-batch output (section "Multi-batch simulator"): the
                             output legs of these qubits (bit q = qubit q, at most 16
                             of them, w = their count) stay open, so each string yields
                             the 2^w amplitudes of the strings that agree with it on
                             every other qubit; the strings' open bits select nothing
                             and only the XEB reads them.  Default 0. */
  int64_t abort_after_slices; /* failure injection for stop / resume (slices are
                             independent, Appendix A, "Slicing", so recovery means
                             contracting the missing slice range): > 0 makes
                             xeb_contract stop once this plan has contracted that many
                             slices over all its calls and return XEB_EABORT (see there).
                             0 = never (default). */
} xeb_options_t;

typedef struct {
  int64_t n_leaves;
  int64_t n_internal;
  int64_t k;                 /* strings passed, duplicates included */
  int64_t k_distinct;        /* distinct strings */
  int32_t n_qubits;
  int32_t n_sliced;          /* s; the plan has 2^s slices */
  int64_t sum_variants;      /* sum over internal nodes of |t_T| (distinct keys: string key
                                and, with stacked slices, low slice key) */
  int64_t max_tensor_elems;  /* largest tensor per variant (after slicing), elements */
  double cmacs_per_slice;    /* sum_T |t_T| 2^(q_T+r_T): one evaluation of every node */
  double cmacs_full;         /* complex MACs for all 2^s slices under the plan's schedule */
  double rw_elems_full;      /* elements read+written by all contractions, all slices */
  double evals_full;         /* node evaluations (kernel launches) for all slices */
  uint64_t workspace_bytes;
  int64_t n_blocks;          /* string blocks chosen by the dry run (1 = all strings at once) */
  int32_t n_stacked;         /* J of xeb_options_t.stack_slices */
  int32_t n_open;            /* w: open output qubits; amps hold k * 2^w values */
  int64_t slices_done;       /* slices contracted by xeb_contract over the plan's life */
} xeb_stats_t;

#define XEB_KERNEL_GENERIC 0  /* per-element kernel (small or sparse nodes) */
#define XEB_KERNEL_MFMA 1     /* FP32-MFMA stacked GEMM */

/* Per internal node; key counts are summed over the string blocks (with one
 * block, `variants` is the node's exact evaluation count |t_T| per slice). */
typedef struct {
  int32_t left, right;       /* child node ids */
  int64_t variants;          /* distinct string keys of this node */
  int64_t left_variants, right_variants;
  int32_t m_bits, n_bits, k_bits; /* free legs of left, free legs of right, shared legs */
  uint64_t slice_mask;       /* bit j set: the node depends on sliced leg j */
  int32_t kernel;            /* XEB_KERNEL_* (first block) */
  int32_t swapped;           /* 1: the kernel runs with the right child as the row operand
                                (per-element kernel, row-streaming form: 1 = the left
                                child's rows are streamed, 0 = the right child's) */
  int32_t tile;              /* per-element kernel: -1 = one thread per output element,
                                -2 = row-streaming form (K <= 16, streamed side >= 8 bits,
                                other side <= 6 bits);
                                MFMA tile shape: 0 = 64x64, 1 = 32x128, 2 = 16x256, 3 = 64x16,
                                4 = 128x128, 5 = 128x128 on eight waves with double-
                                buffered LDS (split forms), 6 = 128x128 and 7 = 256x128
                                on operands converted to hi/lo planes first (split
                                forms, K >= 16, room in the planes region) */
  int32_t ksplit;            /* MFMA: K chunks summed by a second kernel (1 = no split) */
  int32_t k_slab;            /* MFMA: complex K values staged per LDS step */
  int32_t k_groups;          /* MFMA: groups of four waves splitting K inside a workgroup */
  int32_t pair_mode;         /* MFMA key form: 0 = every (left, right) pair is a key,
                                1 = stacked product with a pair table, 2 = keyed (one
                                GEMM per key; the key set is too sparse to stack) */
  double cmacs_per_eval;     /* |t_T| 2^(q+r) */
} xeb_node_stats_t;

/* Fill *opt with the defaults listed above. */
void xeb_options_default(xeb_options_t* opt);

/* Thread-local text of the last error (never NULL). */
const char* xeb_last_error(void);

/*
 * The tensor network of a circuit (section "Multi-batch simulator"), host only,
 * no device needed.  Convention, shared with any independent implementation:
 *  1. Fusion (fuse_1q): walk the gates with a pending one-qubit product P_q per
 *     qubit; a one-qubit gate U on q sets P_q := U P_q; a two-qubit gate W on
 *     (a, b) is emitted as W (P_a (x) P_b) and clears P_a, P_b.  Afterwards each
 *     qubit q with pending P_q (ascending q) left-multiplies it into the last
 *     emitted two-qubit gate touching q (on q's side), or, if none touches q,
 *     is emitted as a one-qubit gate.  Without fusion the gates are emitted as
 *     given.
 *  2. Leaves: ket leaves first (ascending qubit), then one leaf per emitted
 *     gate.  With fold_kets a ket leaf exists only for a qubit no emitted gate
 *     touches; the others are projected onto |0> inside their first gate.
 *  3. Legs are wire segments in creation order: ket segments, then per emitted
 *     gate one output segment per qubit (first qubit's, then second's).
 *  4. A gate leaf's legs: its input segments (a folded input is absent), then
 *     its output segments.  The last segment of each qubit is its open output
 *     leg; it is fixed by that qubit's bit of the string.
 * Outputs (host, any may be NULL to query sizes first):
 *   *n_leaves, *n_legs, *n_leaf_legs (total entries of leaf_legs);
 *   leaf_leg_offsets int32 [n_leaves+1] (CSR offsets into leaf_legs);
 *   leaf_legs int32 [n_leaf_legs];
 *   leg_qubit int32 [n_legs]: q if the leg is qubit q's output leg, else -1.
 * Errors: XEB_EINVAL for a malformed circuit.
 */
int xeb_network_describe(const xeb_circuit_t* circuit, int32_t fuse_1q, int32_t fold_kets,
                         int32_t* n_leaves, int32_t* n_legs, int32_t* n_leaf_legs,
                         int32_t* leaf_leg_offsets, int32_t* leaf_legs, int32_t* leg_qubit);

/*
 * Compile a plan (host only; no device memory is touched until bind).
 *   bitstrings (host) uint64 [k]: bit q = qubit q; duplicates allowed (each
 *     occurrence receives the amplitude).  k >= 0; bits at or above n_qubits
 *     must be zero.
 *   contraction_tree: over the leaves of xeb_network_describe(circuit,
 *     opt->fuse_1q, opt->fold_kets).
 *   sliced_legs (host) int32 [s]: distinct internal (non-output) leg ids; slice
 *     id sigma fixes leg sliced_legs[j] to bit j of sigma (Appendix A,
 *     "Slicing").  0 <= s <= 40.  May be NULL when s == 0.
 *   opt: NULL for defaults.
 * The plan dedupes the strings, orders every node's variants in the
 * lexicographic order of Appendix C, precomputes gather maps, picks a kernel
 * per node, sizes its device workspace by a dry run (Appendix C, "emulation
 * mode") and builds the leaf tensors in FP64 before rounding them to the
 * kernel precision.
 * Errors: XEB_EINVAL (malformed input), XEB_ENOMEM (host memory, or the
 * workspace exceeds opt->memory_budget).
 */
int xeb_plan_create(const xeb_circuit_t* circuit, const uint64_t* bitstrings, int64_t k,
                    const xeb_tree_t* contraction_tree, const int32_t* sliced_legs, int32_t s,
                    const xeb_options_t* opt, xeb_plan_t* out);
/* Memory: every node keeps the table of all its keys among the strings being
 * contracted.  When opt->memory_budget is set and that does not fit, the
 * distinct strings, sorted in the lexicographic tuple order of Appendix C,
 * are cut into 2, 4, 8, ... contiguous blocks contracted one after another
 * (a block's keys share the left spine, as in eval'); the first count that
 * fits is kept (xeb_stats_t.n_blocks). */

/* Device bytes the plan needs (from the dry run). */
int xeb_plan_workspace_bytes(xeb_plan_t plan, uint64_t* bytes);

/*
 * Give the plan its device workspace: dev_ptr (device, 256-byte aligned, at
 * least xeb_plan_workspace_bytes) stays owned by the caller and must outlive
 * the plan's use.  Uploads the leaf tables and gather maps (synchronous).
 * Rebinding is allowed; it invalidates resident tables.
 * Errors: XEB_EINVAL (NULL or misaligned), XEB_ENOMEM (too small), XEB_EHIP.
 */
int xeb_plan_bind_workspace(xeb_plan_t plan, void* dev_ptr, uint64_t bytes);

/*
 * Contract slices [slice_begin, slice_end) (0 <= begin <= end <= 2^s) and add
 * each string's sum over those slices into amps.
 *   amps (device) complex128 [k] ((re, im) doubles), in the order of the
 *     bitstrings passed to xeb_plan_create; zero it before the first call.
 *     With w open qubits it is complex128 [k][2^w]: entry (i, o) is the
 *     amplitude of string i with its open qubits set to o (bit j of o = the
 *     j-th open qubit in increasing order).
 *     Each call adds its slices' partial amplitudes (FP32 complex results of
 *     the contraction, widened to FP64) in increasing slice order with
 *     Neumaier compensation and folds the compensation into amps at the end
 *     of the call, so results are deterministic for a given split of the
 *     slice range.  Repeated calls accumulate; the full amplitude needs the
 *     calls to cover [0, 2^s) exactly once.
 *   stream: hipStream_t (as void*); all work is enqueued on it; the call
 *     returns without waiting.
 * Within a call, a node whose slice bits do not change between consecutive
 * slices keeps its resident table instead of being contracted again; nothing
 * is carried from one call to the next.
 * With xeb_options_t.abort_after_slices = A > 0 and D slices contracted by
 * earlier calls, a call whose range holds more than max(A - D, 0) slices
 * contracts only its first max(A - D, 0) slices [begin, stop), folds them
 * into amps as a complete call over [begin, stop) would, and returns
 * XEB_EABORT; the message names stop.  A later call over [stop, end) gives
 * the same amps as the two calls [begin, stop), [stop, end) without an abort.
 * Errors: XEB_EINVAL (range), XEB_ESTATE (no workspace), XEB_EABORT, XEB_EHIP.
 */
int xeb_contract(xeb_plan_t plan, int64_t slice_begin, int64_t slice_end, void* amps,
                 void* stream);

/*
 * Linear XEB, Eq. (1): F = (2^n / k) sum_i |amps[i]|^2 - 1 over all k strings
 * (duplicates with multiplicity), summed in FP64 with compensation on the
 * device in a fixed order.  amps (device) complex128 [k] (with open qubits
 * [k][2^w], of which each string's own entry, its open bits as o, counts).
 * Waits for the stream and writes *F (host).
 * Errors: XEB_EINVAL (k == 0 or NULL F), XEB_ESTATE (no workspace), XEB_EHIP.
 */
int xeb_fidelity(xeb_plan_t plan, const void* amps, void* stream, double* F);

/*
 * Linear XEB without a plan and without any allocation, for callers that
 * cannot allocate device memory: code running under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same reduction, order and
 * result as xeb_fidelity (bit for bit, for the same amps and k).
 *   amps (device, current device) complex128 [k]; 1 <= k <= XEB_NOALLOC_MAX_STRINGS.
 *   n_qubits: n of Eq. (1), 1 <= n <= 64.
 *   F (device) one double, written on `stream`; the call neither waits for the
 *     stream nor copies to the host.
 * The chunk partials live in an array the library keeps on each device for
 * the life of the process (1 MiB, XEB_NOALLOC_MAX_STRINGS / 4096 slots, taken
 * on the device's first call); the call allocates nothing and frees nothing.
 * Every call on one device shares that array: calls that overlap on a device
 * (concurrent streams or threads) race; serialize them.
 * Errors: XEB_EINVAL (k == 0, NULL pointer, n out of range), XEB_ELIMIT
 * (k above the limit), XEB_EHIP.
 */
#define XEB_NOALLOC_MAX_STRINGS (((int64_t)1) << 28)
int xeb_fidelity_noalloc(const void* amps, int64_t k, int32_t n_qubits, double* F, void* stream);

/* Plan-wide figures (cost measures of Appendix A/C with exact variant counts). */
int xeb_plan_stats(xeb_plan_t plan, xeb_stats_t* stats);

/* Per-node figures; node = n_leaves + i for internal node i. */
int xeb_plan_node_stats(xeb_plan_t plan, int32_t node, xeb_node_stats_t* stats);

/*
 * Kernel timing with HIP events, for measurement.
 * xeb_plan_set_profiling(plan, 1) clears earlier records and makes every later
 * xeb_contract record a HIP event pair on its stream around each contraction
 * launch (and around each slice accumulation); 0 stops recording.
 * xeb_plan_read_profile waits for the recorded events and sums, over the
 * launches of one kernel class (XEB_KERNEL_GENERIC, XEB_KERNEL_MFMA,
 * XEB_KERNEL_ACCUMULATE or XEB_KERNEL_SPLITK), the event-measured seconds and
 * the algorithmic work: complex MACs sum |t_T| 2^(q+r) and bytes
 * 8 (|L| + |R| + |T|) of the tables each contraction launch reads and writes
 * (Appendix A, measures C and RW).  A split-K node's MFMA launch carries that
 * work; its reduction (chunk sum and epilogue, one event pair) carries the
 * bytes of the partial tiles it reads plus the table it writes.
 */
#define XEB_KERNEL_ACCUMULATE 2
#define XEB_KERNEL_SPLITK 3
typedef struct {
  int64_t launches;
  double seconds;
  double cmacs;
  double bytes;
} xeb_kernel_profile_t;
int xeb_plan_set_profiling(xeb_plan_t plan, int32_t enable);
int xeb_plan_read_profile(xeb_plan_t plan, int32_t kernel, xeb_kernel_profile_t* out);
/* The same sums restricted to the launches of one internal node (any kernel). */
int xeb_plan_read_node_profile(xeb_plan_t plan, int32_t node, xeb_kernel_profile_t* out);

/*
 * Autotuning of the contraction kernels (tile shape, row operand, split K, or
 * the per-element kernel), per internal node.  xeb_plan_autotune times on the
 * bound workspace, on `stream` (hipStream_t as void*), every configuration
 * each node's contraction can run with at its real shape and key counts
 * (first string block): `reps` launches (1..1000) after one warm-up, between
 * two events.  It keeps the fastest per node; later blocks take the same
 * choice where they can run it.  The tables in the workspace are
 * overwritten (the next xeb_contract recomputes them); results do not
 * change beyond FP32 summation order.  A batch created before tuning keeps
 * the configuration it captured.  The report (may be NULL):
 *   default_seconds / tuned_seconds: sum over nodes of the measured launch
 *   time of the compile-time / chosen configuration times the node's
 *   evaluations in one call over all 2^s slices (a model of one full call's
 *   kernel time); tuning_seconds: wall time of the tuning.
 * Errors: XEB_EINVAL (reps), XEB_ESTATE (no workspace), XEB_EHIP.
 */
typedef struct {
  int32_t nodes_tuned;
  int32_t nodes_changed;
  int64_t candidates;
  double default_seconds;
  double tuned_seconds;
  double tuning_seconds;
} xeb_autotune_report_t;
int xeb_plan_autotune(xeb_plan_t plan, int32_t reps, void* stream, xeb_autotune_report_t* report);

/*
 * A node's kernel configuration (as reported by xeb_plan_node_stats), for
 * reading the autotuner's choices and applying them, or any valid
 * configuration, to a plan with the same tree.  kernel: XEB_KERNEL_GENERIC
 * with tile -2 (row-streaming form, swapped naming the streamed side as in
 * xeb_node_stats_t; XEB_EINVAL where the shape does not fit it) or any other
 * tile (one thread per output element; the remaining fields are ignored), or
 * XEB_KERNEL_MFMA with tile 0..7, swapped
 * 0/1 (right child as the row operand), ksplit a power of two with K / ksplit
 * >= k_slab, k_slab 16 / 32 (complex64) or 32 / 64 (split forms; 16 on tile
 * 5, which takes no complex64), k_groups 1 or 2 (2 and the larger slab only
 * on some tiles).  A node whose key set is
 * too sparse for the stacked product runs keyed (one GEMM per key): then
 * each key's block must cover whole tiles and ksplit must be 1.
 * xeb_plan_set_node_config applies it to every string block and fails with
 * XEB_EINVAL, changing nothing, if some block cannot run it (variant not
 * built, keyed node with keys smaller than the tile or split K, split-K
 * room exceeded).  A batch created earlier keeps its configuration.
 */
typedef struct {
  int32_t kernel;
  int32_t tile;
  int32_t swapped;
  int32_t ksplit;
  int32_t k_slab;
  int32_t k_groups;
  int32_t keyed;  /* MFMA: 1 = keyed form (one GEMM per key) also where the stacked
                     product applies; a node too sparse to stack is keyed anyway */
} xeb_node_config_t;
int xeb_plan_get_node_config(xeb_plan_t plan, int32_t node, xeb_node_config_t* out);
int xeb_plan_set_node_config(xeb_plan_t plan, int32_t node, const xeb_node_config_t* config);

/*
 * Batched form: several bound plans (different circuits, uneven sizes) as one
 * hipGraph.  xeb_batch_create captures, for every plan, the clearing of its
 * amplitude buffer, the contraction of all its 2^s slices (as xeb_contract
 * over [0, 2^s)) and its XEB reduction, each plan on its own forked capture
 * stream (the plans share nothing), and instantiates the graph.  Every
 * xeb_batch_contract replays the whole batch with one hipGraphLaunch on
 * `stream`; afterwards each amplitude buffer holds its complete amplitudes
 * (a launch overwrites, it does not accumulate).
 *   plans (host) [n]: bound plans on one device, each listed once, n >= 1.
 *   amps (host) [n]: device complex128 [k_i] buffers, caller-owned; their
 *     addresses are captured in the graph (so they are passed here, not to
 *     each replay), and they must stay valid while the batch lives.
 * abort_after_slices does not apply to batch replays.
 * xeb_batch_fidelities waits for `stream` and writes each plan's F (host
 * double [n]; NaN for a plan with k = 0).
 * The plans must not be used by other calls while a launch is in flight;
 * eager calls between launches are fine.
 * One batch graph holds at most XEB_BATCH_MAX_NODES nodes (kernel launches
 * plus the fork / join nodes; xeb_plan_stats' evals_full is the bulk of a
 * plan's share): a larger capture is discarded before it is instantiated
 * and the call fails with XEB_ELIMIT.  Larger workloads are split over
 * several batches (or run eagerly).
 * Errors: XEB_EINVAL, XEB_ESTATE (a plan without workspace), XEB_ELIMIT,
 * XEB_EHIP.
 */
#define XEB_BATCH_MAX_NODES 49152
typedef struct xeb_batch* xeb_batch_t;
int xeb_batch_create(const xeb_plan_t* plans, void* const* amps, int32_t n, xeb_batch_t* out);
int xeb_batch_contract(xeb_batch_t batch, void* stream);
int xeb_batch_fidelities(xeb_batch_t batch, void* stream, double* F);
int xeb_batch_destroy(xeb_batch_t batch);

/* Release the plan's host memory (the workspace stays the caller's). */
int xeb_plan_destroy(xeb_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* XEB_H */
