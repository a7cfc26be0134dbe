"""ctypes binding of libxeb.so (the C ABI in include/xeb.h).

Argument marshalling only: every step of the contraction runs in the
library's gfx950 kernels.  PyTorch supplies device memory (the plan's
workspace and the amplitude buffer) and streams.  If libxeb.so is missing
this module raises at import: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxeb.so")

XEB_OK = 0
XEB_EINVAL = -1
XEB_ENOMEM = -2
XEB_EHIP = -3
XEB_ESTATE = -4
XEB_ELIMIT = -5
XEB_EABORT = -6
BATCH_MAX_NODES = 49152  # nodes of one batch graph (XEB_BATCH_MAX_NODES)

PRECISIONS = {"c64": 0, "split_fp16": 1, "split_bf16": 2}
KERNELS = {0: "generic", 1: "mfma"}

# torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it first
# makes libxeb's libamdhip64.so.7 dependency resolve to that same copy; a second
# runtime in the process would not see the GPU.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "(hipcc --offload-arch=gfx950); there is no CPU fallback"
    )
_lib = ctypes.CDLL(LIB_PATH)


class XebError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"xeb error {code}: {msg}")
        self.code = code


class Circuit(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int32),
        ("n_gates", ctypes.c_int32),
        ("gate_qubits", ctypes.POINTER(ctypes.c_int32)),
        ("gate_mats", ctypes.POINTER(ctypes.c_double)),
    ]


class Tree(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int32), ("children", ctypes.POINTER(ctypes.c_int32))]


class Options(ctypes.Structure):
    _fields_ = [
        ("fuse_1q", ctypes.c_int32),
        ("fold_kets", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("memory_budget", ctypes.c_uint64),
        ("trace", ctypes.c_int32),
        ("force_generic", ctypes.c_int32),
        ("max_ksplit", ctypes.c_int32),
        ("mfma_min_cmacs", ctypes.c_double),
        ("stack_slices", ctypes.c_int32),
        ("open_qubits", ctypes.c_uint64),
        ("abort_after_slices", ctypes.c_int64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_leaves", ctypes.c_int64),
        ("n_internal", ctypes.c_int64),
        ("k", ctypes.c_int64),
        ("k_distinct", ctypes.c_int64),
        ("n_qubits", ctypes.c_int32),
        ("n_sliced", ctypes.c_int32),
        ("sum_variants", ctypes.c_int64),
        ("max_tensor_elems", ctypes.c_int64),
        ("cmacs_per_slice", ctypes.c_double),
        ("cmacs_full", ctypes.c_double),
        ("rw_elems_full", ctypes.c_double),
        ("evals_full", ctypes.c_double),
        ("workspace_bytes", ctypes.c_uint64),
        ("n_blocks", ctypes.c_int64),
        ("n_stacked", ctypes.c_int32),
        ("n_open", ctypes.c_int32),
        ("slices_done", ctypes.c_int64),
    ]


class NodeStats(ctypes.Structure):
    _fields_ = [
        ("left", ctypes.c_int32),
        ("right", ctypes.c_int32),
        ("variants", ctypes.c_int64),
        ("left_variants", ctypes.c_int64),
        ("right_variants", ctypes.c_int64),
        ("m_bits", ctypes.c_int32),
        ("n_bits", ctypes.c_int32),
        ("k_bits", ctypes.c_int32),
        ("slice_mask", ctypes.c_uint64),
        ("kernel", ctypes.c_int32),
        ("swapped", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("ksplit", ctypes.c_int32),
        ("k_slab", ctypes.c_int32),
        ("k_groups", ctypes.c_int32),
        ("pair_mode", ctypes.c_int32),
        ("cmacs_per_eval", ctypes.c_double),
    ]


class KernelProfile(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int64),
        ("seconds", ctypes.c_double),
        ("cmacs", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


KERNEL_IDS = {"generic": 0, "mfma": 1, "accumulate": 2, "splitk": 3}

class NodeConfig(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("swapped", ctypes.c_int32),
        ("ksplit", ctypes.c_int32),
        ("k_slab", ctypes.c_int32),
        ("k_groups", ctypes.c_int32),
        ("keyed", ctypes.c_int32),
    ]


class AutotuneReport(ctypes.Structure):
    _fields_ = [
        ("nodes_tuned", ctypes.c_int32),
        ("nodes_changed", ctypes.c_int32),
        ("candidates", ctypes.c_int64),
        ("default_seconds", ctypes.c_double),
        ("tuned_seconds", ctypes.c_double),
        ("tuning_seconds", ctypes.c_double),
    ]


_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_SIG = {
    "xeb_options_default": (None, [ctypes.POINTER(Options)]),
    "xeb_last_error": (ctypes.c_char_p, []),
    "xeb_network_describe": (ctypes.c_int, [ctypes.POINTER(Circuit), ctypes.c_int32, ctypes.c_int32,
                                            _I32P, _I32P, _I32P, _I32P, _I32P, _I32P]),
    "xeb_plan_create": (ctypes.c_int, [ctypes.POINTER(Circuit), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.c_int64, ctypes.POINTER(Tree), _I32P, ctypes.c_int32,
                                       ctypes.POINTER(Options), ctypes.POINTER(_P)]),
    "xeb_plan_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64)]),
    "xeb_plan_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "xeb_contract": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "xeb_fidelity": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "xeb_fidelity_noalloc": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, _P, _P]),
    "xeb_plan_autotune": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.POINTER(AutotuneReport)]),
    "xeb_plan_get_node_config": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(NodeConfig)]),
    "xeb_plan_set_node_config": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(NodeConfig)]),
    "xeb_plan_stats": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "xeb_plan_node_stats": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(NodeStats)]),
    "xeb_plan_set_profiling": (ctypes.c_int, [_P, ctypes.c_int32]),
    "xeb_plan_read_profile": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(KernelProfile)]),
    "xeb_plan_read_node_profile": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(KernelProfile)]),
    "xeb_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int32,
                                        ctypes.POINTER(_P)]),
    "xeb_batch_contract": (ctypes.c_int, [_P, _P]),
    "xeb_batch_fidelities": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "xeb_batch_destroy": (ctypes.c_int, [_P]),
    "xeb_plan_destroy": (ctypes.c_int, [_P]),
}
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIG)


def _check(rc: int) -> None:
    if rc != XEB_OK:
        raise XebError(rc, _lib.xeb_last_error().decode())


def _circuit_struct(circ):
    gq = np.ascontiguousarray(circ.gate_qubits, dtype=np.int32).reshape(-1, 2)
    gm = np.ascontiguousarray(circ.gate_mats_f64(), dtype=np.float64)
    c = Circuit(int(circ.n_qubits), int(gq.shape[0]),
                gq.ctypes.data_as(_I32P), gm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return c, (gq, gm)  # keep the arrays alive with the struct


def default_options() -> Options:
    o = Options()
    _lib.xeb_options_default(ctypes.byref(o))
    return o


def network_describe(circ, fuse_1q: bool = True, fold_kets: bool = True):
    """Leaves (list of leg-id lists), number of legs, leg -> output qubit (-1)."""
    c, keep = _circuit_struct(circ)
    nl, ng, nt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.xeb_network_describe(ctypes.byref(c), int(fuse_1q), int(fold_kets),
                                     ctypes.byref(nl), ctypes.byref(ng), ctypes.byref(nt),
                                     None, None, None))
    offs = np.zeros(nl.value + 1, dtype=np.int32)
    legs = np.zeros(max(nt.value, 1), dtype=np.int32)
    lq = np.zeros(max(ng.value, 1), dtype=np.int32)
    _check(_lib.xeb_network_describe(ctypes.byref(c), int(fuse_1q), int(fold_kets),
                                     ctypes.byref(nl), ctypes.byref(ng), ctypes.byref(nt),
                                     offs.ctypes.data_as(_I32P), legs.ctypes.data_as(_I32P),
                                     lq.ctypes.data_as(_I32P)))
    leaves = [legs[offs[j]:offs[j + 1]].tolist() for j in range(nl.value)]
    return leaves, ng.value, lq[: ng.value].tolist()


NOALLOC_MAX_STRINGS = 1 << 28


def fidelity_noalloc(amps, n_qubits: int, out, stream=None):
    """xeb_fidelity_noalloc: linear XEB of a device complex128 tensor `amps`
    into the one-element device float64 tensor `out`, enqueued on `stream`
    (torch's current stream by default); returns `out` without waiting."""
    import torch

    if amps.dtype != torch.complex128 or not amps.is_cuda or not amps.is_contiguous():
        raise ValueError("amps must be a contiguous complex128 CUDA tensor")
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < 1:
        raise ValueError("out must be a float64 CUDA tensor with one element")
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(_lib.xeb_fidelity_noalloc(ctypes.c_void_p(amps.data_ptr()), amps.numel(), int(n_qubits),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
    return out


class Plan:
    """A compiled multi-tensor contraction (xeb_plan_create) bound to a
    torch-allocated device workspace."""

    def __init__(self, circ, bitstrings, tree_children, sliced_legs=(), *, fuse_1q=True,
                 fold_kets=True, precision="c64", device=None, memory_budget=0, trace=0,
                 force_generic=False, max_ksplit=0, mfma_min_cmacs=0.0, stack_slices=0,
                 open_qubits=0, abort_after_slices=0, bind=True):
        self._h = _P()
        c, keep = _circuit_struct(circ)
        bs = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint64))
        ch = np.ascontiguousarray(np.asarray(tree_children, dtype=np.int32).reshape(-1))
        n_leaves = ch.size // 2 + 1
        tree = Tree(n_leaves, ch.ctypes.data_as(_I32P) if ch.size else None)
        sl = np.ascontiguousarray(np.asarray(list(sliced_legs), dtype=np.int32))
        o = default_options()
        o.fuse_1q = int(fuse_1q)
        o.fold_kets = int(fold_kets)
        o.precision = PRECISIONS[precision]
        self._device_index = 0 if device is None else int(device)
        o.device = self._device_index
        o.memory_budget = int(memory_budget)
        o.trace = int(trace)
        o.force_generic = int(force_generic)
        o.max_ksplit = int(max_ksplit)
        o.mfma_min_cmacs = float(mfma_min_cmacs)
        o.stack_slices = int(stack_slices)
        o.open_qubits = int(open_qubits)
        o.abort_after_slices = int(abort_after_slices)
        _check(_lib.xeb_plan_create(ctypes.byref(c), bs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                    bs.size, ctypes.byref(tree),
                                    sl.ctypes.data_as(_I32P) if sl.size else None, sl.size,
                                    ctypes.byref(o), ctypes.byref(self._h)))
        self.k = int(bs.size)
        self.n_open = bin(int(open_qubits)).count("1")
        self.n_qubits = int(circ.n_qubits)
        self.n_slices = 1 << int(sl.size)
        self.workspace = None
        if bind:
            self.bind()

    # -- device memory ------------------------------------------------------
    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(_lib.xeb_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def bind(self, workspace=None):
        import torch

        nbytes = self.workspace_bytes()
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                    device=torch.device("cuda", self._device_index))
        ptr = workspace.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        avail = workspace.numel() - (aligned - ptr)
        _check(_lib.xeb_plan_bind_workspace(self._h, ctypes.c_void_p(aligned), avail))
        self.workspace = workspace
        return workspace

    def new_amps(self):
        import torch

        shape = (self.k,) if self.n_open == 0 else (self.k, 1 << self.n_open)
        return torch.zeros(shape, dtype=torch.complex128,
                           device=torch.device("cuda", self._device_index))

    @staticmethod
    def _stream_handle(stream):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream()
        return ctypes.c_void_p(stream.cuda_stream)

    # -- the hot path ---------------------------------------------------------
    def contract(self, amps, slice_begin: int = 0, slice_end: int | None = None, stream=None):
        if slice_end is None:
            slice_end = self.n_slices
        import torch

        if amps.dtype != torch.complex128 or not amps.is_cuda or amps.numel() < (self.k << self.n_open):
            raise ValueError("amps must be a CUDA complex128 tensor with k * 2^w elements")
        if not amps.is_contiguous():
            raise ValueError("amps must be contiguous")
        _check(_lib.xeb_contract(self._h, int(slice_begin), int(slice_end),
                                 ctypes.c_void_p(amps.data_ptr()), self._stream_handle(stream)))
        return amps

    def fidelity(self, amps, stream=None) -> float:
        f = ctypes.c_double()
        _check(_lib.xeb_fidelity(self._h, ctypes.c_void_p(amps.data_ptr()),
                                 self._stream_handle(stream), ctypes.byref(f)))
        return float(f.value)

    # -- introspection ---------------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        _check(_lib.xeb_plan_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def node_stats(self, node: int) -> dict:
        s = NodeStats()
        _check(_lib.xeb_plan_node_stats(self._h, int(node), ctypes.byref(s)))
        d = {name: getattr(s, name) for name, _ in NodeStats._fields_}
        d["kernel"] = KERNELS.get(d["kernel"], d["kernel"])
        return d

    def all_node_stats(self) -> list:
        st = self.stats()
        L = int(st["n_leaves"])
        return [dict(node=L + i, **self.node_stats(L + i)) for i in range(int(st["n_internal"]))]

    # -- measurement -------------------------------------------------------------
    def set_profiling(self, enable: bool) -> None:
        _check(_lib.xeb_plan_set_profiling(self._h, int(bool(enable))))

    def autotune(self, reps: int = 3, stream=None) -> dict:
        """xeb_plan_autotune: per-node kernel configuration by measurement."""
        r = AutotuneReport()
        _check(_lib.xeb_plan_autotune(self._h, int(reps), self._stream_handle(stream), ctypes.byref(r)))
        return {name: getattr(r, name) for name, _ in AutotuneReport._fields_}

    def node_config(self, node: int) -> dict:
        c = NodeConfig()
        _check(_lib.xeb_plan_get_node_config(self._h, int(node), ctypes.byref(c)))
        d = {name: getattr(c, name) for name, _ in NodeConfig._fields_}
        d["kernel"] = KERNELS.get(d["kernel"], d["kernel"])
        return d

    def set_node_config(self, node: int, kernel: str = "mfma", tile: int = 0, swapped: int = 0,
                        ksplit: int = 1, k_slab: int = 16, k_groups: int = 1, keyed: int = 0) -> None:
        c = NodeConfig(KERNEL_IDS[kernel], tile, swapped, ksplit, k_slab, k_groups, keyed)
        _check(_lib.xeb_plan_set_node_config(self._h, int(node), ctypes.byref(c)))

    def read_profile(self, kernel: str) -> dict:
        pr = KernelProfile()
        _check(_lib.xeb_plan_read_profile(self._h, KERNEL_IDS[kernel], ctypes.byref(pr)))
        return {name: getattr(pr, name) for name, _ in KernelProfile._fields_}

    def read_node_profile(self, node: int) -> dict:
        pr = KernelProfile()
        _check(_lib.xeb_plan_read_node_profile(self._h, int(node), ctypes.byref(pr)))
        return {name: getattr(pr, name) for name, _ in KernelProfile._fields_}

    def close(self):
        if self._h:
            _lib.xeb_plan_destroy(self._h)
            self._h = _P()
        self.workspace = None  # the device memory goes back to torch's allocator

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several bound plans replayed as one hipGraph (xeb_batch_*): every launch
    recomputes all amplitudes of all plans into `amps[i]` and their XEB.  One
    graph holds at most BATCH_MAX_NODES nodes (XebError XEB_ELIMIT beyond;
    BatchSet splits larger workloads)."""

    def __init__(self, plans, amps=None):
        self.plans = list(plans)
        self.amps = list(amps) if amps is not None else [p.new_amps() for p in self.plans]
        ph = (_P * len(self.plans))(*[p._h for p in self.plans])
        ah = (_P * len(self.plans))(*[a.data_ptr() for a in self.amps])
        self._h = _P()
        _check(_lib.xeb_batch_create(ph, ah, len(self.plans), ctypes.byref(self._h)))

    def launch(self, stream=None):
        _check(_lib.xeb_batch_contract(self._h, Plan._stream_handle(stream)))

    def fidelities(self, stream=None):
        out = (ctypes.c_double * len(self.plans))()
        _check(_lib.xeb_batch_fidelities(self._h, Plan._stream_handle(stream), out))
        return [float(x) for x in out]

    def close(self):
        if self._h:
            _lib.xeb_batch_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSet:
    """Plans of any total size: grouped into Batch graphs of at most
    BATCH_MAX_NODES nodes each (greedy in list order, by the plans' launch
    counts), and every plan too large for a graph of its own run eagerly
    (zero, contract, XEB) after the graphs, all on one stream.  launch() and
    fidelities() behave as Batch's."""

    def __init__(self, plans, amps=None, max_nodes: int = BATCH_MAX_NODES):
        self.plans = list(plans)
        self.amps = list(amps) if amps is not None else [p.new_amps() for p in self.plans]
        self.batches = []  # (Batch, indices into plans)
        self.eager = []    # indices run eagerly
        groups = self.group([self._estimate(p) for p in self.plans], max_nodes)
        try:
            while groups:
                g = groups.pop(0)
                try:
                    self.batches.append(
                        (Batch([self.plans[i] for i in g], [self.amps[i] for i in g]), g))
                except XebError as err:
                    if err.code != XEB_ELIMIT:
                        raise
                    if len(g) == 1:
                        self.eager.append(g[0])
                    else:
                        groups[:0] = [g[:len(g) // 2], g[len(g) // 2:]]
        except Exception:
            self.close()
            raise
        self.eager.sort()

    @staticmethod
    def group(estimates, max_nodes: int = BATCH_MAX_NODES):
        """Consecutive plan indices grouped greedily so that each group's
        estimated launches stay within 90 % of max_nodes (a plan above that
        alone forms a group of its own)."""
        groups, cur, tot = [], [], 0
        for i, e in enumerate(estimates):
            if cur and tot + e > 0.9 * max_nodes:
                groups.append(cur)
                cur, tot = [], 0
            cur.append(i)
            tot += e
        if cur:
            groups.append(cur)
        return groups

    @staticmethod
    def _estimate(p) -> int:
        """Kernel launches of one full contraction (node evaluations, one
        slice sum per slice and block, two split-K reductions per split
        evaluation counted as two more launches per node evaluation)."""
        st = p.stats()
        extra = sum(1 for ns in p.all_node_stats() if ns["ksplit"] > 1)
        per_slice = (1 << st["n_sliced"]) * st["n_blocks"]
        return int(st["evals_full"]) + per_slice * (1 + 2 * extra) + 8

    def launch(self, stream=None):
        for b, _ in self.batches:
            b.launch(stream)
        if self.eager:
            import torch

            with torch.cuda.stream(stream) if stream is not None else _nullcontext():
                for i in self.eager:
                    self.amps[i].zero_()
                    self.plans[i].contract(self.amps[i], stream=stream)

    def fidelities(self, stream=None):
        F = [float("nan")] * len(self.plans)
        for b, g in self.batches:
            for i, f in zip(g, b.fidelities(stream)):
                F[i] = f
        for i in self.eager:
            F[i] = self.plans[i].fidelity(self.amps[i], stream=stream)
        return F

    def close(self):
        for b, _ in self.batches:
            b.close()
        self.batches = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _nullcontext:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False
