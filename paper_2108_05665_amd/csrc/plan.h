// Plan: the compiled multi-tensor contraction (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace xeb {

// An internal node's keys among one block of strings, with the gather maps
// and the kernel chosen for them.
struct NodeBlock {
  int64_t nvar = 1;                 // distinct keys of the node in this block
  std::vector<int32_t> lidx, ridx;  // child keys of each key (generic kernel)
  int kernel = XEB_KERNEL_GENERIC;
  int pair_mode = 0;                // MFMA: 0 dense, 1 table, 2 keyed (one GEMM per key)
  int keyed = 0;                    // MFMA: keyed form requested where stacking applies
  int swapped = 0;                  // MFMA: right child supplies the tile rows
  int tile = 0;                     // MFMA tile shape (see ContractArgs::tile)
  int8_t ubit[16] = {};             // MFMA epilogue write order
  int ksplit = 1;                   // MFMA: K chunks (partial tiles + reduction)
  int tk = 16;                      // MFMA: K slab (complex per LDS stage)
  int kg = 1;                       // MFMA: K groups of four waves per workgroup
  std::vector<int32_t> pairs;       // MFMA table mode: nvarL * nvarR entries
  uint64_t off_lidx = 0, off_ridx = 0, off_pairs = 0;
};

// A contiguous range of the distinct keyed strings (string, low slice key) in
// lexicographic tuple order.
struct Block {
  int64_t first = 0, count = 0;
  std::vector<NodeBlock> nodes;  // indexed by internal node id - n_leaves
  // Slice accumulation: one entry group per caller position that has keyed
  // strings in this block: idx[g] is the position (in the caller's list),
  // entries eoff[g] .. eoff[g + 1] - 1 its keyed strings in increasing low
  // slice key slo, each with its root key rho.
  std::vector<int32_t> idx;
  std::vector<int32_t> eoff;
  std::vector<int32_t> rho;
  std::vector<int32_t> slo;
  uint64_t off_idx = 0, off_eoff = 0, off_rho = 0, off_slo = 0;
};

// A node of the contraction tree (leaf or internal).
struct Node {
  bool leaf = true;
  int left = -1, right = -1, parent = -1;
  // Tensor legs (internal, unsliced), in layout order: position p of this list
  // is bit p of the element index inside one key's tensor.
  std::vector<int32_t> legs;
  // Key bits whose leg lies in this subtree: qubit q (bit q < n) or stacked
  // slice-id bit j (bit n + j, j < sj).
  uint64_t outmask = 0;
  // Looped slice-id bits whose leg lies in this subtree: bit j is slice-id
  // bit sj + j.
  uint64_t smask = 0;
  // Leaf only: keys over all strings (pext of the string on outmask).
  int64_t leaf_nvar = 1;
  std::vector<uint64_t> leaf_keys;
  int64_t nslicekeys = 1;  // leaf only: 2^popcount(smask)
  float leaf_amax = 0.f;   // leaf only: largest |re|, |im| of its table
  // Internal only.
  int mb = 0, nb = 0, kb = 0;
  int8_t posM[kMaxBits] = {};
  int8_t posN[kMaxBits] = {};
  uint64_t maskM = 0, maskN = 0;  // the same positions as bit masks
  int64_t table_nvar = 1;  // largest key count over the blocks (table capacity)
  // Device placement (byte offset inside the workspace).
  uint64_t off_table = 0;
  // Resident state: block and slice key (sigma & smask) of the table on device.
  bool valid = false;
  uint64_t cur_key = 0;
  int cur_block = -1;
  uint32_t epoch = 0;  // evaluations within the current call (amax epochs)

  int64_t size() const { return int64_t(1) << legs.size(); }
};

struct ProfRecord {
  hipEvent_t start, stop;
  int kernel;
  int node;  // internal node id, -1 for the slice accumulation
  double cmacs, bytes;
};

struct Plan {
  xeb_options_t opt{};
  int n_qubits = 0;
  int s = 0;
  int sj = 0;  // stacked low slice bits (xeb_options_t::stack_slices)
  int w = 0;   // open output qubits (xeb_options_t::open_qubits): 2^w values per string
  uint64_t off_sel = 0;     // static: open bits of each string (int32 [k]), when w > 0
  uint64_t off_gather = 0;  // dynamic: each string's own amplitude (complex128 [k]), w > 0
  std::vector<int32_t> sliced;
  int64_t k = 0, kd = 0;
  int n_leaves = 0;
  int root = 0;
  std::vector<Node> nodes;
  std::vector<Block> blocks;
  std::vector<float> staging;  // static region: leaf tables, maps (uploaded at bind)
  uint64_t off_comp = 0, off_scratch = 0, ws_bytes = 0;
  uint64_t off_leaf_amax = 0;  // static: one slot (epoch 0 | float bits) per leaf
  uint64_t off_amax = 0;       // dynamic: kAmaxSlots (epoch << 32 | bits) slots per node
  uint64_t off_partial = 0;    // dynamic: split-K partial tiles
  uint64_t partial_bytes = 0;  // their capacity (largest need, or the tuning reserve)
  uint64_t off_planes = 0;     // dynamic: plane-format operands of a tile-6 launch
  uint64_t planes_bytes = 0;   // their capacity (0: no node can run tile 6)
  bool capturing = false;      // launches are being captured: no event timing
  void* ws = nullptr;
  uint64_t ws_size = 0;
  xeb_stats_t stats{};
  int64_t slices_done = 0;  // slices contracted by xeb_contract calls
  // Profiling (HIP events around launches).
  bool profiling = false;
  std::vector<ProfRecord> prof;  // records of the current profiling window
  std::vector<hipEvent_t> event_pool;
  ~Plan();
};

void compile_plan(Plan& p, const xeb_circuit_t* c, const uint64_t* bitstrings, int64_t k,
                  const xeb_tree_t* tree, const int32_t* sliced, int32_t s,
                  const xeb_options_t* opt);
void bind_plan(Plan* p, void* dev, uint64_t bytes);
void contract_plan(Plan* p, int64_t b, int64_t e, void* amps, hipStream_t stream);
double fidelity_plan(Plan* p, const void* amps, hipStream_t stream);
// Enqueues the XEB of the plan's amplitudes; F lands in the workspace scratch.
void launch_plan_xeb(Plan* p, const void* amps, hipStream_t stream);

void hip_check(hipError_t e, const char* what);

// Makes `dev` current for the scope and restores the previous device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

// Kernel configuration of one node in one block (compile-time choice or the
// autotuner's).
// Stacked MFMA form (all key pairs, or a pair table): the node's key set is
// dense enough.
bool mfma_capable(const Node& nd, int64_t nvarL, int64_t nvarR, const NodeBlock& nb);
// Keyed MFMA form (one GEMM per key): the stacked form does not apply and
// each key's 2^mb x 2^nb product spans at least half of each side of `tile`
// with the given row operand (at most 4x padding).
bool mfma_keyed_fits(const Node& nd, int tile, int swapped);
bool mfma_keyed(const Node& nd, int64_t nvarL, int64_t nvarR, const NodeBlock& nb);
// Bytes of both operands of a node in plane format (tile 6), either child
// first (the larger of the two orders).
uint64_t planes_need(const Node& nd, int64_t nvarL, int64_t nvarR);
// Whether the MFMA kernel can run the node in this configuration.
bool mfma_can_run(const Node& nd, int64_t nvarL, int64_t nvarR, const NodeBlock& nb, int tile,
                  int swapped, int ksplit, int keyed = 0);
void configure_mfma(const Node& nd, int64_t nvarL, int64_t nvarR, NodeBlock& nb, int tile, int swapped,
                    int ksplit, int tk, int kg = 1, int keyed = 0);
// The per-element kernel: form 0 one thread per output element, form 1 the
// row-streaming form (stream_l: stream L's rows rather than R's).
void configure_generic(NodeBlock& nb, int form, int stream_l);
// Whether the row-streaming form fits the node with that stream side.
bool generic_rows_ok(const Node& nd, int stream_l);
// The row-streaming form where it fits (the wider side streamed), else form 0.
void configure_generic_default(const Node& nd, NodeBlock& nb);
int64_t node_tiles(const Node& nd, int64_t nvarL, int64_t nvarR, int tile, int swapped);
// Key count of node `id` in block `blk` (a leaf's: all its keys).
int64_t nvar_in(const Plan* p, const Block& blk, int id);
// Arguments of internal node T's contraction for slice sigma in block blk.
ContractArgs node_args(Plan* p, const Block& blk, int T, int64_t sigma);
// Launches that contraction (both kernels of a split-K node) on `stream`.
void launch_node(const ContractArgs& a, const NodeBlock& nb, hipStream_t stream);
// Evaluations of a node over one call covering all 2^s slices.
double evals_per_call(const Plan* p, int T);

struct AutotuneReport {
  int nodes_tuned = 0, nodes_changed = 0;
  int64_t candidates = 0;
  double default_seconds = 0, tuned_seconds = 0, tuning_seconds = 0;
};
AutotuneReport autotune_plan(Plan* p, int reps, hipStream_t stream);
// A node's configuration in the first block / applied to all blocks (throws
// XEB_EINVAL, changing nothing, if a block cannot run it).
xeb_node_config_t get_node_config(const Plan* p, int T);
void set_node_config(Plan* p, int T, const xeb_node_config_t& c);

struct Batch;
Batch* create_batch(Plan* const* plans, void* const* amps, int n);
void launch_batch(Batch* b, hipStream_t stream);
void batch_fidelities(Batch* b, hipStream_t stream, double* F);
void destroy_batch(Batch* b);
void set_profiling(Plan* p, bool on);
xeb_kernel_profile_t read_profile(Plan* p, int kernel, int node);

}  // namespace xeb

struct xeb_plan {
  xeb::Plan impl;
};

struct xeb_batch {
  xeb::Batch* impl = nullptr;
};
