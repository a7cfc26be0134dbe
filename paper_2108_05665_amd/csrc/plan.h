// Plan: the compiled multi-tensor contraction (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace xeb {

// A node of the contraction tree (leaf or internal).
struct Node {
  bool leaf = true;
  int left = -1, right = -1, parent = -1;
  // Tensor legs (internal, unsliced), in layout order: position p of this list
  // is bit p of the element index inside one variant.
  std::vector<int32_t> legs;
  uint64_t outmask = 0;  // qubits whose output leg lies in this subtree
  uint64_t smask = 0;    // slice-id bits whose leg lies in this subtree
  int64_t nvar = 1;      // distinct string keys (|t_T| restricted to strings)
  // Leaf only: string keys (pext of the string on outmask) of each variant.
  std::vector<uint64_t> leaf_keys;
  int64_t nslicekeys = 1;  // leaf only: 2^popcount(smask)
  // Internal only.
  int mb = 0, nb = 0, kb = 0;
  std::vector<int32_t> lidx, ridx;  // child variants of each variant
  int kernel = XEB_KERNEL_GENERIC;
  int pair_mode = 0;                // MFMA: 0 dense, 1 table
  int swapped = 0;                  // MFMA: right child supplies the tile rows
  int tile = 0;                     // MFMA tile shape (see ContractArgs::tile)
  int8_t ubit[16] = {};             // MFMA epilogue write order
  std::vector<int32_t> pairs;       // MFMA table mode: nvarL * nvarR entries
  int8_t posM[kMaxBits] = {};
  int8_t posN[kMaxBits] = {};
  // Device placement (byte offsets inside the workspace).
  uint64_t off_table = 0, off_lidx = 0, off_ridx = 0, off_pairs = 0;
  // Resident state: the slice key (sigma & smask) whose table is on device.
  bool valid = false;
  uint64_t cur_key = 0;

  int64_t size() const { return int64_t(1) << legs.size(); }
};

struct ProfRecord {
  hipEvent_t start, stop;
  int kernel;
  double cmacs, bytes;
};

struct Plan {
  xeb_options_t opt{};
  int n_qubits = 0;
  int s = 0;
  std::vector<int32_t> sliced;
  int64_t k = 0, kd = 0;
  int n_leaves = 0;
  int root = 0;
  std::vector<Node> nodes;
  std::vector<int32_t> rho;         // root variant of every input string
  std::vector<float> leaf_staging;  // all leaf tables, complex64 interleaved
  uint64_t leaf_bytes = 0;
  uint64_t off_rho = 0, off_comp = 0, off_scratch = 0, ws_bytes = 0;
  void* ws = nullptr;
  uint64_t ws_size = 0;
  xeb_stats_t stats{};
  // Profiling (HIP events around launches).
  bool profiling = false;
  std::vector<ProfRecord> prof;      // records of the current profiling window
  std::vector<hipEvent_t> event_pool;
  ~Plan();
};

void compile_plan(Plan& p, const xeb_circuit_t* c, const uint64_t* bitstrings, int64_t k,
                  const xeb_tree_t* tree, const int32_t* sliced, int32_t s,
                  const xeb_options_t* opt);
void bind_plan(Plan* p, void* dev, uint64_t bytes);
void contract_plan(Plan* p, int64_t b, int64_t e, void* amps, hipStream_t stream);
double fidelity_plan(Plan* p, const void* amps, hipStream_t stream);

void hip_check(hipError_t e, const char* what);
void set_profiling(Plan* p, bool on);
xeb_kernel_profile_t read_profile(Plan* p, int kernel);

}  // namespace xeb

struct xeb_plan {
  xeb::Plan impl;
};
