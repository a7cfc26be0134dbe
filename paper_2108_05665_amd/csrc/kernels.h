// Launch interfaces of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace xeb {

constexpr int kMaxBits = 48;  // max legs of one tensor (bits of its element index)

// A set of bit positions (`mask`) with the move masks of the compress /
// expand method of H. S. Warren, "Hacker's Delight", sections 7-4 and 7-5:
// mv[i] holds the mask bits that move right by 2^i in the i-th step of
// gathering the mask's bits to the bottom.  With them, PEXT and PDEP over the
// mask take six shift-and-mask steps without branches or table loads.
struct BitMap {
  uint64_t mask;
  uint64_t mv[6];
};

// One pairwise contraction T = L * R over all variants of T (Appendix A:
// 2^(q+r) complex MACs per variant).  Operand layouts: a variant of L is a
// row-major (2^mb x 2^kb) matrix (shared legs in the low bits), a variant of
// R a row-major (2^nb x 2^kb) matrix; element (m, n) of a variant of T lives
// at offset pdep(m, mapM) + pdep(n, mapN): the row index's bits go, lowest
// first, to the set bit positions of mapM.mask (the layout keeps each child's
// free legs in the parent's order, so this is a plain bit deposit), the
// column index's to those of mapN.mask; the two masks partition the mb + nb
// bits.
struct ContractArgs {
  const float2* A;       // L table (variants x 2^(mb+kb))
  const float2* B;       // R table (variants x 2^(nb+kb))
  float2* C;             // T table (variants x 2^(mb+nb))
  const int32_t* lidx;   // generic kernel: L variant of each T variant
  const int32_t* ridx;   // generic kernel: R variant of each T variant
  const int32_t* pairs;  // MFMA kernel, table mode: T variant of (l, r) or -1
  int64_t nvar;          // T variants
  int64_t nvarA, nvarB;  // L and R variants
  int32_t mb, nb, kb;
  int32_t pair_mode;     // 0: dense (a = l * nvarB + r), 1: table, 2: keyed (lidx / ridx)
  int32_t swapped;       // MFMA: rows are R's variants (A <- R, B <- L)
  int32_t tile;          // MFMA tile: 0 = 64 x 64, 1 = 32 x 128, 2 = 16 x 256, 3 = 64 x 16, 4 = 128 x 128,
                         // 5 = 128 x 128 on eight waves (split forms),
                         // 6 = 128 x 128 on plane-format operands (split forms),
                         // 7 = 256 x 128 on plane-format operands (split forms)
  int32_t tk;            // MFMA K slab (complex per LDS stage), see mfma_variant_allowed
  int32_t kg;            // MFMA K groups of four waves per workgroup (1 or 2)
  BitMap mapM;            // output bit positions of the row index's bits
  BitMap mapN;            // output bit positions of the column index's bits
  // MFMA epilogue write order: bit b of an element's number inside the tile is
  // row bit ubit[b] (< 32) or column bit ubit[b] - 32.
  int8_t ubit[16];
  int32_t prec;          // MFMA operand precision: XEB_PREC_C64 / _SPLIT_FP16 / _SPLIT_BF16
  // Largest |re|, |im| of the operand tables, read for the FP16 scale.  A
  // table's value is kept in slots of (epoch << 32) | float bits, kAmaxStride
  // words apart: amaxA / amaxB point at amax_nA / amax_nB such slots, whose
  // largest word is the latest evaluation's (largest epoch) maximum.  The
  // output's is published by atomicMax into slot (workgroup % kAmaxSlots) of
  // amax_out (workgroup 0 always publishes), so slots never need clearing
  // between evaluations.  NULL amax_out: not tracked.
  const unsigned long long* amaxA;
  const unsigned long long* amaxB;
  int32_t amax_nA, amax_nB;
  unsigned long long* amax_out;
  uint32_t epoch;
  // Split K (MFMA): ksplit > 1 cuts K into ksplit equal chunks; the chunk
  // products go to `partial` ([chunk][tile][BM * BN] complex64, row-major
  // inside a tile) and a second kernel sums them in chunk order and writes T.
  int32_t ksplit;
  float2* partial;
  // Tile 6: room for both operands in hi/lo plane format (k_presplit), each
  // (rows x 2^kb complex) x 8 bytes.
  uint16_t* Ap;
  uint16_t* Bp;
};

constexpr int kAmaxSlots = 16;   // atomic slots per table
constexpr int kAmaxStride = 16;  // words between slots (one 128-byte line each)

// Profiling: HIP events attached to the dispatch packets of the next launch
// group on this thread (hipExtLaunchKernel), so that they time the kernels
// alone.  The group's first kernel records `start` as it begins, its last
// kernel `stop` as it ends; each event is cleared once used, and
// take_launch_events returns the ones no kernel used (the caller records
// those itself).
void set_launch_events(hipEvent_t start, hipEvent_t stop);
void take_launch_events(hipEvent_t* start, hipEvent_t* stop);

// The per-element contraction.  a.tile 0: one output element per thread (any
// shape); a.tile 1: the row-streaming form (a.swapped 0 streams R's rows, 1
// streams L's), for the shapes generic_rows_fit accepts.
void launch_contract_generic(const ContractArgs& a, hipStream_t s);
// Stream rows per thread in the row-streaming form (log2), where the stream
// side has at least 8 + kRowsLog2U bits and that leaves at least
// kRowsMinItems work items (one row per thread otherwise).
constexpr int kRowsLog2U = 2;
constexpr int64_t kRowsMinItems = 2048;
// The row-streaming form runs K = 2^kb <= 16, a stream side of at least 8
// bits (256 rows per work item) and at most 64 broadcast rows.
inline bool generic_rows_fit(int kb, int stream_bits, int bcast_bits) {
  return kb >= 0 && kb <= 4 && stream_bits >= 8 && bcast_bits >= 0 && bcast_bits <= 6;
}
// The MFMA contraction; with a.ksplit > 1 it writes the chunk partials only
// and launch_splitk_reduce (same arguments, same stream, right after) sums
// them and writes T.
void launch_contract_mfma(const ContractArgs& a, hipStream_t s);
void launch_splitk_reduce(const ContractArgs& a, hipStream_t s);
constexpr int kMfmaTiles = 8;  // tile shapes 0..7 (see mfma_tile_shape)
void mfma_tile_shape(int tile, int* bm, int* bn);
// MFMA variants that are built: K slab complex64 16 (all tiles) or 32
// (64 x 64, 32 x 128), split forms 32 (all tiles) or 64 (64 x 64); two K
// groups (kg = 2, 512 threads) on the 64 x 64 tile only.  Tile 4 is 128 x 128;
// tile 5 is 128 x 128 with eight waves and double-buffered LDS, split forms
// only, K slab 16; tile 6 is 128 x 128 on operands converted once into hi/lo
// planes (split forms, K slab 16, K >= 16, no split K); tile 7 the same at
// 256 x 128 with eight waves.
bool mfma_variant_allowed(int tile, int prec, int tk, int kg);
int mfma_default_slab(int prec);
// Tiles of an MFMA contraction with rowsA x rowsB outputs on tile shape `tile`.
int64_t mfma_tiles(int tile, int64_t rowsA, int64_t rowsB);
// Queries (once per device) the occupancy the persistent grids use, so that a
// later stream capture makes no occupancy call.
void prepare_mfma_launch(int prec);

// Cross-slice accumulation (Appendix A, "Slicing": sum over assignments) in
// FP64 with Neumaier compensation.  Every root key holds W = 2^w values (w
// open qubits, else W = 1).  Group g < n adds, into amps[idx[g] W + o] for
// o < W, the root partials partial[rho[j] W + o] of its entries
// j = eoff[g] .. eoff[g + 1] - 1 in entry order (increasing low slice key),
// each only if its slice base + slo[j] lies in [lo, hi).
void launch_zero(void* p, uint64_t bytes, hipStream_t s);
void launch_accumulate(const float2* partial, const int32_t* idx, const int32_t* eoff,
                       const int32_t* rho, const int32_t* slo, int64_t base, int64_t lo,
                       int64_t hi, double2* amps, double2* comp, int64_t n, int w, hipStream_t s);
// own[i] = amps[i 2^w + sel[i]], i < k (each string's own amplitude).
void launch_gather_own(const double2* amps, const int32_t* sel, int w, double2* own, int64_t k,
                       hipStream_t s);
void launch_fold_compensation(double2* amps, const double2* comp, int64_t k, hipStream_t s);

// Linear XEB (Eq. 1): F = 2^n / k * sum |amps|^2 - 1, a compensated FP64
// reduction in a fixed order over chunks of kXebChunk strings (two kernels).
// `scratch` (device, 16-byte aligned, xeb_scratch_bytes(k) bytes) receives F
// in its first double; the rest holds the chunks' partial sums.
constexpr int64_t kXebChunk = 4096;
uint64_t xeb_scratch_bytes(int64_t k);
void launch_xeb(const double2* amps, int64_t k, int n_qubits, void* scratch, hipStream_t s);
// The same reduction with its chunk partials in a per-device array that the
// library holds for the life of the process (no allocation, no workspace):
// at most kXebStaticGroups chunks, i.e. kXebStaticMaxStrings strings; F goes
// to F_dev (device).  Runs on the current device.  Calls that overlap on one
// device share the array and race.
constexpr int64_t kXebStaticGroups = int64_t(1) << 16;  // 1 MiB of partial pairs
constexpr int64_t kXebStaticMaxStrings = kXebStaticGroups * kXebChunk;
constexpr int kMaxDevices = 64;
void launch_xeb_static(const double2* amps, int64_t k, int n_qubits, double* F_dev, hipStream_t s);

}  // namespace xeb
