// Plan compiler and executor of the multi-tensor contraction.
//
// Compilation (host, once per plan):
//  * network of the circuit; output legs and sliced legs are projected into
//    the leaves that carry them, which become variables whose values are the
//    projected tensors (section "Multi-batch simulator"; Appendix A, "Slicing");
//  * the distinct strings are sorted in the lexicographic order of their
//    tuples, variables ordered as they occur in the tree (Appendix C), and cut
//    into contiguous blocks; within a block every node gets its distinct keys
//    in lexicographic order of (left key, right key) and gather maps to its
//    children's keys.  |keys| is the exact evaluation count |t_T|;
//  * a top-down pass fixes every tensor's leg order so that the legs a node
//    shares with its sibling are the low (contiguous) bits and each parent's
//    kernel writes its result directly in the order its own parent reads;
//  * a dry run sizes the device workspace (Appendix C, "emulation mode") and
//    picks the smallest number of string blocks whose tables fit the budget.
//
// Execution (xeb_contract): block by block, slices in increasing order; within
// a block a node is contracted again only when the slice bits it depends on
// change (its table of all the block's keys stays resident otherwise), the
// single cached entry per subtree of the paper's K_L cache applied to slice
// variables; a node that sees no output leg keeps its table across blocks.
// The root's partial amplitudes are added into FP64 with compensation.

#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace xeb {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(XEB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
// Index arrays (gather maps, string maps) only need 16-byte alignment.
uint64_t align16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

// Move masks of the compress / expand method (H. S. Warren, "Hacker's
// Delight", 7-4): step i moves the marked bits right by 2^i; mk marks the
// positions whose count of zero mask bits below them (a parallel suffix over
// ~mask) has bit i set.
BitMap bit_map(uint64_t mask) {
  BitMap b{};
  b.mask = mask;
  uint64_t m = mask;
  uint64_t mk = ~m << 1;
  for (int i = 0; i < 6; ++i) {
    uint64_t mp = mk ^ (mk << 1);
    for (int sh = 2; sh < 64; sh <<= 1) mp ^= mp << sh;
    const uint64_t mv = mp & m;
    b.mv[i] = mv;
    m = (m ^ mv) | (mv >> (1 << i));
    mk &= ~mp;
  }
  return b;
}

int rank_in_mask(uint64_t mask, int bit) { return popcount64(mask & ((uint64_t(1) << bit) - 1)); }

std::vector<int32_t> sorted_copy(const std::vector<int32_t>& v) {
  std::vector<int32_t> r(v);
  std::sort(r.begin(), r.end());
  return r;
}

// Times node T is evaluated when slices 0..2^s-1 run in increasing order: its
// key sigma & smask changes exactly at multiples of 2^(lowest set bit).
double evals_over_all_slices(uint64_t smask, int s) {
  if (smask == 0) return 1.0;
  return std::ldexp(1.0, s - __builtin_ctzll(smask));
}

void leaves_dfs(const std::vector<Node>& nodes, int t, std::vector<int>& out) {
  if (nodes[t].leaf) {
    out.push_back(t);
    return;
  }
  leaves_dfs(nodes, nodes[t].left, out);
  leaves_dfs(nodes, nodes[t].right, out);
}

// Kernel choice for one node's keys in one block.  MFMA when the stacked GEMM
// is big enough and its padded tile work stays within 8x the useful MACs; the
// smaller side supplies the tile rows.
// Split K when the tiles alone are far too few for the chip (fewer than 64):
// double the chunk count until about one work item per CU exists, keeping at
// least four K slabs (64 complex) per chunk.  With more tiles the extra
// partial traffic and launches cost more than the added parallelism gains.
constexpr int64_t kSplitBelowTiles = 64, kSplitItems = 256, kMinChunk = 64;
// Largest plane-format operand room (tile 6) a plan reserves.
constexpr uint64_t kMaxPlaneBytes = uint64_t(16) << 30;
// Split-K partial room reserved for the autotuner's candidates.
constexpr uint64_t kTunePartialBytes = uint64_t(32) << 20;

// Default of xeb_options_t::mfma_min_cmacs: below about 2^23 complex MACs an
// MFMA launch (persistent grid, LDS staging, ordered epilogue) costs more
// than the per-element kernel on gfx950.
constexpr double kMfmaMinCmacs = 8388608.0;

}  // namespace

bool mfma_capable(const Node& nd, int64_t nvarL, int64_t nvarR, const NodeBlock& nb) {
  // (K >= 2: operand rows are read as float4; K <= 2^21: in-tile byte
  // offsets of up to 256 rows stay below 2^32.)
  if (nd.kb < 1 || nd.kb > 21) return false;
  const double pairs = double(nvarL) * double(nvarR);
  // A sparse pair set pays for padding in the GEMM and for its table: only a
  // set with at least one key in 8 pairs can run well on MFMA.
  return pairs <= double(1 << 26) && (nb.nvar == nvarL * nvarR || pairs <= 8.0 * double(nb.nvar));
}

bool mfma_keyed_fits(const Node& nd, int tile, int swapped) {
  int bm = 0, bn = 0;
  mfma_tile_shape(tile, &bm, &bn);
  const int rb = swapped ? nd.nb : nd.mb, cb = swapped ? nd.mb : nd.nb;
  return (int64_t(2) << rb) >= bm && (int64_t(2) << cb) >= bn;
}

bool mfma_keyed(const Node& nd, int64_t nvarL, int64_t nvarR, const NodeBlock& nb) {
  if (nd.kb < 1 || nd.kb > 21 || mfma_capable(nd, nvarL, nvarR, nb)) return false;
  for (int tile = 0; tile < kMfmaTiles; ++tile)
    for (int sw = 0; sw < 2; ++sw)
      if (mfma_keyed_fits(nd, tile, sw)) return true;
  return false;
}

uint64_t planes_need(const Node& nd, int64_t nvarL, int64_t nvarR) {
  const uint64_t a = ((uint64_t(nvarL) << nd.mb) * (uint64_t(8) << nd.kb) + 255) & ~uint64_t(255);
  return a + (uint64_t(nvarR) << nd.nb) * (uint64_t(8) << nd.kb) + 256;
}

bool mfma_can_run(const Node& nd, int64_t nvarL, int64_t nvarR, const NodeBlock& nb, int tile,
                  int swapped, int ksplit, int keyed) {
  if ((tile == 6 || tile == 7) && (nd.kb < 4 || nd.kb > 18 || ksplit != 1)) return false;
  const bool stacked = mfma_capable(nd, nvarL, nvarR, nb);
  if (stacked && !keyed) return true;
  return ksplit == 1 && nd.kb >= 1 && nd.kb <= 21 && mfma_keyed_fits(nd, tile, swapped) &&
         (stacked || mfma_keyed(nd, nvarL, nvarR, nb));
}

void configure_mfma(const Node& nd, int64_t nvarL, int64_t nvarR, NodeBlock& nb, int tile, int swapped,
                    int ksplit, int tk, int kg, int want_keyed) {
  nb.kernel = XEB_KERNEL_MFMA;
  nb.tile = tile;
  nb.swapped = swapped;
  nb.ksplit = ksplit;
  nb.tk = tk;
  nb.kg = kg;
  int bm = 0, bn = 0;
  mfma_tile_shape(tile, &bm, &bn);
  if (tile == 6 || tile == 7) bm = 64;  // (their epilogues write 64-row slices)
  // Epilogue write order: tile bits sorted by the output position they feed;
  // bits that select keys come last (columns before rows).
  const int kmb = swapped ? nd.nb : nd.mb, knb = swapped ? nd.mb : nd.nb;
  const int8_t* kpm = swapped ? nd.posN : nd.posM;
  const int8_t* kpn = swapped ? nd.posM : nd.posN;
  std::vector<std::pair<int, int>> keyed;  // (key, code)
  for (int j = 0; (1 << j) < bm; ++j) keyed.push_back({j < kmb ? int(kpm[j]) : 2000 + j, j});
  for (int j = 0; (1 << j) < bn; ++j) keyed.push_back({j < knb ? int(kpn[j]) : 1000 + j, 32 + j});
  std::sort(keyed.begin(), keyed.end());
  std::memset(nb.ubit, 0, sizeof(nb.ubit));
  for (size_t b = 0; b < keyed.size(); ++b) nb.ubit[b] = int8_t(keyed[b].second);
  nb.pair_mode = (want_keyed || !mfma_capable(nd, nvarL, nvarR, nb)) ? 2 : (nb.nvar == nvarL * nvarR ? 0 : 1);
  nb.keyed = nb.pair_mode == 2 ? 1 : 0;
}

void configure_generic(NodeBlock& nb, int form, int stream_l) {
  nb.kernel = XEB_KERNEL_GENERIC;
  nb.keyed = 0;
  nb.tile = form;
  nb.swapped = form == 1 ? stream_l : 0;
  nb.ksplit = 1;
  nb.pair_mode = 0;
}

bool generic_rows_ok(const Node& nd, int stream_l) {
  return stream_l ? generic_rows_fit(nd.kb, nd.mb, nd.nb) : generic_rows_fit(nd.kb, nd.nb, nd.mb);
}

void configure_generic_default(const Node& nd, NodeBlock& nb) {
  // The row-streaming form where it fits, streaming the wider side.
  const int first = nd.mb > nd.nb ? 1 : 0;
  for (int i = 0; i < 2; ++i) {
    const int sl = i == 0 ? first : 1 - first;
    if (generic_rows_ok(nd, sl)) {
      configure_generic(nb, 1, sl);
      return;
    }
  }
  configure_generic(nb, 0, 0);
}

int64_t node_tiles(const Node& nd, int64_t nvarL, int64_t nvarR, int tile, int swapped) {
  // (Stacked form; the keyed form never splits K.)
  int64_t rows = nvarL << nd.mb, cols = nvarR << nd.nb;
  if (swapped) std::swap(rows, cols);
  return mfma_tiles(tile, rows, cols);
}

namespace {

void choose_kernel(const Node& nd, int64_t nvarL, int64_t nvarR, NodeBlock& nb, bool force_generic,
                   int max_ksplit, double min_cmacs, int prec) {
  const double useful = double(nb.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
  const double rowsL = double(nvarL) * std::ldexp(1.0, nd.mb);
  const double rowsR = double(nvarR) * std::ldexp(1.0, nd.nb);
  const int swapped = (rowsR < rowsL && rowsR < 64) ? 1 : 0;
  const double rows = swapped ? rowsR : rowsL;
  const double cols = swapped ? rowsL : rowsR;
  const int tile = rows <= 16 ? 2 : (rows <= 32 ? 1 : 0);
  int bm = 0, bn = 0;
  mfma_tile_shape(tile, &bm, &bn);
  const double work = std::ceil(rows / bm) * bm * std::ceil(cols / bn) * bn *
                      std::max(std::ldexp(1.0, nd.kb), double(mfma_default_slab(prec)));
  // Both index forms are kept for nodes either kernel can run, so that the
  // autotuner may switch between them after compilation.
  if (mfma_capable(nd, nvarL, nvarR, nb) && nb.nvar != nvarL * nvarR) {
    nb.pairs.assign(size_t(nvarL * nvarR), -1);
    for (int64_t v = 0; v < nb.nvar; ++v)
      nb.pairs[size_t(int64_t(nb.lidx[v]) * nvarR + nb.ridx[v])] = int32_t(v);
  }
  configure_generic_default(nd, nb);
  if (force_generic) return;
  if (mfma_keyed(nd, nvarL, nvarR, nb)) {
    // One GEMM per key: the largest tile that each key's block fills, the
    // unswapped orientation first.
    const double keyed_work = useful / std::ldexp(1.0, nd.kb) *
                              std::max(std::ldexp(1.0, nd.kb), double(mfma_default_slab(prec)));
    if (useful < min_cmacs || 8 * useful < keyed_work) return;
    // The fitting tile with the least padding (then the lower tile number).
    int best_t = -1, best_sw = 0;
    double best_pad = 0;
    for (int t = 0; t < kMfmaTiles; ++t)
      for (int sw = 0; sw < 2; ++sw) {
        if (!mfma_keyed_fits(nd, t, sw)) continue;
        int bm = 0, bn = 0;
        mfma_tile_shape(t, &bm, &bn);
        const double M = std::ldexp(1.0, sw ? nd.nb : nd.mb), N = std::ldexp(1.0, sw ? nd.mb : nd.nb);
        const double pad = std::ceil(M / bm) * bm * std::ceil(N / bn) * bn / (M * N);
        if (best_t < 0 || pad < best_pad) {
          best_t = t;
          best_sw = sw;
          best_pad = pad;
        }
      }
    if (best_t >= 0) configure_mfma(nd, nvarL, nvarR, nb, best_t, best_sw, 1, mfma_default_slab(prec));
    return;
  }
  if (!mfma_capable(nd, nvarL, nvarR, nb) || rows < 8 || cols < 64 || useful < min_cmacs ||
      8 * useful < work)
    return;
  int ksplit = 1;
  const int64_t tiles = mfma_tiles(tile, int64_t(rows), int64_t(cols));
  const int64_t K = int64_t(1) << nd.kb;
  const int cap = max_ksplit == 0 ? 64 : max_ksplit;
  if (tiles < kSplitBelowTiles)
    while (ksplit < cap && tiles * ksplit < kSplitItems && K / (2 * ksplit) >= kMinChunk) ksplit *= 2;
  configure_mfma(nd, nvarL, nvarR, nb, tile, swapped, ksplit, mfma_default_slab(prec));
}

}  // namespace

void compile_plan(Plan& p, const xeb_circuit_t* c, const uint64_t* bits, int64_t k,
                  const xeb_tree_t* tree, const int32_t* sliced, int32_t s,
                  const xeb_options_t* opt) {
  xeb_options_t o;
  xeb_options_default(&o);
  if (opt) o = *opt;
  if (o.precision != XEB_PREC_C64 && o.precision != XEB_PREC_SPLIT_FP16 &&
      o.precision != XEB_PREC_SPLIT_BF16)
    fail(XEB_EINVAL, "unknown precision");
  if (o.device < 0) fail(XEB_EINVAL, "device ordinal is negative");
  if (o.max_ksplit < 0 || o.max_ksplit > 64 || (o.max_ksplit & (o.max_ksplit - 1)))
    fail(XEB_EINVAL, "max_ksplit must be 0 or a power of two up to 64");
  if (!(o.mfma_min_cmacs >= 0.0)) fail(XEB_EINVAL, "mfma_min_cmacs must be >= 0");
  if (o.abort_after_slices < 0) fail(XEB_EINVAL, "abort_after_slices must be >= 0");
  p.opt = o;

  Net net = build_net(c, o.fuse_1q != 0, o.fold_kets != 0);
  const int n = net.n_qubits;
  p.n_qubits = n;

  // ---- open output qubits (multi-batch output) ------------------------------
  const uint64_t open = o.open_qubits;
  if (n < 64 && (open >> n) != 0) fail(XEB_EINVAL, "open_qubits names a qubit at or above n_qubits");
  const int w = popcount64(open);
  if (w > 16) fail(XEB_EINVAL, "at most 16 open qubits");
  p.w = w;

  // ---- strings ----------------------------------------------------------
  if (k < 0) fail(XEB_EINVAL, "k is negative");
  if (k > (int64_t(1) << 31) - 1) fail(XEB_EINVAL, "k exceeds 2^31 - 1");
  if (k > 0 && !bits) fail(XEB_EINVAL, "bitstrings is NULL");
  for (int64_t i = 0; i < k; ++i)
    if (n < 64 && (bits[i] >> n) != 0) fail(XEB_EINVAL, "a bitstring has bits at or above n_qubits");

  // ---- tree -------------------------------------------------------------
  if (!tree) fail(XEB_EINVAL, "contraction tree is NULL");
  const int L = tree->n_leaves;
  if (L != int(net.leaves.size()))
    fail(XEB_EINVAL, "tree has " + std::to_string(L) + " leaves, network has " +
                         std::to_string(net.leaves.size()));
  if (L > 1 && !tree->children) fail(XEB_EINVAL, "tree children is NULL");
  const int nn = 2 * L - 1;
  p.n_leaves = L;
  p.root = nn - 1;
  p.nodes.assign(nn, Node());
  std::vector<char> used(nn, 0);
  for (int i = 0; i < L - 1; ++i) {
    const int T = L + i;
    const int a = tree->children[2 * i], b = tree->children[2 * i + 1];
    if (a < 0 || b < 0 || a >= T || b >= T || a == b)
      fail(XEB_EINVAL, "tree node " + std::to_string(T) + " has invalid children");
    if (used[a] || used[b]) fail(XEB_EINVAL, "tree node used twice as a child");
    used[a] = used[b] = 1;
    p.nodes[T].leaf = false;
    p.nodes[T].left = a;
    p.nodes[T].right = b;
    p.nodes[a].parent = T;
    p.nodes[b].parent = T;
  }

  // ---- sliced legs --------------------------------------------------------
  if (s < 0 || s > 40) fail(XEB_EINVAL, "number of sliced legs must be in [0, 40]");
  if (s > 0 && !sliced) fail(XEB_EINVAL, "sliced legs is NULL");
  const int J = o.stack_slices;
  if (J < 0 || J > s) fail(XEB_EINVAL, "stack_slices must be in [0, s]");
  if (n + J > 64) fail(XEB_EINVAL, "n_qubits + stack_slices exceeds 64 key bits");
  p.s = s;
  p.sj = J;
  p.sliced.assign(sliced, sliced + s);
  std::vector<int> slot(net.n_legs, -1);
  for (int j = 0; j < s; ++j) {
    const int l = sliced[j];
    if (l < 0 || l >= net.n_legs) fail(XEB_EINVAL, "sliced leg out of range");
    if (net.leg_qubit[l] >= 0) fail(XEB_EINVAL, "an output leg cannot be sliced");
    if (slot[l] >= 0) fail(XEB_EINVAL, "sliced leg listed twice");
    slot[l] = j;
  }

  // ---- leg sets and masks -------------------------------------------------
  for (int j = 0; j < L; ++j) {
    Node& nd = p.nodes[j];
    for (int32_t leg : net.leaves[j].legs) {
      const int q = net.leg_qubit[leg];
      if (q >= 0 && ((open >> q) & 1))
        nd.legs.push_back(leg);  // open output leg: a tensor leg up to the root
      else if (q >= 0)
        nd.outmask |= uint64_t(1) << q;
      else if (slot[leg] >= 0 && slot[leg] < J)
        nd.outmask |= uint64_t(1) << (n + slot[leg]);  // stacked: a key bit
      else if (slot[leg] >= 0)
        nd.smask |= uint64_t(1) << (slot[leg] - J);
      else
        nd.legs.push_back(leg);
    }
    nd.nslicekeys = int64_t(1) << popcount64(nd.smask);
  }
  for (int T = L; T < nn; ++T) {
    Node& nd = p.nodes[T];
    const Node& a = p.nodes[nd.left];
    const Node& b = p.nodes[nd.right];
    std::vector<int32_t> la = sorted_copy(a.legs), lb = sorted_copy(b.legs);
    std::set_symmetric_difference(la.begin(), la.end(), lb.begin(), lb.end(),
                                  std::back_inserter(nd.legs));
    nd.outmask = a.outmask | b.outmask;
    nd.smask = a.smask | b.smask;
    if (nd.legs.size() > size_t(kMaxBits)) fail(XEB_EINVAL, "intermediate tensor has too many legs");
  }
  // The root keeps exactly the open output legs, ordered by qubit (bit j of a
  // root element's index = the j-th open qubit).
  {
    std::vector<int32_t>& rl = p.nodes[p.root].legs;
    for (int32_t leg : rl)
      if (net.leg_qubit[leg] < 0) fail(XEB_EINVAL, "the tree does not close the network");
    if (int(rl.size()) != w) fail(XEB_EINVAL, "internal: open legs missing at the root");
    std::sort(rl.begin(), rl.end(),
              [&](int32_t x, int32_t y) { return net.leg_qubit[x] < net.leg_qubit[y]; });
  }

  // ---- layouts (top-down) -------------------------------------------------
  std::vector<int> pos(net.n_legs, -1);
  for (int T = nn - 1; T >= L; --T) {
    Node& nd = p.nodes[T];
    Node& a = p.nodes[nd.left];
    Node& b = p.nodes[nd.right];
    for (size_t q = 0; q < nd.legs.size(); ++q) pos[nd.legs[q]] = int(q);
    std::vector<int32_t> la = sorted_copy(a.legs), lb = sorted_copy(b.legs), K, M, N;
    std::set_intersection(la.begin(), la.end(), lb.begin(), lb.end(), std::back_inserter(K));
    std::set_difference(la.begin(), la.end(), K.begin(), K.end(), std::back_inserter(M));
    std::set_difference(lb.begin(), lb.end(), K.begin(), K.end(), std::back_inserter(N));
    auto by_pos = [&](int32_t x, int32_t y) { return pos[x] < pos[y]; };
    std::sort(M.begin(), M.end(), by_pos);
    std::sort(N.begin(), N.end(), by_pos);
    nd.mb = int(M.size());
    nd.nb = int(N.size());
    nd.kb = int(K.size());
    for (int j = 0; j < nd.mb; ++j) nd.posM[j] = int8_t(pos[M[j]]);
    for (int j = 0; j < nd.nb; ++j) nd.posN[j] = int8_t(pos[N[j]]);
    // Sorted by parent position, the row and column bits land in increasing
    // output positions: the kernels' placement is a bit deposit by mask.
    nd.maskM = nd.maskN = 0;
    for (int j = 0; j < nd.mb; ++j) {
      if (j > 0 && nd.posM[j] <= nd.posM[j - 1]) fail(XEB_EINVAL, "internal: row bits out of order");
      nd.maskM |= uint64_t(1) << nd.posM[j];
    }
    for (int j = 0; j < nd.nb; ++j) {
      if (j > 0 && nd.posN[j] <= nd.posN[j - 1]) fail(XEB_EINVAL, "internal: column bits out of order");
      nd.maskN |= uint64_t(1) << nd.posN[j];
    }
    if ((nd.maskM & nd.maskN) || popcount64(nd.maskM | nd.maskN) != nd.mb + nd.nb ||
        (nd.mb + nd.nb < 64 && (nd.maskM | nd.maskN) >> (nd.mb + nd.nb)))
      fail(XEB_EINVAL, "internal: row and column bits do not partition the output");
    for (int32_t x : nd.legs) pos[x] = -1;
    a.legs = K;
    a.legs.insert(a.legs.end(), M.begin(), M.end());
    b.legs = K;
    b.legs.insert(b.legs.end(), N.begin(), N.end());
  }

  // ---- strings in lexicographic tuple order (Appendix C) --------------------
  // Keyed strings: every distinct string with every low slice key, the slice
  // key in bits n .. n + J - 1.  A keyed string's tuple lists its leaf keys
  // in depth-first leaf order; a stacked slice bit sits on the two leaves its
  // leg joins, and only its first occurrence enters the sort key, so the
  // concatenated key has n + J <= 64 bits.
  // (Open bits are no key: strings that differ only there share one entry.)
  std::vector<uint64_t> dr(k);
  for (int64_t i = 0; i < k; ++i) dr[i] = bits[i] & ~open;
  std::sort(dr.begin(), dr.end());
  dr.erase(std::unique(dr.begin(), dr.end()), dr.end());
  const int64_t kdr = int64_t(dr.size());
  const int64_t kd = kdr << J;
  if (kd > (int64_t(1) << 31) - 1) fail(XEB_EINVAL, "distinct strings times 2^stack_slices exceed 2^31 - 1");
  std::vector<uint64_t> ds(kd);
  for (int64_t i = 0; i < kdr; ++i)
    for (int64_t sl = 0; sl < (int64_t(1) << J); ++sl)
      ds[(i << J) | sl] = dr[i] | (J > 0 ? uint64_t(sl) << n : 0);
  p.k = k;
  p.kd = kd;
  std::vector<int> dfs;
  leaves_dfs(p.nodes, p.root, dfs);
  {
    std::vector<uint64_t> first_bits;  // per DFS leaf: its key bits not seen before
    uint64_t seen = 0;
    for (int j : dfs) {
      first_bits.push_back(p.nodes[j].outmask & ~seen);
      seen |= p.nodes[j].outmask;
    }
    std::vector<std::pair<uint64_t, uint64_t>> keyed(kd);
    for (int64_t i = 0; i < kd; ++i) {
      uint64_t key = 0;
      for (uint64_t om : first_bits) {
        if (!om) continue;
        const int w = popcount64(om);
        key = (w == 64 ? 0 : (key << w)) | pext64(ds[i], om);
      }
      keyed[i] = {key, ds[i]};
    }
    std::sort(keyed.begin(), keyed.end());
    for (int64_t i = 0; i < kd; ++i) ds[i] = keyed[i].second;
  }

  // ---- leaf keys (over all strings) -----------------------------------------
  std::vector<std::vector<int32_t>> leaf_var(L);
  for (int j = 0; j < L; ++j) {
    Node& nd = p.nodes[j];
    std::vector<uint64_t> keys(kd);
    for (int64_t i = 0; i < kd; ++i) keys[i] = pext64(ds[i], nd.outmask);
    std::vector<uint64_t> uk(keys);
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    if (uk.empty()) uk.push_back(0);
    nd.leaf_keys = uk;
    nd.leaf_nvar = int64_t(uk.size());
    leaf_var[j].resize(kd);
    for (int64_t i = 0; i < kd; ++i)
      leaf_var[j][i] = int32_t(std::lower_bound(uk.begin(), uk.end(), keys[i]) - uk.begin());
  }
  // Position among the sorted keyed strings of (distinct string r, low slice
  // key sl): pos_of[(r << J) | sl], r indexing the ascending distinct strings.
  std::vector<int64_t> pos_of(kd);
  {
    const uint64_t real = n < 64 ? (uint64_t(1) << n) - 1 : ~uint64_t(0);
    for (int64_t j = 0; j < kd; ++j) {
      const uint64_t x = ds[j];
      const int64_t r = std::lower_bound(dr.begin(), dr.end(), x & real) - dr.begin();
      const int64_t sl = J > 0 ? int64_t(x >> n) : 0;
      pos_of[(r << J) | sl] = j;
    }
  }
  // Distinct string of every input string.
  std::vector<int64_t> where(k);
  for (int64_t i = 0; i < k; ++i)
    where[i] = std::lower_bound(dr.begin(), dr.end(), bits[i] & ~open) - dr.begin();

  // Keys of every internal node among the strings [first, first + count).
  auto build_block = [&](int64_t first, int64_t count) {
    Block blk;
    blk.first = first;
    blk.count = count;
    blk.nodes.resize(nn - L);
    std::vector<std::vector<int32_t>> var(nn);
    auto var_of = [&](int id, int64_t i) -> int32_t {
      return p.nodes[id].leaf ? leaf_var[id][first + i] : var[id][i];
    };
    auto nvar_of = [&](int id) -> int64_t {
      return p.nodes[id].leaf ? p.nodes[id].leaf_nvar : blk.nodes[id - L].nvar;
    };
    for (int T = L; T < nn; ++T) {
      const Node& nd = p.nodes[T];
      NodeBlock& nb = blk.nodes[T - L];
      const int64_t nr = nvar_of(nd.right);
      std::vector<int64_t> codes(count);
      for (int64_t i = 0; i < count; ++i)
        codes[i] = int64_t(var_of(nd.left, i)) * nr + var_of(nd.right, i);
      // Distinct codes in increasing order and each string's rank among them:
      // a mark table over all (left, right) pairs when it is not much larger
      // than the strings, else a sort.
      const int64_t npairs = nvar_of(nd.left) * nr;
      std::vector<int64_t> uc;
      var[T].resize(count);
      if (npairs <= std::max<int64_t>(4 * count, int64_t(1) << 22)) {
        std::vector<int32_t> rank(size_t(npairs), 0);
        for (int64_t i = 0; i < count; ++i) rank[size_t(codes[i])] = 1;
        int32_t next = 0;
        for (int64_t c2 = 0; c2 < npairs; ++c2)
          if (rank[size_t(c2)]) {
            rank[size_t(c2)] = next++;
            uc.push_back(c2);
          }
        for (int64_t i = 0; i < count; ++i) var[T][i] = rank[size_t(codes[i])];
      } else {
        uc = codes;
        std::sort(uc.begin(), uc.end());
        uc.erase(std::unique(uc.begin(), uc.end()), uc.end());
        for (int64_t i = 0; i < count; ++i)
          var[T][i] = int32_t(std::lower_bound(uc.begin(), uc.end(), codes[i]) - uc.begin());
      }
      if (uc.empty()) uc.push_back(0);
      nb.nvar = int64_t(uc.size());
      nb.lidx.resize(nb.nvar);
      nb.ridx.resize(nb.nvar);
      for (int64_t v = 0; v < nb.nvar; ++v) {
        nb.lidx[v] = int32_t(uc[v] / nr);
        nb.ridx[v] = int32_t(uc[v] % nr);
      }
      if (!p.nodes[nd.left].leaf) std::vector<int32_t>().swap(var[nd.left]);
      if (!p.nodes[nd.right].leaf) std::vector<int32_t>().swap(var[nd.right]);
      choose_kernel(nd, nvar_of(nd.left), nr, nb, o.force_generic != 0, o.max_ksplit,
                    o.mfma_min_cmacs > 0 ? o.mfma_min_cmacs : kMfmaMinCmacs, o.precision);
    }
    for (int64_t i = 0; i < k; ++i) {
      bool any = false;
      for (int64_t sl = 0; sl < (int64_t(1) << J); ++sl) {
        const int64_t d = pos_of[(where[i] << J) | sl];
        if (d < first || d >= first + count) continue;
        if (!any) {
          blk.idx.push_back(int32_t(i));
          blk.eoff.push_back(int32_t(blk.rho.size()));
          any = true;
        }
        blk.rho.push_back(L == 1 ? leaf_var[0][d] : var[p.root][d - first]);
        blk.slo.push_back(int32_t(sl));
      }
    }
    blk.eoff.push_back(int32_t(blk.rho.size()));
    return blk;
  };

  // ---- workspace (dry run) --------------------------------------------------
  // Static region (uploaded at bind): leaf tables, per-block gather maps and
  // string maps, leaf amax.  Dynamic region: node tables (sized for the
  // largest block), amax slots, compensation, scratch.
  auto layout = [&](std::vector<Block>& blocks) -> uint64_t {
    uint64_t off = 0;
    for (int j = 0; j < L; ++j) {
      Node& nd = p.nodes[j];
      nd.off_table = off;
      off += align_up(uint64_t(nd.nslicekeys) * nd.leaf_nvar * nd.size() * 8);
    }
    for (Block& blk : blocks) {
      for (NodeBlock& nb : blk.nodes) {
        nb.off_lidx = off;
        off += align16(uint64_t(nb.nvar) * 4);
        nb.off_ridx = off;
        off += align16(uint64_t(nb.nvar) * 4);
        if (!nb.pairs.empty()) {
          nb.off_pairs = off;
          off += align16(nb.pairs.size() * 4);
        }
      }
      blk.off_idx = off;
      off += align16(blk.idx.size() * 4);
      blk.off_eoff = off;
      off += align16(blk.eoff.size() * 4);
      blk.off_rho = off;
      off += align16(blk.rho.size() * 4);
      blk.off_slo = off;
      off += align16(blk.slo.size() * 4);
    }
    p.off_leaf_amax = off;
    off += align_up(uint64_t(nn) * 8);
    if (w > 0) {
      p.off_sel = off;
      off += align_up(uint64_t(k) * 4);
    }
    const uint64_t static_end = off;
    // Node tables.  A table is transient when its parent is only ever
    // evaluated right after it within the same slice step: then it lives from
    // its own evaluation to the parent's (ids are post-order) and shares an
    // arena with other transient tables, packed first-fit by lifetime.  Other
    // tables are read again later without being recomputed and keep their own
    // region.
    const bool many_blocks = blocks.size() > 1;
    auto transient = [&](int T) {
      if (T == p.root) return true;
      const Node& nd = p.nodes[T];
      const Node& par = p.nodes[nd.parent];
      const bool slice_ok =
          par.smask == 0 || (nd.smask != 0 && __builtin_ctzll(nd.smask) == __builtin_ctzll(par.smask));
      if (!slice_ok) return false;
      if (!many_blocks || nd.outmask != 0) return true;
      return par.outmask == 0 && par.smask == 0;
    };
    struct Live {
      int node;
      int begin, end;  // evaluation positions (node ids) where the table is live
      uint64_t bytes;
    };
    std::vector<Live> lives;
    uint64_t persistent_end = off;
    for (int T = L; T < nn; ++T) {
      Node& nd = p.nodes[T];
      nd.table_nvar = 1;
      for (const Block& blk : blocks) nd.table_nvar = std::max(nd.table_nvar, blk.nodes[T - L].nvar);
      const uint64_t bytes = align_up(uint64_t(nd.table_nvar) * nd.size() * 8);
      if (transient(T)) {
        lives.push_back({T, T, T == p.root ? nn : nd.parent, bytes});
      } else {
        nd.off_table = persistent_end;
        persistent_end += bytes;
      }
    }
    // First-fit interval packing (largest tables first).
    std::sort(lives.begin(), lives.end(), [](const Live& x, const Live& y) {
      return x.bytes != y.bytes ? x.bytes > y.bytes : x.node < y.node;
    });
    std::vector<std::pair<uint64_t, const Live*>> placed;  // (arena offset, live)
    uint64_t arena = 0;
    for (const Live& lv : lives) {
      std::vector<std::pair<uint64_t, uint64_t>> busy;  // overlapping [offset, offset + bytes)
      for (auto& pl : placed)
        if (pl.second->begin <= lv.end && lv.begin <= pl.second->end)
          busy.push_back({pl.first, pl.first + pl.second->bytes});
      std::sort(busy.begin(), busy.end());
      uint64_t at = 0;
      for (auto& b : busy) {
        if (at + lv.bytes <= b.first) break;
        at = std::max(at, b.second);
      }
      placed.push_back({at, &lv});
      arena = std::max(arena, at + lv.bytes);
    }
    for (auto& pl : placed) p.nodes[pl.second->node].off_table = persistent_end + pl.first;
    off = persistent_end + arena;
    p.off_amax = off;
    if (o.precision == XEB_PREC_SPLIT_FP16) off += align_up(uint64_t(nn) * kAmaxSlots * kAmaxStride * 8);
    uint64_t partial = 0;
    for (const Block& blk : blocks)
      for (int T = L; T < nn; ++T) {
        const NodeBlock& nb = blk.nodes[T - L];
        if (nb.kernel != XEB_KERNEL_MFMA || nb.ksplit == 1) continue;
        const Node& nd = p.nodes[T];
        const int64_t nl = p.nodes[nd.left].leaf ? p.nodes[nd.left].leaf_nvar : blk.nodes[nd.left - L].nvar;
        const int64_t nr = p.nodes[nd.right].leaf ? p.nodes[nd.right].leaf_nvar : blk.nodes[nd.right - L].nvar;
        int64_t rowsA = nl << nd.mb, rowsB = nr << nd.nb;
        if (nb.swapped) std::swap(rowsA, rowsB);
        int bm = 0, bn = 0;
        mfma_tile_shape(nb.tile, &bm, &bn);
        partial = std::max<uint64_t>(partial, uint64_t(mfma_tiles(nb.tile, rowsA, rowsB)) * nb.ksplit *
                                                  uint64_t(bm) * bn * 8);
      }
    // Room for the autotuner's split-K candidates on long-K nodes.
    bool long_k = false;
    for (const Block& blk : blocks)
      for (int T = L; T < nn; ++T) {
        const Node& nd = p.nodes[T];
        const NodeBlock& nb = blk.nodes[T - L];
        const int64_t nl = p.nodes[nd.left].leaf ? p.nodes[nd.left].leaf_nvar : blk.nodes[nd.left - L].nvar;
        const int64_t nr = p.nodes[nd.right].leaf ? p.nodes[nd.right].leaf_nvar : blk.nodes[nd.right - L].nvar;
        if (nd.kb >= 7 && mfma_capable(nd, nl, nr, nb)) long_k = true;
      }
    // (Under a memory budget the reserve takes at most 1/16 of it.)
    const uint64_t reserve =
        o.memory_budget ? std::min<uint64_t>(kTunePartialBytes, o.memory_budget / 16) : kTunePartialBytes;
    if (long_k) partial = std::max<uint64_t>(partial, reserve);
    p.off_partial = off;
    p.partial_bytes = align_up(partial);
    off += p.partial_bytes;
    // Plane-format operands (tile 6): both children of the largest node that
    // could run it, converted on each launch, up to kMaxPlaneBytes (or 1/8
    // of the budget); larger nodes do not take tile 6.
    const uint64_t plane_cap =
        o.memory_budget ? std::min<uint64_t>(kMaxPlaneBytes, o.memory_budget / 8) : kMaxPlaneBytes;
    uint64_t planes = 0;
    if (o.precision != XEB_PREC_C64)
      for (const Block& blk : blocks)
        for (int T = L; T < nn; ++T) {
          const Node& nd = p.nodes[T];
          const NodeBlock& nb = blk.nodes[T - L];
          const int64_t nl = p.nodes[nd.left].leaf ? p.nodes[nd.left].leaf_nvar : blk.nodes[nd.left - L].nvar;
          const int64_t nr = p.nodes[nd.right].leaf ? p.nodes[nd.right].leaf_nvar : blk.nodes[nd.right - L].nvar;
          if (nd.kb < 4 || nd.kb > 21 || !(mfma_capable(nd, nl, nr, nb) || mfma_keyed(nd, nl, nr, nb)))
            continue;
          const uint64_t need = planes_need(nd, nl, nr);
          if (need <= plane_cap) planes = std::max(planes, need);
        }
    p.off_planes = off;
    p.planes_bytes = planes;
    off += planes;
    p.off_comp = off;
    off += align_up((uint64_t(k) << w) * 16);
    if (w > 0) {
      p.off_gather = off;
      off += align_up(uint64_t(k) * 16);
    }
    p.off_scratch = off;
    off += align_up(xeb_scratch_bytes(k));
    p.ws_bytes = off;
    if (o.trace > 1)
      std::fprintf(stderr,
                   "{\"blocks\":%zu,\"static\":%llu,\"persistent_tables\":%llu,"
                   "\"arena\":%llu,\"workspace\":%llu}\n",
                   blocks.size(), (unsigned long long)static_end,
                   (unsigned long long)(persistent_end - static_end), (unsigned long long)arena,
                   (unsigned long long)off);
    return static_end;
  };

  // Smallest power-of-two block count that fits; give up after three
  // doublings in a row that do not shrink the workspace below its best.
  uint64_t static_bytes = 0;
  uint64_t best_bytes = ~uint64_t(0);
  int stale = 0;
  for (int64_t nblocks = 1;; nblocks *= 2) {
    if (kd > 0 && nblocks > kd) nblocks = kd;
    std::vector<Block> blocks;
    const int64_t nbk = std::max<int64_t>(nblocks, 1);
    for (int64_t b = 0; b < nbk; ++b) {
      const int64_t first = kd * b / nbk, last = kd * (b + 1) / nbk;
      if (last > first || kd == 0) blocks.push_back(build_block(first, last - first));
    }
    static_bytes = layout(blocks);
    p.blocks = std::move(blocks);
    if (!o.memory_budget || p.ws_bytes <= o.memory_budget) break;
    if (p.ws_bytes < best_bytes) {
      best_bytes = p.ws_bytes;
      stale = 0;
    } else {
      ++stale;
    }
    if (nblocks >= std::max<int64_t>(kd, 1) || stale >= 3)
      fail(XEB_ENOMEM, "workspace of at least " + std::to_string(best_bytes) +
                           " bytes exceeds the budget; more string blocks do not shrink it");
  }

  // ---- leaf tables (FP64 -> complex64) --------------------------------------
  p.staging.assign(static_bytes / 4, 0.f);
  for (int j = 0; j < L; ++j) {
    Node& nd = p.nodes[j];
    const NetLeaf& nl = net.leaves[j];
    const int R = int(nl.legs.size());
    const int r = int(nd.legs.size());
    std::vector<int> axis_pos(R, -1);  // position in nd.legs, or -1
    for (int a = 0; a < R; ++a)
      for (int q = 0; q < r; ++q)
        if (nd.legs[q] == nl.legs[a]) axis_pos[a] = q;
    float* dst = p.staging.data() + nd.off_table / 4;
    for (int64_t kappa = 0; kappa < nd.nslicekeys; ++kappa)
      for (int64_t v = 0; v < nd.leaf_nvar; ++v)
        for (int64_t e = 0; e < nd.size(); ++e) {
          int64_t idx = 0;
          for (int a = 0; a < R; ++a) {
            const int32_t leg = nl.legs[a];
            int bit;
            if (axis_pos[a] >= 0)
              bit = int((e >> axis_pos[a]) & 1);
            else if (net.leg_qubit[leg] >= 0)
              bit = int((nd.leaf_keys[v] >> rank_in_mask(nd.outmask, net.leg_qubit[leg])) & 1);
            else if (slot[leg] < J)
              bit = int((nd.leaf_keys[v] >> rank_in_mask(nd.outmask, n + slot[leg])) & 1);
            else
              bit = int((kappa >> rank_in_mask(nd.smask, slot[leg] - J)) & 1);
            idx |= int64_t(bit) << (R - 1 - a);
          }
          const cplx x = nl.data[idx];
          const int64_t o2 = ((kappa * nd.leaf_nvar + v) * nd.size() + e) * 2;
          dst[o2] = float(x.real());
          dst[o2 + 1] = float(x.imag());
          nd.leaf_amax = std::max(nd.leaf_amax, std::max(std::fabs(dst[o2]), std::fabs(dst[o2 + 1])));
        }
    // Largest magnitude of the leaf table (the FP16 scale of a leaf operand),
    // as one amax slot of epoch 0.
    uint32_t bits32 = 0;
    std::memcpy(&bits32, &nd.leaf_amax, 4);
    const uint64_t slot = bits32;
    std::memcpy(p.staging.data() + p.off_leaf_amax / 4 + 2 * j, &slot, 8);
  }
  auto put = [&](uint64_t off, const std::vector<int32_t>& v) {
    if (!v.empty()) std::memcpy(p.staging.data() + off / 4, v.data(), v.size() * 4);
  };
  for (Block& blk : p.blocks) {
    for (NodeBlock& nb : blk.nodes) {
      put(nb.off_lidx, nb.lidx);
      put(nb.off_ridx, nb.ridx);
      if (!nb.pairs.empty()) put(nb.off_pairs, nb.pairs);
    }
    put(blk.off_idx, blk.idx);
    put(blk.off_eoff, blk.eoff);
    put(blk.off_rho, blk.rho);
    put(blk.off_slo, blk.slo);
  }
  if (w > 0) {
    std::vector<int32_t> sel(k);
    for (int64_t i = 0; i < k; ++i) sel[i] = int32_t(pext64(bits[i], open));
    put(p.off_sel, sel);
  }

  // ---- stats -----------------------------------------------------------------
  xeb_stats_t& st = p.stats;
  st = xeb_stats_t{};
  st.n_leaves = L;
  st.n_internal = L - 1;
  st.k = k;
  st.k_distinct = kdr;
  st.n_qubits = n;
  st.n_sliced = s;
  st.n_stacked = J;
  st.n_open = w;
  st.n_blocks = int64_t(p.blocks.size());
  for (int T = 0; T < nn; ++T)
    st.max_tensor_elems = std::max<int64_t>(st.max_tensor_elems, p.nodes[T].size());
  for (const Block& blk : p.blocks) {
    auto nv = [&](int id) {
      return p.nodes[id].leaf ? p.nodes[id].leaf_nvar : blk.nodes[id - L].nvar;
    };
    for (int T = L; T < nn; ++T) {
      const Node& nd = p.nodes[T];
      const NodeBlock& nb = blk.nodes[T - L];
      st.sum_variants += nb.nvar;
      const double cm = double(nb.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
      // A node without output legs keeps its table across blocks when it
      // depends on no slice bit.
      const bool kept = nd.outmask == 0 && nd.smask == 0 && &blk != &p.blocks.front();
      const double ev = kept ? 0.0 : evals_over_all_slices(nd.smask, s - J);
      st.cmacs_per_slice += cm;
      st.cmacs_full += ev * cm;
      st.rw_elems_full += ev * (double(nv(nd.left)) * p.nodes[nd.left].size() +
                                double(nv(nd.right)) * p.nodes[nd.right].size() +
                                double(nb.nvar) * nd.size());
      st.evals_full += ev;
    }
  }
  st.workspace_bytes = p.ws_bytes;

  if (o.trace > 0) {
    const Block& blk = p.blocks.front();
    for (int T = L; T < nn; ++T) {
      const Node& nd = p.nodes[T];
      const NodeBlock& nb = blk.nodes[T - L];
      // Output positions 0, 1, 2, ... taken by the first row (m) or column
      // (n) bits: how many of the lowest output bits each side holds.
      int run_m = 0, run_n = 0;
      while (run_m < nd.mb && nd.posM[run_m] == run_m) ++run_m;
      while (run_n < nd.nb && nd.posN[run_n] == run_n) ++run_n;
      // 128 x 128 output tiles of the stacked (left rows x right rows)
      // product, and those holding at least one key.
      const int64_t nl = p.nodes[nd.left].leaf ? p.nodes[nd.left].leaf_nvar : blk.nodes[nd.left - L].nvar;
      const int64_t nr = p.nodes[nd.right].leaf ? p.nodes[nd.right].leaf_nvar : blk.nodes[nd.right - L].nvar;
      const int64_t tr = ((nl << nd.mb) + 127) / 128, tc = ((nr << nd.nb) + 127) / 128;
      std::vector<uint8_t> hit;
      int64_t used = 0;
      if (tr * tc <= (int64_t(1) << 26)) {
        hit.assign(size_t(tr * tc), 0);
        for (int64_t v = 0; v < nb.nvar; ++v) {
          const int64_t r0 = (int64_t(nb.lidx[v]) << nd.mb) / 128, r1 = ((int64_t(nb.lidx[v] + 1) << nd.mb) - 1) / 128;
          const int64_t c0 = (int64_t(nb.ridx[v]) << nd.nb) / 128, c1 = ((int64_t(nb.ridx[v] + 1) << nd.nb) - 1) / 128;
          for (int64_t r = r0; r <= r1; ++r)
            for (int64_t c = c0; c <= c1; ++c) hit[size_t(r * tc + c)] = 1;
        }
        for (uint8_t h : hit) used += h;
      }
      std::fprintf(stderr,
                   "{\"node\":%d,\"left\":%d,\"right\":%d,\"variants\":%lld,\"m_bits\":%d,"
                   "\"n_bits\":%d,\"k_bits\":%d,\"slice_mask\":%llu,\"kernel\":%d,\"blocks\":%zu,"
                   "\"low_run_m\":%d,\"low_run_n\":%d,\"tiles_128\":%lld,\"key_tiles_128\":%lld}\n",
                   T, nd.left, nd.right, (long long)nb.nvar, nd.mb, nd.nb, nd.kb,
                   (unsigned long long)nd.smask, nb.kernel, p.blocks.size(), run_m, run_n,
                   (long long)(tr * tc), (long long)used);
    }
  }
}

void bind_plan(Plan* p, void* dev, uint64_t bytes) {
  if (!dev) fail(XEB_EINVAL, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(dev) % kAlign) fail(XEB_EINVAL, "workspace is not 256-byte aligned");
  if (bytes < p->ws_bytes)
    fail(XEB_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, plan needs " +
                         std::to_string(p->ws_bytes));
  DeviceGuard g(p->opt.device);
  if (!p->staging.empty())
    hip_check(hipMemcpy(dev, p->staging.data(), p->staging.size() * 4, hipMemcpyHostToDevice),
              "upload of leaf tables");
  p->ws = dev;
  p->ws_size = bytes;
  for (Node& nd : p->nodes) nd.valid = false;
}

Plan::~Plan() {
  for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
  for (ProfRecord& r : prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
}

namespace {

hipEvent_t take_event(Plan* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hip_check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void recycle_records(Plan* p) {
  for (ProfRecord& r : p->prof) {
    p->event_pool.push_back(r.start);
    p->event_pool.push_back(r.stop);
  }
  p->prof.clear();
}

// With profiling on, times `launch` (one launch group) by an event pair
// carried on its kernels' dispatch packets; an event no kernel carried (an
// empty launch) is recorded on the stream instead, so every pair is valid.
template <class F>
void timed(Plan* p, hipStream_t stream, int kernel, int node, double cmacs, double bytes,
           F&& launch) {
  if (!p->profiling || p->capturing) {
    launch();
    return;
  }
  ProfRecord r{take_event(p), take_event(p), kernel, node, cmacs, bytes};
  set_launch_events(r.start, r.stop);
  struct Clear {  // no event stays attached if the launch throws
    ~Clear() {
      hipEvent_t a = nullptr, b = nullptr;
      take_launch_events(&a, &b);
    }
  };
  hipEvent_t start = nullptr, stop = nullptr;
  {
    Clear clear;
    launch();
    take_launch_events(&start, &stop);
  }
  if (start) hip_check(hipEventRecord(start, stream), "hipEventRecord");
  if (stop) hip_check(hipEventRecord(stop, stream), "hipEventRecord");
  p->prof.push_back(r);
}

}  // namespace

void set_profiling(Plan* p, bool on) {
  DeviceGuard g(p->opt.device);
  if (!p->prof.empty()) {
    for (ProfRecord& r : p->prof) hip_check(hipEventSynchronize(r.stop), "hipEventSynchronize");
    recycle_records(p);
  }
  p->profiling = on;
}

xeb_kernel_profile_t read_profile(Plan* p, int kernel, int node) {
  DeviceGuard g(p->opt.device);
  xeb_kernel_profile_t out{};
  for (ProfRecord& r : p->prof) {
    if (kernel >= 0 && r.kernel != kernel) continue;
    if (node >= 0 && r.node != node) continue;
    hip_check(hipEventSynchronize(r.stop), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, r.start, r.stop), "hipEventElapsedTime");
    out.launches += 1;
    out.seconds += double(ms) * 1e-3;
    out.cmacs += r.cmacs;
    out.bytes += r.bytes;
  }
  return out;
}

namespace {

// Current table of a node for slice sigma: internal nodes hold the block's
// keys; a leaf's sub-table is picked by its slice key.
const float2* node_ptr(const Plan* p, int id, int64_t sigma) {
  const Node& nd = p->nodes[id];
  const char* base = static_cast<const char*>(p->ws) + nd.off_table;
  if (nd.leaf) {
    const uint64_t kappa = pext64(uint64_t(sigma), nd.smask);
    base += kappa * uint64_t(nd.leaf_nvar) * nd.size() * 8;
  }
  return reinterpret_cast<const float2*>(base);
}

}  // namespace

int64_t nvar_in(const Plan* p, const Block& blk, int id) {
  return p->nodes[id].leaf ? p->nodes[id].leaf_nvar : blk.nodes[id - p->n_leaves].nvar;
}

double evals_per_call(const Plan* p, int T) {
  return evals_over_all_slices(p->nodes[T].smask, p->s - p->sj);
}

ContractArgs node_args(Plan* p, const Block& blk, int T, int64_t sigma) {
  char* ws = static_cast<char*>(p->ws);
  const Node& nd = p->nodes[T];
  const NodeBlock& nb = blk.nodes[T - p->n_leaves];
  ContractArgs a{};
  const bool sw = nb.kernel == XEB_KERNEL_MFMA && nb.swapped;
  a.A = node_ptr(p, sw ? nd.right : nd.left, sigma);
  a.B = node_ptr(p, sw ? nd.left : nd.right, sigma);
  a.C = reinterpret_cast<float2*>(ws + nd.off_table);
  a.nvar = nb.nvar;
  a.nvarA = nvar_in(p, blk, sw ? nd.right : nd.left);
  a.nvarB = nvar_in(p, blk, sw ? nd.left : nd.right);
  a.mb = sw ? nd.nb : nd.mb;
  a.nb = sw ? nd.mb : nd.nb;
  a.kb = nd.kb;
  a.pair_mode = nb.pair_mode;
  // (The per-element kernel keeps L and R in place; its swapped flag names
  // the stream side of the row-streaming form.)
  a.swapped = nb.kernel == XEB_KERNEL_MFMA ? (sw ? 1 : 0) : nb.swapped;
  a.tile = nb.tile;
  a.tk = nb.tk;
  a.kg = nb.kg;
  a.prec = p->opt.precision;
  a.mapM = bit_map(sw ? nd.maskN : nd.maskM);
  a.mapN = bit_map(sw ? nd.maskM : nd.maskN);
  std::memcpy(a.ubit, nb.ubit, sizeof(a.ubit));
  if (p->opt.precision == XEB_PREC_SPLIT_FP16) {
    // A leaf has one static slot; an internal node kAmaxSlots slots.  The
    // caller sets the epoch.
    const uint64_t amax_words = uint64_t(kAmaxSlots) * kAmaxStride;
    unsigned long long* slots = reinterpret_cast<unsigned long long*>(ws + p->off_amax);
    const unsigned long long* leaf_amax = reinterpret_cast<const unsigned long long*>(ws + p->off_leaf_amax);
    const int ida = sw ? nd.right : nd.left, idb = sw ? nd.left : nd.right;
    auto amax_of = [&](int id) -> const unsigned long long* {
      return p->nodes[id].leaf ? leaf_amax + id : slots + uint64_t(id) * amax_words;
    };
    a.amaxA = amax_of(ida);
    a.amaxB = amax_of(idb);
    a.amax_nA = p->nodes[ida].leaf ? 1 : kAmaxSlots;
    a.amax_nB = p->nodes[idb].leaf ? 1 : kAmaxSlots;
    a.amax_out = slots + uint64_t(T) * amax_words;
  }
  a.ksplit = nb.kernel == XEB_KERNEL_MFMA ? nb.ksplit : 1;
  a.partial = reinterpret_cast<float2*>(ws + p->off_partial);
  if (p->planes_bytes) {
    // Row operand's planes first, the column operand's after them.
    const uint64_t a_bytes = align_up((uint64_t(a.nvarA) << a.mb) * (uint64_t(8) << a.kb));
    a.Ap = reinterpret_cast<uint16_t*>(ws + p->off_planes);
    a.Bp = reinterpret_cast<uint16_t*>(ws + p->off_planes + a_bytes);
  }
  a.pairs = nb.kernel == XEB_KERNEL_MFMA && nb.pair_mode == 1
                ? reinterpret_cast<const int32_t*>(ws + nb.off_pairs)
                : nullptr;
  a.lidx = reinterpret_cast<const int32_t*>(ws + nb.off_lidx);
  a.ridx = reinterpret_cast<const int32_t*>(ws + nb.off_ridx);
  return a;
}

void launch_node(const ContractArgs& a, const NodeBlock& nb, hipStream_t stream) {
  if (nb.kernel == XEB_KERNEL_MFMA) {
    launch_contract_mfma(a, stream);
    if (a.ksplit > 1) launch_splitk_reduce(a, stream);
  } else {
    launch_contract_generic(a, stream);
  }
}

void contract_plan(Plan* p, int64_t b, int64_t e, void* amps, hipStream_t stream) {
  const int64_t total = int64_t(1) << p->s;
  if (b < 0 || e < b || e > total) fail(XEB_EINVAL, "slice range outside [0, 2^s)");
  if (!p->ws) fail(XEB_ESTATE, "no workspace bound");
  if (p->k == 0 || b == e) return;
  if (!amps) fail(XEB_EINVAL, "amps is NULL");
  DeviceGuard g(p->opt.device);
  char* ws = static_cast<char*>(p->ws);
  double2* comp = reinterpret_cast<double2*>(ws + p->off_comp);
  launch_zero(comp, (uint64_t(p->k) << p->w) * 16, stream);
  // Every call starts from its first slice: no table computed by an earlier
  // call is reused, so a call's cost does not depend on its predecessors.
  for (Node& nd : p->nodes) {
    nd.valid = false;
    nd.epoch = 0;
    nd.cur_block = -1;
  }
  const bool fp16 = p->opt.precision == XEB_PREC_SPLIT_FP16;
  const uint64_t amax_words = uint64_t(kAmaxSlots) * kAmaxStride;
  if (fp16) launch_zero(ws + p->off_amax, uint64_t(p->nodes.size()) * amax_words * 8, stream);
  const int L = p->n_leaves;
  // Steps of 2^sj consecutive slices: step c covers slices [c 2^sj, (c + 1) 2^sj)
  // with its low slice keys in the tables' keys; the accumulation keeps the
  // slices inside [b, e).
  const int J = p->sj;
  const int64_t c_begin = b >> J, c_end = ((e - 1) >> J) + 1;
  for (int bi = 0; bi < int(p->blocks.size()); ++bi) {
    const Block& blk = p->blocks[bi];
    for (int64_t sigma = c_begin; sigma < c_end; ++sigma) {
      for (int T = L; T < int(p->nodes.size()); ++T) {
        Node& nd = p->nodes[T];
        const NodeBlock& nb = blk.nodes[T - L];
        const uint64_t key = uint64_t(sigma) & nd.smask;
        if (nd.valid && nd.cur_key == key && (nd.outmask == 0 || nd.cur_block == bi)) continue;
        ContractArgs a = node_args(p, blk, T, sigma);
        if (fp16) a.epoch = ++nd.epoch;
        const double cmacs = double(nb.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
        const double bytes = 8.0 * (double(nvar_in(p, blk, nd.left)) * p->nodes[nd.left].size() +
                                    double(nvar_in(p, blk, nd.right)) * p->nodes[nd.right].size() +
                                    double(nb.nvar) * nd.size());
        if (nb.kernel == XEB_KERNEL_MFMA) {
          timed(p, stream, XEB_KERNEL_MFMA, T, cmacs, bytes,
                [&] { launch_contract_mfma(a, stream); });
          if (a.ksplit > 1) {
            hip_check(hipGetLastError(), "contraction launch");
            int bm = 0, bn = 0;
            mfma_tile_shape(a.tile, &bm, &bn);
            const double partial = 8.0 * double(mfma_tiles(a.tile, a.nvarA << a.mb, a.nvarB << a.nb)) *
                                   bm * bn * (a.ksplit + 2);
            timed(p, stream, XEB_KERNEL_SPLITK, T, 0.0, partial + 8.0 * double(nb.nvar) * nd.size(),
                  [&] { launch_splitk_reduce(a, stream); });
          }
        } else {
          timed(p, stream, XEB_KERNEL_GENERIC, T, cmacs, bytes,
                [&] { launch_contract_generic(a, stream); });
        }
        hip_check(hipGetLastError(), "contraction launch");
        nd.valid = true;
        nd.cur_key = key;
        nd.cur_block = bi;
      }
      const int64_t ng = int64_t(blk.idx.size());
      const double acc_bytes = double(ng) * (4.0 + 8.0 + 2 * 16.0 + 2 * 16.0) +
                               double(blk.rho.size()) * (8.0 + 8.0);
      timed(p, stream, XEB_KERNEL_ACCUMULATE, -1, 0.0, acc_bytes, [&] {
        launch_accumulate(node_ptr(p, p->root, sigma),
                          reinterpret_cast<const int32_t*>(ws + blk.off_idx),
                          reinterpret_cast<const int32_t*>(ws + blk.off_eoff),
                          reinterpret_cast<const int32_t*>(ws + blk.off_rho),
                          reinterpret_cast<const int32_t*>(ws + blk.off_slo), sigma << J, b, e,
                          static_cast<double2*>(amps), comp, ng, p->w, stream);
      });
      hip_check(hipGetLastError(), "accumulate launch");
    }
  }
  launch_fold_compensation(static_cast<double2*>(amps), comp, p->k << p->w, stream);
  hip_check(hipGetLastError(), "fold launch");
}

void launch_plan_xeb(Plan* p, const void* amps, hipStream_t stream) {
  char* ws = static_cast<char*>(p->ws);
  const double2* a = static_cast<const double2*>(amps);
  if (p->w > 0) {
    // Each string's own amplitude: entry (i, open bits of string i).
    double2* own = reinterpret_cast<double2*>(ws + p->off_gather);
    launch_gather_own(a, reinterpret_cast<const int32_t*>(ws + p->off_sel), p->w, own, p->k, stream);
    a = own;
  }
  launch_xeb(a, p->k, p->n_qubits, ws + p->off_scratch, stream);
  hip_check(hipGetLastError(), "xeb launch");
}

double fidelity_plan(Plan* p, const void* amps, hipStream_t stream) {
  if (p->k == 0) fail(XEB_EINVAL, "XEB of an empty batch");
  if (!p->ws) fail(XEB_ESTATE, "no workspace bound");
  if (!amps) fail(XEB_EINVAL, "amps is NULL");
  DeviceGuard g(p->opt.device);
  double* out = reinterpret_cast<double*>(static_cast<char*>(p->ws) + p->off_scratch);
  launch_plan_xeb(p, amps, stream);
  double F = 0.0;
  hip_check(hipMemcpyAsync(&F, out, sizeof(double), hipMemcpyDeviceToHost, stream), "xeb copy");
  hip_check(hipStreamSynchronize(stream), "xeb sync");
  return F;
}

}  // namespace xeb
