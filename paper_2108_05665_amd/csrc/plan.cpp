// Plan compiler and executor of the multi-tensor contraction.
//
// Compilation (host, once per plan):
//  * network of the circuit; output legs and sliced legs are projected into
//    the leaves that carry them, which become variables whose values are the
//    projected tensors (section "Multi-batch simulator"; Appendix A, "Slicing");
//  * the strings are deduplicated; every node gets the distinct keys of its
//    subtree in lexicographic order of (left key, right key), i.e. the order of
//    Appendix C with variables ordered as they occur in the tree, and gather
//    maps to its children's keys.  |keys| is the exact evaluation count |t_T|;
//  * a top-down pass fixes every tensor's leg order so that the legs a node
//    shares with its sibling are the low (contiguous) bits and each parent's
//    kernel writes its result directly in the order its own parent reads;
//  * a dry run of the schedule sizes the device workspace (Appendix C,
//    "emulation mode").
//
// Execution (xeb_contract): slices in increasing order; within one call a
// node is contracted again only when the slice bits it depends on change (its
// table of all string keys stays resident otherwise), which is the single
// cached entry per subtree of the paper's K_L cache applied to slice
// variables; the root's partial amplitudes are added into FP64 with
// compensation.

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

}  // namespace

void compile_plan(Plan& p, const xeb_circuit_t* c, const uint64_t* bits, int64_t k,
                  const xeb_tree_t* tree, const int32_t* sliced, int32_t s,
                  const xeb_options_t* opt) {
  xeb_options_t o;
  xeb_options_default(&o);
  if (opt) o = *opt;
  if (o.precision != XEB_PREC_C64) fail(XEB_EINVAL, "only XEB_PREC_C64 is available");
  if (o.device < 0) fail(XEB_EINVAL, "device ordinal is negative");
  p.opt = o;

  Net net = build_net(c, o.fuse_1q != 0, o.fold_kets != 0);
  const int n = net.n_qubits;
  p.n_qubits = n;

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
  p.s = s;
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
      if (q >= 0)
        nd.outmask |= uint64_t(1) << q;
      else if (slot[leg] >= 0)
        nd.smask |= uint64_t(1) << slot[leg];
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
  if (!p.nodes[p.root].legs.empty()) fail(XEB_EINVAL, "the tree does not close the network");

  // ---- string keys per node (Appendix C: tuples, lexicographic order) ------
  std::vector<uint64_t> ds(bits, bits + k);
  std::sort(ds.begin(), ds.end());
  ds.erase(std::unique(ds.begin(), ds.end()), ds.end());
  const int64_t kd = int64_t(ds.size());
  p.k = k;
  p.kd = kd;
  std::vector<std::vector<int32_t>> var(nn);
  for (int j = 0; j < L; ++j) {
    Node& nd = p.nodes[j];
    std::vector<uint64_t> keys(kd);
    for (int64_t i = 0; i < kd; ++i) keys[i] = pext64(ds[i], nd.outmask);
    std::vector<uint64_t> uk(keys);
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    if (uk.empty()) uk.push_back(0);
    nd.leaf_keys = uk;
    nd.nvar = int64_t(uk.size());
    var[j].resize(kd);
    for (int64_t i = 0; i < kd; ++i)
      var[j][i] = int32_t(std::lower_bound(uk.begin(), uk.end(), keys[i]) - uk.begin());
  }
  for (int T = L; T < nn; ++T) {
    Node& nd = p.nodes[T];
    const int64_t nb_var = p.nodes[nd.right].nvar;
    std::vector<int64_t> codes(kd);
    for (int64_t i = 0; i < kd; ++i) codes[i] = int64_t(var[nd.left][i]) * nb_var + var[nd.right][i];
    std::vector<int64_t> uc(codes);
    std::sort(uc.begin(), uc.end());
    uc.erase(std::unique(uc.begin(), uc.end()), uc.end());
    if (uc.empty()) uc.push_back(0);
    nd.nvar = int64_t(uc.size());
    nd.lidx.resize(nd.nvar);
    nd.ridx.resize(nd.nvar);
    for (int64_t v = 0; v < nd.nvar; ++v) {
      nd.lidx[v] = int32_t(uc[v] / nb_var);
      nd.ridx[v] = int32_t(uc[v] % nb_var);
    }
    var[T].resize(kd);
    for (int64_t i = 0; i < kd; ++i)
      var[T][i] = int32_t(std::lower_bound(uc.begin(), uc.end(), codes[i]) - uc.begin());
    std::vector<int32_t>().swap(var[nd.left]);
    std::vector<int32_t>().swap(var[nd.right]);
  }
  p.rho.resize(k);
  for (int64_t i = 0; i < k; ++i) {
    const int64_t d = std::lower_bound(ds.begin(), ds.end(), bits[i]) - ds.begin();
    p.rho[i] = var[p.root][d];
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
    for (int32_t x : nd.legs) pos[x] = -1;
    a.legs = K;
    a.legs.insert(a.legs.end(), M.begin(), M.end());
    b.legs = K;
    b.legs.insert(b.legs.end(), N.begin(), N.end());
  }

  // ---- kernel per node ------------------------------------------------------
  // MFMA when the stacked GEMM is big enough and its padded tile work stays
  // within 8x the useful MACs; the smaller side supplies the tile rows.
  for (int T = L; T < nn; ++T) {
    Node& nd = p.nodes[T];
    const Node& a = p.nodes[nd.left];
    const Node& b = p.nodes[nd.right];
    const double useful = double(nd.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
    const double rowsL = double(a.nvar) * std::ldexp(1.0, nd.mb);
    const double rowsR = double(b.nvar) * std::ldexp(1.0, nd.nb);
    const double pairs = double(a.nvar) * double(b.nvar);
    nd.swapped = (rowsR < rowsL && rowsR < 64) ? 1 : 0;
    const double rows = nd.swapped ? rowsR : rowsL;
    const double cols = nd.swapped ? rowsL : rowsR;
    nd.tile = rows <= 32 ? 1 : 0;
    int bm = 0, bn = 0;
    mfma_tile_shape(nd.tile, &bm, &bn);
    const double work = std::ceil(rows / bm) * bm * std::ceil(cols / bn) * bn *
                        std::max(std::ldexp(1.0, nd.kb), double(16));
    nd.kernel = XEB_KERNEL_GENERIC;
    if (!o.force_generic && nd.kb >= 1 && rows >= 8 && cols >= 32 && useful >= 65536.0 &&
        8 * useful >= work && pairs <= double(1 << 26)) {
      nd.kernel = XEB_KERNEL_MFMA;
      // Epilogue write order: tile bits sorted by the output position they
      // feed; bits that select variants come last (columns before rows).
      const int kmb = nd.swapped ? nd.nb : nd.mb, knb = nd.swapped ? nd.mb : nd.nb;
      const int8_t* kpm = nd.swapped ? nd.posN : nd.posM;
      const int8_t* kpn = nd.swapped ? nd.posM : nd.posN;
      std::vector<std::pair<int, int>> keyed;  // (key, code)
      for (int j = 0; (1 << j) < bm; ++j) keyed.push_back({j < kmb ? int(kpm[j]) : 2000 + j, j});
      for (int j = 0; (1 << j) < bn; ++j)
        keyed.push_back({j < knb ? int(kpn[j]) : 1000 + j, 32 + j});
      std::sort(keyed.begin(), keyed.end());
      for (size_t b2 = 0; b2 < keyed.size(); ++b2) nd.ubit[b2] = int8_t(keyed[b2].second);
      nd.pair_mode = (nd.nvar == a.nvar * b.nvar) ? 0 : 1;
      if (nd.pair_mode == 1) {
        nd.pairs.assign(size_t(a.nvar * b.nvar), -1);
        for (int64_t v = 0; v < nd.nvar; ++v)
          nd.pairs[size_t(int64_t(nd.lidx[v]) * b.nvar + nd.ridx[v])] = int32_t(v);
      }
    }
  }

  // ---- workspace (dry run) --------------------------------------------------
  // Static region (uploaded at bind): leaf tables, gather maps, rho.
  uint64_t off = 0;
  for (int j = 0; j < L; ++j) {
    Node& nd = p.nodes[j];
    nd.off_table = off;
    off += align_up(uint64_t(nd.nslicekeys) * nd.nvar * nd.size() * 8);
  }
  p.leaf_bytes = off;
  for (int T = L; T < nn; ++T) {
    Node& nd = p.nodes[T];
    if (nd.kernel == XEB_KERNEL_GENERIC) {
      nd.off_lidx = off;
      off += align_up(uint64_t(nd.nvar) * 4);
      nd.off_ridx = off;
      off += align_up(uint64_t(nd.nvar) * 4);
    } else if (nd.pair_mode == 1) {
      nd.off_pairs = off;
      off += align_up(nd.pairs.size() * 4);
    }
  }
  p.off_rho = off;
  off += align_up(uint64_t(k) * 4);
  const uint64_t static_bytes = off;
  // Dynamic region: node tables, compensation, scratch.
  for (int T = L; T < nn; ++T) {
    Node& nd = p.nodes[T];
    nd.off_table = off;
    off += align_up(uint64_t(nd.nvar) * nd.size() * 8);
  }
  p.off_comp = off;
  off += align_up(uint64_t(k) * 16);
  p.off_scratch = off;
  off += kAlign;
  p.ws_bytes = off;
  if (o.memory_budget && p.ws_bytes > o.memory_budget)
    fail(XEB_ENOMEM, "workspace of " + std::to_string(p.ws_bytes) + " bytes exceeds the budget");

  // ---- leaf tables (FP64 -> complex64) --------------------------------------
  p.leaf_staging.assign(static_bytes / 4, 0.f);
  for (int j = 0; j < L; ++j) {
    const Node& nd = p.nodes[j];
    const NetLeaf& nl = net.leaves[j];
    const int R = int(nl.legs.size());
    const int r = int(nd.legs.size());
    std::vector<int> axis_pos(R, -1);  // position in nd.legs, or -1
    for (int a = 0; a < R; ++a)
      for (int q = 0; q < r; ++q)
        if (nd.legs[q] == nl.legs[a]) axis_pos[a] = q;
    float* dst = p.leaf_staging.data() + nd.off_table / 4;
    for (int64_t kappa = 0; kappa < nd.nslicekeys; ++kappa)
      for (int64_t v = 0; v < nd.nvar; ++v)
        for (int64_t e = 0; e < nd.size(); ++e) {
          int64_t idx = 0;
          for (int a = 0; a < R; ++a) {
            const int32_t leg = nl.legs[a];
            int bit;
            if (axis_pos[a] >= 0)
              bit = int((e >> axis_pos[a]) & 1);
            else if (net.leg_qubit[leg] >= 0)
              bit = int((nd.leaf_keys[v] >> rank_in_mask(nd.outmask, net.leg_qubit[leg])) & 1);
            else
              bit = int((kappa >> rank_in_mask(nd.smask, slot[leg])) & 1);
            idx |= int64_t(bit) << (R - 1 - a);
          }
          const cplx x = nl.data[idx];
          const int64_t o2 = ((kappa * nd.nvar + v) * nd.size() + e) * 2;
          dst[o2] = float(x.real());
          dst[o2 + 1] = float(x.imag());
        }
  }
  for (int T = L; T < nn; ++T) {
    const Node& nd = p.nodes[T];
    if (nd.kernel == XEB_KERNEL_GENERIC) {
      std::memcpy(p.leaf_staging.data() + nd.off_lidx / 4, nd.lidx.data(), nd.lidx.size() * 4);
      std::memcpy(p.leaf_staging.data() + nd.off_ridx / 4, nd.ridx.data(), nd.ridx.size() * 4);
    } else if (nd.pair_mode == 1) {
      std::memcpy(p.leaf_staging.data() + nd.off_pairs / 4, nd.pairs.data(), nd.pairs.size() * 4);
    }
  }
  if (k > 0) std::memcpy(p.leaf_staging.data() + p.off_rho / 4, p.rho.data(), size_t(k) * 4);

  // ---- stats -----------------------------------------------------------------
  xeb_stats_t& st = p.stats;
  st = xeb_stats_t{};
  st.n_leaves = L;
  st.n_internal = L - 1;
  st.k = k;
  st.k_distinct = kd;
  st.n_qubits = n;
  st.n_sliced = s;
  for (int T = 0; T < nn; ++T) {
    const Node& nd = p.nodes[T];
    st.max_tensor_elems = std::max<int64_t>(st.max_tensor_elems, nd.size());
    if (nd.leaf) continue;
    const Node& a = p.nodes[nd.left];
    const Node& b = p.nodes[nd.right];
    st.sum_variants += nd.nvar;
    const double cm = double(nd.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
    const double ev = evals_over_all_slices(nd.smask, s);
    st.cmacs_per_slice += cm;
    st.cmacs_full += ev * cm;
    st.rw_elems_full += ev * (double(a.nvar) * a.size() + double(b.nvar) * b.size() +
                              double(nd.nvar) * nd.size());
    st.evals_full += ev;
  }
  st.workspace_bytes = p.ws_bytes;

  if (o.trace > 0) {
    for (int T = L; T < nn; ++T) {
      const Node& nd = p.nodes[T];
      std::fprintf(stderr,
                   "{\"node\":%d,\"left\":%d,\"right\":%d,\"variants\":%lld,\"m_bits\":%d,"
                   "\"n_bits\":%d,\"k_bits\":%d,\"slice_mask\":%llu,\"kernel\":%d}\n",
                   T, nd.left, nd.right, (long long)nd.nvar, nd.mb, nd.nb, nd.kb,
                   (unsigned long long)nd.smask, nd.kernel);
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
  if (!p->leaf_staging.empty())
    hip_check(hipMemcpy(dev, p->leaf_staging.data(), p->leaf_staging.size() * 4,
                        hipMemcpyHostToDevice),
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

// Records an event pair around `launch` when profiling is on.
template <class F>
void timed(Plan* p, hipStream_t stream, int kernel, double cmacs, double bytes, F&& launch) {
  if (!p->profiling) {
    launch();
    return;
  }
  ProfRecord r{take_event(p), take_event(p), kernel, cmacs, bytes};
  hip_check(hipEventRecord(r.start, stream), "hipEventRecord");
  launch();
  hip_check(hipEventRecord(r.stop, stream), "hipEventRecord");
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

xeb_kernel_profile_t read_profile(Plan* p, int kernel) {
  DeviceGuard g(p->opt.device);
  xeb_kernel_profile_t out{};
  for (ProfRecord& r : p->prof) {
    if (r.kernel != kernel) continue;
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

const float2* node_ptr(const Plan* p, int id, int64_t sigma) {
  const Node& nd = p->nodes[id];
  const char* base = static_cast<const char*>(p->ws) + nd.off_table;
  if (nd.leaf) {
    const uint64_t kappa = pext64(uint64_t(sigma), nd.smask);
    base += kappa * uint64_t(nd.nvar) * nd.size() * 8;
  }
  return reinterpret_cast<const float2*>(base);
}

}  // namespace

void contract_plan(Plan* p, int64_t b, int64_t e, void* amps, hipStream_t stream) {
  const int64_t total = int64_t(1) << p->s;
  if (b < 0 || e < b || e > total) fail(XEB_EINVAL, "slice range outside [0, 2^s)");
  if (!p->ws) fail(XEB_ESTATE, "no workspace bound");
  if (p->k == 0 || b == e) return;
  if (!amps) fail(XEB_EINVAL, "amps is NULL");
  DeviceGuard g(p->opt.device);
  char* ws = static_cast<char*>(p->ws);
  double2* comp = reinterpret_cast<double2*>(ws + p->off_comp);
  const int32_t* rho = reinterpret_cast<const int32_t*>(ws + p->off_rho);
  launch_zero(comp, uint64_t(p->k) * 16, stream);
  // Every call starts from its first slice: no table computed by an earlier
  // call is reused, so a call's cost does not depend on its predecessors.
  for (Node& nd : p->nodes) nd.valid = false;
  for (int64_t sigma = b; sigma < e; ++sigma) {
    for (int T = p->n_leaves; T < int(p->nodes.size()); ++T) {
      Node& nd = p->nodes[T];
      const uint64_t key = uint64_t(sigma) & nd.smask;
      if (nd.valid && nd.cur_key == key) continue;
      const Node& na = p->nodes[nd.left];
      const Node& nb = p->nodes[nd.right];
      ContractArgs a{};
      const bool sw = nd.kernel == XEB_KERNEL_MFMA && nd.swapped;
      a.A = node_ptr(p, sw ? nd.right : nd.left, sigma);
      a.B = node_ptr(p, sw ? nd.left : nd.right, sigma);
      a.C = reinterpret_cast<float2*>(ws + nd.off_table);
      a.nvar = nd.nvar;
      a.nvarA = sw ? nb.nvar : na.nvar;
      a.nvarB = sw ? na.nvar : nb.nvar;
      a.mb = sw ? nd.nb : nd.mb;
      a.nb = sw ? nd.mb : nd.nb;
      a.kb = nd.kb;
      a.pair_mode = nd.pair_mode;
      a.swapped = sw ? 1 : 0;
      a.tile = nd.tile;
      std::memcpy(a.posM, sw ? nd.posN : nd.posM, sizeof(a.posM));
      std::memcpy(a.posN, sw ? nd.posM : nd.posN, sizeof(a.posN));
      std::memcpy(a.ubit, nd.ubit, sizeof(a.ubit));
      const double cmacs = double(nd.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
      const double bytes = 8.0 * (double(na.nvar) * na.size() + double(nb.nvar) * nb.size() +
                                  double(nd.nvar) * nd.size());
      if (nd.kernel == XEB_KERNEL_MFMA) {
        a.pairs = nd.pair_mode == 1 ? reinterpret_cast<const int32_t*>(ws + nd.off_pairs) : nullptr;
        timed(p, stream, XEB_KERNEL_MFMA, cmacs, bytes, [&] { launch_contract_mfma(a, stream); });
      } else {
        a.lidx = reinterpret_cast<const int32_t*>(ws + nd.off_lidx);
        a.ridx = reinterpret_cast<const int32_t*>(ws + nd.off_ridx);
        timed(p, stream, XEB_KERNEL_GENERIC, cmacs, bytes,
              [&] { launch_contract_generic(a, stream); });
      }
      hip_check(hipGetLastError(), "contraction launch");
      nd.valid = true;
      nd.cur_key = key;
    }
    const double acc_bytes = double(p->k) * (8.0 + 4.0 + 2 * 16.0 + 2 * 16.0);
    timed(p, stream, XEB_KERNEL_ACCUMULATE, 0.0, acc_bytes, [&] {
      launch_accumulate(node_ptr(p, p->root, sigma), rho, static_cast<double2*>(amps), comp, p->k,
                        stream);
    });
    hip_check(hipGetLastError(), "accumulate launch");
  }
  launch_fold_compensation(static_cast<double2*>(amps), comp, p->k, stream);
  hip_check(hipGetLastError(), "fold launch");
}

double fidelity_plan(Plan* p, const void* amps, hipStream_t stream) {
  if (p->k == 0) fail(XEB_EINVAL, "XEB of an empty batch");
  if (!p->ws) fail(XEB_ESTATE, "no workspace bound");
  if (!amps) fail(XEB_EINVAL, "amps is NULL");
  DeviceGuard g(p->opt.device);
  double* out = reinterpret_cast<double*>(static_cast<char*>(p->ws) + p->off_scratch);
  launch_xeb(static_cast<const double2*>(amps), p->k, p->n_qubits, out, stream);
  hip_check(hipGetLastError(), "xeb launch");
  double F = 0.0;
  hip_check(hipMemcpyAsync(&F, out, sizeof(double), hipMemcpyDeviceToHost, stream), "xeb copy");
  hip_check(hipStreamSynchronize(stream), "xeb sync");
  return F;
}

}  // namespace xeb
