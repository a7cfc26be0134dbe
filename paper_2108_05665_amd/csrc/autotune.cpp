// Autotuner: every kernel configuration a node's contraction can run with
// (per-element kernel; MFMA on each tile shape with either child as the row
// operand and each split-K chunk count) is timed on the bound workspace, at
// the node's real shape and key counts, and the fastest is kept.  The
// timings use whatever the workspace holds (contraction time does not
// depend on the values); the next xeb_contract recomputes every table.

#include <chrono>
#include <cmath>
#include <vector>

#include "plan.h"

namespace xeb {

namespace {

struct Candidate {
  int kernel, tile, swapped, ksplit, tk, kg, keyed;
  bool operator==(const Candidate& o) const {
    return kernel == o.kernel &&
           (kernel == XEB_KERNEL_GENERIC
                ? (tile == o.tile && swapped == o.swapped)
                : (tile == o.tile && swapped == o.swapped && ksplit == o.ksplit && tk == o.tk &&
                   kg == o.kg && keyed == o.keyed));
  }
};

// (Per-element kernel: tile 0 = one thread per output element, tile 1 = the
// row-streaming form with `swapped` naming the stream side.)
constexpr Candidate kGeneric{XEB_KERNEL_GENERIC, 0, 0, 1, 0, 1, 0};

Candidate generic_rows(int stream_l) { return {XEB_KERNEL_GENERIC, 1, stream_l, 1, 0, 1, 0}; }

Candidate current(const NodeBlock& nb) {
  if (nb.kernel == XEB_KERNEL_GENERIC) return {XEB_KERNEL_GENERIC, nb.tile, nb.swapped, 1, 0, 1, 0};
  return {XEB_KERNEL_MFMA, nb.tile, nb.swapped, nb.ksplit, nb.tk, nb.kg, nb.keyed};
}

void apply(const Node& nd, int64_t nl, int64_t nr, NodeBlock& nb, const Candidate& c) {
  if (c.kernel == XEB_KERNEL_GENERIC)
    configure_generic(nb, c.tile, c.swapped);
  else
    configure_mfma(nd, nl, nr, nb, c.tile, c.swapped, c.ksplit, c.tk, c.kg, c.keyed);
}

// Partial-tile bytes a split candidate needs.
uint64_t partial_need(const Node& nd, int64_t nl, int64_t nr, const Candidate& c) {
  if (c.kernel != XEB_KERNEL_MFMA || c.ksplit == 1) return 0;
  int bm = 0, bn = 0;
  mfma_tile_shape(c.tile, &bm, &bn);
  return uint64_t(node_tiles(nd, nl, nr, c.tile, c.swapped)) * c.ksplit * uint64_t(bm) * bn * 8;
}

std::vector<Candidate> candidates(const Plan* p, const Node& nd, int64_t nl, int64_t nr,
                                  const NodeBlock& nb) {
  std::vector<Candidate> out;
  const double useful = double(nb.nvar) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
  // The per-element kernel cannot win on large contractions; leave those out
  // to bound the tuning time.
  if (useful <= std::ldexp(1.0, 30)) out.push_back(kGeneric);
  // (The row-streaming form is HBM-bound at any size.)
  for (int sl = 0; sl < 2; ++sl)
    if (generic_rows_ok(nd, sl)) out.push_back(generic_rows(sl));
  const int64_t K = int64_t(1) << nd.kb;
  // Keyed form: the only MFMA form of a node too sparse to stack, and an
  // alternative to the pair table (which multiplies up to 8x the useful
  // work) where each key fills whole tiles.
  const bool stacked = mfma_capable(nd, nl, nr, nb);
  if (!stacked || nb.nvar != nl * nr) {
    const int lo = mfma_default_slab(p->opt.precision);
    for (int sw = 0; sw < 2; ++sw)
      for (int tile = 0; tile < kMfmaTiles; ++tile) {
        if (!mfma_can_run(nd, nl, nr, nb, tile, sw, 1, 1)) continue;
        if ((tile == 6 || tile == 7) && planes_need(nd, nl, nr) > p->planes_bytes) continue;
        for (int tk = 16; tk <= 2 * lo; tk *= 2)
          for (int kg = 1; kg <= 2; ++kg)
            if (mfma_variant_allowed(tile, p->opt.precision, tk, kg) && !(tk > lo && K < tk) &&
                !(kg > 1 && K < 2 * tk))
              out.push_back({XEB_KERNEL_MFMA, tile, sw, 1, tk, kg, 1});
      }
  }
  if (!stacked) return out;
  // (The 64 x 16 tile serves narrow keyed products only.)
  for (int sw = 0; sw < 2; ++sw) {
    const double rows = double(sw ? nr : nl) * std::ldexp(1.0, sw ? nd.nb : nd.mb);
    const double cols = double(sw ? nl : nr) * std::ldexp(1.0, sw ? nd.mb : nd.nb);
    for (int tile = 0; tile < kMfmaTiles; ++tile) {
      if (tile == 3 || ((tile == 6 || tile == 7) && planes_need(nd, nl, nr) > p->planes_bytes)) continue;
      int bm = 0, bn = 0;
      mfma_tile_shape(tile, &bm, &bn);
      const double padded = std::ceil(rows / bm) * bm * std::ceil(cols / bn) * bn *
                            std::max(double(K), double(mfma_default_slab(p->opt.precision)));
      if (16.0 * useful < padded) continue;  // mostly padding
      const int64_t tiles = node_tiles(nd, nl, nr, tile, sw);
      const int lo = mfma_default_slab(p->opt.precision);
      for (int tk = 16; tk <= 2 * lo; tk *= 2)
        for (int kg = 1; kg <= 2; ++kg) {
          if (!mfma_variant_allowed(tile, p->opt.precision, tk, kg) || (tk > lo && K < tk) ||
              (kg > 1 && K < 2 * tk))
            continue;
          for (int ks = 1; ks <= 64; ks *= 2) {
            if (ks > 1 && (K / ks < 64 || tiles * ks > 2048)) break;
            if (!mfma_can_run(nd, nl, nr, nb, tile, sw, ks, 0)) break;
            const Candidate c{XEB_KERNEL_MFMA, tile, sw, ks, tk, kg, 0};
            if (partial_need(nd, nl, nr, c) > p->partial_bytes) break;
            out.push_back(c);
          }
        }
    }
  }
  return out;
}

}  // namespace

xeb_node_config_t get_node_config(const Plan* p, int T) {
  const NodeBlock& nb = p->blocks.front().nodes[T - p->n_leaves];
  xeb_node_config_t c{};
  c.kernel = nb.kernel;
  if (nb.kernel == XEB_KERNEL_MFMA) {
    c.tile = nb.tile;
    c.swapped = nb.swapped;
    c.ksplit = nb.ksplit;
    c.k_slab = nb.tk;
    c.k_groups = nb.kg;
    c.keyed = nb.pair_mode == 2 ? 1 : 0;
  } else {
    c.tile = nb.tile == 1 ? -2 : -1;
    c.swapped = nb.tile == 1 ? nb.swapped : 0;
    c.ksplit = 1;
    c.k_groups = 1;
  }
  return c;
}

void set_node_config(Plan* p, int T, const xeb_node_config_t& cfg) {
  if (p->capturing) fail(XEB_ESTATE, "cannot change a node while a batch is being captured");
  Candidate c{cfg.kernel, cfg.tile, cfg.swapped, cfg.ksplit, cfg.k_slab, cfg.k_groups, cfg.keyed};
  const Node& nd = p->nodes[T];
  if (c.kernel == XEB_KERNEL_GENERIC) {
    if (cfg.tile == -2) {
      if (cfg.swapped != 0 && cfg.swapped != 1) fail(XEB_EINVAL, "invalid stream side");
      if (!generic_rows_ok(nd, cfg.swapped))
        fail(XEB_EINVAL, "the row-streaming form does not fit the node with that stream side");
      c = generic_rows(cfg.swapped);
    } else {
      c = kGeneric;
    }
  }
  if (c.kernel == XEB_KERNEL_MFMA && c.keyed != 0 && c.keyed != 1) fail(XEB_EINVAL, "keyed must be 0 or 1");
  const int64_t K = int64_t(1) << nd.kb;
  if (c.kernel == XEB_KERNEL_MFMA) {
    if (c.tile < 0 || c.tile >= kMfmaTiles || (c.swapped != 0 && c.swapped != 1))
      fail(XEB_EINVAL, "invalid tile or row operand");
    if (!mfma_variant_allowed(c.tile, p->opt.precision, c.tk, c.kg))
      fail(XEB_EINVAL, "this K slab / K group combination is not built for the tile and precision");
    if (c.ksplit < 1 || c.ksplit > 64 || (c.ksplit & (c.ksplit - 1)) ||
        (c.ksplit > 1 && K % (int64_t(c.ksplit) * c.tk)))
      fail(XEB_EINVAL, "ksplit must be a power of two leaving whole K slabs per chunk");
  } else if (c.kernel != XEB_KERNEL_GENERIC) {
    fail(XEB_EINVAL, "unknown kernel");
  }
  for (const Block& blk : p->blocks) {
    const NodeBlock& nb = blk.nodes[T - p->n_leaves];
    const int64_t nl = nvar_in(p, blk, nd.left), nr = nvar_in(p, blk, nd.right);
    if (c.kernel == XEB_KERNEL_MFMA && !mfma_can_run(nd, nl, nr, nb, c.tile, c.swapped, c.ksplit, c.keyed))
      fail(XEB_EINVAL,
           "the MFMA kernel cannot run the node so (no pair table, or keys smaller than the "
           "tile, or split K on the keyed form)");
    if (partial_need(nd, nl, nr, c) > p->partial_bytes) fail(XEB_EINVAL, "split-K room exceeded");
    if (c.kernel == XEB_KERNEL_MFMA && (c.tile == 6 || c.tile == 7) && planes_need(nd, nl, nr) > p->planes_bytes)
      fail(XEB_EINVAL, "plane-format room exceeded (the node is too large for tile 6)");
  }
  for (Block& blk : p->blocks) {
    const int64_t nl = nvar_in(p, blk, nd.left), nr = nvar_in(p, blk, nd.right);
    apply(nd, nl, nr, blk.nodes[T - p->n_leaves], c);
  }
}

AutotuneReport autotune_plan(Plan* p, int reps, hipStream_t stream) {
  if (!p->ws) fail(XEB_ESTATE, "no workspace bound");
  if (reps < 1 || reps > 1000) fail(XEB_EINVAL, "reps must be in [1, 1000]");
  if (p->capturing) fail(XEB_ESTATE, "cannot autotune while a batch is being captured");
  AutotuneReport rep;
  if (p->k == 0 || p->blocks.empty()) return rep;
  DeviceGuard g(p->opt.device);
  prepare_mfma_launch(p->opt.precision);
  const auto t0 = std::chrono::steady_clock::now();
  char* ws = static_cast<char*>(p->ws);
  const bool fp16 = p->opt.precision == XEB_PREC_SPLIT_FP16;
  // Defined FP16 scales for the timing launches (the tables hold anything).
  if (fp16)
    launch_zero(ws + p->off_amax, uint64_t(p->nodes.size()) * kAmaxSlots * kAmaxStride * 8, stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } events{e0, e1};

  const int L = p->n_leaves;
  const int nn = int(p->nodes.size());
  Block& blk0 = p->blocks.front();
  std::vector<Candidate> chosen(nn, kGeneric);
  for (int T = L; T < nn; ++T) {
    const Node& nd = p->nodes[T];
    NodeBlock& nb = blk0.nodes[T - L];
    const int64_t nl = nvar_in(p, blk0, nd.left), nr = nvar_in(p, blk0, nd.right);
    const Candidate def = current(nb);
    std::vector<Candidate> cands = candidates(p, nd, nl, nr, nb);
    bool has_def = false;
    for (const Candidate& c : cands) has_def = has_def || c == def;
    if (!has_def) cands.push_back(def);
    double best_t = 0, def_t = 0;
    Candidate best = def;
    for (size_t i = 0; i < cands.size(); ++i) {
      const Candidate& c = cands[i];
      apply(nd, nl, nr, nb, c);
      ContractArgs a = node_args(p, blk0, T, 0);
      a.epoch = 1;
      launch_node(a, nb, stream);  // warm-up
      hip_check(hipEventRecord(e0, stream), "hipEventRecord");
      for (int r = 0; r < reps; ++r) launch_node(a, nb, stream);
      hip_check(hipEventRecord(e1, stream), "hipEventRecord");
      hip_check(hipGetLastError(), "autotune launch");
      hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      const double t = 1e-3 * double(ms) / reps;
      ++rep.candidates;
      if (c == def) def_t = t;
      if (i == 0 || t < best_t) {
        best_t = t;
        best = c;
      }
    }
    apply(nd, nl, nr, nb, best);
    chosen[T] = best;
    ++rep.nodes_tuned;
    if (!(best == def)) ++rep.nodes_changed;
    const double ev = evals_per_call(p, T);
    rep.default_seconds += def_t * ev;
    rep.tuned_seconds += best_t * ev;
  }
  // Later string blocks take the first block's choice where they can run it
  // (the key counts differ between blocks, the node shapes do not).
  for (size_t bi = 1; bi < p->blocks.size(); ++bi) {
    Block& blk = p->blocks[bi];
    for (int T = L; T < nn; ++T) {
      const Node& nd = p->nodes[T];
      NodeBlock& nb = blk.nodes[T - L];
      const int64_t nl = nvar_in(p, blk, nd.left), nr = nvar_in(p, blk, nd.right);
      Candidate c = chosen[T];
      if (c.kernel == XEB_KERNEL_MFMA && !mfma_can_run(nd, nl, nr, nb, c.tile, c.swapped, c.ksplit, c.keyed))
        c = kGeneric;
      if (c.kernel == XEB_KERNEL_MFMA && partial_need(nd, nl, nr, c) > p->partial_bytes) c.ksplit = 1;
      if (c.kernel == XEB_KERNEL_MFMA && (c.tile == 6 || c.tile == 7) && planes_need(nd, nl, nr) > p->planes_bytes)
        c = kGeneric;
      apply(nd, nl, nr, nb, c);
    }
  }
  rep.tuning_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (Node& nd : p->nodes) nd.valid = false;
  return rep;
}

}  // namespace xeb
