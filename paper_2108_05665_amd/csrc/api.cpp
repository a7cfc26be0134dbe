// C ABI entry points (xeb.h): argument checks, error capture, no exceptions
// across the boundary.

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plan.h"
#include "xeb.h"

namespace {

thread_local std::string g_last_error = "no error";

template <class F>
int guarded(F&& f) {
  try {
    f();
    g_last_error = "no error";
    return XEB_OK;
  } catch (const xeb::Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return XEB_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return XEB_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return XEB_EINVAL;
  }
}

xeb::Plan& impl(xeb_plan_t p) {
  if (!p) xeb::fail(XEB_EINVAL, "plan handle is NULL");
  return p->impl;
}

}  // namespace

extern "C" {

void xeb_options_default(xeb_options_t* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->fuse_1q = 1;
  opt->fold_kets = 1;
  opt->precision = XEB_PREC_C64;
  opt->device = 0;
  opt->memory_budget = 0;
  opt->trace = 0;
  opt->force_generic = 0;
  opt->max_ksplit = 0;
  opt->mfma_min_cmacs = 0.0;
}

const char* xeb_last_error(void) { return g_last_error.c_str(); }

int xeb_network_describe(const xeb_circuit_t* circuit, int32_t fuse_1q, int32_t fold_kets,
                         int32_t* n_leaves, int32_t* n_legs, int32_t* n_leaf_legs,
                         int32_t* leaf_leg_offsets, int32_t* leaf_legs, int32_t* leg_qubit) {
  return guarded([&] {
    xeb::Net net = xeb::build_net(circuit, fuse_1q != 0, fold_kets != 0);
    int32_t total = 0;
    for (const auto& lf : net.leaves) total += int32_t(lf.legs.size());
    if (n_leaves) *n_leaves = int32_t(net.leaves.size());
    if (n_legs) *n_legs = net.n_legs;
    if (n_leaf_legs) *n_leaf_legs = total;
    if (leaf_leg_offsets) {
      int32_t o = 0;
      for (size_t j = 0; j < net.leaves.size(); ++j) {
        leaf_leg_offsets[j] = o;
        o += int32_t(net.leaves[j].legs.size());
      }
      leaf_leg_offsets[net.leaves.size()] = o;
    }
    if (leaf_legs) {
      int32_t o = 0;
      for (const auto& lf : net.leaves)
        for (int32_t l : lf.legs) leaf_legs[o++] = l;
    }
    if (leg_qubit)
      for (int l = 0; l < net.n_legs; ++l) leg_qubit[l] = net.leg_qubit[l];
  });
}

int xeb_plan_create(const xeb_circuit_t* circuit, const uint64_t* bitstrings, int64_t k,
                    const xeb_tree_t* contraction_tree, const int32_t* sliced_legs, int32_t s,
                    const xeb_options_t* opt, xeb_plan_t* out) {
  return guarded([&] {
    if (!out) xeb::fail(XEB_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    xeb_plan* p = new xeb_plan();
    try {
      xeb::compile_plan(p->impl, circuit, bitstrings, k, contraction_tree, sliced_legs, s, opt);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

int xeb_plan_workspace_bytes(xeb_plan_t plan, uint64_t* bytes) {
  return guarded([&] {
    xeb::Plan& p = impl(plan);
    if (!bytes) xeb::fail(XEB_EINVAL, "bytes is NULL");
    *bytes = p.ws_bytes;
  });
}

int xeb_plan_bind_workspace(xeb_plan_t plan, void* dev_ptr, uint64_t bytes) {
  return guarded([&] { xeb::bind_plan(&impl(plan), dev_ptr, bytes); });
}

int xeb_contract(xeb_plan_t plan, int64_t slice_begin, int64_t slice_end, void* amps,
                 void* stream) {
  return guarded([&] {
    xeb::Plan& p = impl(plan);
    // Injected abort: contract the slices left before the limit, then stop.
    int64_t stop = slice_end;
    if (p.opt.abort_after_slices > 0 && slice_begin >= 0 && slice_end >= slice_begin) {
      const int64_t left = std::max<int64_t>(p.opt.abort_after_slices - p.slices_done, 0);
      if (slice_end - slice_begin > left) stop = slice_begin + left;
    }
    xeb::contract_plan(&p, slice_begin, stop, amps, static_cast<hipStream_t>(stream));
    p.slices_done += stop - slice_begin;
    if (stop < slice_end)
      xeb::fail(XEB_EABORT, "injected abort after " + std::to_string(p.slices_done) +
                                " slices: [" + std::to_string(slice_begin) + ", " + std::to_string(stop) +
                                ") are in amps; resume at slice " + std::to_string(stop));
  });
}

int xeb_plan_get_node_config(xeb_plan_t plan, int32_t node, xeb_node_config_t* out) {
  return guarded([&] {
    xeb::Plan& p = impl(plan);
    if (!out) xeb::fail(XEB_EINVAL, "out is NULL");
    if (node < p.n_leaves || node >= int32_t(p.nodes.size())) xeb::fail(XEB_EINVAL, "not an internal node");
    *out = xeb::get_node_config(&p, node);
  });
}

int xeb_plan_set_node_config(xeb_plan_t plan, int32_t node, const xeb_node_config_t* config) {
  return guarded([&] {
    xeb::Plan& p = impl(plan);
    if (!config) xeb::fail(XEB_EINVAL, "config is NULL");
    if (node < p.n_leaves || node >= int32_t(p.nodes.size())) xeb::fail(XEB_EINVAL, "not an internal node");
    xeb::set_node_config(&p, node, *config);
  });
}

int xeb_plan_autotune(xeb_plan_t plan, int32_t reps, void* stream, xeb_autotune_report_t* report) {
  return guarded([&] {
    const xeb::AutotuneReport r =
        xeb::autotune_plan(&impl(plan), reps, static_cast<hipStream_t>(stream));
    if (report) {
      report->nodes_tuned = r.nodes_tuned;
      report->nodes_changed = r.nodes_changed;
      report->candidates = r.candidates;
      report->default_seconds = r.default_seconds;
      report->tuned_seconds = r.tuned_seconds;
      report->tuning_seconds = r.tuning_seconds;
    }
  });
}

int xeb_fidelity(xeb_plan_t plan, const void* amps, void* stream, double* F) {
  return guarded([&] {
    if (!F) xeb::fail(XEB_EINVAL, "F is NULL");
    *F = xeb::fidelity_plan(&impl(plan), amps, static_cast<hipStream_t>(stream));
  });
}

static_assert(XEB_NOALLOC_MAX_STRINGS == xeb::kXebStaticMaxStrings, "allocation-free XEB limit");

int xeb_fidelity_noalloc(const void* amps, int64_t k, int32_t n_qubits, double* F, void* stream) {
  return guarded([&] {
    xeb::launch_xeb_static(static_cast<const double2*>(amps), k, n_qubits, F,
                           static_cast<hipStream_t>(stream));
  });
}

int xeb_plan_stats(xeb_plan_t plan, xeb_stats_t* stats) {
  return guarded([&] {
    if (!stats) xeb::fail(XEB_EINVAL, "stats is NULL");
    *stats = impl(plan).stats;
    stats->slices_done = impl(plan).slices_done;
  });
}

int xeb_plan_node_stats(xeb_plan_t plan, int32_t node, xeb_node_stats_t* st) {
  return guarded([&] {
    xeb::Plan& p = impl(plan);
    if (!st) xeb::fail(XEB_EINVAL, "stats is NULL");
    if (node < p.n_leaves || node >= int32_t(p.nodes.size()))
      xeb::fail(XEB_EINVAL, "node is not an internal node id");
    const xeb::Node& nd = p.nodes[node];
    std::memset(st, 0, sizeof(*st));
    st->left = nd.left;
    st->right = nd.right;
    auto keys = [&](int id) -> int64_t {
      if (p.nodes[id].leaf) return p.nodes[id].leaf_nvar * int64_t(p.blocks.size());
      int64_t t = 0;
      for (const xeb::Block& b : p.blocks) t += b.nodes[id - p.n_leaves].nvar;
      return t;
    };
    st->variants = keys(node);
    st->left_variants = keys(nd.left);
    st->right_variants = keys(nd.right);
    st->m_bits = nd.mb;
    st->n_bits = nd.nb;
    st->k_bits = nd.kb;
    // Slice-id numbering: looped bits above the stacked ones, stacked bits
    // from the key bits n .. n + sj - 1.
    const uint64_t stacked = p.sj > 0 ? (nd.outmask >> p.n_qubits) & ((uint64_t(1) << p.sj) - 1) : 0;
    st->slice_mask = (nd.smask << p.sj) | stacked;
    const xeb::NodeBlock& nb = p.blocks.front().nodes[node - p.n_leaves];
    st->kernel = nb.kernel;
    st->swapped = nb.kernel == XEB_KERNEL_MFMA || nb.tile == 1 ? nb.swapped : 0;
    st->tile = nb.kernel == XEB_KERNEL_MFMA ? nb.tile : (nb.tile == 1 ? -2 : -1);
    st->ksplit = nb.kernel == XEB_KERNEL_MFMA ? nb.ksplit : 1;
    st->k_slab = nb.kernel == XEB_KERNEL_MFMA ? nb.tk : 0;
    st->k_groups = nb.kernel == XEB_KERNEL_MFMA ? nb.kg : 0;
    st->pair_mode = nb.kernel == XEB_KERNEL_MFMA ? nb.pair_mode : 0;
    st->cmacs_per_eval = double(st->variants) * std::ldexp(1.0, nd.mb + nd.nb + nd.kb);
  });
}

int xeb_plan_set_profiling(xeb_plan_t plan, int32_t enable) {
  return guarded([&] { xeb::set_profiling(&impl(plan), enable != 0); });
}

int xeb_plan_read_profile(xeb_plan_t plan, int32_t kernel, xeb_kernel_profile_t* out) {
  return guarded([&] {
    if (!out) xeb::fail(XEB_EINVAL, "out is NULL");
    if (kernel < 0 || kernel > XEB_KERNEL_SPLITK) xeb::fail(XEB_EINVAL, "unknown kernel class");
    *out = xeb::read_profile(&impl(plan), kernel, -1);
  });
}

int xeb_plan_read_node_profile(xeb_plan_t plan, int32_t node, xeb_kernel_profile_t* out) {
  return guarded([&] {
    xeb::Plan& p = impl(plan);
    if (!out) xeb::fail(XEB_EINVAL, "out is NULL");
    if (node < p.n_leaves || node >= int32_t(p.nodes.size()))
      xeb::fail(XEB_EINVAL, "node is not an internal node id");
    *out = xeb::read_profile(&p, -1, node);
  });
}

int xeb_batch_create(const xeb_plan_t* plans, void* const* amps, int32_t n, xeb_batch_t* out) {
  return guarded([&] {
    if (!out) xeb::fail(XEB_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    if (!plans || n < 1) xeb::fail(XEB_EINVAL, "a batch needs at least one plan");
    std::vector<xeb::Plan*> ps(n);
    for (int i = 0; i < n; ++i) ps[i] = &impl(plans[i]);
    xeb_batch* b = new xeb_batch();
    try {
      b->impl = xeb::create_batch(ps.data(), amps, n);
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
  });
}

int xeb_batch_contract(xeb_batch_t batch, void* stream) {
  return guarded([&] {
    if (!batch) xeb::fail(XEB_EINVAL, "batch handle is NULL");
    xeb::launch_batch(batch->impl, static_cast<hipStream_t>(stream));
  });
}

int xeb_batch_fidelities(xeb_batch_t batch, void* stream, double* F) {
  return guarded([&] {
    if (!batch) xeb::fail(XEB_EINVAL, "batch handle is NULL");
    xeb::batch_fidelities(batch->impl, static_cast<hipStream_t>(stream), F);
  });
}

int xeb_batch_destroy(xeb_batch_t batch) {
  return guarded([&] {
    if (batch) xeb::destroy_batch(batch->impl);
    delete batch;
  });
}

int xeb_plan_destroy(xeb_plan_t plan) {
  return guarded([&] { delete plan; });
}

}  // extern "C"
