// Circuit -> tensor network (section "Multi-batch simulator": one open leg
// per qubit, gate fusion already applied, kets folded into first gates).
// The convention is the one documented at xeb_network_describe in xeb.h.

#include <array>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace xeb {
namespace {

using Mat2 = std::array<cplx, 4>;   // row-major [out][in]
using Mat4 = std::array<cplx, 16>;  // row-major [out][in], index 2*b_q0 + b_q1

struct Emitted {
  int q0, q1;  // q1 = -1: one-qubit gate
  Mat4 u;      // one-qubit gates use u[0..3] as a 2x2
};

Mat2 mul2(const Mat2& a, const Mat2& b) {
  Mat2 r{};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r[i * 2 + j] = a[i * 2] * b[j] + a[i * 2 + 1] * b[2 + j];
  return r;
}

Mat4 mul4(const Mat4& a, const Mat4& b) {
  Mat4 r{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int t = 0; t < 4; ++t) s += a[i * 4 + t] * b[t * 4 + j];
      r[i * 4 + j] = s;
    }
  return r;
}

// (x (x) y) with x acting on the first qubit (the high basis bit).
Mat4 kron2(const Mat2& x, const Mat2& y) {
  Mat4 r{};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) r[(2 * a + b) * 4 + (2 * c + d)] = x[a * 2 + c] * y[b * 2 + d];
  return r;
}

const Mat2 kEye2 = {cplx(1), cplx(0), cplx(0), cplx(1)};

std::vector<Emitted> emit_gates(const xeb_circuit_t* c, bool fuse) {
  const int n = c->n_qubits;
  std::vector<Emitted> out;
  out.reserve(c->n_gates);
  auto read_gate = [&](int g, bool two, Mat4& m) {
    const double* p = c->gate_mats + size_t(g) * 32;
    const int cnt = two ? 16 : 4;
    m.fill(cplx(0));
    for (int e = 0; e < cnt; ++e) {
      double re = p[2 * e], im = p[2 * e + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) fail(XEB_EINVAL, "gate matrix has a non-finite entry");
      m[e] = cplx(re, im);
    }
  };
  if (!fuse) {
    for (int g = 0; g < c->n_gates; ++g) {
      Emitted e;
      e.q0 = c->gate_qubits[2 * g];
      e.q1 = c->gate_qubits[2 * g + 1];
      read_gate(g, e.q1 >= 0, e.u);
      out.push_back(e);
    }
    return out;
  }
  std::vector<Mat2> pend(n, kEye2);
  std::vector<char> has(n, 0);
  std::vector<int> last_two(n, -1);
  for (int g = 0; g < c->n_gates; ++g) {
    const int a = c->gate_qubits[2 * g], b = c->gate_qubits[2 * g + 1];
    Mat4 m;
    read_gate(g, b >= 0, m);
    if (b < 0) {
      Mat2 u = {m[0], m[1], m[2], m[3]};
      pend[a] = has[a] ? mul2(u, pend[a]) : u;
      has[a] = 1;
      continue;
    }
    Emitted e;
    e.q0 = a;
    e.q1 = b;
    e.u = mul4(m, kron2(has[a] ? pend[a] : kEye2, has[b] ? pend[b] : kEye2));
    has[a] = has[b] = 0;
    pend[a] = pend[b] = kEye2;
    out.push_back(e);
    last_two[a] = last_two[b] = int(out.size()) - 1;
  }
  for (int q = 0; q < n; ++q) {
    if (!has[q]) continue;
    if (last_two[q] >= 0) {
      Emitted& e = out[last_two[q]];
      Mat4 side = (q == e.q0) ? kron2(pend[q], kEye2) : kron2(kEye2, pend[q]);
      e.u = mul4(side, e.u);
    } else {
      Emitted e;
      e.q0 = q;
      e.q1 = -1;
      e.u.fill(cplx(0));
      for (int t = 0; t < 4; ++t) e.u[t] = pend[q][t];
      out.push_back(e);
    }
  }
  return out;
}

}  // namespace

Net build_net(const xeb_circuit_t* c, bool fuse_1q, bool fold_kets) {
  if (!c) fail(XEB_EINVAL, "circuit is NULL");
  if (c->n_qubits < 1 || c->n_qubits > 64) fail(XEB_EINVAL, "n_qubits must be in [1, 64]");
  if (c->n_gates < 0) fail(XEB_EINVAL, "n_gates is negative");
  if (c->n_gates > 0 && (!c->gate_qubits || !c->gate_mats)) fail(XEB_EINVAL, "gate arrays are NULL");
  const int n = c->n_qubits;
  for (int g = 0; g < c->n_gates; ++g) {
    const int a = c->gate_qubits[2 * g], b = c->gate_qubits[2 * g + 1];
    if (a < 0 || a >= n) fail(XEB_EINVAL, "gate " + std::to_string(g) + ": qubit out of range");
    if (b < -1 || b >= n || b == a) fail(XEB_EINVAL, "gate " + std::to_string(g) + ": bad second qubit");
  }
  std::vector<Emitted> gates = emit_gates(c, fuse_1q);

  std::vector<char> touched(n, 0);
  for (const Emitted& e : gates) {
    touched[e.q0] = 1;
    if (e.q1 >= 0) touched[e.q1] = 1;
  }
  Net net;
  net.n_qubits = n;
  std::vector<int32_t> wire(n, -1);  // -1: still the initial |0>, folded
  int next_leg = 0;
  for (int q = 0; q < n; ++q) {
    if (fold_kets && touched[q]) continue;
    NetLeaf k;
    k.is_ket = true;
    k.legs = {next_leg};
    k.data = {cplx(1), cplx(0)};
    wire[q] = next_leg++;
    net.leaves.push_back(std::move(k));
  }
  for (const Emitted& e : gates) {
    const int nq = e.q1 >= 0 ? 2 : 1;
    const int qs[2] = {e.q0, e.q1};
    NetLeaf lf;
    bool in_open[2] = {false, false};
    for (int j = 0; j < nq; ++j) {
      if (wire[qs[j]] >= 0) {
        lf.legs.push_back(wire[qs[j]]);
        in_open[j] = true;
      }
    }
    const int n_in = int(lf.legs.size());
    for (int j = 0; j < nq; ++j) {
      wire[qs[j]] = next_leg;
      lf.legs.push_back(next_leg++);
    }
    const int r = n_in + nq;
    lf.data.assign(size_t(1) << r, cplx(0));
    // Enumerate (inputs, outputs); a folded input is fixed to 0.
    for (int idx = 0; idx < (1 << r); ++idx) {
      int bits[4];
      for (int a = 0; a < r; ++a) bits[a] = (idx >> (r - 1 - a)) & 1;
      int in_b[2] = {0, 0}, out_b[2] = {0, 0};
      int p = 0;
      for (int j = 0; j < nq; ++j)
        if (in_open[j]) in_b[j] = bits[p++];
      for (int j = 0; j < nq; ++j) out_b[j] = bits[p++];
      cplx v;
      if (nq == 2)
        v = e.u[(2 * out_b[0] + out_b[1]) * 4 + (2 * in_b[0] + in_b[1])];
      else
        v = e.u[out_b[0] * 2 + in_b[0]];
      lf.data[idx] = v;
    }
    net.leaves.push_back(std::move(lf));
  }
  net.n_legs = next_leg;
  net.leg_qubit.assign(next_leg, -1);
  for (int q = 0; q < n; ++q) net.leg_qubit[wire[q]] = q;
  return net;
}

}  // namespace xeb
