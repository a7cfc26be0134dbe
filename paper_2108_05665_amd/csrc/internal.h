// Internal declarations of the multi-tensor contraction library (host side).
#pragma once

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "xeb.h"

namespace xeb {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

using cplx = std::complex<double>;

// One tensor of the circuit's network.  `data` is row-major over `legs`
// (legs[0] is the slowest axis), every leg of dimension 2.
struct NetLeaf {
  std::vector<int32_t> legs;
  std::vector<cplx> data;
  bool is_ket = false;
};

struct Net {
  int n_qubits = 0;
  int n_legs = 0;
  std::vector<NetLeaf> leaves;
  std::vector<int32_t> leg_qubit;  // q for the output leg of qubit q, else -1
};

// Builds the network of a circuit following the convention documented in
// xeb.h (xeb_network_describe).  Throws Error(XEB_EINVAL) on bad input.
Net build_net(const xeb_circuit_t* c, bool fuse_1q, bool fold_kets);

// Bit helpers on 64-bit masks.
inline uint64_t pext64(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  int b = 0;
  while (mask) {
    uint64_t low = mask & (~mask + 1);
    if (x & low) r |= (uint64_t(1) << b);
    ++b;
    mask &= mask - 1;
  }
  return r;
}

inline int popcount64(uint64_t x) { return __builtin_popcountll(x); }

}  // namespace xeb
