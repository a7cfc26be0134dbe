// gfx950 kernels of the multi-tensor contraction.
//
// * contract_generic: one thread per output element of every variant; the
//   path for small or sparse nodes (latency-bound).
// * contract_mfma (complex64 on FP32 MFMA) and contract_split (hi/lo
//   FP16 / BF16 on 16-bit MFMA): the variants of L stacked as rows
//   (nvarA * 2^mb rows of 2^kb complex) times the variants of R stacked as
//   rows, or, for key sets too sparse to stack, one product per key.  The
//   epilogue scatters each output element straight into the layout the
//   parent node reads (bit deposit), so no separate transpose pass exists.
// * splitk_sum / splitk_reduce: the chunk sum of split-K nodes.
// * accumulate / fold_compensation: FP64 Neumaier sum over slices.
// (The XEB reduction lives in fidelity.hip.)

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>

#include "compensated.h"
#include "kernels.h"

namespace xeb {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Bit deposit (PDEP): the low bits of x go, lowest first, to the set bit
// positions of map.mask; the expand steps of the move-mask method.
__device__ __forceinline__ int64_t deposit(uint64_t x, const BitMap& map) {
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    const uint64_t t = x << (1 << i);
    x = (x & ~map.mv[i]) | (t & map.mv[i]);
  }
  return int64_t(x & map.mask);
}

// ---------------------------------------------------------------------------
// Generic contraction.
// Largest |re|, |im| of a wave's values -> one atomicMax per wave on
// (epoch << 32) | float bits (non-negative floats order like their bits; a
// later evaluation's larger epoch replaces older values).
// Workgroup-wide maximum of v published into the workgroup's slot (called by
// all 256 threads).
__device__ __forceinline__ void publish_amax(float v, unsigned long long* slots, uint32_t epoch) {
  __shared__ float wmax[8];  // up to 512 threads
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (unsigned w = 0; w < (blockDim.x >> 6); ++w) m = fmaxf(m, wmax[w]);
    atomicMax(slots + (blockIdx.x % kAmaxSlots) * kAmaxStride,
              (static_cast<unsigned long long>(epoch) << 32) | __float_as_uint(m));
  }
}

// Bits of x at positions pos[0..bits) gathered into the low bits (the inverse
// of deposit).
// Bit extract (PEXT): the bits of x at the set positions of map.mask,
// gathered to the bottom; the compress steps of the move-mask method.
__device__ __forceinline__ int64_t extract(uint64_t x, const BitMap& map) {
  x &= map.mask;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint64_t t = x & map.mv[i];
    x = (x ^ t) | (t >> (1 << i));
  }
  return int64_t(x);
}

constexpr int kGenericLog2U = 2;  // outputs per thread in a chunk: 4

// A wave-uniform int32 read through the scalar cache (the index is made
// uniform with readfirstlane by the caller).
__device__ __forceinline__ uint32_t load_uniform(const int32_t* p) {
  return *(const __attribute__((address_space(4))) uint32_t*)p;
}

// Complex dot product of two rows of K = 2^kb complex (runtime K).
__device__ __forceinline__ float2 dot_rows(const float2* pa, const float2* pb, int kb) {
  float re = 0.f, im = 0.f;
  if (kb >= 1) {
    const float4* qa = reinterpret_cast<const float4*>(pa);
    const float4* qb = reinterpret_cast<const float4*>(pb);
    const int kv = 1 << (kb - 1);
#pragma unroll 4
    for (int k = 0; k < kv; ++k) {
      const float4 x = qa[k], y = qb[k];
      re += x.x * y.x - x.y * y.y;
      im += x.x * y.y + x.y * y.x;
      re += x.z * y.z - x.w * y.w;
      im += x.z * y.w + x.w * y.z;
    }
  } else {
    const float2 x = pa[0], y = pb[0];
    re = x.x * y.x - x.y * y.y;
    im = x.x * y.y + x.y * y.x;
  }
  return make_float2(re, im);
}

// Dot products of U row pairs at once, K = 2^KB complex (KB < 0: runtime
// kb).  The loads of all U rows for a step of up to two float4 per row are
// issued before any of them is used, so one thread keeps up to 4 U loads in
// flight; each element sums its K terms in ascending k.
template <int U, int KB>
__device__ __forceinline__ void dot_rows_u(const float2* const* pa, const float2* const* pb,
                                           int kb, float2* out) {
  float re[U], im[U];
#pragma unroll
  for (int u = 0; u < U; ++u) re[u] = im[u] = 0.f;
  if constexpr (KB == 0) {
    float2 x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = pa[u][0];
      y[u] = pb[u][0];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the first use
#pragma unroll
    for (int u = 0; u < U; ++u) {
      re[u] = x[u].x * y[u].x - x[u].y * y[u].y;
      im[u] = x[u].x * y[u].y + x[u].y * y[u].x;
    }
  } else {
    const int kv = KB > 0 ? (1 << (KB - 1)) : (1 << (kb - 1));  // float4 per row
    constexpr int STEP = KB == 1 ? 1 : 2;
#pragma unroll
    for (int k = 0; k < (KB > 0 ? (1 << (KB - 1)) : kv); k += STEP) {
      float4 x[U][STEP], y[U][STEP];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < STEP; ++j) {
          x[u][j] = reinterpret_cast<const float4*>(pa[u])[k + j];
          y[u][j] = reinterpret_cast<const float4*>(pb[u])[k + j];
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < STEP; ++j) {
          re[u] += x[u][j].x * y[u][j].x - x[u][j].y * y[u][j].y;
          im[u] += x[u][j].x * y[u][j].y + x[u][j].y * y[u][j].x;
          re[u] += x[u][j].z * y[u][j].z - x[u][j].w * y[u][j].w;
          im[u] += x[u][j].z * y[u][j].w + x[u][j].w * y[u][j].z;
        }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) out[u] = make_float2(re[u], im[u]);
}

// Chunks of 256 * U consecutive output elements (a key's table spans whole
// chunks): thread t takes positions t + 256 u, u < U.  A position's row and
// column bits split by bit range: the thread id's 8 bits (once per thread),
// u's bits (once per thread, U values), and the chunk's high bits (once per
// chunk, wave-uniform).  The chunk's key and its operand variants are
// uniform (scalar loads).
template <int U, int KB>
__device__ __forceinline__ void generic_chunks(const ContractArgs& g, float& amax) {
  const int mn = g.mb + g.nb;
  const int64_t per = int64_t(1) << mn;
  const int64_t chunks = (g.nvar * per) / (256 * U);
  const int kb = KB >= 0 ? KB : g.kb;
  const int64_t sizeA = int64_t(1) << (g.mb + kb);
  const int64_t sizeB = int64_t(1) << (g.nb + kb);
  const int64_t m_lo = extract(threadIdx.x, g.mapM);
  const int64_t n_lo = extract(threadIdx.x, g.mapN);
  int64_t m_u[U], n_u[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    m_u[u] = extract(int64_t(u) << 8, g.mapM) | m_lo;
    n_u[u] = extract(int64_t(u) << 8, g.mapN) | n_lo;
  }
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t e0 = c * (256 * U);
    const int a = __builtin_amdgcn_readfirstlane(int(e0 >> mn));
    // (Variant numbers are non-negative: zero extension.)
    const uint32_t la = load_uniform(g.lidx + a), ra = load_uniform(g.ridx + a);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t o_hi = e0 & (per - 1);
    const int64_t m_hi = extract(o_hi, g.mapM), n_hi = extract(o_hi, g.mapN);
    const float2* A = g.A + uint64_t(la) * sizeA;
    const float2* B = g.B + uint64_t(ra) * sizeB;
    const float2* pa[U];
    const float2* pb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pa[u] = A + ((m_hi | m_u[u]) << kb);
      pb[u] = B + ((n_hi | n_u[u]) << kb);
    }
    float2 v[U];
    dot_rows_u<U, KB>(pa, pb, kb, v);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      g.C[e0 + (u << 8) + threadIdx.x] = v[u];
      amax = fmaxf(amax, fmaxf(fabsf(v[u].x), fabsf(v[u].y)));
    }
  }
}

// Threads walk the output table in its own element order (coalesced stores);
// each finds the row m and column n its element deposits from.  Extraction is
// linear over disjoint bit sets, so when a key's table spans at least one
// 256-element chunk the thread id's 8 low position bits are extracted once per
// thread and the chunk's high bits once per chunk (wave-uniform).  KB is the
// contracted dimension's bit count when it is small (the dot products unroll
// fully), -1 otherwise.
template <int KB>
__global__ void __launch_bounds__(256) k_contract_generic(ContractArgs g) {
  float amax = 0.f;
  const int mn = g.mb + g.nb;
  if (mn >= 8 + kGenericLog2U) {
    generic_chunks<1 << kGenericLog2U, KB>(g, amax);
  } else if (mn >= 8) {
    generic_chunks<1, KB>(g, amax);
  } else {
    const int64_t per = int64_t(1) << mn;
    const int64_t total = g.nvar * per;
    const int64_t sizeA = int64_t(1) << (g.mb + g.kb);
    const int64_t sizeB = int64_t(1) << (g.nb + g.kb);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
      const int64_t a = e >> mn;
      const int64_t o = e & (per - 1);
      const int64_t m = extract(o, g.mapM);
      const int64_t n = extract(o, g.mapN);
      const float2 v = dot_rows(g.A + int64_t(g.lidx[a]) * sizeA + (m << g.kb),
                                g.B + int64_t(g.ridx[a]) * sizeB + (n << g.kb), g.kb);
      g.C[e] = v;
      amax = fmaxf(amax, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
}

// Row-streaming form of the per-element contraction, for a short contracted
// leg (K = 2^KB <= 16) between a wide side (the stream side, >= 8 bits) and a
// narrow one (the broadcast side, <= 6 bits).  A work item is one key and
// 256 U consecutive stream rows: each thread loads its U rows of K complex
// once into registers; the workgroup stages the key's 2^bb broadcast rows in
// LDS (at most 64 x 16 complex), and every thread walks them (same address
// across the wave: broadcast reads), storing one output per (row, b).  The
// per-element form instead loads both K-long rows for every output element,
// which makes it bound by the vector cache rather than by HBM.  (Reading the
// broadcast rows through scalar loads instead measured 3-9 % slower: each
// row's loads stalled the wave right before their use.)  Items run key
// fastest, so the keys that share a stream variant read its rows together.
// g.swapped: 0 = the stream side is R (columns n), 1 = it is L (rows m).
template <int KB, int U>
__global__ void __launch_bounds__(256) k_contract_rows(ContractArgs g) {
  constexpr int K = 1 << KB;
  __shared__ float2 bsh[64 * K];  // the item's broadcast rows
  float amax = 0.f;
  const bool sm = g.swapped != 0;
  const float2* S = sm ? g.A : g.B;
  const float2* Bc = sm ? g.B : g.A;
  const int32_t* sidx = sm ? g.lidx : g.ridx;
  const int32_t* bidx = sm ? g.ridx : g.lidx;
  const int sbits = sm ? g.mb : g.nb, bbits = sm ? g.nb : g.mb;
  const BitMap& mapS = sm ? g.mapM : g.mapN;
  const BitMap& mapB = sm ? g.mapN : g.mapM;
  const int64_t per = int64_t(1) << (g.mb + g.nb);
  const int64_t chunks = (int64_t(1) << sbits) / (256 * U);
  const int64_t items = g.nvar * chunks;
  const int64_t dep_t = deposit(threadIdx.x, mapS);
  int64_t dep_u[U];
#pragma unroll
  for (int u = 0; u < U; ++u) dep_u[u] = deposit(uint64_t(u) << 8, mapS) + dep_t;
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    const int64_t a = w % g.nvar, c = w / g.nvar;
    const int ai = __builtin_amdgcn_readfirstlane(int(a));
    const uint32_t sv = load_uniform(sidx + ai), bv = load_uniform(bidx + ai);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t s0 = c * (256 * U);
    const float2* srow = S + ((uint64_t(sv) << sbits) + s0 + threadIdx.x) * K;
    float2 x[U][K];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (KB == 0) {
        x[u][0] = srow[(u << 8) * K];
      } else {
#pragma unroll
        for (int j = 0; j < K / 2; ++j) {
          const float4 q = reinterpret_cast<const float4*>(srow + (u << 8) * K)[j];
          x[u][2 * j] = make_float2(q.x, q.y);
          x[u][2 * j + 1] = make_float2(q.z, q.w);
        }
      }
    }
    float2* out = g.C + a * per + deposit(uint64_t(s0), mapS);
    const float2* brow0 = Bc + (uint64_t(bv) << (bbits + KB));
    __syncthreads();  // the previous item's reads of bsh are done
    for (int i = threadIdx.x; i < (K << bbits); i += 256) bsh[i] = brow0[i];
    __syncthreads();
    for (int b = 0; b < (1 << bbits); ++b) {
      float2 y[K];
#pragma unroll
      for (int k = 0; k < K; ++k) y[k] = bsh[b * K + k];
      const int64_t db = deposit(uint64_t(b), mapB);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          re += x[u][k].x * y[k].x - x[u][k].y * y[k].y;
          im += x[u][k].x * y[k].y + x[u][k].y * y[k].x;
        }
        out[db + dep_u[u]] = make_float2(re, im);
        amax = fmaxf(amax, fmaxf(fabsf(re), fabsf(im)));
      }
    }
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
}

// ---------------------------------------------------------------------------
// MFMA contraction (complex GEMM  C = A . B^T over stacked keys, or one per
// key in the keyed form; both operands with their K legs contiguous).
//
// Tile shapes (workgroup of four waves):
//   0: 64 x 64,  waves 2 x 2, one 32 x 32 block each
//   1: 32 x 128, waves 1 x 4, one 32 x 32 block each
//   2: 16 x 256, waves 1 x 4, four 16 x 16 blocks each
//   3: 64 x 16,  waves 4 x 1, one 16 x 16 block each (narrow keyed products)
//   4: 128 x 128, waves 2 x 2, four 32 x 32 blocks each (each operand
//      fragment read from LDS feeds two blocks: half the LDS reads and half
//      the operand re-fetch of the 64 x 64 tile per MFMA)
//   5: 128 x 128, eight waves with double-buffered LDS (split forms only,
//      k_contract_split_db)
//   6: 128 x 128, four waves of 64 x 64 on operands converted once into
//      hi/lo planes (split forms only, k_presplit + k_contract_planes)
//   7: 256 x 128, eight waves of 64 x 64 on plane-format operands (split
//      forms only)
// Precisions:
//   PREC 0 (complex64): v_mfma_f32_32x32x2f32 / 16x16x4f32; a complex k costs
//     4 real MACs: the instruction's K runs over (re, im) of the row operand
//     and the column operand supplies (re, -im) for the real part and (im, re)
//     for the imaginary part.  LDS holds re / im planes [k][plane][row].
//   PREC 1 / 2 (split FP16 / BF16): each operand float x, scaled by a power of
//     two 2^e (FP16 only; e from the tensor's largest magnitude so that it lands
//     in [2^14, 2^15)), becomes hi = round(x 2^e), lo = round(x 2^e - hi); the
//     products hi.hi + hi.lo + lo.hi accumulate in FP32 on
//     v_mfma_f32_32x32x16 / 16x16x32 (lo.lo is dropped) and the result is
//     scaled back by 2^-(eA + eB).  LDS holds four planes per operand (hi re,
//     hi im, lo re, lo im), rows of TK + 8 halves (see k_contract_split).
// K is staged TK complex at a time (a template parameter: 16 or 32 for
// complex64, 32 or 64 for the split forms; larger slabs keep more bytes in
// flight per barrier, smaller ones need fewer registers).
//
// The grid is persistent: each workgroup walks tiles p = blockIdx.x,
// blockIdx.x + gridDim.x, ...; the register prefetch of the next K slab runs
// across tile boundaries, so the next tile's first loads overlap the current
// tile's last MFMAs and its epilogue.  Workgroup w runs on XCD w % 8; the walk
// is swizzled so that each XCD covers a contiguous range of tiles in
// column-major order, and tiles sharing one B slab stay in one L2.
//
// Epilogue: the tile is parked in LDS and written in the order of the output
// layout's bit positions (ubit), so each wave stores runs of consecutive
// addresses.  With FP16 operands the epilogue also publishes the output's
// largest magnitude for the consumer's scale.
constexpr int PAD = 1;

template <int CFG>
struct Tile;
template <>
struct Tile<0> { static constexpr int BM = 64, BN = 64, MF = 32, WM = 2; };
template <>
struct Tile<1> { static constexpr int BM = 32, BN = 128, MF = 32, WM = 1; };
template <>
struct Tile<2> { static constexpr int BM = 16, BN = 256, MF = 16, WM = 1; };
template <>
struct Tile<3> { static constexpr int BM = 64, BN = 16, MF = 16, WM = 4; };
template <>
struct Tile<4> { static constexpr int BM = 128, BN = 128, MF = 32, WM = 2; };
// (Tile 5, 128 x 128 with eight waves, is k_contract_split_db's own layout;
// the entry gives its shape to the shared epilogue and tile map.)
template <>
struct Tile<5> { static constexpr int BM = 128, BN = 128, MF = 32, WM = 4; };
// (Tile 6, 128 x 128 on plane-format operands, is k_contract_planes' own
// layout; its epilogue writes half tiles, whose shape is entry 7.)
template <>
struct Tile<6> { static constexpr int BM = 128, BN = 128, MF = 32, WM = 2; };
template <>
struct Tile<7> { static constexpr int BM = 64, BN = 128, MF = 32, WM = 2; };
// (Tile 7 of the API, 256 x 128 on plane-format operands with eight waves.)
template <>
struct Tile<8> { static constexpr int BM = 256, BN = 128, MF = 32, WM = 4; };

template <int CFG, int PREC, int TKV = 16>
struct TileInfo {
  static constexpr int TK = TKV;
  static constexpr int KP = TK + 8;  // halves per split-form plane row
  using B_ = Tile<CFG>;
  static constexpr int BM = B_::BM, BN = B_::BN, MF = B_::MF, WM = B_::WM;
  static constexpr int WN = 4 / WM;
  static constexpr int BMW = BM / WM, BNW = BN / WN;
  static constexpr int FM = BMW / MF, FN = BNW / MF;
  static constexpr int REGS = MF == 32 ? 16 : 4;
  static constexpr int A_F4 = BM * TK / 2;  // float4 loads per tile slab
  static constexpr int B_F4 = BN * TK / 2;
  static constexpr int A_VEC = (A_F4 + 255) / 256;
  static constexpr int B_VEC = (B_F4 + 255) / 256;
  // LDS, in floats.
  // (split forms: four planes of rows of KP halves)
  static constexpr int LDS_A = PREC == 0 ? TK * 2 * (BM + PAD) : 2 * BM * KP;
  static constexpr int LDS_B = PREC == 0 ? TK * 2 * (BN + PAD) : 2 * BN * KP;
  static constexpr int LDS_MAIN = LDS_A + LDS_B;
  static constexpr int LDS_EPI = BM * (BN + 1) * 2;
  static constexpr int LDS = LDS_MAIN > LDS_EPI ? LDS_MAIN : LDS_EPI;
  static constexpr int LOG_BM = BM == 128 ? 7 : (BM == 64 ? 6 : (BM == 32 ? 5 : 4));
  static constexpr int LOG_BN = BN == 16 ? 4 : (BN == 64 ? 6 : (BN == 128 ? 7 : 8));
  static constexpr int UBITS = LOG_BM + LOG_BN;
  static constexpr int PER_THREAD = BM * BN / 256;
};

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Scale exponent e with amax 2^e in [2^14, 2^15) (0 for an all-zero tensor),
// from a table's n amax slots.
// The n <= 64 slots are read by one vector load across the wave (lane i
// reads slot i) and reduced with shuffles: one memory round trip instead of n
// dependent scalar loads at every workgroup's start.
__device__ __forceinline__ int fp16_scale_exp(const unsigned long long* slots, int n) {
  const int lane = threadIdx.x & 63;
  unsigned long long w = lane < n ? slots[lane * kAmaxStride] : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t hi = __shfl_xor(uint32_t(w >> 32), o), lo = __shfl_xor(uint32_t(w), o);
    const unsigned long long v = (static_cast<unsigned long long>(hi) << 32) | lo;
    w = v > w ? v : w;
  }
  const float m = __uint_as_float(uint32_t(w));
  if (!(m > 0.f)) return 0;
  int e = 14 - ilogbf(m);
  return e < -120 ? -120 : (e > 120 ? 120 : e);
}

// Split one float into (hi, lo) 16-bit halves, returned as raw bits.
template <int PREC>
__device__ __forceinline__ void split2(float x, uint32_t& hi, uint32_t& lo) {
  if constexpr (PREC == 1) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  } else {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
}

// Four complex numbers (x = re0 im0 re1 im1, y = re2 im2 re3 im3) scaled by s
// -> their hi and lo halves packed per plane: re_hi, im_hi, re_lo, im_lo
// (uint2 each, k ascending), stored at plane + row offset `at` of four planes
// `plane` halves apart.
template <int PREC>
__device__ __forceinline__ void split_store4(float4 x, float4 y, float s, uint16_t* at, int plane) {
  uint32_t h[8], l[8];
  split2<PREC>(x.x * s, h[0], l[0]);
  split2<PREC>(x.y * s, h[1], l[1]);
  split2<PREC>(x.z * s, h[2], l[2]);
  split2<PREC>(x.w * s, h[3], l[3]);
  split2<PREC>(y.x * s, h[4], l[4]);
  split2<PREC>(y.y * s, h[5], l[5]);
  split2<PREC>(y.z * s, h[6], l[6]);
  split2<PREC>(y.w * s, h[7], l[7]);
  *reinterpret_cast<uint2*>(at) = make_uint2(h[0] | (h[2] << 16), h[4] | (h[6] << 16));
  *reinterpret_cast<uint2*>(at + plane) = make_uint2(h[1] | (h[3] << 16), h[5] | (h[7] << 16));
  *reinterpret_cast<uint2*>(at + 2 * plane) = make_uint2(l[0] | (l[2] << 16), l[4] | (l[6] << 16));
  *reinterpret_cast<uint2*>(at + 3 * plane) = make_uint2(l[1] | (l[3] << 16), l[5] | (l[7] << 16));
}

// One split-form MFMA: 32x32x16 or 16x16x32, FP16 (PREC 1) or BF16 (PREC 2).
template <int MF, int PREC, class Acc>
__device__ __forceinline__ Acc mma_split(const u32x4& x, const u32x4& y, const Acc& acc) {
  if constexpr (MF == 32 && PREC == 1)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, x), __builtin_bit_cast(half8, y), acc, 0, 0, 0);
  else if constexpr (MF == 32)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), acc, 0, 0, 0);
  else if constexpr (PREC == 1)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, x), __builtin_bit_cast(half8, y), acc, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, x), __builtin_bit_cast(bf16x8, y), acc, 0, 0, 0);
}

// Tile numbering of one launch.  Dense and table forms (pair_mode 0 / 1)
// tile the stacked rows x stacked columns; the keyed form (pair_mode 2) tiles
// each key's own 2^mb x 2^nb product (its operand variants from lidx / ridx,
// swapped when A holds R); a key narrower than the tile leaves the tile's
// other rows / columns unused.
struct TileOrigin {
  int64_t row0, col0;        // first stacked row and column
  int64_t key;               // the tile's key (keyed form), else -1
  int64_t row_end, col_end;  // ends (exclusive) of the rows / columns it may use
};

template <int BM, int BN>
struct TileMap {
  int64_t tiles_m = 0, per_key = 0, tiles = 0;
  __device__ explicit TileMap(const ContractArgs& g) {
    if (g.pair_mode == 2) {
      tiles_m = ((int64_t(1) << g.mb) + BM - 1) / BM;
      per_key = tiles_m * (((int64_t(1) << g.nb) + BN - 1) / BN);
      tiles = g.nvar * per_key;
    } else {
      const int64_t rowsA = g.nvarA << g.mb, rowsB = g.nvarB << g.nb;
      tiles_m = (rowsA + BM - 1) / BM;
      tiles = tiles_m * ((rowsB + BN - 1) / BN);
    }
  }
  __device__ TileOrigin at(const ContractArgs& g, int64_t tile) const {
    TileOrigin o;
    origin(g, tile, o.row0, o.col0, o.key, o.row_end, o.col_end);
    return o;
  }
  __device__ void origin(const ContractArgs& g, int64_t tile, int64_t& row0, int64_t& col0,
                         int64_t& key, int64_t& row_end, int64_t& col_end) const {
    if (g.pair_mode == 2) {
      key = tile / per_key;
      const int64_t t = tile - key * per_key;
      const int k32 = __builtin_amdgcn_readfirstlane(int(key));
      const uint32_t vl = load_uniform(g.lidx + k32), vr = load_uniform(g.ridx + k32);
      const uint32_t va = g.swapped ? vr : vl, vb = g.swapped ? vl : vr;
      row0 = (int64_t(va) << g.mb) + (t % tiles_m) * BM;
      col0 = (int64_t(vb) << g.nb) + (t / tiles_m) * BN;
      row_end = int64_t(va + 1) << g.mb;
      col_end = int64_t(vb + 1) << g.nb;
    } else {
      key = -1;
      row0 = (tile % tiles_m) * BM;
      col0 = (tile / tiles_m) * BN;
      row_end = g.nvarA << g.mb;
      col_end = g.nvarB << g.nb;
    }
  }
};

// Epilogue set-up shared by the contraction and the split-K reduction:
// deposit tables of a tile's low row / column bits and this thread's share of
// the write order (tile element bits 0 .. log2(NT) - 1 come from the thread id
// of an NT-thread workgroup).
template <int CFG, int NT = 256>
__device__ __forceinline__ void epilogue_setup(const ContractArgs& g, int64_t* dep_m_lo,
                                               int64_t* dep_n_lo, int& r_tid, int& c_tid) {
  using T = TileInfo<CFG, 0>;
  constexpr int LOG_NT = NT == 512 ? 9 : 8;
  const int64_t M = int64_t(1) << g.mb, N = int64_t(1) << g.nb;
  const int64_t m_lo_mask = (M < T::BM ? M : T::BM) - 1;
  const int64_t n_lo_mask = (N < T::BN ? N : T::BN) - 1;
  for (int i = threadIdx.x; i < T::BM; i += NT) dep_m_lo[i] = deposit(i & m_lo_mask, g.mapM);
  for (int i = threadIdx.x; i < T::BN; i += NT) dep_n_lo[i] = deposit(i & n_lo_mask, g.mapN);
  r_tid = 0;
  c_tid = 0;
#pragma unroll
  for (int b = 0; b < LOG_NT; ++b) {
    if ((threadIdx.x >> b) & 1) {
      const int u = g.ubit[b];
      if (u < 32)
        r_tid |= 1 << u;
      else
        c_tid |= 1 << (u - 32);
    }
  }
}

// Writes a finished tile parked in LDS (Ct, rows of BN + 1) to the output
// table in the write order ubit (NT threads); returns the largest |re|, |im|
// written.
//
// An element's output offset is a sum over the set bits of its row and
// column index inside the tile: a row bit below mb deposits to its output
// position, a row bit at or above mb steps the row operand's variant (dense
// keys: a fixed stride of keys; keyed form: out of the key's rows, masked by
// the bounds); columns alike.  So the offsets of one thread's elements follow
// from its first one by adding one per-bit delta per element, walking the
// element numbers in Gray-code order (one bit changes per step).  The table
// form (pair_mode 1) looks its key up per (row variant, column variant); the
// walk applies when the tile spans one of each, otherwise every element
// looks its key up.
template <int CFG, int NT = 256>
__device__ __forceinline__ float epilogue_write(const ContractArgs& g, const float2* Ct,
                                                int64_t row0, int64_t col0, int64_t key,
                                                int64_t row_end, int64_t col_end,
                                                const int64_t* dep_m_lo, const int64_t* dep_n_lo,
                                                int r_tid, int c_tid) {
  using T = TileInfo<CFG, 0>;
  constexpr int BM = T::BM, BN = T::BN;
  constexpr int LOG_NT = NT == 512 ? 9 : 8;
  constexpr int PER_THREAD = BM * BN / NT;
  constexpr int UB = T::UBITS - LOG_NT;  // element-number bits walked per thread
  const int64_t M = int64_t(1) << g.mb, N = int64_t(1) << g.nb;
  const int64_t sizeC = M * N;
  const int64_t dep_m_hi = M > BM ? deposit(row0 & (M - 1), g.mapM) : 0;
  const int64_t dep_n_hi = N > BN ? deposit(col0 & (N - 1), g.mapN) : 0;
  float amax = 0.f;
  if (g.pair_mode != 1 || (M >= BM && N >= BN)) {
    int64_t a0 = key;
    if (key < 0) {
      const int64_t rv = row0 >> g.mb, cv = col0 >> g.nb;
      a0 = g.swapped ? cv * g.nvarA + rv : rv * g.nvarB + cv;
      if (g.pair_mode == 1) a0 = g.pairs[a0];
      if (a0 < 0) return 0.f;
    }
    // Offset steps of one more row / column variant (dense keys only; in the
    // keyed form such rows and columns lie outside the bounds).
    const int64_t key_r = g.pair_mode == 0 ? (g.swapped ? 1 : g.nvarB) * sizeC : 0;
    const int64_t key_c = g.pair_mode == 0 ? (g.swapped ? g.nvarA : 1) * sizeC : 0;
    float2* out = g.C + a0 * sizeC + dep_m_hi + dep_n_hi + dep_m_lo[r_tid & (BM - 1)] +
                  dep_n_lo[c_tid & (BN - 1)] + (int64_t(r_tid) >> g.mb) * key_r +
                  (int64_t(c_tid) >> g.nb) * key_c;
    int lds = r_tid * (BN + 1) + c_tid;
    // Per element-number bit: offset, LDS and row / column steps.  All are
    // uniform (kernel arguments only), so they stay in scalar registers.
    int64_t dg[UB > 0 ? UB : 1];
    int dl[UB > 0 ? UB : 1], dr[UB > 0 ? UB : 1], dc[UB > 0 ? UB : 1];
#pragma unroll
    for (int k = 0; k < UB; ++k) {
      const int u = g.ubit[LOG_NT + k];
      if (u < 32) {
        dg[k] = (int64_t(1) << u) < M ? deposit(uint64_t(1) << u, g.mapM)
                                      : (int64_t(1) << (u - g.mb)) * key_r;
        dl[k] = (1 << u) * (BN + 1);
        dr[k] = 1 << u;
        dc[k] = 0;
      } else {
        dg[k] = (int64_t(1) << (u - 32)) < N ? deposit(uint64_t(1) << (u - 32), g.mapN)
                                             : (int64_t(1) << (u - 32 - g.nb)) * key_c;
        dl[k] = 1 << (u - 32);
        dr[k] = 0;
        dc[k] = 1 << (u - 32);
      }
    }
    if (row0 + BM <= row_end && col0 + BN <= col_end) {
#pragma unroll
      for (int s = 0; s < PER_THREAD; ++s) {
        if (s > 0) {
          const int k = __builtin_ctz(s);
          const bool up = ((s ^ (s >> 1)) >> k) & 1;
          out += up ? dg[k] : -dg[k];
          lds += up ? dl[k] : -dl[k];
        }
        const float2 val = Ct[lds];
        *out = val;
        amax = fmaxf(amax, fmaxf(fabsf(val.x), fabsf(val.y)));
      }
    } else {
      int r = r_tid, c = c_tid;
#pragma unroll
      for (int s = 0; s < PER_THREAD; ++s) {
        if (s > 0) {
          const int k = __builtin_ctz(s);
          const bool up = ((s ^ (s >> 1)) >> k) & 1;
          out += up ? dg[k] : -dg[k];
          lds += up ? dl[k] : -dl[k];
          r ^= dr[k];
          c ^= dc[k];
        }
        if (row0 + r < row_end && col0 + c < col_end) {
          const float2 val = Ct[lds];
          *out = val;
          amax = fmaxf(amax, fmaxf(fabsf(val.x), fabsf(val.y)));
        }
      }
    }
    return amax;
  }
#pragma unroll 4
  for (int t = 0; t < PER_THREAD; ++t) {
    int r = r_tid, c = c_tid;
#pragma unroll
    for (int b = LOG_NT; b < T::UBITS; ++b) {
      if ((t >> (b - LOG_NT)) & 1) {
        const int u = g.ubit[b];
        if (u < 32)
          r |= 1 << u;
        else
          c |= 1 << (u - 32);
      }
    }
    const int64_t gr = row0 + r, gc = col0 + c;
    if (gr >= row_end || gc >= col_end) continue;
    int64_t a = key;
    if (key < 0) {
      const int64_t rv = gr >> g.mb, cv = gc >> g.nb;
      a = g.swapped ? cv * g.nvarA + rv : rv * g.nvarB + cv;
      if (g.pair_mode == 1) a = g.pairs[a];
      if (a < 0) continue;
    }
    const float2 val = Ct[r * (BN + 1) + c];
    g.C[a * sizeC + dep_m_hi + dep_m_lo[r] + dep_n_hi + dep_n_lo[c]] = val;
    amax = fmaxf(amax, fmaxf(fabsf(val.x), fabsf(val.y)));
  }
  return amax;
}

// KG K groups of four waves each: group g stages and multiplies the K slabs
// g, g + KG, g + 2 KG, ... of every tile in LDS of its own (more loads in
// flight per tile, MFMA of one group overlapping the staging of another), and
// the groups' accumulators are summed through LDS in group order at the end
// of the tile.
template <int CFG, int PREC, int TKV, int KG>
__global__ void __launch_bounds__(256 * KG) k_contract_mfma(ContractArgs g) {
  static_assert(PREC == 0, "the split forms run in k_contract_split");
  using T = TileInfo<CFG, PREC, TKV>;
  constexpr int TK = T::TK;
  constexpr int BM = T::BM, BN = T::BN, MF = T::MF;
  constexpr int LDS_TOTAL = KG * T::LDS_MAIN > T::LDS_EPI ? KG * T::LDS_MAIN : T::LDS_EPI;
  typedef float accv __attribute__((ext_vector_type(T::REGS)));
  __shared__ __attribute__((aligned(16))) float smem[LDS_TOTAL];
  __shared__ int64_t dep_m_lo[BM];
  __shared__ int64_t dep_n_lo[BN];
  const int grp = KG == 1 ? 0 : int(threadIdx.x >> 8);
  float* gsmem = smem + grp * T::LDS_MAIN;
  float(*As)[2][BM + PAD] = reinterpret_cast<float(*)[2][BM + PAD]>(gsmem);
  float(*Bs)[2][BN + PAD] = reinterpret_cast<float(*)[2][BN + PAD]>(gsmem + T::LDS_A);
  float2* Ct = reinterpret_cast<float2*>(smem);

  const int tid = threadIdx.x & 255;  // thread within its K group
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const int64_t rowsA = g.nvarA << g.mb;
  const int64_t rowsB = g.nvarB << g.nb;
  const TileMap<BM, BN> tmap(g);
  const int64_t tiles = tmap.tiles;
  // Work items: (K chunk, tile), item = chunk * tiles + tile.
  const int64_t items = tiles * g.ksplit;
  const int64_t per_xcd = (items + 7) / 8;
  const int64_t walk = per_xcd * 8;
  const int64_t K = int64_t(1) << g.kb;
  const int64_t Kc = K / g.ksplit;

  float amax = 0.f;

  int r_tid = 0, c_tid = 0;
  epilogue_setup<CFG>(g, dep_m_lo, dep_n_lo, r_tid, c_tid);
  __syncthreads();

  // Walk position p -> work item (XCD-contiguous; tiles column-major inside
  // one K chunk).
  auto item_of = [&](int64_t p) -> int64_t { return (p & 7) * per_xcd + (p >> 3); };
  auto next_p = [&](int64_t p) -> int64_t {
    for (p += gridDim.x; p < walk; p += gridDim.x)
      if (item_of(p) < items) return p;
    return walk;
  };
  auto k_begin = [&](int64_t item) -> int64_t { return (item / tiles) * Kc; };

  float4 ra[T::A_VEC], rb[T::B_VEC];
  // Loads the slab at k0 of a work item, zero beyond the item's K chunk end.
  auto fetch = [&](const TileOrigin& o, int64_t k0, int64_t klim) {
    const int64_t row0 = o.row0, col0 = o.col0, row_end = o.row_end, col_end = o.col_end;
#pragma unroll
    for (int t = 0; t < T::A_VEC; ++t) {
      const int e = tid + t * 256;
      const int r = e / (TK / 2), kp = e % (TK / 2);
      const int64_t gr = row0 + r, gk = k0 + 2 * kp;
      ra[t] = (e < T::A_F4 && gr < row_end && gk < klim)
                  ? *reinterpret_cast<const float4*>(g.A + (gr << g.kb) + gk)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int t = 0; t < T::B_VEC; ++t) {
      const int e = tid + t * 256;
      const int r = e / (TK / 2), kp = e % (TK / 2);
      const int64_t gr = col0 + r, gk = k0 + 2 * kp;
      rb[t] = (e < T::B_F4 && gr < col_end && gk < klim)
                  ? *reinterpret_cast<const float4*>(g.B + (gr << g.kb) + gk)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };

  int64_t p = blockIdx.x;
  if (p < walk && item_of(p) >= items) p = next_p(p);
  if (p >= walk) {
    if (g.amax_out) publish_amax(0.f, g.amax_out, g.epoch);
    return;
  }
  // Origin of the tile being multiplied (updated when the next tile's first
  // slab is fetched).
  TileOrigin cur = tmap.at(g, item_of(p) % tiles);
  fetch(cur, k_begin(item_of(p)) + grp * TK, k_begin(item_of(p)) + Kc);

  while (p < walk) {
    const int64_t item = item_of(p);
    const TileOrigin o = cur;
    const int64_t row0 = o.row0, col0 = o.col0, key = o.key, row_end = o.row_end, col_end = o.col_end;
    const int64_t kbeg = k_begin(item), kend = kbeg + Kc;
    const int64_t pn = next_p(p);

    accv acc_re[T::FM][T::FN], acc_im[T::FM][T::FN];
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
        for (int v = 0; v < T::REGS; ++v) {
          acc_re[fm][fn][v] = 0.f;
          acc_im[fm][fn][v] = 0.f;
        }

    for (int64_t k0 = kbeg; k0 < kend; k0 += KG * TK) {
      // Registers -> LDS (this group's slab k0 + grp TK).
#pragma unroll
      for (int t = 0; t < T::A_VEC; ++t) {
        const int e = tid + t * 256;
        if (e < T::A_F4) {
          const int r = e / (TK / 2), kk = 2 * (e % (TK / 2));
          As[kk][0][r] = ra[t].x;
          As[kk][1][r] = ra[t].y;
          As[kk + 1][0][r] = ra[t].z;
          As[kk + 1][1][r] = ra[t].w;
        }
      }
#pragma unroll
      for (int t = 0; t < T::B_VEC; ++t) {
        const int e = tid + t * 256;
        if (e < T::B_F4) {
          const int r = e / (TK / 2), kk = 2 * (e % (TK / 2));
          Bs[kk][0][r] = rb[t].x;
          Bs[kk][1][r] = rb[t].y;
          Bs[kk + 1][0][r] = rb[t].z;
          Bs[kk + 1][1][r] = rb[t].w;
        }
      }
      __syncthreads();
      if (k0 + KG * TK < kend) {
        fetch(o, k0 + (KG + grp) * TK, kend);
      } else if (pn < walk) {
        cur = tmap.at(g, item_of(pn) % tiles);
        fetch(cur, k_begin(item_of(pn)) + grp * TK, k_begin(item_of(pn)) + Kc);
      }

      if constexpr (MF == 32) {
        const int i = lane & 31;
        const int half = lane >> 5;  // 0: real part of the K = 2 pair, 1: imaginary
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
          float a[T::FM], bo_re[T::FN], bo_im[T::FN];
#pragma unroll
          for (int fm = 0; fm < T::FM; ++fm) a[fm] = As[kk][half][wm * T::BMW + fm * 32 + i];
#pragma unroll
          for (int fn = 0; fn < T::FN; ++fn) {
            const float bre = Bs[kk][0][wn * T::BNW + fn * 32 + i];
            const float bim = Bs[kk][1][wn * T::BNW + fn * 32 + i];
            bo_re[fn] = half ? -bim : bre;
            bo_im[fn] = half ? bre : bim;
          }
#pragma unroll
          for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < T::FN; ++fn) {
              acc_re[fm][fn] =
                  __builtin_amdgcn_mfma_f32_32x32x2f32(a[fm], bo_re[fn], acc_re[fm][fn], 0, 0, 0);
              acc_im[fm][fn] =
                  __builtin_amdgcn_mfma_f32_32x32x2f32(a[fm], bo_im[fn], acc_im[fm][fn], 0, 0, 0);
            }
        }
      } else {
        // 16x16x4: lane l holds k = l / 16 of the instruction's K = 4, i.e.
        // complex k (l / 32) of the pair and its part (l / 16) % 2.
        const int i = lane & 15;
        const int q = lane >> 4;
        const int kq = q >> 1, part = q & 1;
#pragma unroll
        for (int kk = 0; kk < TK; kk += 2) {
          float a[T::FM], bo_re[T::FN], bo_im[T::FN];
#pragma unroll
          for (int fm = 0; fm < T::FM; ++fm)
            a[fm] = As[kk + kq][part][wm * T::BMW + fm * 16 + i];
#pragma unroll
          for (int fn = 0; fn < T::FN; ++fn) {
            const float bre = Bs[kk + kq][0][wn * T::BNW + fn * 16 + i];
            const float bim = Bs[kk + kq][1][wn * T::BNW + fn * 16 + i];
            bo_re[fn] = part ? -bim : bre;
            bo_im[fn] = part ? bre : bim;
          }
#pragma unroll
          for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < T::FN; ++fn) {
              acc_re[fm][fn] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(a[fm], bo_re[fn], acc_re[fm][fn], 0, 0, 0);
              acc_im[fm][fn] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(a[fm], bo_im[fn], acc_im[fm][fn], 0, 0, 0);
            }
        }
      }
      __syncthreads();
    }

    // 32x32 results: lane l, register v hold row (v % 4) + 4 (l / 32) +
    // 8 (v / 4), column l % 32.  16x16: row 4 (l / 16) + v, column l % 16.
    auto for_each_result = [&](auto&& f) {
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
          for (int v = 0; v < T::REGS; ++v) {
            int r, c;
            if constexpr (MF == 32) {
              r = wm * T::BMW + fm * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
              c = wn * T::BNW + fn * 32 + (lane & 31);
            } else {
              r = wm * T::BMW + fm * 16 + 4 * (lane >> 4) + v;
              c = wn * T::BNW + fn * 16 + (lane & 15);
            }
            f(r, c, make_float2(acc_re[fm][fn][v], acc_im[fm][fn][v]));
          }
    };
    if constexpr (KG == 2) {
      // Group 1's partial tile through LDS; group 0 adds it to its own.
      if (grp == 1) for_each_result([&](int r, int c, float2 x) { Ct[r * (BN + 1) + c] = x; });
      __syncthreads();
    }
    if (g.ksplit > 1) {
      // A K chunk's product goes to its partial tile, row-major.
      float2* dst = g.partial + item * (BM * BN);
      if (grp == 0)
        for_each_result([&](int r, int c, float2 x) {
          if constexpr (KG == 2) {
            const float2 y = Ct[r * (BN + 1) + c];
            x = make_float2(x.x + y.x, x.y + y.y);
          }
          dst[r * BN + c] = x;
        });
      // (With one group the last slab's barrier already freed LDS for the
      // next item; with two, Ct is read here.)
      if constexpr (KG == 2) __syncthreads();
      p = pn;
      continue;
    }
    // Park the tile in LDS.
    if (grp == 0)
      for_each_result([&](int r, int c, float2 x) {
        if constexpr (KG == 2) {
          const float2 y = Ct[r * (BN + 1) + c];
          x = make_float2(x.x + y.x, x.y + y.y);
        }
        Ct[r * (BN + 1) + c] = x;
      });
    __syncthreads();
    if (grp == 0)
      amax = fmaxf(amax, epilogue_write<CFG>(g, Ct, row0, col0, key, row_end, col_end, dep_m_lo, dep_n_lo, r_tid, c_tid));
    __syncthreads();
    p = pn;
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
}

// Split FP16 / BF16 contraction.  Same walk, tiles, K groups, split K and
// epilogue as k_contract_mfma; the operands are staged in LDS as four planes
// per operand (hi re, hi im, lo re, lo im; rows of TK + 8 halves), so that
//   re = sum ar.br + ai.(-bi),   im = sum ar.bi + ai.br
// take the planes as they are, except that the column operand's imaginary
// fragments are negated for the real part (one sign-bit XOR per packed pair
// in registers): two accumulators per 32 x 32 block.  Each product is
// hi.hi + hi.lo + lo.hi.
// A thread stages pairs of float4 (four consecutive complex of one row), and
// addresses inside a tile are 32-bit byte offsets from the tile's first row;
// rows past the operand's end re-read its last row (their results are never
// written) and only a slab that crosses the end of its K chunk is masked.
template <int CFG, int PREC, int TKV, int KG>
__global__ void __launch_bounds__(256 * KG) k_contract_split(ContractArgs g) {
  using T = TileInfo<CFG, PREC, TKV>;
  constexpr int TK = T::TK, KP = T::KP;
  constexpr int BM = T::BM, BN = T::BN, MF = T::MF;
  constexpr int PL_A = BM * KP, PL_B = BN * KP;  // halves per plane
  constexpr int LDS_G = T::LDS_MAIN;             // floats per K group
  constexpr int LDS_TOTAL = KG * LDS_G > T::LDS_EPI ? KG * LDS_G : T::LDS_EPI;
  constexpr int QR = TK / 4;                     // float4 pairs per row slab
  constexpr int NPA = BM * QR, NPB = BN * QR;    // pairs per slab
  constexpr int VPA = (NPA + 255) / 256, VPB = (NPB + 255) / 256;
  typedef float accv __attribute__((ext_vector_type(T::REGS)));
  __shared__ __attribute__((aligned(16))) float smem[LDS_TOTAL];
  __shared__ int64_t dep_m_lo[BM];
  __shared__ int64_t dep_n_lo[BN];
  const int grp = KG == 1 ? 0 : int(threadIdx.x >> 8);
  uint16_t* As = reinterpret_cast<uint16_t*>(smem + grp * LDS_G);
  uint16_t* Bs = As + 4 * PL_A;
  float2* Ct = reinterpret_cast<float2*>(smem);

  const int tid = threadIdx.x & 255;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const int64_t rowsA = g.nvarA << g.mb;
  const int64_t rowsB = g.nvarB << g.nb;
  const TileMap<BM, BN> tmap(g);
  const int64_t tiles = tmap.tiles;
  const int64_t items = tiles * g.ksplit;
  const int64_t per_xcd = (items + 7) / 8;
  const int64_t walk = per_xcd * 8;
  const int64_t K = int64_t(1) << g.kb;
  const int64_t Kc = K / g.ksplit;
  const int row_shift = g.kb + 3;  // bytes per operand row = 2^row_shift

  int eA = 0, eB = 0;
  if constexpr (PREC == 1) {
    eA = fp16_scale_exp(g.amaxA, g.amax_nA);
    eB = fp16_scale_exp(g.amaxB, g.amax_nB);
  }
  const float sA = ldexpf(1.f, eA), sB = ldexpf(1.f, eB), s_out = ldexpf(1.f, -(eA + eB));
  float amax = 0.f;

  int r_tid = 0, c_tid = 0;
  epilogue_setup<CFG>(g, dep_m_lo, dep_n_lo, r_tid, c_tid);
  __syncthreads();

  auto item_of = [&](int64_t p) -> int64_t { return (p & 7) * per_xcd + (p >> 3); };
  auto next_p = [&](int64_t p) -> int64_t {
    for (p += gridDim.x; p < walk; p += gridDim.x)
      if (item_of(p) < items) return p;
    return walk;
  };
  auto k_begin = [&](int64_t item) -> int64_t { return (item / tiles) * Kc; };

  float4 ra[VPA][2], rb[VPB][2];
  // One operand's slab: pairs p = tid + 256 j of rows [0, BM) (row p / QR,
  // complex 4 (p % QR) onwards).
  auto fetch_op = [&](float4 (*rg)[2], const float2* base, int last_row, int np, int vp,
                      bool full, int64_t k0, int64_t klim) {
    const char* b = reinterpret_cast<const char*>(base);
    for (int j = 0; j < vp; ++j) {
      const int pi = tid + j * 256;
      if (pi < np) {
        const int r = pi / QR, q = pi % QR;
        const int rr = r < last_row ? r : last_row;
        const float4* src = reinterpret_cast<const float4*>(b + ((uint32_t(rr) << row_shift) + 32u * q));
        if (full) {
          rg[j][0] = src[0];
          rg[j][1] = src[1];
        } else {
          const int64_t gk = k0 + 4 * q;
          rg[j][0] = gk < klim ? src[0] : make_float4(0.f, 0.f, 0.f, 0.f);
          rg[j][1] = gk + 2 < klim ? src[1] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
    }
  };
  auto fetch = [&](const TileOrigin& o, int64_t k0, int64_t klim) {
    const int64_t row0 = o.row0, col0 = o.col0, row_end = o.row_end, col_end = o.col_end;
    const int64_t la = row_end - row0 - 1, lb = col_end - col0 - 1;
    const bool full = k0 + TK <= klim;
    if (k0 >= klim) {
#pragma unroll
      for (int j = 0; j < VPA; ++j) ra[j][0] = ra[j][1] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int j = 0; j < VPB; ++j) rb[j][0] = rb[j][1] = make_float4(0.f, 0.f, 0.f, 0.f);
      return;
    }
    fetch_op(ra, g.A + (row0 << g.kb) + k0, la < BM ? int(la) : BM - 1, NPA, VPA, full, k0, klim);
    fetch_op(rb, g.B + (col0 << g.kb) + k0, lb < BN ? int(lb) : BN - 1, NPB, VPB, full, k0, klim);
  };

  int64_t p = blockIdx.x;
  if (p < walk && item_of(p) >= items) p = next_p(p);
  if (p >= walk) {
    if (g.amax_out) publish_amax(0.f, g.amax_out, g.epoch);
    return;
  }
  // Origin of the tile being multiplied (updated when the next tile's first
  // slab is fetched).
  TileOrigin cur = tmap.at(g, item_of(p) % tiles);
  fetch(cur, k_begin(item_of(p)) + grp * TK, k_begin(item_of(p)) + Kc);

  constexpr int GROUPS = MF == 32 ? 2 : 4;  // lane K groups of 8 halves per MFMA
  constexpr int KPM = 8 * GROUPS;           // K per MFMA
  constexpr int STEPS = TK / KPM;
  const int li = MF == 32 ? (lane & 31) : (lane & 15);
  const int lg = MF == 32 ? (lane >> 5) : (lane >> 4);

  while (p < walk) {
    const int64_t item = item_of(p);
    const TileOrigin o = cur;
    const int64_t row0 = o.row0, col0 = o.col0, key = o.key, row_end = o.row_end, col_end = o.col_end;
    const int64_t kbeg = k_begin(item), kend = kbeg + Kc;
    const int64_t pn = next_p(p);

    accv acc_re[T::FM][T::FN], acc_im[T::FM][T::FN];
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
        for (int v = 0; v < T::REGS; ++v) {
          acc_re[fm][fn][v] = 0.f;
          acc_im[fm][fn][v] = 0.f;
        }

    for (int64_t k0 = kbeg; k0 < kend; k0 += KG * TK) {
#pragma unroll
      for (int j = 0; j < VPA; ++j) {
        const int pi = tid + j * 256;
        if (pi < NPA) split_store4<PREC>(ra[j][0], ra[j][1], sA, As + (pi / QR) * KP + 4 * (pi % QR), PL_A);
      }
#pragma unroll
      for (int j = 0; j < VPB; ++j) {
        const int pi = tid + j * 256;
        if (pi < NPB) split_store4<PREC>(rb[j][0], rb[j][1], sB, Bs + (pi / QR) * KP + 4 * (pi % QR), PL_B);
      }
      __syncthreads();
      if (k0 + KG * TK < kend) {
        fetch(o, k0 + (KG + grp) * TK, kend);
      } else if (pn < walk) {
        cur = tmap.at(g, item_of(pn) % tiles);
        fetch(cur, k_begin(item_of(pn)) + grp * TK, k_begin(item_of(pn)) + Kc);
      }

#pragma unroll
      for (int st = 0; st < STEPS; ++st) {
        const int ko = st * KPM + 8 * lg;
        u32x4 arh[T::FM], aih[T::FM], arl[T::FM], ail[T::FM];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm) {
          const uint16_t* a = As + (wm * T::BMW + fm * MF + li) * KP + ko;
          arh[fm] = *reinterpret_cast<const u32x4*>(a);
          aih[fm] = *reinterpret_cast<const u32x4*>(a + PL_A);
          arl[fm] = *reinterpret_cast<const u32x4*>(a + 2 * PL_A);
          ail[fm] = *reinterpret_cast<const u32x4*>(a + 3 * PL_A);
        }
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn) {
          const uint16_t* b = Bs + (wn * T::BNW + fn * MF + li) * KP + ko;
          const u32x4 brh = *reinterpret_cast<const u32x4*>(b);
          const u32x4 bih = *reinterpret_cast<const u32x4*>(b + PL_B);
          const u32x4 brl = *reinterpret_cast<const u32x4*>(b + 2 * PL_B);
          const u32x4 bil = *reinterpret_cast<const u32x4*>(b + 3 * PL_B);
          // -bi: the sign bit of both packed halves (FP16 and BF16 alike).
          const u32x4 nbih = bih ^ 0x80008000u, nbil = bil ^ 0x80008000u;
#pragma unroll
          for (int fm = 0; fm < T::FM; ++fm) {
#define XEB_MMA(acc, x, y) acc = mma_split<MF, PREC>(x, y, acc)
            XEB_MMA(acc_re[fm][fn], arh[fm], brh);
            XEB_MMA(acc_im[fm][fn], arh[fm], bih);
            XEB_MMA(acc_re[fm][fn], aih[fm], nbih);
            XEB_MMA(acc_im[fm][fn], aih[fm], brh);
            XEB_MMA(acc_re[fm][fn], arh[fm], brl);
            XEB_MMA(acc_im[fm][fn], arh[fm], bil);
            XEB_MMA(acc_re[fm][fn], aih[fm], nbil);
            XEB_MMA(acc_im[fm][fn], aih[fm], brl);
            XEB_MMA(acc_re[fm][fn], arl[fm], brh);
            XEB_MMA(acc_im[fm][fn], arl[fm], bih);
            XEB_MMA(acc_re[fm][fn], ail[fm], nbih);
            XEB_MMA(acc_im[fm][fn], ail[fm], brh);
#undef XEB_MMA
          }
        }
      }
      __syncthreads();
    }

    auto for_each_result = [&](auto&& f) {
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
          for (int v = 0; v < T::REGS; ++v) {
            int r, c;
            if constexpr (MF == 32) {
              r = wm * T::BMW + fm * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
              c = wn * T::BNW + fn * 32 + (lane & 31);
            } else {
              r = wm * T::BMW + fm * 16 + 4 * (lane >> 4) + v;
              c = wn * T::BNW + fn * 16 + (lane & 15);
            }
            f(r, c, make_float2(acc_re[fm][fn][v] * s_out, acc_im[fm][fn][v] * s_out));
          }
    };
    if constexpr (KG == 2) {
      if (grp == 1) for_each_result([&](int r, int c, float2 x) { Ct[r * (BN + 1) + c] = x; });
      __syncthreads();
    }
    if (g.ksplit > 1) {
      float2* dst = g.partial + item * (BM * BN);
      if (grp == 0)
        for_each_result([&](int r, int c, float2 x) {
          if constexpr (KG == 2) {
            const float2 y = Ct[r * (BN + 1) + c];
            x = make_float2(x.x + y.x, x.y + y.y);
          }
          dst[r * BN + c] = x;
        });
      if constexpr (KG == 2) __syncthreads();
      p = pn;
      continue;
    }
    if (grp == 0)
      for_each_result([&](int r, int c, float2 x) {
        if constexpr (KG == 2) {
          const float2 y = Ct[r * (BN + 1) + c];
          x = make_float2(x.x + y.x, x.y + y.y);
        }
        Ct[r * (BN + 1) + c] = x;
      });
    __syncthreads();
    if (grp == 0)
      amax = fmaxf(amax, epilogue_write<CFG>(g, Ct, row0, col0, key, row_end, col_end, dep_m_lo, dep_n_lo, r_tid, c_tid));
    __syncthreads();
    p = pn;
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
}

// Split FP16 / BF16 contraction on 128 x 128 tiles with eight waves and
// double-buffered LDS (tile 5).  Waves form a 4 x 2 grid; each computes a
// 32 x 64 block pair (two 32x32x16 MFMA blocks sharing the row fragment)
// with two accumulators per block, as in k_contract_split.  K runs in slabs
// of 16 complex; while the waves multiply slab i out of one LDS buffer, the
// hi/lo planes of slab i + 1 (already in registers) are written to the other
// buffer and the global loads of slab i + 2 are issued, so one barrier per
// slab separates the phases and each SIMD holds two waves whose MFMA and
// staging work interleave.  At the end of a tile the result is parked in LDS
// (over both buffers) and written in the output's bit order; the first slab
// of the next tile is already in registers by then.  Thread t stages row
// t / 4, complex 4 (t % 4) .. 4 (t % 4) + 3 of both operands' slabs.
template <int PREC>
__global__ void __launch_bounds__(512) k_contract_split_db(ContractArgs g) {
  constexpr int BM = 128, BN = 128, TK = 16, KP = TK + 8;  // halves per plane row
  constexpr int PL_A = BM * KP, PL_B = BN * KP;            // halves per plane
  constexpr int BUF = 4 * (PL_A + PL_B);                   // halves per buffer
  constexpr int LDS_MAIN = BUF;                            // floats: two buffers of halves
  constexpr int LDS_EPI = BM * (BN + 1) * 2;
  constexpr int LDS_TOTAL = LDS_MAIN > LDS_EPI ? LDS_MAIN : LDS_EPI;
  typedef float accv __attribute__((ext_vector_type(16)));
  __shared__ __attribute__((aligned(16))) float smem[LDS_TOTAL];
  __shared__ int64_t dep_m_lo[BM];
  __shared__ int64_t dep_n_lo[BN];
  uint16_t* lds = reinterpret_cast<uint16_t*>(smem);
  float2* Ct = reinterpret_cast<float2*>(smem);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // rows 32 wm .., columns 64 wn ..
  const TileMap<BM, BN> tmap(g);
  const int64_t tiles = tmap.tiles;
  const int64_t items = tiles * g.ksplit;
  const int64_t per_xcd = (items + 7) / 8;
  const int64_t walk = per_xcd * 8;
  const int64_t K = int64_t(1) << g.kb;
  const int64_t Kc = K / g.ksplit;
  const int row_shift = g.kb + 3;  // bytes per operand row = 2^row_shift

  int eA = 0, eB = 0;
  if constexpr (PREC == 1) {
    eA = fp16_scale_exp(g.amaxA, g.amax_nA);
    eB = fp16_scale_exp(g.amaxB, g.amax_nB);
  }
  const float sA = ldexpf(1.f, eA), sB = ldexpf(1.f, eB), s_out = ldexpf(1.f, -(eA + eB));
  float amax = 0.f;

  int r_tid = 0, c_tid = 0;
  epilogue_setup<5, 512>(g, dep_m_lo, dep_n_lo, r_tid, c_tid);
  __syncthreads();

  auto item_of = [&](int64_t p) -> int64_t { return (p & 7) * per_xcd + (p >> 3); };
  auto next_p = [&](int64_t p) -> int64_t {
    for (p += gridDim.x; p < walk; p += gridDim.x)
      if (item_of(p) < items) return p;
    return walk;
  };
  auto k_begin = [&](int64_t item) -> int64_t { return (item / tiles) * Kc; };

  const int srow = tid >> 2, sq = tid & 3;
  float4 ra0, ra1, rb0, rb1;
  // One slab of both operands into registers: zero beyond the K chunk end;
  // rows past an operand's end re-read its last row (never written out).
  auto fetch = [&](const TileOrigin& o, int64_t k0, int64_t klim) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t gk = k0 + 4 * sq;
    if (gk >= klim) {
      ra0 = ra1 = rb0 = rb1 = z;
      return;
    }
    const int64_t la = o.row_end - o.row0 - 1, lb = o.col_end - o.col0 - 1;
    const uint32_t rra = uint32_t(srow < la ? srow : la), rrb = uint32_t(srow < lb ? srow : lb);
    const char* pa = reinterpret_cast<const char*>(g.A + (o.row0 << g.kb) + k0) + ((rra << row_shift) + 32u * sq);
    const char* pb = reinterpret_cast<const char*>(g.B + (o.col0 << g.kb) + k0) + ((rrb << row_shift) + 32u * sq);
    const bool two = gk + 2 < klim;
    ra0 = *reinterpret_cast<const float4*>(pa);
    rb0 = *reinterpret_cast<const float4*>(pb);
    ra1 = two ? *reinterpret_cast<const float4*>(pa + 16) : z;
    rb1 = two ? *reinterpret_cast<const float4*>(pb + 16) : z;
  };
  auto stage = [&](uint16_t* buf) {
    split_store4<PREC>(ra0, ra1, sA, buf + srow * KP + 4 * sq, PL_A);
    split_store4<PREC>(rb0, rb1, sB, buf + 4 * PL_A + srow * KP + 4 * sq, PL_B);
  };

  int64_t p = blockIdx.x;
  if (p < walk && item_of(p) >= items) p = next_p(p);
  if (p >= walk) {
    if (g.amax_out) publish_amax(0.f, g.amax_out, g.epoch);
    return;
  }
  TileOrigin cur = tmap.at(g, item_of(p) % tiles);
  fetch(cur, k_begin(item_of(p)), k_begin(item_of(p)) + Kc);

  const int li = lane & 31, lg = lane >> 5;
  while (p < walk) {
    const int64_t item = item_of(p);
    const TileOrigin o = cur;
    const int64_t kbeg = k_begin(item), kend = kbeg + Kc;
    const int nslabs = int((Kc + TK - 1) / TK);
    const int64_t pn = next_p(p);

    accv acc_re[2], acc_im[2];
#pragma unroll
    for (int fn = 0; fn < 2; ++fn)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc_re[fn][v] = acc_im[fn][v] = 0.f;

    // Registers hold this tile's slab 0.
    stage(lds);
    if (nslabs > 1) {
      fetch(o, kbeg + TK, kend);
    } else if (pn < walk) {
      cur = tmap.at(g, item_of(pn) % tiles);
      fetch(cur, k_begin(item_of(pn)), k_begin(item_of(pn)) + Kc);
    }
    __syncthreads();
    for (int i = 0; i < nslabs; ++i) {
      const uint16_t* bc = lds + (i & 1) * BUF;
      if (i + 1 < nslabs) {
        stage(lds + ((i & 1) ^ 1) * BUF);
        if (i + 2 < nslabs) {
          fetch(o, kbeg + int64_t(i + 2) * TK, kend);
        } else if (pn < walk) {
          cur = tmap.at(g, item_of(pn) % tiles);
          fetch(cur, k_begin(item_of(pn)), k_begin(item_of(pn)) + Kc);
        }
      }
      const uint16_t* a = bc + (wm * 32 + li) * KP + 8 * lg;
      const u32x4 arh = *reinterpret_cast<const u32x4*>(a);
      const u32x4 aih = *reinterpret_cast<const u32x4*>(a + PL_A);
      const u32x4 arl = *reinterpret_cast<const u32x4*>(a + 2 * PL_A);
      const u32x4 ail = *reinterpret_cast<const u32x4*>(a + 3 * PL_A);
#pragma unroll
      for (int fn = 0; fn < 2; ++fn) {
        const uint16_t* b = bc + 4 * PL_A + (wn * 64 + fn * 32 + li) * KP + 8 * lg;
        const u32x4 brh = *reinterpret_cast<const u32x4*>(b);
        const u32x4 bih = *reinterpret_cast<const u32x4*>(b + PL_B);
        const u32x4 brl = *reinterpret_cast<const u32x4*>(b + 2 * PL_B);
        const u32x4 bil = *reinterpret_cast<const u32x4*>(b + 3 * PL_B);
        const u32x4 nbih = bih ^ 0x80008000u, nbil = bil ^ 0x80008000u;
#define XEB_MMA(acc, x, y) acc = mma_split<32, PREC>(x, y, acc)
        XEB_MMA(acc_re[fn], arh, brh);
        XEB_MMA(acc_im[fn], arh, bih);
        XEB_MMA(acc_re[fn], aih, nbih);
        XEB_MMA(acc_im[fn], aih, brh);
        XEB_MMA(acc_re[fn], arh, brl);
        XEB_MMA(acc_im[fn], arh, bil);
        XEB_MMA(acc_re[fn], aih, nbil);
        XEB_MMA(acc_im[fn], aih, brl);
        XEB_MMA(acc_re[fn], arl, brh);
        XEB_MMA(acc_im[fn], arl, bih);
        XEB_MMA(acc_re[fn], ail, nbih);
        XEB_MMA(acc_im[fn], ail, brh);
#undef XEB_MMA
      }
      __syncthreads();
    }

    // 32x32 results: lane l, register v hold row (v % 4) + 4 (l / 32) +
    // 8 (v / 4), column l % 32 of the block.
    auto for_each_result = [&](auto&& f) {
#pragma unroll
      for (int fn = 0; fn < 2; ++fn)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int r = wm * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
          const int c = wn * 64 + fn * 32 + (lane & 31);
          f(r, c, make_float2(acc_re[fn][v] * s_out, acc_im[fn][v] * s_out));
        }
    };
    if (g.ksplit > 1) {
      float2* dst = g.partial + item * (BM * BN);
      for_each_result([&](int r, int c, float2 x) { dst[r * BN + c] = x; });
      p = pn;
      continue;
    }
    for_each_result([&](int r, int c, float2 x) { Ct[r * (BN + 1) + c] = x; });
    __syncthreads();
    amax = fmaxf(amax, epilogue_write<5, 512>(g, Ct, o.row0, o.col0, o.key, o.row_end, o.col_end,
                                              dep_m_lo, dep_n_lo, r_tid, c_tid));
    __syncthreads();
    p = pn;
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
}

// ---------------------------------------------------------------------------
// Plane-format split contraction (tile 6).  A pre-pass converts each operand
// table once into hi/lo planes (k_presplit), so that the GEMM stages plain
// 16-byte copies instead of re-splitting every element in every tile that
// reads it.  Plane layout of an operand with K = 2^kb complex per row: row r,
// slab j (complex j TK .. j TK + TK - 1) is one contiguous block of
// 4 * TK halves: hi re, hi im, lo re, lo im, TK halves each (the FP16 form
// scaled by 2^e as in k_contract_split).
constexpr int kPlaneTK = 16;

// Lane l of the conversion writes 16-byte chunk l % 8 (plane (l % 8) / 2,
// complex 8 ((l % 8) % 2) .. + 7 of the slab) of row slab l / 8, so that a
// wave stores 1 KB of contiguous output; the four lanes that need the same
// eight complex inputs read them through the cache.
template <int PREC>
__global__ void __launch_bounds__(256) k_presplit(const float2* src, int64_t rows, int kb,
                                                  const unsigned long long* amax, int amax_n,
                                                  uint16_t* dst) {
  int e = 0;
  if constexpr (PREC == 1) e = fp16_scale_exp(amax, amax_n);
  const float s = ldexpf(1.f, e);
  const int64_t chunks = (rows << kb) >> 1;  // 16-byte output chunks (8 per 16 complex)
  for (int64_t ci = int64_t(blockIdx.x) * 256 + threadIdx.x; ci < chunks;
       ci += int64_t(gridDim.x) * 256) {
    const int c = int(ci & 7);
    const int plane = c >> 1;  // 0 hi re, 1 hi im, 2 lo re, 3 lo im
    const int64_t first = ((ci >> 3) << 4) + 8 * (c & 1);  // flat index of the first complex
    const float4* in = reinterpret_cast<const float4*>(src + first);
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 x = in[q];  // two complex
      uint32_t h0, l0, h1, l1;
      split2<PREC>(((plane & 1) ? x.y : x.x) * s, h0, l0);
      split2<PREC>(((plane & 1) ? x.w : x.z) * s, h1, l1);
      w[q] = (plane < 2) ? (h0 | (h1 << 16)) : (l0 | (l1 << 16));
    }
    reinterpret_cast<u32x4*>(dst)[ci] = u32x4{w[0], w[1], w[2], w[3]};
  }
}

// The GEMM on plane-format operands.  WMT x 2 waves, each a 64 x 64 block
// quad (two 32 x 32 blocks per side, two accumulators per block), so the
// tile is (64 WMT) x 128: tile 6 takes WMT = 2 (128 x 128, four waves, two
// workgroups per CU), tile 7 WMT = 4 (256 x 128, eight waves).  K slabs of
// 16 complex go from global memory straight into LDS (global_load_lds, 16
// bytes per lane: each load instruction of a wave fills 1 KB of LDS, eight
// rows of 128 bytes) through two buffers: while the MFMAs consume slab j,
// the loads of slab j + 1 are in flight, with one barrier per slab.  (A
// third buffer for tile 7, loads two slabs ahead, measured 5-7 % slower.)  Inside a 128-byte row the eight 16-byte chunks (hi re,
// hi im, lo re, lo im; two each) sit at chunk position c ^ (row & 7), so
// that the fragment reads of eight consecutive rows hit distinct banks.
// The epilogue writes 64-row slices of the tile through LDS.  Needs K >= 16
// and no split K.
// s_waitcnt immediate (gfx9 layout: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8) that waits for every vector memory load of the wave and
// for nothing else.
constexpr int kWaitVmcnt0 = (7 << 4) | (15 << 8);
// Word 3 of a raw buffer resource (no format conversion, no swizzle).
constexpr int kBufferFlags = 0x00020000;

template <int PREC, int WMT, int NBUF>
__global__ void __launch_bounds__(128 * WMT, WMT == 2 ? 2 : 1) k_contract_planes(ContractArgs g) {
#if defined(__HIP_DEVICE_COMPILE__)  // buffer resources exist on the device side only
  static_assert(NBUF == 2, "two LDS buffers: slab j + 1 loads while slab j multiplies");
  constexpr int BM = 64 * WMT, BN = 128, TK = kPlaneTK;
  constexpr int NT = 128 * WMT, NW = 2 * WMT;    // threads, waves
  constexpr int ROW_B = 8 * TK;                  // bytes of one row slab (128)
  constexpr int A_B = BM * ROW_B, B_B = BN * ROW_B;
  constexpr int BUF_B = A_B + B_B;
  constexpr int MAIN_F = NBUF * BUF_B / 4;       // floats: the ring
  constexpr int HALF = 64;                       // epilogue rows per pass
  constexpr int EPI_F = HALF * (BN + 1) * 2;
  constexpr int LDS_F = MAIN_F > EPI_F ? MAIN_F : EPI_F;
  constexpr int LA = A_B / 1024 / NW, LB = B_B / 1024 / NW;  // loads per wave and slab
  static_assert(LA * NW * 1024 == A_B && LB * NW * 1024 == B_B, "whole 1 KB blocks per wave");
  typedef float accv __attribute__((ext_vector_type(16)));
  __shared__ __attribute__((aligned(1024))) float smem[LDS_F];
  __shared__ int64_t dep_m_lo[HALF];
  __shared__ int64_t dep_n_lo[BN];
  char* lds = reinterpret_cast<char*>(smem);
  float2* Ct = reinterpret_cast<float2*>(smem);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // rows 64 wm .., columns 64 wn ..
  const TileMap<BM, BN> tmap(g);
  const int64_t tiles = tmap.tiles;
  const int64_t per_xcd = (tiles + 7) / 8;
  const int64_t walk = per_xcd * 8;
  const int nslabs = int((int64_t(1) << g.kb) / TK);
  const uint64_t row_bytes = uint64_t(8) << g.kb;  // 4 planes x K halves

  int eA = 0, eB = 0;
  if constexpr (PREC == 1) {
    eA = fp16_scale_exp(g.amaxA, g.amax_nA);
    eB = fp16_scale_exp(g.amaxB, g.amax_nB);
  }
  const float s_out = ldexpf(1.f, -(eA + eB));
  float amax = 0.f;

  int r_tid = 0, c_tid = 0;
  epilogue_setup<7, NT>(g, dep_m_lo, dep_n_lo, r_tid, c_tid);
  __syncthreads();

  auto item_of = [&](int64_t p) -> int64_t { return (p & 7) * per_xcd + (p >> 3); };
  auto next_p = [&](int64_t p) -> int64_t {
    for (p += gridDim.x; p < walk; p += gridDim.x)
      if (item_of(p) < tiles) return p;
    return walk;
  };

  const char* Ap = reinterpret_cast<const char*>(g.Ap);
  const char* Bp = reinterpret_cast<const char*>(g.Bp);
  // Lane l of the wave's load into 1 KB block b fills its bytes 16 l: row
  // 8 b + l / 8, position l % 8, i.e. chunk (l % 8) ^ (row % 8) of the row.
  const int lrow = lane >> 3, lpos = lane & 7;
  // Loads as buffer loads into LDS: per tile one buffer resource per operand
  // (base = the tile's first row; its rows fit 2^31 bytes, K <= 2^18), a
  // 32-bit offset per lane and load fixed for the tile (rows past the end
  // clamp to the last row), and the slab offset as the scalar offset.
  uint32_t offLA[LA], offLB[LB];
  __amdgpu_buffer_rsrc_t rsA, rsB;
  auto tile_rows = [&](const TileOrigin& o) {
    const int64_t la = o.row_end - o.row0 - 1, lb = o.col_end - o.col0 - 1;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int blk = NW * i + wave, r = 8 * blk + lrow;
      offLA[i] = uint32_t(r < la ? r : la) * uint32_t(row_bytes) + 16u * uint32_t(lpos ^ (r & 7));
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int blk = NW * i + wave, r = 8 * blk + lrow;
      offLB[i] = uint32_t(r < lb ? r : lb) * uint32_t(row_bytes) + 16u * uint32_t(lpos ^ (r & 7));
    }
    rsA = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(Ap + uint64_t(o.row0) * row_bytes), 0,
                                            int(uint32_t(BM) * uint32_t(row_bytes)), kBufferFlags);
    rsB = __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(Bp + uint64_t(o.col0) * row_bytes), 0,
                                            int(uint32_t(BN) * uint32_t(row_bytes)), kBufferFlags);
  };
  auto issue = [&](int j, int buf) {
    char* dst = lds + buf * BUF_B;
#pragma unroll
    for (int i = 0; i < LA; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsA, (__attribute__((address_space(3))) void*)(dst + 1024 * (NW * i + wave)), 16, offLA[i],
          j * ROW_B, 0, 0);
#pragma unroll
    for (int i = 0; i < LB; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsB, (__attribute__((address_space(3))) void*)(dst + A_B + 1024 * (NW * i + wave)), 16, offLB[i],
          j * ROW_B, 0, 0);
  };
  // The 16 fragments of one slab: ar[fm][pl] = A row 64 wm + 32 fm + (lane %
  // 32), chunk 2 pl + lane / 32; br[fn][pl] the same for B row 64 wn + 32 fn
  // + (lane % 32).  Chunk c of row r sits at byte 16 (c ^ (r % 8)) of the
  // row, and r % 8 = lane % 8 for every fragment.
  const int li = lane & 31, lg = lane >> 5;
  int offA[4], offB[4];
#pragma unroll
  for (int pl = 0; pl < 4; ++pl) {
    const int chunk = 16 * ((2 * pl + lg) ^ (li & 7));
    offA[pl] = (wm * 64 + li) * ROW_B + chunk;
    offB[pl] = A_B + (wn * 64 + li) * ROW_B + chunk;
  }
  auto read_frags = [&](const char* buf, u32x4 (&ar)[2][4], u32x4 (&br)[2][4]) {
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        ar[f][pl] = *reinterpret_cast<const u32x4*>(buf + offA[pl] + f * 32 * ROW_B);
        br[f][pl] = *reinterpret_cast<const u32x4*>(buf + offB[pl] + f * 32 * ROW_B);
      }
  };

  int64_t p = blockIdx.x;
  if (p < walk && item_of(p) >= tiles) p = next_p(p);
  while (p < walk) {
    const TileOrigin o = tmap.at(g, item_of(p));
    const int64_t pn = next_p(p);
    accv acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
      for (int fn = 0; fn < 2; ++fn)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc_re[fm][fn][v] = acc_im[fm][fn][v] = 0.f;

    // Per slab j: wait for this wave's loads of slab j, barrier (slab j is in
    // LDS everywhere, and nobody reads slab j - 1's buffer any more), all
    // fragments of slab j into registers, the loads of slab j + 1 into the
    // other buffer, then the MFMAs.  The compiler makes an LDS read wait for
    // every LDS-bound load in flight (it cannot tell the buffers apart), so
    // the reads come before the next slab's loads are issued; those then
    // overlap the MFMAs.
    tile_rows(o);
    issue(0, 0);
    for (int j = 0; j < nslabs; ++j) {
      // The barrier's fence does not wait for loads: wait for this wave's
      // loads of slab j explicitly before it.
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      __syncthreads();
      u32x4 ar[2][4], br[2][4];
      read_frags(lds + (j & 1) * BUF_B, ar, br);
      if (j + 1 < nslabs) issue(j + 1, (j + 1) & 1);
#pragma unroll
      for (int fn = 0; fn < 2; ++fn) {
        const u32x4 brh = br[fn][0], bih = br[fn][1], brl = br[fn][2], bil = br[fn][3];
        const u32x4 nbih = bih ^ 0x80008000u, nbil = bil ^ 0x80008000u;
#pragma unroll
        for (int fm = 0; fm < 2; ++fm) {
#define XEB_MMA(acc, x, y) acc = mma_split<32, PREC>(x, y, acc)
          XEB_MMA(acc_re[fm][fn], ar[fm][0], brh);
          XEB_MMA(acc_im[fm][fn], ar[fm][0], bih);
          XEB_MMA(acc_re[fm][fn], ar[fm][1], nbih);
          XEB_MMA(acc_im[fm][fn], ar[fm][1], brh);
          XEB_MMA(acc_re[fm][fn], ar[fm][0], brl);
          XEB_MMA(acc_im[fm][fn], ar[fm][0], bil);
          XEB_MMA(acc_re[fm][fn], ar[fm][1], nbil);
          XEB_MMA(acc_im[fm][fn], ar[fm][1], brl);
          XEB_MMA(acc_re[fm][fn], ar[fm][2], brh);
          XEB_MMA(acc_im[fm][fn], ar[fm][2], bih);
          XEB_MMA(acc_re[fm][fn], ar[fm][3], nbih);
          XEB_MMA(acc_im[fm][fn], ar[fm][3], brh);
#undef XEB_MMA
        }
      }
    }
    __syncthreads();  // every wave is done with the ring

    // Epilogue in passes of 64 rows: the waves holding rows 64 h .. 64 h + 63
    // park them, then all threads write them out.
#pragma unroll
    for (int h = 0; h < WMT; ++h) {
      if (wm == h) {
#pragma unroll
        for (int fm = 0; fm < 2; ++fm)
#pragma unroll
          for (int fn = 0; fn < 2; ++fn)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int r = fm * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
              const int c = wn * 64 + fn * 32 + (lane & 31);
              Ct[r * (BN + 1) + c] =
                  make_float2(acc_re[fm][fn][v] * s_out, acc_im[fm][fn][v] * s_out);
            }
      }
      __syncthreads();
      amax = fmaxf(amax, epilogue_write<7, NT>(g, Ct, o.row0 + HALF * h, o.col0, o.key, o.row_end,
                                               o.col_end, dep_m_lo, dep_n_lo, r_tid, c_tid));
      __syncthreads();
    }
    p = pn;
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
#endif
}

// Split-K chunk sum: partial[0] += partial[1] + ... + partial[ksplit - 1],
// element by element in chunk order (deterministic), two complex per thread.
__global__ void __launch_bounds__(256) k_splitk_sum(float4* partial, int64_t chunk_f4, int ksplit) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < chunk_f4;
       i += int64_t(gridDim.x) * 256) {
    float4 acc = partial[i];
    int kc = 1;
    for (; kc + 4 <= ksplit; kc += 4) {
      const float4 a = partial[(kc + 0) * chunk_f4 + i], b = partial[(kc + 1) * chunk_f4 + i];
      const float4 c = partial[(kc + 2) * chunk_f4 + i], d = partial[(kc + 3) * chunk_f4 + i];
      acc.x += a.x; acc.y += a.y; acc.z += a.z; acc.w += a.w;
      acc.x += b.x; acc.y += b.y; acc.z += b.z; acc.w += b.w;
      acc.x += c.x; acc.y += c.y; acc.z += c.z; acc.w += c.w;
      acc.x += d.x; acc.y += d.y; acc.z += d.z; acc.w += d.w;
    }
    for (; kc < ksplit; ++kc) {
      const float4 a = partial[kc * chunk_f4 + i];
      acc.x += a.x; acc.y += a.y; acc.z += a.z; acc.w += a.w;
    }
    partial[i] = acc;
  }
}

// Split-K epilogue: each summed tile (chunk 0 of the partials) through LDS to
// the output in the contraction's write order.  Grid-stride over tiles.
template <int CFG>
__global__ void __launch_bounds__(256) k_splitk_reduce(ContractArgs g) {
  using T = TileInfo<CFG, 0>;
  constexpr int BM = T::BM, BN = T::BN;
  __shared__ float2 Ct[BM * (BN + 1)];
  __shared__ int64_t dep_m_lo[BM];
  __shared__ int64_t dep_n_lo[BN];
  const TileMap<BM, BN> tmap(g);
  const int64_t tiles = tmap.tiles;
  int r_tid = 0, c_tid = 0;
  epilogue_setup<CFG>(g, dep_m_lo, dep_n_lo, r_tid, c_tid);
  float amax = 0.f;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    for (int e = threadIdx.x; e < BM * BN; e += 256)
      Ct[(e / BN) * (BN + 1) + (e % BN)] = g.partial[tile * (BM * BN) + e];
    __syncthreads();
    int64_t row0, col0, key, row_end, col_end;
    tmap.origin(g, tile, row0, col0, key, row_end, col_end);
    amax = fmaxf(amax, epilogue_write<CFG>(g, Ct, row0, col0, key, row_end, col_end, dep_m_lo, dep_n_lo, r_tid, c_tid));
    __syncthreads();
  }
  if (g.amax_out) publish_amax(amax, g.amax_out, g.epoch);
}

// ---------------------------------------------------------------------------
__global__ void k_zero(uint32_t* p, uint64_t words) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

// Thread t adds value o = t mod 2^w of group g = t / 2^w.
__global__ void k_accumulate(const float2* partial, const int32_t* idx, const int32_t* eoff,
                             const int32_t* rho, const int32_t* slo, int64_t base, int64_t lo,
                             int64_t hi, double2* amps, double2* comp, int64_t n, int w) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t g = t >> w;
  if (g >= n) return;
  const int64_t o = t & ((int64_t(1) << w) - 1);
  const int64_t i = (int64_t(idx[g]) << w) + o;
  double2 s = amps[i], c = comp[i];
  for (int32_t j = eoff[g], end = eoff[g + 1]; j < end; ++j) {
    const int64_t sigma = base + slo[j];
    if (sigma < lo || sigma >= hi) continue;
    const float2 p = partial[(int64_t(rho[j]) << w) + o];
    neumaier(s.x, c.x, double(p.x));
    neumaier(s.y, c.y, double(p.y));
  }
  amps[i] = s;
  comp[i] = c;
}

__global__ void k_gather_own(const double2* amps, const int32_t* sel, int w, double2* own, int64_t k) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= k) return;
  own[i] = amps[(i << w) + sel[i]];
}

__global__ void k_fold(double2* amps, const double2* comp, int64_t k) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double2 s = amps[i];
  const double2 c = comp[i];
  s.x += c.x;
  s.y += c.y;
  amps[i] = s;
}

struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
thread_local LaunchEvents g_events;

// Launches `kernel`; `first` / `last` mark its place in a timed group.
template <typename... KArgs, typename... Args>
void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, bool first, bool last,
            Args... args) {
  hipEvent_t a = first ? g_events.start : nullptr;
  hipEvent_t b = last ? g_events.stop : nullptr;
  if (a || b) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, static_cast<KArgs>(args)...);
    if (a) g_events.start = nullptr;
    if (b) g_events.stop = nullptr;
  } else {
    kernel<<<grid, block, 0, s>>>(static_cast<KArgs>(args)...);
  }
}

inline int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 262144) g = 262144;
  return int(g);
}

}  // namespace

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_events.start = start;
  g_events.stop = stop;
}

void take_launch_events(hipEvent_t* start, hipEvent_t* stop) {
  *start = g_events.start;
  *stop = g_events.stop;
  g_events = LaunchEvents{};
}

void launch_contract_generic(const ContractArgs& a, hipStream_t s) {
  const int64_t total = a.nvar << (a.mb + a.nb);
  if (total <= 0) return;
  if (a.tile == 1) {
    const int sbits = a.swapped ? a.mb : a.nb, bbits = a.swapped ? a.nb : a.mb;
    if (!generic_rows_fit(a.kb, sbits, bbits))
      throw std::runtime_error("row-streaming form launched on a node it does not fit");
    // Four stream rows per thread, unless that leaves too few work items to
    // fill the chip.
    int lu = sbits >= 8 + kRowsLog2U ? kRowsLog2U : 0;
    if (lu && (a.nvar << (sbits - 8 - lu)) < kRowsMinItems) lu = 0;
    const int64_t items = a.nvar << (sbits - 8 - lu);
    const int grid = int(std::min<int64_t>(items, a.amax_out ? 4096 : (int64_t(1) << 20)));
#define XEB_ROWS_CASE(KB)                                                                   \
  case KB:                                                                                 \
    if (lu)                                                                                \
      launch(k_contract_rows<KB, 1 << kRowsLog2U>, dim3(grid), dim3(256), s, true, true, a); \
    else                                                                                   \
      launch(k_contract_rows<KB, 1>, dim3(grid), dim3(256), s, true, true, a);              \
    break;
    switch (a.kb) {
      XEB_ROWS_CASE(0)
      XEB_ROWS_CASE(1)
      XEB_ROWS_CASE(2)
      XEB_ROWS_CASE(3)
      XEB_ROWS_CASE(4)
      default: break;
    }
#undef XEB_ROWS_CASE
    return;
  }
  // Tracking the FP16 scale costs one atomic per workgroup: keep the grid at
  // a few workgroups per CU then (grid-stride loop).  With a key spanning
  // whole 256-element chunks a workgroup takes one chunk per step.
  int grid = grid_for(total, 256);
  if (a.mb + a.nb >= 8 + kGenericLog2U) grid = int((int64_t(grid) + (1 << kGenericLog2U) - 1) >> kGenericLog2U);
  if (a.amax_out && grid > 4096) grid = 4096;
  switch (a.kb) {
    case 0: launch(k_contract_generic<0>, dim3(grid), dim3(256), s, true, true, a); break;
    case 1: launch(k_contract_generic<1>, dim3(grid), dim3(256), s, true, true, a); break;
    case 2: launch(k_contract_generic<2>, dim3(grid), dim3(256), s, true, true, a); break;
    case 3: launch(k_contract_generic<3>, dim3(grid), dim3(256), s, true, true, a); break;
    case 4: launch(k_contract_generic<4>, dim3(grid), dim3(256), s, true, true, a); break;
    default: launch(k_contract_generic<-1>, dim3(grid), dim3(256), s, true, true, a); break;
  }
}

namespace {

template <int CFG, int PREC, int TKV, int KG>
unsigned persistent_grid(int64_t tiles) {
  // Resident workgroups per device for this kernel, queried once per device.
  static int cached[64] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  int& slot = cached[dev & 63];
  if (slot == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    hipError_t e;
    if constexpr (PREC == 0)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_contract_mfma<CFG, PREC, TKV, KG>, 256 * KG, 0);
    else if constexpr (CFG == 5)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_contract_split_db<PREC>, 512, 0);
    else if constexpr (CFG == 6)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_contract_planes<PREC, 2, 2>, 256, 0);
    else if constexpr (CFG == 8)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_contract_planes<PREC, 4, 2>, 512, 0);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_contract_split<CFG, PREC, TKV, KG>, 256 * KG, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    slot = cus * per_cu;
  }
  // The walk covers ceil(tiles / 8) * 8 positions; a multiple of 8 keeps each
  // workgroup on one XCD's share.
  const int64_t walk = ((tiles + 7) / 8) * 8;
  const int64_t g = walk < slot ? walk : slot;
  return unsigned(g < 1 ? 1 : g);
}

// Tiles of a launch (see TileMap).
int64_t launch_tiles(const ContractArgs& a, int bm, int bn) {
  if (a.pair_mode == 2)
    return a.nvar * ((((int64_t(1) << a.mb) + bm - 1) / bm) * (((int64_t(1) << a.nb) + bn - 1) / bn));
  const int64_t rowsA = a.nvarA << a.mb, rowsB = a.nvarB << a.nb;
  return ((rowsA + bm - 1) / bm) * ((rowsB + bn - 1) / bn);
}

template <int CFG, int PREC, int TKV, int KG = 1>
void launch_cfg(const ContractArgs& a, hipStream_t s, int64_t rowsA, int64_t rowsB) {
  using T = TileInfo<CFG, PREC, TKV>;
  (void)rowsA, (void)rowsB;
  const int64_t tiles = launch_tiles(a, T::BM, T::BN);
  if constexpr (PREC == 0)
    launch(k_contract_mfma<CFG, PREC, TKV, KG>, dim3(persistent_grid<CFG, PREC, TKV, KG>(tiles * a.ksplit)),
           dim3(256 * KG), s, true, true, a);
  else if constexpr (CFG == 5)
    launch(k_contract_split_db<PREC>, dim3(persistent_grid<CFG, PREC, TKV, KG>(tiles * a.ksplit)), dim3(512),
           s, true, true, a);
  else if constexpr (CFG == 6 || CFG == 8) {
    // Both operands into plane format, then the GEMM.
    const int64_t rowsA = a.nvarA << a.mb, rowsB = a.nvarB << a.nb;
    const int64_t chunksA = (rowsA << a.kb) >> 1, chunksB = (rowsB << a.kb) >> 1;
    launch(k_presplit<PREC>, dim3(grid_for(chunksA, 256) < 16384 ? grid_for(chunksA, 256) : 16384), dim3(256),
           s, true, false, a.A, rowsA, int(a.kb), a.amaxA, a.amax_nA, a.Ap);
    launch(k_presplit<PREC>, dim3(grid_for(chunksB, 256) < 16384 ? grid_for(chunksB, 256) : 16384), dim3(256),
           s, false, false, a.B, rowsB, int(a.kb), a.amaxB, a.amax_nB, a.Bp);
    if constexpr (CFG == 6)
      launch(k_contract_planes<PREC, 2, 2>, dim3(persistent_grid<CFG, PREC, TKV, KG>(tiles)), dim3(256), s,
             false, true, a);
    else
      launch(k_contract_planes<PREC, 4, 2>, dim3(persistent_grid<CFG, PREC, TKV, KG>(tiles)), dim3(512), s,
             false, true, a);
  }
  else
    launch(k_contract_split<CFG, PREC, TKV, KG>, dim3(persistent_grid<CFG, PREC, TKV, KG>(tiles * a.ksplit)),
           dim3(256 * KG), s, true, true, a);
}

template <int CFG>
void launch_reduce_cfg(const ContractArgs& a, hipStream_t s, int64_t rowsA, int64_t rowsB) {
  using T = TileInfo<CFG, 0>;
  (void)rowsA, (void)rowsB;
  const int64_t tiles = launch_tiles(a, T::BM, T::BN);
  const int64_t chunk_f4 = tiles * T::BM * T::BN / 2;
  launch(k_splitk_sum, dim3(grid_for(chunk_f4, 256)), dim3(256), s, true, false,
         reinterpret_cast<float4*>(a.partial), chunk_f4, a.ksplit);
  const int64_t grid = tiles < 4096 ? tiles : 4096;
  launch(k_splitk_reduce<CFG>, dim3(unsigned(grid)), dim3(256), s, false, true, a);
}

// The (tile, precision, K slab) combinations that are instantiated.
template <int PREC>
void launch_prec(const ContractArgs& a, hipStream_t s, int64_t rowsA, int64_t rowsB) {
  constexpr int lo = PREC == 0 ? 16 : 32, hi = 2 * lo;
  if (a.tile == 0) {
    if (a.kg == 2) {
      if (a.tk == hi) launch_cfg<0, PREC, hi, 2>(a, s, rowsA, rowsB);
      else launch_cfg<0, PREC, lo, 2>(a, s, rowsA, rowsB);
    } else {
      if (a.tk == hi) launch_cfg<0, PREC, hi>(a, s, rowsA, rowsB);
      else launch_cfg<0, PREC, lo>(a, s, rowsA, rowsB);
    }
  } else if (a.tile == 1) {
    if constexpr (PREC == 0) {
      if (a.tk == hi) {
        launch_cfg<1, 0, hi>(a, s, rowsA, rowsB);
        return;
      }
    }
    launch_cfg<1, PREC, lo>(a, s, rowsA, rowsB);
  } else if (a.tile == 4) {
    launch_cfg<4, PREC, lo>(a, s, rowsA, rowsB);
  } else if (a.tile == 5) {
    if constexpr (PREC != 0) launch_cfg<5, PREC, 16>(a, s, rowsA, rowsB);
  } else if (a.tile == 6) {
    if constexpr (PREC != 0) launch_cfg<6, PREC, 16>(a, s, rowsA, rowsB);
  } else if (a.tile == 7) {
    if constexpr (PREC != 0) launch_cfg<8, PREC, 16>(a, s, rowsA, rowsB);
  } else {
    if (a.tile == 3)
      launch_cfg<3, PREC, lo>(a, s, rowsA, rowsB);
    else
      launch_cfg<2, PREC, lo>(a, s, rowsA, rowsB);
  }
}

}  // namespace

void launch_contract_mfma(const ContractArgs& a, hipStream_t s) {
  const int64_t rowsA = a.nvarA << a.mb;
  const int64_t rowsB = a.nvarB << a.nb;
  if (rowsA <= 0 || rowsB <= 0) return;
  if (!mfma_variant_allowed(a.tile, a.prec, a.tk, a.kg))
    throw std::invalid_argument("MFMA variant not instantiated");
  if (a.kb < 1 || a.kb > 21) throw std::invalid_argument("MFMA kernels take 2 <= K <= 2^21");
  if (a.pair_mode == 2) {
    int bm = 0, bn = 0;
    mfma_tile_shape(a.tile, &bm, &bn);
    if (!a.lidx || !a.ridx || (int64_t(2) << a.mb) < bm || (int64_t(2) << a.nb) < bn || a.ksplit != 1)
      throw std::invalid_argument("keyed MFMA form needs index arrays, keys of at least half a tile side, no split K");
  }
  if (a.ksplit < 1 || (a.ksplit > 1 && (!a.partial || (int64_t(1) << a.kb) % (int64_t(a.ksplit) * a.tk))))
    throw std::invalid_argument("split K needs a partial buffer and chunks of whole K slabs");
  if ((a.tile == 6 || a.tile == 7) && (a.ksplit != 1 || a.kb < 4 || !a.Ap || !a.Bp))
    throw std::invalid_argument("plane-format tiles need K >= 16, no split K and plane buffers");
  if (a.prec == 0)
    launch_prec<0>(a, s, rowsA, rowsB);
  else if (a.prec == 1)
    launch_prec<1>(a, s, rowsA, rowsB);
  else
    launch_prec<2>(a, s, rowsA, rowsB);
}

void launch_splitk_reduce(const ContractArgs& a, hipStream_t s) {
  const int64_t rowsA = a.nvarA << a.mb;
  const int64_t rowsB = a.nvarB << a.nb;
  if (rowsA <= 0 || rowsB <= 0 || a.ksplit <= 1) return;
  if (!a.partial) throw std::invalid_argument("split K needs a partial buffer");
  if (a.tile == 0)
    launch_reduce_cfg<0>(a, s, rowsA, rowsB);
  else if (a.tile == 1)
    launch_reduce_cfg<1>(a, s, rowsA, rowsB);
  else if (a.tile == 2)
    launch_reduce_cfg<2>(a, s, rowsA, rowsB);
  else if (a.tile == 3)
    launch_reduce_cfg<3>(a, s, rowsA, rowsB);
  else if (a.tile == 4)
    launch_reduce_cfg<4>(a, s, rowsA, rowsB);
  else
    launch_reduce_cfg<5>(a, s, rowsA, rowsB);
}

bool mfma_variant_allowed(int tile, int prec, int tk, int kg) {
  if (tile >= 5) return prec != 0 && tk == 16 && kg == 1;
  if (kg != 1 && !(kg == 2 && tile == 0)) return false;
  const int lo = prec == 0 ? 16 : 32;
  if (tk == lo) return tile >= 0 && tile <= 4;
  if (tk == 2 * lo) return tile == 0 || (prec == 0 && tile == 1);
  return false;
}

int mfma_default_slab(int prec) { return prec == 0 ? 16 : 32; }

void prepare_mfma_launch(int prec) {
  if (prec == 0) {
    (void)persistent_grid<0, 0, 16, 1>(1), (void)persistent_grid<1, 0, 16, 1>(1);
    (void)persistent_grid<2, 0, 16, 1>(1), (void)persistent_grid<0, 0, 32, 1>(1);
    (void)persistent_grid<3, 0, 16, 1>(1), (void)persistent_grid<4, 0, 16, 1>(1);
    (void)persistent_grid<1, 0, 32, 1>(1), (void)persistent_grid<0, 0, 16, 2>(1);
    (void)persistent_grid<0, 0, 32, 2>(1);
  } else if (prec == 1) {
    (void)persistent_grid<0, 1, 32, 1>(1), (void)persistent_grid<1, 1, 32, 1>(1);
    (void)persistent_grid<2, 1, 32, 1>(1), (void)persistent_grid<0, 1, 64, 1>(1);
    (void)persistent_grid<3, 1, 32, 1>(1), (void)persistent_grid<4, 1, 32, 1>(1);
    (void)persistent_grid<5, 1, 16, 1>(1), (void)persistent_grid<6, 1, 16, 1>(1);
    (void)persistent_grid<8, 1, 16, 1>(1);
    (void)persistent_grid<0, 1, 32, 2>(1), (void)persistent_grid<0, 1, 64, 2>(1);
  } else {
    (void)persistent_grid<0, 2, 32, 1>(1), (void)persistent_grid<1, 2, 32, 1>(1);
    (void)persistent_grid<2, 2, 32, 1>(1), (void)persistent_grid<0, 2, 64, 1>(1);
    (void)persistent_grid<3, 2, 32, 1>(1), (void)persistent_grid<4, 2, 32, 1>(1);
    (void)persistent_grid<5, 2, 16, 1>(1), (void)persistent_grid<6, 2, 16, 1>(1);
    (void)persistent_grid<8, 2, 16, 1>(1);
    (void)persistent_grid<0, 2, 32, 2>(1), (void)persistent_grid<0, 2, 64, 2>(1);
  }
}

void mfma_tile_shape(int tile, int* bm, int* bn) {
  static const int kBM[kMfmaTiles] = {64, 32, 16, 64, 128, 128, 128, 256};
  static const int kBN[kMfmaTiles] = {64, 128, 256, 16, 128, 128, 128, 128};
  const int t = tile >= 0 && tile < kMfmaTiles ? tile : 0;
  *bm = kBM[t];
  *bn = kBN[t];
}

int64_t mfma_tiles(int tile, int64_t rowsA, int64_t rowsB) {
  int bm = 0, bn = 0;
  mfma_tile_shape(tile, &bm, &bn);
  return ((rowsA + bm - 1) / bm) * ((rowsB + bn - 1) / bn);
}

void launch_zero(void* p, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  if (words == 0) return;
  k_zero<<<grid_for(int64_t(words), 256), 256, 0, s>>>(static_cast<uint32_t*>(p), words);
}

void launch_accumulate(const float2* partial, const int32_t* idx, const int32_t* eoff,
                       const int32_t* rho, const int32_t* slo, int64_t base, int64_t lo,
                       int64_t hi, double2* amps, double2* comp, int64_t n, int w, hipStream_t s) {
  if (n <= 0) return;
  launch(k_accumulate, dim3(grid_for(n << w, 256)), dim3(256), s, true, true, partial, idx, eoff,
         rho, slo, base, lo, hi, amps, comp, n, w);
}

void launch_gather_own(const double2* amps, const int32_t* sel, int w, double2* own, int64_t k,
                       hipStream_t s) {
  if (k <= 0) return;
  k_gather_own<<<grid_for(k, 256), 256, 0, s>>>(amps, sel, w, own, k);
}

void launch_fold_compensation(double2* amps, const double2* comp, int64_t k, hipStream_t s) {
  if (k <= 0) return;
  k_fold<<<grid_for(k, 256), 256, 0, s>>>(amps, comp, k);
}

}  // namespace xeb
