// gfx950 kernels of the multi-tensor contraction.
//
// * contract_generic: one thread per output element of every variant; the
//   path for small or sparse nodes (latency-bound).
// * contract_mfma: the variants of L stacked as rows (nvarA * 2^mb rows of
//   2^kb complex) times the variants of R stacked as rows, on FP32 MFMA
//   (v_mfma_f32_32x32x2_f32).  A complex product takes two MFMAs per complex
//   k: the instruction's K = 2 runs over (re, im) of the row operand, and the
//   column operand supplies (re, -im) for the real part and (im, re) for the
//   imaginary part, so every complex MAC costs exactly 4 real MACs.
//   The epilogue scatters each output element straight into the layout the
//   parent node reads (bit deposit), so no separate transpose pass exists.
// * accumulate / fold_compensation: FP64 Neumaier sum over slices.
// * xeb: compensated FP64 reduction of sum |amp|^2 in a fixed order.

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace xeb {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int64_t deposit(int64_t x, const int8_t* pos, int nbits) {
  int64_t r = 0;
  for (int j = 0; j < nbits; ++j) r |= ((x >> j) & 1) << pos[j];
  return r;
}

// ---------------------------------------------------------------------------
// Generic contraction.
__global__ void __launch_bounds__(256) k_contract_generic(ContractArgs g) {
  const int mn = g.mb + g.nb;
  const int64_t per = int64_t(1) << mn;
  const int64_t total = g.nvar * per;
  const int64_t K = int64_t(1) << g.kb;
  const int64_t sizeA = int64_t(1) << (g.mb + g.kb);
  const int64_t sizeB = int64_t(1) << (g.nb + g.kb);
  const int64_t mmask = (int64_t(1) << g.mb) - 1;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t a = e >> mn;
    const int64_t rem = e & (per - 1);
    const int64_t m = rem & mmask;
    const int64_t n = rem >> g.mb;
    const float2* pa = g.A + int64_t(g.lidx[a]) * sizeA + (m << g.kb);
    const float2* pb = g.B + int64_t(g.ridx[a]) * sizeB + (n << g.kb);
    float re = 0.f, im = 0.f;
    for (int64_t k = 0; k < K; ++k) {
      const float2 x = pa[k], y = pb[k];
      re += x.x * y.x - x.y * y.y;
      im += x.x * y.y + x.y * y.x;
    }
    g.C[a * per + deposit(m, g.posM, g.mb) + deposit(n, g.posN, g.nb)] = make_float2(re, im);
  }
}

// ---------------------------------------------------------------------------
// MFMA contraction.  Workgroup tile BM x BN complex (64 x 64 or 32 x 128), four
// waves, each one 32 x 32 block of v_mfma_f32_32x32x2f32.  K is staged through
// LDS TK = 16 complex at a time as separate re / im planes [k][plane][row]
// (+1 float padding); the next K tile is fetched into registers (16-byte loads,
// consecutive lanes along one contiguous row) while the current one is
// multiplied.  The epilogue parks the tile in LDS and writes it out in the
// order of the output layout's bit positions (ubit), so a wave stores runs of
// consecutive addresses.
constexpr int TK = 16, PAD = 1;

template <int BM, int BN>
struct Tile {
  static constexpr int WM = BM / 32;
  static constexpr int WN = 4 / WM;
  static_assert(WN * 32 == BN, "four 32x32 wave blocks per tile");
  static constexpr int A_VEC = BM * TK / 2 / 256;
  static constexpr int B_VEC = BN * TK / 2 / 256;
  static constexpr int LDS_A = TK * 2 * (BM + PAD);
  static constexpr int LDS_MAIN = LDS_A + TK * 2 * (BN + PAD);
  static constexpr int LDS_EPI = BM * (BN + 1) * 2;
  static constexpr int LDS = LDS_MAIN > LDS_EPI ? LDS_MAIN : LDS_EPI;
  static constexpr int UBITS = (BM == 64 ? 6 : 5) + (BN == 64 ? 6 : 7);
  static constexpr int PER_THREAD = BM * BN / 256;
};

template <int BM, int BN>
__global__ void __launch_bounds__(256) k_contract_mfma(ContractArgs g) {
  using T = Tile<BM, BN>;
  __shared__ float smem[T::LDS];
  __shared__ int64_t dep_m_lo[BM];
  __shared__ int64_t dep_n_lo[BN];
  float(*As)[2][BM + PAD] = reinterpret_cast<float(*)[2][BM + PAD]>(smem);
  float(*Bs)[2][BN + PAD] = reinterpret_cast<float(*)[2][BN + PAD]>(smem + T::LDS_A);
  float2* Ct = reinterpret_cast<float2*>(smem);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const int64_t rowsA = g.nvarA << g.mb;
  const int64_t rowsB = g.nvarB << g.nb;
  const int64_t tiles_n = (rowsB + BN - 1) / BN;
  const int64_t tiles = tiles_n * ((rowsA + BM - 1) / BM);
  const int64_t K = int64_t(1) << g.kb;
  const int64_t M = int64_t(1) << g.mb;
  const int64_t N = int64_t(1) << g.nb;
  const int64_t sizeC = M * N;
  const int64_t m_lo_mask = (M < BM ? M : BM) - 1;
  const int64_t n_lo_mask = (N < BN ? N : BN) - 1;

  for (int i = tid; i < BM; i += 256) dep_m_lo[i] = deposit(i & m_lo_mask, g.posM, g.mb);
  for (int i = tid; i < BN; i += 256) dep_n_lo[i] = deposit(i & n_lo_mask, g.posN, g.nb);
  // Row / column inside the tile of this thread's epilogue elements: bits 0..7
  // of the element number come from tid, the rest from the loop counter.
  int r_tid = 0, c_tid = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if ((tid >> b) & 1) {
      const int u = g.ubit[b];
      if (u < 32)
        r_tid |= 1 << u;
      else
        c_tid |= 1 << (u - 32);
    }
  }
  __syncthreads();

  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row0 = (tile / tiles_n) * BM;
    const int64_t col0 = (tile % tiles_n) * BN;

    floatx16 acc_re, acc_im;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc_re[v] = 0.f;
      acc_im[v] = 0.f;
    }

    float4 ra[T::A_VEC], rb[T::B_VEC];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int t = 0; t < T::A_VEC; ++t) {
        const int e = tid + t * 256;
        const int r = e / (TK / 2), kp = e % (TK / 2);
        const int64_t gr = row0 + r, gk = k0 + 2 * kp;
        ra[t] = (gr < rowsA && gk < K)
                    ? *reinterpret_cast<const float4*>(g.A + (gr << g.kb) + gk)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int t = 0; t < T::B_VEC; ++t) {
        const int e = tid + t * 256;
        const int r = e / (TK / 2), kp = e % (TK / 2);
        const int64_t gr = col0 + r, gk = k0 + 2 * kp;
        rb[t] = (gr < rowsB && gk < K)
                    ? *reinterpret_cast<const float4*>(g.B + (gr << g.kb) + gk)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    fetch(0);
    for (int64_t k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
      for (int t = 0; t < T::A_VEC; ++t) {
        const int e = tid + t * 256;
        const int r = e / (TK / 2), kk = 2 * (e % (TK / 2));
        As[kk][0][r] = ra[t].x;
        As[kk][1][r] = ra[t].y;
        As[kk + 1][0][r] = ra[t].z;
        As[kk + 1][1][r] = ra[t].w;
      }
#pragma unroll
      for (int t = 0; t < T::B_VEC; ++t) {
        const int e = tid + t * 256;
        const int r = e / (TK / 2), kk = 2 * (e % (TK / 2));
        Bs[kk][0][r] = rb[t].x;
        Bs[kk][1][r] = rb[t].y;
        Bs[kk + 1][0][r] = rb[t].z;
        Bs[kk + 1][1][r] = rb[t].w;
      }
      __syncthreads();
      if (k0 + TK < K) fetch(k0 + TK);
      const int i = lane & 31;
      const int half = lane >> 5;  // 0: real part of the K = 2 pair, 1: imaginary
#pragma unroll
      for (int kk = 0; kk < TK; ++kk) {
        const float a = As[kk][half][wm * 32 + i];
        const float bre = Bs[kk][0][wn * 32 + i];
        const float bim = Bs[kk][1][wn * 32 + i];
        const float b_for_re = half ? -bim : bre;
        const float b_for_im = half ? bre : bim;
        acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b_for_re, acc_re, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b_for_im, acc_im, 0, 0, 0);
      }
      __syncthreads();
    }

    // Park the tile: lane l, register v of the MFMA result hold row
    // (v % 4) + 4 (l / 32) + 8 (v / 4), column l % 32 of the wave's block.
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = wm * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
      const int c = wn * 32 + (lane & 31);
      Ct[r * (BN + 1) + c] = make_float2(acc_re[v], acc_im[v]);
    }
    __syncthreads();
    const int64_t dep_m_hi = M > BM ? deposit(row0 & (M - 1), g.posM, g.mb) : 0;
    const int64_t dep_n_hi = N > BN ? deposit(col0 & (N - 1), g.posN, g.nb) : 0;
#pragma unroll 4
    for (int t = 0; t < T::PER_THREAD; ++t) {
      int r = r_tid, c = c_tid;
#pragma unroll
      for (int b = 8; b < T::UBITS; ++b) {
        if ((t >> (b - 8)) & 1) {
          const int u = g.ubit[b];
          if (u < 32)
            r |= 1 << u;
          else
            c |= 1 << (u - 32);
        }
      }
      const int64_t gr = row0 + r, gc = col0 + c;
      if (gr >= rowsA || gc >= rowsB) continue;
      const int64_t rv = gr >> g.mb, cv = gc >> g.nb;
      int64_t a = g.swapped ? cv * g.nvarA + rv : rv * g.nvarB + cv;
      if (g.pair_mode == 1) a = g.pairs[a];
      if (a < 0) continue;
      g.C[a * sizeC + dep_m_hi + dep_m_lo[r] + dep_n_hi + dep_n_lo[c]] = Ct[r * (BN + 1) + c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
__global__ void k_zero(uint32_t* p, uint64_t words) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

__global__ void k_accumulate(const float2* partial, const int32_t* rho, double2* amps,
                             double2* comp, int64_t k) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const float2 p = partial[rho[i]];
  double2 s = amps[i], c = comp[i];
  neumaier(s.x, c.x, double(p.x));
  neumaier(s.y, c.y, double(p.y));
  amps[i] = s;
  comp[i] = c;
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

// Error-free sum of two doubles (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

constexpr int XEB_THREADS = 1024;

__global__ void __launch_bounds__(XEB_THREADS) k_xeb(const double2* amps, int64_t k, int n,
                                                     double* out) {
  __shared__ double ss[XEB_THREADS];
  __shared__ double cc[XEB_THREADS];
  const int t = threadIdx.x;
  double s = 0.0, c = 0.0;
  for (int64_t i = t; i < k; i += XEB_THREADS) {
    const double2 a = amps[i];
    const double p = a.x * a.x + a.y * a.y;
    neumaier(s, c, p);
  }
  ss[t] = s;
  cc[t] = c;
  __syncthreads();
  for (int w = XEB_THREADS / 2; w > 0; w >>= 1) {
    if (t < w) {
      double sum, err;
      two_sum(ss[t], ss[t + w], sum, err);
      ss[t] = sum;
      cc[t] = cc[t] + cc[t + w] + err;
    }
    __syncthreads();
  }
  if (t == 0) {
    const double total = ss[0] + cc[0];
    out[0] = ldexp(total, n) / double(k) - 1.0;
  }
}

inline int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 262144) g = 262144;
  return int(g);
}

}  // namespace

void launch_contract_generic(const ContractArgs& a, hipStream_t s) {
  const int64_t total = a.nvar << (a.mb + a.nb);
  if (total <= 0) return;
  k_contract_generic<<<grid_for(total, 256), 256, 0, s>>>(a);
}

void launch_contract_mfma(const ContractArgs& a, hipStream_t s) {
  const int64_t rowsA = a.nvarA << a.mb;
  const int64_t rowsB = a.nvarB << a.nb;
  if (rowsA <= 0 || rowsB <= 0) return;
  const int bm = a.tile == 0 ? 64 : 32, bn = a.tile == 0 ? 64 : 128;
  const int64_t tiles = ((rowsB + bn - 1) / bn) * ((rowsA + bm - 1) / bm);
  const unsigned grid = unsigned(tiles < (int64_t(1) << 22) ? tiles : (int64_t(1) << 22));
  if (a.tile == 0)
    k_contract_mfma<64, 64><<<grid, 256, 0, s>>>(a);
  else
    k_contract_mfma<32, 128><<<grid, 256, 0, s>>>(a);
}

void mfma_tile_shape(int tile, int* bm, int* bn) {
  *bm = tile == 0 ? 64 : 32;
  *bn = tile == 0 ? 64 : 128;
}

void launch_zero(void* p, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  if (words == 0) return;
  k_zero<<<grid_for(int64_t(words), 256), 256, 0, s>>>(static_cast<uint32_t*>(p), words);
}

void launch_accumulate(const float2* partial, const int32_t* rho, double2* amps, double2* comp,
                       int64_t k, hipStream_t s) {
  if (k <= 0) return;
  k_accumulate<<<grid_for(k, 256), 256, 0, s>>>(partial, rho, amps, comp, k);
}

void launch_fold_compensation(double2* amps, const double2* comp, int64_t k, hipStream_t s) {
  if (k <= 0) return;
  k_fold<<<grid_for(k, 256), 256, 0, s>>>(amps, comp, k);
}

void launch_xeb(const double2* amps, int64_t k, int n_qubits, double* out, hipStream_t s) {
  k_xeb<<<1, XEB_THREADS, 0, s>>>(amps, k, n_qubits, out);
}

}  // namespace xeb
