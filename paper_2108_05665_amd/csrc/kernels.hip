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
// MFMA contraction: workgroup tile 64 x 64 complex, 4 waves (2 x 2), each
// wave one 32 x 32 block; K staged through LDS 16 complex at a time as
// separate re / im planes, [k][plane][row] (+1 float padding per plane row).
constexpr int BM = 64, BN = 64, TK = 16, PAD = 1;

__global__ void __launch_bounds__(256) k_contract_mfma(ContractArgs g) {
  __shared__ float As[TK][2][BM + PAD];
  __shared__ float Bs[TK][2][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t rowsA = g.nvarA << g.mb;
  const int64_t rowsB = g.nvarB << g.nb;
  const int64_t tiles_n = (rowsB + BN - 1) / BN;
  const int64_t tiles = tiles_n * ((rowsA + BM - 1) / BM);
  const int64_t K = int64_t(1) << g.kb;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
  const int64_t row0 = (tile / tiles_n) * BM;
  const int64_t col0 = (tile % tiles_n) * BN;

  floatx16 acc_re, acc_im;
  for (int v = 0; v < 16; ++v) {
    acc_re[v] = 0.f;
    acc_im[v] = 0.f;
  }

  for (int64_t k0 = 0; k0 < K; k0 += TK) {
    // Stage: BM x TK complex of each operand, 4 elements per thread.  A
    // thread's consecutive lanes walk k inside one row (contiguous in HBM).
#pragma unroll
    for (int t = 0; t < (BM * TK) / 256; ++t) {
      const int e = tid + t * 256;
      const int r = e / TK, kk = e % TK;
      const int64_t gr = row0 + r, gk = k0 + kk;
      float2 x = make_float2(0.f, 0.f);
      if (gr < rowsA && gk < K) x = g.A[(gr << g.kb) + gk];
      As[kk][0][r] = x.x;
      As[kk][1][r] = x.y;
    }
#pragma unroll
    for (int t = 0; t < (BN * TK) / 256; ++t) {
      const int e = tid + t * 256;
      const int r = e / TK, kk = e % TK;
      const int64_t gr = col0 + r, gk = k0 + kk;
      float2 x = make_float2(0.f, 0.f);
      if (gr < rowsB && gk < K) x = g.B[(gr << g.kb) + gk];
      Bs[kk][0][r] = x.x;
      Bs[kk][1][r] = x.y;
    }
    __syncthreads();
    const int i = lane & 31;
    const int half = lane >> 5;  // 0: real plane of the K=2 pair, 1: imaginary
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

  // Epilogue.  Output layout of v_mfma_f32_32x32x2f32: lane l, register v hold
  // row (v % 4) + 4 (l / 32) + 8 (v / 4), column l % 32.
  const int64_t mmask = (int64_t(1) << g.mb) - 1;
  const int64_t nmask = (int64_t(1) << g.nb) - 1;
  const int64_t sizeC = int64_t(1) << (g.mb + g.nb);
  const int64_t gc = col0 + wn * 32 + (lane & 31);
  if (gc < rowsB) {
    const int64_t r_var = gc >> g.nb;
    const int64_t n = gc & nmask;
    const int64_t offn = deposit(n, g.posN, g.nb);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gr = row0 + wm * 32 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
      if (gr >= rowsA) continue;
      const int64_t l_var = gr >> g.mb;
      const int64_t m = gr & mmask;
      int64_t a = l_var * g.nvarB + r_var;
      if (g.pair_mode == 1) a = g.pairs[a];
      if (a < 0) continue;
      g.C[a * sizeC + deposit(m, g.posM, g.mb) + offn] = make_float2(acc_re[v], acc_im[v]);
    }
  }
  }  // tile loop
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
  const int64_t tiles = ((rowsB + BN - 1) / BN) * ((rowsA + BM - 1) / BM);
  const int64_t grid = tiles < (int64_t(1) << 22) ? tiles : (int64_t(1) << 22);
  k_contract_mfma<<<unsigned(grid), 256, 0, s>>>(a);
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
