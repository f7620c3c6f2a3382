// gfx950 kernels of the 3D Fourier neural operator (paper Sec. 4, App. A.2):
// one generic BF16-MFMA contraction used for every truncated-DFT stage and
// every pointwise channel map, the per-mode complex channel mixing and its
// adjoints, a Gram kernel for pointwise weight gradients, and elementwise,
// reduction and Adam kernels.  All contractions take BF16 operands and
// accumulate in FP32 (v_mfma_f32_16x16x32_bf16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mfno {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 with round to nearest even, in hardware (v_cvt_pk_bf16_f32);
// f2bf2 packs two values, the first in the low half.
__device__ __forceinline__ uint16_t f2bf(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <typename T> __device__ __forceinline__ float to_f(T v);
template <> __device__ __forceinline__ float to_f<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_f<uint16_t>(uint16_t v) { return bf2f(v); }
template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t from_f<uint16_t>(float v) { return f2bf(v); }
template <typename T> __device__ __forceinline__ uint16_t to_bf(T v);
template <> __device__ __forceinline__ uint16_t to_bf<float>(float v) { return f2bf(v); }
template <> __device__ __forceinline__ uint16_t to_bf<uint16_t>(uint16_t v) { return v; }

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// --------------------------------------------------------------- contract
// out(o, n, i) = alpha * sum_k in(o, k, i) * G[k][n] (+ out if accumulate)
//                (+ bias[n])
// with columns j = o * I + i (I a power of two), index maps
//   in  address = (j >> lgI) * in_so + (j & (I-1)) * in_si
//                 + (k >> lgkd) * in_sk1 + (k & (kd-1)) * in_sk2
//   out address = (j >> lgI) * out_so + (j & (I-1)) * out_si
//                 + (n >> lgnd) * out_sn1 + (n & (nd-1)) * out_sn2
// and G given transposed, gt[n][k] (BF16, row length kp, zero padded to
// kp >= K rounded up to 32 and to np, a multiple of 64 rows).
// Epilogue: the value is stored to out when store_out is set, and its
// activation (GELU or identity) is stored as BF16 to act at the same
// address when act is not null.
struct ContractArgs {
  const void* in;
  void* out;
  const uint16_t* gt;
  const float* bias;
  uint16_t* act;
  int64_t cols;
  int32_t lgI;
  int64_t in_so, in_si, in_sk1, in_sk2;
  int32_t lgkd;
  int64_t out_so, out_si, out_sn1, out_sn2;
  int32_t lgnd;
  int32_t K, N, kp, np;
  float alpha;
  int32_t accumulate;
  int32_t store_out;
  int32_t act_gelu;
  const float* gmul;  // when set: the value is multiplied by GELU'(gmul[addr]) before it is stored
};

constexpr int CT_N = 64;   // rows n per block pass (4 waves x 16)
constexpr int CT_J = 64;   // columns per block
constexpr int CT_K = 32;   // k per step (one MFMA)
constexpr int LDS_KP = 40; // padded k stride of the LDS tile

// Load modes of the 64-column x 32-k input tile (LDS layout [column][k]):
//  LOAD_SCALAR  any index map, one element per load;
//  LOAD_KRUN    k contiguous (lgkd = 0, in_sk1 = 1), K % 8 == 0, column
//               bases 8-element aligned: 8 consecutive k per load;
//  LOAD_JRUN    columns contiguous (in_si = 1) in runs of 8 (I % 8 == 0,
//               cols % 8 == 0), k offsets 8-element aligned: 8 consecutive
//               columns per load, transposed into LDS.
enum { LOAD_SCALAR = 0, LOAD_KRUN = 1, LOAD_JRUN = 2 };

template <typename T> struct Vec8;
template <> struct Vec8<uint16_t> {
  static __device__ __forceinline__ void load(const uint16_t* p, uint16_t (&o)[8]) {
    const uint4 v = *(const uint4*)p;
    o[0] = v.x & 0xffff; o[1] = v.x >> 16; o[2] = v.y & 0xffff; o[3] = v.y >> 16;
    o[4] = v.z & 0xffff; o[5] = v.z >> 16; o[6] = v.w & 0xffff; o[7] = v.w >> 16;
  }
};
template <> struct Vec8<float> {
  static __device__ __forceinline__ void load(const float* p, uint16_t (&o)[8]) {
    const float4 a = *(const float4*)p, b = *(const float4*)(p + 4);
    const uint32_t w[4] = {f2bf2(a.x, a.y), f2bf2(a.z, a.w), f2bf2(b.x, b.y), f2bf2(b.z, b.w)};
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
  }
};

// Makes this wave's earlier LDS stores visible to its later LDS loads from
// other lanes of the same wave.  A wave's LDS operations complete in issue
// order, so no block barrier is needed for a tile that only this wave
// writes and reads; the wavefront-scope fences keep the compiler from
// moving LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// GELU(x) = x Phi(x), Phi the standard normal CDF, without branches:
// Phi(x) = sigma(g(x)), sigma the logistic function and g an odd polynomial
// x (a0 + a1 x^2 + a2 x^4) fitted (minimax of |x (sigma(g) - Phi)| over
// [-60, 60]) to the logit of Phi, with x clamped to [-6, 6] inside g
// (sigma(g(6)) = 1 - 2e-9).  norm_cdf_fit returns sigma(g(x)) as
// 1 / (1 + 2^h), h = -g(x) log2 e, with the coefficients of h.  Errors
// against x Phi(x) and Phi(x) + x phi(x) in FP32: at most 2.6e-5 and 5.1e-5
// absolute, far below the BF16 rounding of the values they feed.
__device__ __forceinline__ float norm_cdf_fit(float x) {
  const float xc = __builtin_amdgcn_fmed3f(x, -6.f, 6.f);
  const float s = xc * xc;
  const float h = xc * fmaf(fmaf(0.0010142630f, s, -0.10677572f), s, -2.3011212f);
  return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(h));
}
__device__ __forceinline__ float gelu(float x) { return x * norm_cdf_fit(x); }
// GELU'(x) = Phi(x) + x phi(x), phi(x) = exp(-x^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_grad(float x) {
  const float xc = __builtin_amdgcn_fmed3f(x, -6.f, 6.f);
  return fmaf(x * 0.39894228f, __builtin_amdgcn_exp2f(-0.72134752f * xc * xc), norm_cdf_fit(x));
}

// Epilogue modes: EP_DIRECT stores from the MFMA layout (each lane owns 16
// outputs); EP_NFAST and EP_JFAST stage the 64 x 64 result tile in LDS and
// store it with consecutive threads on consecutive n (outputs contiguous
// along n) or on consecutive columns (outputs contiguous along columns).
// EP_JVEC and EP_NVEC are the two staged orders with four consecutive
// outputs per thread along the contiguous dimension (one vector access for
// the store, the accumulated value, the GELU' factor and the activation)
// and the address of the fixed index hoisted out of the loop; they need
// 4-element alignment of every address (checked by the host).
enum { EP_DIRECT = 0, EP_NFAST = 1, EP_JFAST = 2, EP_JVEC = 3, EP_NVEC = 4 };

template <typename T> struct Vec4;
template <> struct Vec4<float> {
  static __device__ __forceinline__ void load(const float* p, float (&v)[4]) {
    const float4 x = *(const float4*)p;
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  }
  static __device__ __forceinline__ void store(float* p, const float (&v)[4]) {
    *(float4*)p = float4{v[0], v[1], v[2], v[3]};
  }
};
template <> struct Vec4<uint16_t> {
  static __device__ __forceinline__ void load(const uint16_t* p, float (&v)[4]) {
    const uint2 x = *(const uint2*)p;
    v[0] = bf2f((uint16_t)(x.x & 0xffffu)); v[1] = bf2f((uint16_t)(x.x >> 16));
    v[2] = bf2f((uint16_t)(x.y & 0xffffu)); v[3] = bf2f((uint16_t)(x.y >> 16));
  }
  static __device__ __forceinline__ void store(uint16_t* p, const float (&v)[4]) {
    *(uint2*)p = uint2{f2bf2(v[0], v[1]), f2bf2(v[2], v[3])};
  }
};

constexpr int CT_KT = 64;            // k held in LDS per pass (two MFMA steps)
constexpr int CT_TS = CT_KT + 8;     // padded LDS row of the input tile
constexpr int CT_DS = CT_J + 1;      // padded LDS row of the result tile

// LDS element of the input tile at (column row r, k in [0, 64)): the eight
// 16-byte k chunks of a row are permuted by XOR with (r / 8) mod 8, so that
// the transposing store of LOAD_JRUN (lanes writing rows 8 apart at one k)
// spreads over all banks instead of one; a chunk stays whole and 16-byte
// aligned for the MFMA operand reads.
__device__ __forceinline__ int ct_idx(int r, int k) { return r * CT_TS + (((k >> 3) ^ ((r >> 3) & 7)) << 3) + (k & 7); }

template <typename InT, typename OutT, int LM, int EP>
__global__ __launch_bounds__(256) void contract_kernel(ContractArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t tile[CT_J * CT_TS];
  __shared__ float dst[EP == EP_DIRECT ? 1 : CT_N * CT_DS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t j0 = (int64_t)blockIdx.x * CT_J;
  const InT* in = (const InT*)a.in;
  const int64_t Imask = ((int64_t)1 << a.lgI) - 1;
  const int kdmask = (1 << a.lgkd) - 1;
  auto colbase = [&](int64_t j) { return (j >> a.lgI) * a.in_so + (j & Imask) * a.in_si; };
  auto kaddr = [&](int k) { return (int64_t)(k >> a.lgkd) * a.in_sk1 + (int64_t)(k & kdmask) * a.in_sk2; };

  // per-thread tile coordinates (one 32-k half of the tile per load pass)
  int lk[8], lj[8];
  int64_t cb[8];
  if (LM == LOAD_SCALAR) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      lj[q] = t & 63;
      lk[q] = (t >> 6) * 8 + q;
      const int64_t j = j0 + lj[q];
      cb[q] = j < a.cols ? colbase(j) : -1;
    }
  } else if (LM == LOAD_KRUN) {
    lj[0] = t >> 2;
    lk[0] = (t & 3) * 8;
    cb[0] = j0 + lj[0] < a.cols ? colbase(j0 + lj[0]) : -1;
  } else {
    lk[0] = t >> 3;
    lj[0] = (t & 7) * 8;
    cb[0] = j0 + lj[0] < a.cols ? colbase(j0 + lj[0]) : -1;
  }
  // load k in [k0, k0 + 32) into tile columns [h * 32, h * 32 + 32)
  auto load_half = [&](int k0, int h) {
    if (LM == LOAD_SCALAR) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + lk[q];
        uint16_t v = 0;
        if (cb[q] >= 0 && k < a.K) v = to_bf(in[cb[q] + kaddr(k)]);
        tile[ct_idx(lj[q], h * 32 + lk[q])] = v;
      }
    } else if (LM == LOAD_KRUN) {
      uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      const int k = k0 + lk[0];
      if (cb[0] >= 0 && k < a.K) Vec8<InT>::load(in + cb[0] + k, v);
      uint4 w;
      w.x = v[0] | ((uint32_t)v[1] << 16); w.y = v[2] | ((uint32_t)v[3] << 16);
      w.z = v[4] | ((uint32_t)v[5] << 16); w.w = v[6] | ((uint32_t)v[7] << 16);
      *(uint4*)(tile + ct_idx(lj[0], h * 32 + lk[0])) = w;
    } else {
      uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      const int k = k0 + lk[0];
      if (cb[0] >= 0 && k < a.K) Vec8<InT>::load(in + cb[0] + kaddr(k), v);
#pragma unroll
      for (int q = 0; q < 8; ++q) tile[ct_idx(lj[0] + q, h * 32 + lk[0])] = v[q];
    }
  };

  // K <= 64: the whole input tile stays in LDS for every n-block
  const bool resident = a.K <= CT_KT;
  if (resident) {
    load_half(0, 0);
    if (a.K > CT_K) load_half(CT_K, 1);
    __syncthreads();
  }
  const int akk = 8 * (lane >> 4);
  OutT* out = (OutT*)a.out;
  const int ndm = (1 << a.lgnd) - 1;
  const int nblocks = a.np / CT_N;
  for (int nb = blockIdx.y; nb < nblocks; nb += gridDim.y) {
    const int n0 = nb * CT_N;
    f32x4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int arow = n0 + wave * 16 + (lane & 15);
    for (int k0 = 0; k0 < a.K; k0 += CT_KT) {
      if (!resident) {
        load_half(k0, 0);
        if (k0 + CT_K < a.K) load_half(k0 + CT_K, 1);
        __syncthreads();
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (k0 + h * CT_K >= a.K) break;
        // A: rows of G^T (zero padded beyond N and K)
        const bf16x8 av = *(const bf16x8*)(a.gt + (int64_t)arow * a.kp + k0 + h * CT_K + akk);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 bv = *(const bf16x8*)(tile + ct_idx(c * 16 + (lane & 15), h * 32 + akk));
          acc[c] = mfma16(av, bv, acc[c]);
        }
      }
      if (!resident) __syncthreads();
    }
    auto finish = [&](int n, int64_t j, float v) {
      const int64_t addr = (j >> a.lgI) * a.out_so + (j & Imask) * a.out_si + (int64_t)(n >> a.lgnd) * a.out_sn1 +
                           (int64_t)(n & ndm) * a.out_sn2;
      if (a.bias) v += a.bias[n];
      if (a.accumulate) v += to_f(out[addr]);
      if (a.gmul) v *= gelu_grad(a.gmul[addr]);
      if (a.store_out) out[addr] = from_f<OutT>(v);
      if (a.act) a.act[addr] = f2bf(a.act_gelu ? gelu(v) : v);
    };
    // four consecutive outputs from the staged tile: bias (one per n or per
    // output), accumulation, GELU' factor, store and activation as vectors
    auto finish4 = [&](int64_t addr, const int (&nn)[4], float (&v)[4]) {
      if (a.bias) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += a.bias[nn[q]];
      }
      if (a.accumulate) {
        float o[4];
        Vec4<OutT>::load(out + addr, o);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += o[q];
      }
      if (a.gmul) {
        float h[4];
        Vec4<float>::load(a.gmul + addr, h);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] *= gelu_grad(h[q]);
      }
      if (a.store_out) Vec4<OutT>::store(out + addr, v);
      if (a.act) {
        float g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = a.act_gelu ? gelu(v[q]) : v[q];
        Vec4<uint16_t>::store(a.act + addr, g);
      }
    };
    if (EP == EP_DIRECT) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t j = j0 + c * 16 + (lane & 15);
        if (j >= a.cols) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = n0 + wave * 16 + 4 * (lane >> 4) + r;
          if (n < a.N) finish(n, j, a.alpha * acc[c][r]);
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dst[(wave * 16 + 4 * (lane >> 4) + r) * CT_DS + c * 16 + (lane & 15)] = a.alpha * acc[c][r];
      __syncthreads();
      if (EP == EP_JVEC) {
        // columns jl .. jl + 3 (contiguous outputs, out_si = 1), rows nl
        const int jl = 4 * (t & 15);
        const int64_t j = j0 + jl;
        const int64_t cb = (j >> a.lgI) * a.out_so + (j & Imask);
        for (int nl = t >> 4; nl < CT_N; nl += 16) {
          const int n = n0 + nl;
          if (n >= a.N || j >= a.cols) continue;
          const int64_t addr = cb + (int64_t)(n >> a.lgnd) * a.out_sn1 + (int64_t)(n & ndm) * a.out_sn2;
          float v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = dst[nl * CT_DS + jl + q];
          const int nn[4] = {n, n, n, n};
          finish4(addr, nn, v);
        }
      } else if (EP == EP_NVEC) {
        // rows nl .. nl + 3 (contiguous outputs, out_sn1 = 1, nd = 1), columns jl
        const int nl = 4 * (t & 15);
        const int n = n0 + nl;
        for (int jl = t >> 4; jl < CT_J; jl += 16) {
          const int64_t j = j0 + jl;
          if (n >= a.N || j >= a.cols) continue;
          const int64_t addr = (j >> a.lgI) * a.out_so + (j & Imask) * a.out_si + n;
          float v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) v[q] = dst[(nl + q) * CT_DS + jl];
          const int nn[4] = {n, n + 1, n + 2, n + 3};
          finish4(addr, nn, v);
        }
      } else {
#pragma unroll 4
        for (int e = t; e < CT_N * CT_J; e += 256) {
          const int nl = EP == EP_NFAST ? (e & 63) : (e >> 6);
          const int jl = EP == EP_NFAST ? (e >> 6) : (e & 63);
          const int n = n0 + nl;
          const int64_t j = j0 + jl;
          if (n < a.N && j < a.cols) finish(n, j, dst[nl * CT_DS + jl]);
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------- channel maps
// Pointwise channel map over points p of [B][K][P] activations:
//   out[b][n][p] = alpha * sum_k G[k][n] in[b][k][p] (+ bias[n]) (+ out)
// with the same epilogue as contract_kernel (store_out, BF16 activation).
// A block covers 256 consecutive points of one sample (P % 256 == 0) so
// that every row it touches is a 512 B (BF16) or 1 KB (FP32) run; rows n
// are done 32 at a time, k 32 at a time.
struct PwArgs {
  const void* in;
  float* out;
  const uint16_t* gt;  // [np][kp] BF16, G transposed, zero padded
  const float* bias;
  uint16_t* act;
  int64_t P;
  int32_t K, N, kp;
  float alpha;
  int32_t accumulate, store_out, act_gelu;
  const float* gmul;  // when set: multiplied by GELU'(gmul) (same layout as out) before the store
};

constexpr int PW_J = 256;        // points per block
constexpr int PW_TS = 40;        // padded LDS row (32 k)
constexpr int PW_DS = PW_J + 4;  // padded LDS row of the result tile

// LDS placement of a 256-point x (32 or 64)-channel BF16 tile, [point][k]:
// the threads of one store instruction hold points 8 apart (one 16-byte
// load covers 8 consecutive points), so point p goes to row
// (p % 8) * 32 + p / 8, making those rows consecutive, and its 8-element
// channel groups are XOR-swizzled by p % 4 so the 16-byte fragment reads of
// 16 consecutive points spread over the banks.
__device__ __forceinline__ int tile_row(int p) { return (p & 7) * 32 + (p >> 3); }
__device__ __forceinline__ int tile_col(int k, int p) { return ((((k >> 3) ^ (p & 3))) << 3) | (k & 7); }

// (four waves per SIMD, 128 registers: with 33 KB of LDS, four blocks per CU)
template <typename InT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void pw_kernel(PwArgs a) {
  // one LDS buffer: the input tile during the products, then the result
  // tile for the epilogue (33 KB: four blocks per CU)
  __shared__ __attribute__((aligned(16))) float lds[32 * PW_DS];
  uint16_t* tile = (uint16_t*)lds;
  float* dst = lds;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * PW_J;
  const int64_t b = j0 / a.P, p0 = j0 % a.P;
  const InT* in = (const InT*)a.in + b * a.K * a.P + p0;
  const int nkt = (a.K + 31) / 32;
  // 256 points x 32 k: thread loads 8 consecutive points of one k, 4 times
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = q * 256 + t;
      const int kl = idx >> 5, pl = (idx & 31) * 8;
      uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (k0 + kl < a.K) Vec8<InT>::load(in + (int64_t)(k0 + kl) * a.P + pl, v);
#pragma unroll
      for (int i = 0; i < 8; ++i) tile[tile_row(pl + i) * PW_TS + tile_col(kl, pl + i)] = v[i];
    }
  };
  float* out = a.out ? a.out + b * a.N * a.P + p0 : nullptr;
  uint16_t* act = a.act ? a.act + b * a.N * a.P + p0 : nullptr;
  for (int n0 = 0; n0 < a.N; n0 += 32) {
    f32x4 acc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[h][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < nkt; ++kt) {
      load(kt * 32);
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bf16x8 av = *(const bf16x8*)(a.gt + (int64_t)(n0 + h * 16 + (lane & 15)) * a.kp + kt * 32 + 8 * g);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int pt = wave * 64 + c * 16 + (lane & 15);
          const bf16x8 bv = *(const bf16x8*)(tile + tile_row(pt) * PW_TS + tile_col(8 * g, pt));
          acc[h][c] = mfma16(av, bv, acc[h][c]);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dst[(h * 16 + 4 * g + r) * PW_DS + wave * 64 + c * 16 + (lane & 15)] = a.alpha * acc[h][c][r];
    __syncthreads();
    // 32 rows x 64 float4: a wave stores one contiguous row per step
#pragma unroll 2
    for (int e = t; e < 32 * 64; e += 256) {
      const int nl = e >> 6, p4 = (e & 63) * 4;
      const int n = n0 + nl;
      if (n >= a.N) continue;
      float4 v = *(const float4*)(dst + nl * PW_DS + p4);
      const int64_t off = (int64_t)n * a.P + p4;
      if (a.bias) {
        const float bb = a.bias[n];
        v.x += bb; v.y += bb; v.z += bb; v.w += bb;
      }
      if (a.accumulate) {
        const float4 o = *(const float4*)(out + off);
        v.x += o.x; v.y += o.y; v.z += o.z; v.w += o.w;
      }
      if (a.gmul) {
        const float4 hh = *(const float4*)(a.gmul + b * a.N * a.P + p0 + off);
        v.x *= gelu_grad(hh.x); v.y *= gelu_grad(hh.y); v.z *= gelu_grad(hh.z); v.w *= gelu_grad(hh.w);
      }
      if (a.store_out) *(float4*)(out + off) = v;
      if (act) {
        uint2 w;
        if (a.act_gelu) {
          w.x = f2bf2(gelu(v.x), gelu(v.y));
          w.y = f2bf2(gelu(v.z), gelu(v.w));
        } else {
          w.x = f2bf2(v.x, v.y);
          w.y = f2bf2(v.z, v.w);
        }
        *(uint2*)(act + off) = w;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------- fused y and x forward stages
// The y and x stages of the truncated forward DFT in one pass over one
// (b, w) slab, for Y = 64, 2 my = 2 mx = 32 (64 real rows of each DFT
// operand) and mz = 16:
//   A2[x][n1][kz] = sum_k1 F2[k1][n1] A1[x][k1][kz],  k1 = 2 y + part,
//                                                     n1 = 2 ky + part'
//   modes[n2][ky][kz] = sum_k2 F3[k2][n2] A2[x][2 ky + p][kz],  k2 = 2 x + p
// The y-stage output stays on chip (in LDS, rounded to BF16 as the
// two-pass form stores it), so its 0.27 GB round trip per layer at batch 16
// is gone; both stages accumulate their k steps in the two-pass order, so
// the modes are bitwise those of the separate contractions.  Per chunk of
// 16 x: two halves of 8 x are staged transposed in LDS (t1 [(x, kz)][k1]);
// the y-stage rows are formed in 16-row tiles (the F2 operand held in
// registers for the whole slab) and written as x-stage operands (t2
// [(ky, kz)][k2]); then one x-stage k step of 32.  Eight waves: each owns
// one 16-row tile and half the columns of both stages.
constexpr int DYX_T1 = 136;  // t1 row: 128 k1 + 8
constexpr int DYX_T2 = 40;   // t2 row: 32 k2 + 8

// t2 element (row, k2): the four 16-byte k2 chunks permuted by XOR with
// (ky / 2) mod 4, so that the four lane groups of a stage-1 store (ky two
// apart) hit different banks
__device__ __forceinline__ int dyx_t2(int row, int ky, int k) {
  return row * DYX_T2 + ((((k >> 3) ^ ((ky >> 1) & 3))) << 3) + (k & 7);
}

// (four waves per SIMD, 128 registers: two blocks per CU)
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void dft_yx_kernel(
    const uint16_t* __restrict__ a1, const uint16_t* __restrict__ f2, const uint16_t* __restrict__ f3, int X,
    uint16_t* __restrict__ modes) {
  __shared__ __attribute__((aligned(16))) uint16_t t1[128 * DYX_T1];
  __shared__ __attribute__((aligned(16))) uint16_t t2[512 * DYX_T2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, l16 = lane & 15, kl = 8 * g;
  // eight waves: row tile rt = wave % 4 of both stages; column half ch =
  // wave / 4 (y stage: x columns 4 ch .. 4 ch + 3; x stage: ky 16 ch .. + 15)
  const int rt = wave & 3, ch = wave >> 2;
  const int64_t bw = blockIdx.x;
  const uint16_t* src = a1 + bw * (int64_t)X * 2048;  // [x][y][part][kz]: 2048 values per x
  bf16x8 af2[4];  // F2^T rows 16 rt + l16, the four k steps
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) af2[ks] = *(const bf16x8*)(f2 + (16 * rt + l16) * 128 + 32 * ks + kl);
  f32x4 acc2[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int x0 = 0; x0 < X; x0 += 16) {
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      // x in [x0 + 8 h, x0 + 8 h + 8): 16384 contiguous values, item e =
      // ((xl * 64 + y) * 2 + part) * 2 + q holds kz 8 q .. 8 q + 7; a thread
      // takes both parts of (xl, y, q), so each t1 store is one 4-byte word
      // (k1 = 2 y and 2 y + 1)
      const uint16_t* hs = src + (int64_t)(x0 + 8 * h) * 2048;
      uint4 v[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int pi = t + 512 * i, q = pi & 1, y = (pi >> 1) & 63, xl = pi >> 7;
        const int e0 = ((xl * 64 + y) * 2) * 2 + q;  // part 0; part 1 is e0 + 2
        v[i][0] = *(const uint4*)(hs + 8 * e0);
        v[i][1] = *(const uint4*)(hs + 8 * (e0 + 2));
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int pi = t + 512 * i, q = pi & 1, y = (pi >> 1) & 63, xl = pi >> 7;
        const uint32_t u0[4] = {v[i][0].x, v[i][0].y, v[i][0].z, v[i][0].w};
        const uint32_t u1[4] = {v[i][1].x, v[i][1].y, v[i][1].z, v[i][1].w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t a = u0[j >> 1], b = u1[j >> 1];
          *(uint32_t*)(t1 + (xl * 16 + 8 * q + j) * DYX_T1 + 2 * y) =
              (j & 1) ? (a >> 16) | (b & 0xffff0000u) : (a & 0xffffu) | (b << 16);
        }
      }
      __syncthreads();
      f32x4 acc1[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc1[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 bv = *(const bf16x8*)(t1 + (16 * (4 * ch + c) + l16) * DYX_T1 + 32 * ks + kl);
          acc1[c] = mfma16(af2[ks], bv, acc1[c]);
        }
      // lane holds rows n1 = 16 rt + 4 g + r (ky = 8 rt + 2 g + r / 2,
      // part' = r % 2) of column (x = x0 + 8 h + 4 ch + c, kz = l16); the two
      // parts are adjacent x-stage k values (k2 = 2 x + part')
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k2 = 2 * (8 * h + 4 * ch + c);
#pragma unroll
        for (int rp = 0; rp < 2; ++rp) {
          const int ky = 8 * rt + 2 * g + rp;
          *(uint32_t*)(t2 + dyx_t2(ky * 16 + l16, ky, k2)) = f2bf2(acc1[c][2 * rp], acc1[c][2 * rp + 1]);
        }
      }
      __syncthreads();
    }
    // x-stage k step x0 / 16 for rows n2 = 16 rt .. + 15 and the columns
    // (ky = 16 ch + i, kz = l16)
    const bf16x8 af3 = *(const bf16x8*)(f3 + (int64_t)(16 * rt + l16) * (2 * X) + 2 * x0 + kl);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int ky = 16 * ch + i;
      const bf16x8 bv = *(const bf16x8*)(t2 + dyx_t2(16 * ky + l16, ky, kl));
      acc2[i] = mfma16(af3, bv, acc2[i]);
    }
  }
  // modes[bw][n2][ky][kz], n2 = 16 rt + 4 g + r, ky = 16 ch + i, kz = l16
  uint16_t* mo = modes + bw * 64 * 512;
#pragma unroll
  for (int i = 0; i < 16; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) mo[(16 * rt + 4 * g + r) * 512 + (16 * ch + i) * 16 + l16] = f2bf(acc2[i][r]);
}

// ----------------------------------------- fused x and y inverse stages
// The x and y stages of the truncated inverse DFT in one pass over one
// (b, w) slab, for the same shapes as dft_yx_kernel:
//   R3[n3][ky][kz] = sum_k3 I3[k3][n3] modes[k3][ky][kz],  k3 = 2 kx + part,
//                                                          n3 = 2 x + part'
//   R2[x][n2][kz] = sum_k2 I2[k2][n2] R3[2 x + p][ky][kz],  k2 = 2 ky + p,
//                                                          n2 = 2 y + part'
// The slab's modes (64 KB) are staged once in LDS, transposed
// (t0 [(ky, kz)][k3]); per chunk of 8 x the x-stage rows (16 of them) are
// formed for all 512 (ky, kz) columns, rounded to BF16 as the two-pass form
// stores them and staged as y-stage operands (t3 [(x, kz)][k2]); the y stage
// then writes R2 for those 8 x.  R3's round trip through memory is gone;
// the k steps run in the two-pass order, so R2 is bitwise the same.  Eight
// waves: x stage, four column tiles each; y stage, one 16-row tile each.
// Both LDS tiles have unpadded 128-byte rows (80 KB in all, so two blocks
// share a CU's 160 KB); their eight 16-byte k chunks are XOR-permuted by
// row / 2, so the 16-byte operand reads of 16 consecutive rows cover all
// banks.
constexpr int IXY_T0 = 64;   // t0 row: 64 k3
constexpr int IXY_T3 = 64;   // t3 row: 64 k2

// t0 element (row = (ky, kz), k3)
__device__ __forceinline__ int ixy_t0(int row, int k) {
  return row * IXY_T0 + ((((k >> 3) ^ ((row >> 1) & 7))) << 3) + (k & 7);
}
// t3 element (row = (x - x0) * 16 + kz, k2): the chunks are further
// permuted by XOR with x - x0, so that the x-stage stores of the four lane
// groups (x two apart) spread over the banks
__device__ __forceinline__ int ixy_t3(int row, int k) {
  return row * IXY_T3 + ((((k >> 3) ^ ((row >> 1) & 7) ^ ((row >> 4) & 7))) << 3) + (k & 7);
}

// (four waves per SIMD, 128 registers)
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void idft_xy_kernel(
    const uint16_t* __restrict__ modes, const uint16_t* __restrict__ i3, const uint16_t* __restrict__ i2, int X,
    uint16_t* __restrict__ r2) {
  __shared__ __attribute__((aligned(16))) uint16_t t0[512 * IXY_T0];
  __shared__ __attribute__((aligned(16))) uint16_t t3[128 * IXY_T3];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, l16 = lane & 15, kl = 8 * g;
  const int64_t bw = blockIdx.x;
  // modes[bw][k3][ky][kz]: 64 rows of 512; item e = (col / 8) * 64 + k3, so
  // that the 64 lanes of a wave store one t0 row's 64 k3 values together
  const uint16_t* mi = modes + bw * 64 * 512;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int e = t + 512 * i;
    const int k3 = e & 63, col0 = 8 * (e >> 6);
    const uint4 v = *(const uint4*)(mi + k3 * 512 + col0);
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) t0[ixy_t0(col0 + j, k3)] = (uint16_t)(u[j >> 1] >> (16 * (j & 1)));
  }
  // y-stage A operand: I2^T rows 16 wave + l16 (n2 = 2 y + part'), both k steps
  bf16x8 ai2[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) ai2[ks] = *(const bf16x8*)(i2 + (16 * wave + l16) * 64 + 32 * ks + kl);
  __syncthreads();
  for (int x0 = 0; x0 < X; x0 += 8) {
    // x stage: rows n3 = 2 x0 .. 2 x0 + 15, columns (ky = 4 wave + c, kz = l16)
    bf16x8 ai3[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) ai3[ks] = *(const bf16x8*)(i3 + (2 * x0 + l16) * 64 + 32 * ks + kl);
    f32x4 a3[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a3[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bf16x8 bv = *(const bf16x8*)(t0 + ixy_t0((4 * wave + c) * 16 + l16, 32 * ks + kl));
        a3[c] = mfma16(ai3[ks], bv, a3[c]);
      }
    // lane holds n3 = 2 x0 + 4 g + r (x = x0 + 2 g + r / 2, part = r % 2) of
    // column (ky, kz): y-stage operand t3 [(x - x0, kz)][2 ky + part]
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ky = 4 * wave + c;
#pragma unroll
      for (int rp = 0; rp < 2; ++rp) {
        const int xl = 2 * g + rp;
        *(uint32_t*)(t3 + ixy_t3(xl * 16 + l16, 2 * ky)) = f2bf2(a3[c][2 * rp], a3[c][2 * rp + 1]);
      }
    }
    __syncthreads();
    // y stage: rows n2 = 16 wave .. + 15, columns (x = x0 + c, kz = l16)
    f32x4 a2[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a2[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const bf16x8 bv = *(const bf16x8*)(t3 + ixy_t3(16 * c + l16, 32 * ks + kl));
        a2[c] = mfma16(ai2[ks], bv, a2[c]);
      }
    // R2[bw][x][n2][kz] = [x][y][part][kz]: n2 = 16 wave + 4 g + r
    uint16_t* ro = r2 + (bw * X + x0) * 128 * 16;
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) ro[((int64_t)c * 128 + 16 * wave + 4 * g + r) * 16 + l16] = f2bf(a2[c][r]);
    __syncthreads();  // t3 is read: the next chunk may write it
  }
}

// ------------------------------------------------- fused layer completion
// The end of a Fourier layer in one pass over 256 points of one sample:
//   h[b][w][p] = sum_c Wp[w][c] v[b][c][p]                  (channel map)
//              + sum_k R2[b][w][x][y][k] I1[k][z]          (c2r along z)
//              + bp[w]
// with p = (x, y, z), z fastest, k = (part, kz) the 2 mz contiguous values
// of the y stage's output.  In a 16 x 16 MFMA tile the rows are channels w
// and the columns 16 consecutive z of one (x, y) row, so the channel map
// reads v through LDS and the c2r reads the R2 row of (w, x, y) as its A
// operand directly; each product has its own accumulators, added in the
// epilogue, which stages the sum through LDS: h stored when requested
// (training), its activation (GELU or identity) stored as BF16.
// When a1 is set (Z = 64, W = 32, 2 mz = 32) the block also runs the next
// layer's truncated z-DFT on the activation tile it holds:
//   A1[b][w][x][y][k] = sum_z act[b][w][x][y][z] Fz[k][z]
// with the same operand roles and accumulation order as the stand-alone
// contraction, so the next layer skips its z stage.
// The backward pass uses the same kernel on FP32 input (InT = float) with
// the transposed channel map, the adjoint c2r operand, no bias, gmul set
// (the result times GELU'(gmul), the pre-activation of the layer below)
// and only the FP32 output h.  The lift uses it with cin input channels,
// the lift weights as the channel map and no c2r term (r2 null), so that
// layer 0's z stage is fused as well.
// The hybrid F/FNO layer has no channel map (Win = 0 skips it): forward,
// the kernel yields the spectral convolution s alone; backward, it adds the
// FP32 residual gradient resid to the adjoint c2r term.
struct LayerEndArgs {
  const void* v;        // [B][W][P] layer input, BF16 or FP32 (InT)
  const uint16_t* r2;   // [B W X Y][2 mz] y-stage output (BF16)
  const uint16_t* gwp;  // [64][32] BF16 Wp (rows w_out, k = w_in), zero padded
  const uint16_t* gi1;  // [Z padded to 64][32] BF16 c2r operand (rows z, k), zero padded
  int32_t gi1_kp;
  const float* bias;    // [W]
  float* h;             // [B][W][P] or null
  uint16_t* act;        // [B][W][P] or null
  const float* gmul;    // [B][W][P] or null
  int64_t P;
  int32_t W, Z, K2;     // width, nz, 2 mz
  int32_t Win;          // input channels of the channel map (<= 32; W except for the lift)
  int32_t act_gelu;
  const uint16_t* gz;   // next layer's z-DFT operand [2 mz padded][kp] BF16 (rows k, columns z)
  int32_t gz_kp;
  uint16_t* a1;         // next layer's z-stage output [B W X Y][2 mz] BF16, or null
  const float* resid;   // [B][W][P] FP32 added before gmul, or null
};

// eight consecutive values as packed BF16 (RNE)
template <typename T> __device__ __forceinline__ uint4 load8_bf(const T* p);
template <> __device__ __forceinline__ uint4 load8_bf<uint16_t>(const uint16_t* p) { return *(const uint4*)p; }
template <> __device__ __forceinline__ uint4 load8_bf<float>(const float* p) {
  const float4 x = *(const float4*)p, y = *(const float4*)(p + 4);
  return uint4{f2bf2(x.x, x.y), f2bf2(x.z, x.w), f2bf2(y.x, y.y), f2bf2(y.z, y.w)};
}

// Column of the layer end's FP32 result tile [32 rows][256 points]: the
// 16-point groups are XOR-permuted by row / 4, so the four row groups of
// one accumulator store fall in disjoint banks without padding the rows,
// and the four consecutive points a thread reads stay contiguous.
__device__ __forceinline__ int le_col(int row, int p) { return p ^ (((row >> 2) & 3) << 4); }

// NT = ceil(W / 16), W <= 32; C2R: r2 term present; ROW64: Z = 64, so each
// wave's 64 points are one (x, y) row and its c2r operands are one R2 row
// (six waves per SIMD, 80 registers: with 20 KB of LDS, six blocks per CU)
template <int NT, typename InT, bool C2R = true, bool ROW64 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void layer_end_kernel(LayerEndArgs a) {
  // one LDS region holds in turn the v tile [256 points][PW_TS], the FP32
  // result tile 16 rows at a time [16][PW_J] and the BF16 activation tile
  // [32][PW_J + 8] of the fused z-DFT (20 KB)
  constexpr int AP = PW_J + 8, LDS_BYTES = PW_J * PW_TS * 2;
  static_assert(32 * AP * 2 <= LDS_BYTES && 16 * PW_J * 4 <= LDS_BYTES, "LDS reuse");
  __shared__ __attribute__((aligned(16))) float lds[LDS_BYTES / 4];
  uint16_t* tile = (uint16_t*)lds;
  float* dst = lds;
  uint16_t* at = (uint16_t*)lds;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * PW_J;
  const int64_t b = j0 / a.P, p0 = j0 % a.P;
  // Every global load of the block is issued before the first wait: the v
  // tile (bound for LDS) and this lane's c2r operands from the y-stage
  // output, so that both streams are in flight together.
  const InT* in = (const InT*)a.v + b * a.Win * a.P + p0;
  uint4 vq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = q * 256 + t;
    const int kl = idx >> 5, pl = (idx & 31) * 8;
    vq[q] = kl < a.Win ? load8_bf<InT>(in + (int64_t)kl * a.P + pl) : uint4{0u, 0u, 0u, 0u};
  }
  // c2r operand of column tile c (points pp .. pp + 15 of one (x, y) row) and
  // row tile h: every lane loads (from row 0 where its row or k range does
  // not exist) and selects at use, so no divergent branch feeds the MFMA
  uint4 rq[ROW64 ? 1 : 4][NT];
  // (x, y) row and first z of column tile c, from block-uniform values (the
  // wave index made scalar, so no per-lane 64-bit division is formed)
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int64_t xyb = p0 / a.Z;
  const int zr = (int)(p0 - xyb * a.Z);
  const int64_t XYn = a.P / a.Z;
  int64_t xyc[4];
  int zbc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int o = zr + wv * 64 + c * 16;
    const int q = o / a.Z;
    xyc[c] = xyb + q;
    zbc[c] = o - q * a.Z;
  }
  if (C2R) {
#pragma unroll
    for (int c = 0; c < (ROW64 ? 1 : 4); ++c) {
#pragma unroll
      for (int h = 0; h < NT; ++h) {
        const int w = h * 16 + (lane & 15);
        const bool ok = w < a.W && 8 * g < a.K2;
        rq[c][h] = *(const uint4*)(a.r2 + (ok ? ((b * a.W + w) * XYn + xyc[c]) * a.K2 + 8 * g : 0));
      }
    }
  }
  // v tile [256 points][32 channels] in LDS, zero beyond W
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = q * 256 + t;
    const int kl = idx >> 5, pl = (idx & 31) * 8;
    const uint32_t u[4] = {vq[q].x, vq[q].y, vq[q].z, vq[q].w};
#pragma unroll
    for (int i = 0; i < 8; ++i)
      tile[tile_row(pl + i) * PW_TS + tile_col(kl, pl + i)] = (uint16_t)(u[i >> 1] >> (16 * (i & 1)));
  }
  __syncthreads();
  f32x4 acc[NT][4];
#pragma unroll
  for (int h = 0; h < NT; ++h)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[h][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  // channel map (uniform branch: absent in the hybrid layer)
  if (a.Win > 0) {
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      const bf16x8 av = *(const bf16x8*)(a.gwp + (h * 16 + (lane & 15)) * 32 + 8 * g);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int pt = wave * 64 + c * 16 + (lane & 15);
        const bf16x8 bv = *(const bf16x8*)(tile + tile_row(pt) * PW_TS + tile_col(8 * g, pt));
        acc[h][c] = mfma16(av, bv, acc[h][c]);
      }
    }
  }
  // c2r along z, with its own accumulators, added to the channel map's in
  // the epilogue
  f32x4 acc2[NT][4];
#pragma unroll
  for (int h = 0; h < NT; ++h)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc2[h][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4 * C2R; ++c) {
    const int zb = zbc[c];  // first z of the tile
    const bf16x8 bv = *(const bf16x8*)(a.gi1 + (int64_t)(zb + (lane & 15)) * a.gi1_kp + 8 * g);
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      const int w = h * 16 + (lane & 15);
      const bool ok = w < a.W && 8 * g < a.K2;
      const uint4 rr = rq[ROW64 ? 0 : c][h];
      const uint32_t e[4] = {ok ? rr.x : 0u, ok ? rr.y : 0u, ok ? rr.z : 0u, ok ? rr.w : 0u};
      bf16x8 av;
#pragma unroll
      for (int j = 0; j < 8; ++j) av[j] = __builtin_bit_cast(__bf16, (uint16_t)(e[j >> 1] >> (16 * (j & 1))));
      acc2[h][c] = mfma16(av, bv, acc2[h][c]);
    }
  }
  const int l16 = lane & 15;
  float* hout = a.h ? a.h + b * a.W * a.P + p0 : nullptr;
  uint16_t* act = a.act ? a.act + b * a.W * a.P + p0 : nullptr;
  const float* gm = a.gmul ? a.gmul + b * a.W * a.P + p0 : nullptr;
  // this thread's BF16 activations, kept for the z-DFT tile, which is
  // written over the result tile once every thread has read its values
  uint2 wz[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wz[q] = uint2{0u, 0u};
  // the two products' sum, formed before the staging so the second half
  // waits in 16 registers rather than 32
  f32x4 sum[NT][4];
#pragma unroll
  for (int h = 0; h < NT; ++h)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[h][c][r] = acc[h][c][r] + acc2[h][c][r];
  // the result passes through LDS one 16-row half (channel tile hh) at a
  // time; thread t reads rows wave + 4 qq of the half
#pragma unroll
  for (int hh = 0; hh < NT; ++hh) {
    __syncthreads();  // the v tile, or the previous half, is dead
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dst[(4 * g + r) * PW_J + le_col(4 * g + r, wave * 64 + c * 16 + l16)] = sum[hh][c][r];
    __syncthreads();
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int q = 4 * hh + qq;
    const int e = t + 256 * q;
    const int n = e >> 6, p4 = (e & 63) * 4, nl = n - 16 * hh;
    if (n >= a.W) continue;
    float4 v = *(const float4*)(dst + nl * PW_J + le_col(nl, p4));
    const int64_t off = (int64_t)n * a.P + p4;
    if (a.bias) {
      const float bb = a.bias[n];
      v.x += bb; v.y += bb; v.z += bb; v.w += bb;
    }
    if (a.resid) {
      const float4 rr = *(const float4*)(a.resid + b * a.W * a.P + p0 + off);
      v.x += rr.x; v.y += rr.y; v.z += rr.z; v.w += rr.w;
    }
    if (gm) {
      const float4 hh = *(const float4*)(gm + off);
      v.x *= gelu_grad(hh.x); v.y *= gelu_grad(hh.y); v.z *= gelu_grad(hh.z); v.w *= gelu_grad(hh.w);
    }
    if (hout) *(float4*)(hout + off) = v;
    if (!act) continue;
    uint2 w;
    if (a.act_gelu) {
      w.x = f2bf2(gelu(v.x), gelu(v.y));
      w.y = f2bf2(gelu(v.z), gelu(v.w));
    } else {
      w.x = f2bf2(v.x, v.y);
      w.y = f2bf2(v.z, v.w);
    }
    *(uint2*)(act + off) = w;
    wz[q] = w;
  }
  }
  if (a.a1) {
    __syncthreads();  // the result tile is read: its region becomes the activation tile
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      const int n = e >> 6, p4 = (e & 63) * 4;
      if (n < a.W) *(uint2*)(at + n * AP + p4) = wz[q];
    }
    __syncthreads();
    // columns (w, row) = 16 ct + l16 with w = col / 4 and row = col % 4 the
    // (x, y) row within the block; rows of the result k = 16 rt + 4 g + r
    f32x4 za[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) za[rt][cc] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 ga[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) ga[rt] = *(const bf16x8*)(a.gz + (rt * 16 + l16) * a.gz_kp + ks * 32 + 8 * g);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int col = (2 * wave + cc) * 16 + l16;
        const bf16x8 bv = *(const bf16x8*)(at + (col >> 2) * AP + (col & 3) * 64 + ks * 32 + 8 * g);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) za[rt][cc] = mfma16(ga[rt], bv, za[rt][cc]);
      }
    }
    const int64_t xy0 = p0 / 64, XY = a.P / 64;
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const int col = (2 * wave + cc) * 16 + l16;
      uint16_t* d1 = a.a1 + ((b * a.W + (col >> 2)) * XY + xy0 + (col & 3)) * 32;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        *(uint2*)(d1 + rt * 16 + 4 * g) = uint2{f2bf2(za[rt][cc][0], za[rt][cc][1]),
                                                f2bf2(za[rt][cc][2], za[rt][cc][3])};
    }
  }
}

// ------------------------------------------------------------- projection
// Fused projection (inference): for every point of v [B][W][P] (BF16)
//   y[b][o][p] = q2[o] + sum_h Q2[o][h] bf16(GELU(q1[h] + sum_c Q1[h][c] v[b][c][p]))
// BF16 operands, FP32 accumulation; the GELU output is rounded to BF16 as
// the unfused path stores it.  Q1p [16 NT][32 KS] and Q2p [16][16 NT] are
// BF16 and zero padded, q1p [16 NT] FP32 zero padded (NT even).  A block
// covers 256 consecutive points of one sample (P % 256 == 0); each wave 64
// points as four 16-point MFMA column tiles.  The hidden accumulators feed
// the second contraction directly: for its k-step s, lane group g supplies
// k slots 8g..8g+7 holding hidden rows 32s + 4g + {0..3} (tile 2s) and
// 32s + 16 + 4g + {0..3} (tile 2s+1), and the Q2 operand is gathered with
// the same assignment, so the sum runs over every hidden row once.
// With STORE_A (training) the BF16 hidden activation is also stored to
// aout [B][H][P], for the gradient of Q2.  ACT selects the hidden
// activation: 0 GELU, 1 the SIREN sine sin(w0 h).
// RES selects the residual feed-forward form of the hybrid F/FNO layer:
//   vout[b][o][p] = bf16(resid[b][o][p] + q2[o] + sum_h Q2[o][h] act(...))
// with cout = W <= 32 outputs (two 16-row output tiles, Q2p [32][16 NT]),
// resid and vout BF16 [B][W][P].
// The sine runs on the hardware sine and cosine (argument in revolutions,
// valid within +-256 revolutions) with the library functions beyond that.
__device__ __forceinline__ float sin_w(float x) {
  const float r = x * 0.15915494309189535f;
  return fabsf(r) < 256.f ? __builtin_amdgcn_sinf(r) : sinf(x);
}
__device__ __forceinline__ float cos_w(float x) {
  const float r = x * 0.15915494309189535f;
  return fabsf(r) < 256.f ? __builtin_amdgcn_cosf(r) : cosf(x);
}
template <int ACT>
__device__ __forceinline__ float proj_act(float h, float w0) {
  return ACT == 1 ? sin_w(w0 * h) : gelu(h);
}
template <int ACT>
__device__ __forceinline__ float proj_act_grad(float h, float w0) {
  return ACT == 1 ? w0 * cos_w(w0 * h) : gelu_grad(h);
}
// the activation and its derivative together (one CDF evaluation for GELU)
template <int ACT>
__device__ __forceinline__ void proj_act_both(float h, float w0, float& a, float& da) {
  if (ACT == 1) {
    a = sin_w(w0 * h);
    da = w0 * cos_w(w0 * h);
  } else {
    const float cdf = norm_cdf_fit(h);
    const float hc = __builtin_amdgcn_fmed3f(h, -6.f, 6.f);
    a = h * cdf;
    da = fmaf(h * 0.39894228f, __builtin_amdgcn_exp2f(-0.72134752f * hc * hc), cdf);
  }
}
// (the GELU instances with one k step and no stored activation: four waves
// per SIMD, 128 registers)
template <int NT, int KS, bool STORE_A = false, int ACT = 0, bool RES = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ACT == 0 && KS == 1 && !STORE_A ? 4 : 1)))
void proj_kernel(const uint16_t* __restrict__ v, int W, int64_t P, const uint16_t* __restrict__ Q1p,
                 const float* __restrict__ q1p, const uint16_t* __restrict__ Q2p, const float* __restrict__ q2,
                 int cout, float* __restrict__ y, int H = 0, uint16_t* __restrict__ aout = nullptr, float w0 = 0.f,
                 const uint16_t* __restrict__ resid = nullptr, uint16_t* __restrict__ vout = nullptr) {
  constexpr int WP = 32 * KS, VS = WP + 8, HP = 16 * NT, OT = RES ? 2 : 1;
  // Q2 rows padded by 8: the gather of the second-stage operand reads one
  // column of 16 rows at a time, which with unpadded rows of 64 words would
  // all fall in one LDS bank
  constexpr int Q2S = HP + 8;
  // RES: per wave the FP32 output tile [32][16 points] (row pitch 20, so the
  // four lane groups of a store hit disjoint banks); it reuses the Q2 rows,
  // which are dead once the operand is gathered
  constexpr int SP = 20;
  constexpr int Q2_BYTES = 16 * OT * Q2S * 2, STG_BYTES = RES ? 4 * 32 * SP * 4 : 0;
  __shared__ __attribute__((aligned(16))) uint16_t vt[256 * VS];
  __shared__ __attribute__((aligned(16))) uint16_t q1s[HP * WP];
  __shared__ __attribute__((aligned(16))) unsigned char q2buf[Q2_BYTES > STG_BYTES ? Q2_BYTES : STG_BYTES];
  uint16_t* q2s = (uint16_t*)q2buf;
  float* stg = (float*)q2buf;
  // per wave: the BF16 hidden tile [HP][16 points] of one column tile
  __shared__ __attribute__((aligned(16))) uint16_t hs[STORE_A ? 4 * HP * 16 : 8];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int64_t b = j0 / P, p0 = j0 % P;
  // RES: in the epilogue lane (c, half) = (lane / 2, lane % 2) completes 8
  // consecutive points of channel c; its residual values for every column
  // tile are loaded here, before anything waits, 16 bytes per tile
  const int rc = lane >> 1, rh = lane & 1;
  uint4 rres[RES ? 4 : 1];
  if (RES) {
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      rres[ct] = rc < cout ? *(const uint4*)(resid + (b * cout + rc) * P + p0 + wave * 64 + ct * 16 + 8 * rh)
                           : uint4{0u, 0u, 0u, 0u};
  }
  // operands into LDS
  for (int e = t * 8; e < HP * WP; e += 256 * 8) *(uint4*)(q1s + e) = *(const uint4*)(Q1p + e);
  for (int e = t * 8; e < 16 * OT * HP; e += 256 * 8) *(uint4*)(q2s + (e / HP) * Q2S + e % HP) = *(const uint4*)(Q2p + e);
  // v tile, transposed to [point][channel]
  for (int idx = t; idx < WP * 32; idx += 256) {
    const int c = idx >> 5, g8 = (idx & 31) * 8;
    uint16_t val[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (c < W) Vec8<uint16_t>::load(v + (b * W + c) * P + p0 + g8, val);
#pragma unroll
    for (int i = 0; i < 8; ++i) vt[tile_row(g8 + i) * VS + tile_col(c, g8 + i)] = val[i];
  }
  __syncthreads();
  // second-stage A operand (Q2 rows o = 16 ot + lane % 16), gathered once
  bf16x8 a2[OT][NT / 2];
#pragma unroll
  for (int ot = 0; ot < OT; ++ot)
#pragma unroll
    for (int s = 0; s < NT / 2; ++s)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int h = 32 * s + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
        a2[ot][s][j] = __builtin_bit_cast(__bf16, q2s[(ot * 16 + (lane & 15)) * Q2S + h]);
      }
  if (RES) __syncthreads();  // every wave has its operand: the Q2 rows become the output tiles
  // (unrolled in the residual form, whose prefetched values are indexed by ct)
  constexpr int CT_UNROLL = RES ? 4 : 1;
#pragma unroll CT_UNROLL
  for (int ct = 0; ct < 4; ++ct) {
    const int pt = wave * 64 + ct * 16 + (lane & 15);
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const bf16x8 bv = *(const bf16x8*)(vt + tile_row(pt) * VS + tile_col(ks * 32 + 8 * g, pt));
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8 av = *(const bf16x8*)(q1s + (nt * 16 + (lane & 15)) * WP + ks * 32 + 8 * g);
        acc[nt] = mfma16(av, bv, acc[nt]);
      }
    }
    const int64_t p = p0 + wave * 64 + ct * 16 + (lane & 15);
    f32x4 out[OT];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot) out[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NT / 2; ++s) {
      bf16x8 bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int nt = 2 * s + (j >> 2), r = j & 3;
        const float h = acc[nt][r] + q1p[nt * 16 + 4 * g + r];
        const uint16_t hb = f2bf(proj_act<ACT>(h, w0));
        bv[j] = __builtin_bit_cast(__bf16, hb);
        if (STORE_A) hs[wave * HP * 16 + (nt * 16 + 4 * g + r) * 16 + (lane & 15)] = hb;
      }
#pragma unroll
      for (int ot = 0; ot < OT; ++ot) out[ot] = mfma16(a2[ot][s], bv, out[ot]);
    }
    if (STORE_A) {
      wave_lds_sync();  // the wave's hidden tile is complete
      // rows h of 16 points, two 16-byte halves each
      for (int e = lane; e < HP * 2; e += 64) {
        const int hr = e >> 1, half = e & 1;
        if (hr < H)
          *(uint4*)(aout + (b * H + hr) * P + p0 + wave * 64 + ct * 16 + 8 * half) =
              *(const uint4*)(hs + wave * HP * 16 + hr * 16 + 8 * half);
      }
    }
    if (RES) {
      float* sw = stg + wave * 32 * SP;
#pragma unroll
      for (int ot = 0; ot < OT; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = ot * 16 + 4 * g + r;
          sw[o * SP + (lane & 15)] = out[ot][r] + (o < cout ? q2[o] : 0.f);
        }
      wave_lds_sync();  // the wave's output tile is complete
      if (rc < cout) {
        const uint32_t u[4] = {rres[ct].x, rres[ct].y, rres[ct].z, rres[ct].w};
        const float4 f0 = *(const float4*)(sw + rc * SP + 8 * rh), f1 = *(const float4*)(sw + rc * SP + 8 * rh + 4);
        const float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float lo = f[2 * i] + __uint_as_float(u[i] << 16);
          const float hi = f[2 * i + 1] + __uint_as_float(u[i] & 0xffff0000u);
          w[i] = f2bf2(lo, hi);
        }
        *(uint4*)(vout + (b * cout + rc) * P + p0 + wave * 64 + ct * 16 + 8 * rh) = uint4{w[0], w[1], w[2], w[3]};
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        if (o < cout) y[(b * cout + o) * P + p] = out[0][r] + q2[o];
      }
    }
  }
}

// Fused projection backward (training), per point of v [B][W][P]:
//   h1 = q1 + Q1 v                        (recomputed, as in the forward)
//   ga = GELU'(h1) * (Q2^T gy)            stored BF16 to ga [B][H][P]
//   gv = Q1^T ga                          stored FP32 to gv [B][W][P]
// with gy [B][cout][P] the gradient at the output.  h1 comes from the same
// MFMA products and the same bias add as the forward's, so it is not kept
// between the passes.  Q2t [16 NT][kp2] is Q2 transposed (rows h, k = o),
// BF16, zero padded; the Q1^T operand is gathered from Q1p with the hidden
// rows permuted as the forward's second stage, so that ga feeds it straight
// from the accumulator registers.  Block and wave layout as proj_kernel.
// PF (the hybrid's feed-forward, cout = 32) loads the next column tile's gy
// while the current one computes.
// GQ2 (cout <= 8) also forms the Q2 gradient, so that the forward pass need
// not store the hidden activation: each column tile's BF16 activation
//   a = bf16(act(h1))                     (the forward's value, recomputed)
// goes through the wave's tile, and sum_p gy[o][p] a[h][p] over its 16
// points is formed on MFMA (points as k; the upper 16 k are zero) and
// added, per lane in column-tile order, into the wave's LDS sums of rows
// o < 8.  The block's four waves are summed in a fixed order into
// q2part[block][o][h] (cout x H), reduced over blocks on the host side.
template <int NT, int KS, int ACT = 0, bool PF = false, bool GQ2 = false>
__global__ __launch_bounds__(256) void proj_bwd_kernel(const uint16_t* __restrict__ v, int W, int64_t P,
                                                       const uint16_t* __restrict__ Q1p, const float* __restrict__ q1p,
                                                       const uint16_t* __restrict__ Q2t, int kp2,
                                                       const float* __restrict__ gy, int cout, int H,
                                                       uint16_t* __restrict__ ga, float* __restrict__ gv,
                                                       float w0 = 0.f, float* __restrict__ q2part = nullptr) {
  constexpr int WP = 32 * KS, VS = WP + 8, HP = 16 * NT;
  __shared__ __attribute__((aligned(16))) uint16_t vt[256 * VS];
  __shared__ __attribute__((aligned(16))) uint16_t q1s[HP * WP];
  // the Q1^T operand per (step s, column tile, lane), and per wave the BF16
  // gradient tile [HP][16 points] of one column tile
  __shared__ __attribute__((aligned(16))) bf16x8 q1t[(NT / 2) * (2 * KS) * 64];
  __shared__ __attribute__((aligned(16))) uint16_t hs[4 * HP * 16];
  // GQ2: per wave the Q2 gradient sums [8 rows o][HP]
  __shared__ __attribute__((aligned(16))) float qacc[GQ2 ? 4 * 8 * HP : 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, l16 = lane & 15;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int64_t b = j0 / P, p0 = j0 % P;
  for (int e = t * 8; e < HP * WP; e += 256 * 8) *(uint4*)(q1s + e) = *(const uint4*)(Q1p + e);
  for (int idx = t; idx < WP * 32; idx += 256) {
    const int c = idx >> 5, g8 = (idx & 31) * 8;
    uint16_t val[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (c < W) Vec8<uint16_t>::load(v + (b * W + c) * P + p0 + g8, val);
#pragma unroll
    for (int i = 0; i < 8; ++i) vt[tile_row(g8 + i) * VS + tile_col(c, g8 + i)] = val[i];
  }
  __syncthreads();
  // A operand of Q1^T: rows c = 16 ct2 + l16, k slots of step s holding the
  // hidden rows 32 s + 4 g + {0..3} and 32 s + 16 + 4 g + {0..3}
  for (int e = t; e < (NT / 2) * (2 * KS) * 64; e += 256) {
    const int ln = e & 63, ct2 = (e >> 6) % (2 * KS), s = (e >> 6) / (2 * KS);
    const int gg = ln >> 4, cc = ct2 * 16 + (ln & 15);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int h = 32 * s + (j < 4 ? 4 * gg + j : 16 + 4 * gg + (j - 4));
      o[j] = __builtin_bit_cast(__bf16, q1s[h * WP + cc]);
    }
    q1t[e] = o;
  }
  __syncthreads();
  uint16_t* hw = hs + wave * HP * 16;
  if (GQ2 && g < 2) {
    // lanes of groups 0 and 1 own rows o = 4 g + r, columns 16 nt + l16
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) qacc[(wave * 8 + 4 * g + r) * HP + nt * 16 + l16] = 0.f;
  }
  float gnx[PF ? 8 : 1];
  if (PF) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int o = 8 * g + j;
      gnx[j] = o < cout ? gy[(b * cout + o) * P + p0 + wave * 64 + l16] : 0.f;
    }
  }
#pragma unroll 1
  for (int ct = 0; ct < 4; ++ct) {
    const int pt = wave * 64 + ct * 16 + l16;
    const int64_t p = p0 + pt;
    bf16x8 vb[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) vb[ks] = *(const bf16x8*)(vt + tile_row(pt) * VS + tile_col(ks * 32 + 8 * g, pt));
    // gy operand: column = this point, k = o (zero beyond cout)
    bf16x8 gb;
    if (PF) {
      float gc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) gc[j] = gnx[j];
      if (ct < 3) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int o = 8 * g + j;
          gnx[j] = o < cout ? gy[(b * cout + o) * P + p + 16] : 0.f;
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) gb[j] = __builtin_bit_cast(__bf16, f2bf(gc[j]));
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int o = 8 * g + j;
        gb[j] = __builtin_bit_cast(__bf16, o < cout ? f2bf(gy[(b * cout + o) * P + p]) : (uint16_t)0);
      }
    }
    f32x4 go[2 * KS];
#pragma unroll
    for (int ct2 = 0; ct2 < 2 * KS; ++ct2) go[ct2] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint32_t apk[GQ2 ? NT : 1][2];  // GQ2: packed BF16 activation, (r = 0, 1) and (r = 2, 3)
    // one k step of Q1^T at a time: hidden tiles 2 s and 2 s + 1
#pragma unroll
    for (int s = 0; s < NT / 2; ++s) {
      uint32_t u[4];  // packed BF16 gradient, (tile, r = 0, 1) and (tile, r = 2, 3)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int nt = 2 * s + hh, hr = nt * 16 + 4 * g;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          acc = mfma16(*(const bf16x8*)(q1s + (nt * 16 + l16) * WP + ks * 32 + 8 * g), vb[ks], acc);
        const f32x4 tq = mfma16(*(const bf16x8*)(Q2t + (nt * 16 + l16) * kp2 + 8 * g), gb, f32x4{0.f, 0.f, 0.f, 0.f});
        float d[4];
        if (GQ2) {
          float av[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float da;
            proj_act_both<ACT>(acc[r] + q1p[hr + r], w0, av[r], da);
            d[r] = tq[r] * da;
          }
          apk[GQ2 ? nt : 0][0] = f2bf2(av[0], av[1]);
          apk[GQ2 ? nt : 0][1] = f2bf2(av[2], av[3]);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) d[r] = tq[r] * proj_act_grad<ACT>(acc[r] + q1p[hr + r], w0);
        }
        u[2 * hh] = f2bf2(d[0], d[1]);
        u[2 * hh + 1] = f2bf2(d[2], d[3]);
#pragma unroll
        for (int r = 0; r < 4; ++r) hw[(hr + r) * 16 + l16] = (uint16_t)(u[2 * hh + (r >> 1)] >> (16 * (r & 1)));
      }
      bf16x8 bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[j] = __builtin_bit_cast(__bf16, (uint16_t)(u[j >> 1] >> (16 * (j & 1))));
#pragma unroll
      for (int ct2 = 0; ct2 < 2 * KS; ++ct2) go[ct2] = mfma16(q1t[(s * 2 * KS + ct2) * 64 + lane], bv, go[ct2]);
    }
#pragma unroll
    for (int ct2 = 0; ct2 < 2 * KS; ++ct2)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = ct2 * 16 + 4 * g + r;
        if (c < W) gv[(b * W + c) * P + p] = go[ct2][r];
      }
    wave_lds_sync();  // the wave's gradient tile is complete
    // rows h of 16 points, two 16-byte halves each
    for (int e = lane; e < HP * 2; e += 64) {
      const int hr = e >> 1, half = e & 1;
      if (hr < H)
        *(uint4*)(ga + (b * H + hr) * P + p0 + wave * 64 + ct * 16 + 8 * half) =
            *(const uint4*)(hw + hr * 16 + 8 * half);
    }
    if (GQ2) {
      // the activation tile replaces the gradient tile just stored
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          hw[(nt * 16 + 4 * g + r) * 16 + l16] = (uint16_t)(apk[GQ2 ? nt : 0][r >> 1] >> (16 * (r & 1)));
      wave_lds_sync();
      // A: rows o = l16 (zero from cout on), k = the tile's points 8 g + j
      // for g < 2; B: columns h, the same points, from the tile
      bf16x8 ya;
      const bool live = g < 2 && l16 < cout;
      const float* gr = gy + (b * cout + (live ? l16 : 0)) * P + p0 + wave * 64 + ct * 16 + 8 * (g & 1);
      const float4 y0 = *(const float4*)gr, y1 = *(const float4*)(gr + 4);
      const float yv[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
#pragma unroll
      for (int j = 0; j < 8; ++j) ya[j] = __builtin_bit_cast(__bf16, live ? f2bf(yv[j]) : (uint16_t)0);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        bf16x8 ab = *(const bf16x8*)(hw + (nt * 16 + l16) * 16 + 8 * (g & 1));
        if (g >= 2) {
#pragma unroll
          for (int j = 0; j < 8; ++j) ab[j] = __builtin_bit_cast(__bf16, (uint16_t)0);
        }
        const f32x4 pq = mfma16(ya, ab, f32x4{0.f, 0.f, 0.f, 0.f});
        if (g < 2) {
#pragma unroll
          for (int r = 0; r < 4; ++r) qacc[(wave * 8 + 4 * g + r) * HP + nt * 16 + l16] += pq[r];
        }
      }
    }
  }
  if (GQ2) {
    // the four waves' sums, added in wave order
    __syncthreads();
    for (int e = t; e < cout * H; e += 256) {
      const int o = e / H, h = e % H;
      const float sum = ((qacc[(0 * 8 + o) * HP + h] + qacc[(1 * 8 + o) * HP + h]) + qacc[(2 * 8 + o) * HP + h]) +
                        qacc[(3 * 8 + o) * HP + h];
      q2part[(int64_t)blockIdx.x * cout * H + e] = sum;
    }
  }
}

// ------------------------------------------------------------------ mixing
// Retained modes are stored mode-minor in BF16, [B][C][MX][2][Q] with
// Q = MY * MZ and mode m = kx * Q + q (q = ky * MZ + kz), the layout of the
// DFT intermediates: the x-stage DFT and its inverse then read and write
// whole q-runs.  A mixing block takes one kx and MQ consecutive q (MQ modes)
// for up to 16 batch rows per pass.  It stages the [MQ][rows] slab in LDS
// from 16-byte loads of 2 MQ-byte q-runs, runs each mode's product on MFMA
// (one mode per wave at a time), and writes the result slab back the same
// way.  The capacity class CM bounds the channel count C (C <= CM,
// C % 16 == 0); MQ = 32 for CM = 32 and 16 for CM = 64.
constexpr int MIX_B = 16;          // batch rows per pass
constexpr int MIX_THREADS = 512;   // 8 waves
template <int CM> struct MixCfg {
  static constexpr int MQ = CM <= 32 ? 32 : 16;
  static constexpr int PITCH = MIX_B * 2 * CM + 8;  // slab row of one mode (BF16), 16-byte multiple
};

// slab[ql][ri] = src(b0 + b, k, q0 + ql) for b < nb (0 beyond), k = 2c + part,
// ri = b * 2C + k, or k * 16 + b when KB is set
template <int CM, bool KB>
__device__ __forceinline__ void mix_slab_load(const uint16_t* __restrict__ src, uint16_t* slab, int pitch, int b0,
                                              int nb, int C, int MX, int64_t Q, int kx, int64_t q0) {
  constexpr int MQ = MixCfg<CM>::MQ, HQ = MQ / 8;
  const int K = 2 * C;
  for (int idx = threadIdx.x; idx < MIX_B * K * HQ; idx += MIX_THREADS) {
    const int h = idx % HQ, r = idx / HQ;
    const int b = r / K, k = r - b * K;
    uint4 v = {0u, 0u, 0u, 0u};
    if (b < nb)
      v = *(const uint4*)(src + ((((int64_t)(b0 + b) * C + (k >> 1)) * MX + kx) * 2 + (k & 1)) * Q + q0 + 8 * h);
    const int ri = KB ? k * MIX_B + b : r;
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) slab[(8 * h + i) * pitch + ri] = (uint16_t)(u[i >> 1] >> (16 * (i & 1)));
  }
}

// Per mode m, batch rows b, complex channels:
//   Y[b][o] = sum_c V[b][c] W[m][c][o]                      (MODE 0)
//   gV[b][c] = sum_o gY[b][o] conj(W[m][c][o])              (MODE 1)
// W in BF16 [m][c][o][2] (re, im).  As a real contraction over
// k = (c, part) -> n = (o, part') with the embedding [[Wr, Wi], [-Wi, Wr]]
// (MODE 0) or its transpose (MODE 1).  in and out are mode-minor BF16.
// Grid: MX * Q / MQ blocks of MIX_THREADS.
template <int CM, int MODE>
__global__ __launch_bounds__(MIX_THREADS) void mix_kernel(const uint16_t* __restrict__ in,
                                                          const uint16_t* __restrict__ w,
                                                          uint16_t* __restrict__ out, int B, int C, int MX,
                                                          int64_t Q) {
  constexpr int MQ = MixCfg<CM>::MQ, HQ = MQ / 8, PITCH = MixCfg<CM>::PITCH;
  __shared__ __attribute__((aligned(16))) uint16_t slab[MQ * PITCH];
  const int nqb = (int)(Q / MQ);
  const int kx = blockIdx.x / nqb;
  const int64_t q0 = (int64_t)(blockIdx.x % nqb) * MQ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
  const int K = 2 * C;  // also N
  for (int b0 = 0; b0 < B; b0 += MIX_B) {
    const int nb = min(MIX_B, B - b0);
    mix_slab_load<CM, false>(in, slab, PITCH, b0, nb, C, MX, Q, kx, q0);
    __syncthreads();
    for (int ql = wave; ql < MQ; ql += MIX_THREADS / 64) {
      const uint16_t* wm = w + ((int64_t)kx * Q + q0 + ql) * C * C * 2;
      uint16_t* row = slab + ql * PITCH;
      f32x4 acc[CM / 8];
#pragma unroll
      for (int nt = 0; nt < CM / 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < K / 32; ++ks) {
        // A: row b = l16, k = 32 ks + 8 g + j
        const bf16x8 av = *(const bf16x8*)(row + l16 * K + ks * 32 + 8 * g);
#pragma unroll
        for (int nt = 0; nt < CM / 8; ++nt) {
          if (nt * 16 >= K) break;
          const int n = nt * 16 + l16, o = n >> 1, po = n & 1;
          // B: col n, k = 32 ks + 8 g + j = (c, pi) with c = 16 ks + 4 g + j / 2, pi = j % 2
          uint16_t e[8];
          if (MODE == 0) {
            // element ((c, pi), (o, po)): po = 0 -> (Wr, -Wi), po = 1 -> (Wi, Wr)
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
              const uint32_t wv = *(const uint32_t*)(wm + ((int64_t)(ks * 16 + 4 * g + cc) * C + o) * 2);
              const uint16_t wr = (uint16_t)(wv & 0xffffu), wi = (uint16_t)(wv >> 16);
              e[2 * cc] = po ? wi : wr;
              e[2 * cc + 1] = po ? wr : (uint16_t)(wi ^ 0x8000u);
            }
          } else {
            // k = (o', pi), n = (c', po): W[c'][o'] for four consecutive o';
            // element: po = 0 -> (Wr, Wi), po = 1 -> (-Wi, Wr)
            const uint4 wv = *(const uint4*)(wm + ((int64_t)o * C + ks * 16 + 4 * g) * 2);
            const uint32_t u[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
              const uint16_t wr = (uint16_t)(u[cc] & 0xffffu), wi = (uint16_t)(u[cc] >> 16);
              e[2 * cc] = po ? (uint16_t)(wi ^ 0x8000u) : wr;
              e[2 * cc + 1] = po ? wr : wi;
            }
          }
          bf16x8 bv;
#pragma unroll
          for (int j = 0; j < 8; ++j) bv[j] = __builtin_bit_cast(__bf16, e[j]);
          acc[nt] = mfma16(av, bv, acc[nt]);
        }
      }
      // D: col n = 16 nt + l16, row b = 4 g + r; the mode's own slab row is
      // overwritten only by this wave, after its last read of it
#pragma unroll
      for (int nt = 0; nt < CM / 8; ++nt) {
        if (nt * 16 >= K) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) row[(4 * g + r) * K + nt * 16 + l16] = f2bf(acc[nt][r]);
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < MIX_B * K * HQ; idx += MIX_THREADS) {
      const int h = idx % HQ, r = idx / HQ;
      const int b = r / K, k = r - b * K;
      if (b >= nb) continue;
      uint32_t u[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        u[i] = (uint32_t)slab[(8 * h + 2 * i) * PITCH + r] | ((uint32_t)slab[(8 * h + 2 * i + 1) * PITCH + r] << 16);
      *(uint4*)(out + ((((int64_t)(b0 + b) * C + (k >> 1)) * MX + kx) * 2 + (k & 1)) * Q + q0 + 8 * h) =
          uint4{u[0], u[1], u[2], u[3]};
    }
    __syncthreads();
  }
}

// Spectral weight gradient, per mode: gW[m][c][o] (+)= sum_b conj(V[b][c]) gY[b][o]
// as R[(c,p)][(o,p')] = sum_b V[b][(c,p)] gY[b][(o,p')] (K = batch rows,
// 16 per pass, zero padded to 32), then gWr = R00 + R11, gWi = R01 - R10.
// V and gY are mode-minor BF16; gw is FP32 [m][c][o][2], overwritten unless
// accumulate is set (later passes over the batch always add).
template <int CM>
__global__ __launch_bounds__(MIX_THREADS) void mix_grad_kernel(const uint16_t* __restrict__ v,
                                                               const uint16_t* __restrict__ gy,
                                                               float* __restrict__ gw, int B, int C, int MX,
                                                               int64_t Q, int accumulate) {
  constexpr int MQ = MixCfg<CM>::MQ, PITCH = MixCfg<CM>::PITCH;
  __shared__ __attribute__((aligned(16))) uint16_t sv[MQ * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t sy[MQ * PITCH];
  const int nqb = (int)(Q / MQ);
  const int kx = blockIdx.x / nqb;
  const int64_t q0 = (int64_t)(blockIdx.x % nqb) * MQ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
  const int K2 = 2 * C;
  constexpr int NT = CM / 8;
  for (int b0 = 0; b0 < B; b0 += MIX_B) {
    const int nb = min(MIX_B, B - b0);
    mix_slab_load<CM, true>(v, sv, PITCH, b0, nb, C, MX, Q, kx, q0);
    mix_slab_load<CM, true>(gy, sy, PITCH, b0, nb, C, MX, Q, kx, q0);
    __syncthreads();
    for (int ql = wave; ql < MQ; ql += MIX_THREADS / 64) {
      // A: row (c, p) = 16 rt + l16, k = b = 8 g + j (g < 2; zero beyond 16)
      bf16x8 av[NT], bv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        av[t] = bf16x8{};
        bv[t] = bf16x8{};
        if (t * 16 < K2 && g < 2) {
          av[t] = *(const bf16x8*)(sv + ql * PITCH + (t * 16 + l16) * MIX_B + 8 * g);
          bv[t] = *(const bf16x8*)(sy + ql * PITCH + (t * 16 + l16) * MIX_B + 8 * g);
        }
      }
      float* gm = gw + ((int64_t)kx * Q + q0 + ql) * C * C * 2;
      const bool add = accumulate || b0 > 0;
#pragma unroll
      for (int rt = 0; rt < NT; ++rt) {
        if (rt * 16 >= K2) break;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          if (ct * 16 >= K2) break;
          const f32x4 acc = mfma16(av[rt], bv[ct], f32x4{0.f, 0.f, 0.f, 0.f});
          // lane holds R[row = 16 rt + 4 g + r][col = 16 ct + l16]
          const float nb0 = __shfl_xor(acc[0], 1), nb1 = __shfl_xor(acc[1], 1);
          const float nb2 = __shfl_xor(acc[2], 1), nb3 = __shfl_xor(acc[3], 1);
          if ((l16 & 1) == 0) {
            const int o = (ct * 16 + l16) >> 1;
            const int c0 = (rt * 16 + 4 * g) >> 1;
            // rows r = 0, 1: (c0, re), (c0, im); rows 2, 3: (c0 + 1, re), (c0 + 1, im)
            float2* d0 = (float2*)(gm + ((int64_t)c0 * C + o) * 2);
            float2* d1 = (float2*)(gm + ((int64_t)(c0 + 1) * C + o) * 2);
            float2 x0 = {acc[0] + nb1, nb0 - acc[1]}, x1 = {acc[2] + nb3, nb2 - acc[3]};
            if (add) {
              const float2 p0 = *d0, p1 = *d1;
              x0.x += p0.x; x0.y += p0.y; x1.x += p1.x; x1.y += p1.y;
            }
            *d0 = x0;
            *d1 = x1;
          }
        }
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------- Gram
// part[chunk][a][c] = sum_{t in chunk} X[a][t] Y[c][t], rows of X and Y with
// stride rs (per batch sample) and sample stride bs; t = (b, p), chunks of
// 2048 points within one sample.  One wave per 16 x 16 output tile.
template <typename XT, typename YT>
__global__ __launch_bounds__(64) void gram_kernel(const XT* __restrict__ X, const YT* __restrict__ Y, float* part,
                                                  int A, int Cc, int64_t P, int64_t xbs, int64_t ybs, int chunk) {
  const int lane = threadIdx.x;
  const int64_t ch = blockIdx.x;
  const int64_t per_b = P / chunk;
  const int64_t b = ch / per_b, p0 = (ch % per_b) * chunk;
  const int at = blockIdx.y, ct = blockIdx.z;
  const int row = at * 16 + (lane & 15), col = ct * 16 + (lane & 15);
  const XT* xr = X + b * xbs + (int64_t)row * P + p0;
  const YT* yr = Y + b * ybs + (int64_t)col * P + p0;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < chunk; k0 += 32) {
    bf16x8 av, bv;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + 8 * (lane >> 4) + q;
      av[q] = row < A ? __builtin_bit_cast(__bf16, to_bf(xr[k])) : (__bf16)0.0f;
      bv[q] = col < Cc ? __builtin_bit_cast(__bf16, to_bf(yr[k])) : (__bf16)0.0f;
    }
    acc = mfma16(av, bv, acc);
  }
  float* o = part + ch * (int64_t)A * Cc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ar = at * 16 + 4 * (lane >> 4) + r;
    if (ar < A && col < Cc) o[(int64_t)ar * Cc + col] = acc[r];
  }
}

// Gram over points with K split across waves:
//   part[w][a][c] = sum over the GR_CHUNK points t of chunk w of X[b][a][t] Y[b][c][t]
// One wave per chunk (all chunks within one sample); the wave keeps every
// 16 x 16 tile of the A x C result in MFMA accumulators and loads both
// operands straight from memory in fragment layout (8 consecutive points per
// lane, contiguous along the rows).  Rows beyond A or C read row 0 and are
// zeroed by a select, so no branch feeds an MFMA operand.
constexpr int GR_CHUNK = 2048;
// With partc set, the wave also sums every X row over its chunk in FP32
// (the bias gradient), partc[w][a]; BF16 rows are summed as stored.
template <typename XT, typename YT, int AT, int CT>
__global__ __launch_bounds__(256) void gram2_kernel(const XT* __restrict__ X, const YT* __restrict__ Y, float* part,
                                                    int A, int Cc, int64_t P, float* partc) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const int64_t wg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t per_b = P / GR_CHUNK;
  const int64_t b = wg / per_b, p0 = (wg % per_b) * GR_CHUNK + 8 * g;
  const XT* xr[AT];
  const YT* yr[CT];
  bool xok[AT], yok[CT];
#pragma unroll
  for (int i = 0; i < AT; ++i) {
    const int row = i * 16 + (lane & 15);
    xok[i] = row < A;
    xr[i] = X + (b * A + (xok[i] ? row : 0)) * P + p0;
  }
#pragma unroll
  for (int i = 0; i < CT; ++i) {
    const int row = i * 16 + (lane & 15);
    yok[i] = row < Cc;
    yr[i] = Y + (b * Cc + (yok[i] ? row : 0)) * P + p0;
  }
  f32x4 acc[AT][CT];
  float rs[AT];
#pragma unroll
  for (int i = 0; i < AT; ++i) {
    rs[i] = 0.f;
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (int k0 = 0; k0 < GR_CHUNK; k0 += 32) {
    bf16x8 xa[AT], yb[CT];
#pragma unroll
    for (int i = 0; i < AT; ++i) {
      uint16_t v[8];
      if constexpr (std::is_same<XT, float>::value) {
        const float4 lo = *(const float4*)(xr[i] + k0), hi = *(const float4*)(xr[i] + k0 + 4);
        rs[i] += ((lo.x + lo.y) + (lo.z + lo.w)) + ((hi.x + hi.y) + (hi.z + hi.w));
        v[0] = f2bf(lo.x); v[1] = f2bf(lo.y); v[2] = f2bf(lo.z); v[3] = f2bf(lo.w);
        v[4] = f2bf(hi.x); v[5] = f2bf(hi.y); v[6] = f2bf(hi.z); v[7] = f2bf(hi.w);
      } else {
        Vec8<XT>::load(xr[i] + k0, v);
        rs[i] += ((bf2f(v[0]) + bf2f(v[1])) + (bf2f(v[2]) + bf2f(v[3]))) +
                 ((bf2f(v[4]) + bf2f(v[5])) + (bf2f(v[6]) + bf2f(v[7])));
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) xa[i][q] = __builtin_bit_cast(__bf16, xok[i] ? v[q] : (uint16_t)0);
    }
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      uint16_t v[8];
      Vec8<YT>::load(yr[j] + k0, v);
#pragma unroll
      for (int q = 0; q < 8; ++q) yb[j][q] = __builtin_bit_cast(__bf16, yok[j] ? v[q] : (uint16_t)0);
    }
#pragma unroll
    for (int i = 0; i < AT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[i][j] = mfma16(xa[i], yb[j], acc[i][j]);
  }
  float* o = part + wg * (int64_t)A * Cc;
#pragma unroll
  for (int i = 0; i < AT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = i * 16 + 4 * g + r, c = j * 16 + (lane & 15);
        if (a < A && c < Cc) o[(int64_t)a * Cc + c] = acc[i][j][r];
      }
  if (partc) {
    // lanes l, l + 16, l + 32, l + 48 hold quarter sums of the same row
#pragma unroll
    for (int i = 0; i < AT; ++i) {
      float v = rs[i];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      const int row = i * 16 + (lane & 15);
      if (g == 0 && row < A) partc[wg * (int64_t)A + row] = v;
    }
  }
}

// sum over j = 0 .. n - 1 of p[j * step], added in increasing j from 0 (the
// order of the plain loop, so the result is that loop's to the bit), with
// sixteen loads in flight at a time instead of one
template <typename T>
__device__ __forceinline__ float ordered_sum(const T* p, int64_t n, int64_t step) {
  constexpr int U = 16;
  float acc = 0.f;
  int64_t j = 0;
  for (; j + U <= n; j += U) {
    float x[U];
#pragma unroll
    for (int i = 0; i < U; ++i) x[i] = to_f(p[(j + i) * step]);
#pragma unroll
    for (int i = 0; i < U; ++i) acc += x[i];
  }
  for (; j < n; ++j) acc += to_f(p[j * step]);
  return acc;
}

// part2[s][e] = sum over parts k = s, s + S, s + 2S, ... of part[k][e]
__global__ __launch_bounds__(256) void reduce_slices_kernel(const float* part, int64_t nparts, int64_t E, int S,
                                                            float* part2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= E) return;
  const int64_t n = s < nparts ? (nparts - s + S - 1) / S : 0;  // k = s, s + S, ... below nparts
  part2[(int64_t)s * E + e] = ordered_sum(part + (int64_t)s * E + e, n, (int64_t)S * E);
}

// out[e] (+)= sum_s part[s][e], fixed order
__global__ __launch_bounds__(256) void reduce_parts_kernel(const float* part, int64_t nparts, int64_t E, float* out,
                                                           int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  const float s = ordered_sum(part + e, nparts, E);
  out[e] = accumulate ? out[e] + s : s;
}

// per-block partial sums over (b, p) of X[b][a][p]: part[blk][a]
template <typename XT>  // FP32 rows, or BF16 rows summed as stored
__global__ __launch_bounds__(256) void colsum_kernel(const XT* X, int A, int64_t P, int B, int64_t chunk,
                                                     float* part) {
  __shared__ float red[256];
  const int a = blockIdx.y;
  const int64_t per_b = P / chunk;
  const int64_t b = blockIdx.x / per_b, p0 = (blockIdx.x % per_b) * chunk;
  const XT* x = X + (b * A + a) * P + p0;
  const int64_t n = threadIdx.x < chunk ? (chunk - threadIdx.x + 255) / 256 : 0;
  const float s = ordered_sum(x + threadIdx.x, n, (int64_t)256);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * A + a] = red[0];
}

// ------------------------------------------------------------- elementwise
// masked MSE: per-block partial of sum mask (y - t)^2, and gy = 2 mask (y - t) / cnt
// Number of cells with mask != 0 (one block), and the gradient scale
// 1 / (bc * count) rounded once from FP64 (0 for an empty mask).  16-byte
// loads when the mask is 16-byte aligned and P % 16 == 0, bytes otherwise.
__global__ __launch_bounds__(1024) void mask_count_kernel(const uint8_t* mask, int64_t P, double bc,
                                                          long long* cnt, float* scale) {
  __shared__ long long red[1024];
  const int t = threadIdx.x;
  long long c = 0;
  if (((uintptr_t)mask & 15) == 0 && P % 16 == 0) {
    for (int64_t i = (int64_t)t * 16; i < P; i += 1024 * 16) {
      const uint4 q = *(const uint4*)(mask + i);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int k = 0; k < 16; ++k) c += ((w[k >> 2] >> (8 * (k & 3))) & 0xffu) ? 1 : 0;
    }
  } else {
    for (int64_t i = t; i < P; i += 1024) c += mask[i] ? 1 : 0;
  }
  red[t] = c;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) {
    *cnt = red[0];
    *scale = red[0] ? (float)(1.0 / (bc * (double)red[0])) : 0.f;
  }
}

// loss = (sum of the block partials, fixed order) / (bc * count)
__global__ __launch_bounds__(1024) void loss_reduce_kernel(const double* part, int64_t nparts, const long long* cnt,
                                                           double bc, double* loss) {
  __shared__ double red[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < nparts; i += 1024) s += part[i];
  red[t] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) *loss = red[0] / (bc * (double)*cnt);
}

__global__ __launch_bounds__(256) void mse_kernel(const float* y, const float* t, const uint8_t* mask, int64_t P,
                                                  int64_t n, const float* inv_cnt_d, float* gy, double* part) {
  const float inv_cnt = *inv_cnt_d;
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    const float m = mask[i % P] ? 1.f : 0.f;
    const float d = (y[i] - t[i]) * m;
    s = (double)d * (double)d;
    if (gy) gy[i] = 2.f * d * inv_cnt;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// (also refreshes the BF16 working copy wbf of the updated parameters)
__global__ __launch_bounds__(256) void adam_kernel(float* theta, const float* g, float* m, float* v, int64_t n,
                                                   float lr, float b1, float b2, float c1, float c2, float eps,
                                                   uint16_t* wbf) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float th = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  theta[i] = th;
  wbf[i] = f2bf(th);
}

// BF16 copy of a parameter block
__global__ __launch_bounds__(256) void to_bf16_kernel(const float* src, uint16_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// padded transposed BF16 operand gt[n][k] from W[rows][cols]: transpose = 0
// gives gt[n][k] = W[n][k] (n < rows, k < cols), transpose = 1 gives
// gt[n][k] = W[k][n]; zero elsewhere (npad x kp)
__global__ __launch_bounds__(256) void make_gt_kernel(const float* W, int rows, int cols, int transpose, uint16_t* gt,
                                                      int npad, int kp) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)npad * kp) return;
  const int n = (int)(e / kp), k = (int)(e % kp);
  float v = 0.f;
  if (!transpose) {
    if (n < rows && k < cols) v = W[(int64_t)n * cols + k];
  } else {
    if (k < rows && n < cols) v = W[(int64_t)k * cols + n];
  }
  gt[e] = f2bf(v);
}

// ------------------------------------------------------- min-max scaling
constexpr int MM_CHUNK = 4096;
constexpr int MM_MAXC = 16;

// per (sample, chunk, channel) minimum and maximum of x [S][C][P]:
// part[(c * S * nchunk + blockIdx.x) * 2 + {0, 1}]
__global__ __launch_bounds__(256) void minmax_kernel(const float* x, int C, int64_t P, int64_t nchunk, float* part,
                                                     int64_t nblk) {
  __shared__ float rmin[256], rmax[256];
  const int c = blockIdx.y;
  const int64_t s = blockIdx.x / nchunk, p0 = (blockIdx.x % nchunk) * MM_CHUNK;
  const int64_t p1 = p0 + MM_CHUNK < P ? p0 + MM_CHUNK : P;
  const float* r = x + (s * C + c) * P;
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
    const float v = r[p];
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  rmin[threadIdx.x] = lo;
  rmax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rmin[threadIdx.x] = fminf(rmin[threadIdx.x], rmin[threadIdx.x + w]);
      rmax[threadIdx.x] = fmaxf(rmax[threadIdx.x], rmax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)c * nblk + blockIdx.x) * 2] = rmin[0];
    part[((int64_t)c * nblk + blockIdx.x) * 2 + 1] = rmax[0];
  }
}

struct ScaleArgs {
  float off[MM_MAXC];
  float mul[MM_MAXC];
};

// x [S][C][P] in place: x = (x + off[c]) * mul[c] (forward) or x * mul[c] + off[c]
__global__ __launch_bounds__(256) void scale_kernel(float* x, int C, int64_t P, int64_t n, ScaleArgs a, int inverse) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = (int)((i / P) % C);
  x[i] = inverse ? x[i] * a.mul[c] + a.off[c] : (x[i] + a.off[c]) * a.mul[c];
}

}  // namespace mfno
