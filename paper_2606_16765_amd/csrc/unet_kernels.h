// gfx950 kernels of the 3D U-Net surrogate (paper Sec. 4, Table 2; the
// architecture of App. A.2): implicit-GEMM 3x3x3 convolution on BF16 MFMA
// with FP32 accumulation and fused batch-norm statistics, split-K weight
// gradients, batch normalisation with ReLU and its adjoint, 2x2x2 max
// pooling, trilinear upsampling by two and their adjoints, the 1x1x1
// sigmoid head with the masked MSE, and Adam.
//
// Activations are channels-last, [B][X][Y][Z][C] with C fastest, so that the
// eight consecutive channels an MFMA operand lane needs are one 16-byte load.
// Every channel count on the device is a multiple of 8 (the 4 input channels
// are padded to 8 with zeros).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace munet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 with round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float bflo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bfhi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void unpack8(const uint4& w, float* f) {
  f[0] = bflo(w.x); f[1] = bfhi(w.x); f[2] = bflo(w.y); f[3] = bfhi(w.y);
  f[4] = bflo(w.z); f[5] = bfhi(w.z); f[6] = bflo(w.w); f[7] = bfhi(w.w);
}
__device__ __forceinline__ uint4 pack8(const float* f) {
  return uint4{f2bf2(f[0], f[1]), f2bf2(f[2], f[3]), f2bf2(f[4], f[5]), f2bf2(f[6], f[7])};
}

// ----------------------------------------------------------- convolution
// out[v][co] = sum over taps t and input channels ci of
//              wt[co][t * cin + ci] * in(v + offset(t))[ci]
// (cross-correlation with one cell of zero padding; taps = 27, tap
// t = 9 (dx + 1) + 3 (dy + 1) + (dz + 1), or taps = 1 for a pointwise map).
// The input is the channel concatenation of in0 (c0 channels) and in1 (c1
// channels, may be null with c1 = 0), both channels-last BF16.  wt is BF16
// [coutp][kp], kp = K = taps * cin rounded up to 32, zero padded.  out is
// FP32 [V][cout].  With stats set, each block also writes the sum and the
// sum of squares of its outputs per channel to stats[blockIdx.x][cout][2]
// (batch-norm statistics, reduced in a fixed order afterwards).
//
// Block: four waves, each an MFMA tile of 32 output channels x 64 voxels
// (2 x 4 tiles of 16 x 16); operands are loaded straight from global memory
// (the 27 taps re-read each input row through the caches).  Split over k
// (grids with few voxels and long k, the bottleneck): blockIdx.z takes
// k in [z kchunk, (z + 1) kchunk) and writes its partial sums to
// out + z V cout, without statistics; conv_split_reduce_kernel adds the
// splits.
struct ConvArgs {
  const uint16_t* in0;
  const uint16_t* in1;
  int32_t c0, c1;
  const uint16_t* wt;
  int32_t kp;
  float* out;
  int32_t cout;
  int32_t taps;
  int32_t B, X, Y, Z;
  float* stats;
  int32_t kchunk;  // conv_kernel: k per blockIdx.z (a multiple of 32)
};

constexpr int CV_VOX = 256;  // voxels per block (4 waves x 64)
constexpr int CV_CO = 32;    // output channels per block

__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t YZ = (int64_t)a.Y * a.Z;
  const int64_t V = (int64_t)a.B * a.X * YZ;
  const int cin = a.c0 + a.c1;
  const int K = a.taps * cin;
  const int co0 = blockIdx.y * CV_CO;
  const int64_t vb0 = (int64_t)blockIdx.x * CV_VOX + wave * 64;
  int vx[4], vy[4], vz[4];
  int64_t vv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t v = vb0 + 16 * c + (lane & 15);
    vv[c] = v < V ? v : -1;
    const int64_t w = v < V ? v : 0;
    vz[c] = (int)(w % a.Z);
    vy[c] = (int)((w / a.Z) % a.Y);
    vx[c] = (int)((w / YZ) % a.X);
  }
  f32x4 acc[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[m][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kl = 8 * (lane >> 4);
  const uint16_t* w0 = a.wt + (int64_t)(co0 + (lane & 15)) * a.kp + kl;
  const uint16_t* w1 = w0 + (int64_t)16 * a.kp;
  const int kb = blockIdx.z * a.kchunk, ke = kb + a.kchunk < a.kp ? kb + a.kchunk : a.kp;
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const int k = k0 + kl;
    bf16x8 bv[4];
    if (k < K) {
      const int t = a.taps == 1 ? 0 : k / cin;
      const int ci = k - t * cin;
      const int dx = a.taps == 1 ? 0 : t / 9 - 1, dy = a.taps == 1 ? 0 : (t / 3) % 3 - 1,
                dz = a.taps == 1 ? 0 : t % 3 - 1;
      const bool first = ci < a.c0;
      const uint16_t* src = first ? a.in0 : a.in1;
      const int cs = first ? a.c0 : a.c1;
      const int cc = first ? ci : ci - a.c0;
      const int64_t off = dx * YZ + dy * a.Z + dz;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int nx = vx[c] + dx, ny = vy[c] + dy, nz = vz[c] + dz;
        const bool ok = vv[c] >= 0 && nx >= 0 && nx < a.X && ny >= 0 && ny < a.Y && nz >= 0 && nz < a.Z;
        if (ok) {
          bv[c] = *(const bf16x8*)(src + (vv[c] + off) * cs + cc);
        } else {
          bv[c] = bf16x8{};
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = bf16x8{};
    }
    const bf16x8 a0 = *(const bf16x8*)(w0 + k0);
    const bf16x8 a1 = *(const bf16x8*)(w1 + k0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      acc[0][c] = mfma16(a0, bv[c], acc[0][c]);
      acc[1][c] = mfma16(a1, bv[c], acc[1][c]);
    }
  }
  // lane holds out[voxel vb0 + 16c + (lane & 15)][co0 + 16m + 4 (lane >> 4) + r]
  float* out = a.out + (int64_t)blockIdx.z * V * a.cout;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int cb = co0 + 16 * m + 4 * (lane >> 4);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (vv[c] < 0) continue;
      float* o = out + vv[c] * a.cout + cb;
      if (cb + 3 < a.cout) {
        *(float4*)o = float4{acc[m][c][0], acc[m][c][1], acc[m][c][2], acc[m][c][3]};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (cb + r < a.cout) o[r] = acc[m][c][r];
      }
    }
  }
  if (a.stats) {
    // per channel: sums over this block's voxels (padding voxels hold 0)
    __shared__ float red[4][CV_CO][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float s = 0.f, q = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          s += acc[m][c][r];
          q += acc[m][c][r] * acc[m][c][r];
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          s += __shfl_xor(s, o);
          q += __shfl_xor(q, o);
        }
        if ((lane & 15) == 0) {
          red[wave][16 * m + 4 * (lane >> 4) + r][0] = s;
          red[wave][16 * m + 4 * (lane >> 4) + r][1] = q;
        }
      }
    __syncthreads();
    if (threadIdx.x < 2 * CV_CO) {
      const int col = threadIdx.x >> 1, h = threadIdx.x & 1;
      const float v = red[0][col][h] + red[1][col][h] + red[2][col][h] + red[3][col][h];
      if (co0 + col < a.cout) a.stats[((int64_t)blockIdx.x * a.cout + co0 + col) * 2 + h] = v;
    }
  }
}

// Sum of the k splits of conv_kernel: out[v][c] = sum over z (in order) of
// part[z][v][c], and per-block statistics of the sums as conv_kernel writes
// them, over blocks of CSR_VOX voxels: block (blockIdx.x, blockIdx.y) covers
// voxels [CSR_VOX x, CSR_VOX (x + 1)) and channels [32 y, 32 y + 32); thread
// (column t & 31, row t >> 5) takes every eighth voxel;
// stats[blockIdx.x][c][2] (when stats is set).
constexpr int CSR_VOX = 32;

__global__ __launch_bounds__(256) void conv_split_reduce_kernel(const float* part, int ns, int64_t V, int cout,
                                                                float* out, float* stats) {
  __shared__ float red[8][32][2];
  const int col = threadIdx.x & 31, row = threadIdx.x >> 5;
  const int c = blockIdx.y * 32 + col;
  const int64_t vb = (int64_t)blockIdx.x * CSR_VOX;
  float s = 0.f, q = 0.f;
  if (c < cout)
#pragma unroll
    for (int j = row; j < CSR_VOX; j += 8) {
      const int64_t v = vb + j;
      if (v < V) {
        float acc = 0.f;
#pragma unroll 4
        for (int z = 0; z < ns; ++z) acc += part[((int64_t)z * V + v) * cout + c];
        out[v * cout + c] = acc;
        s += acc;
        q += acc * acc;
      }
    }
  if (!stats) return;
  red[row][col][0] = s;
  red[row][col][1] = q;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int cl = threadIdx.x >> 1, h = threadIdx.x & 1;
    float v = 0.f;
#pragma unroll
    for (int r = 0; r < 8; ++r) v += red[r][cl][h];
    if (blockIdx.y * 32 + cl < cout) stats[((int64_t)blockIdx.x * cout + blockIdx.y * 32 + cl) * 2 + h] = v;
  }
}

// ------------------------------------------------ convolution through LDS
// The same convolution through LDS.  A block owns a 4 x TY x TZ box of
// output voxels of one sample (TY TZ = 64: 4 x 16 on the fine levels, 8 x 8
// on the 8-cell level) and COB output channels.  Per chunk of CC input
// channels it stages the box's (4 + 2) x (TY + 2) x (TZ + 2) halo once in
// LDS and runs all 27 taps from there: each staged value feeds up to 27
// taps instead of being re-read through the caches per tap.  Wave w
// computes the voxels of x-slice w (its 64 voxels, v = 16 c + l: y = v / TZ,
// z = v % TZ, as four 16-voxel MFMA column groups) for all COB channels.
//   CC = 32: inputs in multiples of 32 channels; an MFMA k step is one tap
//            and 32 channels; LDS rows of 40 (the 16 lanes of a column
//            group read disjoint banks).
//   CC = 8:  the 8-channel input layer; a k step is four taps of 8
//            channels (lane group g takes tap 4 s + g), the weight rows'
//            k = tap * 8 + ci order; past tap 26 the weights are zero and
//            the lanes read the centre tap's (finite) values.
// Outputs, statistics and the weight operand are those of conv_kernel; the
// per-block statistics cover the block's 256 voxels (blockIdx.x enumerates
// the boxes).
constexpr int CL_TX = 4;

// (the 32-channel instances: three waves per SIMD, 168 registers)
template <int COB, int CC, int TY, int TZ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(COB == 32 && CC == 32 ? 3 : 1)))
void conv_lds_kernel(ConvArgs a) {
  constexpr int MT = COB / 16;
  constexpr int HX = CL_TX + 2, HY = TY + 2, HZ = TZ + 2, HALO = HX * HY * HZ;
  constexpr int CP = CC == 32 ? 40 : 8;  // LDS row (channels + padding)
  constexpr int Q = CC / 8;              // 16-byte groups per staged voxel
  static_assert(TY * TZ == 64 && (CC == 32 || CC == 8), "box and chunk");
  __shared__ __attribute__((aligned(16))) uint16_t halo[HALO * CP];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nbx = a.X / CL_TX, nby = a.Y / TY, nbz = a.Z / TZ;
  int64_t bi = blockIdx.x;
  const int bz = (int)(bi % nbz); bi /= nbz;
  const int by = (int)(bi % nby); bi /= nby;
  const int bx = (int)(bi % nbx);
  const int64_t b = bi / nbx;
  const int x0 = bx * CL_TX, y0 = by * TY, z0 = bz * TZ;
  const int64_t YZ = (int64_t)a.Y * a.Z;
  const int64_t sbase = b * a.X * YZ;  // first voxel of the sample
  const int cin = a.c0 + a.c1;
  const int co0 = blockIdx.y * COB;
  const int g = lane >> 4, l16 = lane & 15, kl = 8 * g;
  f32x4 acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[m][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* wrow[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) wrow[m] = a.wt + (int64_t)(co0 + 16 * m + l16) * a.kp + kl;
  // halo index of this lane's voxel in column group c at tap offsets (0, 0, 0)
  int hv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int v = 16 * c + l16;
    hv[c] = (wave * HY + v / TZ) * HZ + v % TZ;
  }
  // The halo of a channel chunk is loaded into registers (NI 16-byte
  // items per thread) while the previous chunk computes, and written to
  // LDS once that chunk's taps are done: the global loads of chunk c + 1
  // overlap the MFMA work of chunk c.
  constexpr int NI = (HALO * Q + 255) / 256;
  uint4 pre[NI];
  auto load_chunk = [&](int cb) {
    const bool first = cb < a.c0;
    const uint16_t* src = first ? a.in0 : a.in1;
    const int cs = first ? a.c0 : a.c1;
    const int cc = first ? cb : cb - a.c0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int e = t + 256 * i;
      const int q = e % Q, h = e / Q;
      const int hz = h % HZ, hy = (h / HZ) % HY, hx = h / (HZ * HY);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
      pre[i] = uint4{0u, 0u, 0u, 0u};
      if (e < HALO * Q && gx >= 0 && gx < a.X && gy >= 0 && gy < a.Y && gz >= 0 && gz < a.Z)
        pre[i] = *(const uint4*)(src + (sbase + gx * YZ + (int64_t)gy * a.Z + gz) * cs + cc + 8 * q);
    }
  };
  load_chunk(0);
  for (int cb = 0; cb < cin; cb += CC) {
    // stage the halo: HALO voxels x Q groups of 8 channels
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int e = t + 256 * i;
      if (e < HALO * Q) *(uint4*)(halo + (e / Q) * CP + 8 * (e % Q)) = pre[i];
    }
    __syncthreads();
    if (cb + CC < cin) load_chunk(cb + CC);
    if (CC == 32) {
#pragma unroll 3
      for (int tp = 0; tp < 27; ++tp) {
        const int dx = tp / 9, dy = (tp / 3) % 3, dz = tp % 3;  // offsets + 1
        const int ho = (dx * HY + dy) * HZ + dz;
        bf16x8 av[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) av[m] = *(const bf16x8*)(wrow[m] + tp * cin + cb);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 bv = *(const bf16x8*)(halo + (hv[c] + ho) * CP + kl);
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[m][c] = mfma16(av[m], bv, acc[m][c]);
        }
      }
    } else {
#pragma unroll 1
      for (int s = 0; s < 7; ++s) {
        const int tp = 4 * s + g < 27 ? 4 * s + g : 13;
        const int dx = tp / 9, dy = (tp / 3) % 3, dz = tp % 3;
        const int ho = (dx * HY + dy) * HZ + dz;
        bf16x8 av[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) av[m] = *(const bf16x8*)(wrow[m] + 32 * s);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 bv = *(const bf16x8*)(halo + (hv[c] + ho) * CP);
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[m][c] = mfma16(av[m], bv, acc[m][c]);
        }
      }
    }
    __syncthreads();
  }
  // lane holds out[voxel (x0 + wave, y0 + v / TZ, z0 + v % TZ), v = 16 c + l16][co0 + 16m + 4g + r]
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int cbase = co0 + 16 * m + 4 * g;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int v = 16 * c + l16;
      const int64_t vox = sbase + (int64_t)(x0 + wave) * YZ + (int64_t)(y0 + v / TZ) * a.Z + z0 + v % TZ;
      float* o = a.out + vox * a.cout + cbase;
      if (cbase + 3 < a.cout) {
        *(float4*)o = float4{acc[m][c][0], acc[m][c][1], acc[m][c][2], acc[m][c][3]};
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (cbase + r < a.cout) o[r] = acc[m][c][r];
      }
    }
  }
  if (a.stats) {
    __shared__ float red[4][COB][2];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float s = 0.f, q = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          s += acc[m][c][r];
          q += acc[m][c][r] * acc[m][c][r];
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          s += __shfl_xor(s, o);
          q += __shfl_xor(q, o);
        }
        if (l16 == 0) {
          red[wave][16 * m + 4 * g + r][0] = s;
          red[wave][16 * m + 4 * g + r][1] = q;
        }
      }
    __syncthreads();
    if (t < 2 * COB) {
      const int col = t >> 1, h = t & 1;
      const float v = red[0][col][h] + red[1][col][h] + red[2][col][h] + red[3][col][h];
      if (co0 + col < a.cout) a.stats[((int64_t)blockIdx.x * a.cout + co0 + col) * 2 + h] = v;
    }
  }
}

// the box of the LDS weight-gradient kernel: 4 x 4 x TZ voxels, TZ = 16 on
// the fine levels and 8 on the 8-cell level
constexpr int WL_TY = 4;
constexpr int WL_HX = CL_TX + 2, WL_HY = WL_TY + 2;

// --------------------------------------------------------- weight gradient
// part[chunk][co][k] = sum over the chunk's voxels v of
//                      dz[v][co] * in(v + offset(t))[ci],   k = t * cin + ci
// (the adjoint of conv_kernel with respect to its weights; chunks of the
// voxel range are reduced afterwards in a fixed order).  Block: a 64 x 64
// tile of (co, k), the chunk walked 64 voxels at a time; both operands are
// transposed through LDS so that an MFMA lane reads 8 consecutive voxels.
struct WgradArgs {
  const uint16_t* dz;   // [V][cout] BF16
  int32_t cout;
  const uint16_t* in0;
  const uint16_t* in1;
  int32_t c0, c1;
  int32_t taps;
  int32_t B, X, Y, Z;
  int64_t chunk;        // voxels per chunk, a multiple of 64
  float* part;          // [nchunk][cout][K]
};

constexpr int WG_T = 64;      // tile rows (co) and columns (k)
constexpr int WG_VS = 72;     // LDS row stride in elements (64 voxels + 8)

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t sd[WG_T * WG_VS];
  __shared__ __attribute__((aligned(16))) uint16_t sx[WG_T * WG_VS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
  const int64_t YZ = (int64_t)a.Y * a.Z;
  const int64_t V = (int64_t)a.B * a.X * YZ;
  const int cin = a.c0 + a.c1;
  const int K = a.taps * cin;
  const int co0 = blockIdx.x * WG_T, k0 = blockIdx.y * WG_T;
  const int64_t v0 = (int64_t)blockIdx.z * a.chunk;
  const int64_t v1 = v0 + a.chunk < V ? v0 + a.chunk : V;
  f32x4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  // loader roles: 512 vectors of 8 channels per tile, two per thread
  for (int64_t vs = v0; vs < v1; vs += 64) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = t + 256 * h;         // 0..511
      const int vl = e & 63, g = e >> 6; // voxel in the step, 8-column group
      const int64_t v = vs + vl;
      // dz tile: channels co0 + 8g .. +8 of voxel v -> sd[co][voxel]
      uint4 w = uint4{0u, 0u, 0u, 0u};
      const int cc = co0 + 8 * g;
      if (v < v1 && cc < a.cout) w = *(const uint4*)(a.dz + v * a.cout + cc);
      const uint16_t* wv = (const uint16_t*)&w;
#pragma unroll
      for (int j = 0; j < 8; ++j) sd[(8 * g + j) * WG_VS + vl] = wv[j];
      // input tile: columns k0 + 8g .. +8 (one tap, 8 channels) of voxel v
      uint4 x = uint4{0u, 0u, 0u, 0u};
      const int k = k0 + 8 * g;
      if (v < v1 && k < K) {
        const int tp = a.taps == 1 ? 0 : k / cin;
        const int ci = k - tp * cin;
        const int dx = a.taps == 1 ? 0 : tp / 9 - 1, dy = a.taps == 1 ? 0 : (tp / 3) % 3 - 1,
                  dz = a.taps == 1 ? 0 : tp % 3 - 1;
        const int z = (int)(v % a.Z), y = (int)((v / a.Z) % a.Y), xx = (int)((v / YZ) % a.X);
        const int nx = xx + dx, ny = y + dy, nz = z + dz;
        if (nx >= 0 && nx < a.X && ny >= 0 && ny < a.Y && nz >= 0 && nz < a.Z) {
          const bool first = ci < a.c0;
          const uint16_t* src = first ? a.in0 : a.in1;
          const int cs = first ? a.c0 : a.c1;
          x = *(const uint4*)(src + (v + dx * YZ + dy * a.Z + dz) * cs + (first ? ci : ci - a.c0));
        }
      }
      const uint16_t* xv = (const uint16_t*)&x;
#pragma unroll
      for (int j = 0; j < 8; ++j) sx[(8 * g + j) * WG_VS + vl] = xv[j];
    }
    __syncthreads();
    if (co0 + 16 * wave < a.cout) {  // a wave whose 16 rows are all padding skips its products
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 av = *(const bf16x8*)(sd + (16 * wave + (lane & 15)) * WG_VS + 32 * s + 8 * (lane >> 4));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 bv = *(const bf16x8*)(sx + (16 * c + (lane & 15)) * WG_VS + 32 * s + 8 * (lane >> 4));
          acc[c] = mfma16(av, bv, acc[c]);
        }
      }
    }
    __syncthreads();
  }
  float* part = a.part + (int64_t)blockIdx.z * a.cout * K;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int k = k0 + 16 * c + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = co0 + 16 * wave + 4 * (lane >> 4) + r;
      if (co < a.cout && k < K) part[(int64_t)co * K + k] = acc[c][r];
    }
  }
}

// Weight gradient through LDS, for convolutions with cout % 32 == 0 and
// input channels in multiples of 32 (CI = 32) or the 8-channel input layer
// (CI = 8), on a grid of 4 x 4 x TZ boxes (TZ = 16 or 8).  Grid (nchunk,
// cout / 32, cin / CI); three waves.  A block owns 32 output channels x CI
// input channels x all 27 taps and walks the boxes [blockIdx.x *
// per_chunk, ...).  Per box it stages the box's dz [32 co][4][4][TZ] and
// the input halo [CI][6][6][ZP] (TZ + 2 z, padded) transposed in LDS, z
// contiguous, so that an MFMA lane's k slots are 8 z-consecutive voxels (a
// 32-voxel k step is two (x, y) rows of 16 z, or four rows of 8).  The
// product's 16 columns are (tap pair (dx, dy), input channel) pairs: CI =
// 32: wave w owns the pairs w, w + 3, w + 6, each as two 16-channel column
// tiles; CI = 8: column tile j holds pairs 2j and 2j + 1 x 8 channels, and
// wave w owns the tiles w and w + 3 (of five).  Each lane forms the
// operands of the three dz shifts of its column from one aligned 16-voxel
// window of its halo row in registers (the odd shift by a 16-bit funnel
// shift), so no LDS read is misaligned.  The partials go to
// part[blockIdx.x][co][t * cin + ci], the layout wgrad_reduce_kernel sums.
struct WgradLdsArgs {
  const uint16_t* dz;   // [V][cout] BF16
  int32_t cout;
  const uint16_t* in0;
  const uint16_t* in1;
  int32_t c0, c1;
  int32_t B, X, Y, Z;
  int64_t per_chunk;    // boxes per block
  float* part;          // [nchunk][cout][27 cin]
};

template <int TZ, int CI>
__global__ __launch_bounds__(192) void wgrad_lds_kernel(WgradLdsArgs a) {
  static_assert((TZ == 16 || TZ == 8) && (CI == 32 || CI == 8), "box depth, channel tile");
  constexpr int Q = CI / 8;                 // 16-byte groups per staged voxel
  constexpr int NT = CI == 32 ? 6 : 2;      // column tiles per wave
  constexpr int HZ = TZ + 2;                // halo row
  constexpr int ZP = TZ == 16 ? 24 : 16;    // padded halo row: the 16-voxel windows stay inside
  constexpr int NS = CL_TX * WL_TY * TZ / 32;  // k steps per box
  __shared__ __attribute__((aligned(16))) uint16_t xt[CI * WL_HX * WL_HY * ZP];  // [ci][hx][hy][z]
  __shared__ __attribute__((aligned(16))) uint16_t dt[32 * CL_TX * WL_TY * TZ];  // [co][bx][by][z]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, l16 = lane & 15;
  const int cin = a.c0 + a.c1;
  const int co0 = blockIdx.y * 32, ci0 = blockIdx.z * CI;
  const bool first = ci0 < a.c0;
  const uint16_t* src = first ? a.in0 : a.in1;
  const int cs = first ? a.c0 : a.c1;
  const int cc = first ? ci0 : ci0 - a.c0;
  const int nbx = a.X / CL_TX, nby = a.Y / WL_TY, nbz = a.Z / TZ;
  const int64_t nbox = (int64_t)a.B * nbx * nby * nbz;
  const int64_t YZ = (int64_t)a.Y * a.Z;
  const int64_t bx0 = (int64_t)blockIdx.x * a.per_chunk;
  const int64_t bx1 = bx0 + a.per_chunk < nbox ? bx0 + a.per_chunk : nbox;
  f32x4 acc[NT][3][2];  // [column tile][dz][co tile]
#pragma unroll
  for (int p = 0; p < NT; ++p)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int m = 0; m < 2; ++m) acc[p][d][m] = f32x4{0.f, 0.f, 0.f, 0.f};
  // column tile tau of this wave: the lane's tap pair pr and input channel
  // ci (CI = 8: tiles past the fifth, and the second half of the fifth,
  // hold no pair: live is false there)
  auto column = [&](int tau, int& pr, int& ci, bool& live) {
    if (CI == 32) {
      pr = wave + 3 * (tau >> 1);
      ci = 16 * (tau & 1) + l16;
      live = true;
    } else {
      const int j = wave + 3 * tau;
      pr = 2 * j + (l16 >> 3);
      ci = l16 & 7;
      live = pr < 9;
      if (pr > 8) pr = 8;
    }
  };
  // The first NP of the next box's NH input-halo items per thread are
  // loaded into registers while the current box computes; the rest of the
  // halo and the box's dz are loaded when the box starts.  (Holding more
  // would take the kernel past 256 registers, to one wave per SIMD.)
  constexpr int HITEMS = WL_HX * WL_HY * (HZ / 2) * Q, DITEMS = CL_TX * WL_TY * (TZ / 2) * 4;
  constexpr int NH = (HITEMS + 191) / 192, NP = NH < 3 ? NH : 3;
  uint4 ph[NP][2];
  auto box_origin = [&](int64_t box, int& x0, int& y0, int& z0, int64_t& sbase) {
    int64_t bi = box;
    const int bz = (int)(bi % nbz); bi /= nbz;
    const int by = (int)(bi % nby); bi /= nby;
    const int bxx = (int)(bi % nbx);
    const int64_t b = bi / nbx;
    x0 = bxx * CL_TX; y0 = by * WL_TY; z0 = bz * TZ;
    sbase = b * a.X * YZ;
  };
  // halo item e of a box (origin x0, y0, z0, sample base sbase) into v0, v1
  auto halo_item = [&](int e, int x0, int y0, int z0, int64_t sbase, uint4& v0, uint4& v1) {
    const int q = e % Q, r = e / Q;
    const int hzp = r % (HZ / 2), hy = (r / (HZ / 2)) % WL_HY, hx = r / ((HZ / 2) * WL_HY);
    const int gx = x0 + hx - 1, gy = y0 + hy - 1;
    v0 = uint4{0u, 0u, 0u, 0u};
    v1 = uint4{0u, 0u, 0u, 0u};
    if (e < HITEMS && gx >= 0 && gx < a.X && gy >= 0 && gy < a.Y) {
      const int gz = z0 + 2 * hzp - 1;
      const uint16_t* row = src + (sbase + gx * YZ + (int64_t)gy * a.Z) * cs + cc + 8 * q;
      if (gz >= 0 && gz < a.Z) v0 = *(const uint4*)(row + (int64_t)gz * cs);
      if (gz + 1 >= 0 && gz + 1 < a.Z) v1 = *(const uint4*)(row + (int64_t)(gz + 1) * cs);
    }
  };
  auto prefetch = [&](int64_t box) {
    int x0, y0, z0;
    int64_t sbase;
    box_origin(box, x0, y0, z0, sbase);
#pragma unroll
    for (int i = 0; i < NP; ++i) halo_item(t + 192 * i, x0, y0, z0, sbase, ph[i][0], ph[i][1]);
  };
  // one item's 8 channels at voxels z, z + 1 -> (z, z + 1) pairs of the
  // 8 transposed rows (row stride: stride elements)
  auto put_pairs = [](uint16_t* dst, int stride, const uint4& v0, const uint4& v1) {
    const uint32_t u0[4] = {v0.x, v0.y, v0.z, v0.w}, u1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t lo = (u0[j >> 1] >> (16 * (j & 1))) & 0xffffu, hi = (u1[j >> 1] >> (16 * (j & 1))) & 0xffffu;
      *(uint32_t*)(dst + j * stride) = lo | (hi << 16);
    }
  };
  // the halo item's LDS destination: rows (8 q + j, hx, hy), z pair hzp
  auto put_halo = [&](int e, const uint4& v0, const uint4& v1) {
    const int q = e % Q, r = e / Q;
    const int hzp = r % (HZ / 2), hy = (r / (HZ / 2)) % WL_HY, hx = r / ((HZ / 2) * WL_HY);
    put_pairs(xt + (((8 * q) * WL_HX + hx) * WL_HY + hy) * ZP + 2 * hzp, WL_HX * WL_HY * ZP, v0, v1);
  };
  if (bx0 < bx1) prefetch(bx0);
  for (int64_t box = bx0; box < bx1; ++box) {
    int x0, y0, z0;
    int64_t sbase;
    box_origin(box, x0, y0, z0, sbase);
    // the rest of the halo and the dz of the box (two z-consecutive voxels
    // of 8 channels per item)
#pragma unroll
    for (int i = NP; i < NH; ++i) {
      const int e = t + 192 * i;
      uint4 v0, v1;
      halo_item(e, x0, y0, z0, sbase, v0, v1);
      if (e < HITEMS) put_halo(e, v0, v1);
    }
    for (int e = t; e < DITEMS; e += 192) {
      const int q = e & 3, r = e >> 2;
      const int zp = r % (TZ / 2), yy = (r / (TZ / 2)) % WL_TY, xx = r / ((TZ / 2) * WL_TY);
      const uint16_t* row = a.dz +
                            (sbase + (int64_t)(x0 + xx) * YZ + (int64_t)(y0 + yy) * a.Z + z0 + 2 * zp) * a.cout +
                            co0 + 8 * q;
      put_pairs(dt + (((8 * q) * CL_TX + xx) * WL_TY + yy) * TZ + 2 * zp, CL_TX * WL_TY * TZ,
                *(const uint4*)row, *(const uint4*)(row + a.cout));
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = t + 192 * i;
      if (e < HITEMS) put_halo(e, ph[i][0], ph[i][1]);
    }
    __syncthreads();
    if (box + 1 < bx1) prefetch(box + 1);
    // k steps of 32 voxels: TZ = 16: rows 2s and 2s + 1 of the 16 (x, y)
    // rows, z halves 0 and 8, lane group g takes row 2s + (g >> 1), z half
    // 8 (g & 1); TZ = 8: rows 4s .. 4s + 3, lane group g takes row 4s + g
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
      const int row = TZ == 16 ? 2 * s + (g >> 1) : 4 * s + g, zh = TZ == 16 ? 8 * (g & 1) : 0;
      const int rx = row >> 2, ry = row & 3;
      bf16x8 av[2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
        av[m] = *(const bf16x8*)(dt + (((16 * m + l16) * CL_TX + rx) * WL_TY + ry) * TZ + zh);
#pragma unroll
      for (int tau = 0; tau < NT; ++tau) {
        if (CI == 8 && wave + 3 * tau >= 5) continue;  // wave-uniform: no such tile
        int pr, ci;
        bool live;
        column(tau, pr, ci, live);
        (void)live;
        const int dx = pr / 3, dy = pr % 3;
        {
          const uint16_t* w = xt + ((ci * WL_HX + rx + dx) * WL_HY + ry + dy) * ZP + zh;
          const uint4 lo = *(const uint4*)w, hi = *(const uint4*)(w + 8);
          const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
          uint32_t s1[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) s1[i] = __builtin_amdgcn_alignbit(d[i + 1], d[i], 16);
          const uint4 b0 = uint4{d[0], d[1], d[2], d[3]}, b1 = uint4{s1[0], s1[1], s1[2], s1[3]},
                      b2 = uint4{d[1], d[2], d[3], d[4]};
          const bf16x8 bv[3] = {__builtin_bit_cast(bf16x8, b0), __builtin_bit_cast(bf16x8, b1),
                                __builtin_bit_cast(bf16x8, b2)};
#pragma unroll
          for (int dzi = 0; dzi < 3; ++dzi)
#pragma unroll
            for (int m = 0; m < 2; ++m) acc[tau][dzi][m] = mfma16(av[m], bv[dzi], acc[tau][dzi][m]);
        }
      }
    }
    __syncthreads();
  }
  // D[co][column]: co = co0 + 16m + 4g + r, the lane's column (pr, ci)
  const int64_t K = (int64_t)27 * cin;
  float* part = a.part + (int64_t)blockIdx.x * a.cout * K;
#pragma unroll
  for (int tau = 0; tau < NT; ++tau) {
    if (CI == 8 && wave + 3 * tau >= 5) continue;
    int pr, ci;
    bool live;
    column(tau, pr, ci, live);
    if (!live) continue;
    const int dx = pr / 3, dy = pr % 3;
#pragma unroll
    for (int dzi = 0; dzi < 3; ++dzi) {
      const int tap = 9 * dx + 3 * dy + dzi;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[(int64_t)(co0 + 16 * m + 4 * g + r) * K + (int64_t)tap * cin + ci0 + ci] = acc[tau][dzi][m][r];
    }
  }
}

// dW[co][ci][t] (the parameter layout) = sum over chunks of
// part[.][co][t * cinp + ci] for co < cout, ci < cin (cinp: the device
// channel count the convolution ran with; coutp: the partials' row count).
// A block sums 64 consecutive partial columns (one coalesced 256-byte row
// segment per wave and chunk); its four waves take every fourth chunk and
// the four sums are added in a fixed order.
constexpr int WR_COLS = 64;

__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* part, int nchunk, int coutp, int cout, int cin,
                                                           int cinp, int taps, float* dW) {
  __shared__ float sm[4][WR_COLS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t K = (int64_t)taps * cinp;
  const int64_t col = (int64_t)blockIdx.x * WR_COLS + lane;  // co * K + t * cinp + ci
  const int64_t ncol = (int64_t)cout * K;
  float s = 0.f;
  if (col < ncol) {
    const float* p = part + col;
    const int64_t cs = (int64_t)coutp * K;
    // chunks wave, wave + 4, ... added in that order, eight loads in flight
    int c = wave;
    for (; c + 28 < nchunk; c += 32) {
      float x[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = p[(int64_t)(c + 4 * i) * cs];
#pragma unroll
      for (int i = 0; i < 8; ++i) s += x[i];
    }
    for (; c < nchunk; c += 4) s += p[(int64_t)c * cs];
  }
  sm[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && col < ncol) {
    const int co = (int)(col / K);
    const int r = (int)(col % K);
    const int t = r / cinp, ci = r % cinp;
    if (ci < cin) dW[((int64_t)co * cin + ci) * taps + t] = (sm[0][lane] + sm[1][lane]) + (sm[2][lane] + sm[3][lane]);
  }
}

// FP64 sums of the (first, second) float pairs at p[(b * C + c) * 2] over
// b = b0, b0 + 256, ... below nblk, added in increasing b (the order of the
// plain strided loop, so the sums are that loop's to the bit), with eight
// 8-byte loads in flight at a time
__device__ __forceinline__ void strided_pair_sums(const float* p, int64_t b0, int64_t nblk, int C, int c, double& s,
                                                  double& q) {
  int64_t b = b0;
  for (; b + 7 * 256 < nblk; b += 8 * 256) {
    float2 x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = *(const float2*)(p + ((b + i * 256) * C + c) * 2);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      s += (double)x[i].x;
      q += (double)x[i].y;
    }
  }
  for (; b < nblk; b += 256) {
    const float2 x = *(const float2*)(p + (b * C + c) * 2);
    s += (double)x.x;
    q += (double)x.y;
  }
}

// --------------------------------------------------------- batch norm
// Per channel c: mean and biased variance of the block's conv outputs over
// n voxels from the per-block partial sums (FP64 reduction in a fixed
// order); scale = gamma / sqrt(var + eps), shift = beta - mean * scale;
// running mean/var move 10% of the way (unbiased variance).  One block per
// channel.  With train = 0 the scale and shift come from the running
// statistics instead.
__global__ __launch_bounds__(256) void bn_finalize_kernel(const float* stats, int64_t nblk, int C, double n,
                                                          const float* gamma, const float* beta, float* rmean,
                                                          float* rvar, float* mean_out, float* istd_out,
                                                          float* scale, float* shift, int train) {
  const int c = blockIdx.x;
  __shared__ double rs[256], rq[256];
  double s = 0.0, q = 0.0;
  if (train) strided_pair_sums(stats, threadIdx.x, nblk, C, c, s, q);
  rs[threadIdx.x] = s;
  rq[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rq[threadIdx.x] += rq[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double mean, var;
    if (train) {
      mean = rs[0] / n;
      var = rq[0] / n - mean * mean;
      if (var < 0.0) var = 0.0;
      rmean[c] = (float)(0.9 * (double)rmean[c] + 0.1 * mean);
      rvar[c] = (float)(0.9 * (double)rvar[c] + 0.1 * var * n / (n - 1.0));
    } else {
      mean = rmean[c];
      var = rvar[c];
    }
    const double is = 1.0 / sqrt(var + 1e-5);
    mean_out[c] = (float)mean;
    istd_out[c] = (float)is;
    scale[c] = (float)(gamma[c] * is);
    shift[c] = (float)(beta[c] - mean * gamma[c] * is);
  }
}

// a[v][c] = BF16(max(z[v][c] * scale[c] + shift[c], 0)), eight channels per thread
__global__ __launch_bounds__(256) void bn_relu_kernel(const float* z, int64_t V, int C, const float* scale,
                                                      const float* shift, uint16_t* act) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int g = C / 8;
  if (e >= V * g) return;
  const int c0 = (int)(e % g) * 8;
  const float4 p = *(const float4*)(z + e * 8), q = *(const float4*)(z + e * 8 + 4);
  const float v[8] = {p.x, p.y, p.z, p.w, q.x, q.y, q.z, q.w};
  float o[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = fmaxf(v[j] * scale[c0 + j] + shift[c0 + j], 0.f);
  *(uint4*)(act + e * 8) = pack8(o);
}

// Adjoint of batch norm and ReLU, pass 1: per block and channel, the sums
// of dy and dy * xhat over the block's voxels, with dy = g where the
// activation is positive and xhat = (z - mean) * istd.  Block: 256 voxels x
// all channels, thread (voxel lane, channel group) -> partial[blk][C][2].
__global__ __launch_bounds__(256) void bn_bwd_reduce_kernel(const float* g, const float* z, int64_t V, int C,
                                                            const float* scale, const float* shift,
                                                            const float* mean, const float* istd, float* partial) {
  extern __shared__ float sm[];  // [threads][8][2]
  const int groups = C / 8;
  const int per = 256 / groups;  // voxels handled in parallel (groups divides 256)
  const int gi = threadIdx.x % groups, vi = threadIdx.x / groups;
  const int c0 = gi * 8;
  float s[8], q[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) { s[j] = 0.f; q[j] = 0.f; }
  const int64_t vb = (int64_t)blockIdx.x * 256;
  for (int64_t v = vb + vi; v < vb + 256 && v < V; v += per) {
    const float4 za = *(const float4*)(z + v * C + c0), zb = *(const float4*)(z + v * C + c0 + 4);
    const float4 ga = *(const float4*)(g + v * C + c0), gb = *(const float4*)(g + v * C + c0 + 4);
    const float zz[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
    const float gg[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float y = zz[j] * scale[c0 + j] + shift[c0 + j];
      const float dy = y > 0.f ? gg[j] : 0.f;
      s[j] += dy;
      q[j] += dy * (zz[j] - mean[c0 + j]) * istd[c0 + j];
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    sm[(threadIdx.x * 8 + j) * 2] = s[j];
    sm[(threadIdx.x * 8 + j) * 2 + 1] = q[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < C * 2; e += 256) {
    const int c = e >> 1, h = e & 1, gg = c / 8, j = c % 8;
    float acc = 0.f;
    for (int p = 0; p < per; ++p) acc += sm[((p * groups + gg) * 8 + j) * 2 + h];
    partial[((int64_t)blockIdx.x * C + c) * 2 + h] = acc;
  }
}

// pass 2 coefficients per channel: dbeta = sum dy, dgamma = sum dy * xhat
// (FP64 reduction of the partials in a fixed order), written to the
// gradient vector; k1 = gamma * istd, k2 = dbeta / n, k3 = dgamma / n.
__global__ __launch_bounds__(256) void bn_bwd_finalize_kernel(const float* partial, int64_t nblk, int C, double n,
                                                              const float* gamma, const float* istd, float* dgamma,
                                                              float* dbeta, float* coef) {
  const int c = blockIdx.x;
  __shared__ double rs[256], rq[256];
  double s = 0.0, q = 0.0;
  strided_pair_sums(partial, threadIdx.x, nblk, C, c, s, q);
  rs[threadIdx.x] = s;
  rq[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rq[threadIdx.x] += rq[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dbeta[c] = (float)rs[0];
    dgamma[c] = (float)rq[0];
    coef[3 * c] = gamma[c] * istd[c];
    coef[3 * c + 1] = (float)(rs[0] / n);
    coef[3 * c + 2] = (float)(rq[0] / n);
  }
}

// pass 2: dz = k1 (dy - k2 - xhat k3), stored BF16 (the operand of both
// adjoint convolutions), eight channels per thread
__global__ __launch_bounds__(256) void bn_bwd_apply_kernel(const float* g, const float* z, int64_t V, int C,
                                                           const float* scale, const float* shift, const float* mean,
                                                           const float* istd, const float* coef, uint16_t* dz) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= V * (C / 8)) return;
  const int c0 = (int)(e % (C / 8)) * 8;
  const float4 za = *(const float4*)(z + e * 8), zb = *(const float4*)(z + e * 8 + 4);
  const float4 ga = *(const float4*)(g + e * 8), gb = *(const float4*)(g + e * 8 + 4);
  const float zz[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
  const float gg[8] = {ga.x, ga.y, ga.z, ga.w, gb.x, gb.y, gb.z, gb.w};
  float o[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = c0 + j;
    const float y = zz[j] * scale[c] + shift[c];
    const float dy = y > 0.f ? gg[j] : 0.f;
    const float xh = (zz[j] - mean[c]) * istd[c];
    o[j] = coef[3 * c] * (dy - coef[3 * c + 1] - xh * coef[3 * c + 2]);
  }
  *(uint4*)(dz + e * 8) = pack8(o);
}

// ------------------------------------------------------ pooling, upsampling
// 2x2x2 max pooling, channels-last BF16, eight channels per thread
__global__ __launch_bounds__(256) void maxpool_kernel(const uint16_t* in, int B, int X, int Y, int Z, int C,
                                                      uint16_t* out) {
  const int Xo = X / 2, Yo = Y / 2, Zo = Z / 2, g = C / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)B * Xo * Yo * Zo * g;
  if (e >= n) return;
  const int c0 = (int)(e % g) * 8;
  int64_t r = e / g;
  const int zo = (int)(r % Zo); r /= Zo;
  const int yo = (int)(r % Yo); r /= Yo;
  const int xo = (int)(r % Xo);
  const int b = (int)(r / Xo);
  float m[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) m[j] = -INFINITY;
  for (int d = 0; d < 8; ++d) {
    const int x = 2 * xo + (d >> 2), y = 2 * yo + ((d >> 1) & 1), z = 2 * zo + (d & 1);
    float f[8];
    unpack8(*(const uint4*)(in + ((((int64_t)b * X + x) * Y + y) * Z + z) * C + c0), f);
#pragma unroll
    for (int j = 0; j < 8; ++j) m[j] = fmaxf(m[j], f[j]);
  }
  *(uint4*)(out + e * 8) = pack8(m);
}

// Adjoint of max pooling plus a second gradient of the pooled tensor's
// input: gin[v] = (v is the first maximum of its window, scanned x, y, z
// with z fastest ? gout[window] : 0) + gadd[v], FP32.  gadd has row stride
// sadd and channel offset oadd (the skip part of a concatenation's
// gradient), or is null.
__global__ __launch_bounds__(256) void maxpool_bwd_kernel(const uint16_t* in, const float* gout, int B, int X, int Y,
                                                          int Z, int C, const float* gadd, int sadd, int oadd,
                                                          float* gin) {
  const int Xo = X / 2, Yo = Y / 2, Zo = Z / 2, g = C / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)B * Xo * Yo * Zo * g;
  if (e >= n) return;
  const int c0 = (int)(e % g) * 8;
  int64_t r = e / g;
  const int zo = (int)(r % Zo); r /= Zo;
  const int yo = (int)(r % Yo); r /= Yo;
  const int xo = (int)(r % Xo);
  const int b = (int)(r / Xo);
  float m[8];
  int arg[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) { m[j] = -INFINITY; arg[j] = 0; }
  int64_t vox[8];
  for (int d = 0; d < 8; ++d) {
    const int x = 2 * xo + (d >> 2), y = 2 * yo + ((d >> 1) & 1), z = 2 * zo + (d & 1);
    vox[d] = (((int64_t)b * X + x) * Y + y) * Z + z;
    float f[8];
    unpack8(*(const uint4*)(in + vox[d] * C + c0), f);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (f[j] > m[j]) { m[j] = f[j]; arg[j] = d; }
  }
  const float* go = gout + e * 8;
  for (int d = 0; d < 8; ++d) {
    float o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = arg[j] == d ? go[j] : 0.f;
    if (gadd) {
      const float* ga = gadd + vox[d] * sadd + oadd + c0;
#pragma unroll
      for (int j = 0; j < 8; ++j) o[j] += ga[j];
    }
    float* gi = gin + vox[d] * C + c0;
    *(float4*)gi = float4{o[0], o[1], o[2], o[3]};
    *(float4*)(gi + 4) = float4{o[4], o[5], o[6], o[7]};
  }
}

// one axis of the half-pixel linear upsampling: output index o reads inputs
// i0 (weight 3/4) and i1 (1/4), clamped at the faces
__device__ __forceinline__ void up_taps(int o, int n, int& i0, int& i1) {
  i0 = o >> 1;
  i1 = (o & 1) ? (i0 + 1 < n ? i0 + 1 : n - 1) : (i0 > 0 ? i0 - 1 : 0);
}

// trilinear upsampling by 2 (half-pixel centres), channels-last BF16 in
// [B][X][Y][Z][C] -> out [B][2X][2Y][2Z][C]
__global__ __launch_bounds__(256) void upsample_kernel(const uint16_t* in, int B, int X, int Y, int Z, int C,
                                                       uint16_t* out) {
  const int Xo = 2 * X, Yo = 2 * Y, Zo = 2 * Z, g = C / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)B * Xo * Yo * Zo * g;
  if (e >= n) return;
  const int c0 = (int)(e % g) * 8;
  int64_t r = e / g;
  const int zo = (int)(r % Zo); r /= Zo;
  const int yo = (int)(r % Yo); r /= Yo;
  const int xo = (int)(r % Xo);
  const int b = (int)(r / Xo);
  int xi[2], yi[2], zi[2];
  up_taps(xo, X, xi[0], xi[1]);
  up_taps(yo, Y, yi[0], yi[1]);
  up_taps(zo, Z, zi[0], zi[1]);
  const float w[2] = {0.75f, 0.25f};
  float o[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float f[8];
        unpack8(*(const uint4*)(in + ((((int64_t)b * X + xi[a]) * Y + yi[bb]) * Z + zi[c]) * C + c0), f);
        const float wt = w[a] * w[bb] * w[c];
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] += wt * f[j];
      }
  *(uint4*)(out + e * 8) = pack8(o);
}

// The same upsampling with each thread on a 2 x 2 block of outputs in
// (y, z) for one x and 8 channels: the block draws on a 2 x 3 x 3 input
// neighbourhood (18 loads for 4 outputs instead of 32), loaded once; each
// output then sums its eight terms in upsample_kernel's order, so the
// results are the same to the bit.  Grid: (z pair and channel group,
// y pair, (b, xo)); the host checks B * 2X and Y against the grid limits.
__global__ __launch_bounds__(256) void upsample_block_kernel(const uint16_t* in, int B, int X, int Y, int Z, int C,
                                                             uint16_t* out) {
  const int Xo = 2 * X, Yo = 2 * Y, Zo = 2 * Z, g = C / 8;
  const int zg = blockIdx.x * 256 + threadIdx.x;
  if (zg >= Z * g) return;
  const int zi = zg / g, c0 = (zg - zi * g) * 8;
  const int yi = blockIdx.y, bx = blockIdx.z;
  const int b = bx / Xo, xo = bx - b * Xo;
  int xt[2];
  up_taps(xo, X, xt[0], xt[1]);
  // neighbourhood rows: index 0 the lower neighbour, 1 the centre, 2 the
  // upper neighbour (clamped at the faces as up_taps does)
  const int ys[3] = {yi > 0 ? yi - 1 : 0, yi, yi + 1 < Y ? yi + 1 : Y - 1};
  const int zs[3] = {zi > 0 ? zi - 1 : 0, zi, zi + 1 < Z ? zi + 1 : Z - 1};
  uint4 v[2][3][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        v[a][p][q] = *(const uint4*)(in + ((((int64_t)b * X + xt[a]) * Y + ys[p]) * Z + zs[q]) * C + c0);
  const float w[2] = {0.75f, 0.25f};
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      // taps of up_taps: the centre first, then the neighbour on this side
      const int ty[2] = {1, dy ? 2 : 0}, tz[2] = {1, dz ? 2 : 0};
      float o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) o[j] = 0.f;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            float f[8];
            unpack8(v[a][ty[bb]][tz[c]], f);
            const float wt = w[a] * w[bb] * w[c];
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] += wt * f[j];
          }
      const int yo = 2 * yi + dy, zo = 2 * zi + dz;
      *(uint4*)(out + (((int64_t)bx * Yo + yo) * Zo + zo) * C + c0) = pack8(o);
    }
}

// Adjoint weight of one axis: what output 2 i0 - 1 + j (j = 0..5, the
// window of the input pair i0, i0 + 1) contributes to input x = i0 + i of
// n.  The input x receives from the outputs 2x and 2x + 1 (3/4 each), 2x - 1
// and 2x + 2 (1/4 each, where they exist) and at a face from the clamped
// output (1/4 more): the adjoint of up_taps.
__device__ __forceinline__ float up_adj_w(int j, int i, int x, int n) {
  if (x >= n) return 0.f;
  float w = 0.f;
  if (j == 2 * i + 1) w += x == 0 ? 1.f : 0.75f;
  if (j == 2 * i + 2) w += x == n - 1 ? 1.f : 0.75f;
  if (j == 2 * i && x > 0) w += 0.25f;
  if (j == 2 * i + 3 && x < n - 1) w += 0.25f;
  return w;
}

// Adjoint of upsample_kernel: gin [B][X][Y][Z][C] (FP32) from gout
// [B][2X][2Y][2Z][*] read with row stride sout from channel 0 (the upsampled
// part of a concatenation's gradient).  A thread takes 2 x 2 x 2 inputs
// (x0 = 2 xp, ...) and 8 channels: it reads the 6 x 6 x 6 outputs they draw
// on once (instead of 4 x 4 x 4 per input), contracting z into two partial
// sums per (x, y) output row and those into the eight inputs.
__global__ __launch_bounds__(256) void upsample_bwd_kernel(const float* gout, int sout, int B, int X, int Y, int Z,
                                                           int C, float* gin) {
  const int g = C / 8;
  const int Xp = (X + 1) / 2, Yp = (Y + 1) / 2, Zp = (Z + 1) / 2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)B * Xp * Yp * Zp * g;
  if (e >= n) return;
  const int c0 = (int)(e % g) * 8;
  int64_t r = e / g;
  const int z0 = 2 * (int)(r % Zp); r /= Zp;
  const int y0 = 2 * (int)(r % Yp); r /= Yp;
  const int x0 = 2 * (int)(r % Xp);
  const int b = (int)(r / Xp);
  const int Xo = 2 * X, Yo = 2 * Y, Zo = 2 * Z;
  float acc[2][2][2][8];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[i][j][k][c] = 0.f;
#pragma unroll 1
  for (int jx = 0; jx < 6; ++jx) {
    const int ox = 2 * x0 - 1 + jx;
    if (ox < 0 || ox >= Xo) continue;
    const float wx[2] = {up_adj_w(jx, 0, x0, X), up_adj_w(jx, 1, x0 + 1, X)};
#pragma unroll
    for (int jy = 0; jy < 6; ++jy) {
      const int oy = 2 * y0 - 1 + jy;
      if (oy < 0 || oy >= Yo) continue;
      const float wy[2] = {up_adj_w(jy, 0, y0, Y), up_adj_w(jy, 1, y0 + 1, Y)};
      const float* row = gout + (((int64_t)b * Xo + ox) * Yo + oy) * Zo * sout + c0;
      float tz[2][8];
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 8; ++c) tz[k][c] = 0.f;
#pragma unroll
      for (int jz = 0; jz < 6; ++jz) {
        const int oz = 2 * z0 - 1 + jz;
        if (oz < 0 || oz >= Zo) continue;
        const float4 p = *(const float4*)(row + (int64_t)oz * sout), q = *(const float4*)(row + (int64_t)oz * sout + 4);
        const float gv[8] = {p.x, p.y, p.z, p.w, q.x, q.y, q.z, q.w};
        const float w0 = up_adj_w(jz, 0, z0, Z), w1 = up_adj_w(jz, 1, z0 + 1, Z);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          tz[0][c] += w0 * gv[c];
          tz[1][c] += w1 * gv[c];
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float w = wx[i] * wy[j];
#pragma unroll
          for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[i][j][k][c] += w * tz[k][c];
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (x0 + i >= X || y0 + j >= Y || z0 + k >= Z) continue;
        float* gi = gin + ((((int64_t)b * X + x0 + i) * Y + y0 + j) * Z + z0 + k) * C + c0;
        *(float4*)gi = float4{acc[i][j][k][0], acc[i][j][k][1], acc[i][j][k][2], acc[i][j][k][3]};
        *(float4*)(gi + 4) = float4{acc[i][j][k][4], acc[i][j][k][5], acc[i][j][k][6], acc[i][j][k][7]};
      }
}

// ------------------------------------------------------------------- I/O
// network input [B][cin][X][Y][Z] BF16 -> channels-last [V][8] BF16, zero
// padded beyond cin
__global__ __launch_bounds__(256) void input_kernel(const uint16_t* x, int64_t P, int B, int cin, uint16_t* out) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= (int64_t)B * P) return;
  const int64_t b = v / P, p = v % P;
  uint16_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c < cin; ++c) w[c] = x[(b * cin + c) * P + p];
  *(uint4*)(out + v * 8) = uint4{w[0] | ((uint32_t)w[1] << 16), w[2] | ((uint32_t)w[3] << 16),
                                 w[4] | ((uint32_t)w[5] << 16), w[6] | ((uint32_t)w[7] << 16)};
}

// head: y[b][o][p] = sigmoid(sum_c W[o][c] a[v][c] + bias[o]), FP32
// channels-first output, W FP32 [cout][C] (C % 8 == 0, cout <= 8).  CO:
// cout fixed at compile time (the loops over outputs unrolled, the sums in
// registers), or 0 for any cout.
template <int CO>
__global__ __launch_bounds__(256) void head_kernel(const uint16_t* act, int64_t P, int B, int C, const float* W,
                                                   const float* bias, int cout, float* y) {
  const int co = CO ? CO : cout;
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= (int64_t)B * P) return;
  float s[8];
#pragma unroll
  for (int o = 0; o < co; ++o) s[o] = bias[o];
  for (int c0 = 0; c0 < C; c0 += 8) {
    float f[8];
    unpack8(*(const uint4*)(act + v * C + c0), f);
#pragma unroll
    for (int o = 0; o < co; ++o)
#pragma unroll
      for (int j = 0; j < 8; ++j) s[o] += W[o * C + c0 + j] * f[j];
  }
  const int64_t b = v / P, p = v % P;
#pragma unroll
  for (int o = 0; o < co; ++o) y[(b * co + o) * P + p] = 1.f / (1.f + expf(-s[o]));
}

// number of nonzero mask cells (one block; integer counts, so the result
// does not depend on the order) to out[0], times mul (samples x channels:
// the loss denominator) to out[2].  A 16-byte aligned mask is read sixteen
// cells per load.
__global__ __launch_bounds__(1024) void mask_count_kernel(const uint8_t* mask, int64_t P, double mul, double* out) {
  __shared__ unsigned long long r[1024];
  unsigned long long s = 0;
  int64_t done = 0;
  if (((uintptr_t)mask & 15) == 0) {
    const int64_t n16 = P / 16;
    const uint4* m4 = (const uint4*)mask;
#pragma unroll 4
    for (int64_t i = threadIdx.x; i < n16; i += 1024) {
      const uint4 v = m4[i];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) s += ((w[k] >> (8 * j)) & 0xffu) != 0u;
    }
    done = n16 * 16;
  }
  for (int64_t p = done + threadIdx.x; p < P; p += 1024) s += mask[p] != 0;
  r[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (double)r[0];
    out[2] = (double)r[0] * mul;
  }
}

// Loss and head adjoint: with cnt = B * cout * (mask cells), per voxel
// dlogit[o] = 2 (y - t) mask / cnt * y (1 - y), stored BF16 in dlog[v][8]
// (zero beyond cout; the operand of the head's weight gradient);
// gact[v][c] = sum_o W[o][c] dlogit[o] (FP32); per block partials of the
// loss numerator and of the bias gradient: part[blk][0], part[blk][1 + o].
template <int CO>  // as for head_kernel
__global__ __launch_bounds__(256) void head_bwd_kernel(const uint16_t* act, const float* y, const float* t,
                                                       const uint8_t* mask, const double* cnt, int64_t P, int B, int C,
                                                       const float* W, int cout_rt, float* gact, uint16_t* dlog,
                                                       float* part) {
  const int cout = CO ? CO : cout_rt;
  __shared__ float sm[256][9];
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int i = 0; i < 9; ++i) sm[threadIdx.x][i] = 0.f;
  if (v < (int64_t)B * P) {
    const int64_t b = v / P, p = v % P;
    const float inv = cnt[0] > 0.0 ? (float)(2.0 / cnt[0]) : 0.f;
    const bool in = mask[p] != 0;
    float dl[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float loss = 0.f;
#pragma unroll
    for (int o = 0; o < cout; ++o) {
      const float yy = y[(b * cout + o) * P + p];
      const float d = in ? yy - t[(b * cout + o) * P + p] : 0.f;
      loss += d * d;
      dl[o] = d * inv * yy * (1.f - yy);
      sm[threadIdx.x][1 + o] = dl[o];
    }
    sm[threadIdx.x][0] = loss;
    *(uint4*)(dlog + v * 8) = pack8(dl);
    for (int c0 = 0; c0 < C; c0 += 8) {
      float g[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) g[j] = 0.f;
#pragma unroll
      for (int o = 0; o < cout; ++o)
#pragma unroll
        for (int j = 0; j < 8; ++j) g[j] += W[o * C + c0 + j] * dl[o];
      float* gp = gact + v * C + c0;
      *(float4*)gp = float4{g[0], g[1], g[2], g[3]};
      *(float4*)(gp + 4) = float4{g[4], g[5], g[6], g[7]};
    }
  }
  __syncthreads();
  if (threadIdx.x < 1 + cout) {
    float s = 0.f;
    for (int k = 0; k < 256; ++k) s += sm[k][threadIdx.x];
    part[(int64_t)blockIdx.x * 9 + threadIdx.x] = s;
  }
}

// The same adjoint with G = C / 8 threads per voxel (256 voxels per block
// of 256 G threads), thread cg of a voxel forming channels 8 cg .. 8 cg + 7
// of gact: a wave's stores cover whole contiguous rows instead of one
// 16-byte piece per 128-byte row.  Every value and partial is formed as in
// head_bwd_kernel (the partials over the same 256 voxels, in the same order).
template <int CO, int G>
__global__ __launch_bounds__(256 * G) void head_bwd_grouped_kernel(const uint16_t* act, const float* y, const float* t,
                                                                   const uint8_t* mask, const double* cnt, int64_t P,
                                                                   int B, const float* W, float* gact, uint16_t* dlog,
                                                                   float* part) {
  constexpr int C = 8 * G;
  __shared__ float sm[256][9];
  const int vl = threadIdx.x / G, cg = threadIdx.x % G;
  const int64_t v = (int64_t)blockIdx.x * 256 + vl;
  if (cg == 0)
    for (int i = 0; i < 9; ++i) sm[vl][i] = 0.f;
  if (v < (int64_t)B * P) {
    const int64_t b = v / P, p = v % P;
    const float inv = cnt[0] > 0.0 ? (float)(2.0 / cnt[0]) : 0.f;
    const bool in = mask[p] != 0;
    float dl[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float loss = 0.f;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
      const float yy = y[(b * CO + o) * P + p];
      const float d = in ? yy - t[(b * CO + o) * P + p] : 0.f;
      loss += d * d;
      dl[o] = d * inv * yy * (1.f - yy);
    }
    if (cg == 0) {
#pragma unroll
      for (int o = 0; o < CO; ++o) sm[vl][1 + o] = dl[o];
      sm[vl][0] = loss;
      *(uint4*)(dlog + v * 8) = pack8(dl);
    }
    const int c0 = 8 * cg;
    float g[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = 0.f;
#pragma unroll
    for (int o = 0; o < CO; ++o)
#pragma unroll
      for (int j = 0; j < 8; ++j) g[j] += W[o * C + c0 + j] * dl[o];
    float* gp = gact + v * C + c0;
    *(float4*)gp = float4{g[0], g[1], g[2], g[3]};
    *(float4*)(gp + 4) = float4{g[4], g[5], g[6], g[7]};
  }
  __syncthreads();
  if (threadIdx.x < 1 + CO) {
    float s = 0.f;
    for (int k = 0; k < 256; ++k) s += sm[k][threadIdx.x];
    part[(int64_t)blockIdx.x * 9 + threadIdx.x] = s;
  }
}

// sums of the head partials over blocks in a fixed order: the loss (divided
// by cnt) and the bias gradient; one block per entry (entry 0 the loss)
__global__ __launch_bounds__(256) void head_reduce_kernel(const float* part, int64_t nblk, const double* cnt,
                                                          double* loss, float* dbias) {
  const int i = blockIdx.x;
  __shared__ double r[256];
  double s = 0.0;
  int64_t b = threadIdx.x;
  for (; b + 7 * 256 < nblk; b += 8 * 256) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = part[(b + k * 256) * 9 + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += (double)x[k];
  }
  for (; b < nblk; b += 256) s += (double)part[b * 9 + i];
  r[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (i == 0) loss[0] = cnt[0] > 0.0 ? r[0] / cnt[0] : 0.0;
    else dbias[i - 1] = (float)r[0];
  }
}

// ---------------------------------------------------------- parameters
// forward operand: wt[co][t * cinp + ci] = BF16(W[co][ci][t]) for co < cout,
// ci < cin, zero elsewhere ([coutp][kp])
__global__ __launch_bounds__(256) void pack_fwd_kernel(const float* W, int cout, int cin, int cinp, int taps,
                                                       int coutp, int kp, uint16_t* wt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)coutp * kp) return;
  const int co = (int)(e / kp), k = (int)(e % kp);
  const int t = k / cinp, ci = k % cinp;
  float v = 0.f;
  if (co < cout && t < taps && ci < cin) v = W[((int64_t)co * cin + ci) * taps + t];
  wt[e] = f2bf(v);
}

// adjoint operand (flipped taps, roles of the channels exchanged):
// wb[ci][t * cout + co] = BF16(W[co][ci][taps - 1 - t]) for ci < cin; rows
// up to cinp_out, zero elsewhere ([rows][kp])
__global__ __launch_bounds__(256) void pack_bwd_kernel(const float* W, int cout, int cin, int taps, int rows, int kp,
                                                       uint16_t* wb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * kp) return;
  const int ci = (int)(e / kp), k = (int)(e % kp);
  const int t = k / cout, co = k % cout;
  float v = 0.f;
  if (ci < cin && t < taps) v = W[((int64_t)co * cin + ci) * taps + (taps - 1 - t)];
  wb[e] = f2bf(v);
}

__global__ __launch_bounds__(256) void adam_kernel(float* theta, const float* g, float* m, float* v, int64_t n,
                                                   float lr, float b1, float b2, float c1, float c2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace munet
