// gfx950 kernels of the factorized FNO's spectral convolution (paper Table 2
// and App. A.2, per-axis layers after Tran et al.): per-mode complex channel
// mixing on the modes of one axis, its weight gradient, and the packing of
// the complex weights into the real embedding the MFMA contracts with.  The
// truncated 1D DFTs along each axis and their inverses are contractions of
// the generic kernel in fno_kernels.h.
//
// Modes of axis d are stored BF16 [B][W][OUT][2][M][IN]: the axis replaced by
// (part, k), part 0 the real and 1 the imaginary part, OUT the extent of the
// axes before d and IN of those after it (z: OUT = X Y, IN = 1; y: OUT = X,
// IN = Z; x: OUT = 1, IN = Y Z).  A row is one line along the axis,
// r = o_ * IN + i_ within a sample.  As a real contraction the mixing maps
// kk = 2 c + part to n = 2 o + part' with the embedding
//   E[k][2o][2c] = E[k][2o+1][2c+1] = Wr[k][c][o],
//   E[k][2o][2c+1] = -Wi[k][c][o],  E[k][2o+1][2c] = Wi[k][c][o];
// its transpose is the adjoint (the conjugate-transposed mixing).
#pragma once
#include "fno_kernels.h"

namespace mfno {

struct AxisMixArgs {
  const uint16_t* in;  // [B][W][OUT][2][M][IN]
  uint16_t* out;       // same layout
  const uint16_t* e;   // [M][2W][2W] embedded weights, row n, column kk
  int OUT, IN, M;
  int64_t tiles;       // B * OUT * IN / AX_TR
};

constexpr int AX_TR = 16;        // rows per mixing tile
constexpr int AX_GR = 32;        // rows per weight-gradient step (one MFMA k)
constexpr int FFNO_NCHUNK = 64;  // most blocks (row chunks) of the weight gradient

// Y[row][n] = sum_kk E[k][n][kk] V[row][kk] for every mode k of a tile of 16
// rows.  IN == 1 or IN % 16 == 0; M in {4, 8, 16}.  Dynamic LDS:
// M * (16 * (2W + 8) + 8) BF16 for the input tile, reused for the output
// tile.
// (at least four waves per SIMD: the register budget the 37 KB tile of
// W = 32 leaves room for)
template <int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void axis_mix_kernel(AxisMixArgs a) {
  // KM: the stride of one mode's tile, padded by 16 bytes so that the
  // lanes of a staging store, which differ in the mode, hit different banks
  constexpr int KK = 2 * W, KP = KK + 8, NT = KK / 16, KS = KK / 32, KM = AX_TR * KP + 8;
  extern __shared__ __attribute__((aligned(16))) uint16_t ax_lds[];
  const int M = a.M, OUT = a.OUT, IN = a.IN, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint16_t* tin = ax_lds;   // [M][16][KP] (mode stride KM): rows of kk = 2 c + part
  uint16_t* tout = ax_lds;  // after the MFMAs: [c][part][k][16], ((c * 2 + part) * M + k) * 16 + r
  const int64_t rows = (int64_t)OUT * IN;
  const int64_t tile = blockIdx.x;
  const int64_t b = tile * AX_TR / rows, r0 = tile * AX_TR - b * rows;
  const int64_t line = (int64_t)2 * M * IN;  // one (b, c, o_) block
  // global index of (c, part*M + k, row) within the tile, and its LDS form
  if (IN == 1) {
    // per (c, row): 2M contiguous values, 8 per load
    const int per_row = 2 * M / 8;
    for (int e = t; e < W * AX_TR * per_row; e += 256) {
      const int c = e / (AX_TR * per_row), rem = e - c * AX_TR * per_row;
      const int r = rem / per_row, q = rem - r * per_row;
      const uint4 v = *(const uint4*)(a.in + ((b * W + c) * OUT + r0 + r) * line + 8 * q);
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int pk = 8 * q + j, part = pk >= M, k = pk - part * M;
        tin[k * KM + r * KP + 2 * c + part] = (uint16_t)(u[j >> 1] >> (16 * (j & 1)));
      }
    }
  } else {
    // per (c, part, k): 16 consecutive rows, two loads
    const int64_t o_ = r0 / IN, i0 = r0 - o_ * IN;
    for (int e = t; e < W * 2 * M * 2; e += 256) {
      const int h = e & 1, pk = (e >> 1) % (2 * M), c = (e >> 1) / (2 * M);
      const int part = pk >= M, k = pk - part * M;
      const uint4 v = *(const uint4*)(a.in + ((b * W + c) * OUT + o_) * line + (int64_t)pk * IN + i0 + 8 * h);
      const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 8; ++j)
        tin[k * KM + (8 * h + j) * KP + 2 * c + part] = (uint16_t)(u[j >> 1] >> (16 * (j & 1)));
    }
  }
  __syncthreads();
  const int akk = 8 * (lane >> 4), nk = M / 4;
  f32x4 acc[4][NT];  // modes wave, wave + 4, ... (at most four per wave)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i >= nk) break;
    const int k = wave + 4 * i;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const bf16x8 bv = *(const bf16x8*)(tin + k * KM + (lane & 15) * KP + ks * 32 + akk);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8 av = *(const bf16x8*)(a.e + ((int64_t)k * KK + nt * 16 + (lane & 15)) * KK + ks * 32 + akk);
        acc[i][nt] = mfma16(av, bv, acc[i][nt]);
      }
    }
  }
  __syncthreads();  // every wave has read the input tile
  // D[n][r]: n = nt * 16 + 4 (lane >> 4) + j = 2 o + part', r = lane & 15
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i >= nk) break;
    const int k = wave + 4 * i;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = nt * 16 + 4 * (lane >> 4) + j;
        tout[(((n >> 1) * 2 + (n & 1)) * M + k) * AX_TR + (lane & 15)] = f2bf(acc[i][nt][j]);
      }
  }
  __syncthreads();
  // pk = part * M + k, so ((c * 2) * M + pk) * 16 + r addresses [c][part][k][r]
  if (IN == 1) {
    const int per_row = 2 * M / 8;
    for (int e = t; e < W * AX_TR * per_row; e += 256) {
      const int c = e / (AX_TR * per_row), rem = e - c * AX_TR * per_row;
      const int r = rem / per_row, q = rem - r * per_row;
      uint32_t u[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int pk0 = 8 * q + 2 * j, pk1 = pk0 + 1;
        const uint32_t lo = tout[((c * 2) * M + pk0) * AX_TR + r];
        const uint32_t hi = tout[((c * 2) * M + pk1) * AX_TR + r];
        u[j] = lo | (hi << 16);
      }
      *(uint4*)(a.out + ((b * W + c) * OUT + r0 + r) * line + 8 * q) = uint4{u[0], u[1], u[2], u[3]};
    }
  } else {
    const int64_t o_ = r0 / IN, i0 = r0 - o_ * IN;
    for (int e = t; e < W * 2 * M * 2; e += 256) {
      const int h = e & 1, pk = (e >> 1) % (2 * M), c = (e >> 1) / (2 * M);
      const uint4 v = *(const uint4*)(tout + ((c * 2) * M + pk) * AX_TR + 8 * h);
      *(uint4*)(a.out + ((b * W + c) * OUT + o_) * line + (int64_t)pk * IN + i0 + 8 * h) = v;
    }
  }
}

struct AxisGradArgs {
  const uint16_t* v;  // forward modes [B][W][OUT][2][M][IN]
  const uint16_t* g;  // mode gradient, same layout
  float* part;        // [nchunk][M][2W][2W]: sum over rows g[row][n] v[row][kk]
  int OUT, IN, M;
  int64_t steps;      // B * OUT * IN / 32
  int64_t per_chunk;  // steps per block
};

// Per-block partial Gram matrices of the mixing's weight gradient.  Grid
// (nchunk, M / 4); wave w of a block owns mode 4 blockIdx.y + w and
// accumulates its 2W x 2W matrix over the block's 32-row steps in
// registers.  IN == 1 or IN % 32 == 0.
template <int W>
__global__ __launch_bounds__(256) void axis_mix_grad_kernel(AxisGradArgs a) {
  constexpr int KK = 2 * W, NT = KK / 16, RP = AX_GR + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sv[4 * KK * RP];
  __shared__ __attribute__((aligned(16))) uint16_t sg[4 * KK * RP];
  const int M = a.M, OUT = a.OUT, IN = a.IN, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int k0 = 4 * blockIdx.y;
  const int64_t rows = (int64_t)OUT * IN, line = (int64_t)2 * M * IN;
  f32x4 acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t s0 = (int64_t)blockIdx.x * a.per_chunk;
  const int64_t s1 = s0 + a.per_chunk < a.steps ? s0 + a.per_chunk : a.steps;
  const int akk = 8 * (lane >> 4);
  for (int64_t s = s0; s < s1; ++s) {
    const int64_t R0 = s * AX_GR, b = R0 / rows, r0 = R0 - b * rows;
    if (IN == 1) {
      // per (c, row, part): the block's four modes, 8 bytes
      for (int e = t; e < W * AX_GR * 2; e += 256) {
        const int part = e & 1, r = (e >> 1) % AX_GR, c = (e >> 1) / AX_GR;
        const int64_t off = ((b * W + c) * OUT + r0 + r) * line + part * M + k0;
        const uint2 x = *(const uint2*)(a.v + off), y = *(const uint2*)(a.g + off);
        const int kk = 2 * c + part;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t wx = j < 2 ? x.x : x.y, wy = j < 2 ? y.x : y.y;
          sv[(j * KK + kk) * RP + r] = (uint16_t)(wx >> (16 * (j & 1)));
          sg[(j * KK + kk) * RP + r] = (uint16_t)(wy >> (16 * (j & 1)));
        }
      }
    } else {
      // per (c, part, mode, quarter): 8 consecutive rows, 16 bytes
      const int64_t o_ = r0 / IN, i0 = r0 - o_ * IN;
      for (int e = t; e < W * 2 * 4 * 4; e += 256) {
        const int q = e & 3, j = (e >> 2) & 3, part = (e >> 4) & 1, c = e >> 5;
        const int64_t off = ((b * W + c) * OUT + o_) * line + (int64_t)(part * M + k0 + j) * IN + i0 + 8 * q;
        const int kk = 2 * c + part;
        *(uint4*)(sv + (j * KK + kk) * RP + 8 * q) = *(const uint4*)(a.v + off);
        *(uint4*)(sg + (j * KK + kk) * RP + 8 * q) = *(const uint4*)(a.g + off);
      }
    }
    __syncthreads();
    // D[n][kk] += sum_r g[r][n] v[r][kk] for this wave's mode
    bf16x8 bv[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) bv[mt] = *(const bf16x8*)(sv + (wave * KK + mt * 16 + (lane & 15)) * RP + akk);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bf16x8 av = *(const bf16x8*)(sg + (wave * KK + nt * 16 + (lane & 15)) * RP + akk);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) acc[nt][mt] = mfma16(av, bv[mt], acc[nt][mt]);
    }
    __syncthreads();
  }
  float* out = a.part + ((int64_t)blockIdx.x * M + k0 + wave) * KK * KK;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        out[(nt * 16 + 4 * (lane >> 4) + j) * KK + mt * 16 + (lane & 15)] = acc[nt][mt][j];
}

// The y and z inverses of one layer in one pass, added to the x inverse:
// for every plane (b, o, x) of Y x Z outputs
//   S[y][z] = bf16(sx[y][z] + sum_pk Yz[y][pk] Iz[pk][z] + sum_pk Iy[pk][y] Yy[pk][z])
// with Yz the z modes [B][W][X Y][2 mz] and Yy the y modes [B][W][X][2 my][Z]
// (the per-axis layouts), Iz and Iy the c2r operands given transposed
// (gt[n][k], rows of kp >= 32, zero padded), sx the FP32 x inverse.  Both
// sums are one MFMA k step each (2 m <= 32), on the same accumulators; the
// y modes are transposed through LDS.  One block per plane; Y, Z in
// {32, 64}.
struct AxisYzArgs {
  const uint16_t* yz;
  const uint16_t* yy;
  const uint16_t* iz;  // [Z][kpz]
  const uint16_t* iy;  // [Y][kpy]
  int32_t kpz, kpy;
  const float* sx;     // [B][W][P]
  uint16_t* s;         // [B][W][P]
  int32_t Y, Z, MY2, MZ2;  // 2 my, 2 mz
};

__global__ __launch_bounds__(256) void axis_inverse_yz_kernel(AxisYzArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t yyt[64 * 40];  // [z][pk], pk padded to 40
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, g = lane >> 4, l16 = lane & 15;
  const int64_t plane = blockIdx.x;  // (b, o, x)
  const int Y = a.Y, Z = a.Z;
  const uint16_t* yz = a.yz + plane * Y * a.MZ2;
  const uint16_t* yy = a.yy + plane * a.MY2 * Z;
  // stage Yy transposed: yyt[z][pk] = Yy[pk][z], zero for pk in [2 my, 32)
  for (int e = t; e < 32 * Z; e += 256) {
    const int pk = e / Z, z = e - pk * Z;
    yyt[z * 40 + pk] = pk < a.MY2 ? yy[pk * Z + z] : (uint16_t)0;
  }
  __syncthreads();
  const int ctn = Z / 16, tiles = (Y / 16) * ctn, per = tiles / 4;
  const int64_t obase = plane * Y * Z;
  for (int j = 0; j < per; ++j) {
    const int i = wave * per + j, rt = i / ctn, ct = i - rt * ctn;
    const int y = 16 * rt + l16, z = 16 * ct + l16;
    // z inverse: A = Yz rows y (k = pk), B = Iz^T rows z
    bf16x8 a1 = bf16x8{};
    if (8 * g < a.MZ2) a1 = *(const bf16x8*)(yz + (int64_t)y * a.MZ2 + 8 * g);
    const bf16x8 b1 = *(const bf16x8*)(a.iz + (int64_t)z * a.kpz + 8 * g);
    // y inverse: A = Iy^T rows y, B = Yy^T rows z (from LDS)
    const bf16x8 a2 = *(const bf16x8*)(a.iy + (int64_t)y * a.kpy + 8 * g);
    const bf16x8 b2 = *(const bf16x8*)(yyt + z * 40 + 8 * g);
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    acc = mfma16(a1, b1, acc);
    acc = mfma16(a2, b2, acc);
    // D[16 rt + 4 g + r][16 ct + l16]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t o = obase + (int64_t)(16 * rt + 4 * g + r) * Z + z;
      a.s[o] = f2bf(acc[r] + a.sx[o]);
    }
  }
}

// Weight gradient of the complex mixing from the Gram partials, summed over
// blocks in a fixed order:
//   dWr[k][c][o] = G[2o][2c] + G[2o+1][2c+1],  dWi[k][c][o] = G[2o+1][2c] - G[2o][2c+1]
// written to grad[((k W + c) W + o) 2 + {0, 1}].
__global__ __launch_bounds__(256) void axis_mix_grad_fold_kernel(const float* part, int64_t nchunk, int M, int W,
                                                                 float* grad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * W * W) return;
  const int o = (int)(e % W), c = (int)((e / W) % W), k = (int)(e / ((int64_t)W * W));
  const int KK = 2 * W;
  float re = 0.f, im = 0.f;
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    const float* G = part + (ch * M + k) * KK * KK;
    re += G[(2 * o) * KK + 2 * c] + G[(2 * o + 1) * KK + 2 * c + 1];
    im += G[(2 * o + 1) * KK + 2 * c] - G[(2 * o) * KK + 2 * c + 1];
  }
  grad[2 * e] = re;
  grad[2 * e + 1] = im;
}

// Embedded BF16 operands of one axis's complex weights theta [M][W][W][2]
// (k, c, o, re/im): E[k][n][kk] and its transpose ET[k][kk][n].
__global__ __launch_bounds__(256) void axis_pack_kernel(const float* theta, int M, int W, uint16_t* E, uint16_t* ET) {
  const int KK = 2 * W;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * KK * KK) return;
  const int kk = (int)(e % KK), n = (int)((e / KK) % KK), k = (int)(e / ((int64_t)KK * KK));
  const int o = n >> 1, pr = n & 1, c = kk >> 1, pc = kk & 1;
  const float* w = theta + (((int64_t)k * W + c) * W + o) * 2;
  const float v = pr == pc ? w[0] : (pr == 0 ? -w[1] : w[1]);
  const uint16_t h = f2bf(v);
  E[e] = h;
  ET[((int64_t)k * KK + kk) * KK + n] = h;
}

}  // namespace mfno
