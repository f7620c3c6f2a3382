// MI355X (gfx950) D3Q27 cumulant lattice Boltzmann solver behind the C ABI
// of include/mi355lbm.h.
//
// One fused kernel per time step: two-lattice pull streaming over a
// structure-of-arrays population field (x fastest, 64 cells per wave), the
// central-moment / cumulant transforms and the collision in registers, the
// boundary substitutions (walls, velocity inlet, zero-gradient outlet via a
// ghost column, halfway or linearly interpolated bounce-back at the
// obstacle), and the fused FP64 mean accumulation, snapshot and per-block
// force partials (paper Sec. 2, 3.1, 3.2).
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_device.h"
#include "mi355lbm.h"

using namespace mlbm;

namespace {

constexpr int TX = 64;   // cells along x per wave
constexpr int TY = 2;    // waves (rows along y) per block
constexpr int NTHREADS = TX * TY;

// Population layout, rows of slots: for each padded z plane and padded row,
// the 27 slots of that row follow each other, each a run of slotp = nx + 64
// elements.  Population i of cell (x, y, z) sits at
//   (z + 1) zstride + (y + 1) rowp + i slotp + x,
// rowp = 27 slotp, zstride = rowp (ny + 2).  Columns -1 and nx of every row
// are the inlet and outlet ghosts (column -1 of slot i is the padding of
// slot i - 1); guard rows and planes keep every neighbour address of a
// domain cell inside the array, so loads may be issued before a boundary
// substitution replaces them.  Everything a tile (64 x 2 cells of one z
// plane) touches lies within three consecutive padded planes: one uniform
// base address plus 32-bit lane offsets.
//
// Streaming is a two-lattice pull: a step reads the post-collision
// populations of the previous step from array A at the upstream cells
// x - c_i (the boundary rules substitute at read time) and writes the cell's
// own post-collision populations to array B, aligned; the arrays swap roles
// every step.  After creation or an import, A holds the natural
// pre-collision state instead (the first step reads it in place).
struct StepArgs {
  const void* A;            // populations read by the step
  void* B;                  // populations written by the step
  int32_t nx, ny, nz;
  int32_t slotp;            // elements per slot run = nx + 64
  int32_t rowp;             // elements per padded row = 27 slotp
  int32_t zstride;          // elements per padded plane = rowp (ny + 2)
  int32_t per[3];           // periodic axes
  const uint8_t* flag;      // [N] 0 fluid, 1 fluid next to obstacle, 2 solid
  const int32_t* brow;      // [N] boundary row of flag-1 cells
  const uint32_t* bmask;    // [nb] bit j: cell + c_j is obstacle
  const double* bq;         // [nb][27] wall distance fractions
  int32_t interp;           // 1: linear interpolated bounce-back
  double* acc;              // [4][N] running sums or null
  float* snap;              // [4][N] snapshot slot or null
  const int32_t* bslot;     // [ntiles] force slot of the tile or -1 (null: no forces)
  double* fpart;            // [nslots][3]
  int32_t tiles_x, tiles_y; // tile grid
  int32_t ntiles;
  int32_t remap;            // XCD-contiguous tile order
  int32_t obox[6];          // tile box (x0, x1, y0, y1, z0, z1) around the obstacle
  uint64_t perturb_seed;    // device-generated initial perturbation
  double perturb_amp;
  int32_t* chk;             // stability flag, set on a check step (null: no check)
};

struct Coefs {
  Coef<float> f;
  Coef<double> d;
};

__device__ __forceinline__ int logical_tile(int b, int ntiles, int remap) {
  if (!remap) return b;
  // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous run of tiles so neighbouring tiles share that XCD's L2
  const int per = ntiles >> 3;
  if (b >= (per << 3)) return b;
  return (b & 7) * per + (b >> 3);
}

// element index of population slot 0 of cell (x, y, z)
__device__ __forceinline__ int64_t cell_index(const StepArgs& a, int x, int y, int z) {
  return (int64_t)(z + 1) * a.zstride + (int64_t)(y + 1) * a.rowp + x;
}

// general element access: population slot of the cell whose slot-0 index is idx
template <typename S>
__device__ __forceinline__ typename Storage<S>::T ld(const void* A, const StepArgs& a, int slot, int64_t idx) {
  return Storage<S>::load((const S*)A + idx + (int64_t)slot * a.slotp);
}
template <typename S>
__device__ __forceinline__ void st(void* A, const StepArgs& a, int slot, int64_t idx, typename Storage<S>::T v) {
  Storage<S>::store((S*)A + idx + (int64_t)slot * a.slotp, v);
}

// Per-cell boundary context of the general path.
struct CellCtx {
  int32_t x, y, z;
  int64_t n;        // dense cell index
  int64_t pc;       // element index of slot 0 of the cell
  uint32_t rmask;   // bit i: pull source cell - c_i is not a fluid node (wall, inlet, obstacle)
  uint32_t inlet;   // bit i: that source is the inlet
  uint32_t om;      // bit j: cell + c_j is obstacle
  int32_t row;      // boundary row or -1
  int32_t off[2][3];// x and y source offset for c = -1, 0, +1 (source = cell - c)
  int64_t offz[3];  // z source offset: a periodic wrap spans nz - 1 padded
                    // planes, more elements than int32 holds on large grids
};

__device__ __forceinline__ int64_t src_off(int i, const CellCtx& c) {
  return (int64_t)(c.off[0][cx(i) + 1] + c.off[1][cy(i) + 1]) + c.offz[cz(i) + 1];
}

__device__ __forceinline__ void make_ctx(const StepArgs& a, int x, int y, int z, uint8_t fl, CellCtx& c) {
  c.x = x; c.y = y; c.z = z;
  c.n = ((int64_t)z * a.ny + y) * a.nx + x;
  c.pc = cell_index(a, x, y, z);
  const int rowp = a.rowp;
  const int64_t plane = a.zstride;
  // x: source of c=+1 is x-1, of c=-1 is x+1 (x+1 = nx is the outlet ghost)
  c.off[0][1] = 0; c.off[1][1] = 0; c.offz[1] = 0;
  c.off[0][2] = (a.per[0] && x == 0) ? (a.nx - 1) : -1;
  c.off[0][0] = (a.per[0] && x == a.nx - 1) ? -(a.nx - 1) : 1;
  c.off[1][2] = (a.per[1] && y == 0) ? (a.ny - 1) * rowp : -rowp;
  c.off[1][0] = (a.per[1] && y == a.ny - 1) ? -(a.ny - 1) * rowp : rowp;
  c.offz[2] = (a.per[2] && z == 0) ? (a.nz - 1) * plane : -plane;
  c.offz[0] = (a.per[2] && z == a.nz - 1) ? -(a.nz - 1) * plane : plane;
  uint32_t wall = 0;
  if (!a.per[1]) {
    if (y == 0) wall |= M_YP;
    if (y == a.ny - 1) wall |= M_YN;
  }
  if (!a.per[2]) {
    if (z == 0) wall |= M_ZP;
    if (z == a.nz - 1) wall |= M_ZN;
  }
  c.inlet = (!a.per[0] && x == 0) ? (M_XP & ~wall) : 0u;
  c.om = 0; c.row = -1;
  if (fl == 1) {
    c.row = a.brow[c.n];
    c.om = a.bmask[c.row];
  }
  c.rmask = wall | c.inlet | reverse27(c.om);
}

// Pre-collision populations of a fluid cell, general path: the pull from
// the upstream cells with the boundary rules applied at read time.
//  wall (y, z at -1/2 and n - 1/2): halfway bounce-back, the cell's own
//    opposite population;
//  inlet (x = -1/2): moving-wall bounce-back with rho_w = 1, the own
//    opposite population plus 6 w_i (c_i . u_in);
//  outlet: the source x = nx is the ghost column, which holds the copy of
//    the post-collision column nx - 1 (zero gradient);
//  obstacle: halfway bounce-back, or linear interpolation with the wall
//    distance q of the link: q < 1/2 blends the own opposite population with
//    the one the fluid node behind the cell sent (halfway where that node is
//    not fluid); q >= 1/2 blends it with the cell's own population i.
// natural = true: A holds the pre-collision state itself.
template <typename S>
__device__ __forceinline__ void load_general(const StepArgs& a, const Coef<typename Storage<S>::T>& k,
                                             const CellCtx& c, bool natural, typename Storage<S>::T* g) {
  using T = typename Storage<S>::T;
  if (natural) {
#pragma unroll
    for (int i = 0; i < 27; ++i) g[i] = ld<S>(a.A, a, i, c.pc);
    return;
  }
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const bool r = (c.rmask >> i) & 1u;
    T v = ld<S>(a.A, a, r ? 26 - i : i, r ? c.pc : c.pc + src_off(i, c));
    if (cx(i) == 1 && ((c.inlet >> i) & 1u)) v += T(wgt(i)) * k.u6;
    g[i] = v;
  }
  if (a.interp && c.om) {
    // g[26 - i] of a direction whose source is fluid is never modified here
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      if ((c.om >> (26 - i)) & 1u) {
        const T q = T(a.bq[(int64_t)c.row * 27 + (26 - i)]);
        if (q < T(0.5)) {
          if (!((c.rmask >> (26 - i)) & 1u)) g[i] = T(2) * q * g[i] + (T(1) - T(2) * q) * g[26 - i];
        } else {
          g[i] = g[i] / (T(2) * q) + (T(2) * q - T(1)) / (T(2) * q) * ld<S>(a.A, a, i, c.pc);
        }
      }
    }
  }
}

// Interior fast path: no wall, obstacle or periodic wrap in the wave.  zb
// is the uniform address of the tile's plane, biased back by one padded row
// and one element, p0 the lane's biased byte offset; the neighbour offsets
// are compile-time combinations of the slot, row and plane strides and stay
// non-negative for every domain cell.
template <typename S>
__device__ __forceinline__ const char* plane_base(const void* A, const StepArgs& a, int z) {
  return (const char*)A + ((int64_t)z * a.zstride - (a.rowp + 1)) * (int64_t)sizeof(S);
}
template <typename S>
__device__ __forceinline__ uint32_t lane_off(const StepArgs& a, int x, int y) {
  return (uint32_t)(((y + 2) * a.rowp + x + 1) * (int)sizeof(S));
}
template <typename S>
__device__ __forceinline__ uint32_t fast_off(const StepArgs& a, uint32_t p0, int slot, int dx, int dy, int dz) {
  return p0 + (uint32_t)(((1 + dz) * a.zstride + dy * a.rowp + slot * a.slotp + dx) * (int)sizeof(S));
}

template <typename S>
__device__ __forceinline__ void load_fast(const StepArgs& a, const char* zb, uint32_t p0,
                                          typename Storage<S>::T* g) {
#pragma unroll
  for (int i = 0; i < 27; ++i) g[i] = Storage<S>::load_nt((const S*)(zb + fast_off<S>(a, p0, i, -cx(i), -cy(i), -cz(i))));
}

template <typename T>
__device__ __forceinline__ void macroscopic(const T* g, const Coef<T>& k, T& drho, T& ux, T& uy, T& uz) {
  // pairwise sums of opposite directions
  T d = g[13];
  T jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    const T s = g[i] + g[26 - i], t = g[26 - i] - g[i];  // t carries c of direction 26-i
    d += s;
    const int o = 26 - i;
    if (cx(o)) jx += cx(o) > 0 ? t : -t;
    if (cy(o)) jy += cy(o) > 0 ? t : -t;
    if (cz(o)) jz += cz(o) > 0 ? t : -t;
  }
  const T irho = T(1) / (T(1) + d);
  drho = d;
  ux = (jx + k.hf[0]) * irho;
  uy = (jy + k.hf[1]) * irho;
  uz = (jz + k.hf[2]) * irho;
}

// One cell update.  PATH 0: interior wave (no wall, obstacle, periodic wrap,
// inlet or outlet column in the wave); PATH 1: interior wave of the first or
// last x tile, with the inlet column handled per lane (the outlet column
// pulls from the ghost column like any other source); PATH 2: general
// boundary path.  NAT: the first step after creation or an import, which
// reads the natural pre-collision state in place (PATH 2 only).  Every path
// stores the cell's 27 post-collision populations to B at the cell itself;
// column nx - 1 also fills the outlet ghost column nx with its populations
// that move in -x (zero-gradient outlet).
template <typename S, bool NAT, int MODE, int PATH>
__device__ __forceinline__ void cell_update(const StepArgs& a, const Coef<typename Storage<S>::T>& k, int x, int y,
                                            int z, int64_t n, uint8_t fl, double& fx, double& fy, double& fz) {
  using T = typename Storage<S>::T;
  CellCtx c;
  T g[27];
  T Fx = 0, Fy = 0, Fz = 0;
  const char* zb = plane_base<S>(a.A, a, z);
  const uint32_t p0 = lane_off<S>(a, x, y);
  const bool at_inlet = PATH == 1 && !a.per[0] && x == 0;
  const bool outlet = PATH != 0 && !a.per[0] && x == a.nx - 1;
  if (PATH < 2) {
    load_fast<S>(a, zb, p0, g);
    if (at_inlet) {
#pragma unroll
      for (int i = 0; i < 27; ++i)
        if (cx(i) == 1)
          g[i] = Storage<S>::load((const S*)(zb + fast_off<S>(a, p0, 26 - i, 0, 0, 0))) + T(wgt(i)) * k.u6;
    }
  } else {
    make_ctx(a, x, y, z, fl, c);
    load_general<S>(a, k, c, NAT, g);
    // incoming half of the momentum exchange on obstacle links
    if (c.om) {
#pragma unroll
      for (int j = 0; j < 27; ++j)
        if ((c.om >> j) & 1u) {
          const T v = g[26 - j];
          if (cx(j)) Fx += cx(j) > 0 ? v : -v;
          if (cy(j)) Fy += cy(j) > 0 ? v : -v;
          if (cz(j)) Fz += cz(j) > 0 ? v : -v;
        }
    }
  }

  T drho, rho, irho, ux, uy, uz;
  macro_and_forward(g, k.hf, drho, rho, irho, ux, uy, uz);
  if (a.acc) {
    const int64_t N = (int64_t)a.nx * a.ny * a.nz;
    a.acc[n] += (double)ux;
    a.acc[N + n] += (double)uy;
    a.acc[2 * N + n] += (double)uz;
    a.acc[3 * N + n] += (double)drho * (1.0 / 3.0);
  }
  if (a.chk) {
    // a cell whose density left (0, 2) or whose speed reached the lattice
    // sound speed (or any non-finite value: every comparison fails) marks
    // the run as unstable
    const T usq = ux * ux + uy * uy + uz * uz;
    if (!(usq < T(1.0 / 3.0) && drho > T(-1) && drho < T(1))) *a.chk = 1;
  }
  if (a.snap) {
    const int64_t N = (int64_t)a.nx * a.ny * a.nz;
    a.snap[n] = (float)ux;
    a.snap[N + n] = (float)uy;
    a.snap[2 * N + n] = (float)uz;
    a.snap[3 * N + n] = (float)(drho * T(1.0 / 3.0));
  }
  collide_moments<T, MODE>(g, drho, rho, irho, ux, uy, uz, k);
  inverse_transform(g, ux, uy, uz);

  char* wb = (char*)plane_base<S>(a.B, a, z);
#pragma unroll
  for (int j = 0; j < 27; ++j) {
    S* p = (S*)(wb + fast_off<S>(a, p0, j, 0, 0, 0));
    Storage<S>::store_nt(p, g[j]);
    if (cx(j) == -1 && outlet) Storage<S>::store(p + 1, g[j]);  // ghost column copy
  }
  if (PATH == 2 && c.om) {
#pragma unroll
    for (int j = 0; j < 27; ++j)
      if ((c.om >> j) & 1u) {
        const T v = g[j];
        if (cx(j)) Fx += cx(j) > 0 ? v : -v;
        if (cy(j)) Fy += cy(j) > 0 ? v : -v;
        if (cz(j)) Fz += cz(j) > 0 ? v : -v;
      }
    fx = (double)Fx; fy = (double)Fy; fz = (double)Fz;
  }
}

#ifndef MLBM_WAVES
#define MLBM_WAVES 3
#endif
#ifndef MLBM_EDGE_PATH
#define MLBM_EDGE_PATH 1
#endif
template <typename S, bool NAT, int MODE>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(MLBM_WAVES, 8))) void lbm_step_kernel(
    StepArgs a, Coef<typename Storage<S>::T> k) {
  const int tile = logical_tile(blockIdx.x, a.ntiles, a.remap);
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int z = rest / a.tiles_y;
  const int x = txi * TX + tx, y = tyi * TY + ty;
  const int64_t n = ((int64_t)z * a.ny + y) * a.nx + x;

  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (NAT) {
    const uint8_t fl = a.flag[n];
    if (fl != 2) cell_update<S, true, MODE, 2>(a, k, x, y, z, n, fl, fx, fy, fz);
  } else {
    // Tiles away from the walls, periodic faces and the obstacle's box hold
    // only fluid cells: they skip the cell flags, so their population loads
    // do not wait for a flag load.
    const bool plain_tile = z > 0 && z < a.nz - 1 && tyi > 0 && tyi < a.tiles_y - 1 &&
                            !(a.per[0] && (txi == 0 || txi == a.tiles_x - 1)) &&
                            !(txi >= a.obox[0] && txi <= a.obox[1] && tyi >= a.obox[2] && tyi <= a.obox[3] &&
                              z >= a.obox[4] && z <= a.obox[5]);
    if (plain_tile) {
      if (!a.per[0] && (txi == 0 || txi == a.tiles_x - 1))
        cell_update<S, false, MODE, MLBM_EDGE_PATH>(a, k, x, y, z, n, 0, fx, fy, fz);
      else
        cell_update<S, false, MODE, 0>(a, k, x, y, z, n, 0, fx, fy, fz);
    } else if (const uint8_t fl = a.flag[n]; fl != 2) {
      // periodic axes wrap at their faces and walls bounce back: both take
      // the general path; the inlet and outlet columns take the edge path
      const bool xin = a.per[0] ? (x > 0 && x < a.nx - 1) : true;
      const bool interior = fl == 0 && xin && y > 0 && y < a.ny - 1 && z > 0 && z < a.nz - 1;
      const bool edge_tile = !a.per[0] && (txi == 0 || txi == a.tiles_x - 1);
      if (!__any(!interior)) {
        if (edge_tile) cell_update<S, false, MODE, MLBM_EDGE_PATH>(a, k, x, y, z, n, fl, fx, fy, fz);
        else cell_update<S, false, MODE, 0>(a, k, x, y, z, n, fl, fx, fy, fz);
      } else {
        cell_update<S, false, MODE, 2>(a, k, x, y, z, n, fl, fx, fy, fz);
      }
    }
  }

  // per-block FP64 force partial, deterministic order
  if (a.bslot) {
    const int s = a.bslot[tile];
    if (s >= 0) {
      __shared__ double red[3][NTHREADS];
      red[0][threadIdx.x] = fx; red[1][threadIdx.x] = fy; red[2][threadIdx.x] = fz;
      __syncthreads();
#pragma unroll
      for (int w = NTHREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
          red[0][threadIdx.x] += red[0][threadIdx.x + w];
          red[1][threadIdx.x] += red[1][threadIdx.x + w];
          red[2][threadIdx.x] += red[2][threadIdx.x + w];
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        a.fpart[3 * s + 0] = red[0][0];
        a.fpart[3 * s + 1] = red[1][0];
        a.fpart[3 * s + 2] = red[2][0];
      }
    }
  }
}

// Bandwidth probe: the pull step's memory traffic with the collision left
// out.  Every cell of every tile loads its 27 populations from the
// upstream cells of A and stores them to itself in B, through the same
// addressing, hints and tile order as the stream-and-collide kernel.  A is
// only read, so the state is unchanged.
template <typename S>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(MLBM_WAVES, 8))) void pull_probe_kernel(
    StepArgs a) {
  using T = typename Storage<S>::T;
  const int tile = logical_tile(blockIdx.x, a.ntiles, a.remap);
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int z = rest / a.tiles_y;
  const int x = txi * TX + tx, y = tyi * TY + ty;
  const uint32_t p0 = lane_off<S>(a, x, y);
  T g[27];
  load_fast<S>(a, plane_base<S>(a.A, a, z), p0, g);
  char* wb = (char*)plane_base<S>(a.B, a, z);
#pragma unroll
  for (int j = 0; j < 27; ++j) Storage<S>::store_nt((S*)(wb + fast_off<S>(a, p0, j, 0, 0, 0)), g[j]);
}

// Plain streaming copy: one 16-byte vector per lane, non-temporal stores,
// one pass over the buffer with no loop.  The attainable-bandwidth
// reference of the roofline (the fastest of the copy forms measured on
// MI355X: 6.3 TB/s against 4.5-5.4 TB/s for grid-stride loops).
typedef float float4_v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_probe_kernel(const float4_v* __restrict__ src, float4_v* __restrict__ dst,
                                                         int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n4) __builtin_nontemporal_store(src[i], dst + i);
}

// Sum of the force partials in a fixed order, plus the constant weight part.
__global__ __launch_bounds__(256) void force_reduce_kernel(const double* fpart, int nslots, double c0, double c1,
                                                           double c2, double* out) {
  __shared__ double red[3][256];
  double s0 = 0, s1 = 0, s2 = 0;
  for (int k = threadIdx.x; k < nslots; k += 256) {
    s0 += fpart[3 * k]; s1 += fpart[3 * k + 1]; s2 += fpart[3 * k + 2];
  }
  red[0][threadIdx.x] = s0; red[1][threadIdx.x] = s1; red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
      red[2][threadIdx.x] += red[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0] + c0; out[1] = red[1][0] + c1; out[2] = red[2][0] + c2;
  }
}

// Natural-layout state: the pre-collision populations of a cell written in
// place into dst (the state the next step reads with NAT).
template <typename S>
__device__ __forceinline__ void store_natural(void* dst, const StepArgs& a, int x, int y, int z,
                                              typename Storage<S>::T* g) {
  const int64_t pc = cell_index(a, x, y, z);
#pragma unroll
  for (int i = 0; i < 27; ++i) st<S>(dst, a, i, pc, g[i]);
}

// Equilibrium initial state at rho = 1: fbar = w (Phi - 1) with Phi the
// product of per-axis factors 1 + delta (delta(0) = -3a^2/2,
// delta(+-1) = 3a^2 +- 3a), expanded so that no rest value is subtracted.
template <typename S>
__global__ __launch_bounds__(256) void init_kernel(StepArgs a, const double* u0, void* dst) {
  using T = typename Storage<S>::T;
  const int64_t N = (int64_t)a.nx * a.ny * a.nz;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / ((int64_t)a.nx * a.ny);
  const uint8_t fl = a.flag[n];
  T g[27];
  if (fl == 2) {
    const int64_t pc = cell_index(a, x, y, z);
    for (int i = 0; i < 27; ++i) st<S>(dst, a, i, pc, T(0));
    return;
  }
  T u[3] = {0, 0, 0};
  if (u0) {
    u[0] = T(u0[n]); u[1] = T(u0[N + n]); u[2] = T(u0[2 * N + n]);
  } else if (a.perturb_amp != 0.0) {
    for (int d = 0; d < 3; ++d) {
      // counter-based SplitMix64 (Steele, Lea, Flood 2014), output 3n + d
      uint64_t zz = a.perturb_seed + (uint64_t)(3 * n + d + 1) * 0x9E3779B97F4A7C15ull;
      zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
      zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
      zz ^= zz >> 31;
      const double xi = (double)(zz >> 11) * 0x1.0p-53 * 2.0 - 1.0;
      u[d] = T(a.perturb_amp * xi);
    }
  }
  T del[3][3];
  for (int d = 0; d < 3; ++d) {
    del[d][1] = T(-1.5) * u[d] * u[d];
    del[d][0] = T(3) * u[d] * u[d] - T(3) * u[d];
    del[d][2] = T(3) * u[d] * u[d] + T(3) * u[d];
  }
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const T dx = del[0][cx(i) + 1], dy = del[1][cy(i) + 1], dz = del[2][cz(i) + 1];
    const T ph = dx + dy + dz + dx * dy + dx * dz + dy * dz + dx * dy * dz;
    g[i] = T(wgt(i)) * ph;
  }
  store_natural<S>(dst, a, x, y, z, g);
}

// Natural-layout export of the pre-collision state (pulled from A, or A
// itself when it holds the natural state): populations as double [27][N],
// and/or moments (u, v, w, p) as float [4][N], and/or the per-block mass
// partial.
template <typename S, bool NAT>
__global__ __launch_bounds__(NTHREADS) void export_kernel(StepArgs a, Coef<typename Storage<S>::T> k, double* pops,
                                                          float* mom, double* mass_part) {
  using T = typename Storage<S>::T;
  const int tile = blockIdx.x;
  const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
  const int txi = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int tyi = rest % a.tiles_y;
  const int z = rest / a.tiles_y;
  const int x = txi * TX + tx, y = tyi * TY + ty;
  const int64_t N = (int64_t)a.nx * a.ny * a.nz;
  const int64_t n = ((int64_t)z * a.ny + y) * a.nx + x;
  const uint8_t fl = a.flag[n];
  double dm = 0.0;
  if (fl != 2) {
    CellCtx c;
    make_ctx(a, x, y, z, fl, c);
    T g[27];
    load_general<S>(a, k, c, NAT, g);
    if (pops)
      for (int i = 0; i < 27; ++i) pops[(int64_t)i * N + n] = (double)g[i];
    T drho, ux, uy, uz;
    macroscopic(g, k, drho, ux, uy, uz);
    if (mom) {
      mom[n] = (float)ux; mom[N + n] = (float)uy; mom[2 * N + n] = (float)uz;
      mom[3 * N + n] = (float)(drho * T(1.0 / 3.0));
    }
    dm = (double)drho;
  } else {
    if (pops)
      for (int i = 0; i < 27; ++i) pops[(int64_t)i * N + n] = 0.0;
    if (mom)
      for (int k = 0; k < 4; ++k) mom[k * N + n] = 0.f;
  }
  if (mass_part) {
    __shared__ double red[NTHREADS];
    red[threadIdx.x] = dm;
    __syncthreads();
    for (int w = NTHREADS / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) mass_part[tile] = red[0];
  }
}

// Natural-layout export of a box of cells [x0, x0 + bx) x [y0, y0 + by) x
// [z0, z0 + bz): pops [27][bz][by][bx], the same values export_kernel
// writes for those cells.
template <typename S, bool NAT>
__global__ __launch_bounds__(256) void export_box_kernel(StepArgs a, Coef<typename Storage<S>::T> k, int x0, int y0,
                                                         int z0, int bx, int by, int bz, double* pops) {
  using T = typename Storage<S>::T;
  const int64_t nb = (int64_t)bx * by * bz;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nb) return;
  const int x = x0 + (int)(i % bx), y = y0 + (int)((i / bx) % by), z = z0 + (int)(i / ((int64_t)bx * by));
  const int64_t n = ((int64_t)z * a.ny + y) * a.nx + x;
  const uint8_t fl = a.flag[n];
  if (fl == 2) {
    for (int q = 0; q < 27; ++q) pops[(int64_t)q * nb + i] = 0.0;
    return;
  }
  CellCtx c;
  make_ctx(a, x, y, z, fl, c);
  T g[27];
  load_general<S>(a, k, c, NAT, g);
  for (int q = 0; q < 27; ++q) pops[(int64_t)q * nb + i] = (double)g[q];
}

// Natural-layout import: double fbar [27][N] -> the natural state in dst.
template <typename S>
__global__ __launch_bounds__(256) void import_kernel(StepArgs a, const double* pops, void* dst) {
  using T = typename Storage<S>::T;
  const int64_t N = (int64_t)a.nx * a.ny * a.nz;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / ((int64_t)a.nx * a.ny);
  const uint8_t fl = a.flag[n];
  T g[27];
  for (int i = 0; i < 27; ++i) g[i] = fl == 2 ? T(0) : T(pops[(int64_t)i * N + n]);
  store_natural<S>(dst, a, x, y, z, g);
}

// Mean fields = sums / count, zero in solid cells.
__global__ __launch_bounds__(256) void mean_kernel(const double* acc, int64_t N, double inv, const uint8_t* flag,
                                                   double* out) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const bool sol = flag[n] == 2;
  for (int k = 0; k < 4; ++k) out[k * N + n] = sol ? 0.0 : acc[k * N + n] * inv;
}

// Block means of the running sums over f x f x f cells, written in the
// surrogate's [channel][X][Y][Z] layout (Z fastest), solid cells counting as
// zero; optionally turned by q quarter turns about +x.  The turned field at
// (x, y', z') is R^q applied to the field at R^-q (x, y', z'), where R takes
// +y to +z and +z to -y; on indices (Y == Z) R^-1 maps (y', z') to
// (z', Y - 1 - y') and R maps the vector (u, v, w) to (u, -w, v).
__global__ __launch_bounds__(256) void pool_kernel(const double* acc, int64_t N, double inv, const uint8_t* flag,
                                                   int nx, int ny, int f, int X, int Y, int Z, int turns,
                                                   float* out) {
  const int64_t P = (int64_t)X * Y * Z;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= P) return;
  const int zo = (int)(e % Z), yo = (int)((e / Z) % Y), xo = (int)(e / ((int64_t)Y * Z));
  int ys = yo, zs = zo;
  for (int t = 0; t < turns; ++t) {
    const int yn = zs, zn = Y - 1 - ys;
    ys = yn;
    zs = zn;
  }
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int dz = 0; dz < f; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int64_t n = ((int64_t)(zs * f + dz) * ny + (ys * f + dy)) * nx + (xo * f + dx);
        if (flag[n] == 2) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += acc[k * N + n];
      }
  const double sc = inv / (double)(f * f * f);
  double u = s[0] * sc, v = s[1] * sc, w = s[2] * sc;
  for (int t = 0; t < turns; ++t) {
    const double vn = -w, wn = v;
    v = vn;
    w = wn;
  }
  out[e] = (float)u;
  out[P + e] = (float)v;
  out[2 * P + e] = (float)w;
  out[3 * P + e] = (float)(s[3] * sc);
}

// Boundary tables: mark flag-1 cells and their rows.
__global__ __launch_bounds__(256) void scatter_rows_kernel(const int64_t* cells, int64_t nb, uint8_t* flag,
                                                           int32_t* brow) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nb) return;
  const int64_t n = cells[r];
  flag[n] = 1;
  brow[n] = (int32_t)r;
}

}  // namespace

// ============================================================== host side
struct lbm_sim {
  lbm_params p{};
  double omega1 = 0;
  int mode = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0;
  size_t esize = 0;
  StepArgs args{};
  Coefs coefs{};
  int64_t pop_elems = 0;
  char* block = nullptr;     // device memory of the solver (see Layout)
  bool owns_block = false;   // false: the caller's workspace
  void* arr[2] = {nullptr, nullptr};  // the two population lattices
  int cur = 0;               // lattice holding the state
  bool natural = true;       // true: it holds the natural pre-collision state
  uint8_t* d_flag = nullptr;
  int32_t* d_brow = nullptr;
  uint32_t* d_bmask = nullptr;
  double* d_bq = nullptr;
  int64_t nb = 0;
  int32_t* d_bslot = nullptr;
  int32_t nslots = 0;
  double* d_fpart = nullptr;
  double fconst[3] = {0, 0, 0};
  double* d_forces = nullptr;
  bool force_ring = false;   // true: the last force_cap samples, in the block
  int64_t force_cap = 0, nforces = 0;
  std::vector<int64_t> force_steps;
  double* d_acc = nullptr;
  int64_t nsamples = 0;
  float* d_snap = nullptr;
  int64_t snap_taken = 0;
  std::vector<int64_t> snap_steps;
  int32_t* d_chk = nullptr;  // stability flag written by check steps
  int32_t* h_chk = nullptr;  // its pinned host copy, refreshed after each check step
  int64_t steps = 0;
  int sticky = 0;
  std::string err;
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double prof_ms = 0;
  int64_t prof_launches = 0;
};

static std::string g_err;

static int fail(lbm_sim* s, int code, const std::string& msg) {
  if (s) {
    s->err = msg;
    if (code == LBM_EDEVICE || code == LBM_EUNSTABLE) s->sticky = code;
  }
  g_err = msg;
  return code;
}

#define HIPCHK(s, call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((s), e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,                  \
                  std::string(#call) + ": " + hipGetErrorString(e_));                         \
  } while (0)

static size_t storage_size(int st) {
  switch (st) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16S: return 2;
    case LBM_BF16S: return 2;
  }
  return 0;
}

extern "C" int lbm_default_params(lbm_params* p, int32_t nx, int32_t ny, int32_t nz) {
  if (!p) return LBM_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx; p->ny = ny; p->nz = nz;
  p->storage = LBM_F32;
  p->u_in = 0.05;
  p->nu = 0.05 * ny / 5000.0;
  p->omega2 = 1.0;
  p->mode = LBM_MODE_AUTO;
  p->galilean = 1;
  p->lambda = 0.01;
  p->obstacle_bc = 0;
  p->avg_start = 0;
  p->snap_every = 0;
  p->snap_count = 20;
  p->snap_start = 0;
  p->force_every = 1;
  p->xcd_remap = 1;
  return LBM_OK;
}

static void k17_rates(double w1, double w2, double* o) {
  o[0] = 8.0 * (w1 - 2.0) * (w2 * (3.0 * w1 - 1.0) - 5.0 * w1) /
         (8.0 * (5.0 - 2.0 * w1) * w1 + w2 * (8.0 + w1 * (9.0 * w1 - 26.0)));
  o[1] = 8.0 * (w1 - 2.0) * (w1 + w2 * (3.0 * w1 - 7.0)) / (w2 * (56.0 - 42.0 * w1 + 9.0 * w1 * w1) - 8.0 * w1);
  o[2] = 24.0 * (w1 - 2.0) * (4.0 * w1 * w1 + w1 * w2 * (18.0 - 13.0 * w1) + w2 * w2 * (2.0 + w1 * (6.0 * w1 - 11.0))) /
         (16.0 * w1 * w1 * (w1 - 6.0) - 2.0 * w1 * w2 * (216.0 + 5.0 * w1 * (9.0 * w1 - 46.0)) +
          w2 * w2 * (w1 * (3.0 * w1 - 10.0) * (15.0 * w1 - 28.0) - 48.0));
  o[3] = (4.0 * w1 * w1 + 2.0 * w1 * w2 * (w1 - 6.0) + w2 * w2 * (w1 * (10.0 - 3.0 * w1) - 4.0)) /
         ((w1 - w2) * (w2 * (2.0 + 3.0 * w1) - 8.0 * w1));
  o[4] = (4.0 * w1 * w2 * (9.0 * w1 - 16.0) - 4.0 * w1 * w1 - 2.0 * w2 * w2 * (2.0 + 9.0 * w1 * (w1 - 2.0))) /
         (3.0 * (w1 - w2) * (w2 * (2.0 + 3.0 * w1) - 8.0 * w1));
}

template <typename T>
static void fill_coef(Coef<T>& k, double w1, double w2, double G, double lam, const double* k17, const double* force,
                      double u_in) {
  k.w1 = T(w1); k.w2 = T(w2);
  k.omw1 = T(1.0 - w1); k.omw2 = T(1.0 - w2);
  k.c1 = T(G * 3.0 * (1.0 - 0.5 * w1));
  k.c2 = T(G * 3.0 * (1.0 - 0.5 * w2));
  k.lam = T(lam);
  k.l3 = T((1.0 - k17[0]) * lam);
  k.l4 = T((1.0 - k17[1]) * lam);
  k.l5 = T((1.0 - k17[2]) * lam);
  const double t = 1.0 / w1 - 0.5;
  k.a4 = T(-(2.0 / 3.0) * t * k17[3]);
  k.b4 = T(t * k17[4] * w1);
  for (int d = 0; d < 3; ++d) k.hf[d] = T(0.5 * force[d]);
  k.u6 = T(6.0 * u_in);
}

template <typename S> static const Coef<typename Storage<S>::T>& coef_for(const Coefs& c);
template <> const Coef<double>& coef_for<double>(const Coefs& c) { return c.d; }
template <> const Coef<float>& coef_for<float>(const Coefs& c) { return c.f; }
template <> const Coef<float>& coef_for<f16s>(const Coefs& c) { return c.f; }
template <> const Coef<float>& coef_for<bf16s>(const Coefs& c) { return c.f; }

// Occupancy cap of the FP32 pull step through dynamic LDS the kernel does
// not use.  With its 3 KB of static LDS, 17 KB allows 8 blocks of two waves
// per CU (4 waves per SIMD).  Kernel time per launch at 1024x512x512, three
// to four repeats each: 9.78-9.92 ms capped, 10.22-10.41 ms without; at
// 256x128x128 the cap makes no difference (0.273-0.276 ms), so small grids
// run without it.
#ifndef MLBM_F32_CAP_LDS
#define MLBM_F32_CAP_LDS 17408
#endif
static size_t f32_cap_lds(int64_t ntiles) {
  return ntiles >= (int64_t(1) << 16) ? (size_t)MLBM_F32_CAP_LDS : 0;
}

template <typename S, bool NAT, int MODE>
static void launch_step(const StepArgs& a, const Coefs& c, hipStream_t st) {
  const size_t lds = (!NAT && std::is_same<S, float>::value) ? f32_cap_lds(a.ntiles) : 0;
  hipLaunchKernelGGL((lbm_step_kernel<S, NAT, MODE>), dim3(a.ntiles), dim3(NTHREADS), lds, st, a, coef_for<S>(c));
}

template <typename S>
static void launch_step_s(const StepArgs& a, const Coefs& c, bool nat, int mode, hipStream_t st) {
  if (nat) {
    if (mode) launch_step<S, true, 1>(a, c, st); else launch_step<S, true, 0>(a, c, st);
  } else {
    if (mode) launch_step<S, false, 1>(a, c, st); else launch_step<S, false, 0>(a, c, st);
  }
}

static void launch_step_any(int storage, const StepArgs& a, const Coefs& c, bool nat, int mode, hipStream_t st) {
  switch (storage) {
    case LBM_F64: launch_step_s<double>(a, c, nat, mode, st); break;
    case LBM_F32: launch_step_s<float>(a, c, nat, mode, st); break;
    case LBM_F16S: launch_step_s<f16s>(a, c, nat, mode, st); break;
    case LBM_BF16S: launch_step_s<bf16s>(a, c, nat, mode, st); break;
  }
}

template <typename S>
static void launch_export_s(const StepArgs& a, const Coefs& c, bool nat, double* pops, float* mom, double* mp,
                            hipStream_t st) {
  if (nat)
    hipLaunchKernelGGL((export_kernel<S, true>), dim3(a.ntiles), dim3(NTHREADS), 0, st, a, coef_for<S>(c), pops, mom,
                       mp);
  else
    hipLaunchKernelGGL((export_kernel<S, false>), dim3(a.ntiles), dim3(NTHREADS), 0, st, a, coef_for<S>(c), pops,
                       mom, mp);
}

static void launch_export(int storage, const StepArgs& a, const Coefs& c, bool nat, double* pops, float* mom,
                          double* mp, hipStream_t st) {
  switch (storage) {
    case LBM_F64: launch_export_s<double>(a, c, nat, pops, mom, mp, st); break;
    case LBM_F32: launch_export_s<float>(a, c, nat, pops, mom, mp, st); break;
    case LBM_F16S: launch_export_s<f16s>(a, c, nat, pops, mom, mp, st); break;
    case LBM_BF16S: launch_export_s<bf16s>(a, c, nat, pops, mom, mp, st); break;
  }
}

template <typename S>
static void launch_export_box_s(const StepArgs& a, const Coefs& c, bool nat, const int* box, double* pops,
                                hipStream_t st) {
  const int64_t nb = (int64_t)box[3] * box[4] * box[5];
  const dim3 g((unsigned)((nb + 255) / 256));
  if (nat)
    hipLaunchKernelGGL((export_box_kernel<S, true>), g, dim3(256), 0, st, a, coef_for<S>(c), box[0], box[1], box[2],
                       box[3], box[4], box[5], pops);
  else
    hipLaunchKernelGGL((export_box_kernel<S, false>), g, dim3(256), 0, st, a, coef_for<S>(c), box[0], box[1], box[2],
                       box[3], box[4], box[5], pops);
}

static void launch_init(int storage, const StepArgs& a, const double* u0, void* dst, hipStream_t st) {
  const int64_t N = (int64_t)a.nx * a.ny * a.nz;
  const dim3 g((unsigned)((N + 255) / 256));
  switch (storage) {
    case LBM_F64: hipLaunchKernelGGL(init_kernel<double>, g, dim3(256), 0, st, a, u0, dst); break;
    case LBM_F32: hipLaunchKernelGGL(init_kernel<float>, g, dim3(256), 0, st, a, u0, dst); break;
    case LBM_F16S: hipLaunchKernelGGL(init_kernel<f16s>, g, dim3(256), 0, st, a, u0, dst); break;
    case LBM_BF16S: hipLaunchKernelGGL(init_kernel<bf16s>, g, dim3(256), 0, st, a, u0, dst); break;
  }
}

static void launch_import(int storage, const StepArgs& a, const double* pops, void* dst, hipStream_t st) {
  const int64_t N = (int64_t)a.nx * a.ny * a.nz;
  const dim3 g((unsigned)((N + 255) / 256));
  switch (storage) {
    case LBM_F64: hipLaunchKernelGGL(import_kernel<double>, g, dim3(256), 0, st, a, pops, dst); break;
    case LBM_F32: hipLaunchKernelGGL(import_kernel<float>, g, dim3(256), 0, st, a, pops, dst); break;
    case LBM_F16S: hipLaunchKernelGGL(import_kernel<f16s>, g, dim3(256), 0, st, a, pops, dst); break;
    case LBM_BF16S: hipLaunchKernelGGL(import_kernel<bf16s>, g, dim3(256), 0, st, a, pops, dst); break;
  }
}

static void free_all(lbm_sim* s) {
  if (s->block && s->owns_block) (void)hipFree(s->block);
  s->block = nullptr;
  if (s->d_forces && !s->force_ring) (void)hipFree(s->d_forces);
  s->d_forces = nullptr;
  if (s->h_chk) (void)hipHostFree(s->h_chk);
  s->h_chk = nullptr;
  for (auto& e : s->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  s->events.clear();
}

// Parameters resolved from lbm_params: viscosity (from re and l_ref when
// re > 0, paper Sec. 3.1: Re set through the lattice viscosity), omega1,
// collision mode (paper Sec. 3.2: the fourth-order mode off below Re_c 3000)
// and the fourth-order rates.  Rejects what the step cannot run.
struct Resolved {
  double nu = 0, omega1 = 0;
  int mode = 0;
  double k17[5] = {0, 0, 0, 0, 0};
  int64_t N = 0, slotp = 0, rowp = 0, zstride = 0, pop_elems = 0, ntiles = 0;
};

static int resolve(const lbm_params& p, Resolved& r) {
  if (p.nx <= 0 || p.ny <= 0 || p.nz <= 0 || p.nx % TX || p.ny % TY)
    return fail(nullptr, LBM_EINVAL, "grid must have nx % 64 == 0 and ny % 2 == 0");
  if (storage_size(p.storage) == 0) return fail(nullptr, LBM_EINVAL, "unknown storage type");
  if (p.re > 0.0) {
    if (!(p.u_in > 0.0) || !std::isfinite(p.re)) return fail(nullptr, LBM_EINVAL, "re needs u_in > 0");
    r.nu = p.u_in * (p.l_ref > 0.0 ? p.l_ref : (double)p.ny) / p.re;
  } else {
    r.nu = p.nu;
  }
  if (!(r.nu > 0.0) || !std::isfinite(r.nu)) return fail(nullptr, LBM_EINVAL, "viscosity must be positive");
  if (!(p.omega2 > 0.0 && p.omega2 < 2.0)) return fail(nullptr, LBM_EINVAL, "omega2 must be in (0, 2)");
  if (p.snap_every < 0 || p.snap_count < 0 || p.force_every < 0 || p.check_every < 0 || p.force_capacity < 0)
    return fail(nullptr, LBM_EINVAL, "negative period or capacity");
  if (p.snap_every > 0 && p.snap_count <= 0) return fail(nullptr, LBM_EINVAL, "snap_count must be positive");
  r.omega1 = 1.0 / (3.0 * r.nu + 0.5);
  const double re_c = p.u_in * p.ny / r.nu;
  r.mode = p.mode == LBM_MODE_AUTO ? (re_c >= 3000.0 ? 1 : 0) : (p.mode ? 1 : 0);
  k17_rates(r.omega1, p.omega2, r.k17);
  if (r.mode == 1) {
    // A and B carry 1/(omega1 - omega2), and the rates have poles of their
    // own; the third-order rates must be relaxation rates in (0, 2)
    bool ok = std::fabs(r.omega1 - p.omega2) >= 1e-3;
    for (int i = 0; i < 3; ++i) ok = ok && r.k17[i] > 0.0 && r.k17[i] < 2.0;
    ok = ok && std::isfinite(r.k17[3]) && std::isfinite(r.k17[4]);
    if (!ok)
      return fail(nullptr, LBM_EINVAL,
                  "fourth-order mode undefined at this omega1: needs |omega1 - omega2| >= 1e-3 and rates "
                  "omega3..5 in (0, 2)");
  }
  r.N = (int64_t)p.nx * p.ny * p.nz;
  r.slotp = (int64_t)p.nx + 64;
  r.rowp = 27 * r.slotp;
  r.zstride = r.rowp * (p.ny + 2);
  r.pop_elems = r.zstride * (p.nz + 2);
  if (3 * r.zstride * (int64_t)storage_size(p.storage) >= (int64_t(1) << 31) || r.N >= (int64_t(1) << 31))
    return fail(nullptr, LBM_EINVAL, "grid too large (three padded planes must stay below 2 GiB)");
  r.ntiles = (int64_t)(p.nx / TX) * (p.ny / TY) * p.nz;
  if (r.ntiles >= (int64_t(1) << 31)) return fail(nullptr, LBM_EINVAL, "too many tiles");
  return LBM_OK;
}

// Obstacle tables from the solid mask (host, once): boundary cells (fluid
// cells with a link into the obstacle) in ascending order with their link
// masks, the constant weight part of the momentum exchange, the solid-cell
// box and the force slot of every tile holding a boundary cell.
struct Tables {
  std::vector<int64_t> rcell;
  std::vector<uint32_t> rmask;
  double fc[3] = {0, 0, 0};
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {-1, -1, -1};
  std::vector<int32_t> bslot;
  int32_t nslots = 0;
};

static int build_tables(const lbm_params& p, const Resolved& r, const uint8_t* solid, Tables& t) {
  std::vector<uint64_t> pairs;  // (cell << 5) | j : cell + c_j is obstacle
  if (solid) {
    for (int64_t n = 0; n < r.N; ++n) {
      if (!solid[n]) continue;
      const int x = (int)(n % p.nx), y = (int)((n / p.nx) % p.ny), z = (int)(n / ((int64_t)p.nx * p.ny));
      t.lo[0] = std::min(t.lo[0], x); t.hi[0] = std::max(t.hi[0], x);
      t.lo[1] = std::min(t.lo[1], y); t.hi[1] = std::max(t.hi[1], y);
      t.lo[2] = std::min(t.lo[2], z); t.hi[2] = std::max(t.hi[2], z);
      if (!p.periodic[0] && (x < 3 || x > p.nx - 4))
        return fail(nullptr, LBM_EINVAL, "obstacle must keep 3 cells clear of inlet and outlet");
      for (int j = 0; j < 27; ++j) {
        if (j == 13) continue;
        int fx = x - cx(j), fy = y - cy(j), fz = z - cz(j);
        if (p.periodic[0]) fx = (fx + p.nx) % p.nx; else if (fx < 0 || fx >= p.nx) continue;
        if (p.periodic[1]) fy = (fy + p.ny) % p.ny; else if (fy < 0 || fy >= p.ny) continue;
        if (p.periodic[2]) fz = (fz + p.nz) % p.nz; else if (fz < 0 || fz >= p.nz) continue;
        const int64_t f = ((int64_t)fz * p.ny + fy) * p.nx + fx;
        if (solid[f]) continue;
        pairs.push_back(((uint64_t)f << 5) | (uint64_t)j);
      }
    }
  }
  std::sort(pairs.begin(), pairs.end());
  for (uint64_t pr : pairs) {
    const int64_t cell = (int64_t)(pr >> 5);
    const int j = (int)(pr & 31);
    if (t.rcell.empty() || t.rcell.back() != cell) {
      t.rcell.push_back(cell);
      t.rmask.push_back(0);
    }
    t.rmask.back() |= 1u << j;
    t.fc[0] += 2.0 * wgt(j) * cx(j);
    t.fc[1] += 2.0 * wgt(j) * cy(j);
    t.fc[2] += 2.0 * wgt(j) * cz(j);
  }
  const int tiles_x = p.nx / TX, tiles_y = p.ny / TY;
  if (p.force_every > 0 && !t.rcell.empty()) {
    t.bslot.assign((size_t)r.ntiles, -1);
    for (int64_t cell : t.rcell) {
      const int x = (int)(cell % p.nx), y = (int)((cell / p.nx) % p.ny), z = (int)(cell / ((int64_t)p.nx * p.ny));
      const int64_t tt = ((int64_t)z * tiles_y + y / TY) * tiles_x + x / TX;
      if (t.bslot[(size_t)tt] < 0) t.bslot[(size_t)tt] = t.nslots++;
    }
  }
  return LBM_OK;
}

// Device memory of one solver: one block carved into 256-byte aligned
// regions (populations, cell flags, boundary rows, link masks, wall
// distances, force slots and partials, FP64 accumulators, snapshot ring,
// force ring, stability flag).
struct Layout {
  size_t A = 0, A1 = 0, flag = 0, brow = 0, bmask = 0, bq = 0, bslot = 0, fpart = 0, acc = 0, snap = 0, forces = 0, chk = 0;
  size_t total = 0;
};

static Layout make_layout(const lbm_params& p, const Resolved& r, const Tables& t) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const int64_t nb = std::max<int64_t>((int64_t)t.rcell.size(), 1);
  // each lattice has a 256-byte guard in front: the probe's pull of the
  // corner cell reads one element before element 0 (inlet ghost of slot 0
  // in the guard row of the guard plane)
  (void)take(256);
  L.A = take((size_t)r.pop_elems * storage_size(p.storage));
  (void)take(256);
  L.A1 = take((size_t)r.pop_elems * storage_size(p.storage));
  L.flag = take((size_t)r.N);
  L.brow = take((size_t)r.N * 4);
  L.bmask = take((size_t)nb * 4);
  L.bq = take((size_t)nb * 27 * 8);
  L.bslot = take(t.nslots > 0 ? (size_t)r.ntiles * 4 : 0);
  L.fpart = take((size_t)t.nslots * 24);
  L.acc = take(p.avg_start >= 0 ? (size_t)r.N * 32 : 0);
  L.snap = take(p.snap_every > 0 ? (size_t)p.snap_count * r.N * 16 : 0);
  L.forces = take(p.force_capacity > 0 && t.nslots > 0 ? (size_t)p.force_capacity * 24 : 0);
  L.chk = take(4);
  L.total = off;
  return L;
}

extern "C" int lbm_workspace_size(const lbm_params* pin, const uint8_t* solid, size_t* bytes) {
  if (!pin || !bytes) return fail(nullptr, LBM_EINVAL, "null argument");
  Resolved r;
  int rc = resolve(*pin, r);
  if (rc) return rc;
  Tables t;
  if ((rc = build_tables(*pin, r, solid, t))) return rc;
  *bytes = make_layout(*pin, r, t).total;
  return LBM_OK;
}

extern "C" int lbm_create_in(const lbm_params* pin, const uint8_t* solid, int64_t nlinks, const int64_t* link_cell,
                             const uint8_t* link_dir, const double* link_q, const double* u0, void* d_workspace,
                             size_t workspace_bytes, void* hip_stream, lbm_sim** out) {
  if (!pin || !out) return fail(nullptr, LBM_EINVAL, "null argument");
  *out = nullptr;
  const lbm_params& p = *pin;
  Resolved r;
  int rc = resolve(p, r);
  if (rc) return rc;
  if (nlinks < 0 || (nlinks > 0 && (!link_cell || !link_dir || !link_q)))
    return fail(nullptr, LBM_EINVAL, "bad link arrays");
  if (d_workspace && ((uintptr_t)d_workspace & 255))
    return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
  Tables t;
  if ((rc = build_tables(p, r, solid, t))) return rc;
  if (d_workspace && p.force_every > 0 && !t.rcell.empty() && p.force_capacity <= 0)
    return fail(nullptr, LBM_EINVAL, "a caller workspace needs force_capacity > 0 (the force series is a ring in it)");
  const Layout lay = make_layout(p, r, t);
  if (d_workspace && workspace_bytes < lay.total)
    return fail(nullptr, LBM_EINVAL, "workspace smaller than lbm_workspace_size");
  const int64_t N = r.N;

  lbm_sim* s = new (std::nothrow) lbm_sim();
  if (!s) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
  s->p = p;
  s->p.nu = r.nu;
  s->N = N;
  s->esize = storage_size(p.storage);
  s->stream = (hipStream_t)hip_stream;
  s->omega1 = r.omega1;
  s->mode = r.mode;
  (void)hipGetDevice(&s->device);
  auto bail = [&](int code) {
    free_all(s);
    delete s;
    return code;
  };

  s->nb = (int64_t)t.rcell.size();
  std::vector<double> rq((size_t)std::max<int64_t>(s->nb, 1) * 27, 0.5);
  for (int64_t k = 0; k < nlinks; ++k) {
    const int64_t cell = link_cell[k];
    const int j = link_dir[k];
    if (j < 0 || j >= 27 || cell < 0 || cell >= N) {
      fail(nullptr, LBM_EINVAL, "link out of range");
      return bail(LBM_EINVAL);
    }
    const double q = link_q[k];
    if (!(q > 0.0 && q <= 1.0)) {
      fail(nullptr, LBM_EINVAL, "wall distance fraction must be in (0, 1]");
      return bail(LBM_EINVAL);
    }
    auto it = std::lower_bound(t.rcell.begin(), t.rcell.end(), cell);
    if (it != t.rcell.end() && *it == cell) rq[(size_t)(it - t.rcell.begin()) * 27 + j] = q;
  }
  for (int d = 0; d < 3; ++d) s->fconst[d] = t.fc[d];
  s->nslots = t.nslots;

  // ---- device memory: one block, the caller's or the library's ----
  hipError_t e = hipSuccess;
  if (d_workspace) {
    s->block = (char*)d_workspace;
    s->owns_block = false;
  } else {
    if ((e = hipMalloc((void**)&s->block, lay.total)) != hipSuccess) {
      fail(nullptr, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "device allocation failed");
      return bail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE);
    }
    s->owns_block = true;
  }
  if ((e = hipHostMalloc((void**)&s->h_chk, sizeof(int32_t), hipHostMallocDefault)) != hipSuccess) {
    fail(nullptr, LBM_ENOMEM, "pinned host allocation failed");
    return bail(LBM_ENOMEM);
  }
  *s->h_chk = 0;
  char* B = s->block;
  s->arr[0] = B + lay.A;
  s->arr[1] = B + lay.A1;
  s->cur = 0;
  s->natural = true;
  s->pop_elems = r.pop_elems;
  s->d_flag = (uint8_t*)(B + lay.flag);
  s->d_brow = (int32_t*)(B + lay.brow);
  s->d_bmask = (uint32_t*)(B + lay.bmask);
  s->d_bq = (double*)(B + lay.bq);
  s->d_bslot = s->nslots > 0 ? (int32_t*)(B + lay.bslot) : nullptr;
  s->d_fpart = s->nslots > 0 ? (double*)(B + lay.fpart) : nullptr;
  s->d_acc = p.avg_start >= 0 ? (double*)(B + lay.acc) : nullptr;
  s->d_snap = p.snap_every > 0 ? (float*)(B + lay.snap) : nullptr;
  s->d_chk = (int32_t*)(B + lay.chk);
  if (p.force_capacity > 0 && s->nslots > 0) {
    s->force_ring = true;
    s->d_forces = (double*)(B + lay.forces);
    s->force_cap = p.force_capacity;
  }
  auto dalloc = [&](void** ptr, size_t bytes) -> bool {
    hipError_t ee = hipMalloc(ptr, bytes);
    if (ee != hipSuccess) {
      fail(nullptr, ee == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "device allocation failed");
      return false;
    }
    return true;
  };
  hipStream_t st = s->stream;
  (void)hipMemsetAsync(s->arr[0], 0, (size_t)r.pop_elems * s->esize, st);
  (void)hipMemsetAsync(s->arr[1], 0, (size_t)r.pop_elems * s->esize, st);
  (void)hipMemsetAsync(s->d_brow, 0xff, (size_t)N * 4, st);
  (void)hipMemsetAsync(s->d_chk, 0, sizeof(int32_t), st);
  if (solid) {
    // flags: 2 solid, 0 fluid; the scatter kernel below marks boundary rows 1
    std::vector<uint8_t> fl(solid, solid + N);
    for (auto& v : fl) v = v ? 2 : 0;
    (void)hipMemcpyAsync(s->d_flag, fl.data(), (size_t)N, hipMemcpyHostToDevice, st);
    (void)hipStreamSynchronize(st);
  } else {
    (void)hipMemsetAsync(s->d_flag, 0, (size_t)N, st);
  }
  if (s->nb > 0) {
    int64_t* d_cells = nullptr;
    if (!dalloc((void**)&d_cells, (size_t)s->nb * 8)) return bail(LBM_ENOMEM);
    (void)hipMemcpyAsync(d_cells, t.rcell.data(), (size_t)s->nb * 8, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(s->d_bmask, t.rmask.data(), (size_t)s->nb * 4, hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(s->d_bq, rq.data(), (size_t)s->nb * 27 * 8, hipMemcpyHostToDevice, st);
    hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((s->nb + 255) / 256)), dim3(256), 0, st, d_cells, s->nb,
                       s->d_flag, s->d_brow);
    (void)hipStreamSynchronize(st);
    (void)hipFree(d_cells);
  }
  if (s->nslots > 0)
    (void)hipMemcpyAsync(s->d_bslot, t.bslot.data(), (size_t)r.ntiles * 4, hipMemcpyHostToDevice, st);
  if (s->d_acc) (void)hipMemsetAsync(s->d_acc, 0, (size_t)N * 32, st);
  if (s->d_snap) (void)hipMemsetAsync(s->d_snap, 0, (size_t)p.snap_count * N * 16, st);

  StepArgs& a = s->args;
  a.A = s->arr[0];
  a.B = s->arr[1];
  a.nx = p.nx; a.ny = p.ny; a.nz = p.nz;
  a.slotp = (int32_t)r.slotp;
  a.rowp = (int32_t)r.rowp;
  a.zstride = (int32_t)r.zstride;
  for (int d = 0; d < 3; ++d) a.per[d] = p.periodic[d] ? 1 : 0;
  a.flag = s->d_flag;
  a.brow = s->d_brow;
  a.bmask = s->d_bmask;
  a.bq = s->d_bq;
  a.interp = p.obstacle_bc == 1 ? 1 : 0;
  fill_coef(s->coefs.f, s->omega1, p.omega2, p.galilean, p.lambda, r.k17, p.body_force, p.u_in);
  fill_coef(s->coefs.d, s->omega1, p.omega2, p.galilean, p.lambda, r.k17, p.body_force, p.u_in);
  a.acc = nullptr;
  a.snap = nullptr;
  a.bslot = nullptr;
  a.chk = nullptr;
  a.fpart = s->d_fpart;
  a.tiles_x = p.nx / TX;
  a.tiles_y = p.ny / TY;
  a.ntiles = (int32_t)r.ntiles;
  a.remap = p.xcd_remap ? 1 : 0;
  // tile box around the obstacle: solid cells dilated by two cells (their
  // fluid neighbours and the cells behind them); on a periodic axis a box
  // that reaches a face covers the whole axis
  if (t.hi[0] < 0) {
    a.obox[0] = 1; a.obox[1] = 0; a.obox[2] = 1; a.obox[3] = 0; a.obox[4] = 1; a.obox[5] = 0;
  } else {
    const int ext[3] = {p.nx, p.ny, p.nz}, tsz[3] = {TX, TY, 1};
    for (int d = 0; d < 3; ++d) {
      int b0 = t.lo[d] - 2, b1 = t.hi[d] + 2;
      if (p.periodic[d] && (b0 < 0 || b1 > ext[d] - 1)) {
        b0 = 0;
        b1 = ext[d] - 1;
      }
      b0 = std::max(b0, 0);
      b1 = std::min(b1, ext[d] - 1);
      a.obox[2 * d] = b0 / tsz[d];
      a.obox[2 * d + 1] = b1 / tsz[d];
    }
  }
  a.perturb_seed = p.perturb_seed;
  a.perturb_amp = p.perturb_amp;

  double* d_u0 = nullptr;
  if (u0) {
    if (!dalloc((void**)&d_u0, (size_t)N * 24)) return bail(LBM_ENOMEM);
    (void)hipMemcpyAsync(d_u0, u0, (size_t)N * 24, hipMemcpyHostToDevice, st);
  }
  launch_init(p.storage, a, d_u0, s->arr[0], st);
  e = hipStreamSynchronize(st);
  if (d_u0) (void)hipFree(d_u0);
  if (e != hipSuccess || (e = hipGetLastError()) != hipSuccess) {
    fail(nullptr, LBM_EDEVICE, std::string("initialisation failed: ") + hipGetErrorString(e));
    return bail(LBM_EDEVICE);
  }
  *out = s;
  return LBM_OK;
}

extern "C" int lbm_create(const lbm_params* p, const uint8_t* solid, int64_t nlinks, const int64_t* link_cell,
                          const uint8_t* link_dir, const double* link_q, const double* u0, void* hip_stream,
                          lbm_sim** out) {
  return lbm_create_in(p, solid, nlinks, link_cell, link_dir, link_q, u0, nullptr, 0, hip_stream, out);
}

static int ensure_force_cap(lbm_sim* s, int64_t need) {
  if (s->force_ring || need <= s->force_cap) return LBM_OK;
  int64_t cap = std::max<int64_t>(need, 2 * s->force_cap);
  cap = std::max<int64_t>(cap, 1024);
  double* nb = nullptr;
  HIPCHK(s, hipMalloc(&nb, (size_t)cap * 24));
  if (s->d_forces) {
    HIPCHK(s, hipMemcpyAsync(nb, s->d_forces, (size_t)s->nforces * 24, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    (void)hipFree(s->d_forces);
  }
  s->d_forces = nb;
  s->force_cap = cap;
  return LBM_OK;
}

// Kernel arguments reading the current state (A) and writing the other
// lattice (B).
static StepArgs state_args(const lbm_sim* s) {
  StepArgs a = s->args;
  a.A = s->arr[s->cur];
  a.B = s->arr[s->cur ^ 1];
  return a;
}

// Stability state: the flag a check step set, as last copied to the host.
static int unstable(lbm_sim* s) {
  if (s->h_chk && *(volatile int32_t*)s->h_chk)
    return fail(s, LBM_EUNSTABLE, "a check step found a cell with non-finite, out-of-range density or velocity");
  return LBM_OK;
}

static int guard(lbm_sim* s) {
  if (s->sticky) return s->sticky;
  return unstable(s);
}

// One time step of the method (paper Sec. 3.1-3.2: stream and collide with
// the channel's boundary rules; Sec. 2: mean fields, snapshots, forces).
extern "C" int lbm_step(lbm_sim* s, int64_t nsteps) {
  if (!s) return fail(nullptr, LBM_EINVAL, "null object");
  if (int rc = guard(s)) return rc;
  if (nsteps < 0) return fail(s, LBM_EINVAL, "negative step count");
  const lbm_params& p = s->p;
  if (p.force_every > 0 && s->nslots > 0) {
    const int64_t due = (s->steps + nsteps + p.force_every - 1) / p.force_every - (s->steps + p.force_every - 1) / p.force_every;
    int rc = ensure_force_cap(s, s->nforces + due + 1);
    if (rc) return rc;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t n = s->steps;
    StepArgs a = state_args(s);
    if (s->d_acc && n >= p.avg_start) {
      a.acc = s->d_acc;
      s->nsamples++;
    }
    if (s->d_snap && n >= p.snap_start && (n - p.snap_start) % p.snap_every == 0) {
      const int64_t slotk = s->snap_taken % p.snap_count;
      a.snap = s->d_snap + slotk * 4 * s->N;
      if ((int64_t)s->snap_steps.size() < p.snap_count) s->snap_steps.push_back(n);
      else s->snap_steps[(size_t)slotk] = n;
      s->snap_taken++;
    }
    const bool do_force = p.force_every > 0 && s->nslots > 0 && n % p.force_every == 0;
    if (do_force) a.bslot = s->d_bslot;
    const bool do_chk = p.check_every > 0 && (n + 1) % p.check_every == 0;
    if (do_chk) a.chk = s->d_chk;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s->profiling) {
      HIPCHK(s, hipEventCreate(&e0));
      HIPCHK(s, hipEventCreate(&e1));
      HIPCHK(s, hipEventRecord(e0, s->stream));
    }
    launch_step_any(p.storage, a, s->coefs, s->natural, s->mode, s->stream);
    if (s->profiling) {
      HIPCHK(s, hipEventRecord(e1, s->stream));
      s->events.emplace_back(e0, e1);
    }
    if (do_chk)
      HIPCHK(s, hipMemcpyAsync(s->h_chk, s->d_chk, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream));
    if (do_force) {
      const int64_t slot = s->force_ring ? s->nforces % s->force_cap : s->nforces;
      hipLaunchKernelGGL(force_reduce_kernel, dim3(1), dim3(256), 0, s->stream, s->d_fpart, s->nslots, s->fconst[0],
                         s->fconst[1], s->fconst[2], s->d_forces + 3 * slot);
      if (s->force_ring && (int64_t)s->force_steps.size() == s->force_cap) s->force_steps[(size_t)slot] = n;
      else s->force_steps.push_back(n);
      s->nforces++;
    }
    s->steps++;
    s->cur ^= 1;
    s->natural = false;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s, LBM_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  }
  return LBM_OK;
}

extern "C" int lbm_mean_fields(lbm_sim* s, double* out, int out_on_device, int64_t* nsamples) {
  if (!s || !out) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  if (!s->d_acc) return fail(s, LBM_ESTATE, "averaging is off (avg_start < 0)");
  const int64_t N = s->N;
  double* dst = out;
  double* tmp = nullptr;
  if (!out_on_device) {
    HIPCHK(s, hipMalloc(&tmp, (size_t)N * 32));
    dst = tmp;
  }
  const double inv = s->nsamples > 0 ? 1.0 / (double)s->nsamples : 0.0;
  hipLaunchKernelGGL(mean_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s->stream, s->d_acc, N, inv,
                     s->d_flag, dst);
  if (tmp) {
    HIPCHK(s, hipMemcpyAsync(out, tmp, (size_t)N * 32, hipMemcpyDeviceToHost, s->stream));
  }
  hipError_t e = hipStreamSynchronize(s->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  if (nsamples) *nsamples = s->nsamples;
  return LBM_OK;
}

extern "C" int lbm_mean_fields_pooled(lbm_sim* s, int32_t factor, int32_t quarter_turns, float* d_out) {
  if (!s || !d_out) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  if (!s->d_acc) return fail(s, LBM_ESTATE, "averaging is off (avg_start < 0)");
  const int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
  if (factor < 1 || nx % factor || ny % factor || nz % factor)
    return fail(s, LBM_EINVAL, "pooling factor must divide nx, ny and nz");
  if (quarter_turns < 0 || quarter_turns > 3) return fail(s, LBM_EINVAL, "quarter_turns must be 0..3");
  if (quarter_turns && ny != nz) return fail(s, LBM_EINVAL, "turns about x need ny == nz");
  const int X = nx / factor, Y = ny / factor, Z = nz / factor;
  const int64_t P = (int64_t)X * Y * Z;
  const double inv = s->nsamples > 0 ? 1.0 / (double)s->nsamples : 0.0;
  hipLaunchKernelGGL(pool_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s->stream, s->d_acc, s->N, inv,
                     s->d_flag, nx, ny, (int)factor, X, Y, Z, (int)quarter_turns, d_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int lbm_snapshots(lbm_sim* s, float* out, int out_on_device, int32_t* k, int64_t* steps) {
  if (!s || !k) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  const int64_t taken = s->snap_taken;
  const int64_t cnt = std::min<int64_t>(taken, s->p.snap_count);
  *k = (int32_t)cnt;
  if (!out || cnt == 0) return LBM_OK;
  const size_t one = (size_t)s->N * 16;
  const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int64_t j = 0; j < cnt; ++j) {
    const int64_t idx = taken - cnt + j;
    const int64_t slotk = idx % s->p.snap_count;
    HIPCHK(s, hipMemcpyAsync((char*)out + j * one, (char*)s->d_snap + slotk * one, one, kind, s->stream));
    if (steps) steps[j] = s->snap_steps[(size_t)slotk];
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return LBM_OK;
}

extern "C" int lbm_forces(lbm_sim* s, double* fxyz, int64_t cap, int64_t* n, int64_t* steps) {
  if (!s || !n) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  // retained samples: all of them, or the last force_cap of a ring
  const int64_t kept = s->force_ring ? std::min(s->nforces, s->force_cap) : s->nforces;
  const int64_t first = s->nforces - kept;  // sample index of the oldest kept
  *n = kept;
  const int64_t m = std::min(cap, kept);
  if (fxyz && m > 0) {
    int64_t j = 0;
    while (j < m) {
      // contiguous run of ring slots starting at the slot of sample first + j
      const int64_t slot = s->force_ring ? (first + j) % s->force_cap : first + j;
      const int64_t run = std::min(m - j, s->force_ring ? s->force_cap - slot : m - j);
      HIPCHK(s, hipMemcpyAsync(fxyz + 3 * j, s->d_forces + 3 * slot, (size_t)run * 24, hipMemcpyDeviceToHost,
                               s->stream));
      j += run;
    }
    HIPCHK(s, hipStreamSynchronize(s->stream));
  }
  if (steps)
    for (int64_t j = 0; j < m; ++j)
      steps[j] = s->force_steps[(size_t)(s->force_ring ? (first + j) % s->force_cap : first + j)];
  return LBM_OK;
}

extern "C" int lbm_moments(lbm_sim* s, float* out, int out_on_device) {
  if (!s || !out) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  float* dst = out;
  float* tmp = nullptr;
  if (!out_on_device) {
    HIPCHK(s, hipMalloc(&tmp, (size_t)s->N * 16));
    dst = tmp;
  }
  launch_export(s->p.storage, state_args(s), s->coefs, s->natural, nullptr, dst, nullptr, s->stream);
  if (tmp) HIPCHK(s, hipMemcpyAsync(out, tmp, (size_t)s->N * 16, hipMemcpyDeviceToHost, s->stream));
  hipError_t e = hipStreamSynchronize(s->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int lbm_get_populations(lbm_sim* s, double* fbar) {
  if (!s || !fbar) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  double* tmp = nullptr;
  HIPCHK(s, hipMalloc(&tmp, (size_t)s->N * 27 * 8));
  launch_export(s->p.storage, state_args(s), s->coefs, s->natural, tmp, nullptr, nullptr, s->stream);
  hipError_t e = hipMemcpyAsync(fbar, tmp, (size_t)s->N * 27 * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int lbm_get_populations_box(lbm_sim* s, int32_t x0, int32_t y0, int32_t z0, int32_t bx, int32_t by,
                                       int32_t bz, double* fbar) {
  if (!s || !fbar) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  if (bx <= 0 || by <= 0 || bz <= 0 || x0 < 0 || y0 < 0 || z0 < 0 || x0 > s->p.nx - bx || y0 > s->p.ny - by ||
      z0 > s->p.nz - bz)
    return fail(s, LBM_EINVAL, "box outside the grid");
  const int64_t nb = (int64_t)bx * by * bz;
  double* tmp = nullptr;
  HIPCHK(s, hipMalloc(&tmp, (size_t)nb * 27 * 8));
  const int box[6] = {x0, y0, z0, bx, by, bz};
  switch (s->p.storage) {
    case LBM_F64: launch_export_box_s<double>(state_args(s), s->coefs, s->natural, box, tmp, s->stream); break;
    case LBM_F32: launch_export_box_s<float>(state_args(s), s->coefs, s->natural, box, tmp, s->stream); break;
    case LBM_F16S: launch_export_box_s<f16s>(state_args(s), s->coefs, s->natural, box, tmp, s->stream); break;
    case LBM_BF16S: launch_export_box_s<bf16s>(state_args(s), s->coefs, s->natural, box, tmp, s->stream); break;
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(fbar, tmp, (size_t)nb * 27 * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int lbm_set_populations(lbm_sim* s, const double* fbar) {
  if (!s || !fbar) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  double* tmp = nullptr;
  HIPCHK(s, hipMalloc(&tmp, (size_t)s->N * 27 * 8));
  hipError_t e = hipMemcpyAsync(tmp, fbar, (size_t)s->N * 27 * 8, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) {
    launch_import(s->p.storage, s->args, tmp, s->arr[s->cur], s->stream);
    e = hipStreamSynchronize(s->stream);
  }
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  s->natural = true;
  return LBM_OK;
}

extern "C" int lbm_mass(lbm_sim* s, double* mass) {
  if (!s || !mass) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  double* part = nullptr;
  const int nt = s->args.ntiles;
  HIPCHK(s, hipMalloc(&part, (size_t)nt * 8));
  launch_export(s->p.storage, state_args(s), s->coefs, s->natural, nullptr, nullptr, part, s->stream);
  std::vector<double> h((size_t)nt);
  hipError_t e = hipMemcpyAsync(h.data(), part, (size_t)nt * 8, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(part);
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  double m = 0.0;
  for (double v : h) m += v;
  *mass = m;
  if (!std::isfinite(m)) return fail(s, LBM_EUNSTABLE, "non-finite mass: the run is unstable");
  return LBM_OK;
}

// checkpoint blob: header, raw populations, accumulators, snapshots, forces
struct Blob {
  char magic[8];
  int32_t nx, ny, nz, storage;
  int64_t steps, nsamples, snap_taken, nforces, natural;
  int64_t popbytes, accbytes, snapbytes;
  int64_t fstored;  // force slots stored: every sample, or the ring's filled slots in slot order
};

extern "C" int lbm_export_state(lbm_sim* s, void* blob, size_t cap, size_t* used) {
  if (!s || !used) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  Blob h{};
  std::memcpy(h.magic, "MLBMCKP3", 8);
  h.nx = s->p.nx; h.ny = s->p.ny; h.nz = s->p.nz; h.storage = s->p.storage;
  h.steps = s->steps; h.nsamples = s->nsamples; h.snap_taken = s->snap_taken; h.nforces = s->nforces;
  h.natural = s->natural ? 1 : 0;
  h.popbytes = (int64_t)(s->pop_elems * (int64_t)s->esize);
  h.accbytes = s->d_acc ? s->N * 32 : 0;
  h.snapbytes = s->d_snap ? (int64_t)s->p.snap_count * s->N * 16 : 0;
  h.fstored = (int64_t)s->force_steps.size();
  const size_t need = sizeof(Blob) + h.popbytes + h.accbytes + h.snapbytes + (size_t)h.fstored * 32 +
                      s->snap_steps.size() * 8 + 8;
  *used = need;
  if (!blob) return LBM_OK;
  if (cap < need) return fail(s, LBM_EINVAL, "checkpoint buffer too small");
  char* b = (char*)blob;
  std::memcpy(b, &h, sizeof h);
  b += sizeof h;
  HIPCHK(s, hipMemcpyAsync(b, s->arr[s->cur], (size_t)h.popbytes, hipMemcpyDeviceToHost, s->stream));
  b += h.popbytes;
  if (h.accbytes) HIPCHK(s, hipMemcpyAsync(b, s->d_acc, (size_t)h.accbytes, hipMemcpyDeviceToHost, s->stream));
  b += h.accbytes;
  if (h.snapbytes) HIPCHK(s, hipMemcpyAsync(b, s->d_snap, (size_t)h.snapbytes, hipMemcpyDeviceToHost, s->stream));
  b += h.snapbytes;
  if (h.fstored) HIPCHK(s, hipMemcpyAsync(b, s->d_forces, (size_t)h.fstored * 24, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  b += h.fstored * 24;
  std::memcpy(b, s->force_steps.data(), (size_t)h.fstored * 8);
  b += h.fstored * 8;
  int64_t nss = (int64_t)s->snap_steps.size();
  std::memcpy(b, &nss, 8);
  b += 8;
  std::memcpy(b, s->snap_steps.data(), (size_t)nss * 8);
  return LBM_OK;
}

extern "C" int lbm_import_state(lbm_sim* s, const void* blob, size_t n) {
  if (!s || !blob) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  if (n < sizeof(Blob)) return fail(s, LBM_EINVAL, "checkpoint too short");
  Blob h;
  std::memcpy(&h, blob, sizeof h);
  if (std::memcmp(h.magic, "MLBMCKP3", 8) || h.nx != s->p.nx || h.ny != s->p.ny || h.nz != s->p.nz ||
      h.storage != s->p.storage)
    return fail(s, LBM_EINVAL, "checkpoint does not match this object");
  const int64_t popbytes = (int64_t)(s->pop_elems * (int64_t)s->esize);
  if (h.popbytes != popbytes || h.accbytes != (s->d_acc ? s->N * 32 : 0) ||
      h.snapbytes != (s->d_snap ? (int64_t)s->p.snap_count * s->N * 16 : 0))
    return fail(s, LBM_EINVAL, "checkpoint layout does not match this object");
  const char* b = (const char*)blob + sizeof h;
  if (h.fstored < 0 || (s->force_ring && h.fstored > s->force_cap) || (!s->force_ring && h.fstored != h.nforces))
    return fail(s, LBM_EINVAL, "checkpoint force series does not match this object");
  size_t need = sizeof(Blob) + h.popbytes + h.accbytes + h.snapbytes + (size_t)h.fstored * 32 + 8;
  if (n < need) return fail(s, LBM_EINVAL, "checkpoint truncated");
  HIPCHK(s, hipMemcpyAsync(s->arr[0], b, (size_t)h.popbytes, hipMemcpyHostToDevice, s->stream));
  b += h.popbytes;
  if (h.accbytes) HIPCHK(s, hipMemcpyAsync(s->d_acc, b, (size_t)h.accbytes, hipMemcpyHostToDevice, s->stream));
  b += h.accbytes;
  if (h.snapbytes) HIPCHK(s, hipMemcpyAsync(s->d_snap, b, (size_t)h.snapbytes, hipMemcpyHostToDevice, s->stream));
  b += h.snapbytes;
  if (h.fstored) {
    int rc = ensure_force_cap(s, h.fstored + 1);
    if (rc) return rc;
    HIPCHK(s, hipMemcpyAsync(s->d_forces, b, (size_t)h.fstored * 24, hipMemcpyHostToDevice, s->stream));
  }
  b += h.fstored * 24;
  s->force_steps.assign((const int64_t*)b, (const int64_t*)b + h.fstored);
  b += h.fstored * 8;
  int64_t nss;
  std::memcpy(&nss, b, 8);
  b += 8;
  if (n < need + (size_t)nss * 8) return fail(s, LBM_EINVAL, "checkpoint truncated");
  s->snap_steps.assign((const int64_t*)b, (const int64_t*)b + nss);
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->steps = h.steps; s->nsamples = h.nsamples; s->snap_taken = h.snap_taken; s->nforces = h.nforces;
  s->cur = 0;
  s->natural = h.natural != 0;
  return LBM_OK;
}

extern "C" int lbm_info(const lbm_sim* s, int64_t* steps, double* omega1, int32_t* mode) {
  if (!s) return LBM_EINVAL;
  if (steps) *steps = s->steps;
  if (omega1) *omega1 = s->omega1;
  if (mode) *mode = s->mode;
  return LBM_OK;
}

extern "C" int lbm_profile(lbm_sim* s, int enable) {
  if (!s) return LBM_EINVAL;
  s->profiling = enable != 0;
  return LBM_OK;
}

extern "C" int lbm_profile_read(lbm_sim* s, double* total_ms, int64_t* launches) {
  if (!s) return LBM_EINVAL;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (auto& e : s->events) {
    float ms = 0.f;
    HIPCHK(s, hipEventElapsedTime(&ms, e.first, e.second));
    s->prof_ms += ms;
    s->prof_launches++;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  s->events.clear();
  if (total_ms) *total_ms = s->prof_ms;
  if (launches) *launches = s->prof_launches;
  s->prof_ms = 0;
  s->prof_launches = 0;
  return LBM_OK;
}

extern "C" int lbm_bandwidth_probe(lbm_sim* s, int32_t passes, double* ms_per_pass) {
  if (!s || !ms_per_pass) return fail(s, LBM_EINVAL, "null argument");
  if (int rc = guard(s)) return rc;
  if (passes <= 0 || passes % 2) return fail(s, LBM_EINVAL, "passes must be positive and even");
  const StepArgs a = state_args(s);
  hipEvent_t e0, e1;
  HIPCHK(s, hipEventCreate(&e0));
  HIPCHK(s, hipEventCreate(&e1));
  HIPCHK(s, hipEventRecord(e0, s->stream));
  for (int i = 0; i < passes; ++i) {
    switch (s->p.storage) {
      case LBM_F64: hipLaunchKernelGGL(pull_probe_kernel<double>, dim3(a.ntiles), dim3(NTHREADS), 0, s->stream, a); break;
      case LBM_F32: hipLaunchKernelGGL(pull_probe_kernel<float>, dim3(a.ntiles), dim3(NTHREADS), 0, s->stream, a); break;
      case LBM_F16S: hipLaunchKernelGGL(pull_probe_kernel<f16s>, dim3(a.ntiles), dim3(NTHREADS), 0, s->stream, a); break;
      default: hipLaunchKernelGGL(pull_probe_kernel<bf16s>, dim3(a.ntiles), dim3(NTHREADS), 0, s->stream, a); break;
    }
  }
  HIPCHK(s, hipEventRecord(e1, s->stream));
  HIPCHK(s, hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(s, LBM_EDEVICE, hipGetErrorString(e));
  *ms_per_pass = (double)ms / passes;
  return LBM_OK;
}

extern "C" int lbm_copy_bandwidth(int64_t bytes, int32_t passes, void* hip_stream, double* ms_per_pass) {
  if (!ms_per_pass || bytes <= 0 || bytes % 16 || passes <= 0)
    return fail(nullptr, LBM_EINVAL, "bytes must be a positive multiple of 16, passes positive");
  const int64_t n4 = bytes / 16;
  if ((n4 + 255) / 256 > 0x7fffffff) return fail(nullptr, LBM_EINVAL, "copy too large");
  const hipStream_t st = (hipStream_t)hip_stream;
  void *a = nullptr, *b = nullptr;
  hipError_t e = hipMalloc(&a, (size_t)bytes);
  if (e == hipSuccess) e = hipMalloc(&b, (size_t)bytes);
  if (e != hipSuccess) {
    if (a) (void)hipFree(a);
    return fail(nullptr, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, hipGetErrorString(e));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const dim3 grid((unsigned)((n4 + 255) / 256));
  e = hipMemsetAsync(a, 0, (size_t)bytes, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    for (int w = 0; w < 2; ++w)
      hipLaunchKernelGGL(copy_probe_kernel, grid, dim3(256), 0, st, (const float4_v*)a, (float4_v*)b, n4);
    e = hipEventRecord(e0, st);
  }
  if (e == hipSuccess) {
    for (int i = 0; i < passes; ++i)
      hipLaunchKernelGGL(copy_probe_kernel, grid, dim3(256), 0, st, (const float4_v*)a, (float4_v*)b, n4);
    e = hipEventRecord(e1, st);
  }
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, hipGetErrorString(e));
  *ms_per_pass = (double)ms / passes;
  return LBM_OK;
}

extern "C" void lbm_destroy(lbm_sim* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_all(s);
  delete s;
}

extern "C" const char* lbm_last_error(const lbm_sim* s) { return s ? s->err.c_str() : g_err.c_str(); }
