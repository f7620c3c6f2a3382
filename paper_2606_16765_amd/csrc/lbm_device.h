// Device-side building blocks of the D3Q27 cumulant stream-and-collide step
// for gfx950: storage conversion, the lattice, the well-conditioned central-
// moment transform and the cumulant collision (paper Sec. 3.2, D3Q27
// cumulant operator; fourth-order parametrised mode with limiter).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlbm {

// ---------------------------------------------------------------- storage
// Shifted populations fbar = f - w_i are stored as S; arithmetic runs in T.
struct f16s { uint16_t bits; };
struct bf16s { uint16_t bits; };

template <typename S> struct Storage;
// load/store take the value streamed once per step; the _nt forms may add
// the non-temporal hint (the populations are not reused within a step).
// Measured on MI355X: for 32- and 64-bit storage the hint pays on stores
// and not on loads; 16-bit storage uses it on both.
#ifndef MLBM_NT_LOAD
#define MLBM_NT_LOAD 0
#endif
#ifndef MLBM_NT_STORE
#define MLBM_NT_STORE 1
#endif
template <> struct Storage<double> {
  using T = double;
  static __device__ __forceinline__ double load(const double* p) { return *p; }
  static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
  static __device__ __forceinline__ double load_nt(const double* p) { return MLBM_NT_LOAD ? __builtin_nontemporal_load(p) : *p; }
  static __device__ __forceinline__ void store_nt(double* p, double v) {
    if (MLBM_NT_STORE) __builtin_nontemporal_store(v, p); else *p = v;
  }
};
template <> struct Storage<float> {
  using T = float;
  static __device__ __forceinline__ float load(const float* p) { return *p; }
  static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
  static __device__ __forceinline__ float load_nt(const float* p) { return MLBM_NT_LOAD ? __builtin_nontemporal_load(p) : *p; }
  static __device__ __forceinline__ void store_nt(float* p, float v) {
    if (MLBM_NT_STORE) __builtin_nontemporal_store(v, p); else *p = v;
  }
};
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
// v_cvt_f16_f32 rounds to nearest even in the default mode
__device__ __forceinline__ uint16_t f32_to_f16(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// v_cvt_pk_bf16_f32 rounds to nearest even; a NaN stays a (quiet) NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
template <> struct Storage<f16s> {
  using T = float;
  static __device__ __forceinline__ float load(const f16s* p) { return f16_to_f32(*(const uint16_t*)p); }
  static __device__ __forceinline__ void store(f16s* p, float v) { *(uint16_t*)p = f32_to_f16(v); }
  static __device__ __forceinline__ float load_nt(const f16s* p) {
    return f16_to_f32(__builtin_nontemporal_load((const uint16_t*)p));
  }
  static __device__ __forceinline__ void store_nt(f16s* p, float v) {
    __builtin_nontemporal_store(f32_to_f16(v), (uint16_t*)p);
  }
};
template <> struct Storage<bf16s> {
  using T = float;
  static __device__ __forceinline__ float load(const bf16s* p) { return bf16_to_f32(*(const uint16_t*)p); }
  static __device__ __forceinline__ void store(bf16s* p, float v) { *(uint16_t*)p = f32_to_bf16(v); }
  static __device__ __forceinline__ float load_nt(const bf16s* p) {
    return bf16_to_f32(__builtin_nontemporal_load((const uint16_t*)p));
  }
  static __device__ __forceinline__ void store_nt(bf16s* p, float v) {
    __builtin_nontemporal_store(f32_to_bf16(v), (uint16_t*)p);
  }
};

// ---------------------------------------------------------------- lattice
__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wgt(int i) { return w1d(cx(i)) * w1d(cy(i)) * w1d(cz(i)); }
// rest-state central moment of one axis at order a: 1, 0, 1/3
__host__ __device__ constexpr double rest1d(int a) { return a == 0 ? 1.0 : (a == 1 ? 0.0 : 1.0 / 3.0); }

// bit masks of directions by velocity component
__host__ __device__ constexpr uint32_t mask_of(int axis, int v) {
  uint32_t m = 0;
  for (int i = 0; i < 27; ++i) {
    int c = axis == 0 ? cx(i) : (axis == 1 ? cy(i) : cz(i));
    if (c == v) m |= 1u << i;
  }
  return m;
}
constexpr uint32_t M_XP = mask_of(0, 1), M_XN = mask_of(0, -1);
constexpr uint32_t M_YP = mask_of(1, 1), M_YN = mask_of(1, -1);
constexpr uint32_t M_ZP = mask_of(2, 1), M_ZN = mask_of(2, -1);

__device__ __forceinline__ uint32_t reverse27(uint32_t m) { return __builtin_bitreverse32(m) >> 5; }

template <typename T> __device__ __forceinline__ T fast_rcp(T x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }

// ------------------------------------------------- central-moment transform
// Shifted form: the line holds g = f - K*(1/6, 2/3, 1/6) for a line rest
// factor K; the transform returns (k0 - K, k1, k2 - K/3), i.e. the central
// moments minus their rest-state values.  After the three passes slot
// 9c + 3b + a holds kappa_abc - R_a R_b R_c with R = (1, 0, 1/3).
template <typename T>
__device__ __forceinline__ void fwd_line(T& m, T& z, T& p, T a, T K) {
  const T s = p + m, d = p - m;
  const T k0 = s + z;
  const T kt = k0 + K;
  const T k1 = d - a * kt;
  const T k2 = s + a * (a * kt - T(2) * d);
  m = k0; z = k1; p = k2;
}
template <typename T>
__device__ __forceinline__ void inv_line(T& m, T& z, T& p, T a, T K) {
  const T k0 = m, k1 = z, k2 = p;
  const T kt = k0 + K;
  const T m1 = k1 + a * kt;
  const T m2 = k2 + a * (T(2) * k1 + a * kt);
  z = k0 - m2;
  p = T(0.5) * (m2 + m1);
  m = T(0.5) * (m2 - m1);
}

// Macroscopic quantities and the forward transform in one pass: the z-line
// sums of the first pass give rho - 1 and the momentum, the velocity then
// completes the three passes.  hf is half the body force.
template <typename T>
__device__ __forceinline__ void macro_and_forward(T* g, const T* hf, T& drho, T& rho, T& irho, T& ux, T& uy,
                                                  T& uz) {
  T sz[9], dz[9];
#pragma unroll
  for (int yx = 0; yx < 9; ++yx) {
    const T m = g[yx], z = g[9 + yx], p = g[18 + yx];
    sz[yx] = p + m;
    dz[yx] = p - m;
    g[yx] = sz[yx] + z;  // k0 of the z line (shifted)
  }
  // density and momentum from the line sums: x and y velocities are those of
  // the line, z momentum is the sum of the line differences
  const T c_m = g[0] + g[3] + g[6], c_0 = g[1] + g[4] + g[7], c_p = g[2] + g[5] + g[8];
  const T r_m = g[0] + g[1] + g[2], r_p = g[6] + g[7] + g[8];
  const T d = c_m + c_0 + c_p;
  const T jx = c_p - c_m, jy = r_p - r_m;
  const T jz = ((dz[0] + dz[1]) + (dz[2] + dz[3])) + ((dz[4] + dz[5]) + (dz[6] + dz[7])) + dz[8];
  drho = d;
  rho = T(1) + d;
  irho = fast_rcp(rho);
  ux = (jx + hf[0]) * irho;
  uy = (jy + hf[1]) * irho;
  uz = (jz + hf[2]) * irho;
#pragma unroll
  for (int yx = 0; yx < 9; ++yx) {  // finish the z lines, fixed (cx, cy)
    const int x = yx % 3, y = yx / 3;
    const T K = T(w1d(x - 1) * w1d(y - 1));
    const T kt = g[yx] + K;
    g[9 + yx] = dz[yx] - uz * kt;
    g[18 + yx] = sz[yx] + uz * (uz * kt - T(2) * dz[yx]);
  }
#pragma unroll
  for (int zx = 0; zx < 9; ++zx) {  // y lines, fixed (cx, z order)
    const int x = zx % 3, c = zx / 3;
    fwd_line(g[9 * c + x], g[9 * c + 3 + x], g[9 * c + 6 + x], uy, T(w1d(x - 1) * rest1d(c)));
  }
#pragma unroll
  for (int zy = 0; zy < 9; ++zy) {  // x lines, fixed (y order, z order)
    const int b = zy % 3, c = zy / 3;
    fwd_line(g[9 * c + 3 * b], g[9 * c + 3 * b + 1], g[9 * c + 3 * b + 2], ux, T(rest1d(b) * rest1d(c)));
  }
}

template <typename T>
__device__ __forceinline__ void inverse_transform(T* g, T ux, T uy, T uz) {
#pragma unroll
  for (int zy = 0; zy < 9; ++zy) {
    const int b = zy % 3, c = zy / 3;
    inv_line(g[9 * c + 3 * b], g[9 * c + 3 * b + 1], g[9 * c + 3 * b + 2], ux, T(rest1d(b) * rest1d(c)));
  }
#pragma unroll
  for (int zx = 0; zx < 9; ++zx) {
    const int x = zx % 3, c = zx / 3;
    inv_line(g[9 * c + x], g[9 * c + 3 + x], g[9 * c + 6 + x], uy, T(w1d(x - 1) * rest1d(c)));
  }
#pragma unroll
  for (int yx = 0; yx < 9; ++yx) {
    const int x = yx % 3, y = yx / 3;
    inv_line(g[3 * y + x], g[9 + 3 * y + x], g[18 + 3 * y + x], uz, T(w1d(x - 1) * w1d(y - 1)));
  }
}

// moment slot of orders (a, b, c) in x, y, z
__host__ __device__ constexpr int MI(int a, int b, int c) { return 9 * c + 3 * b + a; }

// Collision constants, precomputed on the host in the compute type.
template <typename T>
struct Coef {
  T w1, w2;        // shear and bulk rates
  T omw1, omw2;    // 1 - omega
  T c1, c2;        // Galilean correction factors G * 3 (1 - omega/2)
  T lam;           // third-order limiter
  T l3, l4, l5;    // (1 - w3) lam, (1 - w4) lam, (1 - w5) lam
  T a4;            // -(2/3) (1/w1 - 1/2) A
  T b4;            // (1/w1 - 1/2) B w1
  T hf[3];         // half body force
  T u6;            // 6 u_in (moving-wall inlet)
};


// Cumulant collision of one cell in the transformed, shifted representation.
// On entry g holds the shifted central moments of orders <= 3 (higher
// orders are never needed: every post-collision cumulant of order >= 4 is
// set, not relaxed from its value); on exit g holds the post-collision
// shifted central moments of all orders.
template <typename T, int MODE>
__device__ __forceinline__ void collide_moments(T* g, T drho, T rho, T irho, T ux, T uy, T uz, const Coef<T>& k) {
  const T third = T(1.0 / 3.0);
  // normalised second-order deviations from the rest state 1/3
  const T d3 = drho * third;
  const T d200 = (g[MI(2, 0, 0)] - d3) * irho;
  const T d020 = (g[MI(0, 2, 0)] - d3) * irho;
  const T d002 = (g[MI(0, 0, 2)] - d3) * irho;
  const T k110 = g[MI(1, 1, 0)] * irho, k101 = g[MI(1, 0, 1)] * irho, k011 = g[MI(0, 1, 1)] * irho;

  // velocity-gradient estimates from the second-order non-equilibrium
  const T m1 = d200 - d020, m2 = d200 - d002, tr = d200 + d020 + d002;
  const T Dxu = T(-0.5) * k.w1 * (m1 + m2) - T(0.5) * k.w2 * tr;
  const T Dyv = Dxu + T(1.5) * k.w1 * m1;
  const T Dzw = Dxu + T(1.5) * k.w1 * m2;
  const T xD = ux * ux * Dxu, yD = uy * uy * Dyv, zD = uz * uz * Dzw;
  const T m1s = k.omw1 * m1 - k.c1 * (xD - yD);
  const T m2s = k.omw1 * m2 - k.c1 * (xD - zD);
  const T trs = k.omw2 * tr - k.c2 * (xD + yD + zD);
  const T a = (m1s + m2s + trs) * third;            // post d200
  const T b = (trs - T(2) * m1s + m2s) * third;     // post d020
  const T c = (trs + m1s - T(2) * m2s) * third;     // post d002
  const T s110 = k.omw1 * k110, s101 = k.omw1 * k101, s011 = k.omw1 * k011;

  // third order (cumulants equal moments) and fourth-order cumulants
  T C210 = 0, C012 = 0, C201 = 0, C021 = 0, C120 = 0, C102 = 0, C111 = 0;
  T C220 = 0, C202 = 0, C022 = 0, C211 = 0, C121 = 0, C112 = 0;
  if (MODE == 1) {
    // relaxed value (1 - omega_lambda) v with omega_lambda the limited rate
    // omega + (1 - omega) |v| / (lambda + |v|)
    auto relax = [&](T lw, T v) { return lw * fast_rcp(k.lam + fabs(v)) * v; };
    {
      const T p = (g[MI(1, 2, 0)] + g[MI(1, 0, 2)]) * irho, d = (g[MI(1, 2, 0)] - g[MI(1, 0, 2)]) * irho;
      const T ps = relax(k.l3, p), ds = relax(k.l4, d);
      C120 = T(0.5) * (ps + ds); C102 = T(0.5) * (ps - ds);
    }
    {
      const T p = (g[MI(2, 1, 0)] + g[MI(0, 1, 2)]) * irho, d = (g[MI(2, 1, 0)] - g[MI(0, 1, 2)]) * irho;
      const T ps = relax(k.l3, p), ds = relax(k.l4, d);
      C210 = T(0.5) * (ps + ds); C012 = T(0.5) * (ps - ds);
    }
    {
      const T p = (g[MI(2, 0, 1)] + g[MI(0, 2, 1)]) * irho, d = (g[MI(2, 0, 1)] - g[MI(0, 2, 1)]) * irho;
      const T ps = relax(k.l3, p), ds = relax(k.l4, d);
      C201 = T(0.5) * (ps + ds); C021 = T(0.5) * (ps - ds);
    }
    C111 = relax(k.l5, g[MI(1, 1, 1)] * irho);
    C220 = k.a4 * (Dxu + Dyv);
    C202 = k.a4 * (Dxu + Dzw);
    C022 = k.a4 * (Dyv + Dzw);
    C211 = k.b4 * k011;   // -(1/3) t B (-3 w1 c011)
    C121 = k.b4 * k101;
    C112 = k.b4 * k110;
  }
  // back to normalised central moments (partition sums over post values)
  const T A2 = third + a, B2 = third + b, C2 = third + c;
  const T k211 = C211 + A2 * s011 + T(2) * s110 * s101;
  const T k121 = C121 + B2 * s101 + T(2) * s110 * s011;
  const T k112 = C112 + C2 * s110 + T(2) * s101 * s011;
  const T d220 = C220 + (a + b) * third + a * b + T(2) * s110 * s110;
  const T d202 = C202 + (a + c) * third + a * c + T(2) * s101 * s101;
  const T d022 = C022 + (b + c) * third + b * c + T(2) * s011 * s011;
  T k221 = 0, k212 = 0, k122 = 0;
  if (MODE == 1) {
    k221 = A2 * C021 + B2 * C201 + T(4) * s110 * C111 + T(2) * (s101 * C120 + s011 * C210);
    k212 = A2 * C012 + C2 * C210 + T(4) * s101 * C111 + T(2) * (s110 * C102 + s011 * C201);
    k122 = B2 * C102 + C2 * C120 + T(4) * s011 * C111 + T(2) * (s110 * C012 + s101 * C021);
  }
  T d222 = (a + b + c) * T(1.0 / 9.0) + (a * b + b * c + c * a) * third + a * b * c +
           T(2) * (A2 * s011 * s011 + B2 * s101 * s101 + C2 * s110 * s110) + T(8) * s110 * s101 * s011;
  if (MODE == 1) {
    d222 += A2 * C022 + B2 * C202 + C2 * C220 + T(4) * (s110 * C112 + s101 * C121 + s011 * C211) +
            T(2) * (C210 * C012 + C201 * C021 + C120 * C102) + T(4) * C111 * C111;
  }
  // post-collision shifted central moments kappa* - rest
  g[MI(0, 0, 0)] = drho;
  g[MI(1, 0, 0)] = -g[MI(1, 0, 0)];
  g[MI(0, 1, 0)] = -g[MI(0, 1, 0)];
  g[MI(0, 0, 1)] = -g[MI(0, 0, 1)];
  g[MI(2, 0, 0)] = rho * a + d3;
  g[MI(0, 2, 0)] = rho * b + d3;
  g[MI(0, 0, 2)] = rho * c + d3;
  g[MI(1, 1, 0)] = rho * s110;
  g[MI(1, 0, 1)] = rho * s101;
  g[MI(0, 1, 1)] = rho * s011;
  g[MI(2, 1, 0)] = rho * C210; g[MI(0, 1, 2)] = rho * C012;
  g[MI(2, 0, 1)] = rho * C201; g[MI(0, 2, 1)] = rho * C021;
  g[MI(1, 2, 0)] = rho * C120; g[MI(1, 0, 2)] = rho * C102;
  g[MI(1, 1, 1)] = rho * C111;
  g[MI(2, 1, 1)] = rho * k211; g[MI(1, 2, 1)] = rho * k121; g[MI(1, 1, 2)] = rho * k112;
  const T d9 = drho * T(1.0 / 9.0);
  g[MI(2, 2, 0)] = rho * d220 + d9;
  g[MI(2, 0, 2)] = rho * d202 + d9;
  g[MI(0, 2, 2)] = rho * d022 + d9;
  g[MI(2, 2, 1)] = rho * k221; g[MI(2, 1, 2)] = rho * k212; g[MI(1, 2, 2)] = rho * k122;
  g[MI(2, 2, 2)] = rho * d222 + drho * T(1.0 / 27.0);
}

}  // namespace mlbm
