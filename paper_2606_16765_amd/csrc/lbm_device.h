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
template <> struct Storage<double> {
  using T = double;
  static __device__ __forceinline__ double load(const double* p) { return *p; }
  static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
};
template <> struct Storage<float> {
  using T = float;
  static __device__ __forceinline__ float load(const float* p) { return *p; }
  static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
};
template <> struct Storage<f16s> {
  using T = float;
  static __device__ __forceinline__ float load(const f16s* p) {
    return (float)__builtin_bit_cast(_Float16, *(const uint16_t*)p);
  }
  static __device__ __forceinline__ void store(f16s* p, float v) {
    // v_cvt_f16_f32 rounds to nearest even in the default mode
    *(uint16_t*)p = __builtin_bit_cast(uint16_t, (_Float16)v);
  }
};
template <> struct Storage<bf16s> {
  using T = float;
  static __device__ __forceinline__ float load(const bf16s* p) {
    return __uint_as_float(((uint32_t) * (const uint16_t*)p) << 16);
  }
  static __device__ __forceinline__ void store(bf16s* p, float v) {
    uint32_t b = __float_as_uint(v);
    // round to nearest, ties to even; quiet NaN stays NaN
    uint32_t r = ((b & 0x7fffffffu) > 0x7f800000u) ? (0x7fc00000u) : (b + 0x7fffu + ((b >> 16) & 1u));
    *(uint16_t*)p = (uint16_t)(r >> 16);
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

template <typename T>
__device__ __forceinline__ void forward_transform(T* g, T ux, T uy, T uz) {
#pragma unroll
  for (int yx = 0; yx < 9; ++yx) {  // z lines, fixed (cx, cy)
    const int x = yx % 3, y = yx / 3;
    fwd_line(g[3 * y + x], g[9 + 3 * y + x], g[18 + 3 * y + x], uz, T(w1d(x - 1) * w1d(y - 1)));
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

struct CollideParams {
  double omega1, omega2;
  double galilean;            // 1, 0 (or -1)
  double lambda;
  double k17[5];              // w3, w4, w5, A, B
  double force[3];
};

// Cumulant collision of one cell in the transformed, shifted representation.
// On entry g holds the shifted central moments of orders <= 3 (higher
// orders are never needed: every post-collision cumulant of order >= 4 is
// set, not relaxed from its value); on exit g holds the post-collision
// shifted central moments of all orders.
template <typename T, int MODE>
__device__ __forceinline__ void collide_moments(T* g, T drho, T rho, T irho, T ux, T uy, T uz,
                                                const CollideParams& cp) {
  const T w1 = T(cp.omega1), w2 = T(cp.omega2), G = T(cp.galilean);
  const T third = T(1.0 / 3.0);
  // normalised second-order deviations from the rest state 1/3
  const T d200 = (g[MI(2, 0, 0)] - drho * third) * irho;
  const T d020 = (g[MI(0, 2, 0)] - drho * third) * irho;
  const T d002 = (g[MI(0, 0, 2)] - drho * third) * irho;
  const T k110 = g[MI(1, 1, 0)] * irho, k101 = g[MI(1, 0, 1)] * irho, k011 = g[MI(0, 1, 1)] * irho;

  // velocity-gradient estimates from the second-order non-equilibrium
  const T Dxu = T(-0.5) * w1 * (T(2) * d200 - d020 - d002) - T(0.5) * w2 * (d200 + d020 + d002);
  const T Dyv = Dxu + T(1.5) * w1 * (d200 - d020);
  const T Dzw = Dxu + T(1.5) * w1 * (d200 - d002);
  const T ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const T m1 = d200 - d020, m2 = d200 - d002, tr = d200 + d020 + d002;
  const T c1 = G * T(3) * (T(1) - T(0.5) * w1), c2 = G * T(3) * (T(1) - T(0.5) * w2);
  const T m1s = (T(1) - w1) * m1 - c1 * (ux2 * Dxu - uy2 * Dyv);
  const T m2s = (T(1) - w1) * m2 - c1 * (ux2 * Dxu - uz2 * Dzw);
  const T trs = (T(1) - w2) * tr - c2 * (ux2 * Dxu + uy2 * Dyv + uz2 * Dzw);
  const T a = (m1s + m2s + trs) * third;            // post d200
  const T b = (trs - T(2) * m1s + m2s) * third;     // post d020
  const T c = (trs + m1s - T(2) * m2s) * third;     // post d002
  const T s110 = (T(1) - w1) * k110, s101 = (T(1) - w1) * k101, s011 = (T(1) - w1) * k011;

  // third order (cumulants equal moments) and fourth-order cumulants
  T C210 = 0, C012 = 0, C201 = 0, C021 = 0, C120 = 0, C102 = 0, C111 = 0;
  T C220 = 0, C202 = 0, C022 = 0, C211 = 0, C121 = 0, C112 = 0;
  if (MODE == 1) {
    const T w3 = T(cp.k17[0]), w4 = T(cp.k17[1]), w5 = T(cp.k17[2]), A = T(cp.k17[3]), B = T(cp.k17[4]);
    const T lam = T(cp.lambda);
    // relaxed value (1 - omega_lambda) c with omega_lambda = omega + (1-omega)|c|/(lambda+|c|)
    auto relax = [&](T wr, T v) { return (T(1) - wr) * lam / (lam + fabs(v)) * v; };
    {
      const T p = (g[MI(1, 2, 0)] + g[MI(1, 0, 2)]) * irho, d = (g[MI(1, 2, 0)] - g[MI(1, 0, 2)]) * irho;
      const T ps = relax(w3, p), ds = relax(w4, d);
      C120 = T(0.5) * (ps + ds); C102 = T(0.5) * (ps - ds);
    }
    {
      const T p = (g[MI(2, 1, 0)] + g[MI(0, 1, 2)]) * irho, d = (g[MI(2, 1, 0)] - g[MI(0, 1, 2)]) * irho;
      const T ps = relax(w3, p), ds = relax(w4, d);
      C210 = T(0.5) * (ps + ds); C012 = T(0.5) * (ps - ds);
    }
    {
      const T p = (g[MI(2, 0, 1)] + g[MI(0, 2, 1)]) * irho, d = (g[MI(2, 0, 1)] - g[MI(0, 2, 1)]) * irho;
      const T ps = relax(w3, p), ds = relax(w4, d);
      C201 = T(0.5) * (ps + ds); C021 = T(0.5) * (ps - ds);
    }
    C111 = relax(w5, g[MI(1, 1, 1)] * irho);
    const T t = T(1) / w1 - T(0.5);
    C220 = T(-2.0 / 3.0) * t * A * (Dxu + Dyv);
    C202 = T(-2.0 / 3.0) * t * A * (Dxu + Dzw);
    C022 = T(-2.0 / 3.0) * t * A * (Dyv + Dzw);
    C211 = t * B * w1 * k011;   // -(1/3) t B (-3 w1 c011)
    C121 = t * B * w1 * k101;
    C112 = t * B * w1 * k110;
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
  g[MI(2, 0, 0)] = rho * a + drho * third;
  g[MI(0, 2, 0)] = rho * b + drho * third;
  g[MI(0, 0, 2)] = rho * c + drho * third;
  g[MI(1, 1, 0)] = rho * s110;
  g[MI(1, 0, 1)] = rho * s101;
  g[MI(0, 1, 1)] = rho * s011;
  g[MI(2, 1, 0)] = rho * C210; g[MI(0, 1, 2)] = rho * C012;
  g[MI(2, 0, 1)] = rho * C201; g[MI(0, 2, 1)] = rho * C021;
  g[MI(1, 2, 0)] = rho * C120; g[MI(1, 0, 2)] = rho * C102;
  g[MI(1, 1, 1)] = rho * C111;
  g[MI(2, 1, 1)] = rho * k211; g[MI(1, 2, 1)] = rho * k121; g[MI(1, 1, 2)] = rho * k112;
  g[MI(2, 2, 0)] = rho * d220 + drho * T(1.0 / 9.0);
  g[MI(2, 0, 2)] = rho * d202 + drho * T(1.0 / 9.0);
  g[MI(0, 2, 2)] = rho * d022 + drho * T(1.0 / 9.0);
  g[MI(2, 2, 1)] = rho * k221; g[MI(2, 1, 2)] = rho * k212; g[MI(1, 2, 2)] = rho * k122;
  g[MI(2, 2, 2)] = rho * d222 + drho * T(1.0 / 27.0);
}

}  // namespace mlbm
