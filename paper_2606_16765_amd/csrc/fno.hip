// Host runtime of the 3D Fourier neural operator surrogate behind the C ABI
// of include/mi355lbm.h (paper Sec. 4 and App. A.2: FNO predicting mean
// flow fields from geometry and Reynolds number).
//
// Layouts (B batch, W width, P = X*Y*Z, modes M = MX*MY*MZ with MX = 2mx,
// MY = 2my, MZ = mz; complex values split into re/im planes next to the
// contracted axis so that every DFT stage is one real contraction):
//   activations      [B][W][X][Y][Z]
//   z stage out  A1  [B W X Y][part][kz]
//   y stage out  A2  [B W X][part][ky][kz]
//   modes            [B][W][kx][part][ky][kz] (mode-minor; m = (kx, ky, kz))
//   inverse x    R3  [B W][x][part][ky][kz]
//   inverse y    R2  [B W X][y][part][kz]
// A1, A2, the modes, R3 and R2 are BF16: each is read only as an MFMA
// operand, which is rounded to BF16 (RNE) in any case, so storing it rounded
// changes no result and halves the traffic of the intermediate stages.
// Real embedding of a complex factor F = c - i s (forward) or c + i s
// (inverse) for input part pi, output part po:
//   forward  (0,0) c  (1,0) s   (0,1) -s  (1,1) c
//   inverse  (0,0) c  (1,0) -s  (0,1) s   (1,1) c
// The factorized FNO (arch 2) keeps per-axis modes [B][W][OUT][2][m][IN]
// instead (ffno_kernels.h), one 1D transform per axis.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ffno_kernels.h"
#include "fno_kernels.h"
#include "mi355lbm.h"

using namespace mfno;

namespace {

uint16_t host_bf16(double v) {
  float f = (float)v;
  uint32_t b;
  std::memcpy(&b, &f, 4);
  uint32_t r = ((b & 0x7fffffffu) > 0x7f800000u) ? 0x7fc00000u : (b + 0x7fffu + ((b >> 16) & 1u));
  return (uint16_t)(r >> 16);
}

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return ((int64_t(1) << l) == v) ? l : -1;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// padded transposed operand gt[n][k] = G[k][n] for a dense G (K x N)
struct GtMat {
  uint16_t* d = nullptr;
  int K = 0, N = 0, kp = 0, np = 0;
};

}  // namespace

struct fno_net {
  fno_params p{};
  hipStream_t st = nullptr;
  std::string err;
  int64_t nparam = 0;
  int W = 0, X = 0, Y = 0, Z = 0, MX = 0, MY = 0, MZ = 0, L = 0, H = 0;
  int64_t P = 0, M = 0;
  // parameter offsets
  int64_t off_P = 0, off_p = 0, off_Q1 = 0, off_q1 = 0, off_Q2 = 0, off_q2 = 0;
  std::vector<int64_t> off_W, off_Wp, off_bp;
  // hybrid F/FNO: feed-forward width and per-layer W1, b1, W2, b2 offsets
  bool hybrid = false;
  int Hf = 0;
  std::vector<int64_t> off_W1, off_b1, off_W2, off_b2;
  // factorized FNO (arch 2; it shares the hybrid's feed-forward blocks):
  // per axis d (0 x, 1 y, 2 z) the length N, retained modes m, the extents
  // OUT and IN of its mode layout, the 1D DFT operands (F forward, I c2r
  // inverse, Ia and Fa their adjoints), the offset of its weights in a
  // layer's spectral block and of its modes in Vh[l]; the embedded mixing
  // weights E and their transposes per (layer, axis)
  bool ffno = false;
  struct Axis {
    int N = 0, m = 0;
    int64_t OUT = 0, IN = 0, woff = 0, voff = 0;
    GtMat F, I, Ia, Fa;
  };
  Axis ax[3];
  std::vector<uint16_t*> Emix, ETmix;
  float* fpart = nullptr;  // Gram partials of the mixing gradient
  uint16_t* Yh2 = nullptr;  // second mode buffer of the fused y/z inverse (null: unfused)
  int64_t fpart_elems = 0;
  float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  int adam_t = 0;
  uint16_t* wspec = nullptr;  // BF16 copy of all parameters (spectral blocks used)
  // DFT operands
  GtMat F1, F1a, F2, F3, I3, I2, I1, I1a;
  // pointwise operands (forward and transposed)
  GtMat Glift, Gq1, Gq1t, Gq2, Gq2t;
  std::vector<GtMat> Gwp, Gwpt;
  // fused projection operands (inference): padded BF16 Q1 [Hp][Wp], Q2 [16][Hp], FP32 q1 [Hp]
  GtMat Pq1, Pq2;
  float* pq1b = nullptr;
  bool fused_proj = false;
  // the projection backward also forms the Q2 gradient (cout <= 8), so the
  // forward pass of a training step stores no hidden activation
  bool q2_in_bwd = false;
  // hybrid feed-forward operands per layer (the fused projection's layout):
  // W1 [Hfp][32], W2 [32][Hfp], W2^T [Hfp][32] BF16, b1 [Hfp] FP32, zero padded
  std::vector<GtMat> Pf1, Pf2, Gf2t;
  std::vector<float*> fb1;
  // c2r along z, channel map, bias and activation in one kernel
  bool fused_layer_end = false;
  // activations and work buffers
  std::vector<uint16_t*> v;  // L + 1, BF16
  std::vector<float*> h;     // L, FP32 pre-activations
  std::vector<uint16_t*> Vh;  // L, BF16 modes (mode-minor)
  // hybrid: spectral convolution s and feed-forward hidden activation per
  // layer (BF16), the hidden gradient and the gradient of s
  std::vector<uint16_t*> S, Aff;
  uint16_t* ffa = nullptr;
  float* gs = nullptr;
  uint16_t *A1 = nullptr, *A2 = nullptr, *R3 = nullptr, *R2 = nullptr;  // BF16 DFT intermediates
  uint16_t* Yh = nullptr;  // BF16 modes (mode-minor)
  float *h1 = nullptr, *y = nullptr, *gy = nullptr, *ga = nullptr, *gv = nullptr, *gvn = nullptr;
  uint16_t* a = nullptr;
  uint16_t* Vg = nullptr;  // mode gradient, BF16 mode-minor
  float* part = nullptr;
  int64_t part_elems = 0;
  float* part2 = nullptr;  // second-stage partials of the Gram reductions
  int64_t part2_elems = 0;
  float* partc = nullptr;  // per-chunk row sums (bias gradients)
  int64_t partc_elems = 0;
  double* lpart = nullptr;
  int64_t lpart_n = 0;
  // device scalars of the loss: [0] mask count (int64), [1] loss (FP64),
  // [2] gradient scale (FP32)
  double* lscal = nullptr;
  int lastB = 0;
  std::vector<void*> allocs;
};

static std::string g_fno_err;

static int ffail(fno_net* n, int code, const std::string& m) {
  if (n) n->err = m;
  g_fno_err = m;
  return code;
}

#define FCHK(n, call)                                                                                        \
  do {                                                                                                       \
    hipError_t e_ = (call);                                                                                  \
    if (e_ != hipSuccess)                                                                                    \
      return ffail((n), e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,                                \
                   std::string(#call) + ": " + hipGetErrorString(e_));                                       \
  } while (0)

static hipError_t falloc(fno_net* n, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) n->allocs.push_back(*p);
  return e;
}

// Build a padded transposed BF16 operand from a host matrix G[k][n].
static hipError_t make_gt_host(fno_net* n, GtMat& m, const std::vector<double>& G, int K, int N) {
  m.K = K;
  m.N = N;
  m.kp = (int)round_up(K, CT_K);
  m.np = (int)round_up(N, CT_N);
  std::vector<uint16_t> h((size_t)m.np * m.kp, 0);
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < N; ++j) h[(size_t)j * m.kp + k] = host_bf16(G[(size_t)k * N + j]);
  hipError_t e = falloc(n, (void**)&m.d, h.size() * 2);
  if (e != hipSuccess) return e;
  e = hipMemcpy(m.d, h.data(), h.size() * 2, hipMemcpyHostToDevice);
  return e;
}

static int mode_value(int j, int m) { return j < m ? j : j - 2 * m; }

// complex-embedded DFT operand along an axis of length Nn with retained
// modes kv[0..Km-1]; forward (sign -1): G[(n, pi)][(k, po)], inverse (sign
// +1): G[(k, pi)][(n, po)].
static std::vector<double> embed_dft(int Nn, const std::vector<int>& kv, int sign) {
  const int Km = (int)kv.size();
  const double tp = 2.0 * M_PI;
  if (sign < 0) {
    std::vector<double> G((size_t)(2 * Nn) * (2 * Km));
    for (int x = 0; x < Nn; ++x)
      for (int k = 0; k < Km; ++k) {
        const double th = tp * kv[k] * x / Nn, c = std::cos(th), s = std::sin(th);
        G[(size_t)(2 * x + 0) * (2 * Km) + 2 * k + 0] = c;
        G[(size_t)(2 * x + 1) * (2 * Km) + 2 * k + 0] = s;
        G[(size_t)(2 * x + 0) * (2 * Km) + 2 * k + 1] = -s;
        G[(size_t)(2 * x + 1) * (2 * Km) + 2 * k + 1] = c;
      }
    return G;
  }
  std::vector<double> G((size_t)(2 * Km) * (2 * Nn));
  for (int k = 0; k < Km; ++k)
    for (int x = 0; x < Nn; ++x) {
      const double th = tp * kv[k] * x / Nn, c = std::cos(th), s = std::sin(th);
      G[(size_t)(2 * k + 0) * (2 * Nn) + 2 * x + 0] = c;
      G[(size_t)(2 * k + 1) * (2 * Nn) + 2 * x + 0] = -s;
      G[(size_t)(2 * k + 0) * (2 * Nn) + 2 * x + 1] = s;
      G[(size_t)(2 * k + 1) * (2 * Nn) + 2 * x + 1] = c;
    }
  return G;
}

// ------------------------------------------------------------- launchers
struct CSpec {
  const void* in;
  bool in_bf16;
  void* out;
  bool out_bf16;
  const GtMat* g;
  int64_t cols;
  int64_t I;
  int64_t in_so, in_si, in_sk1, in_sk2;
  int kd;
  int64_t out_so, out_si, out_sn1, out_sn2;
  int nd;
  float alpha;
  bool accumulate;
  const float* bias;
  bool kcontig;
  bool store_out = true;
  uint16_t* act = nullptr;
  bool act_gelu = false;
  const float* gmul = nullptr;
};

template <typename InT, typename OutT, int LM>
static void launch_contract_ep(const ContractArgs& a, int ep, dim3 grid, hipStream_t st) {
  if (ep == EP_JVEC) hipLaunchKernelGGL((contract_kernel<InT, OutT, LM, EP_JVEC>), grid, dim3(256), 0, st, a);
  else if (ep == EP_NVEC) hipLaunchKernelGGL((contract_kernel<InT, OutT, LM, EP_NVEC>), grid, dim3(256), 0, st, a);
  else if (ep == EP_NFAST) hipLaunchKernelGGL((contract_kernel<InT, OutT, LM, EP_NFAST>), grid, dim3(256), 0, st, a);
  else if (ep == EP_JFAST) hipLaunchKernelGGL((contract_kernel<InT, OutT, LM, EP_JFAST>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((contract_kernel<InT, OutT, LM, EP_DIRECT>), grid, dim3(256), 0, st, a);
}

template <typename InT, typename OutT>
static void launch_contract(const ContractArgs& a, int lm, int ep, dim3 grid, hipStream_t st) {
  if (lm == LOAD_KRUN) launch_contract_ep<InT, OutT, LOAD_KRUN>(a, ep, grid, st);
  else if (lm == LOAD_JRUN) launch_contract_ep<InT, OutT, LOAD_JRUN>(a, ep, grid, st);
  else launch_contract_ep<InT, OutT, LOAD_SCALAR>(a, ep, grid, st);
}

static int contract(fno_net* n, const CSpec& c) {
  ContractArgs a{};
  a.in = c.in;
  a.out = c.out;
  a.gt = c.g->d;
  a.bias = c.bias;
  a.act = c.act;
  a.cols = c.cols;
  a.lgI = ilog2(c.I);
  a.in_so = c.in_so; a.in_si = c.in_si; a.in_sk1 = c.in_sk1; a.in_sk2 = c.in_sk2;
  a.lgkd = ilog2(c.kd);
  a.out_so = c.out_so; a.out_si = c.out_si; a.out_sn1 = c.out_sn1; a.out_sn2 = c.out_sn2;
  a.lgnd = ilog2(c.nd);
  a.K = c.g->K; a.N = c.g->N; a.kp = c.g->kp; a.np = c.g->np;
  a.alpha = c.alpha;
  a.accumulate = c.accumulate ? 1 : 0;
  a.store_out = c.store_out ? 1 : 0;
  a.act_gelu = c.act_gelu ? 1 : 0;
  a.gmul = c.gmul;
  if (a.lgI < 0 || a.lgkd < 0 || a.lgnd < 0) return ffail(n, LBM_EINVAL, "contraction index maps need powers of two");
  if ((a.accumulate || a.store_out) && !a.out) return ffail(n, LBM_EINVAL, "contraction output missing");
  // vector load modes need 8-element alignment of every address they form
  const size_t esz = c.in_bf16 ? 2 : 4;
  const bool base_ok = ((uintptr_t)c.in % (8 * esz)) == 0 && c.in_so % 8 == 0;
  int lm = LOAD_SCALAR;
  if (c.kcontig && c.kd == 1 && c.in_sk1 == 1 && a.K % 8 == 0 && base_ok && (c.I == 1 || c.in_si % 8 == 0))
    lm = LOAD_KRUN;
  else if (!c.kcontig && c.in_si == 1 && c.I % 8 == 0 && c.cols % 8 == 0 && base_ok && c.in_sk1 % 8 == 0 &&
           (c.kd == 1 || c.in_sk2 % 8 == 0))
    lm = LOAD_JRUN;
  // outputs contiguous along n or along (runs of at least 16) columns: store
  // through the LDS-staged epilogue in that order
  int ep = EP_DIRECT;
  if (c.nd == 1 && c.out_sn1 == 1) ep = EP_NFAST;
  else if (c.out_si == 1 && c.I >= 16) ep = EP_JFAST;
  // the vector forms: four consecutive outputs per access, every address a
  // multiple of 4 elements (strides, bases, the contiguous extent)
  auto al4 = [](const void* p, size_t esz) { return p == nullptr || ((uintptr_t)p % (4 * esz)) == 0; };
  const size_t oesz = c.out_bf16 ? 2 : 4;
  const bool bases4 = al4(c.out, oesz) && al4(c.act, 2) && al4(c.gmul, 4);
  if (ep == EP_JFAST && bases4 && c.cols % 4 == 0 && c.out_so % 4 == 0 && c.out_sn1 % 4 == 0 &&
      (c.nd == 1 || c.out_sn2 % 4 == 0))
    ep = EP_JVEC;
  else if (ep == EP_NFAST && bases4 && c.g->N % 4 == 0 && c.out_so % 4 == 0 && c.out_si % 4 == 0)
    ep = EP_NVEC;
  const int nblocks = c.g->np / CT_N;
  const dim3 grid((unsigned)((c.cols + CT_J - 1) / CT_J), (unsigned)(a.K <= CT_KT ? 1 : nblocks));
  if (c.in_bf16 && c.out_bf16) launch_contract<uint16_t, uint16_t>(a, lm, ep, grid, n->st);
  else if (c.in_bf16) launch_contract<uint16_t, float>(a, lm, ep, grid, n->st);
  else if (c.out_bf16) launch_contract<float, uint16_t>(a, lm, ep, grid, n->st);
  else launch_contract<float, float>(a, lm, ep, grid, n->st);
  return LBM_OK;
}

// pointwise channel map on [B][Cin][P] -> [B][Cout][P]
// epilogue: out is written when store_out, act (BF16, same layout) receives
// GELU(value) or the value when act is not null
static int pointwise(fno_net* n, int B, const void* in, bool in_bf16, int cin, void* out, bool out_bf16, int cout,
                     const GtMat* g, const float* bias, bool accumulate, bool store_out = true,
                     uint16_t* act = nullptr, bool act_gelu = false, const float* gmul = nullptr) {
  (void)cout;
  CSpec c{};
  c.in = in; c.in_bf16 = in_bf16; c.out = out; c.out_bf16 = out_bf16; c.g = g;
  c.cols = (int64_t)B * n->P; c.I = n->P;
  c.in_so = (int64_t)cin * n->P; c.in_si = 1; c.in_sk1 = n->P; c.in_sk2 = 0; c.kd = 1;
  c.out_so = (int64_t)g->N * n->P; c.out_si = 1; c.out_sn1 = n->P; c.out_sn2 = 0; c.nd = 1;
  c.alpha = 1.f; c.accumulate = accumulate; c.bias = bias; c.kcontig = false;
  c.store_out = store_out; c.act = act; c.act_gelu = act_gelu; c.gmul = gmul;
  // the dedicated channel-map kernel needs 256-point blocks within a sample
  // and 8-element aligned rows
  const size_t esz = in_bf16 ? 2 : 4;
  if (!out_bf16 && n->P % PW_J == 0 && ((uintptr_t)in % (8 * esz)) == 0 && ((uintptr_t)out % 16) == 0 &&
      ((uintptr_t)act % 16) == 0) {
    if ((accumulate || store_out) && !out) return ffail(n, LBM_EINVAL, "channel map output missing");
    PwArgs a{};
    a.in = in; a.out = (float*)out; a.gt = g->d; a.bias = bias; a.act = act; a.P = n->P;
    a.K = g->K; a.N = g->N; a.kp = g->kp; a.alpha = 1.f;
    a.accumulate = accumulate ? 1 : 0; a.store_out = store_out ? 1 : 0; a.act_gelu = act_gelu ? 1 : 0;
    a.gmul = gmul;
    const dim3 grid((unsigned)((int64_t)B * n->P / PW_J));
    if (in_bf16) hipLaunchKernelGGL(pw_kernel<uint16_t>, grid, dim3(256), 0, n->st, a);
    else hipLaunchKernelGGL(pw_kernel<float>, grid, dim3(256), 0, n->st, a);
    return LBM_OK;
  }
  return contract(n, c);
}

template <int NT, int KS, int ACT>
static void launch_proj_act(fno_net* n, int B, const uint16_t* v, float* y, uint16_t* aout) {
  const unsigned blocks = (unsigned)((int64_t)B * n->P / 256);
  const float w0 = n->p.proj_w0;
  if (aout)
    hipLaunchKernelGGL((proj_kernel<NT, KS, true, ACT>), dim3(blocks), dim3(256), 0, n->st, v, n->W, n->P, n->Pq1.d,
                       n->pq1b, n->Pq2.d, n->theta + n->off_q2, n->p.cout, y, n->H, aout, w0);
  else
    hipLaunchKernelGGL((proj_kernel<NT, KS, false, ACT>), dim3(blocks), dim3(256), 0, n->st, v, n->W, n->P,
                       n->Pq1.d, n->pq1b, n->Pq2.d, n->theta + n->off_q2, n->p.cout, y, 0, nullptr, w0);
}
template <int NT, int KS>
static void launch_proj(fno_net* n, int B, const uint16_t* v, float* y, uint16_t* aout) {
  if (n->p.proj_act == 1) launch_proj_act<NT, KS, 1>(n, B, v, y, aout);
  else launch_proj_act<NT, KS, 0>(n, B, v, y, aout);
}
template <int NT, int KS, bool GQ2>
static void launch_proj_bwd_q(fno_net* n, int B, const uint16_t* v, const float* gy, uint16_t* ga, float* gv,
                              float* q2part) {
  const unsigned blocks = (unsigned)((int64_t)B * n->P / 256);
  if (n->p.proj_act == 1)
    hipLaunchKernelGGL((proj_bwd_kernel<NT, KS, 1, false, GQ2>), dim3(blocks), dim3(256), 0, n->st, v, n->W, n->P,
                       n->Pq1.d, n->pq1b, n->Gq2t.d, n->Gq2t.kp, gy, n->p.cout, n->H, ga, gv, n->p.proj_w0, q2part);
  else
    hipLaunchKernelGGL((proj_bwd_kernel<NT, KS, 0, false, GQ2>), dim3(blocks), dim3(256), 0, n->st, v, n->W, n->P,
                       n->Pq1.d, n->pq1b, n->Gq2t.d, n->Gq2t.kp, gy, n->p.cout, n->H, ga, gv, 0.f, q2part);
}
template <int NT, int KS>
static void launch_proj_bwd(fno_net* n, int B, const uint16_t* v, const float* gy, uint16_t* ga, float* gv,
                            float* q2part) {
  if (q2part) launch_proj_bwd_q<NT, KS, true>(n, B, v, gy, ga, gv, q2part);
  else launch_proj_bwd_q<NT, KS, false>(n, B, v, gy, ga, gv, nullptr);
}

// fused projection; aout (training) also receives the BF16 hidden activation
static void fused_projection(fno_net* n, int B, const uint16_t* v, float* y, uint16_t* aout = nullptr) {
  const int NT = n->Pq1.np / 16, KS = n->Pq1.kp / 32;
  switch (NT * 4 + KS) {
    case 2 * 4 + 1: launch_proj<2, 1>(n, B, v, y, aout); break;
    case 2 * 4 + 2: launch_proj<2, 2>(n, B, v, y, aout); break;
    case 4 * 4 + 1: launch_proj<4, 1>(n, B, v, y, aout); break;
    case 4 * 4 + 2: launch_proj<4, 2>(n, B, v, y, aout); break;
    case 6 * 4 + 1: launch_proj<6, 1>(n, B, v, y, aout); break;
    case 6 * 4 + 2: launch_proj<6, 2>(n, B, v, y, aout); break;
    case 8 * 4 + 1: launch_proj<8, 1>(n, B, v, y, aout); break;
    default: launch_proj<8, 2>(n, B, v, y, aout); break;
  }
}
// fused projection backward: ga (BF16) = GELU'(h1) Q2^T gy, gv = Q1^T ga
static void fused_projection_bwd(fno_net* n, int B, const uint16_t* v, const float* gy, uint16_t* ga, float* gv,
                                 float* q2part = nullptr) {
  const int NT = n->Pq1.np / 16, KS = n->Pq1.kp / 32;
  switch (NT * 4 + KS) {
    case 2 * 4 + 1: launch_proj_bwd<2, 1>(n, B, v, gy, ga, gv, q2part); break;
    case 2 * 4 + 2: launch_proj_bwd<2, 2>(n, B, v, gy, ga, gv, q2part); break;
    case 4 * 4 + 1: launch_proj_bwd<4, 1>(n, B, v, gy, ga, gv, q2part); break;
    case 4 * 4 + 2: launch_proj_bwd<4, 2>(n, B, v, gy, ga, gv, q2part); break;
    case 6 * 4 + 1: launch_proj_bwd<6, 1>(n, B, v, gy, ga, gv, q2part); break;
    case 6 * 4 + 2: launch_proj_bwd<6, 2>(n, B, v, gy, ga, gv, q2part); break;
    case 8 * 4 + 1: launch_proj_bwd<8, 1>(n, B, v, gy, ga, gv, q2part); break;
    default: launch_proj_bwd<8, 2>(n, B, v, gy, ga, gv, q2part); break;
  }
}

// Hybrid F/FNO feed-forward block of layer l, forward:
//   vout = resid + W2 GELU(W1 s + b1) + b2 (BF16), aout (training) the BF16
//   hidden activation
template <int NT>
static void launch_ffn_t(fno_net* n, int l, int B, const uint16_t* s, const uint16_t* resid, uint16_t* vout,
                         uint16_t* aout) {
  const unsigned blocks = (unsigned)((int64_t)B * n->P / 256);
  const float* b2 = n->theta + n->off_b2[l];
  if (aout)
    hipLaunchKernelGGL((proj_kernel<NT, 1, true, 0, true>), dim3(blocks), dim3(256), 0, n->st, s, n->W, n->P,
                       n->Pf1[l].d, n->fb1[l], n->Pf2[l].d, b2, n->W, nullptr, n->Hf, aout, 0.f, resid, vout);
  else
    hipLaunchKernelGGL((proj_kernel<NT, 1, false, 0, true>), dim3(blocks), dim3(256), 0, n->st, s, n->W, n->P,
                       n->Pf1[l].d, n->fb1[l], n->Pf2[l].d, b2, n->W, nullptr, 0, nullptr, 0.f, resid, vout);
}
static void launch_ffn(fno_net* n, int l, int B, const uint16_t* s, const uint16_t* resid, uint16_t* vout,
                       uint16_t* aout) {
  switch (n->Pf1[l].np / 16) {
    case 2: launch_ffn_t<2>(n, l, B, s, resid, vout, aout); break;
    case 4: launch_ffn_t<4>(n, l, B, s, resid, vout, aout); break;
    case 6: launch_ffn_t<6>(n, l, B, s, resid, vout, aout); break;
    default: launch_ffn_t<8>(n, l, B, s, resid, vout, aout); break;
  }
}
// backward: ga (BF16) = GELU'(W1 s + b1) W2^T gv, gsv (FP32) = W1^T ga
template <int NT>
static void launch_ffn_bwd_t(fno_net* n, int l, int B, const uint16_t* s, const float* gv, uint16_t* ga, float* gsv) {
  const unsigned blocks = (unsigned)((int64_t)B * n->P / 256);
  hipLaunchKernelGGL((proj_bwd_kernel<NT, 1, 0, true>), dim3(blocks), dim3(256), 0, n->st, s, n->W, n->P, n->Pf1[l].d,
                     n->fb1[l], n->Gf2t[l].d, n->Gf2t[l].kp, gv, n->W, n->Hf, ga, gsv, 0.f);
}
static void launch_ffn_bwd(fno_net* n, int l, int B, const uint16_t* s, const float* gv, uint16_t* ga, float* gsv) {
  switch (n->Pf1[l].np / 16) {
    case 2: launch_ffn_bwd_t<2>(n, l, B, s, gv, ga, gsv); break;
    case 4: launch_ffn_bwd_t<4>(n, l, B, s, gv, ga, gsv); break;
    case 6: launch_ffn_bwd_t<6>(n, l, B, s, gv, ga, gsv); break;
    default: launch_ffn_bwd_t<8>(n, l, B, s, gv, ga, gsv); break;
  }
}

// ------------------------------------------------ factorized FNO (arch 2)
// Truncated 1D DFT along axis d as one contraction: grid values [B][W][P]
// -> modes [B][W][OUT][2][m][IN] (to_modes, with F or Ia), or modes -> grid
// values (with I or Fa).  The epilogue options are the contraction's.
static int axis_dft(fno_net* n, int d, int B, const void* in, bool in_bf16, const GtMat& G, void* out, bool out_bf16,
                    bool to_modes, bool accumulate, bool store_out = true, uint16_t* act = nullptr) {
  const auto& a = n->ax[d];
  const int64_t W = n->W, N = a.N, m = a.m, OUT = a.OUT, IN = a.IN;
  CSpec c{};
  c.in = in; c.in_bf16 = in_bf16; c.out = out; c.out_bf16 = out_bf16; c.g = &G;
  c.alpha = 1.f; c.accumulate = accumulate; c.store_out = store_out; c.act = act;
  c.cols = (int64_t)B * W * OUT * IN; c.I = IN; c.kd = 1; c.nd = 1;
  if (to_modes) {
    if (IN == 1) {
      c.in_so = N; c.in_sk1 = 1; c.kcontig = true;
      c.out_so = 2 * m; c.out_sn1 = 1;
    } else {
      c.in_so = N * IN; c.in_si = 1; c.in_sk1 = IN;
      c.out_so = 2 * m * IN; c.out_si = 1; c.nd = (int)m; c.out_sn1 = m * IN; c.out_sn2 = IN;
    }
  } else {
    if (IN == 1) {
      c.in_so = 2 * m; c.in_sk1 = 1; c.kcontig = true;
      c.out_so = N; c.out_sn1 = 1;
    } else {
      c.in_so = 2 * m * IN; c.in_si = 1; c.kd = (int)m; c.in_sk1 = m * IN; c.in_sk2 = IN;
      c.out_so = N * IN; c.out_si = 1; c.out_sn1 = IN;
    }
  }
  return contract(n, c);
}

// per-mode channel mixing of axis d's modes by the embedded weights e
// (E for the forward mixing, ET for its adjoint)
static void axis_mix(fno_net* n, int d, int B, const uint16_t* in, const uint16_t* e, uint16_t* out) {
  const auto& a = n->ax[d];
  AxisMixArgs m{};
  m.in = in; m.out = out; m.e = e; m.OUT = (int)a.OUT; m.IN = (int)a.IN; m.M = a.m;
  m.tiles = (int64_t)B * a.OUT * a.IN / AX_TR;
  const size_t lds = (size_t)a.m * (AX_TR * (2 * n->W + 8) + 8) * 2;
  if (n->W == 16) hipLaunchKernelGGL(axis_mix_kernel<16>, dim3((unsigned)m.tiles), dim3(256), lds, n->st, m);
  else hipLaunchKernelGGL(axis_mix_kernel<32>, dim3((unsigned)m.tiles), dim3(256), lds, n->st, m);
}

// weight gradient of axis d's mixing from its forward modes v and mode
// gradient g, stored to grad [m][W][W][2]
static void axis_mix_grad(fno_net* n, int d, int B, const uint16_t* v, const uint16_t* g, float* grad) {
  const auto& a = n->ax[d];
  AxisGradArgs ga{};
  ga.v = v; ga.g = g; ga.part = n->fpart; ga.OUT = (int)a.OUT; ga.IN = (int)a.IN; ga.M = a.m;
  ga.steps = (int64_t)B * a.OUT * a.IN / AX_GR;
  ga.per_chunk = (ga.steps + FFNO_NCHUNK - 1) / FFNO_NCHUNK;
  const int64_t nchunk = (ga.steps + ga.per_chunk - 1) / ga.per_chunk;
  const dim3 grid((unsigned)nchunk, (unsigned)(a.m / 4));
  if (n->W == 16) hipLaunchKernelGGL(axis_mix_grad_kernel<16>, grid, dim3(256), 0, n->st, ga);
  else hipLaunchKernelGGL(axis_mix_grad_kernel<32>, grid, dim3(256), 0, n->st, ga);
  const int64_t e = (int64_t)a.m * n->W * n->W;
  hipLaunchKernelGGL(axis_mix_grad_fold_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, n->st, n->fpart,
                     nchunk, a.m, n->W, grad);
}

// s = sum over the axes of R_d(W_d . T_d(v[l])) into S (BF16), summed in
// FP32 in the buffer of dL/ds (unused in the forward pass); the modes of
// each axis are kept in Vh[l] when training.  Where the y and z extents are
// 32 or 64, the x inverse is stored first and one pass adds the y and z
// inverses to it (axis_inverse_yz_kernel): the FP32 sum is written once and
// read once.
static int ffno_spectral(fno_net* n, int l, int B, bool training, uint16_t* S) {
  int rc;
  float* sacc = n->gs;
  if (n->Yh2) {
    for (int d = 0; d < 3; ++d) {
      auto& a = n->ax[d];
      uint16_t* V = training ? n->Vh[l] + a.voff : n->Vg;
      if ((rc = axis_dft(n, d, B, n->v[l], true, a.F, V, true, true, false))) return rc;
      uint16_t* Y = d == 1 ? n->Yh2 : n->Yh;
      axis_mix(n, d, B, V, n->Emix[3 * l + d], Y);
      if (d == 0 && (rc = axis_dft(n, 0, B, n->Yh, true, a.I, sacc, false, false, false))) return rc;
    }
    AxisYzArgs y{};
    y.yz = n->Yh; y.yy = n->Yh2; y.iz = n->ax[2].I.d; y.kpz = n->ax[2].I.kp; y.iy = n->ax[1].I.d;
    y.kpy = n->ax[1].I.kp; y.sx = sacc; y.s = S; y.Y = n->Y; y.Z = n->Z; y.MY2 = 2 * n->ax[1].m;
    y.MZ2 = 2 * n->ax[2].m;
    hipLaunchKernelGGL(axis_inverse_yz_kernel, dim3((unsigned)((int64_t)B * n->W * n->X)), dim3(256), 0, n->st, y);
    return LBM_OK;
  }
  const int order[3] = {2, 1, 0};
  for (int i = 0; i < 3; ++i) {
    const int d = order[i];
    auto& a = n->ax[d];
    uint16_t* V = training ? n->Vh[l] + a.voff : n->Vg;
    if ((rc = axis_dft(n, d, B, n->v[l], true, a.F, V, true, true, false))) return rc;
    axis_mix(n, d, B, V, n->Emix[3 * l + d], n->Yh);
    const bool last = i == 2;
    if ((rc = axis_dft(n, d, B, n->Yh, true, a.I, sacc, false, false, i > 0, !last, last ? S : nullptr))) return rc;
  }
  return LBM_OK;
}

// backward of the spectral convolution of layer l given dL/ds in gs:
// weight gradients of the three axes, and gv += the adjoint path
static int ffno_spectral_bwd(fno_net* n, int l, int B) {
  int rc;
  for (int d = 0; d < 3; ++d) {
    auto& a = n->ax[d];
    if ((rc = axis_dft(n, d, B, n->gs, false, a.Ia, n->Yh, true, true, false))) return rc;
    axis_mix_grad(n, d, B, n->Vh[l] + a.voff, n->Yh, n->grad + n->off_W[l] + a.woff);
    axis_mix(n, d, B, n->Yh, n->ETmix[3 * l + d], n->Vg);
    if ((rc = axis_dft(n, d, B, n->Vg, true, a.Fa, n->gv, false, false, true))) return rc;
  }
  return LBM_OK;
}

// truncated forward 3D DFT: v [B][W][P] (BF16 or FP32) -> modes [m][B][W][2]
// (z_done: A1 already holds the z stage, written by the previous layer end)
static int forward_dft(fno_net* n, int B, const void* v, bool v_bf16, const GtMat& Gz, uint16_t* modes,
                       bool z_done = false) {
  const int64_t W = n->W, X = n->X, Y = n->Y, Z = n->Z, MY = n->MY, MZ = n->MZ;
  int rc;
  CSpec c{};
  // z: rows (b,w,x,y), k = z contiguous -> A1[row][part][kz]
  if (!z_done) {
    c = CSpec{};
    c.in = v; c.in_bf16 = v_bf16; c.out = n->A1; c.out_bf16 = true; c.g = &Gz;
    c.cols = (int64_t)B * W * X * Y; c.I = 1; c.in_so = Z; c.in_sk1 = 1; c.kd = 1;
    c.out_so = 2 * MZ; c.out_sn1 = 1; c.nd = 1; c.alpha = 1.f; c.kcontig = true;
    if ((rc = contract(n, c))) return rc;
  }
  // y and x in one pass where the shapes are the fused kernel's (Y = 64,
  // 32 x 32 y/x modes, 16 z modes) and there are enough slabs to fill the chip
  if (Y == 64 && MY == 32 && n->MX == 32 && MZ == 16 && X % 16 == 0 && n->F2.kp == 128 &&
      n->F3.kp == 2 * X && (int64_t)B * W >= 256) {
    hipLaunchKernelGGL(dft_yx_kernel, dim3((unsigned)(B * W)), dim3(512), 0, n->st, n->A1, n->F2.d, n->F3.d,
                       (int)X, modes);
    return LBM_OK;
  }
  // y: cols (b,w,x) x kz, k = (y, part) at stride MZ -> A2[bwx][part][ky][kz]
  c = CSpec{};
  c.in = n->A1; c.in_bf16 = true; c.out = n->A2; c.out_bf16 = true; c.g = &n->F2;
  c.cols = (int64_t)B * W * X * MZ; c.I = MZ; c.in_so = Y * 2 * MZ; c.in_si = 1; c.in_sk1 = MZ; c.kd = 1;
  c.out_so = 2 * MY * MZ; c.out_si = 1; c.out_sn1 = MZ; c.out_sn2 = MY * MZ; c.nd = 2; c.alpha = 1.f;
  if ((rc = contract(n, c))) return rc;
  // x: cols (b,w) x (ky,kz), k = (x, part) at stride MY*MZ -> modes
  // [bw][kx][part][ky][kz], n = (kx, part) at stride MY*MZ
  c = CSpec{};
  c.in = n->A2; c.in_bf16 = true; c.out = modes; c.out_bf16 = true; c.g = &n->F3;
  c.cols = (int64_t)B * W * MY * MZ; c.I = MY * MZ; c.in_so = X * 2 * MY * MZ; c.in_si = 1; c.in_sk1 = MY * MZ;
  c.kd = 1;
  c.out_so = (int64_t)n->MX * 2 * MY * MZ; c.out_si = 1; c.out_sn1 = MY * MZ; c.nd = 1;
  c.alpha = 1.f;
  return contract(n, c);
}

// truncated inverse 3D DFT: modes [m][B][W][2] -> out [B][W][P] (FP32),
// with the z operand Gz (c2r with 1/N and c_kz, or its unscaled adjoint)
// out may be null with Gz unused: then only the x and y stages run, leaving
// the y-stage output in R2 for layer_end_kernel.
static int inverse_dft(fno_net* n, int B, const uint16_t* modes, const GtMat& Gz, float* out, bool accumulate,
                       const float* gmul = nullptr) {
  const int64_t W = n->W, X = n->X, Y = n->Y, Z = n->Z, MY = n->MY, MZ = n->MZ;
  int rc;
  CSpec c{};
  // x and y in one pass where the shapes are the fused kernel's
  if (Y == 64 && MY == 32 && n->MX == 32 && MZ == 16 && X % 8 == 0 && n->I3.kp == 64 && n->I2.kp == 64 &&
      (int64_t)B * W >= 256) {
    hipLaunchKernelGGL(idft_xy_kernel, dim3((unsigned)(B * W)), dim3(512), 0, n->st, modes, n->I3.d, n->I2.d,
                       (int)X, n->R2);
  } else {
  // x: cols (b,w) x (ky,kz); k = (kx, part) at stride MY*MZ (mode-minor)
  c.in = modes; c.in_bf16 = true; c.out = n->R3; c.out_bf16 = true; c.g = &n->I3;
  c.cols = (int64_t)B * W * MY * MZ; c.I = MY * MZ; c.in_so = (int64_t)n->MX * 2 * MY * MZ; c.in_si = 1;
  c.in_sk1 = MY * MZ; c.kd = 1;
  c.out_so = X * 2 * MY * MZ; c.out_si = 1; c.out_sn1 = MY * MZ; c.nd = 1; c.alpha = 1.f;
  if ((rc = contract(n, c))) return rc;
  // y: cols (b,w,x) x kz; k = (ky, part): ky at MZ, part at MY*MZ
  c = CSpec{};
  c.in = n->R3; c.in_bf16 = true; c.out = n->R2; c.out_bf16 = true; c.g = &n->I2;
  c.cols = (int64_t)B * W * X * MZ; c.I = MZ; c.in_so = 2 * MY * MZ; c.in_si = 1; c.in_sk1 = MZ; c.in_sk2 = MY * MZ;
  c.kd = 2; c.out_so = Y * 2 * MZ; c.out_si = 1; c.out_sn1 = MZ; c.nd = 1; c.alpha = 1.f;
  if ((rc = contract(n, c))) return rc;
  }
  if (!out) return LBM_OK;
  // z (c2r): rows (b,w,x,y), k = (part, kz) contiguous
  c = CSpec{};
  c.in = n->R2; c.in_bf16 = true; c.out = out; c.g = &Gz;
  c.cols = (int64_t)B * W * X * Y; c.I = 1; c.in_so = 2 * MZ; c.in_sk1 = 1; c.kd = 1;
  c.out_so = Z; c.out_sn1 = 1; c.nd = 1; c.alpha = 1.f; c.accumulate = accumulate; c.kcontig = true;
  c.gmul = gmul;
  return contract(n, c);
}

template <typename XT>
static int colsum(fno_net* n, const XT* Xd, int A, int B, float* out, bool accumulate) {
  const int64_t chunk = 8192;
  const int64_t nb = (int64_t)B * n->P / chunk;
  hipLaunchKernelGGL((colsum_kernel<XT>), dim3((unsigned)nb, (unsigned)A), dim3(256), 0, n->st, Xd, A, n->P, B,
                     chunk, n->part);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((A + 255) / 256)), dim3(256), 0, n->st, n->part, nb,
                     (int64_t)A, out, accumulate ? 1 : 0);
  return LBM_OK;
}

// out[a][c] (+)= sum_{b,p} X[b][a][p] Y[b][c][p]
template <typename XT, typename YT>
static bool launch_gram2(fno_net* n, const XT* Xd, int A, const YT* Yd, int Cc, int64_t nch, float* partc) {
  const int at = (A + 15) / 16, ct = (Cc + 15) / 16;
  const dim3 grid((unsigned)(nch / 4)), blk(256);
#define MFNO_GRAM2(I, J)                                                                                   \
  if (at <= I && ct <= J) {                                                                                \
    hipLaunchKernelGGL((gram2_kernel<XT, YT, I, J>), grid, blk, 0, n->st, Xd, Yd, n->part, A, Cc, n->P,   \
                       partc);                                                                             \
    return true;                                                                                           \
  }
  MFNO_GRAM2(1, 1)
  MFNO_GRAM2(1, 2)
  MFNO_GRAM2(2, 1)
  MFNO_GRAM2(2, 2)
  MFNO_GRAM2(1, 8)
  MFNO_GRAM2(8, 1)
  MFNO_GRAM2(8, 2)
  MFNO_GRAM2(2, 8)
  MFNO_GRAM2(4, 4)
  MFNO_GRAM2(8, 4)
#undef MFNO_GRAM2
  return false;
}

// out[a][c] (+)= sum_{b,p} X[b][a][p] Y[b][c][p]; with bout, also
// bout[a] = sum_{b,p} X[b][a][p] (the bias gradient of the same map)
template <typename XT, typename YT>
static int gram(fno_net* n, const XT* Xd, int A, const YT* Yd, int Cc, int B, float* out, bool accumulate,
                float* bout = nullptr) {
  const int chunk = 2048;
  static_assert(GR_CHUNK == 2048, "gram chunking");
  {
    const int64_t nch = (int64_t)B * n->P / GR_CHUNK;
    const int64_t E = (int64_t)A * Cc;
    constexpr int S = 64;
    const bool with_c = bout && nch * A <= n->partc_elems && S * A <= n->part2_elems;
    // (16-byte operand loads: misaligned rows take the scalar fallback)
    const bool aligned = ((uintptr_t)Xd % 16) == 0 && ((uintptr_t)Yd % 16) == 0;
    if (aligned && nch % 4 == 0 && nch * E <= n->part_elems && S * E <= n->part2_elems && (with_c || !bout) &&
        launch_gram2(n, Xd, A, Yd, Cc, nch, with_c ? n->partc : nullptr)) {
      hipLaunchKernelGGL(reduce_slices_kernel, dim3((unsigned)((E + 255) / 256), S), dim3(256), 0, n->st, n->part,
                         nch, E, S, n->part2);
      hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, n->st, n->part2,
                         (int64_t)S, E, out, accumulate ? 1 : 0);
      if (with_c) {
        hipLaunchKernelGGL(reduce_slices_kernel, dim3((unsigned)((A + 255) / 256), S), dim3(256), 0, n->st, n->partc,
                           nch, (int64_t)A, S, n->part2);
        hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((A + 255) / 256)), dim3(256), 0, n->st, n->part2,
                           (int64_t)S, (int64_t)A, bout, 0);
      }
      return LBM_OK;
    }
  }
  if (bout) colsum(n, Xd, A, B, bout, false);
  const int64_t nch = (int64_t)B * n->P / chunk;
  if (nch * A * Cc > n->part_elems) return ffail(n, LBM_EINVAL, "gram partial buffer too small");
  hipLaunchKernelGGL((gram_kernel<XT, YT>), dim3((unsigned)nch, (unsigned)((A + 15) / 16), (unsigned)((Cc + 15) / 16)),
                     dim3(64), 0, n->st, Xd, Yd, n->part, A, Cc, n->P, (int64_t)A * n->P, (int64_t)Cc * n->P, chunk);
  const int64_t E = (int64_t)A * Cc;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, n->st, n->part, nch, E,
                     out, accumulate ? 1 : 0);
  return LBM_OK;
}

static void elementwise_grid(int64_t cnt, dim3& g) { g = dim3((unsigned)((cnt + 255) / 256)); }

// Refresh the BF16 operands from the FP32 master parameters.
// operands derived from the FP32 parameters (bf16_done: the BF16 working
// copy is already current, written by the optimizer step)
static int refresh(fno_net* n, bool bf16_done = false) {
  dim3 g;
  elementwise_grid(n->nparam, g);
  if (!bf16_done) hipLaunchKernelGGL(to_bf16_kernel, g, dim3(256), 0, n->st, n->theta, n->wspec, n->nparam);
  auto mk = [&](GtMat& m, int64_t off, int rows, int cols, int tr) {
    const int64_t cnt = (int64_t)m.np * m.kp;
    dim3 gg;
    elementwise_grid(cnt, gg);
    hipLaunchKernelGGL(make_gt_kernel, gg, dim3(256), 0, n->st, n->theta + off, rows, cols, tr, m.d, m.np, m.kp);
  };
  mk(n->Glift, n->off_P, n->W, n->p.cin, 0);
  for (int l = 0; l < n->L; ++l) {
    for (int d = 0; n->ffno && d < 3; ++d) {
      const int64_t cnt = (int64_t)n->ax[d].m * (2 * n->W) * (2 * n->W);
      hipLaunchKernelGGL(axis_pack_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, n->st,
                         n->theta + n->off_W[l] + n->ax[d].woff, n->ax[d].m, n->W, n->Emix[3 * l + d],
                         n->ETmix[3 * l + d]);
    }
    if (n->hybrid) {
      mk(n->Pf1[l], n->off_W1[l], n->Hf, n->W, 0);
      mk(n->Pf2[l], n->off_W2[l], n->W, n->Hf, 0);
      mk(n->Gf2t[l], n->off_W2[l], n->W, n->Hf, 1);
      hipError_t ce = hipMemcpyAsync(n->fb1[l], n->theta + n->off_b1[l], (size_t)n->Hf * 4, hipMemcpyDeviceToDevice,
                                     n->st);
      if (ce != hipSuccess) return ffail(n, LBM_EDEVICE, hipGetErrorString(ce));
      continue;
    }
    mk(n->Gwp[l], n->off_Wp[l], n->W, n->W, 0);
    mk(n->Gwpt[l], n->off_Wp[l], n->W, n->W, 1);
  }
  mk(n->Gq1, n->off_Q1, n->H, n->W, 0);
  mk(n->Gq1t, n->off_Q1, n->H, n->W, 1);
  mk(n->Gq2, n->off_Q2, n->p.cout, n->H, 0);
  mk(n->Gq2t, n->off_Q2, n->p.cout, n->H, 1);
  if (n->fused_proj) {
    mk(n->Pq1, n->off_Q1, n->H, n->W, 0);
    mk(n->Pq2, n->off_Q2, n->p.cout, n->H, 0);
    hipError_t ce = hipMemcpyAsync(n->pq1b, n->theta + n->off_q1, (size_t)n->H * 4, hipMemcpyDeviceToDevice, n->st);
    if (ce != hipSuccess) return ffail(n, LBM_EDEVICE, hipGetErrorString(ce));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(n, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

static hipError_t alloc_gt(fno_net* n, GtMat& m, int K, int N) {
  m.K = K;
  m.N = N;
  m.kp = (int)round_up(K, CT_K);
  m.np = (int)round_up(N, CT_N);
  return falloc(n, (void**)&m.d, (size_t)m.np * m.kp * 2);
}

extern "C" int64_t fno_param_count(const fno_params* p) {
  if (!p) return -1;
  const int64_t w = p->width, hf = p->ff_hidden;
  const int64_t M = p->arch == 2 ? (int64_t)p->mx + p->my + p->mz : (int64_t)(2 * p->mx) * (2 * p->my) * p->mz;
  const int64_t layer = M * w * w * 2 + (p->arch == 1 || p->arch == 2 ? 2 * hf * w + hf + w : w * w + w);
  return w * p->cin + w + (int64_t)p->layers * layer + (int64_t)p->proj_hidden * w + p->proj_hidden +
         (int64_t)p->cout * p->proj_hidden + p->cout;
}

static void free_net(fno_net* n) {
  for (void* p : n->allocs) (void)hipFree(p);
  n->allocs.clear();
}

extern "C" int fno_create(const fno_params* pin, uint64_t seed, void* hip_stream, fno_net** out) {
  if (!pin || !out) return ffail(nullptr, LBM_EINVAL, "null argument");
  *out = nullptr;
  const fno_params& p = *pin;
  if (p.nx <= 0 || p.ny <= 0 || p.nz <= 0 || ilog2(p.nx) < 0 || ilog2(p.ny) < 0 || ilog2(p.nz) < 0)
    return ffail(nullptr, LBM_EINVAL, "grid sizes must be powers of two");
  if (p.width <= 0 || p.width % 16 || p.cin <= 0 || p.cout <= 0 || p.layers <= 0 || p.proj_hidden <= 0 ||
      p.proj_hidden % 16 || p.max_batch <= 0)
    return ffail(nullptr, LBM_EINVAL, "width and hidden must be positive multiples of 16");
  if (p.mx <= 0 || p.my <= 0 || p.mz <= 0 || 2 * p.mx > p.nx || 2 * p.my > p.ny || 2 * p.mz > p.nz ||
      ilog2(p.mx) < 0 || ilog2(p.my) < 0 || ilog2(p.mz) < 0)
    return ffail(nullptr, LBM_EINVAL, "modes must be powers of two with 2m <= n (and mz <= nz/2)");
  if (p.arch == 2 && (p.width != 16 && p.width != 32))
    return ffail(nullptr, LBM_EINVAL, "the factorized FNO needs width 16 or 32");
  if (p.arch == 2 && (p.mx < 4 || p.my < 4 || p.mz < 4 || p.mx > 16 || p.my > 16 || p.mz > 16 || p.nz < 32 ||
                      p.nz > 256 || p.ff_hidden <= 0 || p.ff_hidden % 16 || round_up(p.ff_hidden, 32) > 128))
    return ffail(nullptr, LBM_EINVAL,
                 "the factorized FNO needs 4 to 16 modes per axis, nz in [32, 256] and ff_hidden a multiple of 16 "
                 "up to 128");
  const int64_t P = (int64_t)p.nx * p.ny * p.nz;
  if (P % 8192) return ffail(nullptr, LBM_EINVAL, "grid must hold a multiple of 8192 cells");
  if (p.width > 64) return ffail(nullptr, LBM_EINVAL, "width must be at most 64");
  if (p.proj_act != 0 && p.proj_act != 1) return ffail(nullptr, LBM_EINVAL, "proj_act must be 0 (GELU) or 1 (sine)");
  if (p.proj_act == 1 && (!(p.proj_w0 > 0.f) || !std::isfinite(p.proj_w0) || round_up(p.proj_hidden, 32) > 128 ||
                          p.width > 64 || p.cout > 16 || P % 256))
    return ffail(nullptr, LBM_EINVAL, "the sine projection needs proj_w0 > 0, proj_hidden <= 128 and cout <= 16");
  if (p.arch != 2 && 2 * p.my * p.mz < (p.width <= 32 ? MixCfg<32>::MQ : MixCfg<64>::MQ))
    return ffail(nullptr, LBM_EINVAL, "2 my mz must be at least 32 (16 for width above 32)");
  if (p.arch < 0 || p.arch > 2)
    return ffail(nullptr, LBM_EINVAL, "arch must be 0 (FNO), 1 (hybrid F/FNO) or 2 (factorized FNO)");
  if (p.arch == 1 && (p.width > 32 || p.nz < 16 || p.nz > 256 || 2 * p.mz > 32 || P % 256 || p.ff_hidden <= 0 ||
                      p.ff_hidden % 16 || round_up(p.ff_hidden, 32) > 128))
    return ffail(nullptr, LBM_EINVAL,
                 "the hybrid F/FNO needs width <= 32, nz in [16, 256], 2 mz <= 32 and ff_hidden a multiple of 16 "
                 "up to 128");
  fno_net* n = new (std::nothrow) fno_net();
  if (!n) return ffail(nullptr, LBM_ENOMEM, "host allocation failed");
  n->p = p;
  n->st = (hipStream_t)hip_stream;
  n->W = p.width; n->X = p.nx; n->Y = p.ny; n->Z = p.nz;
  n->hybrid = p.arch == 1 || p.arch == 2;
  n->ffno = p.arch == 2;
  n->Hf = n->hybrid ? p.ff_hidden : 0;
  n->MX = 2 * p.mx; n->MY = 2 * p.my; n->MZ = p.mz; n->L = p.layers; n->H = p.proj_hidden;
  n->P = P;
  n->M = (int64_t)n->MX * n->MY * n->MZ;
  if (n->ffno) {
    const int Ns[3] = {p.nx, p.ny, p.nz}, ms[3] = {p.mx, p.my, p.mz};
    int64_t wo = 0, vo = 0;
    for (int d = 0; d < 3; ++d) {
      auto& a = n->ax[d];
      a.N = Ns[d]; a.m = ms[d];
      a.OUT = d == 0 ? 1 : (d == 1 ? p.nx : (int64_t)p.nx * p.ny);
      a.IN = d == 0 ? (int64_t)p.ny * p.nz : (d == 1 ? p.nz : 1);
      a.woff = wo; wo += (int64_t)a.m * p.width * p.width * 2;
      a.voff = vo; vo += (int64_t)p.max_batch * p.width * a.OUT * 2 * a.m * a.IN;
    }
    n->MX = p.mx; n->MY = p.my; n->MZ = p.mz;
    n->M = (int64_t)p.mx + p.my + p.mz;
  }
  n->nparam = fno_param_count(&p);
  // offsets
  int64_t o = 0;
  n->off_P = o; o += (int64_t)n->W * p.cin;
  n->off_p = o; o += n->W;
  for (int l = 0; l < n->L; ++l) {
    n->off_W.push_back(o); o += n->M * n->W * n->W * 2;
    if (n->hybrid) {
      n->off_W1.push_back(o); o += (int64_t)n->Hf * n->W;
      n->off_b1.push_back(o); o += n->Hf;
      n->off_W2.push_back(o); o += (int64_t)n->W * n->Hf;
      n->off_b2.push_back(o); o += n->W;
    } else {
      n->off_Wp.push_back(o); o += (int64_t)n->W * n->W;
      n->off_bp.push_back(o); o += n->W;
    }
  }
  n->off_Q1 = o; o += (int64_t)n->H * n->W;
  n->off_q1 = o; o += n->H;
  n->off_Q2 = o; o += (int64_t)p.cout * n->H;
  n->off_q2 = o; o += p.cout;
  auto bail = [&](int code, const std::string& m) {
    ffail(nullptr, code, m);
    free_net(n);
    delete n;
    return code;
  };
  const int B = p.max_batch;
  const int64_t W = n->W;
  // fused projection: hidden padded to a multiple of 32 (at most 128),
  // width to a multiple of 32 (at most 64), at most 16 outputs
  const int Hp = (int)round_up(n->H, 32), Wp = (int)round_up(n->W, 32);
  n->fused_proj = Hp <= 128 && Wp <= 64 && p.cout <= 16 && P % 256 == 0;
  // the FP32 hidden pre-activation and its gradient exist only without it
  const size_t hid32 = n->fused_proj ? 0 : (size_t)B * n->H * P * 4;
  auto A = [&](void** ptr, size_t bytes) { return falloc(n, ptr, bytes) == hipSuccess; };
  bool ok = A((void**)&n->theta, n->nparam * 4) && A((void**)&n->grad, n->nparam * 4) &&
            A((void**)&n->am, n->nparam * 4) && A((void**)&n->av, n->nparam * 4) &&
            A((void**)&n->wspec, n->nparam * 2);
  n->v.assign(n->L + 1, nullptr);
  n->h.assign(n->L, nullptr);
  n->Vh.assign(n->L, nullptr);
  for (int l = 0; ok && l <= n->L; ++l) ok = A((void**)&n->v[l], (size_t)B * W * P * 2);
  // modes kept for the weight gradient: the FNO's 3D modes, or the three
  // axes' modes of the factorized FNO
  int64_t vh_elems = n->M * B * W * 2, ax_max = 0;
  if (n->ffno) {
    vh_elems = 0;
    for (auto& a : n->ax) {
      const int64_t e = (int64_t)B * W * a.OUT * 2 * a.m * a.IN;
      vh_elems += e;
      ax_max = std::max(ax_max, e);
    }
  }
  for (int l = 0; ok && l < n->L; ++l)
    ok = (n->hybrid || A((void**)&n->h[l], (size_t)B * W * P * 4)) && A((void**)&n->Vh[l], (size_t)vh_elems * 2);
  if (n->hybrid) {
    n->S.assign(n->L, nullptr);
    n->Aff.assign(n->L, nullptr);
    for (int l = 0; ok && l < n->L; ++l)
      ok = A((void**)&n->S[l], (size_t)B * W * P * 2) && A((void**)&n->Aff[l], (size_t)B * n->Hf * P * 2);
    ok = ok && A((void**)&n->ffa, (size_t)B * n->Hf * P * 2) && A((void**)&n->gs, (size_t)B * W * P * 4);
  }
  const int64_t rows = (int64_t)B * W * n->X * n->Y;
  const int64_t mode_elems = n->ffno ? ax_max : n->M * B * W * 2;
  ok = ok && (n->ffno || (A((void**)&n->A1, (size_t)rows * 2 * n->MZ * 2) &&
                          A((void**)&n->A2, (size_t)B * W * n->X * 2 * n->MY * n->MZ * 2) &&
                          A((void**)&n->R3, (size_t)B * W * n->X * 2 * n->MY * n->MZ * 2) &&
                          A((void**)&n->R2, (size_t)rows * 2 * n->MZ * 2))) &&
       A((void**)&n->Yh, (size_t)mode_elems * 2) && A((void**)&n->Vg, (size_t)mode_elems * 2) &&
       (hid32 == 0 || A((void**)&n->h1, hid32)) &&
       A((void**)&n->a, (size_t)B * n->H * P * 2) && A((void**)&n->y, (size_t)B * p.cout * P * 4) &&
       A((void**)&n->gy, (size_t)B * p.cout * P * 4) && (hid32 == 0 || A((void**)&n->ga, hid32)) &&
       A((void**)&n->gv, (size_t)B * W * P * 4) && A((void**)&n->gvn, (size_t)B * W * P * 4);
  // Gram partials: the widest hidden layer is the projection's or the
  // hybrid feed-forward's
  const int64_t Hm = std::max<int64_t>(n->H, n->Hf);
  n->part_elems = std::max<int64_t>((int64_t)B * P / 2048 * std::max<int64_t>(Hm, W) * std::max<int64_t>(W, p.cout) +
                                        (int64_t)B * P / 2048 * Hm * std::max<int64_t>(Hm, W),
                                    (int64_t)B * P / 8192 * std::max<int64_t>(Hm, W));
  n->part_elems = std::max<int64_t>(n->part_elems, (int64_t)B * P / 2048 * Hm * W);
  n->part_elems = std::max<int64_t>(n->part_elems, (int64_t)B * P / 2048 * p.cout * n->H);
  n->lpart_n = ((int64_t)B * p.cout * P + 255) / 256;
  n->part2_elems = 64 * std::max<int64_t>(std::max<int64_t>(Hm * W, (int64_t)p.cout * n->H),
                                           std::max<int64_t>(W * W, W * (int64_t)p.cin));
  n->partc_elems = (int64_t)B * P / 2048 * std::max<int64_t>(std::max<int64_t>(Hm, W), p.cout);
  // per-block Q2 partials of the projection backward (cout x H per 256 points)
  n->q2_in_bwd = n->fused_proj && p.cout <= 8 && (int64_t)B * P / 256 * p.cout * n->H <= n->part_elems &&
                 64 * (int64_t)p.cout * n->H <= n->part2_elems;
  if (n->ffno) {
    // the fused y/z inverse: y and z extents of 32 or 64
    if ((n->Y == 32 || n->Y == 64) && (n->Z == 32 || n->Z == 64)) ok = ok && A((void**)&n->Yh2, (size_t)ax_max * 2);
    n->fpart_elems = (int64_t)FFNO_NCHUNK * 16 * (2 * W) * (2 * W);
    n->Emix.assign(3 * n->L, nullptr);
    n->ETmix.assign(3 * n->L, nullptr);
    ok = ok && A((void**)&n->fpart, (size_t)n->fpart_elems * 4);
    for (int l = 0; ok && l < n->L; ++l)
      for (int d = 0; ok && d < 3; ++d) {
        const size_t eb = (size_t)n->ax[d].m * (2 * W) * (2 * W) * 2;
        ok = A((void**)&n->Emix[3 * l + d], eb) && A((void**)&n->ETmix[3 * l + d], eb);
      }
  }
  ok = ok && A((void**)&n->part, (size_t)n->part_elems * 4) && A((void**)&n->lpart, (size_t)n->lpart_n * 8) &&
       A((void**)&n->lscal, 32) &&
       A((void**)&n->part2, (size_t)n->part2_elems * 4) && A((void**)&n->partc, (size_t)n->partc_elems * 4);
  if (!ok) return bail(LBM_ENOMEM, "device allocation failed");
  // pointwise operands
  hipError_t e = hipSuccess;
  n->Gwp.resize(n->L);
  n->Gwpt.resize(n->L);
  if ((e = alloc_gt(n, n->Glift, p.cin, n->W)) != hipSuccess) return bail(LBM_ENOMEM, "operand allocation");
  for (int l = 0; l < n->L && !n->hybrid; ++l)
    if (alloc_gt(n, n->Gwp[l], n->W, n->W) != hipSuccess || alloc_gt(n, n->Gwpt[l], n->W, n->W) != hipSuccess)
      return bail(LBM_ENOMEM, "operand allocation");
  if (n->hybrid) {
    const int Hfp = (int)round_up(n->Hf, 32);
    n->Pf1.resize(n->L);
    n->Pf2.resize(n->L);
    n->Gf2t.resize(n->L);
    n->fb1.assign(n->L, nullptr);
    for (int l = 0; l < n->L; ++l) {
      GtMat& f1 = n->Pf1[l];
      GtMat& f2 = n->Pf2[l];
      f1.K = n->W; f1.N = n->Hf; f1.kp = 32; f1.np = Hfp;
      f2.K = n->Hf; f2.N = n->W; f2.kp = Hfp; f2.np = 32;
      if (falloc(n, (void**)&f1.d, (size_t)Hfp * 32 * 2) != hipSuccess ||
          falloc(n, (void**)&f2.d, (size_t)32 * Hfp * 2) != hipSuccess ||
          alloc_gt(n, n->Gf2t[l], n->W, n->Hf) != hipSuccess ||
          falloc(n, (void**)&n->fb1[l], (size_t)Hfp * 4) != hipSuccess ||
          hipMemset(n->fb1[l], 0, (size_t)Hfp * 4) != hipSuccess)
        return bail(LBM_ENOMEM, "operand allocation");
    }
  }
  if (alloc_gt(n, n->Gq1, n->W, n->H) != hipSuccess || alloc_gt(n, n->Gq1t, n->H, n->W) != hipSuccess ||
      alloc_gt(n, n->Gq2, n->H, p.cout) != hipSuccess || alloc_gt(n, n->Gq2t, p.cout, n->H) != hipSuccess)
    return bail(LBM_ENOMEM, "operand allocation");
  {
    n->fused_layer_end = !n->ffno && n->W <= 32 && p.nz >= 16 && p.nz <= 256 && 2 * p.mz <= 32 && P % 256 == 0;
    if (n->fused_proj) {
      n->Pq1.K = n->W; n->Pq1.N = n->H; n->Pq1.kp = Wp; n->Pq1.np = Hp;
      n->Pq2.K = n->H; n->Pq2.N = p.cout; n->Pq2.kp = Hp; n->Pq2.np = 16;
      if (falloc(n, (void**)&n->Pq1.d, (size_t)Hp * Wp * 2) != hipSuccess ||
          falloc(n, (void**)&n->Pq2.d, (size_t)16 * Hp * 2) != hipSuccess ||
          falloc(n, (void**)&n->pq1b, (size_t)Hp * 4) != hipSuccess ||
          hipMemset(n->pq1b, 0, (size_t)Hp * 4) != hipSuccess)
        return bail(LBM_ENOMEM, "operand allocation");
    }
  }
  // DFT operands
  if (n->ffno) {
    // per axis, theta = 2 pi k n / N, c_0 = 1, c_k = 2:
    //   F  [n][(part, k)]  (cos, -sin)            forward r2c
    //   I  [(part, k)][n]  c_k (cos, -sin) / N    c2r inverse
    //   Ia [n][(part, k)]  c_k (cos, -sin) / N    adjoint of I
    //   Fa [(part, k)][n]  (cos, -sin)            adjoint of F
    for (auto& a : n->ax) {
      const int N = a.N, m = a.m;
      std::vector<double> f((size_t)N * 2 * m), in((size_t)2 * m * N), ia((size_t)N * 2 * m), fa((size_t)2 * m * N);
      for (int x = 0; x < N; ++x)
        for (int k = 0; k < m; ++k) {
          const double th = 2.0 * M_PI * (double)k * x / N, c = std::cos(th), sn = std::sin(th);
          const double sc = (k == 0 ? 1.0 : 2.0) / N;
          f[(size_t)x * 2 * m + k] = c;
          f[(size_t)x * 2 * m + m + k] = -sn;
          ia[(size_t)x * 2 * m + k] = c * sc;
          ia[(size_t)x * 2 * m + m + k] = -sn * sc;
          in[(size_t)k * N + x] = c * sc;
          in[(size_t)(m + k) * N + x] = -sn * sc;
          fa[(size_t)k * N + x] = c;
          fa[(size_t)(m + k) * N + x] = -sn;
        }
      if (make_gt_host(n, a.F, f, N, 2 * m) || make_gt_host(n, a.I, in, 2 * m, N) ||
          make_gt_host(n, a.Ia, ia, N, 2 * m) || make_gt_host(n, a.Fa, fa, 2 * m, N))
        return bail(LBM_EDEVICE, "DFT operand upload failed");
    }
  } else {
    const int X = n->X, Y = n->Y, Z = n->Z, MZ = n->MZ;
    std::vector<int> kx, ky;
    for (int j = 0; j < n->MX; ++j) kx.push_back(mode_value(j, p.mx));
    for (int j = 0; j < n->MY; ++j) ky.push_back(mode_value(j, p.my));
    const double invN = 1.0 / ((double)X * Y * Z);
    std::vector<double> gz((size_t)Z * 2 * MZ), gza((size_t)Z * 2 * MZ), iz((size_t)2 * MZ * Z),
        iza((size_t)2 * MZ * Z);
    for (int z = 0; z < Z; ++z)
      for (int kz = 0; kz < MZ; ++kz) {
        const double th = 2.0 * M_PI * kz * z / Z, c = std::cos(th), s = std::sin(th);
        const double ck = kz == 0 ? 1.0 : 2.0;
        // forward r2c: out (part, kz) = sum_z v (cos, -sin)
        gz[(size_t)z * 2 * MZ + kz] = c;
        gz[(size_t)z * 2 * MZ + MZ + kz] = -s;
        gza[(size_t)z * 2 * MZ + kz] = c * ck * invN;
        gza[(size_t)z * 2 * MZ + MZ + kz] = -s * ck * invN;
        // c2r: out z = sum (re cos - im sin) c_kz / N
        iz[(size_t)kz * Z + z] = c * ck * invN;
        iz[(size_t)(MZ + kz) * Z + z] = -s * ck * invN;
        iza[(size_t)kz * Z + z] = c;
        iza[(size_t)(MZ + kz) * Z + z] = -s;
      }
    if (make_gt_host(n, n->F1, gz, Z, 2 * MZ) || make_gt_host(n, n->F1a, gza, Z, 2 * MZ) ||
        make_gt_host(n, n->F2, embed_dft(Y, ky, -1), 2 * Y, 2 * n->MY) ||
        make_gt_host(n, n->F3, embed_dft(X, kx, -1), 2 * X, 2 * n->MX) ||
        make_gt_host(n, n->I3, embed_dft(X, kx, +1), 2 * n->MX, 2 * X) ||
        make_gt_host(n, n->I2, embed_dft(Y, ky, +1), 2 * n->MY, 2 * Y) ||
        make_gt_host(n, n->I1, iz, 2 * MZ, Z) || make_gt_host(n, n->I1a, iza, 2 * MZ, Z))
      return bail(LBM_EDEVICE, "DFT operand upload failed");
  }
  // seeded initial parameters (uniform fan-in scaling, spectral 1/width^2)
  {
    std::vector<float> th((size_t)n->nparam, 0.f);
    uint64_t k = 0;
    auto uni = [&](double lo, double hi) {
      uint64_t z = seed + (++k) * 0x9E3779B97F4A7C15ull;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      return lo + (hi - lo) * ((double)(z >> 11) * 0x1.0p-53);
    };
    for (int64_t i = 0; i < (int64_t)W * p.cin; ++i) th[n->off_P + i] = (float)uni(-1, 1) / std::sqrt((float)p.cin);
    for (int l = 0; l < n->L; ++l) {
      for (int64_t i = 0; i < n->M * W * W * 2; ++i) th[n->off_W[l] + i] = (float)(uni(0, 1) / (double)(W * W));
      if (n->hybrid) {
        for (int64_t i = 0; i < (int64_t)n->Hf * W; ++i) th[n->off_W1[l] + i] = (float)uni(-1, 1) / std::sqrt((float)W);
        for (int64_t i = 0; i < (int64_t)W * n->Hf; ++i)
          th[n->off_W2[l] + i] = (float)uni(-1, 1) / std::sqrt((float)n->Hf);
      } else {
        for (int64_t i = 0; i < W * W; ++i) th[n->off_Wp[l] + i] = (float)uni(-1, 1) / std::sqrt((float)W);
      }
    }
    // SIREN (Sitzmann et al.): first layer U(+-1/n), later layers U(+-sqrt(6/n)/w0)
    const bool siren = p.proj_act == 1;
    for (int64_t i = 0; i < (int64_t)n->H * W; ++i)
      th[n->off_Q1 + i] = (float)uni(-1, 1) / (siren ? (float)W : std::sqrt((float)W));
    for (int64_t i = 0; i < (int64_t)p.cout * n->H; ++i)
      th[n->off_Q2 + i] = siren ? (float)(uni(-1, 1) * std::sqrt(6.0 / n->H) / p.proj_w0)
                                : (float)uni(-1, 1) / std::sqrt((float)n->H);
    e = hipMemcpy(n->theta, th.data(), th.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->am, 0, n->nparam * 4);
    if (e == hipSuccess) e = hipMemset(n->av, 0, n->nparam * 4);
    if (e != hipSuccess) return bail(LBM_EDEVICE, "parameter upload failed");
  }
  if (refresh(n) != LBM_OK) return bail(LBM_EDEVICE, n->err);
  if ((e = hipStreamSynchronize(n->st)) != hipSuccess) return bail(LBM_EDEVICE, hipGetErrorString(e));
  *out = n;
  return LBM_OK;
}

extern "C" int fno_set_params(fno_net* n, const float* host, int64_t count) {
  if (!n || !host) return ffail(n, LBM_EINVAL, "null argument");
  if (count != n->nparam) return ffail(n, LBM_EINVAL, "parameter count mismatch");
  FCHK(n, hipMemcpyAsync(n->theta, host, count * 4, hipMemcpyHostToDevice, n->st));
  int rc = refresh(n);
  if (rc) return rc;
  FCHK(n, hipStreamSynchronize(n->st));
  return LBM_OK;
}

extern "C" int fno_get_params(fno_net* n, float* host, int64_t count) {
  if (!n || !host) return ffail(n, LBM_EINVAL, "null argument");
  if (count != n->nparam) return ffail(n, LBM_EINVAL, "parameter count mismatch");
  FCHK(n, hipMemcpyAsync(host, n->theta, count * 4, hipMemcpyDeviceToHost, n->st));
  FCHK(n, hipStreamSynchronize(n->st));
  return LBM_OK;
}

// training keeps what the backward pass reads: FP32 pre-activations of
// every Fourier layer and of the projection's hidden layer, and its BF16
// activations; inference keeps only the BF16 activations of the layers.
// per-mode complex channel mixing on mode-minor BF16 modes (MODE 0: by W,
// MODE 1: by the conjugate transpose of W)
template <int CM>
static void launch_mix(fno_net* n, int mode, int B, const uint16_t* in, const uint16_t* w, uint16_t* out) {
  const int64_t Q = n->MY * n->MZ;
  const dim3 grid((unsigned)(n->MX * (Q / MixCfg<CM>::MQ))), blk(MIX_THREADS);
  if (mode == 0) hipLaunchKernelGGL((mix_kernel<CM, 0>), grid, blk, 0, n->st, in, w, out, B, (int)n->W, n->MX, Q);
  else hipLaunchKernelGGL((mix_kernel<CM, 1>), grid, blk, 0, n->st, in, w, out, B, (int)n->W, n->MX, Q);
}
static void mix(fno_net* n, int mode, int B, const uint16_t* in, const uint16_t* w, uint16_t* out) {
  if (n->W <= 32) launch_mix<32>(n, mode, B, in, w, out);
  else launch_mix<64>(n, mode, B, in, w, out);
}
// spectral weight gradient (overwrites gw)
static void mix_grad(fno_net* n, int B, const uint16_t* v, const uint16_t* gy, float* gw) {
  const int64_t Q = n->MY * n->MZ;
  const dim3 blk(MIX_THREADS);
  if (n->W <= 32)
    hipLaunchKernelGGL((mix_grad_kernel<32>), dim3((unsigned)(n->MX * (Q / MixCfg<32>::MQ))), blk, 0, n->st, v, gy,
                       gw, B, (int)n->W, n->MX, Q, 0);
  else
    hipLaunchKernelGGL((mix_grad_kernel<64>), dim3((unsigned)(n->MX * (Q / MixCfg<64>::MQ))), blk, 0, n->st, v, gy,
                       gw, B, (int)n->W, n->MX, Q, 0);
}

// layer_end_kernel with the one-row c2r operands where Z = 64
template <int NT, typename InT, bool C2R = true>
static void launch_le(const LayerEndArgs& e, dim3 grid, hipStream_t st) {
  if (e.Z == 64) hipLaunchKernelGGL((layer_end_kernel<NT, InT, C2R, true>), grid, dim3(256), 0, st, e);
  else hipLaunchKernelGGL((layer_end_kernel<NT, InT, C2R, false>), grid, dim3(256), 0, st, e);
}

static int forward_impl(fno_net* n, const uint16_t* x, int B, float* yout, bool training) {
  const int64_t W = n->W;
  int rc;
  // the layer end can run the next layer's z stage at the production shape
  const bool fuse_z = !n->ffno && n->fused_layer_end && n->Z == 64 && W == 32 && 2 * n->MZ == 32 && n->F1.kp >= 64;
  bool z_done = false;
  // lift: v0 = P x + p (no activation; the pre-activation is not kept)
  // (16-byte vector loads of x: a misaligned input takes the separate lift)
  if (fuse_z && n->p.cin <= 32 && n->Glift.kp == 32 && ((uintptr_t)x % 16) == 0) {
    LayerEndArgs e{};
    e.v = x; e.r2 = nullptr; e.gwp = n->Glift.d; e.gi1 = nullptr; e.gi1_kp = 0;
    e.bias = n->theta + n->off_p; e.h = nullptr; e.act = n->v[0];
    e.P = n->P; e.W = (int)W; e.Win = n->p.cin; e.Z = n->Z; e.K2 = 2 * n->MZ; e.act_gelu = 0;
    e.gz = n->F1.d; e.gz_kp = n->F1.kp; e.a1 = n->A1;
    launch_le<2, uint16_t, false>(e, dim3((unsigned)((int64_t)B * n->P / PW_J)), n->st);
    z_done = true;
  } else if ((rc = pointwise(n, B, x, true, n->p.cin, nullptr, false, (int)W, &n->Glift, n->theta + n->off_p, false,
                             false, n->v[0], false))) {
    return rc;
  }
  for (int l = 0; l < n->L; ++l) {
    if (n->ffno) {
      // s = sum_d R_d(W_d T_d v) in BF16, then the residual feed-forward block
      uint16_t* sl = n->S[training ? l : 0];
      if ((rc = ffno_spectral(n, l, B, training, sl))) return rc;
      launch_ffn(n, l, B, sl, n->v[l], n->v[l + 1], training ? n->Aff[l] : nullptr);
      continue;
    }
    if ((rc = forward_dft(n, B, n->v[l], true, n->F1, n->Vh[l], z_done))) return rc;
    z_done = false;
    mix(n, 0, B, n->Vh[l], n->wspec + n->off_W[l], n->Yh);
    if (n->hybrid) {
      // s = R(W T v) alone (no channel map, bias or activation), then
      // v' = v + W2 GELU(W1 s + b1) + b2; the next z stage runs on its own
      if ((rc = inverse_dft(n, B, n->Yh, n->I1, nullptr, false))) return rc;
      uint16_t* sl = n->S[training ? l : 0];
      LayerEndArgs e{};
      e.v = n->v[l]; e.r2 = n->R2; e.gwp = nullptr; e.gi1 = n->I1.d; e.gi1_kp = n->I1.kp;
      e.bias = nullptr; e.h = nullptr; e.act = sl;
      e.P = n->P; e.W = (int)W; e.Win = 0; e.Z = n->Z; e.K2 = 2 * n->MZ; e.act_gelu = 0;
      const dim3 grid((unsigned)((int64_t)B * n->P / PW_J));
      if (W <= 16) launch_le<1, uint16_t>(e, grid, n->st);
      else launch_le<2, uint16_t>(e, grid, n->st);
      launch_ffn(n, l, B, sl, n->v[l], n->v[l + 1], training ? n->Aff[l] : nullptr);
      continue;
    }
    // h = R(W T v) + Wp v + bp; v' = GELU(h) (identity after the last layer)
    if (n->fused_layer_end) {
      if ((rc = inverse_dft(n, B, n->Yh, n->I1, nullptr, false))) return rc;
      LayerEndArgs e{};
      e.v = n->v[l]; e.r2 = n->R2; e.gwp = n->Gwp[l].d; e.gi1 = n->I1.d; e.gi1_kp = n->I1.kp;
      e.bias = n->theta + n->off_bp[l]; e.h = training ? n->h[l] : nullptr; e.act = n->v[l + 1];
      e.P = n->P; e.W = (int)W; e.Win = (int)W; e.Z = n->Z; e.K2 = 2 * n->MZ; e.act_gelu = l < n->L - 1 ? 1 : 0;
      if (fuse_z && l < n->L - 1) {
        e.gz = n->F1.d; e.gz_kp = n->F1.kp; e.a1 = n->A1;
        z_done = true;
      }
      const dim3 grid((unsigned)((int64_t)B * n->P / PW_J));
      if (W <= 16) launch_le<1, uint16_t>(e, grid, n->st);
      else launch_le<2, uint16_t>(e, grid, n->st);
    } else {
      if ((rc = inverse_dft(n, B, n->Yh, n->I1, n->h[l], false))) return rc;
      if ((rc = pointwise(n, B, n->v[l], true, (int)W, n->h[l], false, (int)W, &n->Gwp[l], n->theta + n->off_bp[l],
                          true, training, n->v[l + 1], l < n->L - 1)))
        return rc;
    }
  }
  if (n->fused_proj) {
    // training keeps the BF16 hidden activation for the gradient of Q2; the
    // pre-activation is recomputed in the backward pass
    fused_projection(n, B, n->v[n->L], yout, training && !n->q2_in_bwd ? n->a : nullptr);
  } else {
    if ((rc = pointwise(n, B, n->v[n->L], true, (int)W, n->h1, false, n->H, &n->Gq1, n->theta + n->off_q1, false,
                        true, n->a, true)))
      return rc;
    if ((rc = pointwise(n, B, n->a, true, n->H, yout, false, n->p.cout, &n->Gq2, n->theta + n->off_q2, false)))
      return rc;
  }
  n->lastB = B;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(n, LBM_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int fno_forward(fno_net* n, const uint16_t* x, int32_t B, float* y) {
  if (!n || !x || !y) return ffail(n, LBM_EINVAL, "null argument");
  if (B <= 0 || B > n->p.max_batch) return ffail(n, LBM_EINVAL, "batch out of range");
  return forward_impl(n, x, B, y, false);
}

extern "C" int fno_loss_grad(fno_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B,
                             float* loss, float* host_grads) {
  if (!n || !x || !target || !mask) return ffail(n, LBM_EINVAL, "null argument");
  if (B <= 0 || B > n->p.max_batch) return ffail(n, LBM_EINVAL, "batch out of range");
  int rc = forward_impl(n, x, B, n->y, true);
  if (rc) return rc;
  const int64_t W = n->W, P = n->P, cout = n->p.cout;
  // mask cell count and gradient scale on the device: nothing waits for the
  // host unless the loss or the gradients are requested
  long long* dcnt = (long long*)n->lscal;
  double* dloss = n->lscal + 1;
  float* dscale = (float*)(n->lscal + 2);
  const double bc = (double)B * cout;
  hipLaunchKernelGGL(mask_count_kernel, dim3(1), dim3(1024), 0, n->st, mask, P, bc, dcnt, dscale);
  const int64_t ny = (int64_t)B * cout * P;
  const int64_t nblk = (ny + 255) / 256;
  hipLaunchKernelGGL(mse_kernel, dim3((unsigned)nblk), dim3(256), 0, n->st, n->y, target, mask, P, ny,
                     (const float*)dscale, n->gy, n->lpart);
  FCHK(n, hipMemsetAsync(n->grad, 0, n->nparam * 4, n->st));
  // projection
  if (n->q2_in_bwd) {
    // one pass: dL/dh1 (BF16, into the hidden buffer), dL/dv, and per-block
    // sums of the Q2 gradient, reduced here in a fixed order; q2 from gy
    fused_projection_bwd(n, B, n->v[n->L], n->gy, n->a, n->gv, n->part);
    const int64_t nblk = (int64_t)B * P / 256, E2 = cout * n->H;
    constexpr int S = 64;
    hipLaunchKernelGGL(reduce_slices_kernel, dim3((unsigned)((E2 + 255) / 256), S), dim3(256), 0, n->st, n->part, nblk,
                       E2, S, n->part2);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((E2 + 255) / 256)), dim3(256), 0, n->st, n->part2,
                       (int64_t)S, E2, n->grad + n->off_Q2, 0);
    if ((rc = colsum(n, n->gy, (int)cout, B, n->grad + n->off_q2, false))) return rc;
    if ((rc = gram(n, (const uint16_t*)n->a, n->H, n->v[n->L], (int)W, B, n->grad + n->off_Q1, false,
                   n->grad + n->off_q1)))
      return rc;
  } else if ((rc = gram(n, n->gy, (int)cout, n->a, n->H, B, n->grad + n->off_Q2, false, n->grad + n->off_q2))) {
    return rc;
  } else if (n->fused_proj) {
    // dL/dh1 = GELU'(h1) * Q2^T gy in BF16 (the hidden activation's buffer,
    // already consumed) and dL/dv = Q1^T dL/dh1, in one pass
    fused_projection_bwd(n, B, n->v[n->L], n->gy, n->a, n->gv);
    if ((rc = gram(n, (const uint16_t*)n->a, n->H, n->v[n->L], (int)W, B, n->grad + n->off_Q1, false,
                   n->grad + n->off_q1)))
      return rc;
  } else {
    // dL/dh1 = GELU'(h1) * Q2^T gy, the derivative applied in the epilogue
    if ((rc = pointwise(n, B, n->gy, false, (int)cout, n->ga, false, n->H, &n->Gq2t, nullptr, false, true, nullptr,
                        false, n->h1)))
      return rc;
    if ((rc = gram(n, n->ga, n->H, n->v[n->L], (int)W, B, n->grad + n->off_Q1, false, n->grad + n->off_q1)))
      return rc;
    if ((rc = pointwise(n, B, n->ga, false, n->H, n->gv, false, (int)W, &n->Gq1t, nullptr, false))) return rc;
  }
  // Fourier layers in reverse
  // at layer l, gv holds dL/dh[l]: the last layer has no activation, and the
  // GELU' of the layers below is applied where their gradient is completed
  // (hybrid: gv holds dL/dv[l + 1], the gradient of the residual stream)
  for (int l = n->L - 1; l >= 0 && n->hybrid; --l) {
    // feed-forward block: dL/dz = GELU'(z) W2^T gv (BF16), dL/ds = W1^T dL/dz
    launch_ffn_bwd(n, l, B, n->S[l], n->gv, n->ffa, n->gs);
    if ((rc = gram(n, n->gv, (int)W, n->Aff[l], n->Hf, B, n->grad + n->off_W2[l], false, n->grad + n->off_b2[l])))
      return rc;
    if ((rc = gram(n, (const uint16_t*)n->ffa, n->Hf, n->S[l], (int)W, B, n->grad + n->off_W1[l], false,
                   n->grad + n->off_b1[l])))
      return rc;
    if (n->ffno) {
      // per-axis spectral convolutions; gv accumulates dL/dv[l] in place
      if ((rc = ffno_spectral_bwd(n, l, B))) return rc;
      continue;
    }
    // spectral convolution: mode gradient, weight gradient, adjoint path
    if ((rc = forward_dft(n, B, n->gs, false, n->F1a, n->Yh))) return rc;
    mix_grad(n, B, n->Vh[l], n->Yh, n->grad + n->off_W[l]);
    mix(n, 1, B, n->Yh, n->wspec + n->off_W[l], n->Vg);
    if ((rc = inverse_dft(n, B, n->Vg, n->I1a, nullptr, false))) return rc;
    // dL/dv[l] = dL/dv[l + 1] (residual) + adjoint c2r of the y-stage output
    LayerEndArgs e{};
    e.v = n->gv; e.r2 = n->R2; e.gwp = nullptr; e.gi1 = n->I1a.d; e.gi1_kp = n->I1a.kp;
    e.bias = nullptr; e.h = n->gvn; e.act = nullptr; e.gmul = nullptr; e.resid = n->gv;
    e.P = n->P; e.W = (int)W; e.Win = 0; e.Z = n->Z; e.K2 = 2 * n->MZ; e.act_gelu = 0;
    const dim3 grid((unsigned)((int64_t)B * n->P / PW_J));
    if (W <= 16) launch_le<1, float>(e, grid, n->st);
    else launch_le<2, float>(e, grid, n->st);
    std::swap(n->gv, n->gvn);
  }
  for (int l = n->L - 1; l >= 0 && !n->hybrid; --l) {
    if ((rc = gram(n, n->gv, (int)W, n->v[l], (int)W, B, n->grad + n->off_Wp[l], false, n->grad + n->off_bp[l])))
      return rc;
    // gradient on the modes: (c_kz/N) T(gh)
    if ((rc = forward_dft(n, B, n->gv, false, n->F1a, n->Yh))) return rc;
    mix_grad(n, B, n->Vh[l], n->Yh, n->grad + n->off_W[l]);
    mix(n, 1, B, n->Yh, n->wspec + n->off_W[l], n->Vg);
    // gvn = dL/dv[l] = Wp^T gv + (adjoint of the truncated DFT path); for
    // l >= 1 it becomes dL/dh[l - 1] = GELU'(h[l - 1]) dL/dv[l]
    const float* gmul = l >= 1 ? n->h[l - 1] : nullptr;
    if (n->fused_layer_end) {
      if ((rc = inverse_dft(n, B, n->Vg, n->I1a, nullptr, false))) return rc;
      LayerEndArgs e{};
      e.v = n->gv; e.r2 = n->R2; e.gwp = n->Gwpt[l].d; e.gi1 = n->I1a.d; e.gi1_kp = n->I1a.kp;
      e.bias = nullptr; e.h = n->gvn; e.act = nullptr; e.gmul = gmul;
      e.P = n->P; e.W = (int)W; e.Win = (int)W; e.Z = n->Z; e.K2 = 2 * n->MZ; e.act_gelu = 0;
      const dim3 grid((unsigned)((int64_t)B * n->P / PW_J));
      if (W <= 16) launch_le<1, float>(e, grid, n->st);
      else launch_le<2, float>(e, grid, n->st);
    } else {
      if ((rc = pointwise(n, B, n->gv, false, (int)W, n->gvn, false, (int)W, &n->Gwpt[l], nullptr, false)))
        return rc;
      if ((rc = inverse_dft(n, B, n->Vg, n->I1a, n->gvn, true, gmul))) return rc;
    }
    std::swap(n->gv, n->gvn);
  }
  if ((rc = gram(n, n->gv, (int)W, x, n->p.cin, B, n->grad + n->off_P, false, n->grad + n->off_p))) return rc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(n, LBM_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  if (loss) {
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(1024), 0, n->st, n->lpart, nblk, (const long long*)dcnt,
                       bc, dloss);
    double hl[2];
    FCHK(n, hipMemcpyAsync(hl, n->lscal, 16, hipMemcpyDeviceToHost, n->st));
    FCHK(n, hipStreamSynchronize(n->st));
    long long hc;
    std::memcpy(&hc, &hl[0], 8);
    if (hc == 0) return ffail(n, LBM_EINVAL, "empty loss mask");
    *loss = (float)hl[1];
  }
  if (host_grads) {
    FCHK(n, hipMemcpyAsync(host_grads, n->grad, n->nparam * 4, hipMemcpyDeviceToHost, n->st));
    FCHK(n, hipStreamSynchronize(n->st));
  }
  return LBM_OK;
}

extern "C" int fno_adam_step(fno_net* n, float lr) {
  if (!n) return ffail(nullptr, LBM_EINVAL, "null argument");
  n->adam_t++;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, n->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, n->adam_t)));
  dim3 g;
  elementwise_grid(n->nparam, g);
  hipLaunchKernelGGL(adam_kernel, g, dim3(256), 0, n->st, n->theta, n->grad, n->am, n->av, n->nparam, lr, (float)b1,
                     (float)b2, c1, c2, 1e-8f, n->wspec);
  return refresh(n, true);
}

extern "C" int fno_train_step(fno_net* n, const uint16_t* x, const float* target, const uint8_t* mask, int32_t B,
                              float lr, float* loss) {
  int rc = fno_loss_grad(n, x, target, mask, B, loss, nullptr);
  if (rc) return rc;
  return fno_adam_step(n, lr);
}

extern "C" void fno_destroy(fno_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->st);
  free_net(n);
  delete n;
}

extern "C" int fno_field_minmax(const float* x, int64_t S, int32_t C, int64_t P, void* hip_stream, float* lo,
                                float* hi) {
  if (!x || !lo || !hi) return ffail(nullptr, LBM_EINVAL, "null argument");
  if (S <= 0 || C <= 0 || C > MM_MAXC || P <= 0) return ffail(nullptr, LBM_EINVAL, "bad sizes");
  const hipStream_t st = (hipStream_t)hip_stream;
  const int64_t nchunk = (P + MM_CHUNK - 1) / MM_CHUNK, nblk = S * nchunk;
  if (nblk > 0x7fffffff) return ffail(nullptr, LBM_EINVAL, "too many samples");
  float* part = nullptr;
  hipError_t e = hipMalloc((void**)&part, (size_t)nblk * C * 2 * 4);
  if (e != hipSuccess) return ffail(nullptr, LBM_ENOMEM, hipGetErrorString(e));
  hipLaunchKernelGGL(minmax_kernel, dim3((unsigned)nblk, (unsigned)C), dim3(256), 0, st, x, (int)C, P, nchunk, part,
                     nblk);
  std::vector<float> h((size_t)nblk * C * 2);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, h.size() * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  if (e != hipSuccess) return ffail(nullptr, LBM_EDEVICE, hipGetErrorString(e));
  for (int c = 0; c < C; ++c) {
    float a = INFINITY, b = -INFINITY;
    for (int64_t k = 0; k < nblk; ++k) {
      a = std::min(a, h[((size_t)c * nblk + k) * 2]);
      b = std::max(b, h[((size_t)c * nblk + k) * 2 + 1]);
    }
    lo[c] = a;
    hi[c] = b;
  }
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free min-max: the per-block partials of minmax_kernel and the
// final per-channel pair live in a fixed device array instead of a
// hipMalloc'd buffer.  Each GPU the library runs on holds its own copy until
// the process ends; the host reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr int64_t MM_SCRATCH_FLOATS = int64_t(1) << 20;  // 4 MiB
static __device__ __align__(256) float scratch[MM_SCRATCH_FLOATS + 2 * MM_MAXC];

// per channel c: minimum and maximum over the nblk partial pairs of part,
// written to out[2c], out[2c + 1] (NaN partials are skipped, as on the
// host path)
__global__ __launch_bounds__(256) void minmax_reduce_kernel(const float* part, int64_t nblk, float* out) {
  __shared__ float rmin[256], rmax[256];
  const int c = blockIdx.x;
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t k = threadIdx.x; k < nblk; k += 256) {
    lo = fminf(lo, part[((int64_t)c * nblk + k) * 2]);
    hi = fmaxf(hi, part[((int64_t)c * nblk + k) * 2 + 1]);
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
    out[2 * c] = rmin[0];
    out[2 * c + 1] = rmax[0];
  }
}

static std::mutex g_scratch_mu;
static std::vector<float*> g_scratch_ptr;  // device address of scratch, per device

// Device address of the scratch array on the current device, looked up
// once per device.
static hipError_t scratch_ptr(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[(size_t)dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[(size_t)dev] = (float*)p;
  }
  *out = g_scratch_ptr[(size_t)dev];
  return hipSuccess;
}

extern "C" int fno_field_minmax_noalloc(const float* x, int64_t S, int32_t C, int64_t P, void* hip_stream, float* lo,
                                        float* hi) {
  if (!x || !lo || !hi) return ffail(nullptr, LBM_EINVAL, "null argument");
  if (S <= 0 || C <= 0 || C > MM_MAXC || P <= 0) return ffail(nullptr, LBM_EINVAL, "bad sizes");
  const int64_t nchunk = (P + MM_CHUNK - 1) / MM_CHUNK, nblk = S * nchunk;
  if (nblk > 0x7fffffff || nblk * C * 2 > MM_SCRATCH_FLOATS)
    return ffail(nullptr, LBM_EINVAL,
                 "input too large for the fixed scratch: S * ceil(P / 4096) * C must be at most 524288");
  float* part = nullptr;
  hipError_t e = scratch_ptr(&part);
  if (e != hipSuccess) return ffail(nullptr, LBM_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  float* res = part + MM_SCRATCH_FLOATS;
  const hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(minmax_kernel, dim3((unsigned)nblk, (unsigned)C), dim3(256), 0, st, x, (int)C, P, nchunk, part,
                     nblk);
  hipLaunchKernelGGL(minmax_reduce_kernel, dim3((unsigned)C), dim3(256), 0, st, part, nblk, res);
  float h[2 * MM_MAXC];
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h, res, (size_t)C * 2 * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return ffail(nullptr, LBM_EDEVICE, hipGetErrorString(e));
  for (int c = 0; c < C; ++c) {
    lo[c] = h[2 * c];
    hi[c] = h[2 * c + 1];
  }
  return LBM_OK;
}

extern "C" int fno_field_scale(float* x, int64_t S, int32_t C, int64_t P, const float* lo, const float* hi,
                               int32_t inverse, void* hip_stream) {
  if (!x || !lo || !hi) return ffail(nullptr, LBM_EINVAL, "null argument");
  if (S <= 0 || C <= 0 || C > MM_MAXC || P <= 0) return ffail(nullptr, LBM_EINVAL, "bad sizes");
  ScaleArgs a{};
  for (int c = 0; c < C; ++c) {
    const float r = hi[c] - lo[c];
    if (inverse) {
      a.mul[c] = r;
      a.off[c] = lo[c];
    } else {
      a.mul[c] = r > 0.f ? 1.f / r : 0.f;
      a.off[c] = -lo[c];
    }
  }
  const int64_t n = S * C * P;
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, x,
                     (int)C, P, n, a, inverse ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ffail(nullptr, LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

extern "C" const char* fno_last_error(const fno_net* n) { return n ? n->err.c_str() : g_fno_err.c_str(); }
